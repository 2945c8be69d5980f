"""Pins of the three-dimensional oracle (D3Q19 form of Sec. III) against
what the lattice and the mathematics fix, independently of its own code:
the lattice's isotropy, the Appendix moment identities with three velocity
components, the Fourier symbols of the stencils (closed forms summed over an
independently enumerated velocity set), mass conservation, fixed points and
symmetries, walls as a mirror-doubled periodic lattice, an independent
brute-force implementation (tests/brute3d.py), and the Laplace law
Delta P = 2 sigma / R of a spherical droplet.
"""
import itertools
import math

import numpy as np
import pytest
import torch

import brute3d as B
import workloads as wl
from oracle import qilbm_oracle3d as O

torch.set_num_threads(4)


def _co(pb, **kw):
    return O.coefficients(pb.rho_A, pb.rho_B, pb.sigma, pb.W, pb.M, pb.tau_f, pb.tau_g,
                          pb.gx, pb.gy, pb.gz, pb.ref_density, pb.bc, **kw)


def test_d3q19_lattice_isotropy():
    c = np.array(O.C, dtype=float)
    w = np.array(O.WEIGHT)
    assert len(O.C) == 19 and len(set(O.C)) == 19
    assert sorted(map(tuple, c)) == sorted(B.VEL)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.allclose((w[:, None] * c).sum(0), 0.0)
    # second moments c_s^2 delta, fourth moments c_s^4 (dd + dd + dd)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), O.CS2 * np.eye(3))
    m4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    d = np.eye(3)
    iso = O.CS2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                        + np.einsum("ad,bc->abcd", d, d))
    assert np.allclose(m4, iso)
    for i, j in enumerate(O.OPPOSITE):
        assert tuple(-a for a in O.C[i]) == O.C[j]


def test_moment_identities_3d():
    """sum f^eq = p, sum c f^eq = c_s^2 rho u, sum g^eq = phi, sum c g^eq =
    phi u, sum F_i = c_s^2 (u.grad rho - rho gamma D), sum c F_i = c_s^2 F,
    sum G_i = 0, sum c G_i = (phi/rho)(F - grad p) (Appendix, with Gamma_i =
    1 + s_i), at random node values."""
    rng = np.random.default_rng(5)
    n = (6,)
    t = lambda s=1.0: torch.tensor(s * rng.standard_normal(n))
    co = O.coefficients(1.0, 0.3, 0.01, 4.0, 0.1, 0.8, 0.8)
    phi = torch.tensor(rng.random(n))
    rho, p, mu, D = O.density(phi, co), t(1e-2), t(1e-3), t(1e-4)
    u, F, dr, dp = (t(1e-2), t(1e-2), t(1e-2)), (t(), t(), t()), (t(), t(), t()), (t(), t(), t())
    c = [torch.tensor(float(v)) for v in range(1)]
    feq = [O.f_equilibrium(i, p, rho, u) for i in range(O.Q)]
    geq = [O.g_equilibrium(i, phi, mu, u, co) for i in range(O.Q)]
    Fi = [O.f_source(i, u, F, dr, rho, D, co) for i in range(O.Q)]
    Gi = [O.g_source(i, phi, rho, u, dp, F) for i in range(O.Q)]

    def first(vals, a):
        return sum(O.C[i][a] * vals[i] for i in range(O.Q))

    close = lambda x, y: torch.allclose(x, y, rtol=1e-12, atol=1e-15)
    assert close(sum(feq), p)
    assert close(sum(geq), phi)
    assert close(sum(Fi), O.CS2 * (sum(u[a] * dr[a] for a in range(3)) - rho * co.gamma * D))
    assert close(sum(Gi), torch.zeros_like(phi))
    for a in range(3):
        assert close(first(feq, a), O.CS2 * rho * u[a])
        assert close(first(geq, a), phi * u[a])
        assert close(first(Fi, a), O.CS2 * F[a])
        assert close(first(Gi, a), (phi / rho) * (F[a] - dp[a]))


def test_stencil_fourier_symbols_3d():
    """On a periodic lattice a plane wave exp(i k.x) is an eigenfunction of
    both stencils; their symbols, summed over brute3d's independent velocity
    table, are (1/c_s^2) sum_i w_i c_i i sin(k.c_i) and (2/c_s^2) sum_i w_i
    (cos(k.c_i) - 1); the Laplacian's is -|k|^2 (1 + O(k^2)) in every
    direction."""
    nx, ny, nz = 16, 12, 10
    x, y, z = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="xy")
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    for m in [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 2, 3), (3, 1, 2), (5, 4, 2)]:
        k = 2 * math.pi * np.array([m[0] / nx, m[1] / ny, m[2] / nz])
        psi = torch.tensor(np.exp(1j * (k[0] * x + k[1] * y + k[2] * z)))
        lap_sym = 2.0 / B.CS2 * sum(B.W[i] * (math.cos(float(np.dot(k, c))) - 1.0)
                                    for i, c in enumerate(B.VEL))
        grad_sym = [1.0 / B.CS2 * sum(B.W[i] * c[a] * 1j * math.sin(float(np.dot(k, c)))
                                      for i, c in enumerate(B.VEL)) for a in range(3)]
        lp = O.lap(psi, O.PERIODIC)
        assert torch.allclose(lp, lap_sym * psi, atol=1e-12)
        gr = O.grad(psi, O.PERIODIC)
        for a in range(3):
            assert torch.allclose(gr[a], grad_sym[a] * psi, atol=1e-12)
    # isotropy of the leading term on a long lattice
    n = 200
    for dirn in [(1, 0, 0), (1, 1, 0), (1, 1, 1), (2, 1, 0)]:
        k = 2 * math.pi / n * np.array(dirn, dtype=float)
        sym = 2.0 / B.CS2 * sum(B.W[i] * (math.cos(float(np.dot(k, c))) - 1.0)
                                for i, c in enumerate(B.VEL))
        assert sym == pytest.approx(-np.dot(k, k), rel=3e-3)


def _random_state(pb, seed):
    f, g = wl.random_state3d(pb.nx, pb.ny, pb.nz, seed=seed)
    return torch.tensor(f), torch.tensor(g)


def _small(bc, g=(0.0, 0.0, 0.0)):
    return wl.droplet3d(6).with_(nx=6, ny=5, nz=7, bc=bc, gx=g[0], gy=g[1], gz=g[2],
                                 rho_ref=0.5)


@pytest.mark.parametrize("bc", [wl.PERIODIC, wl.WALLS_Z])
def test_mass_conservation_3d(bc):
    pb = _small(bc, (1e-4, 0.0, -2e-4))
    co = _co(pb)
    f, g = _random_state(pb, 3)
    m0 = O.mass(f, g, co)
    f, g = O.run(None, co, 5, state=(f, g))
    m1 = O.mass(f, g, co)
    assert m1[0] == pytest.approx(m0[0], rel=1e-14)
    assert m1[1] == pytest.approx(m0[1], rel=1e-14)


def test_mass_momentum_of_uniform_moving_state_3d():
    """rho u = sum_i c_i f_i + c_s^2 F / 2: a uniform state with
    f = f^eq(p, rho, u) - F_i / 2 and only a body force must report
    sum rho u = N rho u for the chosen u (a velocity without the half-force
    term misses by N F / 2, here ~10 % of rho u)."""
    pb = _small(wl.PERIODIC, (3e-3, -2e-3, -4e-3)).with_(rho_ref=1.0)
    co = _co(pb)
    shape = (pb.nz, pb.ny, pb.nx)
    n = pb.nx * pb.ny * pb.nz
    phi, u0 = 0.3, (0.01, -0.015, -0.02)
    ph = torch.full(shape, phi, dtype=torch.float64)
    rho = O.density(ph, co)
    mu = O.chemical_potential(ph, co)
    u = tuple(torch.full(shape, a, dtype=torch.float64) for a in u0)
    zero = torch.zeros(shape, dtype=torch.float64)
    F = tuple((rho - co.rho_ref) * a for a in (co.gx, co.gy, co.gz))
    f = torch.stack([O.f_equilibrium(i, zero, rho, u)
                     - 0.5 * O.f_source(i, u, F, (zero, zero, zero), rho, zero, co)
                     for i in range(O.Q)])
    g = torch.stack([O.g_equilibrium(i, ph, mu, u, co) for i in range(O.Q)])
    m = O.mass(f, g, co)
    r = float(rho[0, 0, 0])
    assert m[0] == pytest.approx(n * phi, rel=1e-14)
    assert m[1] == pytest.approx(n * r, rel=1e-14)
    for a in range(3):
        assert m[2 + a] == pytest.approx(n * r * u0[a], rel=1e-12)
        assert abs(0.5 * n * float(F[a][0, 0, 0])) > 0.05 * abs(m[2 + a])


def test_mass_momentum_balance_is_trapezoidal_3d():
    """Periodic box: the collision adds c_s^2 F to sum_i c_i f_i and
    streaming permutes populations, so the momentum total of
    rho u = (j + c_s^2 F / 2) / c_s^2 obeys
    sum rho u (t+1) - sum rho u (t) = (sum F(t) + sum F(t+1)) / 2 exactly,
    while F itself changes by ~1e-5 between the levels of a random state."""
    pb = _small(wl.PERIODIC, (1e-4, 0.0, -2e-4))
    co = _co(pb)
    f, g = _random_state(pb, 5)
    m0, M0 = O.mass(f, g, co), O.macroscopic(f, g, co)
    f1, g1 = O.step(f, g, co)
    m1, M1 = O.mass(f1, g1, co), O.macroscopic(f1, g1, co)
    for a in range(3):
        F0 = math.fsum(M0["F"][a].reshape(-1).tolist())
        F1 = math.fsum(M1["F"][a].reshape(-1).tolist())
        assert abs(F1 - F0) > 3e-6
        err = (m1[2 + a] - m0[2 + a]) - 0.5 * (F0 + F1)
        assert abs(err) < 1e-13 * max(abs(m0[2 + a]), 1.0)


def test_bulk_free_energy_3d():
    """psi = beta (phi - phi_A)^2 (phi - phi_B)^2: zero in both phases,
    beta / 16 at phi = 1/2 (p_0 = -beta / 16 there), derivative equal to the
    chemical-potential term, and along the tanh profile int 2 psi dz = sigma
    (equipartition of the interface free energy, Sec. II)."""
    pb = _small(wl.PERIODIC)
    co = _co(pb)
    for ph in (O.PHI_A, O.PHI_B):
        assert float(O.psi_bulk(torch.tensor(ph, dtype=torch.float64), co)) == 0.0
    half = torch.tensor(0.5, dtype=torch.float64)
    assert float(O.psi_bulk(half, co)) == pytest.approx(co.beta / 16, rel=1e-15)
    assert float(half * O.dpsi_dphi(half, co) - O.psi_bulk(half, co)) == \
        pytest.approx(-co.beta / 16, rel=1e-15)
    x = torch.linspace(-0.3, 1.3, 33, dtype=torch.float64).requires_grad_(True)
    (d,) = torch.autograd.grad(O.psi_bulk(x, co).sum(), x)
    torch.testing.assert_close(d, O.dpsi_dphi(x.detach(), co), rtol=1e-13, atol=1e-18)
    z = np.linspace(-5 * pb.W, 5 * pb.W, 8001)
    phi = 0.5 + 0.5 * np.tanh(2 * z / pb.W)
    psi = O.psi_bulk(torch.tensor(phi), co).numpy()
    assert np.trapezoid(2 * psi, z) == pytest.approx(pb.sigma, rel=1e-6)


def test_uniform_state_is_fixed_point_3d():
    pb = _small(wl.PERIODIC)
    co = _co(pb)
    phi0 = np.full((pb.nz, pb.ny, pb.nx), 0.37)
    f, g = O.initial_state(phi0, co)
    f1, g1 = O.run(None, co, 3, state=(f, g))
    # f stays 0; g moves only by the rounding of phi = sum g (a few ulp of 0.37)
    assert float((f1 - f).abs().max()) <= 1e-16
    assert float((g1 - g).abs().max()) <= 2e-15


def test_translation_is_bitwise_3d():
    pb = _small(wl.PERIODIC, (1e-4, 2e-4, -1e-4))
    co = _co(pb)
    f, g = _random_state(pb, 4)
    a = O.run(None, co, 3, state=(f, g))
    sh = (2, 1, 3)
    b = O.run(None, co, 3, state=(torch.roll(f, sh, dims=(1, 2, 3)),
                                 torch.roll(g, sh, dims=(1, 2, 3))))
    assert torch.equal(torch.roll(a[0], sh, dims=(1, 2, 3)), b[0])
    assert torch.equal(torch.roll(a[1], sh, dims=(1, 2, 3)), b[1])


def test_wall_stencils_equal_mirror_doubled_periodic_3d():
    """The mirrored ghost planes at walls are the periodic stencils on the
    field doubled by reflection about z = nz - 1/2 (an arbitrary field)."""
    rng = np.random.default_rng(8)
    v = torch.tensor(rng.standard_normal((7, 5, 6)))
    dbl = torch.cat([v, torch.flip(v, dims=(0,))], dim=0)
    assert torch.allclose(O.lap(v, O.WALLS_Z), O.lap(dbl, O.PERIODIC)[:7], atol=1e-14)
    for a, b in zip(O.grad(v, O.WALLS_Z), O.grad(dbl, O.PERIODIC)):
        assert torch.allclose(a, b[:7], atol=1e-14)


def test_walls_equal_mirror_doubled_periodic_for_layered_states_3d():
    """For a state that depends on z only (no in-plane force), half-way
    bounce-back coincides with specular reflection at the wall, so a walled
    lattice evolves exactly as the periodic lattice doubled by reflection in
    z: 30 steps from a layered initial interface."""
    pb = wl.droplet3d(4).with_(nx=4, ny=3, nz=10, bc=wl.WALLS_Z)
    z = np.arange(pb.nz, dtype=float)[:, None, None] * np.ones((1, pb.ny, pb.nx))
    phi0 = 0.5 + 0.45 * np.tanh(2.0 * (z - 3.7) / pb.W) * np.cos(z / 3.0)
    a = O.run(phi0, _co(pb), 30)
    pp = pb.with_(nz=2 * pb.nz, bc=wl.PERIODIC)
    mirror = [O.C.index((c[0], c[1], -c[2])) for c in O.C]
    b = O.run(np.concatenate([phi0, phi0[::-1]], axis=0), _co(pp), 30)
    assert float((a[0] - b[0][:, :pb.nz]).abs().max()) <= 1e-15
    assert float((a[1] - b[1][:, :pb.nz]).abs().max()) <= 1e-14
    # the upper half is the mirror image
    assert float((b[1][mirror][:, pb.nz:].flip(1) - b[1][:, :pb.nz]).abs().max()) <= 1e-14


@pytest.mark.parametrize("bc,g", [(wl.PERIODIC, (0.0, 0.0, 0.0)),
                                  (wl.WALLS_Z, (1e-4, -5e-5, -2e-4))])
def test_brute_force_equals_oracle_3d(bc, g):
    """tests/brute3d.py (plain floats, push streaming, its own velocity
    order) and the oracle agree over 3 steps on a 4 x 3 x 5 lattice."""
    pb = wl.droplet3d(4).with_(nx=4, ny=3, nz=5, bc=bc, gx=g[0], gy=g[1], gz=g[2],
                               rho_ref=0.55)
    co = _co(pb)
    f, g0 = _random_state(pb, 9)
    k = B.params(pb.rho_A, pb.rho_B, pb.sigma, pb.W, pb.M, pb.tau_f, pb.tau_g, g=g,
                 rho_ref=0.55, walls=bc == wl.WALLS_Z)
    perm = [O.C.index(c) for c in B.VEL]          # brute index -> oracle index
    bf = [f[perm[i]].tolist() for i in range(len(B.VEL))]
    bg = [g0[perm[i]].tolist() for i in range(len(B.VEL))]
    fo, go = f, g0
    for _ in range(3):
        bf, bg = B.step(bf, bg, k)
        fo, go = O.step(fo, go, co)
    bft = torch.tensor(bf, dtype=torch.float64)
    bgt = torch.tensor(bg, dtype=torch.float64)
    for i in range(len(B.VEL)):
        assert float((bft[i] - fo[perm[i]]).abs().max()) <= 1e-13 * float(fo.abs().max())
        assert float((bgt[i] - go[perm[i]]).abs().max()) <= 1e-13


def test_laplace_law_3d():
    """Spherical droplet R = 8 in a 32^3 periodic box (density ratio 10,
    sigma = 0.01, W = 4) after 800 steps: Delta P R / (2 sigma) within 8 %
    (the interface width W/R = 1/2 biases the small droplet; the 2-D check
    uses R = 16)."""
    pb = wl.droplet3d(32, 8.0)
    co = _co(pb)
    with torch.no_grad():
        f, g = O.run(wl.phi0_3d(pb), co, 800)
        dP = O.laplace_pressure(f, g, co)
    ratio = dP * pb.meta["R"] / (2.0 * pb.sigma)
    print("3-D Laplace: Delta P R / (2 sigma) =", ratio)
    assert ratio == pytest.approx(1.0, rel=0.08)


# ------------------------------------------------------------ TRT variant

def _trt_state():
    pb = wl.droplet3d().with_(nx=10, ny=8, nz=6, bc=O.WALLS_Z, gz=-2e-5, rho_ref=0.55,
                              tau_f=0.9)
    f, g = wl.random_state3d(10, 8, 6, seed=3)
    return pb, torch.as_tensor(f), torch.as_tensor(g)


def test_trt_3d_bgk_limit():
    """tau_- = tau_f (magic parameter (tau_f - 1/2)^2) is the BGK step."""
    pb, f, g = _trt_state()
    bgk = O.step(f, g, _co(pb))
    trt = O.step(f, g, _co(pb, trt_magic=(pb.tau_f - 0.5) ** 2))
    assert float((trt[0] - bgk[0]).abs().max() / bgk[0].abs().max()) < 1e-14
    assert torch.equal(trt[1], bgk[1])


@pytest.mark.parametrize("magic", [3.0 / 16.0, 0.25, 1.0])
def test_trt_3d_collision_keeps_mass_and_momentum_change(magic):
    """Post-collision sum f_i and sum c_i f_i do not depend on tau_-:
    sum c_i f* = sum c_i f + c_s^2 F for any magic parameter."""
    pb, f, g = _trt_state()
    m = O.macroscopic(f, g, _co(pb))
    fb, _ = O.collide(f, g, m, _co(pb))
    ft, _ = O.collide(f, g, m, _co(pb, trt_magic=magic))
    scale = float(f.abs().sum(0).max())
    assert float((ft.sum(0) - fb.sum(0)).abs().max()) < 1e-15 * 19 * scale + 1e-18
    for a in range(3):
        c = torch.tensor([O.C[i][a] for i in range(O.Q)], dtype=torch.float64)[:, None, None, None]
        jt = (c * ft).sum(0)
        j = (c * f).sum(0)
        assert float((jt - (j + O.CS2 * m["F"][a])).abs().max()) < 1e-14 * 19 * scale + 1e-18
        assert float((jt - (c * fb).sum(0)).abs().max()) < 1e-14 * 19 * scale + 1e-18
    assert float((ft - fb).abs().max()) > 1e-8


def test_trt_3d_channel_flow_is_exact_at_magic_three_sixteenths():
    """Body-force channel between half-way bounce-back walls normal to z
    (single phase, tau_f = 2, 8 nodes across): the steady profile of the
    Navier-Stokes limit is the parabola u_x = g/(2 nu) (z + 1/2)(nz - 1/2 - z)
    with the walls half a node outside the end nodes. The TRT collision with
    magic parameter 3/16 places the bounce-back walls exactly there, so the
    lattice profile equals the parabola to round-off (Ginzburg, Verhaeghe and
    d'Humieres 2008); BGK at this tau_f misses it by a wall-slip error of
    order (tau_f - 1/2)^2 / nz^2."""
    nz, tau, gx = 8, 2.0, 1e-6
    nu = (tau - 0.5) / 3.0
    pb = wl.droplet3d().with_(nx=1, ny=1, nz=nz, tau_f=tau, bc=O.WALLS_Z, gx=gx, gy=0.0,
                              gz=0.0, rho_ref=0.0)
    z = np.arange(nz, dtype=float)
    exact = gx / (2 * nu) * (z + 0.5) * (nz - 0.5 - z)
    nsteps = int(40 * nz * nz / (math.pi ** 2 * nu))  # e^-40 of the slowest mode left
    err = {}
    for magic in (3.0 / 16.0, 0.0):
        co = _co(pb, trt_magic=magic)
        f, g = O.initial_state(torch.ones((nz, 1, 1), dtype=torch.float64), co)
        for _ in range(nsteps):
            f, g = O.step(f, g, co)
        ux = O.macroscopic(f, g, co)["u"][0][:, 0, 0].numpy()
        err[magic] = float(np.abs(ux - exact).max() / exact.max())
    assert err[3.0 / 16.0] < 1e-12
    assert err[0.0] > 1e-2
