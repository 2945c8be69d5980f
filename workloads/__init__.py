"""Seeded synthetic inputs for the quasi-incompressible phase-field LBE.

This module is shared by the tests, the benchmark and the smoke check. It holds
only problem definitions: the raw physical parameters with which a problem is
stated (densities of the two fluids, surface tension sigma, interface width W,
mobility M, relaxation times, gravity, boundary kind) and the initial
order-parameter field phi0 on the lattice. It contains none of the scheme's
arithmetic: no free-energy coefficients, chemical potential, equilibria,
sources or moments. Each side (the CPU oracle and the HIP library) derives
everything else from these raw numbers itself.

Conventions: arrays are float64 numpy arrays of shape (ny, nx) indexed
[y, x]; node (x, y) has integer coordinates; phi_A = 1 marks fluid A and
phi_B = 0 fluid B, as in every test of the paper (Sec. IV).

Problem sets:

* ``droplet64``  -- static droplet, 64x64 periodic, R = 16, W = 4, density
  ratio 10, sigma = 0.01, M = 0.1, tau_f = tau_g = 0.8 (Laplace-law check).
* ``rt256`` / ``rt2048`` -- Rayleigh-Taylor instability between bounce-back
  walls, Atwood 0.5, sqrt(gL) = 0.04, Re = 3000, Pe = 1000 with
  Re = sqrt(gL) L / nu and Pe = sqrt(gL) L / M (nu = c_s^2 (tau_f - 1/2),
  Sec. III), interface ny/2 + 0.1 nx cos(2 pi x / nx), W = 4; the larger one
  keeps the Bond number Delta_rho g L^2 / sigma of the smaller one.
* ``droplets512`` -- two droplets with radii U[40, 80] and non-overlapping
  centres drawn from a seed, 512x512 periodic (gradient workload), and a
  32x32 copy for finite-difference checks.
* ``bubble4096`` -- rising bubble between walls, R = 256 at (2048, 1536),
  W = 5, Eo = 10 and Mo = 1e-3 closed with sigma = 0.01.
* ``flat_interface`` -- Sec. IV.A: 10x100, fluid A in 25 <= y <= 75.
* ``laplace_droplet`` -- Sec. IV.B / Table 1: 100x100, R in [20, 40].
* ``phase_separation`` -- Sec. IV.D: 100x100 perturbed mixture.
* ``random_state`` -- arbitrary non-equilibrium populations for one-step
  checks.
* ``Problem3`` sets (D3Q19 form): ``droplet3d`` (static droplet in a
  periodic cube, Laplace check), ``rt3d`` (Rayleigh-Taylor between walls in
  z with the two-dimensional problem's settings), ``random_state3d``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

PERIODIC = 0
WALLS_Y = 1

FP64 = 0
FP32 = 1
FP16_STORE = 2


@dataclass(frozen=True)
class Problem:
    """Raw parameters of one lattice problem, as the paper states a problem.

    ``M`` is the mobility (lambda of the Cahn-Hilliard equation), ``gx, gy``
    the gravity vector of the body force (rho - rho_ref) * (gx, gy), and
    ``bc`` is PERIODIC (both axes) or WALLS_Y (periodic in x, bounce-back
    walls below row 0 and above row ny-1).
    """

    name: str
    nx: int
    ny: int
    rho_A: float
    rho_B: float
    sigma: float
    W: float
    M: float
    tau_f: float
    tau_g: float
    gx: float = 0.0
    gy: float = 0.0
    rho_ref: float | None = None
    bc: int = PERIODIC
    steps: int = 1
    meta: dict = field(default_factory=dict, compare=False)

    @property
    def ref_density(self) -> float:
        return self.rho_A if self.rho_ref is None else self.rho_ref

    def with_(self, **kw) -> "Problem":
        return replace(self, **kw)

    def as_dict(self) -> dict:
        return dict(nx=self.nx, ny=self.ny, rho_A=self.rho_A, rho_B=self.rho_B,
                    sigma=self.sigma, W=self.W, M=self.M, tau_f=self.tau_f,
                    tau_g=self.tau_g, gx=self.gx, gy=self.gy,
                    rho_ref=self.ref_density, bc=self.bc)


def _grid(nx: int, ny: int):
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64),
                       np.arange(nx, dtype=np.float64), indexing="ij")
    return x, y


def tanh_step(signed_distance: np.ndarray, W: float) -> np.ndarray:
    """Equilibrium profile 1/2 + 1/2 tanh(2 zeta / W) with phi_A = 1, phi_B = 0
    (Sec. II, equilibrium interface profile); zeta > 0 inside fluid A."""
    return 0.5 + 0.5 * np.tanh(2.0 * signed_distance / W)


# ---------------------------------------------------------------- problems

def droplet64() -> Problem:
    return Problem("droplet64", 64, 64, rho_A=1.0, rho_B=0.1, sigma=0.01, W=4.0,
                   M=0.1, tau_f=0.8, tau_g=0.8, steps=2000,
                   meta=dict(R=16.0, xc=32.0, yc=32.0))


def droplet_phi0(pb: Problem) -> np.ndarray:
    x, y = _grid(pb.nx, pb.ny)
    r = np.sqrt((x - pb.meta["xc"]) ** 2 + (y - pb.meta["yc"]) ** 2)
    return tanh_step(pb.meta["R"] - r, pb.W)


def _rt(name: str, nx: int, ny: int, sigma: float, steps: int) -> Problem:
    L = float(nx)
    U = 0.04                          # sqrt(g L)
    g = U * U / L
    nu = U * L / 3000.0               # Re = 3000
    M = U * L / 1000.0                # Pe = 1000
    return Problem(name, nx, ny, rho_A=1.0, rho_B=1.0 / 3.0, sigma=sigma, W=4.0,
                   M=M, tau_f=0.5 + 3.0 * nu, tau_g=1.0, gx=0.0, gy=-g,
                   bc=WALLS_Y, steps=steps,
                   meta=dict(h0=ny / 2.0, amp=0.1 * nx, U=U, L=L))


def rt256() -> Problem:
    return _rt("rt256", 256, 1024, sigma=5e-5, steps=20000)


def rt2048() -> Problem:
    # Bond number (rho_A - rho_B) g L^2 / sigma kept from rt256 -> sigma = 4e-4
    return _rt("rt2048", 2048, 8192, sigma=4e-4, steps=160000)


def rt_phi0(pb: Problem) -> np.ndarray:
    """Heavy fluid A (phi = 1) above the perturbed interface h(x)."""
    x, y = _grid(pb.nx, pb.ny)
    h = pb.meta["h0"] + pb.meta["amp"] * np.cos(2.0 * math.pi * x / pb.nx)
    return tanh_step(y - h, pb.W)


def bubble4096() -> Problem:
    sigma, D, drho = 0.01, 512.0, 0.9
    g = 10.0 * sigma / (drho * D * D)                               # Eo = 10
    mu_l = (1e-3 * 1.0 * sigma ** 3 / (g * drho)) ** 0.25           # Mo = 1e-3
    return Problem("bubble4096", 4096, 8192, rho_A=1.0, rho_B=0.1, sigma=sigma,
                   W=5.0, M=0.1, tau_f=0.5 + 3.0 * mu_l / 1.0, tau_g=0.8,
                   gy=-g, bc=WALLS_Y, steps=50000,
                   meta=dict(R=256.0, xc=2048.0, yc=1536.0))


def bubble_phi0(pb: Problem) -> np.ndarray:
    """Light bubble (fluid B, phi = 0) inside liquid A."""
    x, y = _grid(pb.nx, pb.ny)
    r = np.sqrt((x - pb.meta["xc"]) ** 2 + (y - pb.meta["yc"]) ** 2)
    return tanh_step(r - pb.meta["R"], pb.W)


def droplets512(small: bool = False, seed: int = 0) -> Problem:
    if small:
        return Problem("droplets32", 32, 32, rho_A=1.0, rho_B=0.1, sigma=1e-3,
                       W=4.0, M=0.05, tau_f=0.8, tau_g=0.8, steps=200,
                       meta=dict(seed=seed, rmin=4.0, rmax=6.0))
    return Problem("droplets512", 512, 512, rho_A=1.0, rho_B=0.1, sigma=1e-3,
                   W=4.0, M=0.05, tau_f=0.8, tau_g=0.8, steps=2000,
                   meta=dict(seed=seed, rmin=40.0, rmax=80.0, checkpoint=100))


def two_droplets_phi0(pb: Problem) -> np.ndarray:
    """Two droplets, radii uniform in [rmin, rmax], centres uniform on the
    periodic domain, redrawn until the minimum-image gap between the two
    circles is at least 2 W (numpy PCG64 stream from ``meta['seed']``)."""
    rng = np.random.default_rng(pb.meta["seed"])
    nx, ny, W = pb.nx, pb.ny, pb.W
    lo, hi = pb.meta["rmin"], pb.meta["rmax"]
    while True:
        R = lo + (hi - lo) * rng.random(2)
        c = rng.random((2, 2)) * np.array([nx, ny])
        d = np.abs(c[0] - c[1])
        d = np.minimum(d, np.array([nx, ny]) - d)
        if np.hypot(*d) >= R[0] + R[1] + 2.0 * W:
            break
    x, y = _grid(nx, ny)
    phi = np.zeros((ny, nx))
    for k in range(2):
        dx = np.abs(x - c[k, 0]); dx = np.minimum(dx, nx - dx)
        dy = np.abs(y - c[k, 1]); dy = np.minimum(dy, ny - dy)
        phi += tanh_step(R[k] - np.hypot(dx, dy), W)
    return phi


def flat_interface(Pe: float = 50.0, Cn: float = 4.0) -> Problem:
    """Sec. IV.A. Pe = U_c L_c / (lambda beta) with U_c = c and L_c = dx
    (lattice units), Cn = W / L_c. The mobility is passed through the
    product lambda*beta via meta['lambda_beta'] = 1/Pe; turning it into M
    needs beta(sigma, W), which is the scheme's own relation, so callers
    pass M explicitly via ``with_`` after deriving it on their side."""
    return Problem("flat_interface", 10, 100, rho_A=1.0, rho_B=0.2, sigma=1e-3,
                   W=Cn, M=float("nan"), tau_f=1.0, tau_g=1.0, steps=4000,
                   meta=dict(lambda_beta=1.0 / Pe, y1=25.0, y2=75.0))


def flat_interface_phi0(pb: Problem) -> np.ndarray:
    x, y = _grid(pb.nx, pb.ny)
    y1 = 2.0 * (y - pb.meta["y1"]) / pb.W
    y2 = 2.0 * (y - pb.meta["y2"]) / pb.W
    return np.where(y <= 50.0, 0.5 + 0.5 * np.tanh(y1), 0.5 - 0.5 * np.tanh(y2))


def laplace_droplet(R: float = 25.0, Pe: float = 200.0, Cn: float = 4.0,
                    n: int = 100) -> Problem:
    """Sec. IV.B / Table 1: n x n periodic, centred droplet of radius R.
    As for ``flat_interface`` the mobility comes as lambda*beta = 1/Pe."""
    return Problem("laplace_droplet", n, n, rho_A=1.0, rho_B=0.2, sigma=1e-3,
                   W=Cn, M=float("nan"), tau_f=1.0, tau_g=1.0, steps=6000,
                   meta=dict(R=R, xc=n / 2.0, yc=n / 2.0, lambda_beta=1.0 / Pe))


def phase_separation(lambda_beta: float = 0.02, W: float = 4.0,
                     rho_r: float = 2.0, n: int = 100) -> Problem:
    """Sec. IV.D: periodic n x n, rho_A = 1, rho_B = rho_A / rho_r."""
    return Problem("phase_separation", n, n, rho_A=1.0, rho_B=1.0 / rho_r,
                   sigma=1e-3, W=W, M=float("nan"), tau_f=1.0, tau_g=1.0,
                   steps=20000, meta=dict(lambda_beta=lambda_beta))


def phase_separation_phi0(pb: Problem) -> np.ndarray:
    x, y = _grid(pb.nx, pb.ny)
    return 0.5 * (1.0 + 0.1 * np.sin(4.0 * math.pi * x / pb.nx)
                  * np.cos(4.0 * math.pi * y / pb.ny))


PHI0 = {
    "droplet64": droplet_phi0,
    "laplace_droplet": droplet_phi0,
    "rt256": rt_phi0,
    "rt2048": rt_phi0,
    "bubble4096": bubble_phi0,
    "droplets512": two_droplets_phi0,
    "droplets32": two_droplets_phi0,
    "flat_interface": flat_interface_phi0,
    "phase_separation": phase_separation_phi0,
}


def phi0(pb: Problem) -> np.ndarray:
    return np.ascontiguousarray(PHI0[pb.name](pb), dtype=np.float64)


def random_phi(nx: int, ny: int, seed: int, lo: float = 0.05,
               hi: float = 0.95) -> np.ndarray:
    """Smooth random order-parameter field in [lo, hi]: a few random Fourier
    modes, so that the stencils see O(1) gradients without aliasing."""
    rng = np.random.default_rng(seed)
    x, y = _grid(nx, ny)
    acc = np.zeros((ny, nx))
    for _ in range(6):
        kx, ky = rng.integers(0, 4, size=2)
        ph = rng.random() * 2.0 * math.pi
        acc += rng.standard_normal() * np.cos(2 * math.pi * (kx * x / nx + ky * y / ny) + ph)
    acc -= acc.min()
    acc /= max(acc.max(), 1e-300)
    return lo + (hi - lo) * acc


def random_state(nx: int, ny: int, seed: int, amp_f: float = 1e-3,
                 amp_g: float = 2e-3):
    """Arbitrary pre-collision populations (f, g) of shape (9, ny, nx): g_0
    carries a smooth field in [0.05, 0.95], every other slot a small uniform
    random deviation. Useful for one-step comparisons far from equilibrium;
    the total order parameter stays inside (0, 1) so densities are positive."""
    rng = np.random.default_rng(seed + 1000003)
    g = amp_g * (2.0 * rng.random((9, ny, nx)) - 1.0)
    g[0] += random_phi(nx, ny, seed)
    f = amp_f * (2.0 * rng.random((9, ny, nx)) - 1.0)
    return np.ascontiguousarray(f), np.ascontiguousarray(g)


def mobility_from_lambda_beta(lambda_beta: float, beta: float) -> float:
    """M = (lambda beta) / beta; beta must come from the caller's own
    free-energy coefficients."""
    return lambda_beta / beta


# ------------------------------------------------------------ three dimensions
# Problems of the D3Q19 form of the scheme. Arrays are float64 numpy arrays of
# shape (nz, ny, nx) indexed [z, y, x]; population sets (19, nz, ny, nx), slot
# 0 the rest population.

WALLS_Z = 1


@dataclass(frozen=True)
class Problem3:
    """Raw parameters of one three-dimensional lattice problem. ``bc`` is
    PERIODIC (all axes) or WALLS_Z (periodic in x and y, bounce-back walls
    below plane z = 0 and above plane nz - 1); gravity (gx, gy, gz)."""

    name: str
    nx: int
    ny: int
    nz: int
    rho_A: float
    rho_B: float
    sigma: float
    W: float
    M: float
    tau_f: float
    tau_g: float
    gx: float = 0.0
    gy: float = 0.0
    gz: float = 0.0
    rho_ref: float | None = None
    bc: int = PERIODIC
    meta: dict = field(default_factory=dict, compare=False)

    @property
    def ref_density(self) -> float:
        return self.rho_A if self.rho_ref is None else self.rho_ref

    def with_(self, **kw) -> "Problem3":
        return replace(self, **kw)

    def as_dict(self) -> dict:
        return dict(nx=self.nx, ny=self.ny, nz=self.nz, rho_A=self.rho_A, rho_B=self.rho_B,
                    sigma=self.sigma, W=self.W, M=self.M, tau_f=self.tau_f,
                    tau_g=self.tau_g, gx=self.gx, gy=self.gy, gz=self.gz,
                    rho_ref=self.ref_density, bc=self.bc)


def _grid3(nx: int, ny: int, nz: int):
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    return x, y, z


def droplet3d(n: int = 32, R: float = 8.0) -> Problem3:
    """Static droplet in a periodic cube (the three-dimensional Laplace
    check, Delta P = 2 sigma / R): density ratio 10, sigma = 0.01, W = 4,
    M = 0.1, tau_f = tau_g = 0.8, centred."""
    return Problem3("droplet3d", n, n, n, rho_A=1.0, rho_B=0.1, sigma=0.01, W=4.0, M=0.1,
                    tau_f=0.8, tau_g=0.8, meta=dict(R=R, xc=n / 2, yc=n / 2, zc=n / 2))


def rt3d(nx: int = 256, nz: int = 256) -> Problem3:
    """Rayleigh-Taylor instability in a box, walls in z: the two-dimensional
    problem's settings (Atwood 0.5, sqrt(g L) = 0.04, Re = 3000, Pe = 1000,
    W = 4, L = nx) with a doubly periodic cosine perturbation
    nz/2 + 0.05 nx (cos 2 pi x / nx + cos 2 pi y / nx)."""
    L = float(nx)
    U = 0.04
    g = U * U / L
    nu = U * L / 3000.0
    M = U * L / 1000.0
    return Problem3("rt3d", nx, nx, nz, rho_A=3.0, rho_B=1.0, sigma=5e-5 * (L / 256.0) ** 2,
                    W=4.0, M=M, tau_f=3.0 * nu + 0.5, tau_g=1.0, gz=-g, rho_ref=2.0,
                    bc=WALLS_Z)


def phi0_3d(pb: Problem3) -> np.ndarray:
    x, y, z = _grid3(pb.nx, pb.ny, pb.nz)
    if pb.name == "droplet3d":
        r = np.sqrt((x - pb.meta["xc"]) ** 2 + (y - pb.meta["yc"]) ** 2
                    + (z - pb.meta["zc"]) ** 2)
        return np.ascontiguousarray(tanh_step(pb.meta["R"] - r, pb.W))
    if pb.name == "rt3d":
        h = pb.nz / 2 + 0.05 * pb.nx * (np.cos(2 * math.pi * x / pb.nx)
                                         + np.cos(2 * math.pi * y / pb.ny))
        return np.ascontiguousarray(tanh_step(z - h, pb.W))
    raise KeyError(pb.name)


def random_phi3d(nx: int, ny: int, nz: int, seed: int, lo: float = 0.05,
                 hi: float = 0.95) -> np.ndarray:
    """Smooth random order parameter in [lo, hi] (a few random Fourier modes)."""
    rng = np.random.default_rng(seed)
    x, y, z = _grid3(nx, ny, nz)
    acc = np.zeros((nz, ny, nx))
    for _ in range(6):
        kx, ky, kz = rng.integers(0, 3, size=3)
        ph = rng.random() * 2.0 * math.pi
        acc += rng.standard_normal() * np.cos(
            2 * math.pi * (kx * x / nx + ky * y / ny + kz * z / nz) + ph)
    acc -= acc.min()
    acc /= max(acc.max(), 1e-300)
    return lo + (hi - lo) * acc


def random_state3d(nx: int, ny: int, nz: int, seed: int, amp_f: float = 1e-3,
                   amp_g: float = 2e-3):
    """Arbitrary pre-collision populations (f, g) of shape (19, nz, ny, nx):
    the rest slot of g carries a smooth field in [0.05, 0.95], every other
    slot a small uniform random deviation."""
    rng = np.random.default_rng(seed + 2000003)
    g = amp_g * (2.0 * rng.random((19, nz, ny, nx)) - 1.0)
    g[0] += random_phi3d(nx, ny, nz, seed)
    f = amp_f * (2.0 * rng.random((19, nz, ny, nx)) - 1.0)
    return np.ascontiguousarray(f), np.ascontiguousarray(g)
