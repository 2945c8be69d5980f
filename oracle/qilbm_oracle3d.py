"""CPU oracle for the three-dimensional form of the quasi-incompressible
phase-field lattice Boltzmann model.

TEST INFRASTRUCTURE, like ``qilbm_oracle``: the plain FP64 statement of one
coupled time step, written from Yang & Guo (Sec. II, Sec. III) with the D2Q9
lattice replaced by D3Q19 -- the paper states its scheme on D2Q9 and notes
that this is without loss of generality, so every term keeps its form with
three velocity components. Only the tests may import it; the library never
does. It shares no code, table or constant with the HIP implementation (nor
with the two-dimensional oracle).

Arrays: a scalar field has shape (nz, ny, nx) indexed [z, y, x]; a population
set has shape (19, nz, ny, nx). Lattice units dx = dt = 1.

Readings (beyond those of the two-dimensional oracle, which carry over):

* D3Q19: c_0 = 0; the six axis vectors (weight 1/18); the twelve vectors
  with two components +-1 (weight 1/36); rest weight 1/3; c_s^2 = 1/3.
* Isotropic central differences on the same stencil:
  grad psi = (1/c_s^2) sum_i w_i c_i psi(x + c_i),
  lap psi = (2/c_s^2) sum_i w_i (psi(x + c_i) - psi(x)).
* H_0 = phi - (1 - w_0) alpha mu with w_0 = 1/3, so sum_i H_i = phi.
* Walls (periodic in x and y): half-way bounce-back below plane z = 0 and
  above plane nz - 1; stencils see mirrored ghost planes.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

DTYPE = torch.float64

# D3Q19 velocity set: rest, the six face neighbours, the twelve edge
# neighbours.
C = ((0, 0, 0),
     (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
     (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
     (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
     (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1))
WEIGHT = tuple([1.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12)
OPPOSITE = tuple(C.index((-a, -b, -c)) for (a, b, c) in C)
Q = len(C)
CS2 = 1.0 / 3.0

PHI_A = 1.0
PHI_B = 0.0

PERIODIC = 0
WALLS_Z = 1


@dataclass
class Coefficients:
    """Model coefficients derived from the physical parameters (Sec. II-III),
    with phi_A = 1, phi_B = 0."""
    beta: float
    kappa: float
    lam: float
    alpha: float
    gamma: float
    rho_A: float
    rho_B: float
    drho_dphi: float
    tau_f: float
    tau_g: float
    gx: float
    gy: float
    gz: float
    rho_ref: float
    bc: int
    trt_magic: float = 0.0          # 0: BGK for f; > 0: TRT with this magic parameter


def coefficients(rho_A, rho_B, sigma, W, M, tau_f, tau_g, gx=0.0, gy=0.0, gz=0.0,
                 rho_ref=None, bc=PERIODIC, no_gamma=False, trt_magic=0.0) -> Coefficients:
    """beta = 12 sigma / W and kappa = 3 sigma W / 2 (the interface-width and
    surface-tension relations of Sec. II), lambda = M, alpha = lambda /
    (c_s^2 (tau_g - 1/2)) (Sec. III), gamma = rho_A / rho_B - 1."""
    return Coefficients(
        beta=12.0 * sigma / W, kappa=1.5 * sigma * W, lam=M,
        alpha=M / (CS2 * (tau_g - 0.5)),
        gamma=0.0 if no_gamma else rho_A / rho_B - 1.0,
        rho_A=rho_A, rho_B=rho_B, drho_dphi=(rho_A - rho_B) / (PHI_A - PHI_B),
        tau_f=tau_f, tau_g=tau_g, gx=gx, gy=gy, gz=gz,
        rho_ref=rho_A if rho_ref is None else rho_ref, bc=bc, trt_magic=float(trt_magic))


# ------------------------------------------------------------- stencils

def neighbour(psi, c, bc):
    """psi(x + c) at every node x (|c_a| <= 1): periodic in x and y; in z
    periodic, or the mirrored boundary plane beyond a wall."""
    cx, cy, cz = c
    out = torch.roll(psi, shifts=(-cy, -cx), dims=(1, 2))
    if cz == 0:
        return out
    if bc == PERIODIC:
        return torch.roll(out, shifts=-cz, dims=0)
    nz = psi.shape[0]
    if cz == 1:
        return torch.cat([out[1:], out[nz - 1:]], dim=0)
    return torch.cat([out[:1], out[:nz - 1]], dim=0)


def grad(psi, bc):
    """(1/c_s^2) sum_i w_i c_i psi(x + c_i), three components."""
    g = [torch.zeros_like(psi) for _ in range(3)]
    for i in range(1, Q):
        nb = neighbour(psi, C[i], bc)
        for a in range(3):
            if C[i][a]:
                g[a] = g[a] + WEIGHT[i] * C[i][a] * nb
    return tuple(ga / CS2 for ga in g)


def lap(psi, bc):
    """(2/c_s^2) sum_i w_i (psi(x + c_i) - psi(x))."""
    acc = torch.zeros_like(psi)
    for i in range(1, Q):
        acc = acc + WEIGHT[i] * (neighbour(psi, C[i], bc) - psi)
    return 2.0 * acc / CS2


# ----------------------------------------------------- free energy (Sec. II)

def psi_bulk(phi, co):
    """Double-well bulk free-energy density beta (phi - phi_A)^2 (phi - phi_B)^2."""
    return co.beta * (phi - PHI_A) ** 2 * (phi - PHI_B) ** 2


def dpsi_dphi(phi, co):
    """4 beta (phi - phi_A)(phi - phi_B)(phi - (phi_A + phi_B)/2)."""
    return 4.0 * co.beta * (phi - PHI_A) * (phi - PHI_B) * (phi - 0.5 * (PHI_A + PHI_B))


def chemical_potential(phi, co, lap_phi=None):
    """mu = d psi/d phi - kappa lap phi."""
    if lap_phi is None:
        lap_phi = lap(phi, co.bc)
    return dpsi_dphi(phi, co) - co.kappa * lap_phi


def density(phi, co):
    """rho = rho_B + (phi - phi_B) d rho/d phi (affine in phi, Sec. II)."""
    return co.rho_B + (phi - PHI_B) * co.drho_dphi


# --------------------------------------------- per-direction terms (Sec. III)

def _dot(c, v):
    return c[0] * v[0] + c[1] * v[1] + c[2] * v[2]


def s_fun(i, u):
    """s_i(u) = c_i.u / c_s^2 + uu:(c_i c_i - c_s^2 I) / (2 c_s^4)."""
    cu = _dot(C[i], u)
    return cu / CS2 + (cu * cu - CS2 * _dot(u, u)) / (2.0 * CS2 * CS2)


def f_equilibrium(i, p, rho, u):
    """f_i^eq = w_i [p + c_s^2 rho s_i(u)]."""
    return WEIGHT[i] * (p + CS2 * rho * s_fun(i, u))


def h_term(i, phi, mu, co):
    """H_0 = phi - (1 - w_0) alpha mu; H_i = w_i alpha mu (i != 0)."""
    if i == 0:
        return phi - (1.0 - WEIGHT[0]) * co.alpha * mu
    return WEIGHT[i] * co.alpha * mu


def g_equilibrium(i, phi, mu, u, co):
    """g_i^eq = H_i + w_i phi s_i(u)."""
    return h_term(i, phi, mu, co) + WEIGHT[i] * phi * s_fun(i, u)


def f_source(i, u, F, dr, rho, D, co):
    """F_i = (c_i - u).[w_i Gamma_i F + w_i s_i c_s^2 grad rho]
    - w_i c_s^2 rho gamma D, with Gamma_i = 1 + s_i and D = lambda lap mu."""
    w = WEIGHT[i]
    s = s_fun(i, u)
    gam = 1.0 + s
    acc = 0.0
    for a in range(3):
        acc = acc + (C[i][a] - u[a]) * (w * F[a] * gam + w * s * CS2 * dr[a])
    return acc - w * CS2 * rho * co.gamma * D


def g_source(i, phi, rho, u, dp, F):
    """G_i = -(phi / (c_s^2 rho)) (c_i - u).(grad p - F) w_i Gamma_i."""
    acc = 0.0
    for a in range(3):
        acc = acc + (C[i][a] - u[a]) * (dp[a] - F[a])
    return -(phi / (CS2 * rho)) * acc * WEIGHT[i] * (1.0 + s_fun(i, u))


# ------------------------------------------------------------- one step

def macroscopic(f, g, co):
    """Macroscopic quantities of one time level from the pre-collision
    populations (Sec. III moments, Sec. II relations)."""
    bc = co.bc
    # sums in direction order, element by element (a library reduction over
    # the direction axis may group its additions by position)
    phi = sum(g[i] for i in range(Q))
    S = sum(f[i] for i in range(Q))
    j = tuple(sum(C[i][a] * f[i] for i in range(Q)) for a in range(3))
    rho = density(phi, co)
    lap_phi = lap(phi, bc)
    gph = grad(phi, bc)
    dr = tuple(co.drho_dphi * ga for ga in gph)
    mu = chemical_potential(phi, co, lap_phi)
    gmu = grad(mu, bc)
    D = co.lam * lap(mu, bc)
    gvec = (co.gx, co.gy, co.gz)
    F = tuple(-phi * gmu[a] + (rho - co.rho_ref) * gvec[a] for a in range(3))
    # u = [sum c_i f_i + (dt/2) c_s^2 F] / (c_s^2 rho)
    u = tuple((j[a] + 0.5 * CS2 * F[a]) / (CS2 * rho) for a in range(3))
    # p = sum f_i + (dt/2) c_s^2 (u.grad rho - gamma rho D)
    p = S + 0.5 * CS2 * (_dot(u, dr) - co.gamma * rho * D)
    dp = grad(p, bc)
    return dict(phi=phi, rho=rho, mu=mu, u=u, p=p, F=F, dr=dr, D=D, dp=dp, j=j, S=S)


def collide(f, g, m, co):
    """BGK collisions with forcing: x_i* = x_i - (x_i - x_i^eq)/tau
    + (1 - 1/(2 tau)) X_i for both LBEs. With ``co.trt_magic`` > 0, f
    collides with two relaxation times instead: f, f^eq and F_i split into
    parts even and odd under c_i -> -c_i, the even part relaxed with tau_f,
    the odd part with tau_- = 1/2 + magic / (tau_f - 1/2), each source part
    with its own 1 - 1/(2 tau) (a variant beyond the paper, which uses
    BGK)."""
    kf = 1.0 - 0.5 / co.tau_f
    kg = 1.0 - 0.5 / co.tau_g
    fs, gs, feqs, Fs = [], [], [], []
    for i in range(Q):
        feq = f_equilibrium(i, m["p"], m["rho"], m["u"])
        Fi = f_source(i, m["u"], m["F"], m["dr"], m["rho"], m["D"], co)
        geq = g_equilibrium(i, m["phi"], m["mu"], m["u"], co)
        Gi = g_source(i, m["phi"], m["rho"], m["u"], m["dp"], m["F"])
        feqs.append(feq)
        Fs.append(Fi)
        fs.append(f[i] - (f[i] - feq) / co.tau_f + kf * Fi)
        gs.append(g[i] - (g[i] - geq) / co.tau_g + kg * Gi)
    if co.trt_magic > 0.0:
        tm = 0.5 + co.trt_magic / (co.tau_f - 0.5)
        fs = []
        for i in range(Q):
            o = OPPOSITE[i]
            fp, fm = 0.5 * (f[i] + f[o]), 0.5 * (f[i] - f[o])
            ep, em = 0.5 * (feqs[i] + feqs[o]), 0.5 * (feqs[i] - feqs[o])
            sp, sm = 0.5 * (Fs[i] + Fs[o]), 0.5 * (Fs[i] - Fs[o])
            fs.append(f[i] - (fp - ep) / co.tau_f - (fm - em) / tm
                      + kf * sp + (1.0 - 0.5 / tm) * sm)
    return torch.stack(fs), torch.stack(gs)


def stream(pop, bc):
    """pop_i(x + c_i) = pop_i*(x); periodic wrap, or at a wall the opposite
    post-collision population of the same node for a source beyond it."""
    nz = pop.shape[1]
    out = []
    for i in range(Q):
        cx, cy, cz = C[i]
        moved = torch.roll(pop[i], shifts=(cz, cy, cx), dims=(0, 1, 2))
        if bc == WALLS_Z and cz != 0:
            back = pop[OPPOSITE[i]]
            if cz == 1:      # plane 0 would come from plane -1
                moved = torch.cat([back[:1], moved[1:]], dim=0)
            else:            # plane nz-1 would come from plane nz
                moved = torch.cat([moved[:nz - 1], back[nz - 1:]], dim=0)
        out.append(moved)
    return torch.stack(out)


def step(f, g, co):
    """One coupled time step t -> t+1."""
    m = macroscopic(f, g, co)
    fs, gs = collide(f, g, m, co)
    return stream(fs, co.bc), stream(gs, co.bc)


def initial_state(phi0, co):
    """f = 0 (u = 0, p = 0) and g_i = H_i(phi0, mu0)."""
    phi0 = torch.as_tensor(phi0, dtype=DTYPE)
    mu0 = chemical_potential(phi0, co)
    g = torch.stack([h_term(i, phi0, mu0, co) for i in range(Q)])
    return torch.zeros_like(g), g


def run(phi0, co, nsteps, state=None):
    f, g = initial_state(phi0, co) if state is None else state
    for _ in range(int(nsteps)):
        f, g = step(f, g, co)
    return f, g


def mass(f, g, co):
    """Totals (sum phi, sum rho, sum rho u_x, sum rho u_y, sum rho u_z)."""
    m = macroscopic(f, g, co)
    rho = m["rho"]
    return (float(m["phi"].sum()), float(rho.sum()),
            *(float((rho * m["u"][a]).sum()) for a in range(3)))


def laplace_pressure(f, g, co):
    """Pressure jump across a droplet interface: the full pressure
    P = p_0 - kappa phi lap phi + kappa |grad phi|^2 / 2 + p, with the bulk
    pressure p_0 = phi psi' - psi, averaged inside (phi > 0.99) minus
    outside (phi < 0.01)."""
    m = macroscopic(f, g, co)
    phi = m["phi"]
    p0 = phi * dpsi_dphi(phi, co) - psi_bulk(phi, co)
    gph = grad(phi, co.bc)
    P = (p0 - co.kappa * phi * lap(phi, co.bc)
         + 0.5 * co.kappa * sum(ga * ga for ga in gph) + m["p"])
    return float(P[phi > 0.99].mean() - P[phi < 0.01].mean())
