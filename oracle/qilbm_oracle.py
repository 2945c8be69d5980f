"""CPU oracle for the quasi-incompressible phase-field lattice Boltzmann model.

TEST INFRASTRUCTURE. This module is the plain, slow FP64 statement of what
one coupled time step of Yang & Guo's model computes ("A lattice Boltzmann
method for binary fluids based on mass-conserved quasi-incompressible
phase-field theory", Sec. II and Sec. III). Only the tests, the smoke check
and the benchmark's CPU-baseline leg may import it; the library never does.
It shares no code, table or constant with the HIP implementation.

Everything is whole-lattice PyTorch CPU arithmetic in float64 with no
blocking, fusion or reordering beyond what the equations state, so it can be
read against the paper line by line. Because every operation is an ordinary
differentiable tensor op, ``torch.autograd`` through :func:`run` is also the
reference for gradients of a final-time loss with respect to sigma, M and the
initial order parameter.

Arrays: a scalar field has shape (ny, nx) indexed [y, x]; a population set
has shape (9, ny, nx). Lattice units dx = dt = 1 (Sec. III).

Readings of points the paper leaves open (each is pinned by a test):

* Gamma_i(u) in the source terms is 1 + s_i(u): the only choice for which the
  moment relations of the Appendix hold (sum F_i^(0) = c_s^2 u.grad rho,
  sum c_i F_i^(0) = c_s^2 F, sum G_i = 0, sum c_i G_i = (phi/rho)(F - grad p)).
* "Isotropic central scheme": grad psi = (1/c_s^2) sum_i w_i c_i psi(x + c_i)
  and lap psi = (2/c_s^2) sum_i w_i (psi(x + c_i) - psi(x)).
* div(lambda grad mu) = lambda lap mu (lambda constant); grad rho =
  (d rho/d phi) grad phi.
* The sources at time t use grad p from the complete pressure field at t.
* Initial state: u = 0, p = 0, so f = f^eq = 0 and g = g^eq = H_i(phi0, mu0).
* M is the mobility lambda; tau_g stays fixed and alpha = lambda/(c_s^2 (tau_g - 1/2)).
* phi_A = 1, phi_B = 0; body force (rho - rho_ref) * (gx, gy).
* Walls (periodic in x; bounce-back below row 0 and above row ny-1): a
  population whose source node lies beyond a wall is the opposite population
  of the same node after collision; stencils see mirrored ghost rows
  psi(x, -1) = psi(x, 0), psi(x, ny) = psi(x, ny - 1).

Variant beyond the paper (its collisions are BGK; it cites generalisations
with multiple relaxation times without specifying one): with
``trt_magic`` > 0 the flow LBE f collides with two relaxation times
(:func:`collide_f_trt`); g keeps the paper's BGK collision.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import torch

DTYPE = torch.float64

# D2Q9 (Sec. III): c_0 = 0, c_1..4 = (cos((i-1) pi/2), sin((i-1) pi/2)),
# c_5..8 = sqrt(2) (cos((2i-1) pi/4), sin((2i-1) pi/4)); w = 4/9, 1/9, 1/36.
C = ((0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1))
WEIGHT = (4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36)
OPPOSITE = (0, 3, 4, 1, 2, 7, 8, 5, 6)
CS2 = 1.0 / 3.0                     # c_s^2 = c^2 / 3

PHI_A = 1.0
PHI_B = 0.0

PERIODIC = 0
WALLS_Y = 1


@dataclass
class Coefficients:
    """Model coefficients derived from the problem parameters (Sec. II-III).

    ``sigma`` and ``M`` may be 0-d tensors requiring grad."""

    beta: object
    kappa: object
    lam: object
    alpha: object
    gamma: float
    drho_dphi: float
    rho_A: float
    rho_B: float
    tau_f: float
    tau_g: float
    gx: float
    gy: float
    rho_ref: float
    bc: int
    trt_magic: float = 0.0          # 0: BGK for f; > 0: TRT with this magic parameter


def coefficients(rho_A, rho_B, sigma, W, M, tau_f, tau_g, gx=0.0, gy=0.0,
                 rho_ref=None, bc=PERIODIC, no_gamma=False, trt_magic=0.0) -> Coefficients:
    """beta and kappa from W = sqrt(8 kappa / beta) / |phi_A - phi_B| and
    sigma = |phi_A - phi_B|^3 sqrt(2 kappa beta) / 6 (Sec. II); lambda = M and
    alpha from lambda = c_s^2 (tau_g - 1/2) alpha (Sec. III); gamma from the
    quasi-incompressible divergence constraint (Sec. II) with
    rho_r = rho_A / rho_B; d rho / d phi of the affine density (Sec. II).

    ``no_gamma`` sets gamma = 0, which removes exactly the two
    quasi-incompressible terms of the scheme (F_i^(1) and the gamma part of p):
    the same LBE written for the incompressible form div u = 0 (Sec. II
    compares the two forms through the extra term gamma phi div(lambda grad mu))."""
    dphi = PHI_A - PHI_B
    beta = 12.0 * sigma / (W * dphi ** 4)
    kappa = 1.5 * sigma * W / dphi ** 2
    lam = M
    alpha = lam / (CS2 * (tau_g - 0.5))
    rho_r = rho_A / rho_B
    gamma = 0.0 if no_gamma else (rho_r - 1.0) / (PHI_A - PHI_B * rho_r)
    drho = (rho_A - rho_B) / (PHI_A - PHI_B)
    return Coefficients(beta, kappa, lam, alpha, gamma, drho, rho_A, rho_B,
                        tau_f, tau_g, gx, gy, rho_A if rho_ref is None else rho_ref, bc,
                        float(trt_magic))


def coefficients_of(problem, sigma=None, M=None, no_gamma=False,
                    trt_magic=0.0) -> Coefficients:
    """Coefficients of a ``workloads.Problem`` (sigma and M overridable)."""
    return coefficients(problem.rho_A, problem.rho_B,
                        problem.sigma if sigma is None else sigma, problem.W,
                        problem.M if M is None else M, problem.tau_f,
                        problem.tau_g, problem.gx, problem.gy,
                        problem.ref_density, problem.bc, no_gamma=no_gamma,
                        trt_magic=trt_magic)


# ------------------------------------------------------------ stencils

def _padded_rows(psi, bc):
    """psi with one ghost row below and above: wrapped (periodic) or the
    mirrored boundary row (walls)."""
    if bc == PERIODIC:
        below, above = psi[-1:], psi[:1]
    else:
        below, above = psi[:1], psi[-1:]
    return torch.cat([below, psi, above], dim=0)


def neighbour(psi, cx, cy, bc):
    """psi(x + c) at every node x, for |cx|, |cy| <= 1."""
    ny = psi.shape[0]
    rows = _padded_rows(psi, bc)[1 + cy:1 + cy + ny]
    return torch.roll(rows, shifts=-cx, dims=1)


def grad(psi, bc):
    """Isotropic central gradient: (1/c_s^2) sum_{i=1..8} w_i c_i psi(x + c_i)."""
    gx = torch.zeros_like(psi)
    gy = torch.zeros_like(psi)
    for i in range(1, 9):
        cx, cy = C[i]
        nb = neighbour(psi, cx, cy, bc)
        gx = gx + WEIGHT[i] * cx * nb
        gy = gy + WEIGHT[i] * cy * nb
    return gx / CS2, gy / CS2


def lap(psi, bc):
    """Isotropic central Laplacian: (2/c_s^2) sum_{i=1..8} w_i (psi(x + c_i) - psi(x))."""
    acc = torch.zeros_like(psi)
    for i in range(1, 9):
        cx, cy = C[i]
        acc = acc + WEIGHT[i] * (neighbour(psi, cx, cy, bc) - psi)
    return 2.0 * acc / CS2


# ----------------------------------------------------- free energy (Sec. II)

def psi_bulk(phi, co):
    """Double-well bulk free-energy density beta (phi-phi_A)^2 (phi-phi_B)^2."""
    return co.beta * (phi - PHI_A) ** 2 * (phi - PHI_B) ** 2


def dpsi_dphi(phi, co):
    """d psi / d phi = 4 beta (phi - phi_A)(phi - phi_B)(phi - (phi_A + phi_B)/2)."""
    return 4.0 * co.beta * (phi - PHI_A) * (phi - PHI_B) * (phi - 0.5 * (PHI_A + PHI_B))


def chemical_potential(phi, co, lap_phi=None):
    """mu = d psi/d phi - kappa lap phi (Sec. II)."""
    if lap_phi is None:
        lap_phi = lap(phi, co.bc)
    return dpsi_dphi(phi, co) - co.kappa * lap_phi


def density(phi, co):
    """Affine density rho = rho_B + (phi - phi_B)(rho_A - rho_B)/(phi_A - phi_B) (Sec. II)."""
    return co.rho_B + (phi - PHI_B) * co.drho_dphi


# --------------------------------------------- per-direction terms (Sec. III)

def s_fun(i, ux, uy):
    """s_i(u) = c_i.u / c_s^2 + uu:(c_i c_i - c_s^2 I) / (2 c_s^4)."""
    cx, cy = C[i]
    cu = cx * ux + cy * uy
    return cu / CS2 + (cu * cu - CS2 * (ux * ux + uy * uy)) / (2.0 * CS2 * CS2)


def gamma_fun(i, ux, uy):
    """Gamma_i(u) = 1 + s_i(u) (see module docstring)."""
    return 1.0 + s_fun(i, ux, uy)


def f_equilibrium(i, p, rho, ux, uy):
    """f_i^eq = w_i [p + c_s^2 rho s_i(u)] (Sec. III)."""
    return WEIGHT[i] * (p + CS2 * rho * s_fun(i, ux, uy))


def h_term(i, phi, mu, co):
    """H_0 = phi - (1 - w_0) alpha mu, H_i = w_i alpha mu for i != 0 (Sec. III)."""
    if i == 0:
        return phi - (1.0 - WEIGHT[0]) * co.alpha * mu
    return WEIGHT[i] * co.alpha * mu


def g_equilibrium(i, phi, mu, ux, uy, co):
    """g_i^eq = H_i + w_i phi s_i(u) (Sec. III)."""
    return h_term(i, phi, mu, co) + WEIGHT[i] * phi * s_fun(i, ux, uy)


def f_source_0(i, ux, uy, Fx, Fy, drx, dry):
    """F_i^(0) = (c_i - u).[w_i Gamma_i F + w_i s_i c_s^2 grad rho] (Appendix)."""
    cx, cy = C[i]
    w = WEIGHT[i]
    s = s_fun(i, ux, uy)
    gam = gamma_fun(i, ux, uy)
    return ((cx - ux) * (w * Fx * gam + w * s * CS2 * drx)
            + (cy - uy) * (w * Fy * gam + w * s * CS2 * dry))


def f_source_1(i, rho, D, co):
    """F_i^(1) = -w_i c_s^2 rho gamma div(lambda grad mu), with D = lambda lap mu (Appendix)."""
    return -WEIGHT[i] * CS2 * rho * co.gamma * D


def f_source(i, ux, uy, Fx, Fy, drx, dry, rho, D, co):
    """F_i = F_i^(0) + F_i^(1) (Sec. III)."""
    return f_source_0(i, ux, uy, Fx, Fy, drx, dry) + f_source_1(i, rho, D, co)


def g_source(i, phi, rho, ux, uy, dpx, dpy, Fx, Fy):
    """G_i = -(phi / (c_s^2 rho)) (c_i - u).(grad p - F) w_i Gamma_i(u) (Sec. III)."""
    cx, cy = C[i]
    return (-(phi / (CS2 * rho)) * ((cx - ux) * (dpx - Fx) + (cy - uy) * (dpy - Fy))
            * WEIGHT[i] * gamma_fun(i, ux, uy))


def velocity(jx, jy, Fx, Fy, rho):
    """u = [sum_i c_i f_i + (dt/2) c_s^2 F] / (c_s^2 rho) (Sec. III)."""
    return (jx + 0.5 * CS2 * Fx) / (CS2 * rho), (jy + 0.5 * CS2 * Fy) / (CS2 * rho)


def pressure(S, ux, uy, drx, dry, rho, D, co):
    """p = sum_i f_i + (dt/2) c_s^2 (u.grad rho - gamma rho div(lambda grad mu)) (Sec. III)."""
    return S + 0.5 * CS2 * (ux * drx + uy * dry - co.gamma * rho * D)


# ------------------------------------------------------------- one step

def macroscopic(f, g, co):
    """All macroscopic quantities at one time level from the pre-collision
    populations f, g (Sec. III moments, Sec. II constitutive relations)."""
    bc = co.bc
    phi = g.sum(dim=0)
    S = f.sum(dim=0)
    jx = sum(C[i][0] * f[i] for i in range(9))
    jy = sum(C[i][1] * f[i] for i in range(9))
    rho = density(phi, co)
    lap_phi = lap(phi, bc)
    gphx, gphy = grad(phi, bc)
    drx, dry = co.drho_dphi * gphx, co.drho_dphi * gphy
    mu = chemical_potential(phi, co, lap_phi)
    gmux, gmuy = grad(mu, bc)
    D = co.lam * lap(mu, bc)
    # total force: surface tension -phi grad mu plus body force (Sec. II, IV.C)
    Fx = -phi * gmux + (rho - co.rho_ref) * co.gx
    Fy = -phi * gmuy + (rho - co.rho_ref) * co.gy
    ux, uy = velocity(jx, jy, Fx, Fy, rho)
    p = pressure(S, ux, uy, drx, dry, rho, D, co)
    dpx, dpy = grad(p, bc)
    return dict(phi=phi, rho=rho, mu=mu, ux=ux, uy=uy, p=p, Fx=Fx, Fy=Fy,
                drx=drx, dry=dry, D=D, dpx=dpx, dpy=dpy, jx=jx, jy=jy, S=S,
                lap_phi=lap_phi, gphx=gphx, gphy=gphy)


def collide(f, g, m, co):
    """BGK collisions with forcing (Sec. III, both LBEs):
    f_i* = f_i - (f_i - f_i^eq)/tau_f + (1 - 1/(2 tau_f)) F_i and likewise g.
    With ``co.trt_magic`` > 0, f collides by :func:`collide_f_trt` instead."""
    fs, gs = [], []
    kf = 1.0 - 0.5 / co.tau_f
    kg = 1.0 - 0.5 / co.tau_g
    feqs, Fs = [], []
    for i in range(9):
        feq = f_equilibrium(i, m["p"], m["rho"], m["ux"], m["uy"])
        Fi = f_source(i, m["ux"], m["uy"], m["Fx"], m["Fy"], m["drx"], m["dry"],
                      m["rho"], m["D"], co)
        geq = g_equilibrium(i, m["phi"], m["mu"], m["ux"], m["uy"], co)
        Gi = g_source(i, m["phi"], m["rho"], m["ux"], m["uy"], m["dpx"], m["dpy"],
                      m["Fx"], m["Fy"])
        feqs.append(feq)
        Fs.append(Fi)
        fs.append(f[i] - (f[i] - feq) / co.tau_f + kf * Fi)
        gs.append(g[i] - (g[i] - geq) / co.tau_g + kg * Gi)
    if co.trt_magic > 0.0:
        fs = collide_f_trt(f, feqs, Fs, co)
    return torch.stack(fs), torch.stack(gs)


def tau_minus(co):
    """Relaxation time of the odd part: the magic parameter is
    Lambda = (tau_f - 1/2)(tau_- - 1/2)."""
    return 0.5 + co.trt_magic / (co.tau_f - 0.5)


def collide_f_trt(f, feq, F, co):
    """Two-relaxation-time collision of f with forcing (Ginzburg, Verhaeghe
    and d'Humieres, 2008): populations, equilibria and sources are split into
    parts even and odd under c_i -> -c_i, x_i^(+-) = (x_i +- x_opp(i)) / 2;
    the even part relaxes with tau_f (it carries the viscous stress), the odd
    part with tau_- (:func:`tau_minus`), and each source part takes its own
    factor 1 - 1/(2 tau):
    f_i* = f_i - (f_i^+ - f_i^eq+)/tau_f - (f_i^- - f_i^eq-)/tau_-
           + (1 - 1/(2 tau_f)) F_i^+ + (1 - 1/(2 tau_-)) F_i^-.
    tau_- = tau_f (Lambda = (tau_f - 1/2)^2) is the BGK collision."""
    tm = tau_minus(co)
    out = []
    for i in range(9):
        o = OPPOSITE[i]
        fp, fm = 0.5 * (f[i] + f[o]), 0.5 * (f[i] - f[o])
        ep, em = 0.5 * (feq[i] + feq[o]), 0.5 * (feq[i] - feq[o])
        sp, sm = 0.5 * (F[i] + F[o]), 0.5 * (F[i] - F[o])
        out.append(f[i] - (fp - ep) / co.tau_f - (fm - em) / tm
                   + (1.0 - 0.5 / co.tau_f) * sp + (1.0 - 0.5 / tm) * sm)
    return out


def stream(pop, bc):
    """pop_i(x + c_i, t + 1) = pop_i*(x, t); periodic wrap. With walls a
    population whose source x - c_i lies beyond a wall is the bounced-back
    opposite population pop_opp(i)* of the same node."""
    ny = pop.shape[1]
    out = []
    for i in range(9):
        cx, cy = C[i]
        moved = torch.roll(pop[i], shifts=(cy, cx), dims=(0, 1))
        if bc == WALLS_Y and cy != 0:
            back = pop[OPPOSITE[i]]
            if cy == 1:      # row 0 would come from row -1
                moved = torch.cat([back[:1], moved[1:]], dim=0)
            else:            # row ny-1 would come from row ny
                moved = torch.cat([moved[:ny - 1], back[ny - 1:]], dim=0)
        out.append(moved)
    return torch.stack(out)


def step(f, g, co):
    """One coupled time step t -> t+1 of both LBEs (Sec. III)."""
    m = macroscopic(f, g, co)
    fs, gs = collide(f, g, m, co)
    return stream(fs, co.bc), stream(gs, co.bc)


def initial_state(phi0, co):
    """Pre-collision populations at t = 0: f = 0 (u = 0, p = 0) and
    g_i = H_i(phi0, mu0), so that sum_i g_i = phi0."""
    phi0 = torch.as_tensor(phi0)
    if not (phi0.is_floating_point() or phi0.is_complex()):
        phi0 = phi0.to(DTYPE)
    mu0 = chemical_potential(phi0, co)
    g = torch.stack([h_term(i, phi0, mu0, co) for i in range(9)])
    f = torch.zeros_like(g)
    return f, g


def run(phi0, co, nsteps, state=None):
    """Initial state from phi0 (or the given (f, g)) advanced by nsteps."""
    f, g = initial_state(phi0, co) if state is None else state
    for _ in range(int(nsteps)):
        f, g = step(f, g, co)
    return f, g


# ------------------------------------------------------------- outputs

def moments(f, g, co):
    """(phi, rho, ux, uy, p, mu) at the time level of the populations."""
    m = macroscopic(f, g, co)
    return tuple(m[k] for k in ("phi", "rho", "ux", "uy", "p", "mu"))


def _fsum(t):
    return math.fsum(t.detach().reshape(-1).tolist())


def mass(f, g, co):
    """(sum phi, sum rho, sum rho ux, sum rho uy) over the lattice, each a
    correctly rounded FP64 sum; rho u = (sum_i c_i f_i + c_s^2 F / 2) / c_s^2."""
    m = macroscopic(f, g, co)
    rux = m["rho"] * m["ux"]
    ruy = m["rho"] * m["uy"]
    return (_fsum(m["phi"]), _fsum(m["rho"]), _fsum(rux), _fsum(ruy))


def laplace_pressure(f, g, co):
    """P = p_0 - kappa phi lap phi + kappa |grad phi|^2 / 2 + p with
    p_0 = phi dpsi/dphi - psi (Sec. IV.B)."""
    m = macroscopic(f, g, co)
    phi = m["phi"]
    p0 = phi * dpsi_dphi(phi, co) - psi_bulk(phi, co)
    return (p0 - co.kappa * phi * m["lap_phi"]
            + 0.5 * co.kappa * (m["gphx"] ** 2 + m["gphy"] ** 2) + m["p"])


# ------------------------------------------------------------- gradients

def loss_and_gradients(phi0, problem, nsteps, loss_of_phi, sigma=None, M=None,
                       state=None):
    """L(phi_K) and dL/dsigma, dL/dM, dL/dphi0 by reverse-mode automatic
    differentiation through :func:`run`. sigma enters through beta and kappa
    (W fixed); M through lambda and alpha (tau_g fixed); phi0 through the
    initial state. ``loss_of_phi`` maps the final phi field to a 0-d tensor."""
    sig = torch.tensor(problem.sigma if sigma is None else sigma, dtype=DTYPE,
                       requires_grad=True)
    mob = torch.tensor(problem.M if M is None else M, dtype=DTYPE, requires_grad=True)
    p0 = torch.as_tensor(phi0, dtype=DTYPE).clone().requires_grad_(True)
    co = coefficients_of(problem, sigma=sig, M=mob)
    f, g = run(p0, co, nsteps, state=state)
    L = loss_of_phi(g.sum(dim=0))
    dsig, dmob, dphi0 = torch.autograd.grad(L, (sig, mob, p0))
    return float(L.detach()), float(dsig), float(dmob), dphi0


def step_vjp(f, g, problem, fbar, gbar):
    """Vector-Jacobian product of one step: given the cotangents (fbar, gbar)
    of the state at t+1, return those of the state at t and the parameter
    cotangents (sigma_bar, M_bar)."""
    sig = torch.tensor(problem.sigma, dtype=DTYPE, requires_grad=True)
    mob = torch.tensor(problem.M, dtype=DTYPE, requires_grad=True)
    f = torch.as_tensor(f, dtype=DTYPE).clone().requires_grad_(True)
    g = torch.as_tensor(g, dtype=DTYPE).clone().requires_grad_(True)
    co = coefficients_of(problem, sigma=sig, M=mob)
    f1, g1 = step(f, g, co)
    out = (f1 * torch.as_tensor(fbar, dtype=DTYPE)).sum() + \
          (g1 * torch.as_tensor(gbar, dtype=DTYPE)).sum()
    df, dg, dsig, dmob = torch.autograd.grad(out, (f, g, sig, mob))
    return df, dg, float(dsig), float(dmob)


def step_jvp(f, g, problem, df, dg, dsigma=0.0, dM=0.0):
    """Jacobian-vector product of one step by forward-mode differentiation
    (dual numbers, ``torch.func.jvp``): the tangent of the state at t+1 for a
    tangent (df, dg) of the state at t and (dsigma, dM) of the parameters.
    Independent of the reverse mode of :func:`step_vjp`, so the pair checks
    <J^T w, v> = <w, J v>."""
    def one(f, g, sig, mob):
        return step(f, g, coefficients_of(problem, sigma=sig, M=mob))
    t = lambda a: torch.as_tensor(a, dtype=DTYPE)
    _, (tf, tg) = torch.func.jvp(
        one, (t(f), t(g), t(problem.sigma), t(problem.M)),
        (t(df), t(dg), t(dsigma), t(dM)))
    return tf, tg


def loss_jvp(phi0, problem, nsteps, loss_of_phi, dphi0, dsigma=0.0, dM=0.0):
    """Directional derivative of L(phi_K) along (dphi0, dsigma, dM) by
    forward-mode differentiation through :func:`run`."""
    def L(p0, sig, mob):
        co = coefficients_of(problem, sigma=sig, M=mob)
        f, g = run(p0, co, nsteps)
        return loss_of_phi(g.sum(dim=0))
    t = lambda a: torch.as_tensor(a, dtype=DTYPE)
    _, dL = torch.func.jvp(L, (t(phi0), t(problem.sigma), t(problem.M)),
                           (t(dphi0), t(dsigma), t(dM)))
    return float(dL)
