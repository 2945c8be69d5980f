"""Brute-force second implementation of one coupled three-dimensional step,
for pinning the 3-D oracle on tiny lattices.

Written independently of ``oracle/``: plain Python floats, one node and one
direction at a time, explicit neighbour indices, push streaming, and its own
velocity table (every vector of {-1, 0, 1}^3 with at most two non-zero
components, in enumeration order, weight by length: 1/3, 1/18, 1/36). The
readings are those of the oracle (Gamma_i = 1 + s_i, isotropic central
stencils on the same vectors, same-time grad p, half-way bounce-back with
mirrored ghost planes in z).

State: nested lists ``f[i][z][y][x]`` in this module's own direction order;
``VEL`` maps an index to its vector.
"""
from __future__ import annotations

import itertools

VEL = [c for c in itertools.product((-1, 0, 1), repeat=3) if sum(a != 0 for a in c) <= 2]
W = [{0: 1.0 / 3.0, 1: 1.0 / 18.0, 2: 1.0 / 36.0}[sum(a * a for a in c)] for c in VEL]
BACK = [VEL.index(tuple(-a for a in c)) for c in VEL]
REST = VEL.index((0, 0, 0))
CS2 = 1.0 / 3.0


def params(rho_A, rho_B, sigma, Wd, M, tau_f, tau_g, g=(0.0, 0.0, 0.0), rho_ref=None,
           walls=False):
    return dict(beta=12.0 * sigma / Wd, kappa=1.5 * sigma * Wd, lam=M,
                alpha=M / (CS2 * (tau_g - 0.5)), gamma=rho_A / rho_B - 1.0,
                rho_A=rho_A, rho_B=rho_B, tau_f=tau_f, tau_g=tau_g, g=tuple(g),
                rho_ref=rho_A if rho_ref is None else rho_ref, walls=walls)


def _at(psi, x, y, z, shape, walls):
    nz, ny, nx = shape
    x %= nx
    y %= ny
    if walls:
        z = 0 if z < 0 else (nz - 1 if z >= nz else z)
    else:
        z %= nz
    return psi[z][y][x]


def _grad_lap(psi, x, y, z, shape, walls):
    gr = [0.0, 0.0, 0.0]
    lp = 0.0
    c0 = psi[z][y][x]
    for i, c in enumerate(VEL):
        if i == REST:
            continue
        v = _at(psi, x + c[0], y + c[1], z + c[2], shape, walls)
        for a in range(3):
            gr[a] += W[i] * c[a] * v
        lp += W[i] * (v - c0)
    return [ga / CS2 for ga in gr], 2.0 * lp / CS2


def _field(shape):
    nz, ny, nx = shape
    return [[[0.0] * nx for _ in range(ny)] for _ in range(nz)]


def _nodes(shape):
    nz, ny, nx = shape
    return itertools.product(range(nz), range(ny), range(nx))


def step(f, g, k):
    """One coupled time step; returns new (f, g)."""
    shape = (len(f[0]), len(f[0][0]), len(f[0][0][0]))
    nz = shape[0]
    wl = k["walls"]
    q = len(VEL)
    phi, S = _field(shape), _field(shape)
    j = [_field(shape) for _ in range(3)]
    for z, y, x in _nodes(shape):
        phi[z][y][x] = sum(g[i][z][y][x] for i in range(q))
        S[z][y][x] = sum(f[i][z][y][x] for i in range(q))
        for a in range(3):
            j[a][z][y][x] = sum(VEL[i][a] * f[i][z][y][x] for i in range(q))
    drho = k["rho_A"] - k["rho_B"]
    mu = _field(shape)
    for z, y, x in _nodes(shape):
        ph = phi[z][y][x]
        _, lphi = _grad_lap(phi, x, y, z, shape, wl)
        mu[z][y][x] = 4.0 * k["beta"] * ph * (ph - 1.0) * (ph - 0.5) - k["kappa"] * lphi
    node = {}
    p = _field(shape)
    for z, y, x in _nodes(shape):
        ph = phi[z][y][x]
        rho = k["rho_B"] + drho * ph
        gph, _ = _grad_lap(phi, x, y, z, shape, wl)
        gmu, lmu = _grad_lap(mu, x, y, z, shape, wl)
        F = [-ph * gmu[a] + (rho - k["rho_ref"]) * k["g"][a] for a in range(3)]
        u = [(j[a][z][y][x] + 0.5 * CS2 * F[a]) / (CS2 * rho) for a in range(3)]
        D = k["lam"] * lmu
        dr = [drho * gph[a] for a in range(3)]
        p[z][y][x] = S[z][y][x] + 0.5 * CS2 * (sum(u[a] * dr[a] for a in range(3))
                                               - k["gamma"] * rho * D)
        node[(z, y, x)] = (ph, rho, mu[z][y][x], F, u, D, dr)
    fo = [_field(shape) for _ in range(q)]
    go = [_field(shape) for _ in range(q)]
    af = 1.0 - 0.5 / k["tau_f"]
    ag = 1.0 - 0.5 / k["tau_g"]
    for z, y, x in _nodes(shape):
        ph, rho, m, F, u, D, dr = node[(z, y, x)]
        dp, _ = _grad_lap(p, x, y, z, shape, wl)
        usq = sum(a * a for a in u)
        for i, c in enumerate(VEL):
            cu = sum(c[a] * u[a] for a in range(3))
            s = cu / CS2 + (cu * cu - CS2 * usq) / (2.0 * CS2 * CS2)
            gam = 1.0 + s
            feq = W[i] * (p[z][y][x] + CS2 * rho * s)
            Fi = sum((c[a] - u[a]) * W[i] * (gam * F[a] + s * CS2 * dr[a]) for a in range(3)) \
                - W[i] * CS2 * rho * k["gamma"] * D
            H = ph - (1.0 - W[REST]) * k["alpha"] * m if i == REST else W[i] * k["alpha"] * m
            geq = H + W[i] * ph * s
            Gi = -(ph / (CS2 * rho)) * sum((c[a] - u[a]) * (dp[a] - F[a]) for a in range(3)) \
                * W[i] * gam
            fs = f[i][z][y][x] - (f[i][z][y][x] - feq) / k["tau_f"] + af * Fi
            gs = g[i][z][y][x] - (g[i][z][y][x] - geq) / k["tau_g"] + ag * Gi
            tz = z + c[2]
            if wl and (tz < 0 or tz >= nz):
                fo[BACK[i]][z][y][x] = fs
                go[BACK[i]][z][y][x] = gs
            else:
                ty, tx = (y + c[1]) % shape[1], (x + c[0]) % shape[2]
                fo[i][tz % nz][ty][tx] = fs
                go[i][tz % nz][ty][tx] = gs
    return fo, go
