"""Brute-force second implementation of one coupled step, for pinning the
oracle on tiny lattices.

Written independently of ``oracle/``: plain Python floats, one node and one
direction at a time, explicit neighbour indices, push streaming (the oracle
pulls with whole-array shifts), its own lattice table built from the
paper's closed-form velocity set (Sec. III). It follows the same readings of
the paper as the oracle (Gamma_i = 1 + s_i, isotropic central stencils,
same-time grad p, half-way bounce-back with mirrored stencil ghosts), so a
disagreement points at an indexing, sign or transposition mistake in one of
the two, not at a reading.

State: lists ``f[i][y][x]``, ``g[i][y][x]`` (pre-collision populations).
"""
from __future__ import annotations

import math

# D2Q9 from the closed form of Sec. III: c_0 = 0; c_1..4 on the axes at
# angles (i-1) pi/2; c_5..8 on the diagonals at angles (2i-1) pi/4 with
# length sqrt(2). Weights 4/9, 1/9, 1/36.
VEL = [(0, 0)]
for i in range(1, 5):
    a = (i - 1) * math.pi / 2
    VEL.append((round(math.cos(a)), round(math.sin(a))))
for i in range(5, 9):
    a = (2 * i - 1) * math.pi / 4
    VEL.append((round(math.sqrt(2) * math.cos(a)), round(math.sqrt(2) * math.sin(a))))
W = [4.0 / 9.0] + [1.0 / 9.0] * 4 + [1.0 / 36.0] * 4
BACK = [VEL.index((-cx, -cy)) for (cx, cy) in VEL]
CS2 = 1.0 / 3.0


def params(rho_A, rho_B, sigma, Wd, M, tau_f, tau_g, gx=0.0, gy=0.0, rho_ref=None,
           walls=False):
    """Derived coefficients with phi_A = 1, phi_B = 0 (Sec. II-III)."""
    return dict(beta=12.0 * sigma / Wd, kappa=1.5 * sigma * Wd, lam=M,
                alpha=M / (CS2 * (tau_g - 0.5)), gamma=rho_A / rho_B - 1.0,
                rho_A=rho_A, rho_B=rho_B, tau_f=tau_f, tau_g=tau_g, gx=gx, gy=gy,
                rho_ref=rho_A if rho_ref is None else rho_ref, walls=walls)


def _at(psi, x, y, nx, ny, walls):
    """psi at node (x, y) of the lattice extended by periodic x, and in y by
    periodic wrap or mirrored ghost rows at walls."""
    x %= nx
    if walls:
        y = 0 if y < 0 else (ny - 1 if y >= ny else y)
    else:
        y %= ny
    return psi[y][x]


def _grad_lap(psi, x, y, nx, ny, walls):
    gx = gy = lp = 0.0
    c = psi[y][x]
    for i in range(1, 9):
        cx, cy = VEL[i]
        v = _at(psi, x + cx, y + cy, nx, ny, walls)
        gx += W[i] * cx * v
        gy += W[i] * cy * v
        lp += W[i] * (v - c)
    return gx / CS2, gy / CS2, 2.0 * lp / CS2


def _field(ny, nx):
    return [[0.0] * nx for _ in range(ny)]


def step(f, g, k):
    """One coupled time step; returns new (f, g)."""
    ny, nx = len(f[0]), len(f[0][0])
    wl = k["walls"]
    phi, S, jx, jy = _field(ny, nx), _field(ny, nx), _field(ny, nx), _field(ny, nx)
    for y in range(ny):
        for x in range(nx):
            phi[y][x] = sum(g[i][y][x] for i in range(9))
            S[y][x] = sum(f[i][y][x] for i in range(9))
            jx[y][x] = sum(VEL[i][0] * f[i][y][x] for i in range(9))
            jy[y][x] = sum(VEL[i][1] * f[i][y][x] for i in range(9))
    drho = k["rho_A"] - k["rho_B"]
    mu = _field(ny, nx)
    for y in range(ny):
        for x in range(nx):
            ph = phi[y][x]
            _, _, lphi = _grad_lap(phi, x, y, nx, ny, wl)
            mu[y][x] = 4.0 * k["beta"] * ph * (ph - 1.0) * (ph - 0.5) - k["kappa"] * lphi
    node = [[None] * nx for _ in range(ny)]
    p = _field(ny, nx)
    for y in range(ny):
        for x in range(nx):
            ph = phi[y][x]
            rho = k["rho_B"] + drho * ph
            gpx, gpy, _ = _grad_lap(phi, x, y, nx, ny, wl)
            gmx, gmy, lmu = _grad_lap(mu, x, y, nx, ny, wl)
            Fx = -ph * gmx + (rho - k["rho_ref"]) * k["gx"]
            Fy = -ph * gmy + (rho - k["rho_ref"]) * k["gy"]
            ux = (jx[y][x] + 0.5 * CS2 * Fx) / (CS2 * rho)
            uy = (jy[y][x] + 0.5 * CS2 * Fy) / (CS2 * rho)
            D = k["lam"] * lmu
            rx, ry = drho * gpx, drho * gpy
            p[y][x] = S[y][x] + 0.5 * CS2 * (ux * rx + uy * ry - k["gamma"] * rho * D)
            node[y][x] = (ph, rho, mu[y][x], Fx, Fy, ux, uy, D, rx, ry)
    fo = [_field(ny, nx) for _ in range(9)]
    go = [_field(ny, nx) for _ in range(9)]
    af = 1.0 - 0.5 / k["tau_f"]
    ag = 1.0 - 0.5 / k["tau_g"]
    for y in range(ny):
        for x in range(nx):
            ph, rho, m, Fx, Fy, ux, uy, D, rx, ry = node[y][x]
            dpx, dpy, _ = _grad_lap(p, x, y, nx, ny, wl)
            for i in range(9):
                cx, cy = VEL[i]
                cu = cx * ux + cy * uy
                s = cu / CS2 + (cu * cu - CS2 * (ux * ux + uy * uy)) / (2.0 * CS2 * CS2)
                gam = 1.0 + s
                feq = W[i] * (p[y][x] + CS2 * rho * s)
                Fi = ((cx - ux) * W[i] * (gam * Fx + s * CS2 * rx)
                      + (cy - uy) * W[i] * (gam * Fy + s * CS2 * ry)
                      - W[i] * CS2 * rho * k["gamma"] * D)
                H = ph - (1.0 - W[0]) * k["alpha"] * m if i == 0 else W[i] * k["alpha"] * m
                geq = H + W[i] * ph * s
                Gi = -(ph / (CS2 * rho)) * ((cx - ux) * (dpx - Fx) + (cy - uy) * (dpy - Fy)) \
                    * W[i] * gam
                fs = f[i][y][x] - (f[i][y][x] - feq) / k["tau_f"] + af * Fi
                gs = g[i][y][x] - (g[i][y][x] - geq) / k["tau_g"] + ag * Gi
                # push to the neighbour, or back into this node (opposite
                # direction) when the neighbour lies beyond a wall
                ty = y + cy
                if wl and (ty < 0 or ty >= ny):
                    fo[BACK[i]][y][x] = fs
                    go[BACK[i]][y][x] = gs
                else:
                    fo[i][ty % ny][(x + cx) % nx] = fs
                    go[i][ty % ny][(x + cx) % nx] = gs
    return fo, go
