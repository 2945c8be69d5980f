"""Sampled-window comparison of a full-size GPU run with the oracle.

A lattice too large for the oracle is checked on small windows: the oracle
steps a crop of the GPU's stored starting state that extends ``margin`` nodes
beyond the window on every side that is not a wall (k steps depend on nodes
within 4k: one pull plus the phi/mu/p stencils of radius 3 per step), and
the window of the oracle's result is compared with the same window of the
GPU's state after the run."""
import numpy as np
import torch

from oracle import qilbm_oracle as O


def rel(a, b):
    a = torch.as_tensor(a).cpu().double()
    b = torch.as_tensor(b).cpu().double()
    return float((a - b).abs().max() / b.abs().max().clamp_min(1e-300))


def compare_windows(pb, before, after, picks, nsteps, tol, trt_magic=0.0, size=12, margin=10):
    """before: (f, g) on the CPU, the stored state the GPU started from;
    after: (f, g) on any device after nsteps GPU steps; picks: (y0, x0)
    window corners (x wraps). Returns the worst (rel f, rel g)."""
    fa, ga = before
    fs, gs = after
    ny, nx = pb.ny, pb.nx
    assert margin >= 4 * nsteps
    worst = (0.0, 0.0)
    for y0, x0 in picks:
        h = w = size
        lo, hi = max(0, y0 - margin), min(ny, y0 + h + margin)
        rows = torch.arange(lo, hi)
        cols = torch.as_tensor(np.arange(x0 - margin, x0 + w + margin) % nx)
        # the crop keeps the problem's boundary kind; where its edges are not
        # the lattice's own walls they are artificial (walls or wrap), and the
        # compared nodes lie margin >= 4 * nsteps nodes inside them
        co = O.coefficients_of(pb.with_(nx=len(cols), ny=len(rows)), trt_magic=trt_magic)
        st = (fa[:, rows][:, :, cols], ga[:, rows][:, :, cols])
        with torch.no_grad():
            for _ in range(nsteps):
                st = O.step(*st, co)
        r0 = y0 - lo
        fr, gr = st[0][:, r0:r0 + h, margin:margin + w], st[1][:, r0:r0 + h, margin:margin + w]
        cc = cols[margin:margin + w].to(fs.device)
        fg = fs[:, y0:y0 + h][:, :, cc].cpu()
        gg = gs[:, y0:y0 + h][:, :, cc].cpu()
        ef, eg = rel(fg, fr), rel(gg, gr)
        print(f"  window y0={y0} x0={x0}: rel f {ef:.2e} g {eg:.2e}", flush=True)
        assert ef < tol[0] and eg < tol[1], (y0, x0, ef, eg)
        worst = (max(worst[0], ef), max(worst[1], eg))
    return worst
