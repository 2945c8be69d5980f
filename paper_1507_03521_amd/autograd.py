"""Gradients of a final-time loss through the GPU lattice: a
``torch.autograd.Function`` whose backward runs the library's hand-written
adjoint step with checkpoint-and-recompute."""
from __future__ import annotations

import torch

from .lattice import Lattice


class PhaseFieldRun(torch.autograd.Function):
    """phi_K = run(phi0; sigma, M) for K steps. Differentiable in phi0,
    sigma and M.

    Forward keeps a raw snapshot of the state every ``checkpoint`` steps
    (including t = 0) and advances each segment with one library call.
    Backward walks the segments last to first: it restores the segment's
    snapshot, replays the segment with one call that also writes the records
    (the forward quantities phi, mu, p, S, j each adjoint step needs) -- the
    same launches as the forward segment, pairs of steps included -- and
    applies the adjoint step to the records in reverse time order. Memory:
    ceil(K / C) raw states plus C records (a record is a third of a raw
    state). With two steps per kernel pass, an even C keeps the launches of
    a run without checkpoints (pairs from even t), so the gradients do not
    depend on C bitwise; an odd C moves the pairs and changes only rounding.
    """

    @staticmethod
    def forward(ctx, phi0, sigma, M, params: dict, nsteps: int, checkpoint: int,
                precision: str = "fp64", flags: int = 0):
        p = dict(params)
        p["sigma"] = float(sigma)
        p["M"] = float(M)
        lat = Lattice(p, phi0.detach(), precision=precision, flags=flags, device=phi0.device)
        C = max(1, int(checkpoint))
        snaps = []
        for t0 in range(0, int(nsteps), C):
            snaps.append(lat.save_raw())
            lat.step(min(C, int(nsteps) - t0))
        phi = lat.moments(("phi",))["phi"]
        ctx.lat = lat
        ctx.param_meta = [(x.device, x.dtype) if torch.is_tensor(x) else None for x in (sigma, M)]
        ctx.snaps = snaps
        ctx.C = C
        ctx.K = int(nsteps)
        ctx.save_for_backward(phi0.detach())
        return phi

    @staticmethod
    def backward(ctx, dphi):
        (phi0,) = ctx.saved_tensors
        lat, snaps, C, K = ctx.lat, ctx.snaps, ctx.C, ctx.K
        lat.adjoint_begin(dphi.detach().to(torch.float64).contiguous())
        records = [torch.empty(lat.record_bytes, dtype=torch.uint8, device=phi0.device)
                   for _ in range(min(C, max(K, 1)))]
        for s in reversed(range(len(snaps))):
            t0 = s * C
            t1 = min(t0 + C, K)
            lat.load_raw(snaps[s], t0)
            lat.step_records(records[:t1 - t0])
            for t in reversed(range(t0, t1)):
                lat.adjoint_step_record(records[t - t0])
        dphi0, dsigma, dM = lat.adjoint_init(phi0)
        grads = []
        for val, meta in zip((dsigma, dM), ctx.param_meta):
            grads.append(None if meta is None else torch.tensor(val, dtype=meta[1], device=meta[0]))
        return (dphi0.to(phi0.dtype), grads[0], grads[1], None, None, None, None, None)


def simulate(phi0: torch.Tensor, sigma: torch.Tensor, M: torch.Tensor, params: dict,
             nsteps: int, checkpoint: int = 100, precision: str = "fp64",
             flags: int = 0) -> torch.Tensor:
    """Order parameter after ``nsteps`` steps from ``phi0``; differentiable
    with respect to phi0, sigma and M (0-d tensors)."""
    return PhaseFieldRun.apply(phi0, sigma, M, params, nsteps, checkpoint, precision, flags)
