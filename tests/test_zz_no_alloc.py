"""lbm_mass_noalloc (the allocation-free form of lbm_mass, scratch in the
library's static device array) against lbm_mass of a context holding the
same state, through the C ABI: several calls in a row on one GPU, each on a
smaller lattice than the one before (the array keeps the previous call's
larger contents), in all three storage precisions; and its refusals."""
import numpy as np
import pytest
import torch

import workloads as wl

pytestmark = pytest.mark.gpu


def _lattice(nx, ny, bc, precision, seed):
    from paper_1507_03521_amd import Lattice
    pb = wl.droplet64().with_(nx=nx, ny=ny, bc=bc, gy=-2e-5 * bc, gx=1e-5, rho_ref=0.55)
    f, g = wl.random_state(nx, ny, seed=seed)
    lat = Lattice(pb.as_dict(), np.full((ny, nx), 0.5), precision=precision, device="cuda:0")
    lat.set_state(f, g)
    lat.step(3)
    return pb, lat


# decreasing sizes; the first is the largest lattice the scratch holds
CASES = [(1024, 2048, wl.WALLS_Y, "fp64"), (1000, 1500, wl.PERIODIC, "fp32"),
         (300, 70, wl.WALLS_Y, "fp16"), (37, 29, wl.PERIODIC, "fp64"), (5, 4, wl.WALLS_Y, "fp32")]


def test_mass_noalloc_equals_lbm_mass_on_calls_in_a_row():
    from paper_1507_03521_amd.lattice import MASS_NOALLOC_MAX_NODES, mass_noalloc
    assert CASES[0][0] * CASES[0][1] == MASS_NOALLOC_MAX_NODES
    out = torch.empty(4, dtype=torch.float64, device="cuda:0")
    for k, (nx, ny, bc, precision) in enumerate(CASES):
        print(f"case noalloc {nx}x{ny} bc={bc} {precision}", flush=True)
        pb, lat = _lattice(nx, ny, bc, precision, seed=k + 3)
        ref = lat.mass()
        raw = lat.save_raw()
        out.fill_(float("nan"))
        mass_noalloc(pb.as_dict(), precision, raw, out)
        got = tuple(out.cpu().tolist())
        print(f"  lbm_mass {ref}\n  noalloc  {got}", flush=True)
        assert got == ref              # same kernels, same order: bit for bit
        # a second call on the same input gives the same again
        mass_noalloc(pb.as_dict(), precision, raw, out)
        assert tuple(out.cpu().tolist()) == ref
        lat.close()
        del lat, raw
        torch.cuda.empty_cache()


def test_mass_noalloc_refusals():
    from paper_1507_03521_amd import QilbmError
    from paper_1507_03521_amd.lattice import mass_noalloc
    out = torch.full((4,), 7.0, dtype=torch.float64, device="cuda:0")
    pb, lat = _lattice(64, 32, wl.PERIODIC, "fp32", seed=1)
    raw = lat.save_raw()
    big = pb.with_(nx=2049, ny=1024)                       # 2^21 + 1024 nodes
    with pytest.raises(QilbmError):
        mass_noalloc(big.as_dict(), "fp32", raw, out)
    with pytest.raises(QilbmError):                        # state not 256-byte aligned
        mass_noalloc(pb.as_dict(), "fp32", raw[8:], out)
    with pytest.raises(QilbmError):                        # invalid parameters
        mass_noalloc(pb.with_(tau_f=0.4).as_dict(), "fp32", raw, out)
    torch.cuda.synchronize()
    assert out.cpu().tolist() == [7.0] * 4                 # nothing was enqueued
