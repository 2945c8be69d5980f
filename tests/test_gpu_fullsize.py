"""The headline kernel at full size against the oracle, in the launch shape
the benchmark times: the BGK two-steps-per-launch kernel on the 2048 x 8192
Rayleigh-Taylor lattice (FP64 and FP32), and on the 4096 x 8192 rising-bubble
lattice (FP32), two steps from a random pre-collision state, compared with
the oracle on sampled windows at the walls, a segment boundary, a strip
boundary, the periodic seam and the middle.

Tolerances (max |gpu - oracle| / max |oracle| per window and population set)
are those of the one-step checks from random states: FP64 1e-12; FP32 3e-5
for f and 1e-6 for g (binary32 arithmetic, Q2.29 g)."""
import numpy as np
import pytest
import torch

import workloads as wl
from windows import compare_windows

pytestmark = pytest.mark.gpu

torch.set_num_threads(8)

TOL = {"fp64": (1e-12, 1e-12), "fp32": (3e-5, 1e-6)}


def _run_two_steps(pb, precision, seed):
    from paper_1507_03521_amd import Lattice
    f0, g0 = wl.random_state(pb.nx, pb.ny, seed=seed)
    lat = Lattice(pb.as_dict(), np.full((pb.ny, pb.nx), 0.5), precision=precision,
                  device="cuda:0")
    lat.set_state(f0, g0)
    del f0, g0
    before = tuple(t.cpu() for t in lat.get_state())     # exactly what is stored
    info = lat.pass_info()
    print(f"  launch: {info}", flush=True)
    assert info["steps"] == 2
    lat.step(2)
    return lat, before, lat.get_state(), info


def _picks(pb, info):
    nx, ny = pb.nx, pb.ny
    seg, width = info["seg_rows"], -(-nx // info["strips"])
    return [(0, 250), (ny - 12, 1000), (seg - 6, width - 6), (2 * seg - 6, 3 * width - 6),
            (ny // 2 - 6, nx - 6), (ny // 2 - 6, nx // 4 - 6)]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_bgk_two_step_pass_rt2048_windows(precision):
    print(f"case bgk full size rt2048 {precision}", flush=True)
    pb = wl.rt2048()
    lat, before, after, info = _run_two_steps(pb, precision, seed=43)
    assert info["strips"] == 9 and info["threads"] == 256
    compare_windows(pb, before, after, _picks(pb, info), 2, TOL[precision])
    lat.close()
    del lat, before, after
    torch.cuda.empty_cache()


def test_bgk_two_step_pass_bubble4096_windows_fp32():
    print("case bgk full size bubble4096 fp32", flush=True)
    pb = wl.bubble4096()
    lat, before, after, info = _run_two_steps(pb, "fp32", seed=47)
    compare_windows(pb, before, after, _picks(pb, info), 2, TOL["fp32"])
    lat.close()
    del lat, before, after
    torch.cuda.empty_cache()
