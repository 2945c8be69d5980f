"""Two time steps per pass of the fused kernel (the default for FP64 and
FP32; FP16 storage on request).

The two-step kernel keeps the first step's post-collision populations on
chip (FP64 and FP32 in their storage format, binary64 or binary32 f with
Q2.29 g; FP16 storage in that FP32 format, so it rounds to binary16 once
per pass) and runs the second step on them. It evaluates the same
expressions as the one-step kernel, but the compiler contracts
multiply-adds per kernel (measured: with contraction off the two write
identical bytes), so the two agree to rounding (FP16 storage: to binary16
rounding), and both conserve the exact integer total of the stored g. Checked here against the FP64 oracle and against one step per launch, on
lattices with one strip and with several ragged strips, periodic and
walled, narrower than the kernel's 7-column halo, with segment lengths from
1 row to the whole lattice, for even and odd step counts, and at the full
2048 x 8192 size in the benchmark's launch shape.

Tolerances (max |a - b| / max |b| per population set), from a random state
(test_gpu_forward's reduced-precision bounds): FP32 f 3e-5, g 1e-6 (measured
after 6 steps: 5.5e-6 and 7.7e-8 against the oracle, 2.2e-6 and 6.5e-8
between the two kernels: rounding differences grow through the steps);
FP16 storage 4e-3 for both; FP64 the one-step bounds of multi-step runs
(test_gpu_forward): f 2e-11, g 1e-12. FP64 has no fixed-point total.
"""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import qilbm_oracle as O
from q229 import q229_total

pytestmark = pytest.mark.gpu

TOL = {"fp64": (2e-11, 1e-12), "fp32": (3e-5, 1e-6), "fp16": (4e-3, 4e-3)}


def _rel(a, b):
    a = torch.as_tensor(a).cpu().double()
    b = torch.as_tensor(b).cpu().double()
    return float((a - b).abs().max() / b.abs().max().clamp_min(1e-300))


def _lattice(pb, phi0, precision):
    from paper_1507_03521_amd import Lattice
    return Lattice(pb.as_dict(), phi0, precision=precision, device="cuda:0")


def _run_pair(pb, precision, nsteps, seg_rows, seed):
    """From a random pre-collision state: the states after nsteps with one
    step per launch and with two, the oracle's, and the exact Q2.29 totals
    before and after (one per run)."""
    f, g = wl.random_state(pb.nx, pb.ny, seed=seed)
    states, totals = [], []
    for steps in (1, 2):
        lat = _lattice(pb, np.full((pb.ny, pb.nx), 0.5), precision)
        lat.set_pass(steps, seg_rows if steps == 2 else 0)
        assert lat.pass_info()["steps"] == steps
        lat.set_state(f, g)
        fixed = precision != "fp64"
        q0 = q229_total(lat.save_raw(), precision, pb.nx, pb.ny) if fixed else 0
        lat.step(nsteps)
        assert lat.time == nsteps
        totals.append((q0, q229_total(lat.save_raw(), precision, pb.nx, pb.ny) if fixed else 0))
        states.append(lat.get_state())
        lat.close()
    with torch.no_grad():
        ref = O.run(None, O.coefficients_of(pb), nsteps, state=(torch.tensor(f), torch.tensor(g)))
    return states, ref, totals


def _check(precision, states, ref, totals):
    (f1, g1), (f2, g2) = states
    tf, tg = TOL[precision]
    e = dict(two_oracle=(_rel(f2, ref[0]), _rel(g2, ref[1])),
             one_oracle=(_rel(f1, ref[0]), _rel(g1, ref[1])), two_one=(_rel(f2, f1), _rel(g2, g1)))
    print("  rel (f, g):", {k: f"{a:.2e} {b:.2e}" for k, (a, b) in e.items()}, flush=True)
    for a, b in e.values():
        assert a <= tf and b <= tg
    # exact mass: each run keeps its initial integer total, and both start equal
    assert totals[0][0] == totals[1][0]
    assert totals[0][1] == totals[0][0] and totals[1][1] == totals[1][0]


# one strip (ragged), several strips with ragged tails, walls, lattices
# narrower than the halo, a single row band
SHAPES = [(37, 29, wl.PERIODIC, 0.0), (300, 70, wl.WALLS_Y, -1e-5), (520, 45, wl.PERIODIC, 0.0),
          (485, 33, wl.WALLS_Y, -2e-5), (3, 3, wl.PERIODIC, 0.0), (5, 4, wl.WALLS_Y, -1e-5),
          (10, 40, wl.PERIODIC, 0.0), (243, 12, wl.WALLS_Y, -1e-5)]


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16"])
@pytest.mark.parametrize("nx,ny,bc,gy", SHAPES)
def test_two_step_pass_matches_oracle_and_one_step_launches(precision, nx, ny, bc, gy):
    print(f"case pass2 {precision} {nx}x{ny} bc={bc}", flush=True)
    pb = wl.droplet64().with_(nx=nx, ny=ny, bc=bc, gy=gy, rho_ref=0.55)
    _check(precision, *_run_pair(pb, precision, 6, 0, seed=nx + 7 * ny))


@pytest.mark.parametrize("seg_rows", [1, 2, 5, 16, 64, 1000])
@pytest.mark.parametrize("nsteps", [7, 8])
def test_two_step_pass_segment_lengths_and_odd_counts(seg_rows, nsteps):
    print(f"case pass2 seg_rows={seg_rows} nsteps={nsteps}", flush=True)
    pb = wl.droplet64().with_(nx=300, ny=41, bc=wl.WALLS_Y, gy=-1e-5, rho_ref=0.55)
    _check("fp32", *_run_pair(pb, "fp32", nsteps, seg_rows, seed=5))


@pytest.mark.parametrize("precision,tol", [("fp64", (5e-12, 1e-12)), ("fp32", (2e-3, 1e-6))])
def test_two_step_pass_full_size_rt2048(precision, tol):
    """2048 x 8192 Rayleigh-Taylor lattice between walls, automatic launch
    shapes (the benchmark's): 4 steps from the initial interface plus a
    small random perturbation, one step per launch vs two. Bounds: those of
    the full-size checks against the oracle (test_gpu_forward; f is small
    near rest and formed by cancellation); in FP32 the exact Q2.29 totals
    are equal."""
    print(f"case pass2 full size rt2048 {precision}", flush=True)
    pb = wl.rt2048()
    phi0 = wl.phi0(pb)
    rng = np.random.default_rng(3)
    phi0 = np.clip(phi0 + 0.02 * (rng.random(phi0.shape) - 0.5), 0.0, 1.0)
    states, totals = [], []
    for steps in (1, 2):
        lat = _lattice(pb, phi0, precision)
        lat.set_pass(steps)
        info = lat.pass_info()
        print(f"  steps per pass {steps}: {info}", flush=True)
        if steps == 2:
            assert info["strips"] == 9 and info["threads"] == 256
        lat.step(4)
        if precision != "fp64":
            totals.append(q229_total(lat.save_raw(), precision, pb.nx, pb.ny))
        states.append(lat.get_state())
        lat.close()
        torch.cuda.empty_cache()
    (f1, g1), (f2, g2) = states
    ef, eg = _rel(f2, f1), _rel(g2, g1)
    print(f"  two vs one: rel f {ef:.2e} g {eg:.2e}", flush=True)
    assert ef <= tol[0] and eg <= tol[1]
    if totals:
        assert totals[0] == totals[1]
    del states
    torch.cuda.empty_cache()


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-4), ("fp16", 5e-2)])
def test_two_step_pass_droplet_vs_oracle(precision, tol):
    """The 64 x 64 droplet for 200 steps (100 two-step passes) against the
    FP64 oracle: phi within the reduced-precision bounds of the one-step
    runs."""
    pb = wl.droplet64()
    phi0 = wl.phi0(pb)
    lat = _lattice(pb, phi0, precision)
    lat.set_pass(2)
    assert lat.pass_info()["steps"] == 2
    lat.step(200)
    m = lat.moments(("phi",))
    with torch.no_grad():
        _, gr = O.run(phi0, O.coefficients_of(pb), 200)
    err = float((m["phi"].cpu() - gr.sum(0)).abs().max())
    print(precision, "two-step pass: phi max abs error after 200 steps", err, flush=True)
    assert err <= tol


def test_pass_settings():
    """Defaults and argument checks of lbm_set_pass / lbm_pass_info."""
    from paper_1507_03521_amd import QilbmError
    pb = wl.droplet64()
    phi0 = wl.phi0(pb)
    l64 = _lattice(pb, phi0, "fp64")
    assert l64.pass_info()["steps"] == 2
    l16 = _lattice(pb, phi0, "fp16")
    assert l16.pass_info()["steps"] == 1
    l32 = _lattice(pb, phi0, "fp32")
    info = l32.pass_info()
    assert info["steps"] == 2 and info["strips"] == 1 and info["threads"] == 256
    for bad in ((0, 0), (3, 0), (2, -1)):
        with pytest.raises(QilbmError):
            l32.set_pass(*bad)
    l32.set_pass(2, 20)
    assert l32.pass_info()["seg_rows"] == 20 and l32.pass_info()["segments"] == 4
    l32.set_pass(1)
    one = l32.pass_info()
    launch = l32.launch_info()
    assert one["steps"] == 1 and one["seg_rows"] == launch["seg_rows"]
