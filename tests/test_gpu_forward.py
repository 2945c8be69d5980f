"""GPU forward step vs the CPU oracle, element by element, through the C ABI.

FP64 tolerance: 1e-12 normwise (max |gpu - oracle| / max |oracle| per
population set or field), the target the method's FP64 implementation is
held to. FP32 / FP16-storage tolerances follow from the storage rounding
(2^-24 and 2^-11 relative) amplified by the O(10) terms of a step.
"""
import math

import numpy as np
import pytest
import torch

import workloads as wl
from oracle import qilbm_oracle as O

pytestmark = pytest.mark.gpu

torch.set_num_threads(4)


def _rel(a, b):
    a = torch.as_tensor(a).cpu().double()
    b = torch.as_tensor(b).cpu().double()
    return float((a - b).abs().max() / b.abs().max().clamp_min(1e-300))


def _lattice(pb, phi0, precision="fp64", flags=0):
    from paper_1507_03521_amd import Lattice
    return Lattice(pb.as_dict(), phi0, precision=precision, flags=flags, device="cuda:0")


def _problem(nx, ny, bc, gy=0.0):
    return wl.droplet64().with_(nx=nx, ny=ny, bc=bc, gy=gy, rho_ref=0.55)


# shapes: one strip (ragged), two and three strips with ragged tails, walls
SHAPES = [(37, 29, wl.PERIODIC, 0.0), (300, 70, wl.WALLS_Y, -1e-5), (520, 45, wl.PERIODIC, 0.0),
          (64, 64, wl.WALLS_Y, -2e-5), (3, 3, wl.PERIODIC, 0.0), (5, 4, wl.WALLS_Y, -1e-5)]


def _flags_id(fl):
    return "unfused" if fl else "fused"


@pytest.mark.parametrize("flags", [0, 2], ids=_flags_id)
@pytest.mark.parametrize("nx,ny,bc,gy", SHAPES)
def test_one_step_fp64_random_state(nx, ny, bc, gy, flags):
    print(f"case one-step fp64 {nx}x{ny} bc={bc} flags={flags}", flush=True)
    pb = _problem(nx, ny, bc, gy)
    f, g = wl.random_state(nx, ny, seed=nx * 1000 + ny)
    lat = _lattice(pb, np.full((ny, nx), 0.5), flags=flags)
    lat.set_state(f, g)
    lat.step(1)
    fg, gg = lat.get_state()
    co = O.coefficients_of(pb)
    with torch.no_grad():
        fr, gr = O.step(torch.tensor(f), torch.tensor(g), co)
    assert _rel(fg, fr) <= 1e-12
    assert _rel(gg, gr) <= 1e-12


@pytest.mark.parametrize("seg_rows", [1, 3, 7, 64])
def test_fused_segment_lengths(seg_rows):
    """Results do not depend on the fused kernel's segment length."""
    print(f"case seg_rows={seg_rows}", flush=True)
    pb = _problem(300, 41, wl.WALLS_Y, -1e-5)
    f, g = wl.random_state(300, 41, seed=5)
    lat = _lattice(pb, np.full((41, 300), 0.5))
    lat.set_launch(seg_rows)
    lat.set_state(f, g)
    lat.step(2)
    fg, gg = lat.get_state()
    co = O.coefficients_of(pb)
    with torch.no_grad():
        fr, gr = O.run(None, co, 2, state=(torch.tensor(f), torch.tensor(g)))
    assert _rel(fg, fr) <= 1e-12 and _rel(gg, gr) <= 1e-12


def test_initial_state_matches_oracle():
    pb = wl.droplet64()
    phi0 = wl.phi0(pb)
    lat = _lattice(pb, phi0)
    fg, gg = lat.get_state()
    fr, gr = O.initial_state(phi0, O.coefficients_of(pb))
    assert float(fg.abs().max()) == 0.0
    assert _rel(gg, gr) <= 1e-14


def test_moments_match_oracle():
    pb = _problem(70, 50, wl.WALLS_Y, -3e-5)
    f, g = wl.random_state(70, 50, seed=8)
    lat = _lattice(pb, np.full((50, 70), 0.5))
    lat.set_state(f, g)
    m = lat.moments()
    ref = O.moments(torch.tensor(f), torch.tensor(g), O.coefficients_of(pb))
    for k, r in zip(("phi", "rho", "ux", "uy", "p", "mu"), ref):
        assert _rel(m[k], r) <= 1e-13, k


def test_droplet64_2000_steps_fp64():
    """64x64 static droplet, 2000 steps: state within 1e-12 of the oracle,
    sum phi and sum rho conserved to 1e-12, Laplace law within 5 %."""
    pb = wl.droplet64()
    phi0 = wl.phi0(pb)
    lat = _lattice(pb, phi0)
    m0 = lat.mass()
    lat.step(pb.steps)
    m1 = lat.mass()
    fg, gg = lat.get_state()
    co = O.coefficients_of(pb)
    with torch.no_grad():
        fr, gr = O.run(phi0, co, pb.steps)
    print("droplet64 rel f", _rel(fg, fr), "g", _rel(gg, gr), flush=True)
    assert _rel(fg, fr) <= 1e-12
    assert _rel(gg, gr) <= 1e-12
    assert abs(m1[0] - m0[0]) <= 1e-12 * abs(m0[0])
    assert abs(m1[1] - m0[1]) <= 1e-12 * abs(m0[1])
    ref = O.mass(fr, gr, co)
    for a, b in zip(m1[:2], ref[:2]):
        assert a == pytest.approx(b, rel=1e-13)


def test_rayleigh_taylor_walls_fp64():
    """Walls + gravity: a 64x128 Rayleigh-Taylor lattice with the 256x1024
    problem's parameters, 300 steps."""
    pb = wl.rt256().with_(nx=64, ny=128, meta=dict(h0=64.0, amp=6.4))
    phi0 = wl.phi0(pb)
    lat = _lattice(pb, phi0)
    lat.step(300)
    fg, gg = lat.get_state()
    with torch.no_grad():
        fr, gr = O.run(phi0, O.coefficients_of(pb), 300)
    assert _rel(fg, fr) <= 1e-12
    assert _rel(gg, gr) <= 1e-12


def test_gamma_ablation_flag():
    pb = _problem(40, 30, wl.PERIODIC)
    f, g = wl.random_state(40, 30, seed=3)
    from paper_1507_03521_amd import LBM_FLAG_NO_GAMMA
    lat = _lattice(pb, np.full((30, 40), 0.5), flags=LBM_FLAG_NO_GAMMA)
    lat.set_state(f, g)
    lat.step(1)
    fg, gg = lat.get_state()
    with torch.no_grad():
        fr, gr = O.step(torch.tensor(f), torch.tensor(g), O.coefficients_of(pb, no_gamma=True))
    assert _rel(fg, fr) <= 1e-12 and _rel(gg, gr) <= 1e-12


@pytest.mark.parametrize("precision,tol", [("fp32", 2e-6), ("fp16", 4e-3)])
@pytest.mark.parametrize("bc", [wl.PERIODIC, wl.WALLS_Y])
def test_one_step_reduced_precision(precision, tol, bc):
    print(f"case one-step {precision} bc={bc}", flush=True)
    nx, ny = 300, 37
    pb = _problem(nx, ny, bc, -1e-5)
    f, g = wl.random_state(nx, ny, seed=17)
    lat = _lattice(pb, np.full((ny, nx), 0.5), precision=precision)
    lat.set_state(f, g)
    lat.step(1)
    fg, gg = lat.get_state()
    with torch.no_grad():
        fr, gr = O.step(torch.tensor(f), torch.tensor(g), O.coefficients_of(pb))
    assert _rel(fg, fr) <= tol
    assert _rel(gg, gr) <= tol


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-4), ("fp16", 5e-2)])
def test_droplet_reduced_precision_200_steps(precision, tol):
    pb = wl.droplet64()
    phi0 = wl.phi0(pb)
    lat = _lattice(pb, phi0, precision=precision)
    lat.step(200)
    m = lat.moments(("phi",))
    with torch.no_grad():
        fr, gr = O.run(phi0, O.coefficients_of(pb), 200)
    err = float((m["phi"].cpu() - gr.sum(0)).abs().max())
    print(precision, "phi max abs error after 200 steps", err, flush=True)
    assert err <= tol


def test_translation_is_bitwise_on_gpu():
    pb = _problem(96, 48, wl.PERIODIC)
    phi0 = wl.random_phi(96, 48, seed=2)
    a = _lattice(pb, phi0)
    b = _lattice(pb, np.roll(phi0, (5, 17), axis=(0, 1)))
    a.step(7)
    b.step(7)
    fa, ga = a.get_state()
    fb, gb = b.get_state()
    assert torch.equal(torch.roll(fa, (5, 17), dims=(1, 2)), fb)
    assert torch.equal(torch.roll(ga, (5, 17), dims=(1, 2)), gb)


def test_run_to_run_bitwise_and_raw_restore():
    pb = wl.droplet64()
    phi0 = wl.phi0(pb)
    a = _lattice(pb, phi0)
    a.step(10)
    snap = a.save_raw()
    a.step(15)
    fa, ga = a.get_state()
    ma = a.mass()
    b = _lattice(pb, phi0)
    b.load_raw(snap, 10)
    b.step(15)
    fb, gb = b.get_state()
    assert b.time == 25
    assert torch.equal(fa, fb) and torch.equal(ga, gb)
    assert ma == b.mass()


def test_set_get_state_roundtrip():
    pb = _problem(33, 21, wl.WALLS_Y)
    f, g = wl.random_state(33, 21, seed=4)
    lat = _lattice(pb, np.full((21, 33), 0.5))
    lat.set_state(f, g)
    fg, gg = lat.get_state()
    assert torch.equal(fg.cpu(), torch.tensor(f)) and torch.equal(gg.cpu(), torch.tensor(g))


def test_nan_input_reports_divergence():
    from paper_1507_03521_amd import QilbmError
    pb = wl.droplet64()
    phi0 = wl.phi0(pb)
    phi0[10, 10] = float("nan")
    lat = _lattice(pb, phi0)
    lat.step(3)
    with pytest.raises(QilbmError):
        lat.mass()


# ------------------------------------------------- full-size sampled parity
def _window_check(state, pb, phi0, y0, x0, h, w):
    """One step from the initial state; the oracle runs on a window whose
    rows [y0, y0+h) and columns [x0, x0+w) (wrapped in x) surround the
    compared nodes by 6 on every side that is not a wall."""
    co = O.coefficients_of(pb)
    ny = pb.ny
    lo = max(0, y0 - 6) if pb.bc == wl.WALLS_Y else y0 - 6
    hi = min(ny, y0 + h + 6) if pb.bc == wl.WALLS_Y else y0 + h + 6
    rows = np.arange(lo, hi) % ny
    cols = np.arange(x0 - 6, x0 + w + 6) % pb.nx
    win = phi0[np.ix_(rows, cols)]
    sub = pb.with_(nx=len(cols), ny=len(rows))
    with torch.no_grad():
        fr, gr = O.run(win, O.coefficients_of(sub), 1)
    r0 = y0 - lo
    fr = fr[:, r0:r0 + h, 6:6 + w]
    gr = gr[:, r0:r0 + h, 6:6 + w]
    fg, gg = state
    rr = torch.as_tensor(np.arange(y0, y0 + h) % ny)
    cc = torch.as_tensor(np.arange(x0, x0 + w) % pb.nx)
    fg = fg[:, rr][:, :, cc].cpu()
    gg = gg[:, rr][:, :, cc].cpu()
    return _rel(fg, fr), _rel(gg, gr)


@pytest.mark.parametrize("name", ["rt2048", "bubble4096"])
def test_full_size_sampled_one_step(name):
    """At the full problem sizes, in the benchmark's launch shape: one step
    from the initial state compared on windows at the walls, at strip and
    segment boundaries and in the bulk. FP64 for the Rayleigh-Taylor problem,
    FP32 (relative 2e-6) for the bubble."""
    print(f"case full-size {name}", flush=True)
    pb = wl.rt2048() if name == "rt2048" else wl.bubble4096()
    precision, tol = ("fp64", 1e-12) if name == "rt2048" else ("fp32", 2e-6)
    phi0 = wl.phi0(pb)
    lat = _lattice(pb, phi0, precision=precision)
    info = lat.launch_info()
    lat.step(1)
    state = lat.get_state()
    sr = info["seg_rows"]
    picks = [(0, 250, 12, 12), (pb.ny - 12, 1000, 12, 12), (sr - 6, 250, 12, 12),
             (pb.ny // 2 - 6, 2 * 256 - 6, 12, 12), (1536 - 260, 2048 - 6, 12, 12),
             (pb.ny // 2 + 3, pb.nx - 6, 12, 12)]
    for (y0, x0, h, w) in picks:
        ef, eg = _window_check(state, pb, phi0, y0, x0, h, w)
        print(f"  window y0={y0} x0={x0}: rel f {ef:.2e} g {eg:.2e}", flush=True)
        assert ef <= tol and eg <= tol
    del lat, state
    torch.cuda.empty_cache()
