"""Hand-written GPU adjoint vs the CPU oracle's reverse mode (autograd through
the plain FP64 step) and vs central finite differences of the GPU forward."""
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


CASES = [(23, 17, wl.PERIODIC, 0.0), (20, 14, wl.WALLS_Y, -2e-5), (300, 9, wl.WALLS_Y, -1e-5)]


@pytest.mark.parametrize("nx,ny,bc,gy", CASES)
def test_step_vjp_matches_oracle(nx, ny, bc, gy):
    """One adjoint step from arbitrary state and cotangent: population
    cotangents and dL/dsigma, dL/dM of that step."""
    print(f"case vjp {nx}x{ny} bc={bc}", flush=True)
    pb = wl.droplet64().with_(nx=nx, ny=ny, bc=bc, gy=gy, rho_ref=0.5)
    f, g = wl.random_state(nx, ny, seed=31)
    rng = np.random.default_rng(7)
    fbar = rng.standard_normal((9, ny, nx))
    gbar = rng.standard_normal((9, ny, nx))
    lat = _lattice(pb, np.full((ny, nx), 0.5))
    lat.set_state(f, g)
    raw = lat.save_raw()
    lat.adjoint_begin(torch.zeros((ny, nx), dtype=torch.float64, device="cuda:0"))
    lat.adjoint_set(fbar, gbar)
    lat.adjoint_step(raw)
    df, dg, ds, dm = lat.adjoint_get()
    rf, rg, rs, rm = O.step_vjp(f, g, pb, fbar, gbar)
    assert _rel(df, rf) <= 1e-12
    assert _rel(dg, rg) <= 1e-12
    assert ds == pytest.approx(rs, rel=1e-11)
    assert dm == pytest.approx(rm, rel=1e-11)


@pytest.mark.parametrize("nx,ny,bc,gy", CASES)
def test_step_vjp_dot_product_with_forward_mode(nx, ny, bc, gy):
    """Dot-product test of the hand-written adjoint step: for random state
    tangents v = (df, dg, dsigma, dM) and cotangents w = (fbar, gbar),
    <J^T w, v> from the GPU adjoint equals <w, J v> with J v from the
    oracle's forward mode (dual numbers: no transposition involved)."""
    print(f"case dot product {nx}x{ny} bc={bc}", flush=True)
    pb = wl.droplet64().with_(nx=nx, ny=ny, bc=bc, gy=gy, rho_ref=0.5)
    f, g = wl.random_state(nx, ny, seed=37)
    rng = np.random.default_rng(11)
    fbar, gbar, vf, vg = (rng.standard_normal((9, ny, nx)) for _ in range(4))
    vs, vm = 0.4 * pb.sigma, -0.3 * pb.M
    lat = _lattice(pb, np.full((ny, nx), 0.5))
    lat.set_state(f, g)
    raw = lat.save_raw()
    lat.adjoint_begin(torch.zeros((ny, nx), dtype=torch.float64, device="cuda:0"))
    lat.adjoint_set(fbar, gbar)
    lat.adjoint_step(raw)
    df, dg, ds, dm = lat.adjoint_get()
    tf, tg = O.step_jvp(f, g, pb, vf, vg, vs, vm)
    t = lambda a: torch.as_tensor(a, dtype=torch.float64)
    lhs = float((t(fbar) * tf).sum() + (t(gbar) * tg).sum())
    rhs = float((df.cpu() * t(vf)).sum() + (dg.cpu() * t(vg)).sum()) + ds * vs + dm * vm
    print(f"  <w, Jv> = {lhs:.15e}  <J^T w, v> = {rhs:.15e}", flush=True)
    assert rhs == pytest.approx(lhs, rel=1e-10)


def test_gradient_dot_direction_matches_forward_mode():
    """End to end (15 steps with checkpoints): the GPU reverse-mode gradient
    of L dotted with a direction (dphi0, dsigma, dM) equals the directional
    derivative of the oracle's forward map by forward mode."""
    from paper_1507_03521_amd import simulate
    pb = wl.droplets512(small=True).with_(nx=16, ny=13, bc=wl.WALLS_Y, gy=-1e-5)
    phi0 = wl.random_phi(pb.nx, pb.ny, seed=21, lo=0.1, hi=0.9)
    target = _loss_target(pb.nx, pb.ny)
    K = 15
    loss = lambda ph: ((ph - target.to(ph.device)) ** 2).sum()
    v = np.random.default_rng(5).standard_normal(phi0.shape)
    vs, vm = 0.2 * pb.sigma, 0.2 * pb.M
    dL = O.loss_jvp(phi0, pb, K, loss, v, vs, vm)
    dev = "cuda:0"
    p0 = torch.tensor(phi0, device=dev, requires_grad=True)
    sig = torch.tensor(pb.sigma, dtype=torch.float64, requires_grad=True)
    mob = torch.tensor(pb.M, dtype=torch.float64, requires_grad=True)
    loss(simulate(p0, sig, mob, pb.as_dict(), K, checkpoint=4)).backward()
    got = float((p0.grad.cpu() * torch.as_tensor(v)).sum()) + float(sig.grad) * vs + \
        float(mob.grad) * vm
    print(f"  forward mode {dL:.15e}  GPU reverse mode {got:.15e}", flush=True)
    assert got == pytest.approx(dL, rel=1e-10)


def _loss_target(nx, ny, seed=22):
    return torch.as_tensor(wl.random_phi(nx, ny, seed=seed, lo=0.2, hi=0.8))


@pytest.mark.parametrize("bc", [wl.PERIODIC, wl.WALLS_Y])
def test_end_to_end_gradients_match_oracle(bc):
    from paper_1507_03521_amd import simulate
    pb = wl.droplets512(small=True).with_(nx=16, ny=13, bc=bc, gy=-1e-5 * bc)
    phi0 = wl.random_phi(pb.nx, pb.ny, seed=21, lo=0.1, hi=0.9)
    target = _loss_target(pb.nx, pb.ny)
    K = 15
    L, ds, dm, dp = O.loss_and_gradients(phi0, pb, K, lambda ph: ((ph - target) ** 2).sum())
    dev = "cuda:0"
    p0 = torch.tensor(phi0, device=dev, requires_grad=True)
    sig = torch.tensor(pb.sigma, dtype=torch.float64, requires_grad=True)
    mob = torch.tensor(pb.M, dtype=torch.float64, requires_grad=True)
    phi = simulate(p0, sig, mob, pb.as_dict(), K, checkpoint=4)
    Lg = ((phi - target.to(dev)) ** 2).sum()
    Lg.backward()
    assert float(Lg.detach()) == pytest.approx(L, rel=1e-12)
    assert float(sig.grad) == pytest.approx(ds, rel=1e-10)
    assert float(mob.grad) == pytest.approx(dm, rel=1e-10)
    assert _rel(p0.grad, dp) <= 1e-10


def test_checkpoint_interval_does_not_change_gradients():
    """Gradients do not depend on the checkpoint interval C. With two steps
    per kernel pass (the FP64 default) the forward and every replay launch
    pairs of steps from the start of each segment, so for even C the run is
    the same sequence of launches as without checkpoints and the gradients
    are bitwise equal; an odd C moves the pairs, which changes only the
    rounding (the two kernels contract multiply-adds differently): 1e-12."""
    from paper_1507_03521_amd import simulate
    pb = wl.droplets512(small=True)
    phi0 = torch.tensor(wl.phi0(pb), device="cuda:0")
    target = _loss_target(pb.nx, pb.ny).to("cuda:0")
    res = {}
    for C in (2, 8, 40, 1, 7):
        p0 = phi0.clone().requires_grad_(True)
        sig = torch.tensor(pb.sigma, dtype=torch.float64, requires_grad=True)
        mob = torch.tensor(pb.M, dtype=torch.float64, requires_grad=True)
        L = ((simulate(p0, sig, mob, pb.as_dict(), 40, checkpoint=C) - target) ** 2).sum()
        L.backward()
        res[C] = (float(sig.grad), float(mob.grad), p0.grad.clone())
    ref = res[40]
    for C in (2, 8):
        assert res[C][0] == ref[0] and res[C][1] == ref[1]
        assert torch.equal(res[C][2], ref[2])
    for C in (1, 7):
        assert res[C][0] == pytest.approx(ref[0], rel=1e-12)
        assert res[C][1] == pytest.approx(ref[1], rel=1e-12)
        assert _rel(res[C][2], ref[2]) <= 1e-12


def test_finite_differences_droplets32():
    """32x32, 200-step copy of the two-droplet gradient workload: loss
    sum (phi_K - phi_target)^2 with phi_target from a run at 1.2 sigma.
    Adjoint dL/dsigma, dL/dM and dL/dphi0 entries vs central differences of
    the GPU forward with relative step 1e-6; agreement 1e-6."""
    from paper_1507_03521_amd import Lattice, simulate
    pb = wl.droplets512(small=True)
    phi0 = wl.phi0(pb)
    K = pb.steps
    dev = "cuda:0"
    tgt_lat = Lattice(pb.with_(sigma=1.2 * pb.sigma).as_dict(), phi0, device=dev)
    tgt_lat.step(K)
    target = tgt_lat.moments(("phi",))["phi"]

    def loss(sigma=pb.sigma, M=pb.M, ph=phi0):
        lat = Lattice(pb.with_(sigma=sigma, M=M).as_dict(), ph, device=dev)
        lat.step(K)
        return float(((lat.moments(("phi",))["phi"] - target) ** 2).sum())

    p0 = torch.tensor(phi0, device=dev, requires_grad=True)
    sig = torch.tensor(pb.sigma, dtype=torch.float64, requires_grad=True)
    mob = torch.tensor(pb.M, dtype=torch.float64, requires_grad=True)
    L = ((simulate(p0, sig, mob, pb.as_dict(), K, checkpoint=20) - target) ** 2).sum()
    L.backward()
    h = 1e-6
    fd_s = (loss(sigma=pb.sigma * (1 + h)) - loss(sigma=pb.sigma * (1 - h))) / (2 * h * pb.sigma)
    fd_m = (loss(M=pb.M * (1 + h)) - loss(M=pb.M * (1 - h))) / (2 * h * pb.M)
    print("dL/dsigma adjoint", float(sig.grad), "fd", fd_s, flush=True)
    print("dL/dM adjoint", float(mob.grad), "fd", fd_m, flush=True)
    assert float(sig.grad) == pytest.approx(fd_s, rel=1e-6)
    assert float(mob.grad) == pytest.approx(fd_m, rel=1e-6)
    g = p0.grad.cpu().numpy()
    idx = np.unravel_index(np.argsort(np.abs(g).ravel())[-3:], g.shape)
    for yy, xx in zip(*idx):
        e = np.zeros_like(phi0)
        e[yy, xx] = 1e-6
        fd = (loss(ph=phi0 + e) - loss(ph=phi0 - e)) / 2e-6
        assert g[yy, xx] == pytest.approx(fd, rel=1e-6)


def test_fp32_adjoint_close_to_fp64():
    from paper_1507_03521_amd import simulate
    pb = wl.droplets512(small=True)
    phi0 = torch.tensor(wl.phi0(pb), device="cuda:0")
    target = _loss_target(pb.nx, pb.ny).to("cuda:0")
    out = {}
    for prec in ("fp64", "fp32"):
        p0 = phi0.clone().requires_grad_(True)
        sig = torch.tensor(pb.sigma, dtype=torch.float64, requires_grad=True)
        mob = torch.tensor(pb.M, dtype=torch.float64, requires_grad=True)
        L = ((simulate(p0, sig, mob, pb.as_dict(), 50, checkpoint=10, precision=prec) - target) ** 2).sum()
        L.backward()
        out[prec] = (float(sig.grad), float(mob.grad), p0.grad.cpu())
    assert out["fp32"][0] == pytest.approx(out["fp64"][0], rel=1e-3)
    assert out["fp32"][1] == pytest.approx(out["fp64"][1], rel=1e-3)
    assert _rel(out["fp32"][2], out["fp64"][2]) <= 1e-3


def test_two_droplets_512_full_size_gradients_vs_finite_differences():
    """The two-droplet gradient workload at full size: 512x512 periodic,
    K = 2000 steps, checkpoints every 100, loss sum (phi_K - phi_target)^2
    with phi_target from a run at 1.2 sigma. Adjoint dL/dsigma and dL/dM,
    and the directional derivative <dL/dphi0, v> along a smooth random
    field v, vs central differences of the GPU forward (relative step
    1e-6): agreement 1e-6. Also reports the FP32 adjoint's deviation."""
    from paper_1507_03521_amd import Lattice, simulate
    pb = wl.droplets512()
    phi0 = wl.phi0(pb)
    K, C = pb.steps, pb.meta["checkpoint"]
    dev = "cuda:0"
    tgt = Lattice(pb.with_(sigma=1.2 * pb.sigma).as_dict(), phi0, device=dev)
    tgt.step(K)
    target = tgt.moments(("phi",))["phi"]
    v = torch.tensor(wl.random_phi(pb.nx, pb.ny, seed=5, lo=-1.0, hi=1.0), device=dev)

    def loss(sigma=pb.sigma, M=pb.M, ph=None):
        ph = torch.tensor(phi0, device=dev) if ph is None else ph
        lat = Lattice(pb.with_(sigma=sigma, M=M).as_dict(), ph, device=dev)
        lat.step(K)
        return float(((lat.moments(("phi",))["phi"] - target) ** 2).sum())

    grads = {}
    for prec in ("fp64", "fp32"):
        p0 = torch.tensor(phi0, device=dev, requires_grad=True)
        sig = torch.tensor(pb.sigma, dtype=torch.float64, requires_grad=True)
        mob = torch.tensor(pb.M, dtype=torch.float64, requires_grad=True)
        L = ((simulate(p0, sig, mob, pb.as_dict(), K, checkpoint=C, precision=prec)
              - target) ** 2).sum()
        L.backward()
        grads[prec] = (float(sig.grad), float(mob.grad), float((p0.grad * v).sum()))
    h = 1e-6
    p = torch.tensor(phi0, device=dev)
    fd = ((loss(sigma=pb.sigma * (1 + h)) - loss(sigma=pb.sigma * (1 - h))) / (2 * h * pb.sigma),
          (loss(M=pb.M * (1 + h)) - loss(M=pb.M * (1 - h))) / (2 * h * pb.M),
          (loss(ph=p + h * v) - loss(ph=p - h * v)) / (2 * h))
    names = ("dL/dsigma", "dL/dM", "<dL/dphi0, v>")
    for name, a, a32, f in zip(names, grads["fp64"], grads["fp32"], fd):
        print(f"{name}: adjoint FP64 {a:.10e} FP32 {a32:.6e} (rel {abs(a32 - a) / abs(a):.1e}), "
              f"central difference {f:.10e} (rel {abs(a - f) / abs(f):.1e})", flush=True)
        assert a == pytest.approx(f, rel=1e-6)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16"])
@pytest.mark.parametrize("flags", [0, 2], ids=["fused", "unfused"])
def test_step_record_matches_step_and_oracle(precision, flags):
    """lbm_step_record advances the state exactly as lbm_step (raw state
    bitwise equal) and its record holds the forward quantities of the state
    it started from: phi, mu, p, S, jx, jy equal to the oracle's (FP64:
    1e-12 of each field's largest magnitude; FP32 arithmetic: 1e-5)."""
    from paper_1507_03521_amd import Lattice
    nx, ny = 300, 41
    pb = wl.droplet64().with_(nx=nx, ny=ny, bc=wl.WALLS_Y, gy=-1e-5, rho_ref=0.5)
    f, g = wl.random_state(nx, ny, seed=8)
    lats = []
    for _ in range(2):
        lat = Lattice(pb.as_dict(), np.full((ny, nx), 0.5), precision=precision, flags=flags,
                      device="cuda:0")
        lat.set_state(f, g)
        lats.append(lat)
    fs, gs = (t.cpu() for t in lats[0].get_state())   # stored (rounded) start state
    rec = lats[0].step_record()
    lats[1].step(1)
    assert torch.equal(lats[0].save_raw(), lats[1].save_raw())
    dt = torch.float64 if precision == "fp64" else torch.float32
    Ns = rec.numel() // (6 * (8 if precision == "fp64" else 4))
    planes = rec.view(dt)[:6 * Ns].view(6, Ns)[:, :nx * ny].double().cpu().view(6, ny, nx)
    m = O.macroscopic(fs, gs, O.coefficients_of(pb))
    tol = 1e-12 if precision == "fp64" else 1e-5
    for k, name in enumerate(("phi", "mu", "p", "S", "jx", "jy")):
        assert _rel(planes[k], m[name]) <= tol, name


@pytest.mark.parametrize("per_pass", [1, 2])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-4), ("fp16", 2e-3)])
def test_step_records_match_steps_and_oracle(precision, tol, per_pass):
    """lbm_step_records over 5 steps (two pairs and a single step with two
    steps per pass) launches what lbm_step launches: the raw state after it
    is bitwise equal to lbm_step's. Record k holds the forward quantities of
    the state after k steps: equal to the oracle's at step k (FP64 1e-12 of
    each field's largest magnitude; FP32 arithmetic 1e-4 and FP16 storage
    2e-3, which include the drift of the reduced-precision trajectory from
    the oracle's over 4 steps from a random state)."""
    from paper_1507_03521_amd import Lattice
    nx, ny, n = 300, 41, 5
    pb = wl.droplet64().with_(nx=nx, ny=ny, bc=wl.WALLS_Y, gy=-1e-5, rho_ref=0.5)
    f, g = wl.random_state(nx, ny, seed=18)
    lats = []
    for _ in range(2):
        lat = Lattice(pb.as_dict(), np.full((ny, nx), 0.5), precision=precision,
                      device="cuda:0")
        lat.set_pass(per_pass)
        lat.set_state(f, g)
        lats.append(lat)
    fs, gs = (t.cpu() for t in lats[0].get_state())   # stored (rounded) start state
    recs = [torch.empty(lats[0].record_bytes, dtype=torch.uint8, device="cuda:0")
            for _ in range(n)]
    lats[0].step_records(recs)
    lats[1].step(n)
    assert lats[0].time == n
    assert torch.equal(lats[0].save_raw(), lats[1].save_raw())
    dt = torch.float64 if precision == "fp64" else torch.float32
    co = O.coefficients_of(pb)
    state = (fs, gs)
    for k in range(n):
        Ns = recs[k].numel() // (6 * (8 if precision == "fp64" else 4))
        planes = recs[k].view(dt)[:6 * Ns].view(6, Ns)[:, :nx * ny].double().cpu().view(6, ny, nx)
        m = O.macroscopic(*state, co)
        errs = {name: _rel(planes[j], m[name])
                for j, name in enumerate(("phi", "mu", "p", "S", "jx", "jy"))}
        print(f"  record {k}:", {a: f"{b:.1e}" for a, b in errs.items()}, flush=True)
        assert max(errs.values()) <= tol, (k, errs)
        with torch.no_grad():
            state = O.step(*state, co)


def test_step_records_unfused_path():
    """lbm_step_records with LBM_FLAG_UNFUSED (one launch sequence per step,
    records from the unfused kernels): the raw state equals lbm_step's
    bitwise and the records equal those of the fused two-step passes to
    rounding (FP64 1e-13)."""
    from paper_1507_03521_amd import LBM_FLAG_UNFUSED
    nx, ny, n = 120, 37, 4
    pb = wl.droplet64().with_(nx=nx, ny=ny, bc=wl.WALLS_Y, gy=-1e-5, rho_ref=0.5)
    f, g = wl.random_state(nx, ny, seed=23)
    recs, raws = [], []
    for flags in (LBM_FLAG_UNFUSED, 0):
        a = _lattice(pb, np.full((ny, nx), 0.5), flags=flags)
        b = _lattice(pb, np.full((ny, nx), 0.5), flags=flags)
        a.set_state(f, g)
        b.set_state(f, g)
        r = [torch.empty(a.record_bytes, dtype=torch.uint8, device="cuda:0") for _ in range(n)]
        a.step_records(r)
        b.step(n)
        assert torch.equal(a.save_raw(), b.save_raw())
        recs.append(r)
        raws.append(a.save_raw())
    Ns = recs[0][0].numel() // 48
    for k in range(n):
        u = recs[0][k].view(torch.float64)[:6 * Ns].view(6, Ns)[:, :nx * ny]
        v = recs[1][k].view(torch.float64)[:6 * Ns].view(6, Ns)[:, :nx * ny]
        for j in range(6):
            assert _rel(u[j], v[j]) <= 1e-13, (k, j)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_step_records_large_lattice(precision):
    """Past the 4 GiB plane-group limit (the recording two-step kernel then
    addresses every plane with its own descriptor): two steps with records
    leave the raw state of two plain steps bitwise, and the two records
    match those of the unfused kernels to rounding: near rest p, S and j
    are small and formed by cancellation, so the bounds are the from-rest
    ones of the full-size forward checks (FP64 5e-12, FP32 2e-3 of each
    field's largest magnitude)."""
    from paper_1507_03521_amd import LBM_FLAG_UNFUSED
    nx, ny = (4000, 15000) if precision == "fp64" else (8000, 15000)
    print(f"case step records large {precision} {nx}x{ny}", flush=True)
    pb = wl.rt2048().with_(nx=nx, ny=ny)
    dev = torch.device("cuda:0")
    y = torch.arange(ny, device=dev, dtype=torch.float64)[:, None]
    x = torch.arange(nx, device=dev, dtype=torch.float64)[None, :]
    phi0 = 0.5 + 0.5 * torch.tanh(2.0 * (y - ny / 2 - 40.0 * torch.cos(2 * math.pi * 3 * x / nx))
                                  / pb.W)
    del x, y
    dt = torch.float64 if precision == "fp64" else torch.float32
    tol = 5e-12 if precision == "fp64" else 2e-3
    out = []
    for flags in (0, LBM_FLAG_UNFUSED):
        lat = _lattice(pb, phi0, precision=precision, flags=flags)
        lat.step(1)
        recs = [torch.empty(lat.record_bytes, dtype=torch.uint8, device=dev) for _ in range(2)]
        if flags == 0:
            ref = _lattice(pb, phi0, precision=precision)
            ref.step(1)
            ref.step(2)          # the same launches: one step, then one pair
            lat.step_records(recs)
            assert lat.pass_info()["steps"] == 2
            assert torch.equal(lat.save_raw(), ref.save_raw())
            ref.close()
            del ref
        else:
            lat.step_records(recs)
        out.append(recs)
        lat.close()
        del lat
        torch.cuda.empty_cache()
    Ns = out[0][0].numel() // (6 * (8 if precision == "fp64" else 4))
    N = nx * ny
    for k in range(2):
        u = out[0][k].view(dt)[:6 * Ns].view(6, Ns)[:, :N]
        v = out[1][k].view(dt)[:6 * Ns].view(6, Ns)[:, :N]
        for j in range(6):
            e = float((u[j] - v[j]).abs().max() / v[j].abs().max().clamp_min(1e-300))
            assert e <= tol, (k, j, e)
    del out
    torch.cuda.empty_cache()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-13), ("fp32", 1e-4), ("fp16", 1e-4)])
def test_adjoint_step_from_record_matches_raw_state_path(precision, tol):
    """One adjoint step from a record (lbm_step_record) equals the step from
    the raw state (lbm_adjoint_step, which recomputes the record with the
    unfused kernels): the two records differ only by the rounding of two
    evaluation orders, so FP64 cotangents agree within 1e-13 (sigma/M 1e-12)
    and FP32-arithmetic ones within 1e-4."""
    from paper_1507_03521_amd import Lattice
    nx, ny = 300, 41
    pb = wl.droplet64().with_(nx=nx, ny=ny, bc=wl.WALLS_Y, gy=-1e-5, rho_ref=0.5)
    f, g = wl.random_state(nx, ny, seed=9)
    rng = np.random.default_rng(3)
    fbar = rng.standard_normal((9, ny, nx))
    gbar = rng.standard_normal((9, ny, nx))
    zero = torch.zeros((ny, nx), dtype=torch.float64, device="cuda:0")
    out = []
    for use_record in (False, True):
        lat = _lattice(pb, np.full((ny, nx), 0.5), precision=precision)
        lat.set_state(f, g)
        raw = lat.save_raw().clone()
        rec = lat.step_record()
        lat.adjoint_begin(zero)
        lat.adjoint_set(fbar, gbar)
        if use_record:
            lat.adjoint_step_record(rec)
        else:
            lat.adjoint_step(raw)
        out.append(lat.adjoint_get())
    (f0, g0, s0, m0), (f1, g1, s1, m1) = out
    assert _rel(f1, f0) <= tol and _rel(g1, g0) <= tol
    assert s1 == pytest.approx(s0, rel=10 * tol) and m1 == pytest.approx(m0, rel=10 * tol)


ADJ_SHAPES = [(300, 41, wl.WALLS_Y, -1e-5), (520, 37, wl.PERIODIC, 0.0), (16, 13, wl.WALLS_Y, -1e-5),
              (3, 3, wl.PERIODIC, 0.0), (249, 20, wl.WALLS_Y, -2e-5)]


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-13), ("fp32", 1e-5)])
@pytest.mark.parametrize("nx,ny,bc,gy", ADJ_SHAPES)
def test_fused_adjoint_matches_three_kernel_path(precision, tol, nx, ny, bc, gy):
    """The fused adjoint kernel (default) and the three-kernel adjoint
    (LBM_FLAG_UNFUSED) on the same record and the same incoming cotangents:
    the same transposes in a different grouping, so the outgoing cotangents
    agree to rounding (FP64 1e-13, FP32 1e-5 of the largest magnitude) and
    the parameter sums to 10x that; shapes with one and several strips,
    ragged tails, walls and a lattice narrower than the halo."""
    from paper_1507_03521_amd import LBM_FLAG_UNFUSED
    print(f"case fused adjoint {precision} {nx}x{ny} bc={bc}", flush=True)
    pb = wl.droplet64().with_(nx=nx, ny=ny, bc=bc, gy=gy, rho_ref=0.5)
    f, g = wl.random_state(nx, ny, seed=nx + ny)
    rng = np.random.default_rng(nx)
    fbar = rng.standard_normal((9, ny, nx))
    gbar = rng.standard_normal((9, ny, nx))
    zero = torch.zeros((ny, nx), dtype=torch.float64, device="cuda:0")
    lat = _lattice(pb, np.full((ny, nx), 0.5), precision=precision)
    lat.set_state(f, g)
    rec = lat.step_record()
    out = []
    for flags in (0, LBM_FLAG_UNFUSED):
        la = _lattice(pb, np.full((ny, nx), 0.5), precision=precision, flags=flags)
        la.adjoint_begin(zero)
        la.adjoint_set(fbar, gbar)
        la.adjoint_step_record(rec)
        la.adjoint_step_record(rec)      # twice: the second reads the first's output
        out.append(la.adjoint_get())
    (f0, g0, s0, m0), (f1, g1, s1, m1) = out
    ef, eg = _rel(f0, f1), _rel(g0, g1)
    print(f"  fused vs three kernels: rel f {ef:.2e} g {eg:.2e}; sigma {s0:.6e} {s1:.6e}, "
          f"M {m0:.6e} {m1:.6e}", flush=True)
    assert ef <= tol and eg <= tol
    assert s0 == pytest.approx(s1, rel=10 * tol, abs=1e-300)
    assert m0 == pytest.approx(m1, rel=10 * tol, abs=1e-300)


@pytest.mark.parametrize("precision,nx,ny,tol", [("fp64", 4096, 8192, 1e-13),
                                                  ("fp32", 8000, 8000, 1e-5)])
def test_fused_adjoint_large_lattice_matches_three_kernels(precision, nx, ny, tol):
    """Where the 18 cotangent planes span 4 GiB or more (the fused adjoint
    then addresses every plane with its own descriptor): the 4096 x 8192
    rising-bubble lattice in FP64 and an 8000 x 8000 Rayleigh-Taylor
    lattice in FP32. Two adjoint steps from the record of a state one step
    past the initial interface, seeded with a random dL/dphi: the fused and
    three-kernel adjoints agree to rounding, as on small lattices."""
    from paper_1507_03521_amd import LBM_FLAG_UNFUSED
    print(f"case fused adjoint large {precision} {nx}x{ny}", flush=True)
    dev = torch.device("cuda:0")
    if precision == "fp64":
        pb = wl.bubble4096()
        assert (pb.nx, pb.ny) == (nx, ny)
        phi0 = torch.tensor(wl.phi0(pb), device=dev)
    else:
        pb = wl.rt2048().with_(nx=nx, ny=ny)
        y = torch.arange(ny, device=dev, dtype=torch.float64)[:, None]
        x = torch.arange(nx, device=dev, dtype=torch.float64)[None, :]
        h = ny / 2 + 40.0 * torch.cos(2 * math.pi * 3 * x / nx)
        phi0 = 0.5 + 0.5 * torch.tanh(2.0 * (y - h) / pb.W)
        del x, y, h
    lat = _lattice(pb, phi0, precision=precision)
    per_node, tb = (144, 8) if precision == "fp64" else (72, 4)
    assert 18 * (lat.state_bytes // per_node) * tb > 2**32 - 1
    lat.step(1)
    rec = lat.step_record()
    lat.close()
    del lat
    gen = torch.Generator(device=dev).manual_seed(7)
    seed = torch.randn((ny, nx), generator=gen, device=dev, dtype=torch.float64)
    out = []
    for flags in (0, LBM_FLAG_UNFUSED):
        la = _lattice(pb, phi0, precision=precision, flags=flags)
        la.adjoint_begin(seed)
        la.adjoint_step_record(rec)
        la.adjoint_step_record(rec)
        out.append(la.adjoint_get())
        la.close()
        del la
        torch.cuda.empty_cache()
    (f0, g0, s0, m0), (f1, g1, s1, m1) = out

    def rel_dev(a, b):   # on the device: the arrays hold ~300 M values each
        return float((a - b).abs().max() / b.abs().max())

    ef, eg = rel_dev(f0, f1), rel_dev(g0, g1)
    print(f"  fused vs three kernels: rel f {ef:.2e} g {eg:.2e}; sigma {s0:.8e} {s1:.8e}, "
          f"M {m0:.8e} {m1:.8e}", flush=True)
    assert ef <= tol and eg <= tol
    assert s0 == pytest.approx(s1, rel=10 * tol) and m0 == pytest.approx(m1, rel=10 * tol)
    del out, f0, g0, f1, g1, rec
    torch.cuda.empty_cache()


def test_adjoint_seed_reuses_the_workspace():
    """lbm_adjoint_seed restarts the adjoint with the bound workspace: a
    second loss after re-seeding gives bitwise the same cotangents and
    parameter sums as a fresh lbm_adjoint_begin with that loss; before any
    lbm_adjoint_begin it reports LBM_ESTATE."""
    from paper_1507_03521_amd import QilbmError
    nx, ny = 40, 33
    pb = wl.droplet64().with_(nx=nx, ny=ny, bc=wl.WALLS_Y, gy=-1e-5, rho_ref=0.5)
    f, g = wl.random_state(nx, ny, seed=12)
    rng = np.random.default_rng(4)
    s1 = torch.tensor(rng.standard_normal((ny, nx)), device="cuda:0")
    s2 = torch.tensor(rng.standard_normal((ny, nx)), device="cuda:0")

    def run(lat, seeds):
        lat.set_state(f, g)
        recs = [lat.step_record() for _ in range(3)]
        out = None
        for k, sd in enumerate(seeds):
            if k == 0:
                lat.adjoint_begin(sd)
            else:
                lat.adjoint_seed(sd)
            for rec in reversed(recs):
                lat.adjoint_step_record(rec)
            out = lat.adjoint_get()
        return out

    lat = _lattice(pb, np.full((ny, nx), 0.5))
    with pytest.raises(QilbmError) as err:
        lat.adjoint_seed(s1)
    assert err.value.status == -5
    a = run(lat, [s1, s2])
    b = run(_lattice(pb, np.full((ny, nx), 0.5)), [s2])
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    assert a[2] == b[2] and a[3] == b[3]
