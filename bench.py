"""Benchmark of the coupled phase-field LBE step on one MI355X.

Workload: the 2048 x 8192 Rayleigh-Taylor problem between bounce-back walls
(Atwood 0.5, Re 3000, Pe 1000, W 4), synthetic initial interface, no
datasets. A step is one coupled f+g update of the whole lattice (moments,
chemical potential, gradients, force, velocity, pressure, both collisions,
streaming). FP64 and FP32 run two steps per launch of the fused kernel
(the state between them stays on chip); FP16 storage one step per launch.

Printed: ONE JSON line. ``value`` is the FP32 rate in MLUPS (million lattice
updates per second), the median of five timed windows of ``--steps`` steps;
the line also carries the FP64 and FP16-storage rates, the adjoint/forward
step-time ratio, the roofline position of the fused kernel, the 4096 x 8192
rising bubble's FP32 rate and its gradient cost with checkpoint-and-recompute,
the stated error of FP32 and FP16 storage against FP64 (tip positions and
phi on the 256 x 1024 Rayleigh-Taylor problem over 10 000 steps), the
CPU-oracle rates (host model and core count stated), the rate with the
two-relaxation-time collision variant and the three-dimensional (D3Q19,
256^3 box) step's rates.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS (coupled f+g) FP64 vs FP32 at stated error; adjoint/forward step ratio"
PEAK_HBM_GBS = 8000.0
BYTES_PER_LU = {"fp64": 288, "fp32": 144, "fp16": 76}
PROFILE_TRAFFIC = {1: os.path.join(ROOT, "profiles", "fused_step_rt2048_fp32_pmc.txt"),
                   2: os.path.join(ROOT, "profiles", "fused_step2_rt2048_fp32_pmc.txt")}
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1507_03521_amd", "csrc", f)
                  for f in ("qilbm_kernels.hip", "qilbm_device.hpp")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


REPEATS = 5


def timed_runs(lat, steps: int, warmup: int, repeats: int = REPEATS):
    """``warmup`` untimed steps, then ``repeats`` timed windows of exactly
    ``steps`` steps, each bracketed by device synchronisations and timed with
    HIP events on the lattice's stream: ms per step of each window."""
    import torch
    lat.step(warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    runs = []
    for _ in range(repeats):
        torch.cuda.synchronize()
        start.record(lat.stream)
        lat.step(steps)
        stop.record(lat.stream)
        torch.cuda.synchronize()
        runs.append(start.elapsed_time(stop) / steps)
    return runs


def timed_steps(lat, steps: int, warmup: int):
    """Median ms per step over the timed windows of :func:`timed_runs`."""
    import statistics
    return statistics.median(timed_runs(lat, steps, warmup))


def run_precision(pb, phi0, precision, steps, warmup, seg_rows, pass_steps):
    from paper_1507_03521_amd import Lattice
    lat = Lattice(pb.as_dict(), phi0, precision=precision, device="cuda:0")
    if pass_steps:
        lat.set_pass(pass_steps, seg_rows if pass_steps == 2 else 0)
    if seg_rows and lat.pass_info()["steps"] == 1:
        lat.set_launch(seg_rows)
    m0 = lat.mass()
    runs = timed_runs(lat, steps, warmup)
    m1 = lat.mass()
    info = lat.pass_info()
    del lat
    return runs, m0, m1, info


def copy_gbps(reps: int = 10) -> float:
    """Achievable HBM rate of a plain device copy (1 GiB read + 1 GiB
    written per copy), HIP events around `reps` copies."""
    import torch
    src = torch.empty(1 << 28, dtype=torch.float32, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    gbps = 2.0 * (1 << 30) * reps / (a.elapsed_time(b) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbps


def run_trt(pb, phi0, steps: int, warmup: int, magic: float = 0.25):
    """FP32 step with the two-relaxation-time collision of f next to the BGK
    step on the same lattice, both two steps per launch of the fused kernel."""
    from paper_1507_03521_amd import Lattice
    N = pb.nx * pb.ny
    out = {"magic": magic, "precision": "fp32", "steps_per_launch": 2}
    for name, m in (("bgk", 0.0), ("trt", magic)):
        lat = Lattice(dict(pb.as_dict(), trt_magic=m), phi0, precision="fp32", device="cuda:0")
        lat.set_pass(2)
        ms = timed_steps(lat, steps, warmup)
        del lat
        out[name] = dict(mlups=round(N / ms / 1e3, 2), ms_per_step=round(ms, 5),
                         hbm_roofline_frac=round(BYTES_PER_LU["fp32"] * N / (ms * 1e-3) / 1e9
                                                 / PEAK_HBM_GBS, 4))
        log(f"  {name}: {ms:.4f} ms/step")
    return out


# D3Q19: 19 f and 19 g read and written once per node and step
BYTES_PER_LU_3D = {"fp64": 608, "fp32": 304}


def run_3d(steps: int, warmup: int):
    """The three-dimensional step on the 256^3 Rayleigh-Taylor box (walls
    normal to z): rate per precision, the step's algorithmic HBM rate (19 f
    and 19 g per node read and written once) and the totals' drift."""
    import workloads as wl
    from paper_1507_03521_amd import Lattice3D
    pb = wl.rt3d()
    phi0 = wl.phi0_3d(pb)
    N = pb.nx * pb.ny * pb.nz
    out = {"workload": "rt3d: Rayleigh-Taylor 256x256x256, walls in z, Atwood 0.5, "
                       "Re 3000, Pe 1000, W 4"}
    kernels = {"fp32": "k_zero_words (next step's phi words) + k3_fused (one z-sweep kernel)",
               "fp64": "k3_phi, k3_mu, k3_pf (pressure, f collision), k3_g (g collision)"}
    # key, storage precision, TRT magic parameter of the f collision (0: BGK)
    for key, prec, magic in (("fp32", "fp32", 0.0), ("fp64", "fp64", 0.0),
                             ("fp32_trt", "fp32", 0.25)):
        lat = Lattice3D(dict(pb.as_dict(), trt_magic=magic), phi0, precision=prec,
                        device="cuda:0")
        m0 = lat.mass()
        ms = timed_steps(lat, steps, warmup)
        m1 = lat.mass()
        del lat
        gbs = BYTES_PER_LU_3D[prec] * N / (ms * 1e-3) / 1e9
        out[key] = dict(kernels=kernels[prec], mlups=round(N / ms / 1e3, 2),
                        ms_per_step=round(ms, 5),
                        alg_gbps=round(gbs, 1), hbm_roofline_frac=round(gbs / PEAK_HBM_GBS, 4),
                        phi_total_drift=abs(m1[0] - m0[0]) / abs(m0[0]))
        if magic:
            out[key]["trt_magic"] = magic
        log(f"  3-D {key}: {ms:.4f} ms/step, {N / ms / 1e3:.1f} MLUPS")
    return out


def adjoint_ratio(pb, phi0, precision, fwd_ms, nadj=10):
    """Adjoint step time (from a step record) and, with the replay of the
    forward steps that write the records (as checkpoint-recompute does), over
    the forward step time."""
    import torch
    from paper_1507_03521_amd import Lattice
    lat = Lattice(pb.as_dict(), phi0, precision=precision, device="cuda:0")
    lat.step(5)
    rec = lat.step_record()
    seed = torch.zeros((pb.ny, pb.nx), dtype=torch.float64, device="cuda:0")
    lat.adjoint_begin(seed)
    lat.adjoint_step_record(rec)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(lat.stream)
    for _ in range(nadj):
        lat.adjoint_step_record(rec)
    stop.record(lat.stream)
    torch.cuda.synchronize()
    adj_ms = start.elapsed_time(stop) / nadj
    # the replay as checkpoint-and-recompute runs it: nadj steps with one
    # record each, pairs of steps per launch where the forward uses them
    recs = [torch.empty(lat.record_bytes, dtype=torch.uint8, device="cuda:0")
            for _ in range(nadj)]
    lat.step_records(recs)
    torch.cuda.synchronize()
    start.record(lat.stream)
    lat.step_records(recs)
    stop.record(lat.stream)
    torch.cuda.synchronize()
    rec_ms = start.elapsed_time(stop) / nadj
    del recs
    del lat
    # algorithmic bytes of one adjoint step per node: the record (phi, mu, p,
    # S, jx, jy) read, the 18 population cotangents read and written
    tb = 8 if precision == "fp64" else 4
    alg = (6 + 18 + 18) * tb
    n = pb.nx * pb.ny
    return dict(adjoint_ms_per_step=round(adj_ms, 4), ratio=round(adj_ms / fwd_ms, 3),
                ratio_with_recompute=round((adj_ms + rec_ms) / fwd_ms, 3), precision=precision,
                alg_bytes_per_lu=alg,
                hbm_roofline_frac=round(alg * n / (adj_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4))


def traffic_from_profile(pass_steps):
    """HBM bytes per launch of the fused kernel (one or two steps per pass)
    from the committed PMC summary, if it was taken on the current kernel
    source; else None."""
    path = PROFILE_TRAFFIC[pass_steps]
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha") != source_digest():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _oracle_crop_rate(pb, phi0, rows: int, target_s: float, threads: int):
    """Oracle rate (MLUPS) on the middle ``rows`` rows of the lattice (all
    columns, walls), with ``threads`` torch threads; steps chosen so that the
    timed part takes about ``target_s`` seconds (at least 2)."""
    import torch
    from oracle import qilbm_oracle as O
    saved = torch.get_num_threads()
    torch.set_num_threads(threads)
    try:
        y0 = pb.ny // 2 - rows // 2
        sub = pb.with_(ny=rows)
        co = O.coefficients_of(sub)
        with torch.no_grad():
            f, g = O.initial_state(phi0[y0:y0 + rows], co)
            t0 = time.perf_counter()
            f, g = O.step(f, g, co)               # first touch, also sizes the run
            one = time.perf_counter() - t0
            steps = max(2, min(50, int(target_s / max(one, 1e-6))))
            t0 = time.perf_counter()
            for _ in range(steps):
                f, g = O.step(f, g, co)
            dt = time.perf_counter() - t0
        return dict(value=round(sub.nx * rows * steps / dt / 1e6, 4), unit="MLUPS",
                    cores=torch.get_num_threads(), steps=steps, seconds=round(dt, 2))
    finally:
        torch.set_num_threads(saved)


def _oracle_droplet_run(threads: int, repeats: int = 3):
    """The 64x64 static droplet's full 2000-step run by the oracle; median
    wall time of up to ``repeats`` runs (one more run only while a run takes
    under 15 s)."""
    import statistics
    import torch
    import workloads as wl
    from oracle import qilbm_oracle as O
    pb = wl.droplet64()
    co = O.coefficients_of(pb)
    saved = torch.get_num_threads()
    torch.set_num_threads(threads)
    times = []
    try:
        for _ in range(repeats):
            t0 = time.perf_counter()
            with torch.no_grad():
                O.run(wl.phi0(pb), co, pb.steps)
            times.append(time.perf_counter() - t0)
            if times[-1] > 15.0:
                break
    finally:
        torch.set_num_threads(saved)
    med = statistics.median(times)
    return dict(value=round(pb.nx * pb.ny * pb.steps / med / 1e6, 4), unit="MLUPS",
                cores=threads, seconds=[round(t, 2) for t in times])


def cpu_baseline(pb, phi0, rows: int, target_s: float):
    """The oracle as it stands (plain PyTorch-CPU FP64, never tuned) on the
    host: the headline rate on a crop of the same workload (all columns, the
    middle ``rows`` rows between walls) with all the threads torch uses, the
    same crop with one thread, and the 64x64 droplet's full 2000-step run
    with one thread and all threads. Small lattices gain nothing from
    threads (each operation on 4096 nodes is shorter than a thread hand-off),
    so the crop is what shows the host's throughput."""
    import torch
    threads = torch.get_num_threads()
    allc = _oracle_crop_rate(pb, phi0, rows, target_s, threads)
    one = _oracle_crop_rate(pb, phi0, rows, target_s / 2, 1)
    c0 = {"all_threads": _oracle_droplet_run(threads), "single_thread": _oracle_droplet_run(1)}
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = None
    return dict(value=allc["value"], unit="MLUPS", cores=allc["cores"], kind="oracle",
                sample=f"{allc['steps']} FP64 steps of a {pb.nx}x{rows} crop (middle rows, "
                       f"walls) of the {pb.nx}x{pb.ny} Rayleigh-Taylor lattice, "
                       f"{allc['seconds']} s",
                cpu_model=_cpu_model(), host_cpus=os.cpu_count(), affinity_cpus=affinity,
                single_thread=dict(one, sample=f"{one['steps']} FP64 steps of the same crop"),
                droplet64_full_run=dict(c0, workload="64x64 static droplet, 2000 FP64 steps "
                                                     "(median of up to 3 runs)"))


def _crossings(col):
    """Positions of the phi = 1/2 crossings along a column (linear
    interpolation between nodes)."""
    c = col.cpu().numpy()
    return [y + (0.5 - c[y]) / (c[y + 1] - c[y]) for y in range(len(c) - 1)
            if (c[y] - 0.5) * (c[y + 1] - 0.5) < 0]


def interface_tips(phi, nx):
    """Spike tip: lowest phi = 1/2 crossing along x = nx/2 (heavy fluid
    falling); bubble tip: highest crossing along x = 0 (light fluid rising)."""
    lo, hi = _crossings(phi[:, nx // 2]), _crossings(phi[:, 0])
    return (min(lo) if lo else float("nan")), (max(hi) if hi else float("nan"))


def interface_tips_3d(phi):
    """The same in the 3-D box ([nz, ny, nx]): spike along the column
    (nx/2, ny/2), where the initial interface is lowest; bubble along (0, 0),
    where it is highest."""
    nz, ny, nx = phi.shape
    lo, hi = _crossings(phi[:, ny // 2, nx // 2]), _crossings(phi[:, 0, 0])
    return (min(lo) if lo else float("nan")), (max(hi) if hi else float("nan"))


def precision_study_3d(steps: int, every: int):
    """The 256^3 Rayleigh-Taylor box in FP64 and FP32: tip positions every
    ``every`` steps, drift of the phi total, and the deviation of the FP32
    run from the FP64 run."""
    import torch
    import workloads as wl
    from paper_1507_03521_amd import Lattice3D, QilbmError
    pb = wl.rt3d()
    phi0 = wl.phi0_3d(pb)
    t_unit = math.sqrt(abs(pb.gz) / pb.nx)        # t* = t sqrt(g / L), L = nx
    out, phi64, tips64 = {}, None, None
    for prec in ("fp64", "fp32"):
        lat = Lattice3D(pb.as_dict(), phi0, precision=prec, device="cuda:0")
        m0 = lat.mass()
        tips, diverged, t0, done = [], None, time.perf_counter(), 0
        while done < steps:
            n = min(every, steps - done)
            lat.step(n)
            done += n
            try:
                m = lat.mass()
            except QilbmError:
                m = (float("nan"),)
            if not math.isfinite(m[0]):
                diverged = done
                log(f"  3-D {prec}: non-finite state by step {done}")
                break
            s, b = interface_tips_3d(lat.moments(("phi",))["phi"])
            tips.append((done, round(s, 4), round(b, 4)))
            log(f"  3-D {prec}: step {done}/{steps} (t* {done * t_unit:.3f}) spike {s:.3f} "
                f"bubble {b:.3f}, {time.perf_counter() - t0:.0f} s")
        r = dict(tips_every=every, tips=tips, diverged_at=diverged,
                 seconds=round(time.perf_counter() - t0, 1))
        if diverged is None:
            r["phi_total_drift_rel"] = abs(lat.mass()[0] - m0[0]) / abs(m0[0])
            phi = lat.moments(("phi",))["phi"]
            if prec == "fp64":
                phi64, tips64 = phi, tips
            elif phi64 is not None:
                r["phi_max_abs_dev_vs_fp64"] = float((phi - phi64).abs().max())
                r["phi_rms_dev_vs_fp64"] = float((phi - phi64).square().mean().sqrt())
                r["tip_max_abs_dev_vs_fp64"] = max(
                    max(abs(a[1] - b[1]), abs(a[2] - b[2])) for a, b in zip(tips, tips64))
        out[prec] = r
        del lat
        torch.cuda.empty_cache()
    return dict(study="precision", workload="rt3d 256x256x256", steps=steps,
                t_star=round(steps * t_unit, 4), **out)


def precision_study(pb, phi0, steps: int, every: int):
    """Long run of the same workload in FP64, FP32 and FP16 storage: tip
    positions every ``every`` steps, mass drift, and the deviation of the
    reduced-precision runs from the FP64 GPU run."""
    import torch
    from paper_1507_03521_amd import Lattice, QilbmError
    out, phi64, tips64 = {}, None, None
    t_unit = math.sqrt(abs(pb.gy) / pb.nx)        # t* = t sqrt(g / L), L = nx
    for prec in ("fp64", "fp32", "fp16"):
        lat = Lattice(pb.as_dict(), phi0, precision=prec, device="cuda:0")
        m0 = lat.mass()
        tips, diverged, t0 = [], None, time.perf_counter()
        done = 0
        while done < steps:
            n = min(every, steps - done)
            lat.step(n)
            done += n
            try:
                lat.mass()
            except QilbmError:
                diverged = done
                log(f"  {prec}: non-finite state by step {done}")
                break
            s, b = interface_tips(lat.moments(("phi",))["phi"], pb.nx)
            tips.append((done, round(s, 4), round(b, 4)))
            log(f"  {prec}: step {done}/{steps} (t* {done * t_unit:.3f}) spike {s:.3f} "
                f"bubble {b:.3f}, {time.perf_counter() - t0:.0f} s")
        r = dict(tips_every=every, tips=tips, diverged_at=diverged,
                 seconds=round(time.perf_counter() - t0, 1))
        if diverged is None:
            m1 = lat.mass()
            r["mass_drift_rel"] = abs(m1[1] - m0[1]) / abs(m0[1])
            phi = lat.moments(("phi",))["phi"]
            if prec == "fp64":
                phi64, tips64 = phi, tips
            elif phi64 is not None:
                r["phi_max_abs_dev_vs_fp64"] = float((phi - phi64).abs().max())
                r["tip_max_abs_dev_vs_fp64"] = max(
                    max(abs(a[1] - b[1]), abs(a[2] - b[2])) for a, b in zip(tips, tips64))
        out[prec] = r
        del lat
        torch.cuda.empty_cache()
    return dict(study="precision", workload=f"{pb.name} {pb.nx}x{pb.ny}", steps=steps,
                t_star=round(steps * t_unit, 4), **out)


def exact_phi(lat):
    """phi = sum_i g_i from the stored populations, read back exactly in
    binary64 (not the compute type's moment)."""
    return lat.get_state()[1].sum(0)


def precision_window(steps: int, every: int):
    """The stated error of the reduced-precision runs on the 256 x 1024
    Rayleigh-Taylor problem (Re 3000, Pe 1000, walls): FP32 and FP16 storage
    against the FP64 GPU run (which test_gpu_physics compares with the
    oracle), from the same initial interface for ``steps`` steps: the
    largest deviation of the spike and bubble tips sampled every ``every``
    steps, the largest |phi - phi_FP64| at the end (phi summed exactly from
    the stored g) and the mass drift."""
    import torch
    import workloads as wl
    from paper_1507_03521_amd import Lattice
    pb = wl.rt256()
    phi0 = wl.phi0(pb)
    t_unit = math.sqrt(abs(pb.gy) / pb.nx)
    out, ref = {}, None
    for prec in ("fp64", "fp32", "fp16"):
        lat = Lattice(pb.as_dict(), phi0, precision=prec, device="cuda:0")
        m0 = lat.mass()
        tips, done = [], 0
        while done < steps:
            n = min(every, steps - done)
            lat.step(n)
            done += n
            tips.append(interface_tips(exact_phi(lat), pb.nx))
        m1 = lat.mass()
        phi = exact_phi(lat)
        r = dict(mass_drift_rel=abs(m1[1] - m0[1]) / abs(m0[1]),
                 spike_tip=round(tips[-1][0], 4), bubble_tip=round(tips[-1][1], 4))
        if ref is None:
            ref = (phi, tips)
        else:
            r["tip_max_abs_dev_vs_fp64"] = round(max(
                max(abs(a[0] - b[0]), abs(a[1] - b[1])) for a, b in zip(tips, ref[1])), 5)
            r["phi_max_abs_dev_vs_fp64"] = float((phi - ref[0]).abs().max())
        out[prec] = r
        del lat
        torch.cuda.empty_cache()
        log(f"  {prec}: {r}")
    return dict(workload="rt256: Rayleigh-Taylor 256x1024, walls in y, Atwood 0.5, Re 3000, "
                         "Pe 1000, W 4", steps=steps, t_star=round(steps * t_unit, 4),
                tips_every=every, initial_tips=(wl.rt256().meta["h0"] - wl.rt256().meta["amp"],
                                                wl.rt256().meta["h0"] + wl.rt256().meta["amp"]),
                **out)


def bubble_leg(steps: int, warmup: int, window: int, C: int):
    """The 4096 x 8192 rising bubble in FP32: the forward rate (two steps per
    launch), and the gradient's cost by checkpoint-and-recompute over a
    ``window`` of steps with a raw checkpoint every ``C`` steps (replay of
    each segment with step records, then the adjoint steps in reverse) over
    the forward window with its checkpoints."""
    import statistics
    import torch
    import workloads as wl
    from paper_1507_03521_amd import Lattice
    pb = wl.bubble4096()
    N = pb.nx * pb.ny
    lat = Lattice(pb.as_dict(), wl.phi0(pb), precision="fp32", device="cuda:0")
    runs = timed_runs(lat, steps, warmup)
    ms = statistics.median(runs)
    info = lat.pass_info()
    y = torch.arange(pb.ny, device="cuda:0", dtype=torch.float64)[:, None].expand(pb.ny, pb.nx)
    records = [torch.empty(lat.record_bytes, dtype=torch.uint8, device="cuda:0")
               for _ in range(C)]
    snaps = [torch.empty(lat.state_bytes, dtype=torch.uint8, device="cuda:0")
             for _ in range(-(-window // C))]
    lat.adjoint_begin((-y).contiguous())
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fwd, bwd = [], []
    for _ in range(REPEATS):
        t = lat.time
        torch.cuda.synchronize()
        ev0.record(lat.stream)
        for k in range(len(snaps)):
            lat.save_raw(snaps[k])
            lat.step(min(C, window - k * C))
        ev1.record(lat.stream)
        torch.cuda.synchronize()
        fwd.append(ev0.elapsed_time(ev1))
        lat.adjoint_seed((-y).contiguous())
        torch.cuda.synchronize()
        ev0.record(lat.stream)
        for k in reversed(range(len(snaps))):
            n = min(C, window - k * C)
            lat.load_raw(snaps[k], t + k * C)
            lat.step_records(records[:n])
            for j in reversed(range(n)):
                lat.adjoint_step_record(records[j])
        ev1.record(lat.stream)
        torch.cuda.synchronize()
        bwd.append(ev0.elapsed_time(ev1))
    fwd_ms, bwd_ms = statistics.median(fwd), statistics.median(bwd)
    del records, snaps, lat
    torch.cuda.empty_cache()
    return dict(workload="bubble4096: rising bubble 4096x8192, walls in y, R 256, Eo 10, "
                         "Mo 1e-3, W 5", precision="fp32",
                mlups=round(N / ms / 1e3, 2), ms_per_step=round(ms, 5),
                ms_per_step_runs=[round(r, 5) for r in runs], launch=info,
                hbm_roofline_frac=round(BYTES_PER_LU["fp32"] * N / (ms * 1e-3) / 1e9
                                        / PEAK_HBM_GBS, 4),
                adjoint=dict(window=window, checkpoint=C, forward_window_ms=round(fwd_ms, 3),
                             backward_ms=round(bwd_ms, 3),
                             ratio_with_recompute=round(bwd_ms / fwd_ms, 3)))


def adjoint_study(warm: int, window: int, C: int, precision: str = "fp64", h: float = 1e-6):
    """The 4096 x 8192 rising-bubble problem: ``warm`` forward steps, then
    the gradient of L = sum_x y (1 - phi_K) (the bubble's height moment)
    over the last ``window`` steps with respect to sigma and M (the state at
    the window start held fixed), by checkpoint-and-recompute with a raw
    checkpoint every ``C`` steps and C step records; timed against the
    plain forward window, and checked against central differences of the
    forward with relative step ``h`` (meaningful in FP64: in FP32 the
    rounding of L exceeds the differences)."""
    import torch
    import workloads as wl
    from paper_1507_03521_amd import Lattice
    pb = wl.bubble4096()
    dev = "cuda:0"
    lat = Lattice(pb.as_dict(), wl.phi0(pb), precision=precision, device=dev)
    t0 = time.perf_counter()
    done = 0
    while done < warm:
        n = min(5000, warm - done)
        lat.step(n)
        done += n
        torch.cuda.synchronize()
        log(f"  warm-up step {done}/{warm}, {time.perf_counter() - t0:.0f} s")
    start_raw = lat.save_raw().clone()
    y = torch.arange(pb.ny, device=dev, dtype=torch.float64)[:, None].expand(pb.ny, pb.nx)

    def loss_of(l):
        return float((y * (1.0 - l.moments(("phi",))["phi"])).sum())

    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # forward window with checkpoints
    torch.cuda.synchronize()
    ev0.record(lat.stream)
    snaps = []
    for t0 in range(0, window, C):
        snaps.append(lat.save_raw())
        lat.step(min(C, window - t0))
    ev1.record(lat.stream)
    torch.cuda.synchronize()
    fwd_ms = ev0.elapsed_time(ev1)
    L = loss_of(lat)
    # backward: replay each segment with records, adjoint steps in reverse
    records = [torch.empty(lat.record_bytes, dtype=torch.uint8, device=dev) for _ in range(C)]
    lat.adjoint_begin((-y).contiguous())
    torch.cuda.synchronize()
    ev0.record(lat.stream)
    for sgm in reversed(range(len(snaps))):
        a, b = sgm * C, min(sgm * C + C, window)
        lat.load_raw(snaps[sgm], warm + a)
        lat.step_records(records[:b - a])
        for t in reversed(range(a, b)):
            lat.adjoint_step_record(records[t - a])
    ev1.record(lat.stream)
    torch.cuda.synchronize()
    bwd_ms = ev0.elapsed_time(ev1)
    _, _, dsig, dM = lat.adjoint_get()
    peak_gb = torch.cuda.max_memory_allocated() / 1e9
    del snaps, records
    torch.cuda.empty_cache()

    def window_loss(sigma=pb.sigma, M=pb.M):
        l2 = Lattice(pb.with_(sigma=sigma, M=M).as_dict(), wl.phi0(pb), precision=precision,
                     device=dev)
        l2.load_raw(start_raw, warm)
        l2.step(window)
        v = loss_of(l2)
        l2.close()
        return v

    N = pb.nx * pb.ny
    out = dict(study="adjoint", workload=f"{pb.name} {pb.nx}x{pb.ny} rising bubble",
               precision=precision, warm_steps=warm, window=window, checkpoint=C,
               loss=L, dL_dsigma=dsig, dL_dM=dM)
    if h > 0:
        fd_sig = (window_loss(sigma=pb.sigma * (1 + h))
                  - window_loss(sigma=pb.sigma * (1 - h))) / (2 * h * pb.sigma)
        fd_M = (window_loss(M=pb.M * (1 + h)) - window_loss(M=pb.M * (1 - h))) / (2 * h * pb.M)
        out.update(fd_step=h, fd_dL_dsigma=fd_sig, fd_dL_dM=fd_M,
                   rel_dev_sigma=abs(dsig - fd_sig) / abs(fd_sig),
                   rel_dev_M=abs(dM - fd_M) / abs(fd_M))
    return dict(out, forward_window_ms=round(fwd_ms, 1), backward_ms=round(bwd_ms, 1),
                backward_over_forward=round(bwd_ms / fwd_ms, 3),
                forward_mlups=round(N * window / (fwd_ms * 1e-3) / 1e6, 1),
                peak_device_memory_gb=round(peak_gb, 1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--seg-rows", type=int, default=0)
    ap.add_argument("--pass-steps", type=int, choices=[1, 2], default=0,
                    help="time steps per fused launch (default: the library's choice per "
                         "precision: 2 for fp64 and fp32, 1 for fp16 storage)")
    ap.add_argument("--only", choices=["fp32", "fp64", "fp16"], default=None,
                    help="time one precision only (for profiler runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-3d", action="store_true",
                    help="skip the three-dimensional (D3Q19) 256^3 leg")
    ap.add_argument("--steps-3d", type=int, default=200)
    ap.add_argument("--no-trt", action="store_true",
                    help="skip the two-relaxation-time (FP32) leg")
    ap.add_argument("--cpu-rows", type=int, default=512,
                    help="rows of the crop of the workload that the CPU oracle steps")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="about how long the oracle's all-thread crop run takes")
    ap.add_argument("--no-bubble", action="store_true",
                    help="skip the 4096x8192 rising-bubble leg (rate and adjoint cost)")
    ap.add_argument("--bubble-window", type=int, nargs=2, default=(32, 16),
                    metavar=("WINDOW", "C"))
    ap.add_argument("--no-precision-window", action="store_true",
                    help="skip the FP32/FP16-vs-FP64 error run on the 256x1024 lattice")
    ap.add_argument("--window-steps", type=int, default=10000)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (PMC byte-counter calibration)")
    ap.add_argument("--precision-study", type=int, default=0, metavar="STEPS",
                    help="instead of timing: run STEPS steps in each precision and print "
                         "tip positions, mass drift and deviation from FP64 (one JSON line)")
    ap.add_argument("--precision-study-3d", type=int, default=0, metavar="STEPS",
                    help="instead of timing: the same for the 256^3 box in FP64 and FP32")
    ap.add_argument("--study-every", type=int, default=5000)
    ap.add_argument("--adjoint-study", type=int, nargs=3, default=None,
                    metavar=("WARM", "WINDOW", "C"),
                    help="instead of timing: 4096x8192 bubble, WARM forward steps, then the "
                         "sigma/M gradient over the last WINDOW steps with checkpoints every C "
                         "(one JSON line)")
    ap.add_argument("--study-precision", choices=["fp64", "fp32", "fp16"], default="fp64")
    ap.add_argument("--fd-step", type=float, default=1e-4,
                    help="relative central-difference step of the adjoint study (0: none)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              f"(the multi-GPU decomposition is a design only)", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as wl

    pb = wl.rt2048()
    phi0 = wl.phi0(pb)
    N = pb.nx * pb.ny
    if args.adjoint_study:
        print(json.dumps(adjoint_study(*args.adjoint_study, precision=args.study_precision,
                                       h=args.fd_step)), flush=True)
        return
    if args.precision_study:
        print(json.dumps(precision_study(pb, phi0, args.precision_study, args.study_every)),
              flush=True)
        return
    if args.precision_study_3d:
        print(json.dumps(precision_study_3d(args.precision_study_3d, args.study_every)),
              flush=True)
        return
    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda:0").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 x 1 GiB read + 1 GiB write")

    achievable = copy_gbps()
    log(f"device copy: {achievable:.0f} GB/s")
    precisions = [args.only] if args.only else ["fp32", "fp64", "fp16"]
    res = {}
    import statistics
    for prec in precisions:
        log(f"timing {prec}: {REPEATS} x {args.steps} steps after {args.warmup} warm-up")
        runs, m0, m1, info = run_precision(pb, phi0, prec, args.steps, args.warmup,
                                           args.seg_rows, args.pass_steps)
        ms = statistics.median(runs)
        res[prec] = dict(ms=ms, runs=runs, m0=m0, m1=m1, info=info)
        log(f"  {prec}: {ms:.4f} ms/step (median; runs {[round(r, 4) for r in runs]}), "
            f"{N / ms / 1e3:.1f} MLUPS, launch {info}")

    def entry(prec):
        r = res[prec]
        return dict(mlups=round(N / r["ms"] / 1e3, 2), ms_per_step=round(r["ms"], 5),
                    ms_per_step_runs=[round(x, 5) for x in r["runs"]],
                    steps_per_launch=r["info"]["steps"],
                    hbm_roofline_frac=round(BYTES_PER_LU[prec] * N / (r["ms"] * 1e-3) / 1e9
                                            / PEAK_HBM_GBS, 4),
                    mass_drift_rel=abs(r["m1"][1] - r["m0"][1]) / abs(r["m0"][1]))

    main_prec = args.only or "fp32"
    ms = res[main_prec]["ms"]
    # per launch of the fused kernel: it advances the lattice by `per` steps;
    # algorithmic bytes = B/LU x nodes x steps (what `per` one-step launches
    # would move), over the launch's average duration
    per = res[main_prec]["info"]["steps"]
    alg_bytes = BYTES_PER_LU[main_prec] * N * per
    achieved = alg_bytes / (ms * per * 1e-3) / 1e9
    traffic = traffic_from_profile(per) if main_prec == "fp32" else None
    kname = "k_step2_fused" if per == 2 else "k_step_fused"
    line = {
        "metric": METRIC,
        "value": round(N / ms / 1e3, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64", "fp16": "f16-store/f32"}[main_prec],
        "data": "synthetic",
        "config": {"workload": "rt2048: Rayleigh-Taylor 2048x8192, walls in y, Atwood 0.5, "
                               "Re 3000, Pe 1000, W 4",
                   "nx": pb.nx, "ny": pb.ny, "precision": main_prec,
                   "launch": res[main_prec]["info"]},
        "roofline": {"bound": "hbm", "kernel": f"{kname}<{main_prec}>",
                     "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "steps_per_launch": per,
                     "ms_per_launch": round(ms * per, 5),
                     "alg_bytes_per_launch": alg_bytes,
                     "traffic": None if traffic is None else round(traffic, 0),
                     "achievable_copy_gbps": round(achievable, 1),
                     "moved_gbps": None if traffic is None
                     else round(traffic / (ms * per * 1e-3) / 1e9, 1)},
    }
    for prec in res:
        line[{"fp64": "fp64", "fp32": "fp32", "fp16": "fp16_store"}[prec]] = entry(prec)
    if not args.no_adjoint and main_prec in ("fp32", "fp64"):
        log("timing adjoint")
        line["adjoint"] = adjoint_ratio(pb, phi0, main_prec, ms)
    if not args.no_trt:
        log("timing the two-relaxation-time collision variant")
        line["trt"] = run_trt(pb, phi0, 200, 20)
    if not args.no_bubble and not args.only:
        log("timing the 4096x8192 rising bubble (FP32 rate, adjoint with checkpoints)")
        line["bubble4096"] = bubble_leg(args.steps, args.warmup, *args.bubble_window)
    if not args.no_precision_window and not args.only:
        log(f"reduced-precision error window: 256x1024, {args.window_steps} steps")
        line["precision_error"] = precision_window(args.window_steps,
                                                   max(1, args.window_steps // 10))
    if not args.no_3d:
        log("timing the three-dimensional step")
        line["d3q19"] = run_3d(args.steps_3d, max(1, args.steps_3d // 10))
    if not args.no_cpu_baseline:
        log("timing CPU oracle sample")
        line["cpu_baseline"] = cpu_baseline(pb, phi0, args.cpu_rows, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
