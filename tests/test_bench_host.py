"""Host-side checks of bench.py (no GPU): the one-GPU contract, the interface
tip detection of the stated-error leg, the lookup of the HBM traffic in a
counter summary, and the CPU oracle's crop timing."""
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import workloads as wl  # noqa: E402


def test_more_than_one_gpu_is_refused_before_any_device_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT, timeout=300)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def test_interface_tips_of_linear_profiles():
    """phi linear in y near the crossings: the linear interpolation between
    nodes is exact, so the spike tip (lowest phi = 1/2 crossing along
    x = nx/2) and the bubble tip (highest crossing along x = 0) come out at
    the constructed positions; the other columns do not count."""
    ny, nx = 1024, 16
    y = torch.arange(ny, dtype=torch.float64)
    phi = torch.zeros((ny, nx), dtype=torch.float64)
    phi[:, :] = torch.clamp(0.5 + (y[:, None] - 512.0) / 32.0, 0.0, 1.0)
    phi[:, nx // 2] = torch.clamp(0.5 + (y - 300.25) / 32.0, 0.0, 1.0)
    phi[:, 0] = torch.clamp(0.5 + (y - 700.75) / 32.0, 0.0, 1.0)
    spike, bubble = bench.interface_tips(phi, nx)
    assert spike == pytest.approx(300.25, abs=1e-12)
    assert bubble == pytest.approx(700.75, abs=1e-12)
    # several crossings in a column: the lowest one for the spike, the
    # highest for the bubble
    phi[:, nx // 2] = 0.5 + 0.4 * torch.cos(2 * np.pi * (y + 0.125) / 256.0)
    lo = bench._crossings(phi[:, nx // 2])
    assert len(lo) == 8
    spike, _ = bench.interface_tips(phi, nx)
    assert spike == min(lo)
    # a column without a crossing gives nan, not an error
    phi[:, 0] = 0.25
    assert np.isnan(bench.interface_tips(phi, nx)[1])


def test_interface_tips_3d_columns():
    nz, ny, nx = 64, 8, 8
    z = torch.arange(nz, dtype=torch.float64)
    phi = torch.zeros((nz, ny, nx), dtype=torch.float64)
    phi[:, ny // 2, nx // 2] = torch.clamp(0.5 + (z - 20.5) / 8.0, 0.0, 1.0)
    phi[:, 0, 0] = torch.clamp(0.5 + (z - 40.25) / 8.0, 0.0, 1.0)
    spike, bubble = bench.interface_tips_3d(phi)
    assert spike == pytest.approx(20.5, abs=1e-12)
    assert bubble == pytest.approx(40.25, abs=1e-12)


def test_traffic_is_taken_only_from_a_summary_of_the_current_sources(tmp_path, monkeypatch):
    """The bench reports the counter-derived HBM bytes per launch only when
    the summary names the digest of the kernel sources it was taken on."""
    digest = bench.source_digest()
    assert len(digest) == 16 and int(digest, 16) >= 0
    good = tmp_path / "good.txt"
    good.write_text(f"# a comment = ignored\nkernel_source_sha = {digest}\n"
                    "hbm_bytes_per_launch = 2524912486\n")
    stale = tmp_path / "stale.txt"
    stale.write_text("kernel_source_sha = 0000000000000000\nhbm_bytes_per_launch = 1\n")
    monkeypatch.setitem(bench.PROFILE_TRAFFIC, 2, str(good))
    monkeypatch.setitem(bench.PROFILE_TRAFFIC, 1, str(stale))
    assert bench.traffic_from_profile(2) == 2524912486.0
    assert bench.traffic_from_profile(1) is None
    monkeypatch.setitem(bench.PROFILE_TRAFFIC, 1, str(tmp_path / "missing.txt"))
    assert bench.traffic_from_profile(1) is None


def test_committed_summaries_parse_to_plausible_traffic():
    """The committed FP32 counter summaries, when they match the sources:
    two steps per launch move about one read and one write of the state
    (0.5 of the algorithmic bytes of two steps), one step a little more
    than its algorithmic bytes."""
    alg = {1: 144 * 2048 * 8192, 2: 2 * 144 * 2048 * 8192}
    for steps, (lo, hi) in ((1, (1.0, 1.3)), (2, (0.5, 0.65))):
        t = bench.traffic_from_profile(steps)
        if t is None:
            continue
        assert lo * alg[steps] < t < hi * alg[steps]


def test_oracle_crop_rate_on_a_few_rows():
    pb = wl.rt2048()
    phi0 = wl.phi0(pb)
    r = bench._oracle_crop_rate(pb, phi0, rows=8, target_s=0.05, threads=1)
    assert r["unit"] == "MLUPS" and r["cores"] == 1
    assert r["steps"] >= 2 and r["value"] > 0.0 and r["seconds"] >= 0.0
    assert torch.get_num_threads() >= 1
