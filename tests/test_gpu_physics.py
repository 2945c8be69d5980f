"""Physics checks of the GPU path at the settings the paper and the workload
definitions state, where the CPU oracle would be too slow for the step
counts involved. Diagnostics that need the oracle's definitions (the Laplace
pressure of Sec. IV.B) are evaluated with the oracle on the GPU's state."""
import json
import math
import os

import numpy as np
import pytest
import torch

import workloads as wl
from oracle import qilbm_oracle as O

pytestmark = pytest.mark.gpu
torch.set_num_threads(4)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _lattice(pb, phi0, precision="fp64", flags=0):
    from paper_1507_03521_amd import Lattice
    return Lattice(pb.as_dict(), phi0, precision=precision, flags=flags, device="cuda:0")


def _with_mobility(pb):
    beta = O.coefficients_of(pb.with_(M=1.0)).beta
    return pb.with_(M=pb.meta["lambda_beta"] / beta)


def _laplace_jump(lat, pb, steps, every=200):
    """R * Delta P averaged over the last third of the run (the pressure
    jump breathes with a slowly damped acoustic mode)."""
    co = O.coefficients_of(pb)
    samples = []
    done = 0
    start = steps - steps // 3
    while done < steps:
        lat.step(every)
        done += every
        if done >= start:
            f, g = (t.cpu() for t in lat.get_state())
            P = O.laplace_pressure(f, g, co)
            phi = g.sum(0)
            R = math.sqrt(float(phi.sum()) / math.pi)
            samples.append((R, float(P[phi > 0.99].mean() - P[phi < 0.01].mean())))
    R = np.mean([s[0] for s in samples])
    dP = np.mean([s[1] for s in samples])
    return R, dP


@pytest.mark.parametrize("Pe,Cn", [(50, 4), (125, 4), (200, 4), (200, 6), (200, 8)])
def test_table1_surface_tension(Pe, Cn):
    """Sec. IV.B, Table 1: sigma_LBM = R * Delta P for droplets of radius
    20..40 on a 100x100 lattice (rho_A = 1, rho_B = 0.2, tau = 1,
    sigma = 1e-3). The paper prints one value per (Pe, Cn), 0.989..0.993e-3,
    without saying which radius; R * Delta P drifts with R by an O(W/R)
    finite-width term, so the value is taken at the largest droplet (R = 40,
    nearest the sharp-interface limit) and must agree within 2 %; every
    radius must satisfy the Laplace law within 6 %."""
    gold = {(r["Pe"], r["Cn"]): r["sigma_LBM"]
            for r in json.load(open(os.path.join(GOLDEN, "table1_surface_tension.json")))["rows"]}
    sig = {}
    for R0 in (20.0, 25.0, 30.0, 35.0, 40.0):
        pb = _with_mobility(wl.laplace_droplet(R=R0, Pe=Pe, Cn=Cn))
        lat = _lattice(pb, wl.phi0(pb))
        R, dP = _laplace_jump(lat, pb, 24000)
        sig[R0] = R * dP
    print(f"Pe {Pe} Cn {Cn}: R*dP/1e-3 per radius {[round(v / 1e-3, 4) for v in sig.values()]}, "
          f"paper {gold[(Pe, Cn)] / 1e-3:.3f}", flush=True)
    assert sig[40.0] == pytest.approx(gold[(Pe, Cn)], rel=0.02)
    for v in sig.values():
        assert v == pytest.approx(1e-3, rel=0.06)


def _tips(phi, nx):
    """Spike tip: lowest phi = 1/2 crossing along x = nx/2 (heavy fluid
    falling); bubble tip: highest crossing along x = 0 (light fluid rising)."""
    def crossings(col):
        c = col.cpu().numpy()
        out = []
        for y in range(len(c) - 1):
            if (c[y] - 0.5) * (c[y + 1] - 0.5) < 0:
                out.append(y + (0.5 - c[y]) / (c[y + 1] - c[y]))
        return out
    return min(crossings(phi[:, nx // 2])), max(crossings(phi[:, 0]))


def test_rayleigh_taylor_256x1024_fp64_vs_oracle():
    """The 256x1024 Rayleigh-Taylor problem at full size: 200 FP64 steps
    equal the oracle's (f within 2e-11, g within 1e-12)."""
    pb = wl.rt256()
    phi0 = wl.phi0(pb)
    lat = _lattice(pb, phi0)
    lat.step(200)
    fg, gg = (t.cpu() for t in lat.get_state())
    torch.set_num_threads(16)
    with torch.no_grad():
        fr, gr = O.run(phi0, O.coefficients_of(pb), 200)
    ef = float((fg - fr).abs().max() / fr.abs().max())
    eg = float((gg - gr).abs().max() / gr.abs().max())
    print(f"rt256 200 steps: rel f {ef:.2e} g {eg:.2e}", flush=True)
    assert ef <= 2e-11 and eg <= 1e-12


def test_rayleigh_taylor_256x1024_tips_fp32_vs_fp64():
    """The 256x1024 problem over 10000 steps (t* = t sqrt(g/L) = 1.56; with
    the paper's BGK collision it diverges later, see the next test): spike
    and bubble tips of the FP32 run within 0.05 lattice units of the FP64
    run, mass conserved (FP64 to 1e-12, FP32 exactly), spike falling and
    bubble rising."""
    pb = wl.rt256()
    phi0 = wl.phi0(pb)
    res = {}
    for prec in ("fp64", "fp32"):
        lat = _lattice(pb, phi0, precision=prec)
        m0 = lat.mass()
        tips = []
        for k in range(4):
            lat.step(2500)
            tips.append(_tips(lat.moments(("phi",))["phi"], pb.nx))
        res[prec] = (tips, m0, lat.mass())
        print(prec, "tips (spike, bubble) every 2500 steps:",
              [tuple(round(v, 3) for v in t) for t in tips], flush=True)
    for (s64, b64), (s32, b32) in zip(res["fp64"][0], res["fp32"][0]):
        assert abs(s64 - s32) <= 0.05 and abs(b64 - b32) <= 0.05
    for prec in ("fp64", "fp32"):
        _, m0, m1 = res[prec]
        assert abs(m1[0] - m0[0]) <= 1e-12 * m0[0]
    spike, bubble = res["fp64"][0][-1]
    h0, amp = pb.meta["h0"], pb.meta["amp"]
    assert spike < h0 - amp - 20 and bubble > h0 + amp + 10


def test_rayleigh_taylor_re3000_bgk_divergence_is_reported():
    """At Re = 3000 on 256x1024 (tau_f = 0.5102) the BGK scheme is unstable:
    the run is finite at step 10000 and non-finite by step 15000, and
    lbm_mass reports it as LBM_EDIVERGED (the library's failure signal;
    a multiple-relaxation-time collision would be the remedy and is not part
    of the paper's scheme)."""
    from paper_1507_03521_amd import QilbmError
    pb = wl.rt256()
    lat = _lattice(pb, wl.phi0(pb))
    lat.step(10000)
    lat.mass()
    lat.step(5000)
    with pytest.raises(QilbmError) as err:
        lat.mass()
    assert err.value.status == -4


def test_phase_separation_quasi_vs_incompressible_form():
    """Sec. IV.D workload (100x100 periodic, lambda*beta = 0.02, W = 4,
    rho_r = 2 so gamma = 1): GPU matches the oracle for both the
    quasi-incompressible step and the gamma-ablation over 100 steps, and the
    two forms separate at different rates (the paper's quasi/incompressible
    difference when mu is not uniform)."""
    from paper_1507_03521_amd import LBM_FLAG_NO_GAMMA
    pb = _with_mobility(wl.phase_separation(lambda_beta=0.02, W=4.0, rho_r=2.0))
    phi0 = wl.phi0(pb)
    var = {}
    for flags, no_gamma in ((0, False), (LBM_FLAG_NO_GAMMA, True)):
        lat = _lattice(pb, phi0, flags=flags)
        lat.step(100)
        fg, gg = (t.cpu() for t in lat.get_state())
        with torch.no_grad():
            fr, gr = O.run(phi0, O.coefficients_of(pb, no_gamma=no_gamma), 100)
        assert float((gg - gr).abs().max() / gr.abs().max()) <= 1e-12
        assert float((fg - fr).abs().max() / fr.abs().max()) <= 2e-11
        lat.step(900)
        var[no_gamma] = float(lat.moments(("phi",))["phi"].var())
    print("phi variance after 1000 steps: quasi", var[False], "incompressible form", var[True], flush=True)
    assert var[False] > 1.05 * var[True]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_static_droplet_64_laplace_mass_spurious_velocity(precision):
    """The 64x64 static droplet (R = 16, W = 4, sigma = 0.01, rho 1 / 0.1,
    M = 0.1, tau = 0.8) after 2000 steps on the GPU: total phi conserved
    (FP64 to 1e-12 relative, FP32 exactly in fixed point), the Laplace
    pressure jump within 5 % of sigma / R (Sec. IV.B; R from the droplet
    area, averaged over the last third of the run) and the largest spurious
    velocity reported (bounded by 1e-3 lattice units)."""
    pb = wl.droplet64()
    lat = _lattice(pb, wl.phi0(pb), precision=precision)
    m0 = lat.mass()
    R, dP = _laplace_jump(lat, pb, pb.steps, every=100)
    m1 = lat.mass()
    mo = lat.moments(("ux", "uy"))
    umax = float(torch.sqrt(mo["ux"] ** 2 + mo["uy"] ** 2).max())
    print(f"{precision}: R {R:.3f}, dP {dP:.4e} vs sigma/R {pb.sigma / R:.4e} "
          f"({dP * R / pb.sigma - 1:+.2%}), max |u| {umax:.2e}, "
          f"mass drift {abs(m1[0] - m0[0]) / m0[0]:.1e}", flush=True)
    if precision == "fp64":
        assert abs(m1[0] - m0[0]) <= 1e-12 * abs(m0[0])
    else:
        assert m1[0] == m0[0]
    assert dP == pytest.approx(pb.sigma / R, rel=0.05)
    assert umax <= 1e-3
