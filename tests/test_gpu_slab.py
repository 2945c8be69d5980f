"""One GPU's share of a y-slab decomposition, at its real shape.

A multi-GPU run of the 2-D step would give each GPU a band of rows and
exchange ghost rows before each two-step pass (the two-step kernel reads 8
rows beyond its segment: 4 per step, the distance from which a node's new
state draws). Here the exchange is a local copy: an interior band of the
4096 x 8192 rising-bubble lattice plus 8 ghost rows per side is cut into a
lattice of its own (periodic in y; the wrap only touches ghost rows), one
two-step pass runs on both, and the band's rows must equal the full
lattice's bit for bit (the same kernel does the same arithmetic per node,
whatever the lattice height, y boundary or segment layout).
"""
import pytest
import torch

import workloads as wl

pytestmark = pytest.mark.gpu

GHOST = 8


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_y_slab_with_ghost_rows_reproduces_the_full_lattice(precision):
    from paper_1507_03521_amd import Lattice
    pb = wl.bubble4096()
    full = Lattice(pb.as_dict(), wl.phi0(pb), precision=precision, device="cuda:0")
    full.step(200)                                   # a developed state
    y0, y1 = 1024, 2048                              # the band holding the bubble
    f, g = full.get_state()
    band = pb.with_(ny=(y1 - y0) + 2 * GHOST, bc=wl.PERIODIC)
    slab = Lattice(band.as_dict(), g[:, y0 - GHOST:y1 + GHOST].sum(0), precision=precision,
                   device="cuda:0")
    slab.set_state(f[:, y0 - GHOST:y1 + GHOST], g[:, y0 - GHOST:y1 + GHOST])
    del f, g
    assert full.pass_info()["steps"] == 2 and slab.pass_info()["steps"] == 2
    full.step(2)
    slab.step(2)
    ff, gf = full.get_state()
    fs, gs = slab.get_state()
    assert torch.equal(fs[:, GHOST:GHOST + (y1 - y0)], ff[:, y0:y1])
    assert torch.equal(gs[:, GHOST:GHOST + (y1 - y0)], gf[:, y0:y1])
    del ff, gf, fs, gs
    # the band's own rate at this shape (4096 x 1040, two steps per pass)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(slab.stream)
    slab.step(200)
    b.record(slab.stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / 200
    print(f"{precision} slab 4096x{band.ny}: {ms:.4f} ms/step, "
          f"{4096 * band.ny / ms / 1e6:.2f} GLUPS", flush=True)
