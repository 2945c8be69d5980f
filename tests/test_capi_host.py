"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every symbol include/*.h declares, and rejects invalid arguments before any
device work."""
import ctypes
import glob
import os
import re
from ctypes import c_int32, byref, c_double, c_void_p

import pytest

import workloads as wl
from paper_1507_03521_amd import _lib

HEADERS = sorted(glob.glob(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                                        "include", "*.h")))


def _declared():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(lbm3?_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(HEADERS) >= 2 and len(names) >= 29
    assert any(n.startswith("lbm3_") for n in names)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.SIGNATURES), set(names) ^ set(_lib.SIGNATURES)


def _params(**kw):
    d = wl.droplet64().as_dict()
    d.update(kw)
    return _lib.make_params(d)


@pytest.mark.parametrize("bad", [dict(nx=2), dict(ny=0), dict(tau_f=0.5), dict(tau_g=0.4),
                                 dict(sigma=0.0), dict(W=-1.0), dict(M=0.0), dict(rho_B=0.0),
                                 dict(rho_A=float("nan")), dict(gx=float("inf")), dict(bc=7)])
def test_invalid_parameters_rejected(lib, bad):
    p = _params(**bad)
    assert lib.lbm_workspace_bytes(byref(p)) == 0
    out = (c_double * 6)()
    assert lib.lbm_coefficients(byref(p), out) == _lib.LBM_EINVAL
    ctx = c_void_p()
    assert lib.lbm_init(byref(ctx), byref(p), c_void_p(256), 1 << 30, c_void_p(256), None) == _lib.LBM_EINVAL
    assert not ctx.value


def test_bad_precision_and_flags_rejected(lib):
    p = _params()
    p.precision = 3
    assert lib.lbm_workspace_bytes(byref(p)) == 0
    p = _params()
    p.flags = 64
    assert lib.lbm_workspace_bytes(byref(p)) == 0


def test_init_argument_checks(lib):
    p = _params()
    nbytes = lib.lbm_workspace_bytes(byref(p))
    assert nbytes > 0
    ctx = c_void_p()
    # null workspace, null phi0, misaligned workspace, short workspace
    assert lib.lbm_init(byref(ctx), byref(p), None, nbytes, c_void_p(256), None) == _lib.LBM_EINVAL
    assert lib.lbm_init(byref(ctx), byref(p), c_void_p(256), nbytes, None, None) == _lib.LBM_EINVAL
    assert lib.lbm_init(byref(ctx), byref(p), c_void_p(264), nbytes, c_void_p(256), None) == _lib.LBM_EINVAL
    assert lib.lbm_init(byref(ctx), byref(p), c_void_p(256), nbytes - 1, c_void_p(256), None) == _lib.LBM_ENOMEM
    assert lib.lbm_init(None, byref(p), c_void_p(256), nbytes, c_void_p(256), None) == _lib.LBM_EINVAL


def test_null_context_calls(lib):
    assert lib.lbm_step(None, 1) == _lib.LBM_EINVAL
    assert lib.lbm_mass(None, (c_double * 4)()) == _lib.LBM_EINVAL
    assert lib.lbm_moments(None, *([None] * 6)) == _lib.LBM_EINVAL
    assert lib.lbm_get_state(None, None, None) == _lib.LBM_EINVAL
    assert lib.lbm_time(None) == -1
    assert lib.lbm_state_bytes(None) == 0
    assert lib.lbm_adjoint_step(None, None) == _lib.LBM_EINVAL
    assert lib.lbm_adjoint_seed(None, None) == _lib.LBM_EINVAL
    assert lib.lbm_adjoint_step_record(None, None) == _lib.LBM_EINVAL
    assert lib.lbm_step_record(None, None) == _lib.LBM_EINVAL
    assert lib.lbm_record_bytes(None) == 0
    assert lib.lbm_set_launch(None, 0) == _lib.LBM_EINVAL
    assert lib.lbm_launch_info(None, (c_int32 * 4)()) == _lib.LBM_EINVAL
    assert lib.lbm_set_pass(None, 2, 0) == _lib.LBM_EINVAL
    assert lib.lbm_pass_info(None, (c_int32 * 5)()) == _lib.LBM_EINVAL
    assert lib.lbm_step_records(None, 1, (c_void_p * 1)()) == _lib.LBM_EINVAL
    lib.lbm_destroy(None)
    assert lib.lbm_strerror(_lib.LBM_EDIVERGED).decode().startswith("non-finite")


def test_abi_version_matches_header_and_binding():
    """The library reports the QILBM_ABI_VERSION of the header it was built
    with, and the binding's structs follow that same version."""
    hdr = open([h for h in HEADERS if h.endswith("qilbm.h")][0]).read()
    version = int(re.search(r"#define QILBM_ABI_VERSION (\d+)", hdr).group(1))
    lib = _lib.load()
    assert lib.lbm_abi_version() == version == _lib.ABI_VERSION


def test_workspace_sizes_scale_with_precision(lib):
    b = {}
    for prec in (0, 1, 2):
        p = _params(nx=2048, ny=8192)
        p.precision = prec
        b[prec] = lib.lbm_workspace_bytes(byref(p))
    N = 2048 * 8192
    # two population buffers of 288, 144 and 76 bytes per node, plus fields
    assert b[0] >= 2 * 144 * N and b[1] >= 2 * 72 * N and b[2] >= 2 * 38 * N
    assert b[0] > b[1] > b[2]


def test_coefficients_match_paper_relations(lib):
    """Host derivation (beta, kappa, lambda, alpha, gamma, d rho/d phi) of the
    64x64 static-droplet problem: 0.03, 0.06, 0.1, 1, 9, 0.9."""
    p = _params()
    out = (c_double * 6)()
    assert lib.lbm_coefficients(byref(p), out) == 0
    assert list(out) == pytest.approx([0.03, 0.06, 0.1, 1.0, 9.0, 0.9], rel=1e-15)
    p.flags = _lib.LBM_FLAG_NO_GAMMA
    assert lib.lbm_coefficients(byref(p), out) == 0
    assert out[4] == 0.0


def _params3(**kw):
    d = wl.droplet3d().as_dict()
    d.update(kw)
    return _lib.make_params3(d)


@pytest.mark.parametrize("bad", [dict(nx=2), dict(nz=0), dict(tau_f=0.5), dict(tau_g=0.4),
                                 dict(sigma=0.0), dict(M=0.0), dict(rho_B=0.0),
                                 dict(gz=float("nan")), dict(bc=2)])
def test_3d_invalid_parameters_rejected(lib, bad):
    p = _params3(**bad)
    assert lib.lbm3_workspace_bytes(byref(p)) == 0
    ctx = c_void_p()
    assert lib.lbm3_init(byref(ctx), byref(p), c_void_p(256), 1 << 30, c_void_p(256),
                         None) == _lib.LBM_EINVAL
    assert not ctx.value


def test_3d_precision_flags_and_init_checks(lib):
    p = _params3()
    p.precision = _lib.LBM_FP16_STORE            # not offered in 3-D
    assert lib.lbm3_workspace_bytes(byref(p)) == 0
    p = _params3()
    p.flags = 4                                  # only LBM_FLAG_NO_GAMMA and LBM_FLAG_UNFUSED
    assert lib.lbm3_workspace_bytes(byref(p)) == 0
    p.flags = _lib.LBM_FLAG_NO_GAMMA | _lib.LBM_FLAG_UNFUSED
    assert lib.lbm3_workspace_bytes(byref(p)) > 0
    p = _params3()
    nbytes = lib.lbm3_workspace_bytes(byref(p))
    # two population sets of 38 planes (FP64) plus fields
    assert nbytes >= 2 * 38 * 8 * 32 ** 3
    ctx = c_void_p()
    assert lib.lbm3_init(byref(ctx), byref(p), None, nbytes, c_void_p(256), None) == _lib.LBM_EINVAL
    assert lib.lbm3_init(byref(ctx), byref(p), c_void_p(256), nbytes, None, None) == _lib.LBM_EINVAL
    assert lib.lbm3_init(byref(ctx), byref(p), c_void_p(264), nbytes, c_void_p(256), None) == _lib.LBM_EINVAL
    assert lib.lbm3_init(byref(ctx), byref(p), c_void_p(256), nbytes - 1, c_void_p(256), None) == _lib.LBM_ENOMEM
    p.precision = _lib.LBM_FP32
    assert 0 < lib.lbm3_workspace_bytes(byref(p)) < nbytes


def test_3d_null_context_calls(lib):
    assert lib.lbm3_step(None, 1) == _lib.LBM_EINVAL
    assert lib.lbm3_mass(None, (c_double * 5)()) == _lib.LBM_EINVAL
    assert lib.lbm3_moments(None, *([None] * 7)) == _lib.LBM_EINVAL
    assert lib.lbm3_get_state(None, None, None) == _lib.LBM_EINVAL
    assert lib.lbm3_set_state(None, None, None) == _lib.LBM_EINVAL
    assert lib.lbm3_time(None) == -1
    lib.lbm3_destroy(None)


def test_trt_parameter_checks(lib):
    """trt_magic: finite and >= 0 (0 is the BGK collision); the adjoint
    refuses the two-relaxation-time variant."""
    for bad in (-0.1, float("nan"), float("inf")):
        assert lib.lbm_workspace_bytes(byref(_params(trt_magic=bad))) == 0
    p = _params(trt_magic=0.25)
    assert lib.lbm_workspace_bytes(byref(p)) == lib.lbm_workspace_bytes(byref(_params()))
    assert lib.lbm_adjoint_workspace_bytes(byref(p)) == 0
    assert lib.lbm_adjoint_workspace_bytes(byref(_params())) > 0


def test_binding_refuses_a_library_of_another_abi_version(monkeypatch):
    monkeypatch.setattr(_lib, "ABI_VERSION", _lib.ABI_VERSION + 1)
    with pytest.raises(ImportError, match="interface version"):
        _lib.load(_lib.LIB_PATH)
