"""ctypes declarations of the C ABI in include/qilbm.h and include/qilbm3d.h
(argument marshalling only)."""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int32, c_int64, c_size_t, c_uint32, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqilbm.so")
# QILBM_ABI_VERSION of include/qilbm.h that SIGNATURES and the structs below follow
ABI_VERSION = 2

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_EDIVERGED, LBM_ESTATE = 0, -1, -2, -3, -4, -5
LBM_FP64, LBM_FP32, LBM_FP16_STORE = 0, 1, 2
LBM_BC_PERIODIC, LBM_BC_WALLS_Y = 0, 1
LBM_FLAG_NO_GAMMA, LBM_FLAG_UNFUSED = 1, 2

PRECISIONS = {"fp64": LBM_FP64, "fp32": LBM_FP32, "fp16": LBM_FP16_STORE,
              "fp16_store": LBM_FP16_STORE}


class LbmParams(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("rho_A", c_double), ("rho_B", c_double),
                ("sigma", c_double), ("W", c_double), ("M", c_double), ("tau_f", c_double),
                ("tau_g", c_double), ("gx", c_double), ("gy", c_double), ("rho_ref", c_double),
                ("bc", c_int32), ("precision", c_int32), ("flags", c_uint32),
                ("trt_magic", c_double)]


class Lbm3Params(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("nz", c_int32), ("rho_A", c_double),
                ("rho_B", c_double), ("sigma", c_double), ("W", c_double), ("M", c_double),
                ("tau_f", c_double), ("tau_g", c_double), ("gx", c_double), ("gy", c_double),
                ("gz", c_double), ("rho_ref", c_double), ("bc", c_int32),
                ("precision", c_int32), ("flags", c_uint32), ("trt_magic", c_double)]


LBM3_BC_WALLS_Z = 1

_P = POINTER(LbmParams)
_P3 = POINTER(Lbm3Params)
_D = POINTER(c_double)
# name -> (restype, argtypes); every symbol declared in include/qilbm.h and
# include/qilbm3d.h
SIGNATURES = {
    "lbm_workspace_bytes": (c_size_t, [_P]),
    "lbm_coefficients": (c_int32, [_P, _D]),
    "lbm_init": (c_int32, [POINTER(c_void_p), _P, c_void_p, c_size_t, c_void_p, c_void_p]),
    "lbm_step": (c_int32, [c_void_p, c_int64]),
    "lbm_record_bytes": (c_size_t, [c_void_p]),
    "lbm_step_record": (c_int32, [c_void_p, c_void_p]),
    "lbm_moments": (c_int32, [c_void_p] + [c_void_p] * 6),
    "lbm_mass": (c_int32, [c_void_p, _D]),
    "lbm_mass_noalloc": (c_int32, [_P, c_void_p, c_void_p, c_void_p]),
    "lbm_get_state": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "lbm_set_state": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "lbm_state_bytes": (c_size_t, [c_void_p]),
    "lbm_save_raw": (c_int32, [c_void_p, c_void_p]),
    "lbm_load_raw": (c_int32, [c_void_p, c_void_p, c_int64]),
    "lbm_time": (c_int64, [c_void_p]),
    "lbm_set_stream": (c_int32, [c_void_p, c_void_p]),
    "lbm_set_launch": (c_int32, [c_void_p, c_int32]),
    "lbm_launch_info": (c_int32, [c_void_p, POINTER(c_int32)]),
    "lbm_set_pass": (c_int32, [c_void_p, c_int32, c_int32]),
    "lbm_step_records": (c_int32, [c_void_p, c_int64, POINTER(c_void_p)]),
    "lbm_pass_info": (c_int32, [c_void_p, POINTER(c_int32)]),
    "lbm_adjoint_workspace_bytes": (c_size_t, [_P]),
    "lbm_adjoint_begin": (c_int32, [c_void_p, c_void_p, c_size_t, c_void_p]),
    "lbm_adjoint_seed": (c_int32, [c_void_p, c_void_p]),
    "lbm_adjoint_step": (c_int32, [c_void_p, c_void_p]),
    "lbm_adjoint_step_record": (c_int32, [c_void_p, c_void_p]),
    "lbm_adjoint_init": (c_int32, [c_void_p, c_void_p, c_void_p, _D]),
    "lbm_adjoint_set": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "lbm_adjoint_get": (c_int32, [c_void_p, c_void_p, c_void_p, _D]),
    "lbm_destroy": (None, [c_void_p]),
    "lbm_strerror": (ctypes.c_char_p, [c_int32]),
    "lbm_abi_version": (c_int32, []),
    "lbm3_workspace_bytes": (c_size_t, [_P3]),
    "lbm3_init": (c_int32, [POINTER(c_void_p), _P3, c_void_p, c_size_t, c_void_p, c_void_p]),
    "lbm3_step": (c_int32, [c_void_p, c_int64]),
    "lbm3_moments": (c_int32, [c_void_p] + [c_void_p] * 7),
    "lbm3_mass": (c_int32, [c_void_p, _D]),
    "lbm3_get_state": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "lbm3_set_state": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "lbm3_time": (c_int64, [c_void_p]),
    "lbm3_destroy": (None, [c_void_p]),
}


class QilbmError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = _strerror(status)
        super().__init__(f"{what}: {msg} (status {status})" if what else msg)


_lib = None


def _strerror(status: int) -> str:
    try:
        return load().lbm_strerror(status).decode()
    except Exception:  # library missing: fall back to the code
        return f"status {status}"


def load(path: str | None = None) -> ctypes.CDLL:
    """The HIP library. Raises FileNotFoundError when it has not been built
    (run ``python -m paper_1507_03521_amd.build``); there is no fallback."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise FileNotFoundError(f"HIP library not built: {p} (run python -m paper_1507_03521_amd.build)")
    lib = ctypes.CDLL(p)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if lib.lbm_abi_version() != ABI_VERSION:
        raise ImportError(f"{p}: interface version {lib.lbm_abi_version()}, the binding expects "
                          f"{ABI_VERSION} (rebuild with python -m paper_1507_03521_amd.build)")
    if path is None:
        _lib = lib
    return lib


def check(status: int, what: str = "") -> None:
    if status != LBM_OK:
        raise QilbmError(status, what)


def make_params(p: dict, precision="fp64", flags: int = 0) -> LbmParams:
    """lbm_params from a mapping with keys nx, ny, rho_A, rho_B, sigma, W, M,
    tau_f, tau_g and optionally gx, gy, rho_ref (default rho_A), bc and
    trt_magic (0: BGK collision of f; > 0: two-relaxation-time collision)."""
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    rho_ref = p.get("rho_ref")
    return LbmParams(int(p["nx"]), int(p["ny"]), float(p["rho_A"]), float(p["rho_B"]),
                     float(p["sigma"]), float(p["W"]), float(p["M"]), float(p["tau_f"]),
                     float(p["tau_g"]), float(p.get("gx", 0.0)), float(p.get("gy", 0.0)),
                     float(p["rho_A"] if rho_ref is None else rho_ref), int(p.get("bc", 0)),
                     prec, int(flags), float(p.get("trt_magic", 0.0)))


def make_params3(p: dict, precision="fp64", flags: int = 0) -> Lbm3Params:
    """lbm3_params from a mapping with keys nx, ny, nz, rho_A, rho_B, sigma,
    W, M, tau_f, tau_g and optionally gx, gy, gz, rho_ref (default rho_A),
    bc (0 periodic, 1 walls normal to z), trt_magic (0: BGK)."""
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    rho_ref = p.get("rho_ref")
    return Lbm3Params(int(p["nx"]), int(p["ny"]), int(p["nz"]), float(p["rho_A"]),
                      float(p["rho_B"]), float(p["sigma"]), float(p["W"]), float(p["M"]),
                      float(p["tau_f"]), float(p["tau_g"]), float(p.get("gx", 0.0)),
                      float(p.get("gy", 0.0)), float(p.get("gz", 0.0)),
                      float(p["rho_A"] if rho_ref is None else rho_ref), int(p.get("bc", 0)),
                      prec, int(flags), float(p.get("trt_magic", 0.0)))
