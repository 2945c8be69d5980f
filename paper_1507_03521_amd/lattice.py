"""Python handle of one lattice context. PyTorch provides the device memory
(workspaces, inputs, outputs) and the stream; every step of the method runs
in the HIP library behind the C ABI."""
from __future__ import annotations

import ctypes
from ctypes import byref, c_double, c_int32, c_void_p

import torch

from . import _lib


def _ptr(t: torch.Tensor) -> int:
    return t.data_ptr()


MASS_NOALLOC_MAX_NODES = 1 << 21


def mass_noalloc(params: dict, precision: str, state: torch.Tensor, out: torch.Tensor,
                 flags: int = 0, stream: torch.cuda.Stream | None = None) -> None:
    """lbm_mass_noalloc: the four totals of a raw state (``Lattice.save_raw``
    layout, device uint8 tensor) into ``out`` (device float64 tensor of 4),
    asynchronously on ``stream``, with no context and no allocation (the
    kernels' scratch is the library's static device array)."""
    lib = _lib.load()
    prm = _lib.make_params(params, precision, flags)
    assert state.is_cuda and state.is_contiguous()
    assert out.is_cuda and out.dtype == torch.float64 and out.numel() >= 4
    stream = stream or torch.cuda.current_stream(state.device)
    _lib.check(lib.lbm_mass_noalloc(byref(prm), _ptr(state), _ptr(out),
                                    c_void_p(stream.cuda_stream)), "lbm_mass_noalloc")


class Lattice:
    """A D2Q9 lattice of the quasi-incompressible phase-field LBE on one GPU.

    ``params``: mapping with nx, ny, rho_A, rho_B, sigma, W, M, tau_f, tau_g
    and optional gx, gy, rho_ref, bc. ``phi0``: initial order parameter
    (ny, nx), any array-like; copied to the device as FP64.
    ``precision``: "fp64", "fp32" or "fp16" (binary16 storage, FP32 arithmetic).
    """

    def __init__(self, params: dict, phi0, precision="fp64", flags: int = 0,
                 device: str | torch.device = "cuda", stream: torch.cuda.Stream | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("qilbm needs a ROCm GPU; none is visible")
        self.lib = _lib.load()
        self.device = torch.device(device)
        self.params = _lib.make_params(params, precision, flags)
        self.nx, self.ny = self.params.nx, self.params.ny
        nbytes = self.lib.lbm_workspace_bytes(byref(self.params))
        if nbytes == 0:
            raise _lib.QilbmError(_lib.LBM_EINVAL, "lbm_workspace_bytes")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream or torch.cuda.current_stream(self.device)
        self.phi0 = torch.as_tensor(phi0, dtype=torch.float64).to(self.device).contiguous()
        assert self.phi0.shape == (self.ny, self.nx)
        self._ctx = c_void_p()
        _lib.check(self.lib.lbm_init(byref(self._ctx), byref(self.params), _ptr(self.workspace),
                                     nbytes, _ptr(self.phi0), c_void_p(self.stream.cuda_stream)),
                   "lbm_init")
        self._adj_ws = None

    # ------------------------------------------------------------ basics
    @property
    def ctx(self):
        if not self._ctx:
            raise RuntimeError("lattice destroyed")
        return self._ctx

    def coefficients(self) -> dict:
        out = (c_double * 6)()
        _lib.check(self.lib.lbm_coefficients(byref(self.params), out), "lbm_coefficients")
        return dict(zip(("beta", "kappa", "lam", "alpha", "gamma", "drho_dphi"), list(out)))

    def step(self, n: int = 1) -> None:
        _lib.check(self.lib.lbm_step(self.ctx, int(n)), "lbm_step")

    @property
    def record_bytes(self) -> int:
        return int(self.lib.lbm_record_bytes(self.ctx))

    def step_record(self, out: torch.Tensor | None = None) -> torch.Tensor:
        """One step that also writes the record of the state it started
        from (phi, mu, p, S, jx, jy planes), the input of
        :meth:`adjoint_step_record`."""
        if out is None:
            out = torch.empty(self.record_bytes, dtype=torch.uint8, device=self.device)
        assert out.numel() >= self.record_bytes and out.is_contiguous()
        _lib.check(self.lib.lbm_step_record(self.ctx, _ptr(out)), "lbm_step_record")
        return out

    @property
    def time(self) -> int:
        return int(self.lib.lbm_time(self.ctx))

    def _field(self):
        return torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device)

    def moments(self, names=("phi", "rho", "ux", "uy", "p", "mu")) -> dict:
        out = {k: self._field() for k in names}
        args = [c_void_p(_ptr(out[k])) if k in out else c_void_p(0)
                for k in ("phi", "rho", "ux", "uy", "p", "mu")]
        _lib.check(self.lib.lbm_moments(self.ctx, *args), "lbm_moments")
        return out

    def mass(self):
        out = (c_double * 4)()
        st = self.lib.lbm_mass(self.ctx, out)
        if st not in (_lib.LBM_OK, _lib.LBM_EDIVERGED):
            _lib.check(st, "lbm_mass")
        vals = tuple(out)
        if st == _lib.LBM_EDIVERGED:
            raise _lib.QilbmError(st, f"lbm_mass {vals}")
        return vals

    def get_state(self):
        f = torch.empty((9, self.ny, self.nx), dtype=torch.float64, device=self.device)
        g = torch.empty_like(f)
        _lib.check(self.lib.lbm_get_state(self.ctx, _ptr(f), _ptr(g)), "lbm_get_state")
        return f, g

    def set_state(self, f, g) -> None:
        f = torch.as_tensor(f, dtype=torch.float64).to(self.device).contiguous()
        g = torch.as_tensor(g, dtype=torch.float64).to(self.device).contiguous()
        assert f.shape == (9, self.ny, self.nx) and g.shape == f.shape
        _lib.check(self.lib.lbm_set_state(self.ctx, _ptr(f), _ptr(g)), "lbm_set_state")
        self.stream.synchronize()

    @property
    def state_bytes(self) -> int:
        return int(self.lib.lbm_state_bytes(self.ctx))

    def save_raw(self, out: torch.Tensor | None = None) -> torch.Tensor:
        if out is None:
            out = torch.empty(self.state_bytes, dtype=torch.uint8, device=self.device)
        assert out.numel() >= self.state_bytes and out.is_contiguous()
        _lib.check(self.lib.lbm_save_raw(self.ctx, _ptr(out)), "lbm_save_raw")
        return out

    def load_raw(self, src: torch.Tensor, t: int) -> None:
        assert src.numel() >= self.state_bytes and src.is_contiguous()
        _lib.check(self.lib.lbm_load_raw(self.ctx, _ptr(src), int(t)), "lbm_load_raw")

    def set_launch(self, seg_rows: int) -> None:
        _lib.check(self.lib.lbm_set_launch(self.ctx, int(seg_rows)), "lbm_set_launch")

    def launch_info(self) -> dict:
        out = (c_int32 * 4)()
        _lib.check(self.lib.lbm_launch_info(self.ctx, out), "lbm_launch_info")
        return dict(zip(("strips", "segments", "seg_rows", "threads"), list(out)))

    def step_records(self, records) -> None:
        """len(records) steps, writing the record of the state step k starts
        from into records[k] (uint8 device tensors of record_bytes each)."""
        for r in records:
            assert r.numel() >= self.record_bytes and r.is_contiguous()
        arr = (c_void_p * max(len(records), 1))(*[_ptr(r) for r in records])
        _lib.check(self.lib.lbm_step_records(self.ctx, len(records), arr), "lbm_step_records")

    def set_pass(self, steps: int, seg_rows: int = 0) -> None:
        """Time steps per fused launch in step() (2: temporal blocking, the
        default for fp64 and fp32; 1: one launch per step, the default for
        fp16 storage)."""
        _lib.check(self.lib.lbm_set_pass(self.ctx, int(steps), int(seg_rows)), "lbm_set_pass")

    def pass_info(self) -> dict:
        out = (c_int32 * 5)()
        _lib.check(self.lib.lbm_pass_info(self.ctx, out), "lbm_pass_info")
        return dict(zip(("steps", "strips", "segments", "seg_rows", "threads"), list(out)))

    # ------------------------------------------------------------ adjoint
    def adjoint_begin(self, dL_dphi: torch.Tensor) -> None:
        nbytes = self.lib.lbm_adjoint_workspace_bytes(byref(self.params))
        if self._adj_ws is None or self._adj_ws.numel() < nbytes:
            self._adj_ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._seed = torch.as_tensor(dL_dphi, dtype=torch.float64).to(self.device).contiguous()
        _lib.check(self.lib.lbm_adjoint_begin(self.ctx, _ptr(self._adj_ws), nbytes,
                                              _ptr(self._seed)), "lbm_adjoint_begin")

    def adjoint_seed(self, dL_dphi: torch.Tensor) -> None:
        """Re-seeds the adjoint (workspace from :meth:`adjoint_begin`)."""
        self._seed = torch.as_tensor(dL_dphi, dtype=torch.float64).to(self.device).contiguous()
        _lib.check(self.lib.lbm_adjoint_seed(self.ctx, _ptr(self._seed)), "lbm_adjoint_seed")

    def adjoint_step(self, fwd_raw: torch.Tensor) -> None:
        _lib.check(self.lib.lbm_adjoint_step(self.ctx, _ptr(fwd_raw)), "lbm_adjoint_step")

    def adjoint_step_record(self, record: torch.Tensor) -> None:
        _lib.check(self.lib.lbm_adjoint_step_record(self.ctx, _ptr(record)),
                   "lbm_adjoint_step_record")

    def adjoint_init(self, phi0: torch.Tensor | None = None):
        phi0 = self.phi0 if phi0 is None else \
            torch.as_tensor(phi0, dtype=torch.float64).to(self.device).contiguous()
        dphi0 = torch.empty_like(phi0)
        out = (c_double * 2)()
        _lib.check(self.lib.lbm_adjoint_init(self.ctx, _ptr(phi0), _ptr(dphi0), out),
                   "lbm_adjoint_init")
        return dphi0, out[0], out[1]

    def adjoint_set(self, fbar, gbar) -> None:
        self._fbar = torch.as_tensor(fbar, dtype=torch.float64).to(self.device).contiguous()
        self._gbar = torch.as_tensor(gbar, dtype=torch.float64).to(self.device).contiguous()
        _lib.check(self.lib.lbm_adjoint_set(self.ctx, _ptr(self._fbar), _ptr(self._gbar)),
                   "lbm_adjoint_set")

    def adjoint_get(self):
        f = torch.empty((9, self.ny, self.nx), dtype=torch.float64, device=self.device)
        g = torch.empty_like(f)
        out = (c_double * 2)()
        _lib.check(self.lib.lbm_adjoint_get(self.ctx, _ptr(f), _ptr(g), out), "lbm_adjoint_get")
        return f, g, out[0], out[1]

    # ------------------------------------------------------------ teardown
    def close(self) -> None:
        if getattr(self, "_ctx", None):
            self.lib.lbm_destroy(self._ctx)
            self._ctx = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
