"""Python handle of one three-dimensional (D3Q19) lattice context; PyTorch
provides device memory and the stream, the HIP library runs the step."""
from __future__ import annotations

from ctypes import byref, c_double, c_void_p

import torch

from . import _lib


class Lattice3D:
    """A D3Q19 lattice of the quasi-incompressible phase-field LBE on one GPU.

    ``params``: mapping with nx, ny, nz, rho_A, rho_B, sigma, W, M, tau_f,
    tau_g and optional gx, gy, gz, rho_ref, bc (0 periodic, 1 walls normal to
    z). ``phi0``: initial order parameter (nz, ny, nx), copied to the device
    as FP64. ``precision``: "fp64" or "fp32" (g in Q2.29 fixed point).
    """

    def __init__(self, params: dict, phi0, precision="fp64", flags: int = 0,
                 device: str | torch.device = "cuda", stream: torch.cuda.Stream | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("qilbm needs a ROCm GPU; none is visible")
        self.lib = _lib.load()
        self.device = torch.device(device)
        self.params = _lib.make_params3(params, precision, flags)
        self.nx, self.ny, self.nz = self.params.nx, self.params.ny, self.params.nz
        nbytes = self.lib.lbm3_workspace_bytes(byref(self.params))
        if nbytes == 0:
            raise _lib.QilbmError(_lib.LBM_EINVAL, "lbm3_workspace_bytes")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream or torch.cuda.current_stream(self.device)
        self.phi0 = torch.as_tensor(phi0, dtype=torch.float64).to(self.device).contiguous()
        assert self.phi0.shape == (self.nz, self.ny, self.nx)
        self._ctx = c_void_p()
        _lib.check(self.lib.lbm3_init(byref(self._ctx), byref(self.params),
                                      self.workspace.data_ptr(), nbytes, self.phi0.data_ptr(),
                                      c_void_p(self.stream.cuda_stream)), "lbm3_init")

    @property
    def ctx(self):
        if not self._ctx:
            raise RuntimeError("lattice destroyed")
        return self._ctx

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def step(self, n: int = 1) -> None:
        _lib.check(self.lib.lbm3_step(self.ctx, int(n)), "lbm3_step")

    @property
    def time(self) -> int:
        return int(self.lib.lbm3_time(self.ctx))

    def moments(self, names=("phi", "rho", "ux", "uy", "uz", "p", "mu")) -> dict:
        out = {k: torch.empty(self.shape, dtype=torch.float64, device=self.device)
               for k in names}
        args = [c_void_p(out[k].data_ptr()) if k in out else c_void_p(0)
                for k in ("phi", "rho", "ux", "uy", "uz", "p", "mu")]
        _lib.check(self.lib.lbm3_moments(self.ctx, *args), "lbm3_moments")
        return out

    def mass(self):
        out = (c_double * 5)()
        st = self.lib.lbm3_mass(self.ctx, out)
        vals = tuple(out)
        if st == _lib.LBM_EDIVERGED:
            raise _lib.QilbmError(st, f"lbm3_mass {vals}")
        _lib.check(st, "lbm3_mass")
        return vals

    def get_state(self):
        f = torch.empty((19,) + self.shape, dtype=torch.float64, device=self.device)
        g = torch.empty_like(f)
        _lib.check(self.lib.lbm3_get_state(self.ctx, f.data_ptr(), g.data_ptr()),
                   "lbm3_get_state")
        return f, g

    def set_state(self, f, g) -> None:
        f = torch.as_tensor(f, dtype=torch.float64).to(self.device).contiguous()
        g = torch.as_tensor(g, dtype=torch.float64).to(self.device).contiguous()
        assert f.shape == (19,) + self.shape and g.shape == f.shape
        _lib.check(self.lib.lbm3_set_state(self.ctx, f.data_ptr(), g.data_ptr()),
                   "lbm3_set_state")
        self.stream.synchronize()

    def close(self) -> None:
        if getattr(self, "_ctx", None):
            self.lib.lbm3_destroy(self._ctx)
            self._ctx = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
