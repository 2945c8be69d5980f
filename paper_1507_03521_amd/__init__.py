"""MI355X (gfx950) implementation of the quasi-incompressible phase-field
lattice Boltzmann step of Yang & Guo: HIP kernels behind a C ABI
(include/qilbm.h, libqilbm.so), ctypes bindings (:class:`Lattice`; the
D3Q19 form, include/qilbm3d.h: :class:`Lattice3D`) and an
autograd wrapper around the hand-written adjoint (:func:`simulate`)."""
from ._lib import (LBM_BC_PERIODIC, LBM_BC_WALLS_Y, LBM_FLAG_NO_GAMMA, LBM_FLAG_UNFUSED,
                   QilbmError, load)
from .autograd import PhaseFieldRun, simulate
from .lattice import Lattice
from .lattice3d import Lattice3D

__all__ = ["Lattice", "Lattice3D", "simulate", "PhaseFieldRun", "QilbmError", "load", "LBM_BC_PERIODIC",
           "LBM_BC_WALLS_Y", "LBM_FLAG_NO_GAMMA", "LBM_FLAG_UNFUSED"]
