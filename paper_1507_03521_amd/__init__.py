"""MI355X (gfx950) implementation of the quasi-incompressible phase-field
lattice Boltzmann step of Yang & Guo: HIP kernels behind a C ABI
(include/qilbm.h, libqilbm.so), a ctypes binding (:class:`Lattice`) and an
autograd wrapper around the hand-written adjoint (:func:`simulate`)."""
from ._lib import (LBM_BC_PERIODIC, LBM_BC_WALLS_Y, LBM_FLAG_NO_GAMMA, LBM_FLAG_UNFUSED,
                   QilbmError, load)
from .autograd import PhaseFieldRun, simulate
from .lattice import Lattice

__all__ = ["Lattice", "simulate", "PhaseFieldRun", "QilbmError", "load", "LBM_BC_PERIODIC",
           "LBM_BC_WALLS_Y", "LBM_FLAG_NO_GAMMA", "LBM_FLAG_UNFUSED"]
