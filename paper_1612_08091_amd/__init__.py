"""MI355X-native state-vector simulator core (the data-parallel hot path of the
ProjectQ high-performance simulator, arXiv:1612.08091 Sec. 4.3.2).

The computation lives in libqsv.so (HIP kernels for gfx950 behind the C ABI
of include/qsv.h); ``qsv`` is its ctypes binding and ``autograd`` wraps the
adjoint gradient as a torch.autograd.Function.
"""
from . import qsv  # noqa: F401  (fails loudly when libqsv.so is missing)
from .qsv import (Batch, NotClassicalError, QsvError, Simulator,  # noqa: F401
                  adjoint_gradient)

__all__ = ["qsv", "Simulator", "Batch", "adjoint_gradient", "QsvError", "NotClassicalError"]
