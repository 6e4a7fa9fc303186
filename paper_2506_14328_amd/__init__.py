"""MI355X (gfx950) implementation of one RK3 step of the implicit second-order
discrete-forcing immersed-boundary method with FFT/tridiagonal projection.

The compute path is the HIP library libibm.so (C ABI in include/ibm.h);
`IbmGrid` is its ctypes binding.  Importing the package does not load the
library; creating an `IbmGrid` does, and raises if it has not been built.
"""
from .ibm import (IBM_B_EULER, IBM_B_EXP, IBM_B_TAYLOR2, IBM_CFR, IBM_CPG, IBM_FP32_STORAGE, IBM_FP64,  # noqa
                  IbmError, IbmGrid, IbmGridDesc, IbmStats, load_library, LIB_PATH, EXPORTED, stream_copy, stream_mix,
                  solve_pressure_noalloc)
