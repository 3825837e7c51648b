"""MI355X-native structured-operator conic solver (arXiv 1609.03488, Sections IV-V).

The computation runs in ``libcgs.so`` (hand-written HIP kernels for gfx950,
C ABI in ``include/cgs.h``).  This package is a thin ctypes binding with the
same names: it marshals arguments and uses PyTorch only to own the device
workspace and to name the HIP stream.  There is no CPU fallback: importing the
binding raises if the library is missing.
"""
from ._lib import (  # noqa: F401
    CgsError, Settings, Info, Operator, Solver, Server, lib, library_path, solve_noalloc,
    NOALLOC_SCRATCH_BYTES, DTYPE_F64, DTYPE_F32, MEM_HOST_COPY, MEM_DEVICE_BORROW,
    FP64, FP32, BF16, SOLVED, MAX_ITERS, INFEASIBLE, UNBOUNDED, NUMERICAL, RUNNING,
    STATUS_NAMES,
)
from .problems import deconv_problem, lasso_problem, conv_lasso_problem, ConeProblem  # noqa: F401
from .regls import RegLS  # noqa: F401
