"""MI355X (gfx950) direct-sum N-body library: HIP kernels behind a C ABI
(include/nbody.h) and a thin ctypes binding (``nbody``)."""
from . import nbody  # noqa: F401  (loads libnbody.so; raises if it is not built)
from .nbody import (Context, Params, System, NBodyError, NB_FP64, NB_MIXED, NB_FP32,  # noqa: F401
                    PREC, DIAG_KEYS)
