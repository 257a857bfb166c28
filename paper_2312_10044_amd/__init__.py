"""MI355X-native direct-sum boundary-integral Poisson-Boltzmann solver.

The compute path is the HIP library ``libpbdsbi.so`` (C ABI in
``include/pbsolve.h``); :mod:`.pbsolve` is its ctypes binding.
"""
from .pbsolve import (  # noqa: F401
    Context,
    Info,
    Params,
    PbError,
    PB_OK,
    PB_NOT_CONVERGED,
    PB_ERR_ARG,
    PB_ERR_GEOMETRY,
    PB_ERR_CHARGE,
    PB_ERR_HIP,
    PB_ERR_OOM,
    PB_FP64,
    PB_FP32_IR,
    PB_SWEEP_PAIRWISE,
    PB_SWEEP_BANDED,
    load_library,
    exported_symbols,
)
