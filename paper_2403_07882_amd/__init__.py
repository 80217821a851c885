"""MI355X-native solver for the coupled block-sparse systems of arXiv 2403.07882.

The computation lives in ``libcbs.so`` (HIP kernels for gfx950 behind the C
ABI in ``include/cbs.h``); this package is its thin ctypes binding.
"""
from .binding import (  # noqa: F401
    Allocator, CbsError, Options, Stats, System, coupled_solve, default_options, lib, pack_fields, torch_allocator,
    unpack_fields, OK, NOT_CONVERGED, ERR_ARG, ERR_PATTERN, ERR_SINGULAR, ERR_BREAKDOWN,
    ERR_NONFINITE, ERR_STATE, ERR_OOM, ERR_HIP, SOLVER_BICGSTAB, SOLVER_FGMRES, SOLVER_GMRES, PREC_NONE,
    PREC_BJACOBI, PREC_AMG, PREC_SGS, SMOOTH_BJACOBI, SMOOTH_DILU, SMOOTH_SGS, SMOOTH_ILU0, PRECISION_FP64, PRECISION_MIXED,
    LEVEL_SWEEP, LEVEL_RESIDUAL,
)
