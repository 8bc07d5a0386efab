"""MI355X-native Jacobi-preconditioned block BiCGGR for the clover
Wilson-Dirac system A X = B with L right-hand sides.

The numerical work lives in the HIP library ``libwdsolve.so`` (C ABI in
``include/wdsolve.h``); this package holds its sources (``csrc/``), the
build script and a thin ctypes binding.
"""

from ._binding import (  # noqa: F401
    Context, WDError, load, strerror, LIB_PATH,
    WD_F64, WD_F32, WD_BF16, WD_F64_COEF_F32, WD_F64_COEF_BF16, WD_PRECOND_NONE, WD_PRECOND_JACOBI, WD_PRECOND_LEARNED,
    WD_JACOBI_BLOCK, WD_JACOBI_POINT, WD_MAX_L, WD_LAYOUT_STANDARD, WD_LAYOUT_TILED,
    WD_OK, WD_EINVAL, WD_ENOMEM, WD_EHIP, WD_ENAN, WD_ESTATE,
    WD_NOT_CONVERGED, WD_BREAKDOWN, WD_DIVERGED, WD_STAGNATED,
)
