"""MI355X-native resolvent-sampling Rayleigh-Ritz (RSRR) for T(lambda) v = 0.

The computation lives in librsrr.so (HIP kernels for gfx950 behind the C ABI
of include/rsrr.h); this package is its ctypes binding.
"""
from ._binding import (  # noqa: F401
    PREC_C128, PREC_C64_IR, Problem, RsrrError, check, contour, default_params, from_device,
    gemm, gesv, load, orthonormalize, to_device, empty_device, timers_enable, timers_reset,
    timers_read, timers_only, Server, solve_batched, tune_lu, tune_save, tune_load,
)
