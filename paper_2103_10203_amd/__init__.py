"""MI355X-native reduced-frequency Lippmann-Schwinger solver (arXiv 2103.10203).

The product is ``libmor.so`` (HIP kernels for gfx950 behind the C ABI in
``include/mor.h``); this package holds its sources (``csrc/``), the build
script (``build.py``) and the thin ctypes binding (``_native``).
"""
from ._native import (  # noqa: F401
    Phase, Plan, PlanList, SolveResult, MorError, make_plans, solve, solve_multi, solve_path, solve_path_multi, compat, stress_error,
    PATTERN_ADAPTED, PATTERN_RADIAL,
    profile_enable, profile_reset, profile_query, version, lib,
    GAMMA_ROTATED, GAMMA_CONTINUOUS, PREC_FP32, PREC_BF16X3, PREC_FP64,
    TRANSFORM_AUTO, TRANSFORM_FFT, TRANSFORM_DFT,
    MOR_OK, MOR_E_INVALID_ARG, MOR_E_NOT_CONVERGED, MOR_E_NONFINITE, MOR_E_UNSUPPORTED,
    MLP, MLP_FP32, MLP_BF16, warm_features, warm_targets, warm_apply,
    KERNEL_ROW, KERNEL_COL, SCHED_GRID, SCHED_PERSISTENT, tune_variants, tune_get, tune_set, tune_subbatch, autotune,
)
