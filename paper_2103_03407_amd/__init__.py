"""MI355X two-grid MLQMC eigen-samples (Gilbert & Scheichl, arXiv:2103.03407).

The computation lives in ``libmlqmc.so`` (hand-written HIP kernels for gfx950
behind the C ABI of ``include/mlqmc.h``); this package is its ctypes binding.
"""

from .binding import (  # noqa: F401
    Context, Level, Opts, Islands, MlqmcError, default_opts, load, EXPORTS,
    MLQMC_OK, MLQMC_EINVAL, MLQMC_ENOMEM, MLQMC_EDEVICE, MLQMC_ENOCONV, MLQMC_HOST_ONLY,
    MLQMC_FP64, MLQMC_MIXED,
    FLAG_RQ_NOCONV, FLAG_LIN_NOCONV, FLAG_BREAKDOWN, FLAG_NONFINITE, FLAG_WRONG_PAIR,
    K_NONE, K_COEFF, K_APPLY, K_SMOOTH, K_COARSE, K_PRE, K_TG_LDS,
    mlqmc_create, mlqmc_create_islands, mlqmc_destroy, mlqmc_last_error, mlqmc_default_opts,
    mlqmc_lattice_points, mlqmc_coefficient, mlqmc_apply_operator, mlqmc_edge_weights,
    mlqmc_prolong,
    mlqmc_eig_level, mlqmc_eig_level_noalloc, mlqmc_estimate, mlqmc_set_tuning, mlqmc_set_timing, mlqmc_get_timing,
    mlqmc_embedded_points, mlqmc_estimate_nested, mlqmc_estimate_nested_extend,
    mlqmc_adaptive_decide, mlqmc_estimate_adaptive, AdaptiveOpts,
    ADAPT_DONE, ADAPT_DOUBLE, ADAPT_ADD, ADAPT_BUDGET, ADAPT_LEVELS,
)
