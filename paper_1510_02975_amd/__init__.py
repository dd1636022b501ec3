"""MI355X (gfx950) evaluation of continuous functions through their
near-optimal continuous piecewise-linear approximation (Berjon et al., IEEE
TCYB 2015, arXiv 1510.02975).

The compute path is the HIP library libpwl.so (C ABI in include/pwl.h);
`binding` marshals PyTorch tensors and streams into it.  Importing the
package does not load the library; the first call does, and fails loudly if
it has not been built.
"""

from .binding import (  # noqa: F401
    BESSEL_J0, EXP, FLAG_DEGENERATE, FLAG_KNOTS_COLLAPSED, FLAG_NONFINITE, GAUSSIAN, INTERP,
    KDE_EXPF, KDE_FAST_EXPF, KDE_TABLE, KERNEL_BACKWARD, KERNEL_BATCH, KERNEL_BATCH_BACKWARD, KERNEL_FORWARD,
    LOCATE_MAP, LOCATE_SEARCH, RECORDS_PACKED, RECORDS_SOA, RECORDS_PAIRS,
    LORENTZIAN, MAX_N, NORM_L2,
    NORM_LINF, OPTIMAL, POLY, PROJ, SAMPLED, UNIFORM, Batch, PWLError, PWLFunction, PWLTable, Table, load_library,
    pwl_abi_version, pwl_batch_capture, pwl_batch_create, pwl_batch_eval, pwl_batch_eval_backward,
    pwl_batch_free, pwl_batch_info, pwl_batch_replay, pwl_build, pwl_build_sampled, pwl_build_tol, pwl_copy,
    pwl_direct_eval, pwl_direct_gaussian, pwl_eval, pwl_eval_backward, pwl_eval_backward_noalloc, pwl_kde, pwl_get_launch, pwl_get_locate, pwl_last_error,
    pwl_locate, pwl_set_locate, pwl_set_records, pwl_get_records,
    pwl_plan_tol, pwl_rebuild, pwl_set_launch, pwl_table_check, pwl_table_download, pwl_table_free,
    pwl_table_info)
