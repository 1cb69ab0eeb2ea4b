"""tqr: tiled QR factorization on one AMD Instinct MI355X.

Thin Python binding of libtqr.so (the C ABI in include/tqr.h).  Every step
of the factorization, Q^T application and least-squares solve runs in the
library's HIP kernels; this module only marshals arguments.  PyTorch
supplies device memory and the current stream.

Matrices are float64 column-major device tensors (stride (1, ld)).
"""
from ._binding import (  # noqa: F401
    ASAP, BF16, BINARY, EXEC_PERSISTENT, EXEC_SEQUENTIAL, F32, F64, FIBONACCI, FLAT,
    GRASAP, GREEDY, debug_graph, debug_ready, debug_spin_limit, debug_succ, debug_timing, debug_timing_read, debug_trace, executor_grid, wallclock_khz, HYBRID, PLASMA, TREES, TT, AUTO, Opts, TqrError, default_opts, lib,
    library_path, tqr_apply_qt, tqr_factor, tqr_factor_ex, tqr_graph_stats, tqr_lstsq,
    tqr_lstsq_work_size, tqr_schedule_bounds, tqr_cholinv, tqr_cholinv_work_size, tqr_cholinv_graph_stats,
    tqr_zworkspace_size, tqr_zfactor, tqr_zapply_qh,
    CHOLINV_INPLACE, CHOLINV_RENAMED, CHOLINV_UUU, PRIO_BOTTOM, PRIO_LIST, PRIO_STATIC, REFINE_AUTO, REFINE_CLASSICAL, REFINE_GMRES, tqr_solve_r, tqr_tree_cp, tqr_tree_list, tqr_workspace_size,
)
from .api import (apply_qt, autotune_batched, cholinv, colmajor, factor, lstsq, lstsq_batched,  # noqa: F401
                  zapply_qh, zcolmajor, zfactor,
                  lstsq_batched_workspace, lstsq_workspace, refine_report, refine_reports, solve_r, workspace)  # noqa: F401
