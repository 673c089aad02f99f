"""MI355X-native reduced-KKT (Schur complement) hot path of a block-structured
interior-point method (arXiv 2301.04869), FP64, behind the C ABI of
include/rkkt.h.  The Python layer only marshals arguments to librkkt.so."""
from ._lib import (RkktError, lib, rkkt_analyze, rkkt_create, rkkt_set_loads, rkkt_set_line_status, rkkt_dims_get,
                   rkkt_evaluate, rkkt_condense, rkkt_factor, rkkt_step, rkkt_status,
                   rkkt_destroy, rkkt_last_error, rkkt_profile_begin, rkkt_profile_end,
                   rkkt_solve, rkkt_solve_warm, rkkt_iterate, rkkt_graph_capture, rkkt_graph_launch,
                   rkkt_batch_create, rkkt_batch_launch, rkkt_batch_destroy, rkkt_autotune,
                   rkkt_analyze_lu, rkkt_analyze_schedule, rkkt_probe_peaks, SCHEDULES, EXPORTS, STAGES, LIB_PATH,
                   Mlp, Multi, mlp_layout, MLP_EXPORTS)

__all__ = ["RkktError", "lib", "rkkt_analyze", "rkkt_create", "rkkt_set_loads", "rkkt_set_line_status", "rkkt_dims_get",
           "rkkt_evaluate", "rkkt_condense", "rkkt_factor", "rkkt_step", "rkkt_status",
           "rkkt_destroy", "rkkt_last_error", "rkkt_profile_begin", "rkkt_profile_end",
           "rkkt_solve", "rkkt_solve_warm", "rkkt_iterate", "rkkt_graph_capture",
           "rkkt_graph_launch", "rkkt_batch_create", "rkkt_batch_launch", "rkkt_batch_destroy",
           "rkkt_autotune", "rkkt_analyze_lu", "rkkt_analyze_schedule", "rkkt_probe_peaks", "SCHEDULES", "EXPORTS",
           "STAGES", "LIB_PATH", "Mlp", "Multi", "mlp_layout", "MLP_EXPORTS"]
