"""Randomly Pivoted LU on MI355X (gfx950): Python binding of librplu.

The binding marshals torch device tensors and the current HIP stream into the
C ABI of include/rplu.h; all computation runs in the library's HIP kernels.
Importing fails if the library has not been built (there is no CPU path).
"""
from ._binding import (  # noqa: F401
    RPLU_C64, RPLU_C128, RPLU_FLAG_COLMASS, RPLU_FLAG_GRAPH, RPLU_FLAG_NO_GRAPH,
    RPLU_FLAG_STALL_STOP, RPLU_FLAG_SPLIT_SAMPLER, RPLU_FLAG_C2PLU, RPLU_FLAG_REFRESH, RPLU_FLAG_CERTIFY, RPLU_FLAG_KEEP_INPUT, RPLU_FLAG_LAZY_SWEEP, RPLU_FLAG_EAGER_SWEEP, RPLU_FLAG_CPLU, RPLU_FLAG_BOUNDS, RPLU_FLAG_MAXMASS_STOP, RPLU_CUR_MAX_RANK, RPLU_LAZY_STEPS, RPLU_MAX_REFRESH, RPLU_STALL_WINDOW, RPLU_STOP_STALL,
    RPLU_ORDER_AREA, RPLU_ORDER_CUBE, RPLU_ORDER_GIVEN, RPLU_R32, RPLU_R64,
    RPLU_STOP_EXHAUSTED, RPLU_STOP_RANK, RPLU_STOP_TOL, RPLU_STOP_TOL_UNREACHED,
    RPLU_SERVER_SIMULATE, RPLU_TRACE_WORDS, BatchPlan, Context, CURResult, Result, RPLUError, Server,
    default_context, lib,
    rplu_batched, rplu_batched_tune, rplu_cauchy, rplu_create, rplu_cur, rplu_cur_aaa, AAAResult, rplu_dense, rplu_dense_noalloc,
    rplu_profile_begin, rplu_profile_end, rplu_verify,
)
