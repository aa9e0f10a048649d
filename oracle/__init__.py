"""CPU oracle for Randomly Pivoted LU (FP64 / complex128).

TEST INFRASTRUCTURE: only tests, the smoke check and the bench's CPU-baseline
leg import this package. The product path (the HIP library and its binding)
never imports it, and the two share no code.
"""
from .philox import philox4x64_10, step_uniforms, word_to_unit  # noqa: F401
from .rplu import (  # noqa: F401
    STALL_RATIO, STALL_WINDOW, STOP_EXHAUSTED, STOP_RANK, STOP_STALL, STOP_TOL,
    STOP_TOL_UNREACHED, Draw,
    NonFiniteInput, RPLUResult, ZeroPivot, cauchy_col, cauchy_entries,
    cauchy_generator_update, cauchy_row, cauchy_row_masses, first_exceeding,
    inverse_cdf, rplu_cauchy, rplu_dense, schur_closed_form, schur_update,
    squared_magnitude,
)
