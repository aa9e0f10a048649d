"""Parity protocol between the HIP path and the CPU oracle.

The oracle replays the pivots the GPU chose (forced mode) and, at every step,
still makes its own draw. A GPU pivot counts as a match when the oracle's own
draw selects the same index, or when the oracle's draw target u*T lies within
tau*T (FP64: tau = 1e-12) of the CDF bin of the GPU's index in the oracle's
own prefix sums, i.e. the two sides landed in the same bin up to rounding of
the prefix sums. For a single-precision sweep the window also admits the
measured difference between the two sides' masses (delta_t).
"""
from __future__ import annotations

import math

import numpy as np


def fro(x) -> float:
    return float(np.sqrt(np.sum(np.abs(x) ** 2)))


def rel(a, b, scale=None) -> float:
    d = fro(np.asarray(a) - np.asarray(b))
    s = fro(b) if scale is None else scale
    return d / s if s > 0 else d


def check_draws(orc, tau=1e-12, delta=None):
    """orc: oracle result forced on the GPU pivots. Returns (#exact, #steps);
    raises AssertionError at a pivot outside the tolerance window."""
    exact = 0
    for t, st in enumerate(orc.trace):
        for stage, d in (("row", st.row), ("col", st.col)):
            if not math.isfinite(d.total):
                continue            # step replayed without masses
            if d.drawn == d.used:
                exact += stage == "row"
                continue
            win = tau * d.total
            if delta is not None:
                win += delta[t] * d.total if stage == "row" else 0.0
            assert d.lo - win <= d.target < d.hi + win, (
                f"step {t} {stage}: GPU index {d.used} bin [{d.lo}, {d.hi}) vs oracle draw "
                f"{d.drawn} target {d.target} (T={d.total}, window {win})")
    return exact, len(orc.trace)


def check_trace_self(trace, piv):
    """GPU sampler exactness: each drawn index's bin, in the GPU's own prefix
    sums, contains the GPU's own target (trace words 0..11)."""
    tr = np.asarray(trace)
    for t in range(tr.shape[0]):
        T, ti, lo, hi, Ti, tj, loj, hij = tr[t, :8]
        assert lo <= ti < hi, (t, lo, ti, hi)
        assert loj <= tj < hij, (t, loj, tj, hij)
        assert 0 <= ti < T and 0 <= tj < Ti
        assert int(tr[t, 10]) == int(piv[t, 0]) and int(tr[t, 11]) == int(piv[t, 1])


def check_draws_ref(trace, tau=1e-12):
    """As check_draws, for the C++ oracle's trace words (oracle/ref.py): per
    step its own row target u1*T and the edges [lo, hi) of the used (GPU)
    row's bin in its own prefix sums, and the same for the column. The
    oracle's own draw equals the GPU index exactly when lo <= target < hi.
    Returns (#rows exact, #columns exact, #steps)."""
    tr = np.asarray(trace)
    ex_r = ex_c = 0
    for t in range(tr.shape[0]):
        for stage, (T, tgt, lo, hi) in (("row", tr[t, 0:4]), ("col", tr[t, 4:8])):
            if not math.isfinite(T):
                continue
            if lo <= tgt < hi:
                ex_r += stage == "row"
                ex_c += stage == "col"
                continue
            win = tau * T
            assert lo - win <= tgt < hi + win, (
                f"step {t} {stage}: GPU bin [{lo}, {hi}) in the oracle's prefix sums vs the "
                f"oracle's target {tgt} (T={T}, window {win})")
    return ex_r, ex_c, tr.shape[0]
