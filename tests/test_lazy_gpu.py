"""The deferred dense sweep (RPLU_FLAG_LAZY_SWEEP) against the eager sweep.

The deferred sweep keeps S^(tb) in memory, applies the pending rank-1
updates of the window tb..t in registers in the eager sweep's order, and
writes S back every RPLU_LAZY_STEPS steps (and at the last step, or after a
stop in the middle of a window). It must give the eager sweep's results bit
for bit: pivots, L, U, the final Schur complement, every step's row masses,
the trace words and the totals, in all four dtypes, through both pivot-draw
forms, with tolerance, stall and rank stops landing inside and at the end of
windows, forced pivots, unaligned rows and residual replacement; and agree
with the oracle (FP64: the oracle's own draws, 1e-10).
"""
import numpy as np
import pytest
import torch

import parity
import workloads as W
from oracle import ref as R

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

DT = {"r32": torch.float32, "r64": torch.float64, "c64": torch.complex64,
      "c128": torch.complex128}


def _input(n, m, dt, seed, lda=None):
    A = W.random_dense(n, m, seed=seed, complex_=DT[dt].is_complex)
    t = torch.from_numpy(np.ascontiguousarray(A)).to(DT[dt]).to(DEV)
    if lda is None:
        return t
    buf = torch.zeros((n, lda), dtype=DT[dt], device=DEV)
    buf[:, :m] = t
    return buf[:, :m]


def _clone(A0):
    """A copy with A0's row pitch."""
    if A0.is_contiguous():
        return A0.clone()
    n, m = A0.shape
    buf = torch.zeros((n, A0.stride(0)), dtype=A0.dtype, device=A0.device)
    buf[:, :m] = A0
    return buf[:, :m]


def _run(rplu, A0, flags, **kw):
    A = _clone(A0)
    r = rplu.rplu_dense(A, flags=flags, want_trace=True, want_rowmass=True, **kw)
    torch.cuda.synchronize()
    return r, A


def _equal(rplu, A0, **kw):
    flags = kw.pop("flags", 0)
    a, Sa = _run(rplu, A0, flags | rplu.RPLU_FLAG_EAGER_SWEEP, **kw)
    b, Sb = _run(rplu, A0, flags | rplu.RPLU_FLAG_LAZY_SWEEP, **kw)
    assert (a.rank, a.stop) == (b.rank, b.stop)
    assert a.a_fro2 == b.a_fro2 and a.res_fro2 == b.res_fro2
    for x, y in ((a.piv, b.piv), (a.L, b.L), (a.U, b.U), (Sa, Sb), (a.trace, b.trace),
                 (a.rowmass, b.rowmass)):
        assert torch.equal(x, y)
    return a, b


@pytest.mark.parametrize("dt", ["r32", "r64", "c64", "c128"])
@pytest.mark.parametrize("n,m,k", [(1, 1, 1), (7, 5, 0), (300, 257, 40), (513, 257, 16),
                                   (130, 1100, 23)])
def test_lazy_equals_eager(rplu_lib, dt, n, m, k):
    A0 = _input(n, m, dt, seed=n * 7 + m)
    _equal(rplu_lib, A0, k=k, seed=3, stream=n)


@pytest.mark.parametrize("dt", ["r32", "r64"])
def test_lazy_stops_inside_windows(rplu_lib, dt):
    """Tolerance stops at steps that are not window ends (the write-back after
    the run), the stall rule, exhaustion of a rank-r input, forced pivots."""
    A0 = torch.from_numpy(W.dense_with_spectrum(400, 350, 0.8 ** np.arange(350), seed=5))
    A0 = A0.to(DT[dt]).to(DEV)
    ranks = []
    for tol in (3e-2, 1e-3, 2e-5):
        a, _ = _equal(rplu_lib, A0, k=0, tol=tol, seed=1)
        assert a.stop == rplu_lib.RPLU_STOP_TOL
        ranks.append(a.rank)
    assert any(r % 8 != 0 for r in ranks), ranks       # a stop inside a window
    _equal(rplu_lib, A0, k=0, tol=1e-30, seed=2, flags=rplu_lib.RPLU_FLAG_STALL_STOP)
    Ar = torch.from_numpy(W.rank_r_dense(200, 180, 11, seed=6)).to(DT[dt]).to(DEV)
    a, _ = _equal(rplu_lib, Ar, k=0, seed=3)
    assert a.stop == rplu_lib.RPLU_STOP_EXHAUSTED
    b, _ = _equal(rplu_lib, A0, k=37, seed=9)           # another draw sequence on A0,
    _equal(rplu_lib, A0, k=37, seed=3, forced=b.piv.flatten())   # replayed


def test_lazy_unaligned_and_wide_draws(rplu_lib):
    """Rows of odd pitch (element packs instead of 16-byte ones), and more
    than 12288 rows (the wide pivot-draw kernels read the pivot row through
    the window)."""
    A0 = _input(333, 301, "r32", seed=9, lda=305)
    _equal(rplu_lib, A0, k=30, seed=4)
    A1 = _input(12289, 24, "r32", seed=10)
    _equal(rplu_lib, A1, k=20, seed=5)
    A2 = _input(24, 12289, "r64", seed=11)
    _equal(rplu_lib, A2, k=20, seed=6)


def test_lazy_with_refresh(rplu_lib):
    sig = 0.9 ** np.arange(1, 1201)
    A0 = torch.from_numpy(W.dense_with_spectrum(1200, 1100, sig[:1100], seed=7)).float().to(DEV)
    a, b = _equal(rplu_lib, A0, k=0, tol=1e-6, seed=2, flags=rplu_lib.RPLU_FLAG_STALL_STOP,
                  A_orig=A0)
    assert a.refreshes >= 1 and a.stop == rplu_lib.RPLU_STOP_TOL


def test_lazy_against_oracle(rplu_lib):
    """The deferred sweep on its own, FP64, against the oracle: every pivot is
    the oracle's own draw, factors and Schur complement within 1e-10."""
    A = W.random_dense(640, 520, seed=12)
    r, S = _run(rplu_lib, torch.from_numpy(A).to(DEV), rplu_lib.RPLU_FLAG_LAZY_SWEEP, k=60,
                seed=7, stream=1)
    piv = r.piv.cpu().numpy()
    o = R.rplu_dense(A, k=60, seed=7, stream=1, forced=[tuple(p) for p in piv])
    ex_r, ex_c, steps = parity.check_draws_ref(o.trace, tau=1e-12)
    assert steps == 60 and ex_r == 60
    assert parity.rel(r.U.cpu().numpy(), o.U) <= 1e-10
    assert parity.fro(S.cpu().numpy() - o.S) <= 1e-10 * np.sqrt(o.a_fro2)
