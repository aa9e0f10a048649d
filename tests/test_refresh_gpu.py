"""Residual replacement (RPLU_FLAG_REFRESH) on the GPU.

A single-precision sweep keeps the rounding errors of every earlier update in
S, which puts a floor under ||S|| (about 1e-6 ||A||_F for sigma_i = 0.9^i at
n = 2000), so a tolerance of 1e-6 stalls. With the flag, the run replaces S
by the true residual A - L U formed in FP64 each time ||S|| has fallen
100-fold (and when the stall rule fires) and goes on. Checked: the run
reaches the tolerance where the plain run stalls, in at most 1.5 times the
steps of an FP64 run; the FP64 check ||A - L U|| of the returned factors is within the
tolerance; the factors agree with the oracle replaying the same pivots on the
FP64 A (1e-5 of ||A||, over the steps above the 1e-5 residual); batches
reproduce rplu_dense bit for bit with the flag; the flag's argument errors.
"""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import ref as R

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _compare_steps(o, target=1e-5):
    """Steps of a forced oracle replay over which FP32 factors are compared
    with it: those taken while the oracle's residual is above target ||A||_F
    (trace word 0 is T = ||S^(t)||^2 before step t). Pivots drawn once the
    residual is at the single-precision rounding floor select entries whose
    exact values can be far smaller than the rounded ones, and the exact
    Schur complements under them grow; there the FP64 check of the factors
    is the bar."""
    tr = np.asarray(o.trace)
    for t in range(tr.shape[0]):
        if tr[t, 0] <= target * target * o.a_fro2:
            return t
    return tr.shape[0]


def _distinct_prefix(piv):
    """Steps before the first pivot row or column that was a pivot before
    (after a residual replacement an earlier pivot row holds the residual
    the stored factors leave there and may be drawn again; an exact replay
    has an exact zero there)."""
    rows, cols = set(), set()
    for t, (i, j) in enumerate(np.asarray(piv)):
        if int(i) in rows or int(j) in cols:
            return t
        rows.add(int(i))
        cols.add(int(j))
    return len(piv)


def _decaying(n, m, seed, r=0.9):
    k = min(n, m)
    sig = r ** np.arange(1, k + 1)
    sig[sig < 1e-16] = 0.0
    return W.dense_with_spectrum(n, m, sig, seed=seed)


@pytest.mark.parametrize("n,m", [(2000, 2000), (1500, 1800)])
def test_refresh_reaches_tolerance(rplu_lib, n, m):
    A64 = _decaying(n, m, seed=n + m)
    A = torch.from_numpy(A64).float().to(DEV)
    tol = 1e-6
    flags = rplu_lib.RPLU_FLAG_STALL_STOP
    plain = rplu_lib.rplu_dense(A.clone(), k=0, tol=tol, seed=1, stream=2, flags=flags)
    ref = rplu_lib.rplu_dense(A.clone(), k=0, tol=tol, seed=1, stream=2, flags=flags, A_orig=A)
    print(f"plain: stop {plain.stop} rank {plain.rank} residual "
          f"{math.sqrt(plain.res_fro2 / plain.a_fro2):.2e}; refreshed: stop {ref.stop} rank "
          f"{ref.rank} residual {math.sqrt(ref.res_fro2 / ref.a_fro2):.2e}", flush=True)
    assert plain.stop == rplu_lib.RPLU_STOP_STALL      # the rounding floor is above 1e-6
    assert ref.stop == rplu_lib.RPLU_STOP_TOL
    # with replacements the run needs a few more steps than an FP64 run (the
    # FP32 rounding of the stored factors, about u32 ||L|| ||U||, is part of
    # every replaced residual), far fewer than the plain run spends stalling
    r64 = rplu_lib.rplu_dense(A.double(), k=0, tol=tol, seed=1, stream=2, flags=flags)
    print(f"FP64 run: stop {r64.stop} rank {r64.rank}", flush=True)
    assert r64.stop == rplu_lib.RPLU_STOP_TOL and ref.rank <= 1.5 * r64.rank
    v = rplu_lib.rplu_verify(A, ref.L, ref.U)
    err = math.sqrt(v["err_fro2"] / v["a_fro2"])
    print(f"FP64 check of the factors: ||A - LU|| / ||A|| = {err:.3e}", flush=True)
    assert err <= tol
    # the first replacement comes when ||S|| has fallen 100-fold, long before
    # the plain run's stall; the two runs are the same up to it
    assert ref.refreshes >= 2 and 0 < ref.first_refresh < plain.rank
    assert torch.equal(ref.piv[:ref.first_refresh], plain.piv[:ref.first_refresh])
    # the oracle replays the GPU pivots on the FP64 values of A (protocol P2)
    piv = ref.piv.cpu().numpy()
    kd = _distinct_prefix(piv)
    o = R.rplu_dense(A.double().cpu().numpy(), k=kd, forced=[tuple(p) for p in piv[:kd]])
    tc = _compare_steps(o)
    LU_g = ref.L[:, :tc].double().cpu().numpy() @ ref.U[:tc].double().cpu().numpy()
    LU_o = o.L[:, :tc] @ o.U[:tc]
    d = np.linalg.norm(LU_g - LU_o) / math.sqrt(o.a_fro2)
    print(f"first {tc} steps: ||L U (GPU) - L U (oracle, same pivots)|| / ||A|| = {d:.3e}",
          flush=True)
    assert d <= 1e-5


def test_refresh_batched_equals_dense(rplu_lib):
    """Batches with the flag: every instance bit for bit rplu_dense alone
    with the flag (the residual replacement at the same step, the resumed
    launch from there), including instances that never stall."""
    rng = np.random.default_rng(5)
    As, origs = [], []
    for q in range(6):
        n = int(rng.integers(900, 2048))
        m = int(rng.integers(900, 2048))
        A = torch.from_numpy(_decaying(n, m, seed=100 + q, r=0.88 + 0.01 * q)).float().to(DEV)
        origs.append(A)
        As.append(A.clone())
    tol = 1e-6
    flags = rplu_lib.RPLU_FLAG_STALL_STOP | rplu_lib.RPLU_FLAG_REFRESH
    plan = rplu_lib.BatchPlan(As, k=0, tol=tol, seed=3, streams=list(range(6)), flags=flags,
                              A_origs=origs)
    plan.run()
    res = plan.results()
    n_ref = 0
    for q in range(6):
        Aa = origs[q].clone()
        a = rplu_lib.rplu_dense(Aa, k=0, tol=tol, seed=3, stream=q,
                                flags=rplu_lib.RPLU_FLAG_STALL_STOP, A_orig=origs[q])
        b = res[q]
        assert (b.rank, b.stop) == (a.rank, a.stop), q
        assert torch.equal(b.piv, a.piv) and torch.equal(b.U, a.U) and torch.equal(b.L, a.L), q
        assert torch.equal(As[q], Aa), q               # the final Schur complements
        n_ref += plan.infos[q].refreshes
    print(f"{n_ref} residual replacements over 6 instances", flush=True)
    assert n_ref >= 1


def test_refresh_argument_errors(rplu_lib):
    A = torch.randn(40, 30, device=DEV)
    with pytest.raises(rplu_lib.RPLUError) as e:
        rplu_lib.rplu_dense(A.clone(), k=5, flags=rplu_lib.RPLU_FLAG_REFRESH)   # no A_orig
    assert e.value.status == -1
    Ac = torch.randn(40, 30, device=DEV, dtype=torch.complex64)
    with pytest.raises(rplu_lib.RPLUError) as e:
        rplu_lib.rplu_dense(Ac.clone(), k=5, A_orig=Ac)
    assert e.value.status == -6
