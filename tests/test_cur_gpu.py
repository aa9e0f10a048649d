"""RPLU in CUR form (rplu_cur, Alg. 2) on the GPU against the oracle's
rplu_cur.

Every GPU operation other than reading A is FP64, so single-precision
storage is compared like double: the oracle runs in FP64 on the stored
values (FP32 -> FP64 is exact) and replays the GPU pivots, making its own
draw at every step. Checked, in all four dtypes and on shapes that span
several chunks with ragged tails: every pivot is the oracle's own draw (or
within 1e-12 T of the shared CDF edge); the row-norm estimates before every
draw agree within 1e-11 ||A||_F^2; the core agrees within 1e-13 cond(A[I,J])
relative and the approximation A[:, J] U A[I, :] within (1e-12 + 1e-15
cond(A[I,J])) ||A||_F; A is
not written. Also: the dense path's pivots and factors on the same seed,
tolerance and exhaustion stops, C2PLU, the wide draw kernels, unaligned rows,
graph replay against plain launches, refusals.
"""
import numpy as np
import pytest
import torch

import parity
import workloads as W
from oracle import rplu as O

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TORCH = {"r64": torch.float64, "c128": torch.complex128, "r32": torch.float32, "c64": torch.complex64}
WIDE = {"r64": torch.float64, "c128": torch.complex128, "r32": torch.float64, "c64": torch.complex128}


def _input(n, m, dt, seed, lda=None):
    A = W.random_dense(n, m, seed=seed, complex_=dt in ("c128", "c64"))
    t = torch.from_numpy(np.ascontiguousarray(A)).to(TORCH[dt])
    if lda is None:
        return t.to(DEV)
    buf = torch.zeros((n, lda), dtype=TORCH[dt])
    buf[:, :m] = t
    return buf.to(DEV)[:, :m]


def _approx(A, I, J, Uc):
    return A[:, J] @ Uc @ A[I, :]


def _check(rplu, Ad, r, tag, seed=0, stream=0, greedy=False, tol=0.0, k=0):
    A64 = Ad.cpu().to(WIDE[{torch.float32: "r32", torch.float64: "r64", torch.complex64: "c64",
                            torch.complex128: "c128"}[Ad.dtype]]).numpy()
    piv = r.piv.cpu().numpy()
    o = O.rplu_cur(A64, k=k, tol=tol, seed=seed, stream=stream, greedy=greedy,
                   forced=[tuple(p) for p in piv] + [None], keep_masses=True)
    assert (o.rank, o.stop) == (r.rank, r.stop), (tag, o.rank, r.rank, o.stop, r.stop)
    assert np.array_equal(o.piv, piv), tag
    if not greedy:
        exact, steps = parity.check_draws(o, tau=1e-12)
    else:
        exact = steps = r.rank
        assert all(st.row.drawn == st.row.used and st.col.drawn == st.col.used for st in o.trace)
    T0 = o.a_fro2
    assert abs(r.a_fro2 - T0) <= 1e-13 * T0 and abs(r.res_fro2 - o.res_fro2) <= 1e-11 * T0, tag
    if r.rowmass is not None and r.rank:
        dm = np.abs(r.rowmass.cpu().numpy() - np.stack(o.masses)).max()
        assert dm <= 1e-11 * T0, (tag, dm / T0)
    if r.rank:
        I, J = o.I, o.J
        Wm = A64[np.ix_(I, J)]
        Ug = r.Ucore.cpu().numpy()
        du = parity.rel(Ug, o.Uc)
        assert du <= 1e-13 * np.linalg.cond(Wm) + 1e-13, (tag, du)
        da = parity.fro(_approx(A64, I, J, Ug) - _approx(A64, I, J, o.Uc)) / np.sqrt(T0)
        assert da <= 1e-15 * np.linalg.cond(Wm) + 1e-12, (tag, da)
    print(f"{tag}: rank {r.rank} stop {r.stop}, {exact}/{steps} own draws", flush=True)
    return o


@pytest.mark.parametrize("dt", ["r64", "c128", "r32", "c64"])
@pytest.mark.parametrize("n,m,k", [(300, 257, 60), (1000, 90, 40), (130, 1100, 50),
                                   (513, 700, 100)])
def test_cur_matches_oracle(rplu_lib, dt, n, m, k):
    Ad = _input(n, m, dt, seed=n + 3 * m)
    A0 = Ad.clone()
    r = rplu_lib.rplu_cur(Ad, k=k, seed=7, stream=n, want_rowmass=True, want_trace=True)
    torch.cuda.synchronize()
    assert torch.equal(Ad, A0), "rplu_cur wrote A"
    parity.check_trace_self(r.trace.cpu().numpy(), r.piv.cpu().numpy())
    _check(rplu_lib, Ad, r, f"{dt} {n}x{m}", seed=7, stream=n, k=k)


def test_cur_matches_dense_path(rplu_lib):
    """FP64: the dense path on the same seed and stream takes the same pivots
    (the estimates are the dense row masses up to rounding), and
    A[:, J] U A[I, :] equals its L U."""
    A = W.random_dense(600, 500, seed=21)
    Ad = torch.from_numpy(A).to(DEV)
    c = rplu_lib.rplu_cur(Ad, k=80, seed=3, stream=9)
    d = rplu_lib.rplu_dense(Ad.clone(), k=80, seed=3, stream=9)
    assert torch.equal(c.piv, d.piv)
    piv = c.piv.cpu().numpy()
    LU = d.L.cpu().numpy() @ d.U.cpu().numpy()
    ap = _approx(A, piv[:, 0], piv[:, 1], c.Ucore.cpu().numpy())
    assert parity.fro(ap - LU) <= 1e-11 * np.linalg.norm(A)


@pytest.mark.parametrize("dt", ["r32", "r64"])
def test_cur_tolerance_and_exhaustion(rplu_lib, dt):
    """A tolerance stop at the oracle's step where the core is moderately
    conditioned (tol 1e-4, cond(A[I, J]) about 1e6). At tol 1e-6 on the same
    spectrum cond(A[I, J]) reaches 1e9 and the estimates carry relative
    errors of about 1e-2 on both sides (the block-inverse update loses
    accuracy with the conditioning of the core), so the stop step is only
    compared within a few steps; the true residual of the returned index
    sets (closed form) is then within 1.2 tol."""
    sig = 0.8 ** np.arange(350)
    Ad = torch.from_numpy(W.dense_with_spectrum(400, 350, sig, seed=5)).to(TORCH[dt]).to(DEV)
    r = rplu_lib.rplu_cur(Ad, k=0, tol=1e-4, seed=1, want_rowmass=True)
    assert r.stop == rplu_lib.RPLU_STOP_TOL
    _check(rplu_lib, Ad, r, f"tol 1e-4 {dt}", seed=1, tol=1e-4)
    r = rplu_lib.rplu_cur(Ad, k=0, tol=1e-6, seed=1)
    assert r.stop == rplu_lib.RPLU_STOP_TOL
    A64 = Ad.cpu().double().numpy()
    o = O.rplu_cur(A64, tol=1e-6, seed=1)
    assert o.stop == O.STOP_TOL and abs(o.rank - r.rank) <= 4, (o.rank, r.rank)
    piv = r.piv.cpu().numpy()
    S = O.schur_closed_form(A64, piv[:, 0], piv[:, 1])
    res = np.linalg.norm(S) / np.sqrt(r.a_fro2)
    print(f"tol 1e-6 {dt}: rank {r.rank} (oracle {o.rank}), true residual {res:.3e}", flush=True)
    assert res <= 1.2e-6
    # rank 11 (in single precision, rank 11 plus rounding of relative size 1e-7)
    Ar = torch.from_numpy(W.rank_r_dense(200, 180, 11, seed=6)).to(TORCH[dt]).to(DEV)
    tol = 1e-7 if dt == "r64" else 1e-5
    r = rplu_lib.rplu_cur(Ar, k=0, tol=tol, seed=3)
    assert r.rank == 11 and r.stop == rplu_lib.RPLU_STOP_TOL
    A64 = Ar.cpu().double().numpy()
    piv = r.piv.cpu().numpy()
    ap = _approx(A64, piv[:, 0], piv[:, 1], r.Ucore.cpu().numpy())
    assert parity.fro(ap - A64) <= (1e-10 if dt == "r64" else 1e-6) * np.linalg.norm(A64)


@pytest.mark.parametrize("dt", ["r64", "c128"])
def test_cur_c2plu(rplu_lib, dt):
    Ad = _input(260, 230, dt, seed=31)
    r = rplu_lib.rplu_cur(Ad, k=40, flags=rplu_lib.RPLU_FLAG_C2PLU, want_rowmass=True)
    _check(rplu_lib, Ad, r, f"c2plu {dt}", greedy=True, k=40)


def test_cur_wide_unaligned_and_graph(rplu_lib):
    """More than 12288 rows or columns (several wide workgroups per draw),
    rows of odd pitch (element loads), and graph replay against plain
    launches, bit for bit."""
    A1 = _input(12300, 40, "r64", seed=41)
    _check(rplu_lib, A1, rplu_lib.rplu_cur(A1, k=20, seed=4, want_rowmass=True), "tall", seed=4,
           k=20)
    A2 = _input(40, 12300, "r32", seed=42)
    _check(rplu_lib, A2, rplu_lib.rplu_cur(A2, k=20, seed=5, want_rowmass=True), "wide", seed=5,
           k=20)
    A3 = _input(333, 301, "r32", seed=43, lda=305)
    r3 = rplu_lib.rplu_cur(A3, k=45, seed=6, want_rowmass=True)
    _check(rplu_lib, A3, r3, "unaligned", seed=6, k=45)
    r4 = rplu_lib.rplu_cur(A3, k=45, seed=6, flags=rplu_lib.RPLU_FLAG_NO_GRAPH)
    assert torch.equal(r3.piv, r4.piv) and torch.equal(r3.Ucore, r4.Ucore)
    assert r3.res_fro2 == r4.res_fro2


def test_cur_refusals(rplu_lib):
    A = torch.randn(30, 20, device=DEV, dtype=torch.float64)
    for f in (rplu_lib.RPLU_FLAG_CPLU, rplu_lib.RPLU_FLAG_COLMASS, rplu_lib.RPLU_FLAG_REFRESH):
        with pytest.raises(rplu_lib.RPLUError) as e:
            rplu_lib.rplu_cur(A, k=3, flags=f)
        assert e.value.status == -6
    B = torch.randn(2100, 2100, device=DEV, dtype=torch.float32)
    with pytest.raises(rplu_lib.RPLUError) as e:
        rplu_lib.rplu_cur(B, k=0)
    assert e.value.status == -6
