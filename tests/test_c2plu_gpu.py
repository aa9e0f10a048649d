"""C2PLU (complete 2-norm pivoting, Sec. 2.3.3; RPLU_FLAG_C2PLU) on the GPU
against the oracle's C2PLU.

The choice is an argmax, taken on both sides in FP64 over masses that agree
to rounding; the random inputs keep the largest masses well apart, so the
pivots must be identical. FP64 / complex128: L, U and the final Schur
complement agree within 1e-10. FP32 / complex64: the oracle runs in FP64 on
the single-precision input and the factors agree within 1e-5 (printed). Ties: on
+-1 Hadamard inputs every step has exact ties on both sides (small integers
are exact in every precision), which go to the smallest index. The fused
and the wide pivot forms agree bit for bit; the Cauchy-like path agrees with
the oracle's Cauchy-like C2PLU; batches and the server reject the flag.
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


def _check(res, orc, tol):
    assert res.rank == orc.rank and res.stop == orc.stop
    assert np.array_equal(res.piv.cpu().numpy(), orc.piv), (res.piv.cpu().numpy(), orc.piv)
    fa = np.sqrt(orc.a_fro2)
    if orc.rank:
        a_t = np.array([orc.U[t, orc.piv[t, 1]] for t in range(orc.rank)])
        assert parity.fro((res.L.cpu().numpy() - orc.L) * a_t) <= tol * fa
        assert parity.rel(res.U.cpu().numpy(), orc.U) <= tol


@pytest.mark.parametrize("dt", ["r64", "c128", "r32", "c64"])
@pytest.mark.parametrize("shape", [(60, 45), (33, 700), (513, 129)])
def test_c2plu_dense_matches_oracle(rplu_lib, dt, shape):
    n, m = shape
    A = W.random_dense(n, m, seed=71 + n, complex_=dt in ("c128", "c64"))
    t = torch.from_numpy(A).to(TORCH[dt])
    A_in = t.to(WIDE[dt]).numpy()
    k = min(20, n, m)
    Ad = t.to(DEV)
    res = rplu_lib.rplu_dense(Ad, k=k, flags=rplu_lib.RPLU_FLAG_C2PLU)
    orc = O.rplu_dense(A_in, k=k, greedy=True)
    tol = 1e-10 if dt in ("r64", "c128") else 1e-5
    _check(res, orc, tol)
    S_g = Ad.cpu().to(WIDE[dt]).numpy()
    err = parity.rel(S_g, orc.S, scale=np.sqrt(orc.a_fro2))
    print(f"c2plu {dt} {n}x{m}: ||S_gpu - S_orc|| / ||A|| = {err:.2e}", flush=True)
    assert err <= tol


def test_c2plu_dense_wide_form_matches_oracle(rplu_lib):
    """n > 12288 takes the wide pivot kernels (last-arriving workgroup)."""
    A = W.random_dense(12300, 40, seed=5)
    Ad = torch.from_numpy(A).to(DEV)
    res = rplu_lib.rplu_dense(Ad, k=12, flags=rplu_lib.RPLU_FLAG_C2PLU)
    _check(res, O.rplu_dense(A, k=12, greedy=True), 1e-10)


@pytest.mark.parametrize("dt", ["r32", "c128"])
def test_c2plu_forms_bitwise(rplu_lib, dt):
    A = W.random_dense(200, 150, seed=17, complex_=dt == "c128")
    t = torch.from_numpy(A).to(TORCH[dt]).to(DEV)
    a1, a2 = t.clone(), t.clone()
    F = rplu_lib.RPLU_FLAG_C2PLU
    r1 = rplu_lib.rplu_dense(a1, k=40, flags=F)
    r2 = rplu_lib.rplu_dense(a2, k=40, flags=F | rplu_lib.RPLU_FLAG_SPLIT_SAMPLER)
    assert r1.rank == r2.rank == 40
    assert torch.equal(r1.piv, r2.piv) and torch.equal(r1.L, r2.L) and torch.equal(r1.U, r2.U)
    assert torch.equal(a1, a2)


@pytest.mark.parametrize("dt", ["r64", "r32"])
def test_c2plu_ties_go_to_smallest_index(rplu_lib, dt):
    H = np.array([[1.0]])
    for _ in range(4):
        H = np.block([[H, H], [H, -H]])        # 16 x 16, all row masses equal
    Ad = torch.from_numpy(H).to(TORCH[dt]).to(DEV)
    res = rplu_lib.rplu_dense(Ad, flags=rplu_lib.RPLU_FLAG_C2PLU)
    orc = O.rplu_dense(H, greedy=True)
    assert tuple(int(v) for v in orc.piv[0]) == (0, 0)
    _check(res, orc, 1e-12)
    assert torch.count_nonzero(Ad) == 0          # a full-rank run ends at S = 0


@pytest.mark.parametrize("p", [1, 2])
def test_c2plu_cauchy_matches_oracle(rplu_lib, p):
    x, y, G, B = W.cauchy_like_random(300, 250, p, seed=9 + p)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)   # noqa: E731
    res = rplu_lib.rplu_cauchy(t(x), t(y), t(G), t(B), k=15, flags=rplu_lib.RPLU_FLAG_C2PLU)
    orc = O.rplu_cauchy(x, y, G, B, k=15, greedy=True)
    _check(res, orc, 1e-10)


def test_c2plu_rejected_in_batches(rplu_lib):
    mats = [torch.from_numpy(W.random_dense(8, 8, seed=1)).to(torch.float32).to(DEV)]
    with pytest.raises(rplu_lib.RPLUError):
        rplu_lib.rplu_batched(mats, k=2, flags=rplu_lib.RPLU_FLAG_C2PLU)
