"""CPLU (complete pivoting, Sec. 1; RPLU_FLAG_CPLU) on the GPU against the
oracle's CPLU.

The choice is an argmax of |S_ij|^2, taken on both sides in FP64 over
values that agree to rounding; the random inputs keep the largest entries
well apart, so the pivots must be the oracle's own. FP64 / complex128: L, U
and the final Schur complement within 1e-10. FP32 / complex64: the oracle
runs in FP64 on the single-precision input; L a_t, U and the final Schur
complement within 1e-5 of ||A||_F (the errors are printed). Ties: on +-1
Hadamard inputs and on [[1, 2], [2, 0]] the equal entries go to the first in
row-major order on both sides. The fused and wide pivot forms, and the eager
and deferred sweeps, agree bit for bit. Cauchy-like runs, batches, the
server and the combinations with C2PLU or column masses are refused.
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


def _check(res, orc, tol, S_g=None, tag=""):
    assert res.rank == orc.rank and res.stop == orc.stop, tag
    assert np.array_equal(res.piv.cpu().numpy(), orc.piv), (tag, res.piv.cpu().numpy(), orc.piv)
    fa = np.sqrt(orc.a_fro2)
    errs = {}
    if orc.rank:
        a_t = np.array([orc.U[t, orc.piv[t, 1]] for t in range(orc.rank)])
        errs["L"] = parity.fro((res.L.cpu().numpy() - orc.L) * a_t) / fa
        errs["U"] = parity.fro(res.U.cpu().numpy() - orc.U) / fa
    if S_g is not None:
        errs["S"] = parity.fro(S_g - orc.S) / fa
    print(f"{tag}: rank {res.rank} " + " ".join(f"{k} {v:.2e}" for k, v in errs.items()),
          flush=True)
    for k, v in errs.items():
        assert v <= tol, (tag, k, v)


@pytest.mark.parametrize("dt", ["r64", "c128", "r32", "c64"])
@pytest.mark.parametrize("shape", [(60, 45), (33, 700), (513, 129)])
def test_cplu_dense_matches_oracle(rplu_lib, dt, shape):
    n, m = shape
    A = W.random_dense(n, m, seed=91 + n, complex_=dt in ("c128", "c64"))
    t = torch.from_numpy(A).to(TORCH[dt])
    A_in = t.to(WIDE[dt]).numpy()
    k = min(24, n, m)
    Ad = t.to(DEV)
    res = rplu_lib.rplu_dense(Ad, k=k, flags=rplu_lib.RPLU_FLAG_CPLU)
    orc = O.rplu_dense(A_in, k=k, complete=True)
    tol = 1e-10 if dt in ("r64", "c128") else 1e-5
    _check(res, orc, tol, Ad.cpu().to(WIDE[dt]).numpy(), f"{dt} {n}x{m}")


def test_cplu_tolerance_stop(rplu_lib):
    """A tolerance run stops at the oracle's step (FP64, decaying spectrum)."""
    A = W.dense_with_spectrum(300, 260, 0.7 ** np.arange(260), seed=4)
    Ad = torch.from_numpy(A).to(DEV)
    res = rplu_lib.rplu_dense(Ad, k=0, tol=1e-6, flags=rplu_lib.RPLU_FLAG_CPLU)
    orc = O.rplu_dense(A, tol=1e-6, complete=True)
    assert orc.stop == O.STOP_TOL
    _check(res, orc, 1e-10, Ad.cpu().numpy(), "tol 1e-6")


def test_cplu_wide_form_matches_oracle(rplu_lib):
    """n > 12288 takes the wide pivot kernels (last-arriving workgroup)."""
    A = W.random_dense(12300, 40, seed=6)
    Ad = torch.from_numpy(A).to(DEV)
    res = rplu_lib.rplu_dense(Ad, k=12, flags=rplu_lib.RPLU_FLAG_CPLU)
    _check(res, O.rplu_dense(A, k=12, complete=True), 1e-10, Ad.cpu().numpy(), "wide")


@pytest.mark.parametrize("dt", ["r32", "c128"])
def test_cplu_forms_and_sweeps_bitwise(rplu_lib, dt):
    A = W.random_dense(300, 257, seed=19, complex_=dt == "c128")
    t = torch.from_numpy(A).to(TORCH[dt]).to(DEV)
    F = rplu_lib.RPLU_FLAG_CPLU
    runs = []
    for extra in (rplu_lib.RPLU_FLAG_EAGER_SWEEP,
                  rplu_lib.RPLU_FLAG_EAGER_SWEEP | rplu_lib.RPLU_FLAG_SPLIT_SAMPLER,
                  rplu_lib.RPLU_FLAG_LAZY_SWEEP,
                  rplu_lib.RPLU_FLAG_LAZY_SWEEP | rplu_lib.RPLU_FLAG_SPLIT_SAMPLER):
        a = t.clone()
        r = rplu_lib.rplu_dense(a, k=45, flags=F | extra)
        torch.cuda.synchronize()
        runs.append((r, a))
    r0, a0 = runs[0]
    assert r0.rank == 45
    for r, a in runs[1:]:
        assert torch.equal(r0.piv, r.piv) and torch.equal(r0.L, r.L) and torch.equal(r0.U, r.U)
        assert torch.equal(a0, a)


@pytest.mark.parametrize("dt", ["r64", "r32"])
def test_cplu_ties_go_to_first_in_row_major_order(rplu_lib, dt):
    H = np.array([[1.0]])
    for _ in range(4):
        H = np.block([[H, H], [H, -H]])        # 16 x 16: every entry of equal modulus
    Ad = torch.from_numpy(H).to(TORCH[dt]).to(DEV)
    res = rplu_lib.rplu_dense(Ad, flags=rplu_lib.RPLU_FLAG_CPLU)
    orc = O.rplu_dense(H, complete=True)
    assert [tuple(int(v) for v in p) for p in orc.piv[:2]] == [(0, 0), (1, 1)]
    _check(res, orc, 1e-12, tag=f"hadamard {dt}")
    assert torch.count_nonzero(Ad) == 0          # a full-rank run ends at S = 0
    B = torch.tensor([[1.0, 2.0], [2.0, 0.0]], dtype=TORCH[dt], device=DEV)
    r = rplu_lib.rplu_dense(B, k=1, flags=rplu_lib.RPLU_FLAG_CPLU)
    assert tuple(int(v) for v in r.piv[0]) == (0, 1)


def test_cplu_refusals(rplu_lib):
    A = torch.randn(20, 30, device=DEV, dtype=torch.float64)
    F = rplu_lib.RPLU_FLAG_CPLU
    with pytest.raises(rplu_lib.RPLUError) as e:
        rplu_lib.rplu_dense(A.clone(), k=3, flags=F | rplu_lib.RPLU_FLAG_C2PLU)
    assert e.value.status == -1
    with pytest.raises(rplu_lib.RPLUError) as e:
        rplu_lib.rplu_dense(A.clone(), k=3, flags=F | rplu_lib.RPLU_FLAG_COLMASS)
    assert e.value.status == -6
    x, y, G, B = W.cauchy_like_random(40, 30, 1, seed=2)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)   # noqa: E731
    with pytest.raises(rplu_lib.RPLUError) as e:
        rplu_lib.rplu_cauchy(t(x), t(y), t(G), t(B), k=3, flags=F)
    assert e.value.status == -6
    mats = [torch.from_numpy(W.random_dense(8, 8, seed=1)).to(torch.float32).to(DEV)]
    with pytest.raises(rplu_lib.RPLUError):
        rplu_lib.rplu_batched(mats, k=2, flags=F)
