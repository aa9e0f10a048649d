"""FP64 matrix-core verification (rplu_verify) against the oracle in FP64.

The kernel forms A - L U tile by tile with v_mfma_f64_16x16x4f64 and reduces
three squared Frobenius norms; the oracle (factorization_check) computes the
same three numbers from the same (widened) values by their definitions with
a library matmul. Sums of squares of the same
terms in another order agree to a few ulps of the total, and the FP64
products of L U differ by at most k ulps per entry, so 1e-10 relative to
||A||^2 (or to the summed magnitudes for the near-zero gap) is a safe bar.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import rplu as O

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _ref(A, L, U, S):
    A, L, U = (x.detach().cpu().double().numpy() for x in (A, L, U))
    out = O.factorization_check(A, L, U, None if S is None else S.detach().cpu().double().numpy())
    scale = float(np.sum(np.abs(A) ** 2) + np.sum((np.abs(L) @ np.abs(U)) ** 2))
    return out, scale


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n,m,k", [(1, 1, 1), (5, 7, 0), (130, 257, 19), (128, 128, 16),
                                   (300, 129, 37), (257, 1000, 64), (1025, 513, 3)])
def test_verify_random(rplu_lib, dtype, n, m, k):
    g = torch.Generator().manual_seed(n * 7 + m * 3 + k)
    A = torch.randn(n, m, generator=g, dtype=torch.float64).to(dtype).to(DEV)
    S = torch.randn(n, m, generator=g, dtype=torch.float64).to(dtype).to(DEV)
    Lt = torch.randn(max(k, 1), n + 3, generator=g, dtype=torch.float64).to(dtype).to(DEV)
    L = Lt[:k, :n].T                       # n x k view with column stride n + 3
    U = torch.randn(k, m, generator=g, dtype=torch.float64).to(dtype).to(DEV)
    got = rplu_lib.rplu_verify(A, L if k else None, U if k else None, S)
    ref, scale = _ref(A, L, U, S)
    assert abs(got["a_fro2"] - ref["a_fro2"]) <= 1e-12 * ref["a_fro2"]
    assert abs(got["err_fro2"] - ref["err_fro2"]) <= 1e-10 * scale
    assert abs(got["schur_gap_fro2"] - ref["schur_gap_fro2"]) <= 1e-10 * scale
    again = rplu_lib.rplu_verify(A, L if k else None, U if k else None, S)
    assert again == got                    # fixed reduction order


def test_verify_exact_factorisation(rplu_lib):
    """A = L U exactly (integer-valued factors, FP64): every product and sum
    is exact, so ||A - L U|| must be exactly 0."""
    g = torch.Generator().manual_seed(5)
    n, m, k = 300, 200, 40
    L = torch.randint(-3, 4, (n, k), generator=g).double()
    U = torch.randint(-3, 4, (k, m), generator=g).double()
    A = (L @ U).to(DEV)
    Lc = L.T.contiguous().to(DEV).T        # column-major n x k
    got = rplu_lib.rplu_verify(A, Lc, U.to(DEV))
    assert got["err_fro2"] == 0.0
    assert got["a_fro2"] == float((A.cpu() ** 2).sum())


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_verify_after_rplu(rplu_lib, dtype):
    """After a dense run, A - L U equals the Schur complement left in the
    buffer up to rounding, and ||A - L U||^2 matches the run's own total."""
    A0 = torch.from_numpy(W.random_dense(400, 300, seed=12)).to(dtype).to(DEV)
    S = A0.clone()
    res = rplu_lib.rplu_dense(S, k=60, seed=3)
    v = rplu_lib.rplu_verify(A0, res.L, res.U, S)
    u = 2.0 ** -52 if dtype == torch.float64 else 2.0 ** -23
    assert v["schur_gap_fro2"] <= (60 * 4 * u) ** 2 * v["a_fro2"] * 60
    assert abs(v["err_fro2"] - res.res_fro2) <= 1e-3 * res.res_fro2 + (60 * 4 * u) ** 2 * v["a_fro2"] * 60
    assert abs(v["a_fro2"] - res.a_fro2) <= 1e-12 * res.a_fro2


def test_verify_errors(rplu_lib):
    A = torch.zeros(4, 4, dtype=torch.complex128, device=DEV)
    with pytest.raises(ValueError):
        rplu_lib.rplu_verify(A, None, None)
    B = torch.zeros(4, 4, dtype=torch.float64, device=DEV)
    L = torch.zeros(5, 2, dtype=torch.float64, device=DEV)
    U = torch.zeros(2, 4, dtype=torch.float64, device=DEV)
    with pytest.raises(ValueError):
        rplu_lib.rplu_verify(B, L, U)
