"""Distribution of whole GPU runs against exact enumeration (beyond the
first-pivot chi-square test): Monte Carlo means over many Philox streams of
the GPU's residual ||S^(k)||_F^2 against the exact expectation over every
pivot sequence (the oracle's Schur update, enumerated in tests/pins.py), to
within 4 standard errors. The streams are fixed, so each test is
deterministic.

- E||S^(k)||^2, k = 1, 2, 3, for 4 x 4 FP64 inputs (thm. doubling's
  quantity), through the batched kernel (one launch of 20000 instances per k)
  and, for a complex input, through rplu_dense;
- the unitary example of Sec. 3.1: E||A^(1)||^2 = 2(n - 1) for the
  normalised DFT;
- one step of the Cauchy-like form on a small Cauchy matrix.
"""
import math

import numpy as np
import pytest
import torch

import pins
import workloads as W
from oracle import rplu as O

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _within(samples, expected, tag):
    s = np.asarray(samples, dtype=np.float64)
    se = s.std(ddof=1) / math.sqrt(len(s))
    assert abs(s.mean() - expected) <= 4 * se + 1e-12 * abs(expected), \
        f"{tag}: mean {s.mean():.6g} vs exact {expected:.6g} (se {se:.3g})"


@pytest.mark.parametrize("seed", [21, 23])
def test_expected_error_4x4_batched(rplu_lib, seed):
    A = W.random_dense(4, 4, seed=seed)
    E = pins._enumerate(A, 3)
    N = 20000
    At = torch.from_numpy(A).to(DEV)
    for k in (1, 2, 3):
        mats = [At.clone() for _ in range(N)]
        res = rplu_lib.rplu_batched(mats, k=k, seed=5, streams=list(range(N)), store_L=False,
                                    store_U=False)
        assert all(r.rank == k for r in res)
        _within([r.res_fro2 for r in res], E[k], f"seed {seed}, k = {k}")


def test_expected_error_4x4_complex_dense(rplu_lib):
    A = W.random_dense(4, 4, seed=22, complex_=True)
    E = pins._enumerate(A, 2)
    At = torch.from_numpy(A).to(DEV)
    N = 4000
    for k in (1, 2):
        out = []
        for s in range(N):
            r = rplu_lib.rplu_dense(At.clone(), k=k, seed=9, stream=s,
                                    flags=rplu_lib.RPLU_FLAG_NO_GRAPH)
            out.append(r.res_fro2)
        _within(out, E[k], f"complex, k = {k}")


def test_unitary_dft_one_step(rplu_lib):
    n = 6
    F = np.exp(-2j * np.pi * np.outer(np.arange(n), np.arange(n)) / n) / math.sqrt(n)
    Ft = torch.from_numpy(F).to(DEV)
    N = 4000
    out = []
    for s in range(N):
        r = rplu_lib.rplu_dense(Ft.clone(), k=1, seed=3, stream=s,
                                flags=rplu_lib.RPLU_FLAG_NO_GRAPH)
        out.append(r.res_fro2)
    _within(out, 2.0 * (n - 1), "normalised DFT")


def test_cauchy_one_step(rplu_lib):
    x, y, G, B = W.cauchy_like_random(6, 5, 1, seed=4)
    A = O.cauchy_entries(x, y, G, B)
    E = pins._enumerate(A, 1)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)   # noqa: E731
    xd, yd, G0, B0 = t(x), t(y), t(G), t(B)
    N = 3000
    out = []
    for s in range(N):
        r = rplu_lib.rplu_cauchy(xd, yd, G0.clone(), B0.clone(), k=1, seed=2, stream=s,
                                 flags=rplu_lib.RPLU_FLAG_NO_GRAPH)
        out.append(r.res_fro2)
    _within(out, E[1], "Cauchy, k = 1")
