"""Dense path: the fused one-workgroup pivot draw (the default when
n, m <= 12288) against the wide form (RPLU_FLAG_SPLIT_SAMPLER: a row-draw
kernel and a pivot-row kernel, each finishing in its last workgroup, the
form used above 12288): the same pivots, trace words, masses, factors and
final Schur complement, bit for bit, for every element type, for shapes with
ragged chunks, groups and wide workgroups, at the largest fused sizes, with
forced pivots, under the tolerance and stall stops, and on every error path.
(Both forms are checked against the oracle by the other parity tests; this
file pins that they are one computation.)
"""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TORCH = {"r64": torch.float64, "c128": torch.complex128, "r32": torch.float32, "c64": torch.complex64}


def _dense_input(n, m, dt, seed):
    A = W.random_dense(n, m, seed=seed, complex_=dt in ("c128", "c64"))
    return torch.from_numpy(A).to(TORCH[dt]).to(DEV)


def _dense_run(rplu, A, flags, **kw):
    Ad = A.clone()
    r = rplu.rplu_dense(Ad, flags=flags, want_trace=True, want_rowmass=True, **kw)
    torch.cuda.synchronize()
    out = dict(rank=r.rank, stop=r.stop, a_fro2=r.a_fro2, res_fro2=r.res_fro2, piv=r.piv, L=r.L,
               U=r.U, trace=r.trace, rowmass=r.rowmass, S=Ad)
    if kw.get("want_colmass"):
        out["colmass"] = r.colmass
    return out


def _same(a, b, tag):
    assert a.keys() == b.keys()
    for key in a:
        x, y = a[key], b[key]
        if torch.is_tensor(x):
            assert x.shape == y.shape, f"{tag}: {key} shape"
            # bit patterns, so that -0.0 / +0.0 and NaN payloads count too
            xv = torch.view_as_real(x) if x.is_complex() else x
            yv = torch.view_as_real(y) if y.is_complex() else y
            assert torch.equal(xv.contiguous().reshape(-1).view(torch.uint8),
                               yv.contiguous().reshape(-1).view(torch.uint8)), \
                f"{tag}: {key} differs"
        else:
            assert x == y, f"{tag}: {key} {x} != {y}"


def _dense_both(rplu, A, extra=0, **kw):
    f = _dense_run(rplu, A, extra, **kw)
    s = _dense_run(rplu, A, extra | rplu.RPLU_FLAG_SPLIT_SAMPLER, **kw)
    return f, s


@pytest.mark.parametrize("dt", ["r32", "r64", "c64", "c128"])
@pytest.mark.parametrize("n,m", [(1, 1), (1, 700), (700, 1), (513, 511), (1025, 4097), (2048, 1024),
                                 (12288, 33)])
def test_dense_forms_equal(rplu_lib, dt, n, m):
    A = _dense_input(n, m, dt, seed=n + 3 * m)
    k = min(n, m, 60)
    f, s = _dense_both(rplu_lib, A, k=k, seed=4, stream=2)
    assert f["rank"] == k
    _same(f, s, f"{dt} {n}x{m}")


@pytest.mark.parametrize("n,m", [(12288, 40), (40, 12288)])
def test_dense_forms_equal_at_fused_limit(rplu_lib, n, m):
    A = _dense_input(n, m, "r32", seed=5)
    f, s = _dense_both(rplu_lib, A, k=25, seed=1)
    assert f["rank"] == 25
    _same(f, s, f"{n}x{m}")


def test_dense_forms_equal_options(rplu_lib):
    A = _dense_input(300, 2100, "r64", seed=8)
    f, s = _dense_both(rplu_lib, A, k=40, seed=3, want_colmass=True)
    _same(f, s, "colmass")
    f, s = _dense_both(rplu_lib, A, k=40, seed=3, extra=rplu_lib.RPLU_FLAG_NO_GRAPH)
    _same(f, s, "plain launches")
    rng = np.random.default_rng(0)
    forced = torch.tensor(np.stack([rng.permutation(300)[:40], rng.permutation(2100)[:40]], 1),
                          dtype=torch.int32)
    f, s = _dense_both(rplu_lib, A, k=40, forced=forced)
    _same(f, s, "forced")
    D = torch.from_numpy(W.dense_with_spectrum(300, 2100, 0.8 ** np.arange(300), seed=6)).to(DEV)
    f, s = _dense_both(rplu_lib, D, k=0, tol=1e-4, seed=6)
    assert f["stop"] == rplu_lib.RPLU_STOP_TOL and 20 < f["rank"] < 300
    _same(f, s, "tolerance")


def test_dense_forms_equal_stall(rplu_lib):
    # identity 4096: T_t = 4096 - t first falls below 63/64 of T_0 at t = 65,
    # so the run stalls at t = 64 whatever the draws
    D = torch.eye(4096, dtype=torch.float32, device=DEV)
    f, s = _dense_both(rplu_lib, D, extra=rplu_lib.RPLU_FLAG_STALL_STOP, k=0, tol=1e-6, seed=2)
    assert f["stop"] == rplu_lib.RPLU_STOP_STALL and f["rank"] == 64
    _same(f, s, "stall")


def test_dense_forms_same_errors(rplu_lib):
    Z = torch.zeros((5, 9), dtype=torch.float64, device=DEV)
    f, s = _dense_both(rplu_lib, Z, k=3)
    assert f["rank"] == 0 and f["stop"] == rplu_lib.RPLU_STOP_EXHAUSTED
    _same(f, s, "zero matrix")
    N = _dense_input(6, 4, "r64", seed=2)
    N[3, 1] = float("nan")
    F = _dense_input(6, 6, "r64", seed=2)
    F[2, 3] = 0.0
    for A, kw, status in ((N, dict(k=2), -4), (F, dict(k=1, forced=torch.tensor([2, 3])), -7),
                          (F, dict(k=1, forced=torch.tensor([9, 0])), -1),
                          (F, dict(k=1, forced=torch.tensor([0, 6])), -1)):
        for flags in (0, rplu_lib.RPLU_FLAG_SPLIT_SAMPLER):
            with pytest.raises(rplu_lib.RPLUError) as e:
                rplu_lib.rplu_dense(A.clone(), flags=flags, **kw)
            assert e.value.status == status, (kw, flags)
