"""rplu_dense_noalloc (the allocation-free dense entry point) against
rplu_dense through the C ABI: same pivots, factors, Schur complement, trace
and info bit for bit (the same kernels on the fixed scratch array instead of
context workspace), on two calls in a row whose second input is smaller, and
the size limit rejected before anything runs."""
import ctypes as C

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _lib():
    from paper_2601_22344_amd import _binding as Bd
    return Bd


def _run(Bd, fn, A0, k, tol, seed, stream, flags, ctx=None):
    n, m = A0.shape
    A = A0.clone()
    kmax = min(n, m, k) if k > 0 else min(n, m)
    piv = torch.full((kmax, 2), -7, dtype=torch.int32, device=DEV)
    Lt = torch.full((kmax, n), 3.0, dtype=A.dtype, device=DEV)
    U = torch.full((kmax, m), 5.0, dtype=A.dtype, device=DEV)
    tr = torch.zeros((kmax, Bd.RPLU_TRACE_WORDS), dtype=torch.float64, device=DEV)
    rm = torch.zeros((kmax, n), dtype=torch.float64, device=DEV)
    opts = Bd._opts(k, tol, seed, stream, flags, None, tr, rm, None)
    info = Bd.rplu_info()
    dt = Bd._DTYPES[A.dtype]
    strm = Bd._cur_stream(A.device)
    if fn == "noalloc":
        st = Bd.lib.rplu_dense_noalloc(dt, n, m, Bd._ptr(A), A.stride(0), C.byref(opts),
                                       Bd._ptr(piv), Bd._ptr(Lt), n, Bd._ptr(U), m,
                                       C.byref(info), strm)
    else:
        st = Bd.lib.rplu_dense(ctx.handle, dt, n, m, Bd._ptr(A), A.stride(0), C.byref(opts),
                               Bd._ptr(piv), Bd._ptr(Lt), n, Bd._ptr(U), m, C.byref(info), strm)
    torch.cuda.synchronize()
    return st, info, A, piv, Lt, U, tr, rm


def _same(r1, r2):
    st1, i1, *t1 = r1
    st2, i2, *t2 = r2
    assert st1 == st2 == 0
    assert (i1.rank, i1.stop, i1.status) == (i2.rank, i2.stop, i2.status)
    assert i1.a_fro2 == i2.a_fro2 and i1.res_fro2 == i2.res_fro2
    for a, b in zip(t1, t2):
        assert torch.equal(a, b)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.complex128])
def test_noalloc_matches_rplu_dense_twice(dtype):
    Bd = _lib()
    ctx = Bd.Context(0)
    cases = [((700, 533), 40, 0.0, 11, 3, 0),
             ((129, 77), 0, 1e-3, 12, 4, Bd.RPLU_FLAG_STALL_STOP)]   # second: smaller
    for (n, m), k, tol, seed, stream, flags in cases:
        print(f"noalloc case dtype={dtype} n={n} m={m} k={k}", flush=True)
        A = W.random_dense(n, m, seed=n + m)
        if dtype.is_complex:
            A = A + 1j * W.random_dense(n, m, seed=n + m + 1)
        A0 = torch.from_numpy(np.ascontiguousarray(A)).to(DEV).to(dtype)
        r_ref = _run(Bd, "dense", A0, k, tol, seed, stream, flags | Bd.RPLU_FLAG_NO_GRAPH, ctx)
        r_na = _run(Bd, "noalloc", A0, k, tol, seed, stream, flags)
        _same(r_ref, r_na)
        assert r_na[1].rank > 0
    ctx.close()


def test_noalloc_wide_draws_and_limit():
    """Past the fused-draw limit (12289 rows: the wide draw kernels and their
    arrival counter in the scratch state), then a problem whose scratch is
    beyond the array: RPLU_E_ARG, its buffers untouched."""
    Bd = _lib()
    ctx = Bd.Context(0)
    A0 = torch.from_numpy(W.random_dense(12289, 24, seed=5)).to(DEV).to(torch.float32)
    _same(_run(Bd, "dense", A0, 10, 0.0, 2, 9, Bd.RPLU_FLAG_NO_GRAPH, ctx),
          _run(Bd, "noalloc", A0, 10, 0.0, 2, 9, 0))
    limit = 16 << 20
    n = 2_200_000                      # row masses alone: 17.6 MB > 16 MiB
    need = Bd.lib.rplu_dense_noalloc_bytes(Bd.RPLU_R32, n, 1, 0, 1)
    assert need > limit
    A = torch.ones((n, 1), dtype=torch.float32, device=DEV)
    piv = torch.full((1, 2), -7, dtype=torch.int32, device=DEV)
    opts = Bd._opts(1, 0.0, 0, 0, 0, None, None, None, None)
    info = Bd.rplu_info()
    st = Bd.lib.rplu_dense_noalloc(Bd.RPLU_R32, n, 1, Bd._ptr(A), 1, C.byref(opts), Bd._ptr(piv),
                                   None, n, None, 1, C.byref(info), Bd._cur_stream(A.device))
    torch.cuda.synchronize()
    assert st == Bd.RPLU_E_ARG
    assert "scratch" in Bd.lib.rplu_last_error().decode()
    assert torch.equal(piv.cpu(), torch.full((1, 2), -7, dtype=torch.int32))
    assert bool((A == 1).all())
    ctx.close()


def test_noalloc_binding_against_oracle():
    """The binding's wrapper (caller-owned outputs) on a FP64 input: the
    oracle's own draws at every step and its Schur complement within 1e-10."""
    import paper_2601_22344_amd as rplu
    from oracle import rplu as O
    A = W.random_dense(150, 90, seed=21)
    Ad = torch.from_numpy(A).to(DEV)
    k = 30
    piv = torch.empty((k, 2), dtype=torch.int32, device=DEV)
    L = torch.empty((k, 150), dtype=torch.float64, device=DEV)
    U = torch.empty((k, 90), dtype=torch.float64, device=DEV)
    r = rplu.rplu_dense_noalloc(Ad, piv, L, U, k=k, seed=8, stream=2)
    o = O.rplu_dense(A, k=k, seed=8, stream=2)
    assert np.array_equal(r.piv.cpu().numpy(), o.piv)
    assert np.linalg.norm(Ad.cpu().numpy() - o.S) <= 1e-10 * np.linalg.norm(A)
    assert np.linalg.norm(r.U.cpu().numpy() - o.U) <= 1e-10 * np.linalg.norm(o.U)
