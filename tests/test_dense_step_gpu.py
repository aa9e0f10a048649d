"""Small dense runs in one launch per step (k_dense_step, n and m up to
DENSE_STEP_MAX): every workgroup makes both draws of the step itself and
sweeps its own rows. Against the two-kernel form on the same input (forced
with RPLU_FLAG_SPLIT_SAMPLER, whose draws are bit for bit those of the fused
draw kernel): the same rank, stop and totals, and the same bits in the
pivots, L, U, the trace, the per-step row masses and the final Schur
complement left in A, in all four dtypes, on shapes with ragged row ends
and row blocks, unaligned rows, the stop rules and pivot choices of the
dense path, graph and plain launches. Parity with the oracle on these sizes
is the other dense tests' (they take this form by default)."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TORCH = {"r64": torch.float64, "c128": torch.complex128, "r32": torch.float32,
         "c64": torch.complex64}


def _bits(x):
    x = x.contiguous()
    if x.is_complex():
        x = torch.view_as_real(x).contiguous()
    return x.view(torch.int32 if x.element_size() == 4 else torch.int64)


def _mat(n, m, dt, seed, lda=None, spectrum=None):
    if spectrum is not None:
        A = W.dense_with_spectrum(n, m, spectrum, seed=seed)
    else:
        A = W.random_dense(n, m, seed=seed, complex_=dt in ("c128", "c64"))
    t = torch.from_numpy(np.ascontiguousarray(A)).to(TORCH[dt])
    if lda is None:
        return t.to(DEV)
    buf = torch.zeros((n, lda), dtype=TORCH[dt])
    buf[:, :m] = t
    return buf.to(DEV)[:, :m]


def _run(rplu, A0, flags, **kw):
    if A0.is_contiguous():
        A = A0.clone()
    else:                                   # keep the row pitch
        buf = torch.zeros((A0.shape[0], A0.stride(0)), dtype=A0.dtype, device=DEV)
        buf[:, :A0.shape[1]] = A0
        A = buf[:, :A0.shape[1]]
    r = rplu.rplu_dense(A, flags=flags, want_trace=True, want_rowmass=True, **kw)
    torch.cuda.synchronize()
    return r, A


def _compare(rplu, A0, tag, flags=0, **kw):
    outs = []
    for extra in (0, rplu.RPLU_FLAG_NO_GRAPH, rplu.RPLU_FLAG_SPLIT_SAMPLER,
                  rplu.RPLU_FLAG_SPLIT_SAMPLER | rplu.RPLU_FLAG_NO_GRAPH):
        outs.append(_run(rplu, A0, flags | extra, **kw))
    r0, A_0 = outs[0]
    bad = []
    for q, (r, A) in enumerate(outs[1:], 1):
        if (r.rank, r.stop, r.a_fro2, r.res_fro2) != (r0.rank, r0.stop, r0.a_fro2, r0.res_fro2):
            bad.append((q, "totals", (r0.rank, r0.stop, r0.a_fro2, r0.res_fro2),
                        (r.rank, r.stop, r.a_fro2, r.res_fro2)))
        for name in ("piv", "L", "U", "trace", "rowmass"):
            a, b = getattr(r0, name), getattr(r, name)
            if a is None or b is None:
                if (a is None) != (b is None):
                    bad.append((q, name, "missing"))
                continue
            if a.shape != b.shape or not torch.equal(_bits(a), _bits(b)):
                first = None
                if a.shape == b.shape:
                    d = (_bits(a) != _bits(b)).nonzero()
                    first = d[0].tolist() if len(d) else None
                bad.append((q, name, "first differing index", first))
        if not torch.equal(_bits(A_0), _bits(A)):
            bad.append((q, "final A"))
    # runs: 0 one launch + graph, 1 one launch plain, 2 two kernels + graph, 3 plain
    assert not bad, (tag, bad)
    print(f"{tag}: rank {r0.rank} stop {r0.stop}", flush=True)
    return r0


@pytest.mark.parametrize("dt", ["r64", "c128", "r32", "c64"])
@pytest.mark.parametrize("n,m,k", [(512, 512, 50), (301, 257, 60), (1000, 90, 40),
                                   (130, 1000, 50), (1024, 1023, 80)])
def test_step_matches_two_kernels(rplu_lib, dt, n, m, k):
    A = _mat(n, m, dt, seed=n + 7 * m)
    _compare(rplu_lib, A, f"{dt} {n}x{m}", k=k, seed=5, stream=n)


def test_step_unaligned_and_no_factors(rplu_lib):
    """Rows of odd pitch (element accesses), and runs that store neither L
    nor U (the pivot row in the workspace)."""
    A = _mat(333, 301, "r32", seed=3, lda=305)
    _compare(rplu_lib, A, "unaligned", k=45, seed=2)
    B = _mat(400, 380, "r64", seed=4)
    _compare(rplu_lib, B, "no L, U", k=30, seed=1, store_L=False, store_U=False)


@pytest.mark.parametrize("case", ["tol", "stall", "c2plu", "maxmass", "forced", "rank_r"])
def test_step_stop_rules_and_choices(rplu_lib, case):
    sig = 0.8 ** np.arange(300)
    A = _mat(320, 300, "r64", seed=9, spectrum=sig)
    kw = dict(seed=3)
    flags = 0
    if case == "tol":
        kw.update(k=0, tol=1e-6)
    elif case == "stall":
        A = A.to(torch.float32)
        kw.update(k=0, tol=1e-9)
        flags = rplu_lib.RPLU_FLAG_STALL_STOP
    elif case == "c2plu":
        kw.update(k=40)
        flags = rplu_lib.RPLU_FLAG_C2PLU
    elif case == "maxmass":
        kw.update(k=0, tol=1e-5)
        flags = rplu_lib.RPLU_FLAG_MAXMASS_STOP
    elif case == "forced":
        rng = np.random.default_rng(6)
        f = np.stack([rng.permutation(320)[:30], rng.permutation(300)[:30]], 1).astype(np.int32)
        kw.update(k=30, forced=torch.from_numpy(f))
    elif case == "rank_r":
        A = torch.from_numpy(W.rank_r_dense(200, 180, 11, seed=6)).to(DEV)
        kw.update(k=0, tol=1e-12)
    r = _compare(rplu_lib, A, case, flags=flags, **kw)
    if case == "rank_r":
        assert r.rank == 11
    if case == "forced":
        assert r.rank == 30


def test_step_reports_errors_like_two_kernels(rplu_lib):
    """A forced row out of range, and a zero pivot: both forms report the
    same status."""
    A = _mat(64, 64, "r64", seed=1)
    f = torch.tensor([[3, 4], [70, 2]], dtype=torch.int32)
    for flags in (0, rplu_lib.RPLU_FLAG_SPLIT_SAMPLER):
        with pytest.raises(rplu_lib.RPLUError) as e:
            rplu_lib.rplu_dense(A.clone(), k=2, forced=f, flags=flags)
        assert e.value.status == -1
    Z = torch.zeros((64, 64), dtype=torch.float64, device=DEV)
    Z[5, 7] = 1.0
    Z[9, 9] = 1.0                                # mass left after the first pivot
    f = torch.tensor([[5, 7], [6, 8]], dtype=torch.int32)
    st = []
    for flags in (0, rplu_lib.RPLU_FLAG_SPLIT_SAMPLER):
        with pytest.raises(rplu_lib.RPLUError) as e:
            rplu_lib.rplu_dense(Z.clone(), k=2, forced=f, flags=flags)
        st.append(e.value.status)
    assert st[0] == st[1]
