"""Batched dense RPLU (one persistent launch) on the GPU.

Every instance of a batch must give bitwise the results of rplu_dense run on
that instance alone (pivots, L, U, final Schur complement, totals), under
every launch configuration: the batched kernel reduces each row in the
single-instance order, and the schedule knobs (rows per pass, workgroups per
CU, queue order) do not touch the arithmetic. rplu_dense itself is checked
against the FP64 oracle in test_dense_gpu.py; here two batched instances are
also compared with the oracle directly.
"""
import math

import numpy as np
import pytest
import torch

import parity
import workloads as W
from oracle import rplu as O

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _instances(dtype, seed=11):
    """Shapes that cover tiny, ragged (m % 4 != 0), one- to eight-wave rows,
    multi-pass rows, unaligned rows (lda * size % 16 != 0) and misaligned
    starts, plus rank-deficient inputs (exhausted before k). The block pass
    (rows the pivot row's LDS copy holds: 4..1024 FP32 columns, 2..512 FP64;
    single-element packs for rows not 16-byte aligned, 1..1024 FP32 and
    1..512 FP64, up to four virtual waves of one column per lane, then all
    eight of one or two) is taken at and just past each of its limits:
    m = 2, 3, 4, 256, 512, 768, 769, 1024, 1025 and, unaligned, 256, 257,
    511, 512, 513, 1023, 1024 and 1025."""
    rng = np.random.default_rng(seed)
    shapes = [(1, 1), (1, 7), (7, 1), (3, 5), (64, 64), (100, 37), (37, 100), (130, 257),
              (257, 130), (513, 20), (20, 513), (997, 1000), (64, 1024), (1024, 64), (40, 3001),
              (33, 2100), (200, 555), (9, 4), (6, 2), (11, 3), (25, 256), (30, 512),
              (12, 768), (12, 769), (40, 1025), (15, 511), (15, 1023)]
    mats, meta = [], []
    for q, (n, m) in enumerate(shapes):
        A = torch.from_numpy(rng.standard_normal((n, m))).to(dtype)
        mats.append(A.to(DEV))
        meta.append(("plain", n, m))
    # unaligned row pitch: lda = m + 1
    for (n, m) in [(50, 71), (129, 64), (30, 256), (30, 257), (30, 512), (12, 1024)]:
        buf = torch.zeros((n, m + 1), dtype=dtype)
        buf[:, :m] = torch.from_numpy(rng.standard_normal((n, m))).to(dtype)
        mats.append(buf.to(DEV)[:, :m])
        meta.append(("lda+1", n, m))
    # misaligned start (4 bytes in)
    n, m = 60, 96
    flat = torch.zeros(n * m + 4, dtype=dtype)
    flat[1:1 + n * m] = torch.from_numpy(rng.standard_normal(n * m)).to(dtype)
    mats.append(flat.to(DEV)[1:1 + n * m].view(n, m))
    meta.append(("offset", n, m))
    # rank 3: EXHAUSTED after 3 steps
    for (n, m) in [(80, 90), (5, 300)]:
        A = rng.standard_normal((n, 3)) @ rng.standard_normal((3, m))
        mats.append(torch.from_numpy(A).to(dtype).to(DEV))
        meta.append(("rank3", n, m))
    return mats, meta


def _clone(t):
    """A copy with the same row pitch and the same address offset mod 16."""
    n, m = t.shape
    lda = t.stride(0)
    off = (t.data_ptr() % 16) // t.element_size()
    buf = torch.zeros(n * lda + off + 16, dtype=t.dtype, device=t.device)
    v = buf[off:off + (n - 1) * lda + m].as_strided((n, m), (lda, 1))
    v.copy_(t)
    assert v.data_ptr() % 16 == t.data_ptr() % 16
    return v


def _equal(a, b):
    return a is None and b is None or (a is not None and b is not None and torch.equal(a, b))


def _compare(rplu, mats, k, tol, seeds, cfg):
    alone_in = [_clone(A) for A in mats]
    batch_in = [_clone(A) for A in mats]
    streams = [1000 + b for b in range(len(mats))]
    res_b = rplu.rplu_batched(batch_in, k=k, tol=tol, seed=seeds, streams=streams, cfg=cfg)
    for b, A in enumerate(alone_in):
        ks = k[b] if isinstance(k, list) else k
        ts = tol[b] if isinstance(tol, list) else tol
        r1 = rplu.rplu_dense(A, k=ks, tol=ts, seed=seeds[b], stream=streams[b])
        r2 = res_b[b]
        tag = f"job {b} shape {tuple(A.shape)} cfg {cfg}"
        assert r2.status == 0, tag
        assert (r1.rank, r1.stop) == (r2.rank, r2.stop), tag
        assert r1.a_fro2 == r2.a_fro2 and r1.res_fro2 == r2.res_fro2, tag
        assert torch.equal(r1.piv, r2.piv), tag
        assert _equal(r1.U, r2.U), tag
        assert _equal(r1.L, r2.L), tag
        assert torch.equal(A, batch_in[b]), tag


CFGS = [None,
        {"rows_per_pass": 1, "wg_per_cu": 1, "order": 3},
        {"rows_per_pass": 2, "wg_per_cu": 3, "order": 1},
        {"rows_per_pass": 4, "wg_per_cu": 2, "order": 2},
        {"rows_per_pass": 8, "wg_per_cu": 1, "order": 1}]


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("cfg", CFGS, ids=["tuned", "r1w1given", "r2w3area", "r4w2cube", "r8w1area"])
def test_batched_bitwise_equals_single(rplu_lib, dtype, cfg):
    mats, meta = _instances(dtype)
    count = len(mats)
    seeds = [7 + b for b in range(count)]
    # mixed stop rules: fixed rank, tolerance, full rank
    k = [min(40, min(A.shape)) if b % 3 == 0 else 0 for b, A in enumerate(mats)]
    tol = [1e-3 if b % 3 == 1 else 0.0 for b in range(count)]
    _compare(rplu_lib, mats, k, tol, seeds, cfg)


def test_batched_without_factors(rplu_lib):
    """L and U not stored (U rows in per-workgroup scratch): same pivots and
    Schur complements as rplu_dense without factors."""
    mats, _ = _instances(torch.float32, seed=5)
    a1 = [_clone(A) for A in mats]
    a2 = [_clone(A) for A in mats]
    rb = rplu_lib.rplu_batched(a2, k=25, seed=3, store_L=False, store_U=False)
    for b, A in enumerate(a1):
        r1 = rplu_lib.rplu_dense(A, k=25, seed=3, stream=b, store_L=False, store_U=False)
        assert torch.equal(r1.piv, rb[b].piv) and torch.equal(A, a2[b])
        assert rb[b].L is None and rb[b].U is None


def test_batched_matches_oracle(rplu_lib):
    """Two FP64 instances of the batch against the oracle directly."""
    hosts = [W.random_dense(70, 45, seed=31), W.random_dense(33, 120, seed=32)]
    mats = [torch.from_numpy(h).to(DEV) for h in hosts]
    res = rplu_lib.rplu_batched(mats, k=[30, 20], seed=[5, 6], streams=[2, 3])
    for b, h in enumerate(hosts):
        orc = O.rplu_dense(h, k=[30, 20][b], seed=[5, 6][b], stream=[2, 3][b])
        assert res[b].rank == orc.rank
        assert np.array_equal(res[b].piv.cpu().numpy(), orc.piv)
        fa = math.sqrt(orc.a_fro2)
        a_t = np.array([orc.U[t, orc.piv[t, 1]] for t in range(orc.rank)])
        assert parity.fro((res[b].L.cpu().numpy() - orc.L) * a_t) <= 1e-10 * fa
        assert parity.rel(res[b].U.cpu().numpy(), orc.U) <= 1e-10
        assert parity.rel(mats[b].cpu().numpy(), orc.S, scale=fa) <= 1e-10


def test_batched_errors(rplu_lib):
    rplu = rplu_lib
    good = [torch.randn(30, 40, dtype=torch.float64, device=DEV) for _ in range(3)]
    bad = good[1].clone()
    bad[4, 5] = float("nan")
    mats = [good[0].clone(), bad, good[2].clone()]
    res = rplu.rplu_batched(mats, k=10, seed=1, raise_on_error=False)
    assert res[1].status == -4                      # RPLU_E_NONFINITE
    assert res[0].status == 0 and res[2].status == 0 and res[0].rank == 10
    with pytest.raises(rplu.RPLUError):
        rplu.rplu_batched([good[0].clone(), bad.clone()], k=10)
    # mixed dtypes, too large, unknown configuration
    with pytest.raises(rplu.RPLUError):
        rplu.rplu_batched([good[0].clone(), good[1].float()], k=4)
    with pytest.raises(rplu.RPLUError):
        rplu.rplu_batched([torch.zeros(8193, 4, device=DEV)], k=2)
    with pytest.raises(rplu.RPLUError):
        rplu.rplu_batched([good[0].clone()], k=2, cfg={"rows_per_pass": 3})
    assert rplu.rplu_batched([], k=2) == []


def test_batched_tall_instances(rplu_lib):
    """Row masses of up to 8192 rows in LDS (16 chunks, one CDF group)."""
    rplu = rplu_lib
    cases = [(4100, 50, torch.float32), (8192, 17, torch.float32), (6000, 40, torch.float64)]
    for n, m, dt in cases:
        A = torch.randn(n, m, dtype=dt, device=DEV)
        a1, a2 = A.clone(), A.clone()
        try:
            rb = rplu.rplu_batched([a2], k=12, seed=4, streams=[9])[0]
        except rplu.RPLUError as e:
            # a device whose workgroups get less LDS than n * (8 + size) bytes
            assert e.status == -6, (n, m, dt)
            continue
        r1 = rplu.rplu_dense(a1, k=12, seed=4, stream=9)
        assert torch.equal(r1.piv, rb.piv) and torch.equal(a1, a2) and torch.equal(r1.L, rb.L)


def test_batched_tuner_keeps_inputs(rplu_lib):
    mats, _ = _instances(torch.float32, seed=9)
    before = [A.clone() for A in mats]
    cfg, ms = rplu_lib.rplu_batched_tune(mats, k=0, tol=1e-6, seed=0)
    assert cfg["rows_per_pass"] in (1, 2, 4, 8) and 1 <= cfg["wg_per_cu"] <= 8 and ms > 0
    for a, b in zip(mats, before):
        assert torch.equal(a, b)


@pytest.mark.slow
def test_batched_full_size_sampled(rplu_lib):
    """4096 FP32 instances, n, m ~ U{64..1024}, sigma_i = r^i, tol 1e-6, in
    one tuned launch; a size-stratified sample of 24 instances is re-run
    alone (bitwise equal), and every instance's stop is checked."""
    specs = W.batched_instance_specs()
    print(f"generating {len(specs)} instances", flush=True)
    mats = W.batched_instances_device(specs)
    order = sorted(range(len(specs)), key=lambda b: specs[b].n * specs[b].m)
    sample = [order[q] for q in np.linspace(0, len(order) - 1, 24).astype(int)]
    keep = {b: mats[b].clone() for b in sample}
    print("running the batch", flush=True)
    res = rplu_lib.rplu_batched(mats, k=0, tol=1e-6, seed=0, streams=list(range(len(specs))),
                                store_L=False, store_U=True)
    for b, r in enumerate(res):
        assert r.status == 0
        assert r.stop in (rplu_lib.RPLU_STOP_TOL, rplu_lib.RPLU_STOP_TOL_UNREACHED,
                          rplu_lib.RPLU_STOP_EXHAUSTED)
        if r.stop == rplu_lib.RPLU_STOP_TOL:
            assert r.res_fro2 <= 1e-12 * r.a_fro2
    for b in sample:
        A = keep[b]
        r1 = rplu_lib.rplu_dense(A, k=0, tol=1e-6, seed=0, stream=b, store_L=False)
        assert torch.equal(r1.piv, res[b].piv) and torch.equal(A, mats[b]), b
        assert torch.equal(r1.U, res[b].U) and r1.res_fro2 == res[b].res_fro2, b


def test_batched_stall_rule(rplu_lib):
    """The stall rule in the batched kernel stops where rplu_dense does. On
    an identity of size N every step removes one unit of mass, so an
    improvement by 1/64 of the best total takes N/64 steps: N = 4096 stalls
    at t = 64 (4032 is not below 63/64 of 4096), N = 4095 improves just in
    time in every window and reaches the rank limit."""
    F = rplu_lib.RPLU_FLAG_STALL_STOP
    mats = [torch.eye(4096, device=DEV), torch.eye(4095, device=DEV)]
    try:
        res = rplu_lib.rplu_batched([m.clone() for m in mats], k=150, seed=1, flags=F)
    except rplu_lib.RPLUError as e:
        assert e.status == -6          # workgroups get less LDS than 4096 rows need
        pytest.skip("4096 rows exceed this device's LDS per workgroup")
    assert [(r.stop, r.rank) for r in res] == [(rplu_lib.RPLU_STOP_STALL, 64),
                                                (rplu_lib.RPLU_STOP_RANK, 150)]
    for b, m in enumerate(mats):
        a = rplu_lib.rplu_dense(m.clone(), k=150, seed=1, stream=b, flags=F)
        assert (a.stop, a.rank) == (res[b].stop, res[b].rank)
        assert torch.equal(a.piv, res[b].piv)
