"""Queueing logic of the continuous-batching server, on the host only.

RPLU_SERVER_SIMULATE runs the real admission, FIFO, slot pool, step-tick
and statistics code with a stand-in executor (no device: a worker job "runs"
for footprint / 1e10 s, a tick advances every resident small job by
tick_steps steps for its share of that), so these tests need no GPU. Inputs
are never read in this mode, so host tensors stand in for device buffers.
"""
import time

import pytest
import torch

import paper_2601_22344_amd as rplu

MB = 1 << 20


def _dense(n, m=None, dtype=torch.float32):
    return torch.zeros((n, m or n), dtype=dtype)


def _rup(v):
    return (v + 255) // 256 * 256


def _footprint(n, m, k=0, es=4):
    """Work block (the input copy) plus the server-owned outputs (piv, L, U of
    kmax steps); the dense workspace of a worker job adds a little more."""
    kmax = min(n, m) if k <= 0 else min(k, n, m)
    return _rup(n * m * es + 16) + _rup(kmax * 8) + _rup(n * kmax * es) + _rup(kmax * m * es)


def _wait_all(S, tickets, timeout=30.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t not in out:
                r = S.poll(t)
                if r is not None:
                    out[t] = r
        assert time.time() - t0 < timeout, "server did not finish"
        time.sleep(0.001)
    return out


def test_all_jobs_complete_and_stats():
    S = rplu.Server(budget_bytes=64 * MB, workers=2, simulate=True)
    ts = [S.submit_dense(_dense(256 + 16 * q)) for q in range(20)]
    res = _wait_all(S, ts)
    assert all(res[t].status == 0 and res[t].rank == 256 + 16 * q for q, t in enumerate(ts))
    st = S.stats()
    assert st["submitted"] == 20 and st["completed"] == 20 and st["rejected"] == 0
    assert st["queued"] == 0 and st["active"] == 0 and st["hbm_in_use"] == 0
    assert 0.0 <= st["p50_ms"] <= st["p99_ms"]
    assert st["p99_cauchy_ms"] == 0.0                 # no Cauchy jobs
    # every job goes through the step ticks: 256 steps / 32 per tick at least
    assert st["tick_jobs"] == 20 and st["ticks"] >= 8
    S.close()


def test_poll_once_then_forgotten():
    S = rplu.Server(budget_bytes=8 * MB, simulate=True)
    t = S.submit_dense(_dense(64))
    _wait_all(S, [t])
    with pytest.raises(rplu.RPLUError):
        S.poll(t)
    with pytest.raises(rplu.RPLUError):
        S.poll(12345)
    S.close()


def test_admission_by_footprint_is_fifo_and_bounded():
    """Jobs of about 42 MB (input copy, outputs and workspace) in a 100 MB
    pool: at most two resident at once and the pool never over-commits. A
    finished job keeps its output block until it is polled, so at every
    observation the bytes in use are at most (running jobs) x footprint +
    (finished, not yet polled) x outputs."""
    n = 3240                                    # 3240^2 * 4 B ~ 40 MB
    fp = _footprint(n, n, k=64) + 2 * MB        # + the dense workspace (masses, totals)
    out_fp = _footprint(n, n, k=64) - _rup(n * n * 4 + 16)
    S = rplu.Server(budget_bytes=100 * MB, workers=3, batch_max_dim=1024, simulate=True)
    ts = [S.submit_dense(_dense(n), k=64) for _ in range(8)]
    peak_active = 0
    done = {}
    t0 = time.time()
    while len(done) < len(ts):
        st = S.stats()
        peak_active = max(peak_active, st["active"])
        assert st["hbm_in_use"] <= 100 * MB
        held = st["completed"] - len(done)
        assert st["hbm_in_use"] <= st["active"] * fp + held * out_fp, (st, held)
        for t in ts:
            if t not in done:
                r = S.poll(t)
                if r is not None:
                    done[t] = time.time()
        assert time.time() - t0 < 30
    assert peak_active <= 2
    st = S.stats()
    assert st["ticks"] == 0                     # all above batch_max_dim: run alone
    assert st["hbm_peak"] <= 100 * MB and st["hbm_peak"] >= fp - 2 * MB
    S.close()


def test_footprint_counts_outputs_and_workspace():
    """A dense job whose input copy alone fits the pool but whose outputs do
    not is refused; the outputs are part of the footprint."""
    n = 1024                                    # input copy 4 MB, L and U 8 MB at k = n
    S = rplu.Server(budget_bytes=8 * MB, simulate=True)
    with pytest.raises(rplu.RPLUError) as e:
        S.submit_dense(_dense(n), k=0)
    assert e.value.status == -1
    t = S.submit_dense(_dense(n), k=64)         # 4 MB + 0.5 MB of outputs
    _wait_all(S, [t])
    assert S.stats()["hbm_in_use"] == 0         # output block released by poll
    S.close()


def test_max_slots_limits_residency():
    S = rplu.Server(budget_bytes=1 << 30, max_slots=3, workers=4, batch_max_dim=64, simulate=True)
    ts = [S.submit_dense(_dense(2000)) for _ in range(10)]
    t0 = time.time()
    pending = set(ts)
    while pending:
        assert S.stats()["active"] <= 3
        for t in list(pending):
            if S.poll(t) is not None:
                pending.discard(t)
        assert time.time() - t0 < 30
    S.close()


def test_queue_capacity_rejects_with_busy():
    # one huge job occupies the pool; the queue then fills
    S = rplu.Server(budget_bytes=1100 * MB, queue_capacity=2, workers=1, simulate=True)
    A = _dense(16000)                            # 1 GB: ~0.1 s of simulated work
    big = S.submit_dense(A, k=1)
    q1 = S.submit_dense(A, k=1)
    q2 = S.submit_dense(A, k=1)
    with pytest.raises(rplu.RPLUError) as e:
        S.submit_dense(A, k=1)
    assert e.value.status == -5                  # RPLU_E_BUSY
    assert S.stats()["rejected"] == 1
    _wait_all(S, [big, q1, q2])
    S.close()


def test_job_larger_than_pool_is_refused():
    S = rplu.Server(budget_bytes=1 * MB, simulate=True)
    with pytest.raises(rplu.RPLUError) as e:
        S.submit_dense(_dense(1024))             # 4 MB
    assert e.value.status == -1
    S.close()


def test_small_jobs_join_the_ticks_while_a_large_job_runs():
    """Step-level batching: small jobs do not wait for a large job on the only
    worker; they are admitted into the resident set and finish in ticks while
    it still runs, and jobs arriving later join at a tick boundary."""
    S = rplu.Server(budget_bytes=8 << 30, workers=1, batch_max_dim=512, tick_steps=16,
                    simulate=True)
    # runs alone on the worker for ~0.4 s of simulated work (the zero pages
    # of the 4 GB host tensor are never touched in simulation)
    big = S.submit_dense(_dense(16000, 64000), k=1)
    time.sleep(0.01)
    first = [S.submit_dense(_dense(128 + q), k=64) for q in range(8)]
    time.sleep(0.002)
    later = [S.submit_dense(_dense(200 + q), k=64) for q in range(8)]
    res = _wait_all(S, first + later)
    assert all(r.rank == 64 for r in res.values())
    assert S.poll(big) is None                   # the large job is still running
    st = S.stats()
    assert st["tick_jobs"] == 16 and st["ticks"] >= 4     # 64 steps / 16 per tick
    _wait_all(S, [big])
    S.close()


def test_destroy_drains():
    """close() returns only after every submitted job ran: six 36 MB jobs on
    two workers need at least 3 x 3.6 ms of simulated work."""
    S = rplu.Server(budget_bytes=256 * MB, workers=2, simulate=True)
    A = _dense(3000)
    t0 = time.time()
    for _ in range(6):
        S.submit_dense(A, k=1)
    S.close()
    assert time.time() - t0 >= 0.9 * 3 * _footprint(3000, 3000, k=1) / 1e10


def test_cauchy_jobs_counted_per_class():
    S = rplu.Server(budget_bytes=64 * MB, workers=2, simulate=True)
    x = torch.zeros(5000, dtype=torch.complex128)
    y = torch.zeros(4000, dtype=torch.complex128)
    G = torch.zeros((5000, 2), dtype=torch.complex128)
    B = torch.zeros((2, 4000), dtype=torch.complex128)
    ts = [S.submit_cauchy(x, y, G, B, k=5) for _ in range(3)] + [S.submit_dense(_dense(300))]
    _wait_all(S, ts)
    st = S.stats()
    assert st["p50_cauchy_ms"] > 0.0 and st["p50_dense_ms"] > 0.0 and st["completed"] == 4
    S.close()


def test_c2plu_flag_is_refused():
    """C2PLU is a single-run option (rplu_dense / rplu_cauchy); a served job
    carrying RPLU_FLAG_C2PLU is refused at submission with RPLU_E_ARG."""
    S = rplu.Server(budget_bytes=64 * MB, simulate=True)
    with pytest.raises(rplu.RPLUError) as e:
        S.submit_dense(_dense(64), k=4, flags=rplu.RPLU_FLAG_C2PLU)
    assert e.value.status == -1
    t = S.submit_dense(_dense(64), k=4)            # the server keeps working
    assert t in _wait_all(S, [t])
    S.close()
