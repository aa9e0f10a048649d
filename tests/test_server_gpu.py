"""Continuous-batching server on the GPU: every served result is the one the
job gets alone, and every served result is checked against the oracle.

A mix of small dense jobs (FP32 and FP64; they go through the step ticks,
pausing every 8 steps), larger dense jobs (workers) and Cauchy-like jobs is
submitted at once and in a trickle, under a slot pool that holds only a few
jobs. For every job:
  * alone vs mix: rank, stop, totals, pivots and factors equal, bit for bit,
    to rplu_dense / rplu_cauchy on the same inputs, seed, stream and flags;
  * oracle: the C++ oracle replays the served pivots. FP64 and complex128
    jobs (protocol P1): every pivot is the oracle's own draw (or within
    1e-12 T of the shared bin edge), U and the columns L(:,t) a_t within
    1e-10. FP32 jobs: L U within 1e-5 ||A||_F of the oracle's L U on the
    same pivots, over the steps taken while the residual is above 1e-5
    ||A||_F (before the single-precision rounding floor), and, for the
    tolerance jobs (stall rule, residual replacement, certification), a TOL
    stop with the certified FP64 ||A - L U|| within the tolerance, equal to
    rplu_verify on the returned factors.
The server leaves its inputs untouched.
"""
import math
import time

import numpy as np
import pytest
import torch

import parity
import workloads as W
from oracle import ref as R
from test_refresh_gpu import _compare_steps, _distinct_prefix

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
MB = 1 << 20
TOL = 1e-6


def _decaying(n, seed):
    sig = 0.9 ** np.arange(1, n + 1)
    sig[sig < 1e-16] = 0.0
    return W.dense_with_spectrum(n, n, sig, seed=seed)


def _mix(rplu, seed=3):
    rng = np.random.default_rng(seed)
    tolf = rplu.RPLU_FLAG_STALL_STOP | rplu.RPLU_FLAG_REFRESH | rplu.RPLU_FLAG_CERTIFY
    jobs = []
    for q in range(10):
        n, m = int(rng.integers(40, 700)), int(rng.integers(40, 700))
        dt = torch.float64 if q % 4 == 3 else torch.float32
        A = torch.from_numpy(rng.standard_normal((n, m))).to(dt).to(DEV)
        jobs.append(dict(kind="dense", A=A, k=0 if q % 2 else 30, tol=1e-2 if q % 2 else 0.0,
                         seed=q, stream=100 + q, flags=0))
    for q in range(2):                      # FP32 at tolerance 1e-6 through the ticks
        n = 1400 + 300 * q
        A = torch.from_numpy(_decaying(n, seed=60 + q)).float().to(DEV)
        jobs.append(dict(kind="dense", A=A, k=0, tol=TOL, seed=4, stream=150 + q, flags=tolf))
    for q in range(2):                      # larger: workers
        n = 2100 + 37 * q
        if q == 0:
            A = torch.from_numpy(W.random_dense(n, n - 50, seed=40 + q)).float().to(DEV)
            jobs.append(dict(kind="dense", A=A, k=40, tol=0.0, seed=7, stream=200 + q, flags=0))
        else:
            A = torch.from_numpy(_decaying(n, seed=70)).float().to(DEV)
            jobs.append(dict(kind="dense", A=A, k=0, tol=TOL, seed=7, stream=200 + q, flags=tolf))
    for q in range(2):
        x, y, G, B = W.cauchy_like_random(1500 + 300 * q, 1200, 1 + q, seed=50 + q)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)   # noqa: E731
        jobs.append(dict(kind="cauchy", x=t(x), y=t(y), G=t(G), B=t(B), k=25, tol=0.0, seed=9,
                         stream=300 + q, flags=0))
    return jobs


def _submit(S, j):
    if j["kind"] == "dense":
        return S.submit_dense(j["A"], k=j["k"], tol=j["tol"], seed=j["seed"], stream=j["stream"],
                              flags=j["flags"])
    return S.submit_cauchy(j["x"], j["y"], j["G"], j["B"], k=j["k"], tol=j["tol"], seed=j["seed"],
                           stream=j["stream"], flags=j["flags"])


def _alone(rplu, j):
    if j["kind"] == "dense":
        refresh = bool(j["flags"] & rplu.RPLU_FLAG_REFRESH)
        fl = j["flags"] & rplu.RPLU_FLAG_STALL_STOP
        return rplu.rplu_dense(j["A"].clone(), k=j["k"], tol=j["tol"], seed=j["seed"],
                               stream=j["stream"], flags=fl, A_orig=j["A"] if refresh else None)
    return rplu.rplu_cauchy(j["x"], j["y"], j["G"].clone(), j["B"].clone(), k=j["k"],
                            tol=j["tol"], seed=j["seed"], stream=j["stream"])


def _run(rplu, jobs, budget, workers, trickle):
    before = [{k: v.clone() for k, v in j.items() if torch.is_tensor(v)} for j in jobs]
    S = rplu.Server(budget_bytes=budget, workers=workers, tick_steps=8)
    tickets = []
    for j in jobs:
        tickets.append(_submit(S, j))
        if trickle:
            time.sleep(0.002)
    out = {}
    t0 = time.time()
    peak = 0
    while len(out) < len(tickets):
        peak = max(peak, S.stats()["hbm_in_use"])
        for q, t in enumerate(tickets):
            if q not in out:
                r = S.poll(t)
                if r is not None:
                    out[q] = r
        assert time.time() - t0 < 100, "server did not finish"
        time.sleep(0.001)
    st = S.stats()
    S.close()
    assert peak <= budget and st["hbm_peak"] <= budget
    for j, b in zip(jobs, before):
        for k, v in b.items():
            assert torch.equal(j[k], v), "the server modified an input"
    return out, st


def _oracle_check(rplu, j, r, tag):
    piv = r.piv.cpu().numpy()
    forced = [tuple(p) for p in piv]
    fp64 = j["kind"] == "cauchy" or j["A"].dtype == torch.float64
    ts = r.rank if fp64 else _distinct_prefix(piv)
    if j["kind"] == "cauchy":
        x, y, G, B = (j[k].cpu().numpy() for k in ("x", "y", "G", "B"))
        o = R.rplu_cauchy(x, y, G, B, k=ts, seed=j["seed"], stream=j["stream"], forced=forced)
    else:
        A64 = j["A"].double().cpu().numpy()
        o = R.rplu_dense(A64, k=ts, seed=j["seed"], stream=j["stream"], forced=forced[:ts])
    assert o.rank == ts, tag
    if fp64:
        ex_r, ex_c, steps = parity.check_draws_ref(o.trace, tau=1e-12)
        assert steps == r.rank, tag
        assert parity.rel(r.U.cpu().numpy(), o.U) <= 1e-10, tag
        a_t = np.array([o.U[t, o.piv[t, 1]] for t in range(o.rank)])
        if o.rank:
            assert parity.rel(r.L.cpu().numpy() * a_t, o.L * a_t) <= 1e-10, tag
        return "P1", ex_r, steps
    tc = _compare_steps(o)
    LU_g = r.L[:, :tc].double().cpu().numpy() @ r.U[:tc].double().cpu().numpy()
    d = np.linalg.norm(LU_g - o.L[:, :tc] @ o.U[:tc]) / math.sqrt(o.a_fro2)
    assert d <= 1e-5, (tag, d)
    if j["tol"] == TOL:
        assert r.stop == rplu.RPLU_STOP_TOL, tag
        assert 0.0 <= r.err_fro2 <= TOL * TOL * r.a_fro2, (tag, r.err_fro2 / r.a_fro2)
        v = rplu.rplu_verify(j["A"], r.L, r.U)
        assert abs(v["err_fro2"] - r.err_fro2) <= 1e-12 * r.a_fro2, tag
    return "P2", d, r.refreshes


@pytest.mark.parametrize("budget_mb,workers,trickle", [(4096, 3, False), (80, 2, True)],
                         ids=["roomy", "tight-pool"])
def test_server_results_equal_alone_and_oracle(rplu_lib, budget_mb, workers, trickle):
    jobs = _mix(rplu_lib)
    out, st = _run(rplu_lib, jobs, budget_mb * MB, workers, trickle)
    assert st["completed"] == len(jobs) and st["queued"] == 0 and st["active"] == 0
    assert st["ticks"] >= 1 and st["tick_jobs"] == 12
    assert st["hbm_in_use"] == 0 and st["p50_ms"] <= st["p99_ms"]
    for q, j in enumerate(jobs):
        a = _alone(rplu_lib, j)
        r = out[q]
        tag = f"job {q} ({j['kind']})"
        assert r.status == 0, tag
        assert (r.rank, r.stop) == (a.rank, a.stop), tag
        assert r.res_fro2 == a.res_fro2 and r.a_fro2 == a.a_fro2, tag
        assert torch.equal(r.piv, a.piv), tag
        assert torch.equal(r.U, a.U) and torch.equal(r.L, a.L), tag
        res = _oracle_check(rplu_lib, j, r, tag)
        print(f"{tag}: rank {r.rank} stop {r.stop} oracle {res}", flush=True)


def test_server_reports_job_errors(rplu_lib):
    """Inputs written on the submitter's stream just before submission (the
    admission copy waits for them); a NaN job fails alone."""
    A = torch.randn(50, 60, device=DEV)
    A[3, 3] = float("nan")
    good = torch.randn(50, 60, device=DEV)
    S = rplu_lib.Server(budget_bytes=64 * MB, workers=1)
    tb, tg = S.submit_dense(A, k=5), S.submit_dense(good, k=5)
    t0 = time.time()
    res = {}
    while len(res) < 2:
        for name, t in (("bad", tb), ("good", tg)):
            if name in res:
                continue
            try:
                r = S.poll(t)
            except rplu_lib.RPLUError as e:
                res[name] = e.status
                continue
            if r is not None:
                res[name] = r
        assert time.time() - t0 < 30
    st = S.stats()
    S.close()
    assert res["bad"] == -4                      # RPLU_E_NONFINITE
    assert res["good"].rank == 5
    assert st["hbm_in_use"] == 0
