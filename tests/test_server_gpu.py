"""Continuous-batching server on the GPU: every job's result in the mix is
the result it gets alone.

A mix of small dense jobs (batched together), larger dense jobs (run alone)
and Cauchy-like jobs is submitted at once and in a trickle, under a slot pool
that holds only a few jobs; each result must equal, bit for bit, that of
rplu_dense / rplu_cauchy on the same inputs, seed and stream, and the
server must leave its inputs untouched.
"""
import time

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
MB = 1 << 20


def _mix(seed=3):
    rng = np.random.default_rng(seed)
    jobs = []
    for q in range(12):
        n, m = int(rng.integers(40, 700)), int(rng.integers(40, 700))
        dt = torch.float64 if q % 4 == 3 else torch.float32
        A = torch.from_numpy(rng.standard_normal((n, m))).to(dt).to(DEV)
        jobs.append(dict(kind="dense", A=A, k=0 if q % 2 else 30, tol=1e-2 if q % 2 else 0.0,
                         seed=q, stream=100 + q))
    for q in range(2):
        n = 2100 + 37 * q
        A = torch.from_numpy(W.random_dense(n, n - 50, seed=40 + q)).float().to(DEV)
        jobs.append(dict(kind="dense", A=A, k=40, tol=0.0, seed=7, stream=200 + q))
    for q in range(2):
        x, y, G, B = W.cauchy_like_random(1500 + 300 * q, 1200, 1 + q, seed=50 + q)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)   # noqa: E731
        jobs.append(dict(kind="cauchy", x=t(x), y=t(y), G=t(G), B=t(B), k=25, tol=0.0, seed=9,
                         stream=300 + q))
    return jobs


def _submit(S, j):
    if j["kind"] == "dense":
        return S.submit_dense(j["A"], k=j["k"], tol=j["tol"], seed=j["seed"], stream=j["stream"])
    return S.submit_cauchy(j["x"], j["y"], j["G"], j["B"], k=j["k"], tol=j["tol"], seed=j["seed"],
                           stream=j["stream"])


def _alone(rplu, j):
    if j["kind"] == "dense":
        return rplu.rplu_dense(j["A"].clone(), k=j["k"], tol=j["tol"], seed=j["seed"],
                               stream=j["stream"])
    return rplu.rplu_cauchy(j["x"], j["y"], j["G"].clone(), j["B"].clone(), k=j["k"],
                            tol=j["tol"], seed=j["seed"], stream=j["stream"])


def _run(rplu, jobs, budget, workers, trickle):
    before = [{k: v.clone() for k, v in j.items() if torch.is_tensor(v)} for j in jobs]
    S = rplu.Server(budget_bytes=budget, workers=workers)
    tickets = []
    for j in jobs:
        tickets.append(_submit(S, j))
        if trickle:
            time.sleep(0.002)
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for q, t in enumerate(tickets):
            if q not in out:
                r = S.poll(t)
                if r is not None:
                    out[q] = r
        assert time.time() - t0 < 100, "server did not finish"
        time.sleep(0.001)
    st = S.stats()
    S.close()
    for j, b in zip(jobs, before):
        for k, v in b.items():
            assert torch.equal(j[k], v), "the server modified an input"
    return out, st


@pytest.mark.parametrize("budget_mb,workers,trickle", [(4096, 3, False), (40, 2, True)],
                         ids=["roomy", "tight-pool"])
def test_server_results_equal_alone(rplu_lib, budget_mb, workers, trickle):
    jobs = _mix()
    out, st = _run(rplu_lib, jobs, budget_mb * MB, workers, trickle)
    assert st["completed"] == len(jobs) and st["queued"] == 0 and st["active"] == 0
    assert st["batches"] >= 1 and st["batched_jobs"] == 12
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


def test_server_reports_job_errors(rplu_lib):
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
    S.close()
    assert res["bad"] == -4                      # RPLU_E_NONFINITE
    assert res["good"].rank == 5
