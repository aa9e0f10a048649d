"""Dense FP32 32768 x 32768, k = 512 (the configuration bench.py times, with
its default hipGraph replay) checked by properties that hold at any size and
by the oracle on sampled outputs.

The oracle cannot replay 512 steps on a 4.3 GB matrix, but the Schur
complement after pivots on rows I and columns J has the closed form
A - A[:,J] A[I,J]^-1 A[I,:] (the oracle's schur_closed_form, pinned), whose
entries on sampled rows and columns only need A on those rows and columns
and on I, J. The GPU's final S is compared with it on 96 x 96 sampled
entries, in FP64 on the host, to the FP32 target 1e-5 relative to ||A||_F
(the sampled RMS error scaled to the whole matrix). Also: every draw target
is u * T with u from the oracle's Philox stream, lands in its bin (trace
words), the pivots are distinct, L(i_t, t) = 1, pivot rows and columns of S
are exactly 0, and ||A - L U - S||_F from the FP64 matrix-core check is
within the same target.
"""
import math

import numpy as np
import pytest
import torch

import parity
import workloads as W
from oracle import rplu as O
from oracle.philox import step_uniforms

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

DEV = "cuda:0"


def test_config3_dense_32768_fp32(rplu_lib):
    n, k = 32768, 512
    print("generating the 32768^2 input", flush=True)
    A0 = W.dense_reflector_matrix_device(n, sigma_power=-2.0, q=256, seed=3, device=DEV,
                                         dtype=torch.float32)
    S = A0.clone()
    print("running rank 512", flush=True)
    res = rplu_lib.rplu_dense(S, k=k, seed=0, want_trace=True)
    assert res.rank == k and res.stop == rplu_lib.RPLU_STOP_RANK
    piv = res.piv.cpu().numpy().astype(np.int64)
    tr = res.trace.cpu().numpy()
    parity.check_trace_self(tr, piv)
    for t in range(k):
        u1, u2 = step_uniforms(0, 0, t)
        assert tr[t, 1] == u1 * tr[t, 0] and tr[t, 5] == u2 * tr[t, 4], t
    I, J = piv[:, 0], piv[:, 1]
    assert len(set(I.tolist())) == k and len(set(J.tolist())) == k
    L, U = res.L, res.U
    It = torch.from_numpy(I).to(DEV)
    Jt = torch.from_numpy(J).to(DEV)
    assert torch.all(L[It, torch.arange(k, device=DEV)] == 1.0)
    assert int(torch.count_nonzero(S[It, :])) == 0
    assert int(torch.count_nonzero(S[:, Jt])) == 0

    fa = math.sqrt(res.a_fro2)
    # FP64 matrix-core check of the whole factorisation
    v = rplu_lib.rplu_verify(A0, L, U, S)
    assert abs(v["a_fro2"] - res.a_fro2) <= 1e-9 * res.a_fro2
    assert math.sqrt(v["schur_gap_fro2"]) <= 1e-5 * fa

    # closed-form Schur complement on sampled entries (FP64, host)
    rng = np.random.default_rng(7)
    rows = np.setdiff1d(rng.choice(n, 160, replace=False), I)[:96]
    cols = np.setdiff1d(rng.choice(n, 160, replace=False), J)[:96]
    R = np.concatenate([rows, I])
    Cc = np.concatenate([cols, J])
    Rt, Ct = torch.from_numpy(R).to(DEV), torch.from_numpy(Cc).to(DEV)
    sub = A0[Rt][:, Ct].double().cpu().numpy()          # (96 + k) x (96 + k)
    nr, nc = len(rows), len(cols)
    S_sub = O.schur_closed_form(sub, range(nr, nr + k), range(nc, nc + k))[:nr, :nc]
    S_gpu = S[torch.from_numpy(rows).to(DEV)][:, torch.from_numpy(cols).to(DEV)].double().cpu().numpy()
    rms = float(np.sqrt(np.mean((S_gpu - S_sub) ** 2)))
    est = rms * n                                        # Frobenius-norm estimate (n = m)
    print(f"sampled rms error {rms:.3e}, whole-matrix estimate {est / fa:.3e} of ||A||_F; "
          f"||A - LU - S|| = {math.sqrt(v['schur_gap_fro2']) / fa:.3e}; "
          f"residual {math.sqrt(res.res_fro2 / res.a_fro2):.3e}", flush=True)
    assert est <= 1e-5 * fa
    # the residual reported by the run is the FP64 total of the FP32 S
    assert abs(math.sqrt(res.res_fro2) - math.sqrt(v["err_fro2"])) <= 1e-5 * fa


SAMPLED_STEPS = [0, 1, 2, 3, 7, 15, 31, 63, 95, 127, 191, 255, 319, 383, 447, 511]


@pytest.mark.timeout(900)
def test_config3_draws_against_closed_form_masses(rplu_lib):
    """Draw agreement (protocol P2) at 16 sampled steps of the 32768^2 FP32
    run: the oracle's FP64 row masses of S^(t) from the closed-form Schur
    complement of the same (FP32-valued) A under the GPU's first t pivots;
    the oracle's target u1*T lands in the GPU's row bin within delta_t*T,
    delta_t = sum_i |m_gpu,i - m_orc,i| / T the measured mass discrepancy, and
    the same for the column draw in the pivot row. Each step's delta and
    whether the draw matched exactly are printed."""
    n, k = 32768, 512
    print("generating the 32768^2 input", flush=True)
    A0 = W.dense_reflector_matrix_device(n, sigma_power=-2.0, q=256, seed=3, device=DEV,
                                         dtype=torch.float32)
    S = A0.clone()
    res = rplu_lib.rplu_dense(S, k=k, seed=0, want_trace=True, want_rowmass=True)
    assert res.rank == k
    piv = res.piv.cpu().numpy().astype(np.int64)
    rm_gpu = res.rowmass[SAMPLED_STEPS].cpu().numpy()
    U_gpu = res.U[SAMPLED_STEPS].double().cpu().numpy()
    tr = res.trace.cpu().numpy()
    del S, res
    A_host = A0.cpu().numpy()                      # FP32, 4.3 GB
    del A0
    torch.cuda.empty_cache()
    print("closed-form masses at 16 steps on the host", flush=True)
    get_rows = lambda a, b: A_host[a:b].astype(np.float64)      # noqa: E731
    orc = O.schur_closed_form_masses(get_rows, n, piv[:, 0], piv[:, 1], SAMPLED_STEPS,
                                     row_block=2048)
    exact = 0
    for q, t in enumerate(SAMPLED_STEPS):
        m_orc, row_orc = orc[t]
        i, j = int(piv[t, 0]), int(piv[t, 1])
        u1, u2 = step_uniforms(0, 0, t)
        P = np.cumsum(m_orc)
        T = P[-1]
        delta = float(np.sum(np.abs(rm_gpu[q] - m_orc)) / T)
        lo, hi = (P[i - 1] if i else 0.0), P[i]
        tgt = u1 * T
        win = delta * T
        assert lo - win <= tgt < hi + win, (t, lo, tgt, hi, delta)
        w_orc = row_orc ** 2
        Pc = np.cumsum(w_orc)
        Ti = Pc[-1]
        delta_c = float(np.sum(np.abs(U_gpu[q] ** 2 - w_orc)) / Ti)
        loc, hic = (Pc[j - 1] if j else 0.0), Pc[j]
        tgc = u2 * Ti
        assert loc - delta_c * Ti <= tgc < hic + delta_c * Ti, (t, loc, tgc, hic, delta_c)
        ok = lo <= tgt < hi and loc <= tgc < hic
        exact += ok
        # the GPU's own T against the oracle's
        print(f"t={t:3d} delta_row={delta:.2e} delta_col={delta_c:.2e} "
              f"T_gpu/T_orc-1={tr[t, 0] / T - 1:+.2e} exact={ok}", flush=True)
    print(f"{exact}/{len(SAMPLED_STEPS)} sampled draws land in the GPU's bins exactly", flush=True)
