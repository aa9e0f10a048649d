"""Plain CPU oracle for Randomly Pivoted LU (RPLU), FP64 / complex128.

TEST INFRASTRUCTURE. This module exists to check the HIP implementation.
Only tests, the smoke check and the bench's CPU-baseline leg may import it;
the product path never does, and it shares no code with the HIP path.

What it computes (Gilles & Wilber, "Low-Rank Approximation by Randomly
Pivoted LU"):

* Dense RPLU, Alg. 1. At step t the Schur complement S = A^(t) (S^(0) = A)
  gives a pivot (i, j) drawn with probability |S_ij|^2 / ||S||_F^2 (Sec. 1,
  the RPLU pivot distribution), realised in two stages: a row with
  probability ||S_i,:||^2 / ||S||_F^2, then a column of that row with
  probability |S_ij|^2 / ||S_i,:||^2 (Sec. 4.1, two-stage sampling). Then
  L(:,t) = S_:,j / S_ij, U(t,:) = S_i,:, and S <- S - L(:,t) U(t,:)
  (eq. residual_update).
* Cauchy-like RPLU, Alg. 3 with exact row masses. S is never formed: its
  entries are s_ij = (G_i,: B_:,j) / (x_i - y_j) (eq. cauchy-like), the row
  masses are sum_j |s_ij|^2 (Sec. 5.1, row-norm formula), and each step
  updates the generators with eqs. generator_update_g / generator_update_b.
  With exact masses the rejection step of Alg. 3 accepts with probability 1,
  so no acceptance draw is consumed.

Readings where the paper is silent (each also listed in the design notes):

* Inverse CDF: for weights w, P = inclusive prefix sums (np.cumsum,
  sequential), T := P[-1], and the drawn index is the first idx with
  P[idx] > u*T. The strict inequality never selects a zero-weight bin.
* The column draw uses the pivot row's own total (last prefix of |S_i,:|^2),
  not the row mass from the row stage.
* Pivot row i and column j of the updated S are set to exactly 0 (they are 0
  in exact arithmetic, eq. residual_update) and L(i,t) := 1.
* U is not conjugated for complex inputs; a mass is |z|^2 = re^2 + im^2.
* Stop test before each draw, in this order: T == 0 -> EXHAUSTED;
  tol > 0 and T <= tol^2 * T0 -> TOL; t == kmax -> RANK (or TOL_UNREACHED
  when tol > 0). kmax = min(n, m) when k == 0, else min(k, n, m).
* Random numbers come from oracle.philox.step_uniforms(seed, stream, t).
* C2PLU (complete 2-norm pivoting, Sec. 2.3.3), the greedy counterpart:
  i = a row of largest mass ||S_i,:||^2, then j = a column of largest
  |S_ij| in that row; ties go to the smallest index. Same update and stop
  test; no random numbers.
* RPLU in CUR form, Alg. 2 (Sec. 4.1): the same draws on row norms of the
  residual that are updated from A, the index sets and the core matrix
  U_k = A[I, J]^{-1} (eq. block-inverse-update), A never written.
* CPLU (complete pivoting, Sec. 1 and Sec. 2.3.2): (i, j) = an entry of
  largest |S_ij| over the whole Schur complement; moduli are compared as
  |S_ij|^2 in FP64 (squared_magnitude), and ties go to the first entry in
  row-major order (smallest i, then smallest j). Same update and stop test;
  no random numbers.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

from . import cauchy_bounds as CB
from .philox import step_uniforms, trial_uniforms

STOP_RANK = 1
STOP_TOL = 2
STOP_EXHAUSTED = 3
STOP_TOL_UNREACHED = 4
STOP_STALL = 5

# Optional stall rule (a library extension, not from the paper): the run
# keeps the best total T_best and the step t_best at which T last fell below
# STALL_RATIO * T_best (T_best = T_0, t_best = 0 at the start); it stops at
# step t when t - t_best reaches STALL_WINDOW. This ends tolerance runs whose
# target lies under the rounding floor of the working precision, where T
# stops falling, while a transient rise of T (a step can increase the
# residual) does not end the run.
STALL_WINDOW = 64
STALL_RATIO = 63.0 / 64.0


class NonFiniteInput(ValueError):
    pass


class ZeroPivot(ValueError):
    pass


# ------------------------------------------------------------------ sampling

def squared_magnitude(z: np.ndarray) -> np.ndarray:
    """|z|^2 elementwise, in FP64."""
    if np.iscomplexobj(z):
        return z.real * z.real + z.imag * z.imag
    z = np.asarray(z, dtype=np.float64)
    return z * z


def first_exceeding(prefix: np.ndarray, target: float) -> int:
    """First index idx with prefix[idx] > target (prefix non-decreasing)."""
    idx = int(np.searchsorted(prefix, target, side="right"))
    if idx >= prefix.shape[0]:
        raise ValueError("target is not below the last prefix value")
    return idx


@dataclass
class Draw:
    """One inverse-CDF draw and the CDF bin of the index actually used."""
    drawn: int          # index the draw selects
    used: int           # index used (== drawn unless forced)
    total: float        # T = last inclusive prefix
    target: float       # u * T
    lo: float           # lower edge of the used index's bin (0 for idx 0)
    hi: float           # upper edge of the used index's bin


def largest(weights: np.ndarray, forced: Optional[int] = None) -> Draw:
    """C2PLU's choice (Sec. 2.3.3): the first index of the largest weight."""
    w = np.asarray(weights, dtype=np.float64)
    drawn = int(np.argmax(w))
    used = drawn if forced is None else int(forced)
    return Draw(drawn, used, float(np.sum(w)), float("nan"), float("nan"), float("nan"))


def largest_entry(S: np.ndarray, forced=(None, None)):
    """CPLU's choice (Sec. 1, complete pivoting): the entry of largest
    |S_ij|^2 over all of S, the first in row-major order among equal ones.
    Returns the row and column Draws (forced: an (i, j) to use instead)."""
    W = squared_magnitude(S)
    i, j = np.unravel_index(int(np.argmax(W)), W.shape)   # argmax: first in C order
    return _entry_draws(int(i), int(j), float(np.sum(W)), forced)


def _entry_draws(i: int, j: int, T: float, forced):
    fi, fj = forced
    nan = float("nan")
    rd = Draw(i, i if fi is None else int(fi), T, nan, nan, nan)
    cd = Draw(j, j if fj is None else int(fj), nan, nan, nan, nan)
    return rd, cd


def inverse_cdf(weights: np.ndarray, u: float, forced: Optional[int] = None) -> Draw:
    P = np.cumsum(np.asarray(weights, dtype=np.float64))
    T = float(P[-1])
    target = u * T
    drawn = first_exceeding(P, target)
    used = drawn if forced is None else int(forced)
    lo = float(P[used - 1]) if used > 0 else 0.0
    return Draw(drawn, used, T, target, lo, float(P[used]))


# ------------------------------------------------------------------- results

@dataclass
class StepTrace:
    t: int
    row: Draw
    col: Draw
    a: complex


@dataclass
class RPLUResult:
    L: np.ndarray                 # n x rank
    U: np.ndarray                 # rank x m
    piv: np.ndarray               # rank x 2 (i_t, j_t)
    rank: int
    stop: int
    a_fro2: float                 # ||A||_F^2 (T at step 0)
    res_fro2: float               # T at the stop test
    S: Optional[np.ndarray] = None            # final Schur complement (dense)
    G: Optional[np.ndarray] = None            # final generators (Cauchy)
    B: Optional[np.ndarray] = None
    trace: list = field(default_factory=list)
    masses: list = field(default_factory=list)   # rowmass per step if asked
    trials: list = field(default_factory=list)   # rejection trials per step (bounds)


def _stop_reason(t: int, T: float, T0: float, kmax: int, tol: float, stall_ref=None,
                 M=None, M0=None) -> int:
    """Stop test before the draw of step t. stall_ref: None (no stall rule)
    or a two-element list [T_best, t_best], updated here. M, M0: the largest
    row mass now and at step 0, for the max-mass rule (CUR-AAA, Alg. 4:
    stop when max_i u_i <= tol^2 max_i u^(0)_i) in place of the total."""
    if T == 0.0:
        return STOP_EXHAUSTED
    if tol > 0.0 and ((M <= (tol * tol) * M0) if M is not None else (T <= (tol * tol) * T0)):
        return STOP_TOL
    if stall_ref is not None:
        if t == 0:
            stall_ref[0], stall_ref[1] = T, 0
        elif T < STALL_RATIO * stall_ref[0]:
            stall_ref[0], stall_ref[1] = T, t
        if t - stall_ref[1] >= STALL_WINDOW:
            return STOP_STALL
    if t == kmax:
        return STOP_TOL_UNREACHED if tol > 0.0 else STOP_RANK
    return 0


def _forced_at(forced, t: int):
    """Forced (i, j) for step t, or (None, None) to use the draw. A forced
    sequence may hold None entries for steps that draw freely."""
    if forced is None or t >= len(forced) or forced[t] is None:
        return None, None
    return int(forced[t][0]), int(forced[t][1])


def _kmax(n: int, m: int, k: int) -> int:
    return min(n, m) if k <= 0 else min(k, n, m)


# --------------------------------------------------------------- dense form

def schur_update(S: np.ndarray, i: int, j: int):
    """Apply pivot (i, j) to S in place (eq. residual_update; Alg. 1 body).

    Returns (l, u, a): l = S_:,j / a with l[i] = 1, u = S_i,: and a = S_ij.
    Row i and column j of the result are set to exactly zero.
    """
    a = S[i, j]
    if a == 0:
        raise ZeroPivot(f"pivot ({i},{j}) is zero")
    u = S[i, :].copy()
    l = S[:, j] / a
    l[i] = 1.0
    S -= np.outer(l, u)
    S[i, :] = 0.0
    S[:, j] = 0.0
    return l, u, a


def rplu_dense(A: np.ndarray, k: int = 0, tol: float = 0.0, seed: int = 0,
               stream: int = 0, forced: Optional[Sequence] = None,
               keep_masses: bool = False, stall: bool = False,
               greedy: bool = False, complete: bool = False) -> RPLUResult:
    """Alg. 1 with two-stage exact sampling (Sec. 4.1).

    forced: optional sequence of (i, j) pivots to use instead of the draws
    (the draws are still made and recorded, so a caller can check where a
    draw landed relative to the forced pivot's CDF bin).
    greedy: C2PLU (Sec. 2.3.3) instead of the random draws.
    complete: CPLU (Sec. 1, complete pivoting) instead of the random draws.
    """
    if greedy and complete:
        raise ValueError("C2PLU and CPLU are exclusive")
    S = np.array(A, dtype=np.complex128 if np.iscomplexobj(A) else np.float64,
                 copy=True)
    n, m = S.shape
    kmax = _kmax(n, m, k)
    L = np.zeros((n, kmax), dtype=S.dtype)
    U = np.zeros((kmax, m), dtype=S.dtype)
    piv = np.full((kmax, 2), -1, dtype=np.int64)
    trace, masses = [], []
    T0 = None
    stall_ref = [0.0, 0] if stall else None
    t = 0
    while True:
        rowmass = np.sum(squared_magnitude(S), axis=1)
        T = float(np.cumsum(rowmass)[-1]) if n else 0.0
        if not np.isfinite(T):
            raise NonFiniteInput("non-finite entry in the input")
        if t == 0:
            T0 = T
        stop = _stop_reason(t, T, T0, kmax, tol, stall_ref)
        if stop:
            break
        if keep_masses:
            masses.append(rowmass)
        u1, u2 = step_uniforms(seed, stream, t)
        fi, fj = _forced_at(forced, t)
        if complete:
            rd, cd = largest_entry(S, (fi, fj))
        else:
            rd = largest(rowmass, fi) if greedy else inverse_cdf(rowmass, u1, fi)
            w_row = squared_magnitude(S[rd.used, :])
            cd = largest(w_row, fj) if greedy else inverse_cdf(w_row, u2, fj)
        i, j = rd.used, cd.used
        l, u, a = schur_update(S, i, j)
        L[:, t] = l
        U[t, :] = u
        piv[t] = (i, j)
        trace.append(StepTrace(t, rd, cd, complex(a)))
        t += 1
    return RPLUResult(L[:, :t].copy(), U[:t].copy(), piv[:t].copy(), t, stop,
                      T0, T, S=S, trace=trace, masses=masses)


def factorization_check(A: np.ndarray, L: np.ndarray, U: np.ndarray,
                        S: Optional[np.ndarray] = None) -> dict:
    """The three sums of squares of the verification, by their definitions,
    in FP64 (complex128 for complex data): ||A||_F^2; ||A - L U||_F^2, the
    error of the rank-k approximation L U (Sec. 2, the error measure); and,
    with S given, ||A - L U - S||_F^2, which is 0 in exact arithmetic when S
    is the run's Schur complement (A - L U = A^(k), eq. approximation_update).
    L U is a library matrix product."""
    wide = np.complex128 if any(np.iscomplexobj(v) for v in (A, L, U)) else np.float64
    A = np.asarray(A, dtype=wide)
    E = A - np.asarray(L, dtype=wide) @ np.asarray(U, dtype=wide)
    out = {"a_fro2": float(np.sum(squared_magnitude(A))),
           "err_fro2": float(np.sum(squared_magnitude(E)))}
    if S is not None:
        out["schur_gap_fro2"] = float(np.sum(squared_magnitude(E - np.asarray(S, dtype=wide))))
    return out


def schur_closed_form(A: np.ndarray, I: Sequence[int], J: Sequence[int]) -> np.ndarray:
    """Schur complement after pivots on rows I, columns J, by its definition
    A - A[:,J] A[I,J]^{-1} A[I,:] (depends on the sets only; Sec. 4.1, the
    interpolative CUR form C U R with U = A[I,J]^{-1})."""
    I = list(I)
    J = list(J)
    if not I:
        return np.array(A, copy=True)
    W = A[np.ix_(I, J)]
    return A - A[:, J] @ np.linalg.solve(W, A[I, :])


def schur_closed_form_masses(get_rows, n: int, I: Sequence[int], J: Sequence[int],
                             steps: Sequence[int], row_block: int = 1024):
    """Row masses ||S^(t)_r,:||^2 (all n rows) and the row i_t of S^(t), for
    each t in `steps`, where S^(t) is the closed-form Schur complement after
    the first t pivots (I[:t], J[:t]): A - A[:,J_t] A[I_t,J_t]^{-1} A[I_t,:]
    (as in schur_closed_form), streamed a block of rows at a time so that no
    n x m FP64 array is held. get_rows(r0, r1) returns rows r0..r1-1 of A in
    FP64. Returns {t: (masses, pivot_row)}."""
    I = np.asarray(I, dtype=np.int64)
    J = np.asarray(J, dtype=np.int64)
    AI = get_rows_at(get_rows, I)                    # all pivot rows of A
    X = {}
    for t in steps:
        X[t] = np.linalg.solve(AI[:t][:, J[:t]], AI[:t]) if t else None
    out = {t: [np.empty(n), None] for t in steps}
    for r0 in range(0, n, row_block):
        r1 = min(n, r0 + row_block)
        blk = get_rows(r0, r1)
        for t in steps:
            S = blk if t == 0 else blk - blk[:, J[:t]] @ X[t]
            out[t][0][r0:r1] = np.sum(squared_magnitude(S), axis=1)
    for t in steps:
        if t < len(I):
            row = AI[t:t + 1]
            out[t][1] = (row if t == 0 else row - row[:, J[:t]] @ X[t])[0]
    return {t: (v[0], v[1]) for t, v in out.items()}


def get_rows_at(get_rows, idx):
    """Rows idx of A (FP64) through a row-range accessor."""
    return np.stack([get_rows(int(r), int(r) + 1)[0] for r in idx]) if len(idx) else None


# ------------------------------------------------------------- CUR form

@dataclass
class CURResult:
    """RPLU in CUR form: A ~ A[:, J] Uc A[I, :] with Uc = A[I, J]^{-1}."""
    I: np.ndarray                 # rank row indices, in selection order
    J: np.ndarray                 # rank column indices
    Uc: np.ndarray                # rank x rank core matrix
    rank: int
    stop: int
    a_fro2: float                 # sum of the initial row norms, ||A||_F^2
    res_fro2: float               # sum of the row-norm estimates at the stop test
    rownorms: np.ndarray          # the row-norm estimates at the stop test
    trace: list = field(default_factory=list)
    masses: list = field(default_factory=list)

    @property
    def piv(self) -> np.ndarray:
        return np.stack([self.I, self.J], axis=1) if self.rank else np.zeros((0, 2), np.int64)


def block_inverse_update(Uc: np.ndarray, z: np.ndarray, w: np.ndarray, omega):
    """U_{k+1} = A[I+i, J+j]^{-1} from U_k = A[I, J]^{-1} (eq.
    block-inverse-update): with W_{k+1} = [[W_k, w], [z^T, omega]] and
    sigma = omega - z^T U_k w, the blocks U_k + U_k w z^T U_k / sigma,
    -U_k w / sigma, -z^T U_k / sigma and 1 / sigma. Returns (U_{k+1}, sigma)."""
    Uw = Uc @ w
    zU = z @ Uc
    sigma = omega - zU @ w
    if sigma == 0:
        raise ZeroPivot("zero Schur complement of the core matrix")
    k = Uc.shape[0]
    out = np.empty((k + 1, k + 1), dtype=np.result_type(Uc, z, w, omega))
    out[:k, :k] = Uc + np.outer(Uw, zU) / sigma
    out[:k, k] = -Uw / sigma
    out[k, :k] = -zU / sigma
    out[k, k] = 1.0 / sigma
    return out, sigma


def cur_rownorm_update(A, I, J, Uc, nrm, l, chat):
    """Row norms of A^(k+1) = A^(k) - chat l^T from those of A^(k) (Sec. 4.1,
    row-norm updates): n - 2 Re((g - v) conj(chat)) + ||l||^2 |chat|^2 with
    g = A conj(l) and v = A[:, J] U_k g[I], so that g - v = A^(k) conj(l)."""
    g = A @ np.conj(l)
    v = A[:, J] @ (Uc @ g[I]) if I else np.zeros_like(g)
    l2 = float(np.sum(squared_magnitude(l)))
    return nrm - 2.0 * np.real((g - v) * np.conj(chat)) + l2 * squared_magnitude(chat)


def rplu_cur(A: np.ndarray, k: int = 0, tol: float = 0.0, seed: int = 0, stream: int = 0,
             forced: Optional[Sequence] = None, keep_masses: bool = False, stall: bool = False,
             greedy: bool = False) -> CURResult:
    """Alg. 2 (Sec. 4.1, RPLU in CUR form): A is only read. The state is the
    index sets I, J, the core U_k = A[I, J]^{-1} and the row norms n_k of
    the residual A^(k) = A - A[:, J] U_k A[I, :], which are updated (not
    recomputed) each step. Same draws, stop test and stall rule as
    rplu_dense; greedy: C2PLU (Sec. 2.3.3) instead of the draws.

    Readings: the residual's entries in the selected columns (of its pivot
    row) and selected rows (of its pivot column) are set to exactly 0, as in
    the dense form; the row-norm step uses g = A conj(l) (the derivation of
    the row-norm recurrence for complex A; Alg. 2 prints A l, the same for
    real A); the estimates of selected rows are set to 0 and negative
    estimates (rounding) to 0."""
    A = np.asarray(A)
    A = A.astype(np.complex128 if np.iscomplexobj(A) else np.float64, copy=False)
    n, m = A.shape
    kmax = _kmax(n, m, k)
    I: list = []
    J: list = []
    Uc = np.zeros((0, 0), dtype=A.dtype)
    nrm = np.sum(squared_magnitude(A), axis=1)           # initial row norms
    sel = np.zeros(n, dtype=bool)
    trace, masses = [], []
    T0 = None
    stall_ref = [0.0, 0] if stall else None
    t = 0
    while True:
        T = float(np.cumsum(nrm)[-1]) if n else 0.0
        if not np.isfinite(T):
            raise NonFiniteInput("non-finite entry in the input")
        if t == 0:
            T0 = T
        stop = _stop_reason(t, T, T0, kmax, tol, stall_ref)
        if stop:
            break
        if keep_masses:
            masses.append(nrm.copy())
        u1, u2 = step_uniforms(seed, stream, t)
        fi, fj = _forced_at(forced, t)
        # Step 1: pivot row of the residual, its column
        rd = largest(nrm, fi) if greedy else inverse_cdf(nrm, u1, fi)
        i = rd.used
        r = A[i, :]
        rhat = r - A[I, :].T @ (Uc.T @ r[J]) if I else r.copy()
        rhat[J] = 0.0
        w_row = squared_magnitude(rhat)
        cd = largest(w_row, fj) if greedy else inverse_cdf(w_row, u2, fj)
        j = cd.used
        if rhat[j] == 0:
            raise ZeroPivot(f"pivot ({i},{j}) is zero")
        c = A[:, j]
        chat = c - A[:, J] @ (Uc @ c[I]) if I else c.copy()
        chat[I] = 0.0
        # Step 2: row norms of A^(k+1) = A^(k) - chat l^T
        nrm = cur_rownorm_update(A, I, J, Uc, nrm, rhat / rhat[j], chat)
        sel[i] = True
        nrm[sel] = 0.0
        nrm = np.maximum(nrm, 0.0)
        # Step 3: core matrix
        Uc, _ = block_inverse_update(Uc, A[i, J], A[I, j], A[i, j])
        I.append(i)
        J.append(j)
        trace.append(StepTrace(t, rd, cd, complex(rhat[j])))
        t += 1
    return CURResult(np.array(I, dtype=np.int64), np.array(J, dtype=np.int64), Uc, t, stop,
                     T0, T, nrm, trace=trace, masses=masses)


# -------------------------------------------------------- Cauchy-like form

def cauchy_entries(x, y, G, B) -> np.ndarray:
    """Dense n x m matrix with entries (G_i,: B_:,j) / (x_i - y_j)
    (eq. cauchy-like)."""
    return (G @ B) / (x[:, None] - y[None, :])


def cauchy_row(x, y, G, B, i: int) -> np.ndarray:
    """Row i: (G_i,: B) / (x_i - y) (Alg. 3, row of A^(k))."""
    return (G[i, :] @ B) / (x[i] - y)


def cauchy_col(x, y, G, B, j: int) -> np.ndarray:
    """Column j: (G B_:,j) / (x - y_j) (Alg. 3, column of A^(k))."""
    return (G @ B[:, j]) / (x - y[j])


def cauchy_row_masses(x, y, G, B, rows_per_block: int = 512) -> np.ndarray:
    """sum_j |s_ij|^2 for every row i (Sec. 5.1, exact row norms), one block
    of rows at a time so that no n x m array is held."""
    n = x.shape[0]
    out = np.empty(n, dtype=np.float64)
    for i0 in range(0, n, rows_per_block):
        i1 = min(n, i0 + rows_per_block)
        s = (G[i0:i1] @ B) / (x[i0:i1, None] - y[None, :])
        out[i0:i1] = np.sum(squared_magnitude(s), axis=1)
    return out


def cauchy_largest_entry(x, y, G, B, rows_per_block: int = 512):
    """CPLU's choice on a Cauchy-like matrix (Sec. 1, complete pivoting):
    (i, j) of the largest |s_ij|^2 over all entries, the first in row-major
    order among equal ones, one block of rows at a time (a later block
    replaces the best only when strictly larger)."""
    n = x.shape[0]
    best, bi, bj = -1.0, -1, -1
    for i0 in range(0, n, rows_per_block):
        i1 = min(n, i0 + rows_per_block)
        W = squared_magnitude((G[i0:i1] @ B) / (x[i0:i1, None] - y[None, :]))
        r, c = np.unravel_index(int(np.argmax(W)), W.shape)
        if W[r, c] > best:
            best, bi, bj = float(W[r, c]), i0 + int(r), int(c)
    return bi, bj


def cauchy_generator_update(x, y, G, B, i: int, j: int):
    """One pivot step on the generators, in place (eqs. generator_update_g,
    generator_update_b): regenerate r = row i and c = column j, then
    G <- G - (1/a) c G_i,:  and  B <- B - (1/a) B_:,j r, and zero G_i,: and
    B_:,j exactly. Returns (c, r, a)."""
    r = cauchy_row(x, y, G, B, i)
    a = r[j]
    if a == 0:
        raise ZeroPivot(f"pivot ({i},{j}) is zero")
    c = cauchy_col(x, y, G, B, j)
    gi = G[i, :].copy()
    bj = B[:, j].copy()
    G -= np.outer(c, gi) / a
    B -= np.outer(bj, r) / a
    G[i, :] = 0.0
    B[:, j] = 0.0
    return c, r, a


def rplu_cauchy(x, y, G, B, k: int = 0, tol: float = 0.0, seed: int = 0,
                stream: int = 0, forced: Optional[Sequence] = None,
                keep_masses: bool = False, mass_steps: Optional[set] = None,
                stall: bool = False, greedy: bool = False,
                complete: bool = False, bounds=None, maxmass: bool = False) -> RPLUResult:
    """Alg. 3 with exact row masses (no rejection), generators in complex128.

    bounds: (nu, leaf) for Alg. 3 as printed: certified row-norm upper
    bounds (App. C, oracle.cauchy_bounds) and the rejection-sampled row draw
    (Step 1); the trace's row Draw is then the accepted trial's, over the
    bounds, result.trials counts the trials of every step and keep_masses
    keeps the bounds. The stop test runs on the bound total with tol^2 / nu
    (see oracle.cauchy_bounds).
    maxmass: the tolerance stop compares the largest row mass (or bound)
    with tol^2 times its value at step 0 (Alg. 4), unscaled by nu.

    greedy: C2PLU (Sec. 2.3.3) instead of the random draws (needs the masses
    at every step).
    complete: CPLU (Sec. 1, complete pivoting) instead of the random draws.

    mass_steps: if given, row masses (and hence the draw check) are computed
    only at these steps; elsewhere the run must be forced. This keeps
    full-size forced replays cheap (the generator update is O((n+m)p)).
    """
    x = np.asarray(x, dtype=np.complex128)
    y = np.asarray(y, dtype=np.complex128)
    G = np.array(G, dtype=np.complex128, copy=True)
    B = np.array(B, dtype=np.complex128, copy=True)
    n, m = x.shape[0], y.shape[0]
    assert G.shape[0] == n and B.shape[1] == m and G.shape[1] == B.shape[0]
    kmax = _kmax(n, m, k)
    L = np.zeros((n, kmax), dtype=np.complex128)
    U = np.zeros((kmax, m), dtype=np.complex128)
    piv = np.full((kmax, 2), -1, dtype=np.int64)
    trace, masses = [], []
    T0 = None
    T = float("nan")
    stall_ref = [0.0, 0] if stall else None
    if bounds is not None and (complete or mass_steps is not None):
        raise ValueError("row-norm bounds replace the exact masses")
    plan = CB.interaction_lists(x, y, bounds[0], bounds[1]) if bounds is not None else None
    tol2_scale = 1.0 / bounds[0] if bounds is not None and not maxmass else 1.0
    M0 = None
    trials = []
    if (greedy or complete) and mass_steps is not None:
        raise ValueError("C2PLU and CPLU need the row masses at every step")
    if greedy and complete:
        raise ValueError("C2PLU and CPLU are exclusive")
    if stall and mass_steps is not None:
        raise ValueError("the stall rule needs the total at every step")
    t = 0
    while True:
        need_mass = mass_steps is None or t in mass_steps or t == 0
        if need_mass:
            rowmass = (CB.row_norm_bounds(plan, x, y, G, B) if plan is not None
                       else cauchy_row_masses(x, y, G, B))
            T = float(np.cumsum(rowmass)[-1])
            if not np.isfinite(T):
                raise NonFiniteInput("non-finite generator or node data")
            if t == 0:
                T0 = T
            M = float(np.max(rowmass)) if maxmass else None
            if t == 0:
                M0 = M
            stop = _stop_reason(t, T, T0, kmax, tol * np.sqrt(tol2_scale), stall_ref, M, M0)
        else:
            stop = STOP_RANK if t == kmax else 0
        if stop:
            break
        u1, u2 = step_uniforms(seed, stream, t)
        fi, fj = _forced_at(forced, t)
        if not need_mass and fi is None:
            raise ValueError("a step without row masses needs a forced pivot")
        if need_mass and keep_masses:
            masses.append(rowmass)
        if complete:
            rd, cd = _entry_draws(*cauchy_largest_entry(x, y, G, B), T, (fi, fj))
        else:
            if plan is not None and not greedy and fi is None:
                rd, q = _rejection_row(x, y, G, B, rowmass, seed, stream, t)
                trials.append(q)
            elif need_mass:
                rd = largest(rowmass, fi) if greedy else inverse_cdf(rowmass, u1, fi)
            else:
                rd = Draw(-1, fi, float("nan"), float("nan"), float("nan"), float("nan"))
            w_row = squared_magnitude(cauchy_row(x, y, G, B, rd.used))
            cd = largest(w_row, fj) if greedy else inverse_cdf(w_row, u2, fj)
        i, j = rd.used, cd.used
        c, r, a = cauchy_generator_update(x, y, G, B, i, j)
        l = c / a
        l[i] = 1.0
        L[:, t] = l
        U[t, :] = r
        piv[t] = (i, j)
        trace.append(StepTrace(t, rd, cd, complex(a)))
        t += 1
    return RPLUResult(L[:, :t].copy(), U[:t].copy(), piv[:t].copy(), t, stop,
                      T0, T, G=G, B=B, trace=trace, masses=masses, trials=trials)


def _rejection_row(x, y, G, B, u, seed, stream, t):
    """Alg. 3, Step 1: draw i from the bounds u, regenerate row i, accept
    with probability ||row||^2 / u_i; repeat. Returns (Draw of the accepted
    trial over u, number of trials)."""
    for q in range(CB.MAX_TRIALS):
        v_row, v_acc = trial_uniforms(seed, stream, t, q)
        d = inverse_cdf(u, v_row)
        rho = float(np.sum(squared_magnitude(cauchy_row(x, y, G, B, d.used))))
        if v_acc * u[d.used] < rho:
            return d, q + 1
    raise ValueError(f"step {t}: no row accepted in {CB.MAX_TRIALS} trials (bounds below the masses?)")
