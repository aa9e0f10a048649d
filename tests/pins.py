"""Pins of the CPU oracle: checks against facts the paper and the
mathematics fix, not against the oracle's own formulas.

Each pin is a function that raises AssertionError on failure, so that the
mutation tests can plant a mistake in the oracle and confirm that some pin
catches it. Pins reach the oracle through the module object `O` so that a
monkeypatched oracle function is the one exercised.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
from scipy import stats

import workloads as W
from oracle import philox as PH
from oracle import rplu as O


# ----------------------------------------------------------------- helpers

def _numpy_philox_block(seed: int, stream: int, t: int):
    """numpy's Philox4x64-10 output for counter (t, stream, 0, 0): numpy
    pre-increments its 256-bit counter, so start it one below."""
    c = (t | (stream << 64)) - 1
    c %= 1 << 256
    words = [(c >> (64 * q)) & PH.MASK64 for q in range(4)]
    bg = np.random.Philox(key=np.array([seed, 0], dtype=np.uint64),
                          counter=np.array(words, dtype=np.uint64))
    return [int(v) for v in bg.random_raw(4)]


def _p_of(S):
    """The RPLU pivot distribution |S_ij|^2 / ||S||_F^2 (Sec. 1), computed
    with numpy's abs, independently of the oracle's mass routine."""
    w = np.abs(S) ** 2
    return w / w.sum()


def _enumerate(S, depth, prob=1.0, out=None, k=0):
    """Accumulate E||S^(k)||_F^2 (k = 0..depth) over every pivot sequence,
    weighting each by the product of the step probabilities."""
    if out is None:
        out = np.zeros(depth + 1)
    out[k] += prob * float(np.sum(np.abs(S) ** 2))
    if k == depth:
        return out
    P = _p_of(S) if np.any(S != 0) else None
    if P is None:
        for kk in range(k + 1, depth + 1):
            out[kk] += 0.0
        return out
    for (i, j), pij in np.ndenumerate(P):
        if pij == 0:
            continue
        S2 = S.copy()
        O.schur_update(S2, i, j)
        _enumerate(S2, depth, prob * pij, out, k + 1)
    return out


def _one_step_moments(A):
    """E[S^(1)] and E[S^(1)* S^(1)] by enumeration over the first pivot."""
    P = _p_of(A)
    E1 = np.zeros_like(A)
    G1 = np.zeros((A.shape[1], A.shape[1]), dtype=A.dtype)
    for (i, j), pij in np.ndenumerate(P):
        if pij == 0:
            continue
        S = A.copy()
        O.schur_update(S, i, j)
        E1 = E1 + pij * S
        G1 = G1 + pij * (S.conj().T @ S)
    return E1, G1


def _chi2_pvalue(counts, probs):
    counts = np.asarray(counts, dtype=np.float64).ravel()
    probs = np.asarray(probs, dtype=np.float64).ravel()
    keep = probs > 0
    assert np.all(counts[~keep] == 0), "a zero-probability pivot was drawn"
    N = counts.sum()
    c = counts[keep]
    exp = N * probs[keep]
    small = exp < 5          # pool sparse cells into one, as usual for chi-square
    if small.any():
        c = np.append(c[~small], c[small].sum())
        exp = np.append(exp[~small], exp[small].sum())
    stat = float(np.sum((c - exp) ** 2 / exp))
    return float(stats.chi2.sf(stat, len(c) - 1))


def _mixed_6x6(seed=11):
    rng = np.random.default_rng(seed)
    mag = rng.uniform(0.5, 2.0, (6, 6))
    sgn = rng.choice([-1.0, 1.0], (6, 6))
    return mag * sgn


# --------------------------------------------------------------------- pins

def pin_philox_numpy():
    """Philox4x64-10 equals numpy.random.Philox (a library implementation of
    the same published generator) word for word."""
    cases = [(0, 0, 0), (0, 0, 1), (0, 3, 0), (7, 0, 5), (2**63 + 5, 2**40 + 1, 123456),
             (12345, 4095, 511), (1, 2**64 - 1, 2**64 - 1)]
    for seed, stream, t in cases:
        mine = list(PH.philox4x64_10((t, stream, 0, 0), (seed, 0)))
        ref = _numpy_philox_block(seed, stream, t)
        assert mine == ref, (seed, stream, t, mine, ref)
        u1, u2 = PH.step_uniforms(seed, stream, t)
        assert u1 == (ref[0] >> 11) / 2.0**53 and u2 == (ref[1] >> 11) / 2.0**53


def pin_inverse_cdf_bruteforce():
    """First prefix strictly above u*T, brute force on tiny vectors with
    zero-weight runs, targets exactly on edges, u = 0 and u = 1 - 2^-53."""
    rng = np.random.default_rng(3)
    # power-of-two weights make every prefix exact, so edges can be hit exactly
    for trial in range(300):
        n = int(rng.integers(1, 9))
        w = np.where(rng.random(n) < 0.35, 0.0, 2.0 ** rng.integers(-3, 4, n))
        if w.sum() == 0:
            w[int(rng.integers(0, n))] = 1.0
        P = np.cumsum(w)
        T = P[-1]
        us = [0.0, 1.0 - 2.0**-53] + [float(v) / T for v in P[:-1] if v < T] + list(rng.random(4))
        for u in us:
            d = O.inverse_cdf(w, u)
            target = u * T
            brute = next(idx for idx in range(n) if P[idx] > target)
            assert d.drawn == brute, (w, u, d.drawn, brute)
            assert w[d.drawn] > 0, "zero-weight bin selected"
            assert d.total == T and d.target == target
            assert d.lo <= d.target < d.hi


def pin_chi2_first_pivot(N=40000):
    """First pivots over N independent streams follow |a_ij|^2/||A||_F^2
    (Sec. 1, the RPLU distribution): chi-square on 36 cells, p > 1e-3."""
    A = _mixed_6x6()
    counts = np.zeros((6, 6))
    for s in range(N):
        r = O.rplu_dense(A, k=1, seed=9, stream=s)
        counts[tuple(r.piv[0])] += 1
    p = _chi2_pvalue(counts, _p_of(A))
    assert p > 1e-3, p


def pin_chi2_second_pivot(N=40000):
    """With the first pivot forced to (i1, j1), the second pivot follows
    |S_ij|^2/||S||_F^2 of the closed-form one-step Schur complement."""
    A = _mixed_6x6(12)
    i1, j1 = 2, 4
    S1 = A - np.outer(A[:, j1], A[i1, :]) / A[i1, j1]
    S1[i1, :] = 0
    S1[:, j1] = 0
    counts = np.zeros((6, 6))
    for s in range(N):
        r = O.rplu_dense(A, k=2, seed=4, stream=s, forced=[(i1, j1), None])
        counts[tuple(r.piv[1])] += 1
    p = _chi2_pvalue(counts, _p_of(S1))
    assert p > 1e-3, p


def pin_one_step_expectation():
    """E[A^(1) | A] = A - A A^* A / ||A||_F^2 (Sec. 3.1), and when every
    a_ij != 0 the Gram identity E[A^(1)* A^(1)] = 2 A^*A - 2 (A^*A)^2/||A||_F^2
    (eq. G1_bound, equality case), real and complex."""
    rng = np.random.default_rng(5)
    for cplx in (False, True):
        for shape in ((4, 4), (3, 5), (5, 3)):
            A = W.random_dense(*shape, seed=int(rng.integers(1 << 30)), complex_=cplx)
            f2 = float(np.sum(np.abs(A) ** 2))
            E1, G1 = _one_step_moments(A)
            E1_cf = A - A @ A.conj().T @ A / f2
            AhA = A.conj().T @ A
            G1_cf = 2 * AhA - 2 * AhA @ AhA / f2
            assert np.allclose(E1, E1_cf, rtol=0, atol=1e-12 * np.abs(A).max()), cplx
            assert np.allclose(G1, G1_cf, rtol=0, atol=1e-12 * np.abs(AhA).max()), cplx


def pin_unitary_dft():
    """Dense unitary with no zero entry (normalised DFT): E||A^(1)||_F^2 =
    2(n - 1) (Sec. 3.1, the unitary example)."""
    for n in (4, 5, 6, 8):
        F = np.exp(-2j * np.pi * np.outer(np.arange(n), np.arange(n)) / n) / math.sqrt(n)
        E = _enumerate(F, 1)
        assert abs(E[1] - 2 * (n - 1)) <= 1e-12 * n, (n, E[1])


def pin_doubling_enumeration():
    """Exact expected error over all 576 pivot sequences of a 4x4 matrix:
    E||A - A_hat^(k)||_F^2 <= 4^k * sum_{j>k} sigma_j^2 (thm. doubling) for
    k = 1, 2, 3, and the error is exactly 0 at k = 4. The k = 1 value equals
    the trace of the Gram identity, 2||A||^2 - 2||A^*A||_F^2/||A||^2."""
    for seed, cplx in ((21, False), (22, True), (23, False)):
        A = W.random_dense(4, 4, seed=seed, complex_=cplx)
        sig = np.linalg.svd(A, compute_uv=False)
        E = _enumerate(A, 4)
        f2 = float(np.sum(np.abs(A) ** 2))
        AhA = A.conj().T @ A
        assert abs(E[1] - (2 * f2 - 2 * np.sum(np.abs(AhA) ** 2) / f2)) <= 1e-12 * f2
        for k in (1, 2, 3):
            assert E[k] <= 4**k * np.sum(sig[k:] ** 2) * (1 + 1e-12), (k, E[k])
            assert E[k] >= np.sum(sig[k:] ** 2) * (1 - 1e-12), (k, E[k])
        assert E[4] == 0.0, E[4]


def _check_schur_relations(A, res, tol):
    I = [int(v) for v in res.piv[:, 0]]
    J = [int(v) for v in res.piv[:, 1]]
    scale = np.abs(A).max()
    S_cf = O.schur_closed_form(A, I, J) if I else A
    # the closed form via numpy.linalg.solve, written out again here so that
    # this check does not rest on the oracle's own helper
    if I:
        S_np = A - A[:, J] @ np.linalg.solve(A[np.ix_(I, J)], A[I, :])
        assert np.allclose(S_cf, S_np, rtol=0, atol=tol * scale)
    assert np.allclose(res.S, S_cf, rtol=0, atol=tol * scale), np.abs(res.S - S_cf).max()
    LU = res.L @ res.U
    assert np.allclose(LU + res.S, A, rtol=0, atol=tol * scale)
    if I:
        assert np.allclose(LU[I, :], A[I, :], rtol=0, atol=tol * scale)      # interpolation
        assert np.allclose(LU[:, J], A[:, J], rtol=0, atol=tol * scale)
        prod = np.prod(np.array([res.U[t, J[t]] for t in range(len(I))]))
        det = np.linalg.det(A[np.ix_(I, J)])
        assert abs(prod - det) <= 1e-9 * abs(det), (prod, det)
        for t in range(len(I)):
            assert res.L[I[t], t] == 1.0
            for s_ in range(t):
                assert res.L[I[s_], t] == 0.0 and res.U[t, J[s_]] == 0.0


def pin_closed_form_schur():
    """The Schur complement after pivots (I, J) is A - A[:,J] A[I,J]^{-1} A[I,:]
    (depends only on the sets; Sec. 4.1 CUR form), A = LU + S^(k)
    (eqs. residual_update / approximation_update), LU interpolates A on the
    pivot rows and columns, the pivot product equals det A[I,J], and L, U are
    triangular up to the pivot order (Sec. 1, PAQ = LU)."""
    rng = np.random.default_rng(8)
    for trial in range(12):
        n, m = int(rng.integers(3, 12)), int(rng.integers(3, 12))
        cplx = bool(trial % 2)
        A = W.random_dense(n, m, seed=100 + trial, complex_=cplx)
        k = int(rng.integers(1, min(n, m) + 1))
        res = O.rplu_dense(A, k=k, seed=trial, stream=0)
        _check_schur_relations(A, res, 1e-10)
        # and under arbitrary forced pivots
        rows = rng.permutation(n)[:k]
        cols = rng.permutation(m)[:k]
        res2 = O.rplu_dense(A, k=k, forced=list(zip(rows, cols)))
        _check_schur_relations(A, res2, 1e-8)


def pin_exact_recovery():
    """A rank-r matrix is recovered after r steps (the rank-r Schur
    complement is 0 in exact arithmetic, eq. residual_update)."""
    for seed, (n, m, r, cplx) in enumerate(((30, 20, 3, False), (25, 40, 7, True), (64, 64, 10, False))):
        A = W.rank_r_dense(n, m, r, seed=seed, complex_=cplx)
        res = O.rplu_dense(A, k=r, seed=seed)
        rel = math.sqrt(float(np.sum(np.abs(res.S) ** 2)) / float(np.sum(np.abs(A) ** 2)))
        assert rel <= 1e-12, rel
        assert np.allclose(res.L @ res.U, A, rtol=0, atol=1e-11 * np.abs(A).max())


def pin_eckart_young_floor():
    """No rank-k approximation beats the truncated SVD (Sec. 2.2):
    ||S^(k)||_F >= (sum_{j>k} sigma_j^2)^{1/2}, and T = ||S||_F^2."""
    sigma = 0.8 ** np.arange(1, 97)
    A = W.dense_with_spectrum(96, 96, sigma, seed=3)
    for seed in range(4):
        res = O.rplu_dense(A, k=20, seed=seed)
        fro2 = float(np.sum(np.abs(res.S) ** 2))
        assert abs(res.res_fro2 - fro2) <= 1e-13 * fro2
        assert math.sqrt(fro2) >= math.sqrt(np.sum(sigma[20:] ** 2)) * (1 - 1e-12)


def pin_mass_bookkeeping():
    """Row masses and column masses both sum to ||S||_F^2 at every step, and
    the row masses of a step equal the squared row norms of that step's
    Schur complement from the closed form."""
    A = W.random_dense(17, 23, seed=5, complex_=True)
    res = O.rplu_dense(A, k=8, seed=1, keep_masses=True)
    for t, rm in enumerate(res.masses):
        I = [int(v) for v in res.piv[:t, 0]]
        J = [int(v) for v in res.piv[:t, 1]]
        S = O.schur_closed_form(A, I, J)
        w = np.abs(S) ** 2
        assert np.allclose(rm, w.sum(axis=1), rtol=1e-10, atol=1e-12 * w.sum())
        assert abs(w.sum(axis=0).sum() - rm.sum()) <= 1e-12 * w.sum()


def pin_stop_rules():
    """Stop test before each draw: tolerance, exhaustion, rank limit."""
    A = W.config1_dense_512()[:128, :128]
    full = O.rplu_dense(A, k=60, seed=2)
    # rel. residual history from the closed form of each prefix of pivots
    fro2 = float(np.sum(A * A))
    hist = []
    for t in range(61):
        I = [int(v) for v in full.piv[:t, 0]]
        J = [int(v) for v in full.piv[:t, 1]]
        hist.append(float(np.sum(O.schur_closed_form(A, I, J) ** 2)))
    tol = math.sqrt(hist[25] / fro2) * 1.0000001
    first = next(t for t in range(61) if hist[t] <= tol * tol * fro2)
    res = O.rplu_dense(A, k=60, tol=tol, seed=2)
    assert res.stop == O.STOP_TOL and res.rank == first, (res.stop, res.rank, first)
    res = O.rplu_dense(A, k=10, tol=1e-30, seed=2)
    assert res.stop == O.STOP_TOL_UNREACHED and res.rank == 10
    res = O.rplu_dense(A, k=10, seed=2)
    assert res.stop == O.STOP_RANK and res.rank == 10
    # exactly representable rank-1 matrix: the Schur complement is exactly 0
    X = np.outer([1.0, 2.0, 4.0, 0.5], [3.0, -1.0, 2.0])
    res = O.rplu_dense(X, k=3)
    assert res.stop == O.STOP_EXHAUSTED and res.rank == 1
    res = O.rplu_dense(np.zeros((3, 4)), k=2)
    assert res.stop == O.STOP_EXHAUSTED and res.rank == 0 and res.a_fro2 == 0.0
    res = O.rplu_dense(W.random_dense(5, 3, seed=1), k=0)
    assert res.rank == 3 and res.stop == O.STOP_EXHAUSTED


def stall_cases():
    """Diagonal inputs whose totals are exact in FP32 and FP64: entries are
    powers of two and a pivot on the diagonal removes exactly its own mass.
    Each case: (diagonal squared, forced pivot order, k, expected stop,
    expected rank)."""
    eps = 2.0 ** -40
    # one unit of mass that is never pivoted; pivots on tiny entries leave T
    # flat: no improvement after t = 0, stall at t = 64
    flat = ([1.0] + [eps] * 71, list(range(1, 72)), 70, O.STOP_STALL, 64)
    # the first pivot removes 4 of 5 (an improvement at t = 1), then flat:
    # stall at t = 65
    late = ([4.0, 1.0] + [eps] * 70, [0] + list(range(2, 72)), 70, O.STOP_STALL, 65)
    # unit masses: T_t = 72 - t keeps improving by more than 1/64 every
    # few steps: no stall, the rank limit ends the run
    unit = ([1.0] * 72, list(range(72)), 70, O.STOP_RANK, 70)
    return [flat, late, unit]


def pin_stall_rule():
    """Stall rule on diagonal inputs with forced pivots (totals exact, see
    stall_cases): the stop step pins the window length, the >= comparison and
    the refresh of the best total."""
    for d2, order, k, stop, rank in stall_cases():
        D = np.diag(np.sqrt(np.array(d2)))
        forced = [(q, q) for q in order[:k]]
        r = O.rplu_dense(D, k=k, seed=1, forced=forced, stall=True)
        assert (r.stop, r.rank) == (stop, rank), (r.stop, r.rank, stop, rank)
        r = O.rplu_dense(D, k=k, seed=1, forced=forced, stall=False)
        assert (r.stop, r.rank) == (O.STOP_RANK, k)
    return True


def pin_nonfinite():
    A = W.random_dense(4, 4, seed=1)
    A[2, 1] = np.nan
    try:
        O.rplu_dense(A, k=2)
    except O.NonFiniteInput:
        return
    raise AssertionError("NaN input was not rejected")


def pin_cauchy_vs_dense():
    """Generator updates (eqs. generator_update_g/_b) reproduce the dense
    Schur complement entrywise under the same pivots, and the Sylvester
    identity X S - S Y = G B holds at every step (eq. cauchy-like-Sylvester);
    free-running, both forms draw the same pivots."""
    for p, (n, m) in ((1, (40, 30)), (2, (25, 45)), (3, (33, 33))):
        x, y, G, B = W.cauchy_like_random(n, m, p, seed=p)
        A = O.cauchy_entries(x, y, G, B)
        rc = O.rplu_cauchy(x, y, G, B, k=12, seed=p)
        rd = O.rplu_dense(A, k=12, seed=p)
        assert np.array_equal(rc.piv, rd.piv), (rc.piv, rd.piv)
        scale = np.abs(A).max()
        # L(:,t) = c/a_t: compare the columns c = L(:,t) a_t of S^(t), since
        # late pivots a_t are small and the division amplifies rounding
        a_t = np.array([rd.U[t, rd.piv[t, 1]] for t in range(rd.rank)])
        assert np.allclose(rc.L * a_t, rd.L * a_t, rtol=0, atol=1e-12 * scale)
        assert np.allclose(rc.U, rd.U, rtol=0, atol=1e-12 * scale)
        S_gen = O.cauchy_entries(x, y, rc.G, rc.B)
        assert np.allclose(S_gen, rd.S, rtol=0, atol=1e-12 * scale)
        # Sylvester identity at every step, with the dense oracle's S^(t)
        Gt, Bt = G.astype(np.complex128).copy(), B.astype(np.complex128).copy()
        S = A.copy()
        gb0 = np.abs(Gt @ Bt).max()        # rounding scales with the input
        for t in range(rc.rank):
            i, j = (int(v) for v in rc.piv[t])
            O.cauchy_generator_update(x, y, Gt, Bt, i, j)
            O.schur_update(S, i, j)
            lhs = x[:, None] * S - S * y[None, :]
            assert np.allclose(lhs, Gt @ Bt, rtol=0, atol=1e-12 * gb0)


def pin_cauchy_determinant():
    """For a pure Cauchy matrix (G = B = 1), the pivot product equals the
    Cauchy determinant of A[I, J] (textbook closed form)."""
    x, y, G, B = W.cauchy_like_random(30, 26, 1, seed=7)
    G = np.ones_like(G)
    B = np.ones_like(B)
    res = O.rplu_cauchy(x, y, G, B, k=9, seed=3)
    I = [int(v) for v in res.piv[:, 0]]
    J = [int(v) for v in res.piv[:, 1]]
    xi, yj = x[I], y[J]
    num = 1.0 + 0j
    for a, b in itertools.combinations(range(len(I)), 2):
        num *= (xi[b] - xi[a]) * (yj[a] - yj[b])
    den = np.prod(xi[:, None] - yj[None, :])
    det = num / den
    prod = np.prod([res.U[t, J[t]] for t in range(len(I))])
    assert abs(prod - det) <= 1e-12 * len(I) * abs(det), (prod, det)


def pin_loewner_entries():
    """With Loewner generators (eq. loewner-generators), regenerated entries
    equal (f^x_i - f^y_j)/(x_i - y_j) (eq. aaa-loewner)."""
    rng = np.random.default_rng(4)
    x = rng.uniform(-1, 1, 50).astype(np.complex128)
    y = rng.uniform(-1, 1, 40).astype(np.complex128) + 1e-3j
    fx, fy = np.sin(10 * x), np.sin(10 * y)
    G, B = W.loewner_generators(fx, fy)
    A = O.cauchy_entries(x, y, G, B)
    ref = (fx[:, None] - fy[None, :]) / (x[:, None] - y[None, :])
    assert np.allclose(A, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
    row = O.cauchy_row(x, y, G, B, 7)
    col = O.cauchy_col(x, y, G, B, 5)
    assert np.allclose(row, ref[7], rtol=1e-13, atol=0) and np.allclose(col, ref[:, 5], rtol=1e-13, atol=0)
    rm = O.cauchy_row_masses(x, y, G, B, rows_per_block=7)
    assert np.allclose(rm, np.sum(np.abs(ref) ** 2, axis=1), rtol=1e-12)


def pin_c2plu():
    """C2PLU (Sec. 2.3.3): on diag(d) with distinct |d_i| the pivots are the
    diagonal in decreasing |d_i| and S ends exactly 0; on a rank-one u v^T
    the first pivot is (argmax |u_i|, argmax |v_j|) and one step leaves S ~ 0;
    equal masses go to the smallest index; the first row is a row of largest
    2-norm (numpy.linalg.norm) and the first column the largest |A_ij| in it;
    the Schur relations hold as for RPLU; the Cauchy-like form makes the same
    choices as the dense form on its entries."""
    d = np.array([3.0, -5.0, 1.0, 4.0])
    r = O.rplu_dense(np.diag(d), greedy=True)
    assert [tuple(int(v) for v in p_) for p_ in r.piv] == [(1, 1), (3, 3), (0, 0), (2, 2)]
    assert r.stop == O.STOP_EXHAUSTED and np.all(r.S == 0.0)
    u = np.array([1.0, -3.0, 2.0])
    v = np.array([0.5, 4.0, -1.0, 2.0])
    r = O.rplu_dense(np.outer(u, v), k=1, greedy=True)
    assert tuple(int(x) for x in r.piv[0]) == (1, 1)
    assert np.abs(r.S).max() <= 1e-15 * np.abs(np.outer(u, v)).max()
    r = O.rplu_dense(np.array([[1.0, 1.0], [1.0, -1.0]]), k=1, greedy=True)
    assert tuple(int(x) for x in r.piv[0]) == (0, 0)
    rng = np.random.default_rng(31)
    for trial in range(8):
        n, m = int(rng.integers(3, 12)), int(rng.integers(3, 12))
        A = W.random_dense(n, m, seed=300 + trial, complex_=bool(trial % 2))
        k = int(rng.integers(1, min(n, m) + 1))
        res = O.rplu_dense(A, k=k, greedy=True)
        i0 = int(np.argmax(np.linalg.norm(A, axis=1)))
        assert int(res.piv[0, 0]) == i0
        assert int(res.piv[0, 1]) == int(np.argmax(np.abs(A[i0, :])))
        _check_schur_relations(A, res, 1e-10)
    for p_, (n, m) in ((1, (30, 24)), (2, (21, 35))):
        x, y, G, B = W.cauchy_like_random(n, m, p_, seed=40 + p_)
        A = O.cauchy_entries(x, y, G, B)
        rc = O.rplu_cauchy(x, y, G, B, k=10, greedy=True)
        rd = O.rplu_dense(A, k=10, greedy=True)
        assert np.array_equal(rc.piv, rd.piv), (rc.piv, rd.piv)
        assert np.allclose(rc.U, rd.U, rtol=0, atol=1e-12 * np.abs(A).max())


def _first_largest_bruteforce(S):
    """The first row-major (i, j) of largest |S_ij|^2, by explicit loops."""
    best, bi, bj = -1.0, -1, -1
    for i in range(S.shape[0]):
        for j in range(S.shape[1]):
            z = complex(S[i, j])
            v = z.real * z.real + z.imag * z.imag
            if v > best:
                best, bi, bj = v, i, j
    return bi, bj


def pin_cplu():
    """CPLU (complete pivoting, Sec. 1): on diag(d) the pivots are the
    diagonal in decreasing |d_i| and S ends exactly 0; where the largest
    entry is not in the row of largest norm CPLU and C2PLU differ; on a
    rank-one u v^T with dyadic entries the pivot is (argmax |u_i|,
    argmax |v_j|) and one step leaves S exactly 0; ties go to the first entry
    in row-major order, not column-major ([[1, 2], [2, 0]]) nor the last
    (Sylvester-Hadamard 8 x 8: (0,0) then (1,1), |a| = 1 then 2); at every
    step of random real and complex runs the pivot is the first largest
    entry found by explicit loops and |a_t| <= 2 |a_(t-1)| (an entry of the
    next Schur complement is at most twice the largest one); the Schur
    relations hold as for RPLU; the Cauchy-like form makes the dense form's
    choices, also for equal entries in different row blocks."""
    d = np.array([3.0, -5.0, 1.0, 4.0])
    r = O.rplu_dense(np.diag(d), complete=True)
    assert [tuple(int(v) for v in p_) for p_ in r.piv] == [(1, 1), (3, 3), (0, 0), (2, 2)]
    assert r.stop == O.STOP_EXHAUSTED and np.all(r.S == 0.0)
    A = np.array([[3.0, 0.0, 0.0], [2.0, 2.0, 2.0]])
    assert tuple(int(v) for v in O.rplu_dense(A, k=1, complete=True).piv[0]) == (0, 0)
    assert tuple(int(v) for v in O.rplu_dense(A, k=1, greedy=True).piv[0]) == (1, 0)
    u = np.array([1.0, 2.0, -4.0, 3.0])
    v = np.array([2.0, -1.0, 5.0])
    r = O.rplu_dense(np.outer(u, v), complete=True)
    assert r.rank == 1 and tuple(int(x) for x in r.piv[0]) == (2, 2)
    assert r.stop == O.STOP_EXHAUSTED and np.all(r.S == 0.0)
    r = O.rplu_dense(np.array([[1.0, 2.0], [2.0, 0.0]]), k=1, complete=True)
    assert tuple(int(x) for x in r.piv[0]) == (0, 1)
    H = np.array([[(-1.0) ** bin(i & j).count("1") for j in range(8)] for i in range(8)])
    r = O.rplu_dense(H, k=2, complete=True)
    assert [tuple(int(x) for x in p_) for p_ in r.piv] == [(0, 0), (1, 1)]
    assert abs(r.U[0, 0]) == 1.0 and abs(r.U[1, 1]) == 2.0
    rng = np.random.default_rng(37)
    for trial in range(8):
        n, m = int(rng.integers(3, 12)), int(rng.integers(3, 12))
        A = W.random_dense(n, m, seed=500 + trial, complex_=bool(trial % 2))
        if trial == 2:
            A = np.round(A * 2.0)                # small integers: many equal moduli
        k = int(rng.integers(1, min(n, m) + 1))
        res = O.rplu_dense(A, k=k, complete=True)
        S = np.array(A, dtype=np.complex128 if np.iscomplexobj(A) else np.float64)
        prev = None
        for t in range(res.rank):
            assert tuple(int(x) for x in res.piv[t]) == _first_largest_bruteforce(S), (trial, t)
            i, j = (int(x) for x in res.piv[t])
            a = abs(S[i, j])
            assert prev is None or a <= 2.0 * prev * (1 + 1e-12)
            prev = a
            O.schur_update(S, i, j)
        _check_schur_relations(A, res, 1e-10)
    for p_, (n, m) in ((1, (30, 24)), (2, (21, 35))):
        x, y, G, B = W.cauchy_like_random(n, m, p_, seed=60 + p_)
        A = O.cauchy_entries(x, y, G, B)
        rc = O.rplu_cauchy(x, y, G, B, k=10, complete=True)
        rd = O.rplu_dense(A, k=10, complete=True)
        assert np.array_equal(rc.piv, rd.piv), (rc.piv, rd.piv)
        assert np.allclose(rc.U, rd.U, rtol=0, atol=1e-12 * np.abs(A).max())
    # equal largest entries in different row blocks: rows 0 and 2 repeat
    x = np.array([1.0, 2.0, 1.0, 2.0, 3.0], dtype=np.complex128)
    y = np.array([0.0, -1.0], dtype=np.complex128)
    G = np.ones((5, 1), dtype=np.complex128)
    B = np.ones((1, 2), dtype=np.complex128)
    assert O.cauchy_largest_entry(x, y, G, B, rows_per_block=2) == (0, 0)
    assert O.cauchy_largest_entry(x, y, G, B, rows_per_block=1) == (0, 0)


def pin_cur_form():
    """RPLU in CUR form (Alg. 2): at every step of real and complex runs the
    core U_k equals numpy.linalg.inv(A[I, J]) and the updated row norms equal
    the row norms of the closed-form Schur complement
    A - A[:, J] A[I, J]^{-1} A[I, :] (1e-12 of ||A||^2); the pivots are the
    dense Alg. 1's for the same seed and stream (the same two-stage
    distribution), also for C2PLU; a rank-r input is reproduced by
    A[:, J] U_r A[I, :] after r steps; a tolerance run stops where the dense
    form does; A is not written; eq. block-inverse-update grows W^{-1} as the
    library inverse does."""
    for trial, cplx in enumerate((False, True, False, True)):
        n, m = (37, 29) if trial < 2 else (23, 41)
        A = W.random_dense(n, m, seed=600 + trial, complex_=cplx)
        A0 = A.copy()
        kk = min(n, m) - 3
        r = O.rplu_cur(A, k=kk, seed=trial, stream=5)
        assert np.array_equal(A, A0)
        d = O.rplu_dense(A, k=kk, seed=trial, stream=5)
        assert np.array_equal(r.piv, d.piv), trial
        for t in (1, 2, kk // 2, kk):
            rt = O.rplu_cur(A, k=t, seed=trial, stream=5)
            W_ = A[np.ix_(rt.I, rt.J)]
            Winv = np.linalg.inv(W_)
            assert np.abs(rt.Uc - Winv).max() <= 1e-10 * np.abs(Winv).max() * np.linalg.cond(W_)
            S = O.schur_closed_form(A, rt.I, rt.J)
            exact = np.sum(np.abs(S) ** 2, axis=1)
            assert np.abs(rt.rownorms - exact).max() <= 1e-12 * r.a_fro2, (trial, t)
            assert np.all(rt.rownorms[rt.I] == 0.0)
        g = O.rplu_cur(A, k=kk, greedy=True)
        assert np.array_equal(g.piv, O.rplu_dense(A, k=kk, greedy=True).piv)
    Ar = W.rank_r_dense(30, 26, 5, seed=7)
    r = O.rplu_cur(Ar, k=5, seed=2)
    approx = Ar[:, r.J] @ r.Uc @ Ar[r.I, :]
    assert np.abs(approx - Ar).max() <= 1e-12 * np.abs(Ar).max()
    assert r.res_fro2 <= 1e-13 * r.a_fro2          # the downdates cancel to rounding
    Ad = W.dense_with_spectrum(60, 50, 0.6 ** np.arange(50), seed=8)
    rc = O.rplu_cur(Ad, tol=1e-5, seed=4)
    rd = O.rplu_dense(Ad, tol=1e-5, seed=4)
    assert rc.stop == rd.stop == O.STOP_TOL and rc.rank == rd.rank
    assert np.array_equal(rc.piv, rd.piv)
    rng = np.random.default_rng(9)
    M = rng.standard_normal((8, 8))
    U = np.zeros((0, 0))
    for q in range(8):
        U, sig = O.block_inverse_update(U, M[q, :q], M[:q, q], M[q, q])
        assert np.allclose(U, np.linalg.inv(M[:q + 1, :q + 1]), rtol=0, atol=1e-11)


def _bounds_geometries():
    """(name, x, y, G, B) on separated, interleaved and degenerate point sets."""
    from oracle import cauchy_bounds as CB  # noqa: F401
    out = []
    for p_ in (1, 2, 3):
        x, y, G, B = W.cauchy_like_random(300, 260, p_, seed=700 + p_)
        out.append((f"separated p={p_}", x, y, G, B))
    x, y, G, B = W.cauchy_like_random(280, 240, 2, seed=710, separated=False)
    out.append(("near annulus", x, y, G, B))
    x, y = W.spiral_cluster_points(400, 400, seed=2)
    out.append(("spirals vs cluster", x, y, np.ones((400, 1), np.complex128),
                np.ones((1, 400), np.complex128)))
    rng = np.random.default_rng(711)
    z = rng.standard_normal(500) + 1j * rng.standard_normal(500)
    x, y = z[::2], z[1::2] + 1e-3                 # interleaved in one cloud
    G = rng.standard_normal((250, 2)) + 1j * rng.standard_normal((250, 2))
    B = rng.standard_normal((2, 250)) + 1j * rng.standard_normal((2, 250))
    out.append(("interleaved", x, y, G, B))
    x = np.concatenate([np.full(70, 0.25 + 0.5j), rng.random(50) + 1j * rng.random(50)])
    y = 3.0 + rng.random(90) + 1j * rng.random(90)
    G = rng.standard_normal((120, 1)) + 0j
    B = rng.standard_normal((1, 90)) + 0j
    out.append(("repeated targets", x, y, G, B))
    return out


def pin_cauchy_bounds():
    """Certified row-norm bounds (App. C, Alg. C.1 and C.2): on separated,
    interleaved, spiral-vs-cluster and repeated-point geometries, every
    u_i lies between the exact row mass (brute force) and nu times it; the
    source points reached from every target leaf through A_l and E_l are all
    m points, each once; every aggregated pair is admissible over its actual
    points and alpha is at least 1 / (smallest squared distance); leaves hold
    at most `leaf` points (or identical points) and the leaves of each tree
    partition its points; every H_s equals B[:, s] B[:, s]^* (library
    product)."""
    from oracle import cauchy_bounds as CB
    nu, leaf = 5.0, 16
    for name, x, y, G, B in _bounds_geometries():
        plan = CB.interaction_lists(x, y, nu, leaf)
        u = CB.row_norm_bounds(plan, x, y, G, B)
        ex = O.cauchy_row_masses(x, y, G, B)
        assert np.all(ex <= u * (1 + 1e-12)), name
        assert np.all(u <= nu * ex * (1 + 1e-12)), name
        m = y.shape[0]
        for l in plan.tgt_leaves:
            cover = np.concatenate([plan.src[s].idx for s, _ in plan.A[l]] +
                                   [plan.src[s].idx for s in plan.E[l]])
            assert np.array_equal(np.sort(cover), np.arange(m)), (name, l)
            xl = x[plan.tgt[l].idx]
            for s, alpha in plan.A[l]:
                d2 = np.abs(xl[:, None] - y[None, plan.src[s].idx]) ** 2
                assert d2.max() <= nu * d2.min() * (1 + 1e-12), (name, l, s)
                assert alpha * d2.min() >= 1 - 1e-12
        for tree, pts in ((plan.tgt, x), (plan.src, y)):
            leaves = CB.leaves_under(tree, 0)
            allidx = np.concatenate([tree[l].idx for l in leaves])
            assert np.array_equal(np.sort(allidx), np.arange(pts.shape[0]))
            for l in leaves:
                q = pts[tree[l].idx]
                assert len(q) <= leaf or np.all(q == q[0]), name
        H = CB.gram_matrices(plan.src, B)
        for s, nd in enumerate(plan.src):
            Bs = B[:, nd.idx]
            assert np.allclose(H[s], Bs @ Bs.conj().T, rtol=1e-12, atol=1e-12 * np.abs(Bs).max() ** 2)


def _bounds_chi2_case():
    """A 10 x 96 Cauchy-like problem whose bounds are far from proportional
    to the masses (u_i / ||S_i,:||^2 from 1.0 to 3.8 with leaf size 4):
    targets on a segment, sources in a square cluster beside its middle."""
    rng = np.random.default_rng(720)
    x = np.linspace(0, 3, 10) + 0.05j * rng.random(10)
    y = 1.5 + 0.8j + 0.6 * (rng.random(96) - 0.5) + 0.6j * (rng.random(96) - 0.5)
    G = rng.standard_normal((10, 2)) + 1j * rng.standard_normal((10, 2))
    B = rng.standard_normal((2, 96)) + 1j * rng.standard_normal((2, 96))
    return x, y, G, B


def pin_rejection_sampling(N=20000):
    """Alg. 3, Step 1 with the bounds: over N streams the accepted first row
    follows the exact row masses (chi-square p > 1e-3) and not the bounds
    (p < 1e-6); the mean number of trials is sum(u) / sum(rho) within 5
    standard errors; with leaves holding every point (no aggregation) the
    bounds are the exact masses, every step accepts its first trial and the
    run takes the exact form's pivots; a tolerance run stops at TOL with the
    exact residual within the tolerance."""
    from oracle import cauchy_bounds as CB
    x, y, G, B = _bounds_chi2_case()
    plan = CB.interaction_lists(x, y, 5.0, 4)
    u = CB.row_norm_bounds(plan, x, y, G, B)
    ex = O.cauchy_row_masses(x, y, G, B)
    assert (u / ex).max() / (u / ex).min() > 1.3
    counts = np.zeros(10)
    trials = []
    for s in range(N):
        d, q = O._rejection_row(x, y, G, B, u, 0, s, 0)
        counts[d.used] += 1
        trials.append(q)
    assert _chi2_pvalue(counts, ex / ex.sum()) > 1e-3
    assert _chi2_pvalue(counts, u / u.sum()) < 1e-6
    mean_q = u.sum() / ex.sum()
    se = np.std(trials) / np.sqrt(N)
    assert abs(np.mean(trials) - mean_q) <= 5 * se + 1e-9, (np.mean(trials), mean_q)
    xs, ys, Gs, Bs = W.cauchy_like_random(60, 50, 2, seed=721)
    r_all = O.rplu_cauchy(xs, ys, Gs, Bs, k=12, seed=3, bounds=(5.0, 1000))
    r_ex = O.rplu_cauchy(xs, ys, Gs, Bs, k=12, seed=3)
    assert r_all.trials == [1] * 12 and np.array_equal(r_all.piv, r_ex.piv)
    r = O.rplu_cauchy(xs, ys, Gs, Bs, tol=1e-6, seed=4, bounds=(5.0, 8))
    assert r.stop == O.STOP_TOL
    A = O.cauchy_entries(xs, ys, Gs, Bs)
    S = O.schur_closed_form(A, r.piv[:, 0], r.piv[:, 1])
    assert np.linalg.norm(S) <= 1e-6 * np.linalg.norm(A)


def _bary_poles(t, w):
    """Poles of the barycentric form with support t and weights w: the finite
    eigenvalues of the (k+1) x (k+1) arrowhead pencil (scipy.linalg.eig)."""
    import scipy.linalg as sl
    k = len(t)
    E = np.zeros((k + 1, k + 1), dtype=np.complex128)
    E[0, 1:] = w
    E[1:, 0] = 1.0
    E[1:, 1:] = np.diag(t)
    Bm = np.eye(k + 1)
    Bm[0, 0] = 0.0
    ev = sl.eig(E, Bm, right=False)
    return ev[np.isfinite(ev)]


def pin_cur_aaa():
    """CUR-AAA (Alg. 4) on 3000 samples in the unit disk: for f = tan(2z)
    the interpolant's poles include +-pi/4, for f = tan(2z^2) the four
    points +-sqrt(pi/4), +-i sqrt(pi/4), each within 1e-10; the error is
    below 1e-7 on the samples and on a hold-out circle of radius 0.95; r
    equals f at the support points; the Loewner matrix of eq. Laaa times
    the weights is below 1e-8 of its norm (eq. linearization-aaa); the run
    stops on the tolerance within 30 steps (ranks 9 and 18); the split
    has ceil(m/2) and floor(m/2) points, disjoint; the final residual's
    largest row mass (closed form from the dense Loewner matrix) is within
    eps^2 of the initial one (the max-mass stop)."""
    from oracle import cur_aaa as A
    rng = np.random.default_rng(730)
    m = 3000
    z = np.sqrt(rng.random(m)) * np.exp(2j * np.pi * rng.random(m))
    zt = 0.95 * np.exp(2j * np.pi * np.linspace(0, 1, 300))
    r0 = np.sqrt(np.pi / 4)
    for fn, poles in ((lambda q: np.tan(2 * q), [np.pi / 4, -np.pi / 4]),
                      (lambda q: np.tan(2 * q * q), [r0, -r0, 1j * r0, -1j * r0])):
        f = fn(z)
        eps = 1e-11
        r = A.cur_aaa(z, f, eps, seed=3, kmax=60)
        assert r.cur.stop == O.STOP_TOL and r.cur.rank <= 30, (r.cur.stop, r.cur.rank)
        t, w = z[r.support], r.weights
        ev = _bary_poles(t, w)
        for p_ in poles:
            assert np.abs(ev - p_).min() <= 1e-10, (p_, np.abs(ev - p_).min())
        assert r.max_err <= 1e-7
        assert np.abs(A.bary_eval(zt, t, f[r.support], w) - fn(zt)).max() <= 1e-7
        assert np.array_equal(A.bary_eval(t, t, f[r.support], w), f[r.support])
        rest = np.setdiff1d(np.arange(m), r.support)
        Lm = (f[rest, None] - f[r.support][None, :]) / (z[rest, None] - t[None, :])
        assert np.linalg.norm(Lm @ w) <= 1e-8 * np.linalg.norm(Lm, 2)
        X, Y = r.X, r.Y
        assert len(X) == (m + 1) // 2 and len(Y) == m // 2
        assert np.array_equal(np.sort(np.concatenate([X, Y])), np.arange(m))
        Lt = (f[X, None] - f[Y][None, :]) / (z[X, None] - z[Y][None, :])
        S = O.schur_closed_form(Lt, r.cur.piv[:, 0], r.cur.piv[:, 1])
        M0 = np.max(np.sum(np.abs(Lt) ** 2, axis=1))
        assert np.max(np.sum(np.abs(S) ** 2, axis=1)) <= eps * eps * M0 * (1 + 1e-3) + 1e-28 * M0


def pin_factorization_check():
    """The verification's sums of squares: exact integer data checked against
    sums formed term by term in Python integers (tiny sizes, brute force);
    k = 0 (the error is ||A||^2); and after an oracle run the identity
    A - L U = S^(k) (eq. approximation_update): the gap is at rounding level
    and the error equals the run's own ||S||_F^2."""
    rng = np.random.default_rng(21)
    for n, m, k in ((3, 4, 2), (5, 2, 1), (1, 1, 1), (4, 6, 3)):
        L = rng.integers(-3, 4, size=(n, k))
        U = rng.integers(-3, 4, size=(k, m))
        D = rng.integers(-2, 3, size=(n, m))
        A = L @ U + D
        S = rng.integers(-2, 3, size=(n, m))
        a2 = sum(int(A[r, c]) ** 2 for r in range(n) for c in range(m))
        e2 = sum((int(A[r, c]) - sum(int(L[r, q]) * int(U[q, c]) for q in range(k))) ** 2
                 for r in range(n) for c in range(m))
        g2 = sum((int(A[r, c]) - sum(int(L[r, q]) * int(U[q, c]) for q in range(k))
                  - int(S[r, c])) ** 2 for r in range(n) for c in range(m))
        out = O.factorization_check(A.astype(float), L.astype(float), U.astype(float), S.astype(float))
        assert (out["a_fro2"], out["err_fro2"], out["schur_gap_fro2"]) == (a2, e2, g2), (out, a2, e2, g2)
    # complex integers: |z|^2 = re^2 + im^2 term by term
    Lc = np.array([[1 + 2j], [0 - 1j]])
    Uc = np.array([[2 - 1j, 1j, 3]])
    Ac = np.array([[4 + 3j, -2 + 1j, 3 + 6j], [-1 - 2j, 1, 1j]])
    Ec = Ac - Lc @ Uc
    e2c = sum(int(z.real) ** 2 + int(z.imag) ** 2 for z in Ec.ravel())
    a2c = sum(int(z.real) ** 2 + int(z.imag) ** 2 for z in Ac.ravel())
    out = O.factorization_check(Ac, Lc, Uc)
    assert (out["a_fro2"], out["err_fro2"]) == (a2c, e2c) and "schur_gap_fro2" not in out
    # k = 0: nothing approximated
    A0 = rng.standard_normal((6, 5))
    out = O.factorization_check(A0, np.zeros((6, 0)), np.zeros((0, 5)))
    assert out["err_fro2"] == out["a_fro2"] > 0
    # after a run: A - L U is the Schur complement
    for seed, cplx in ((3, False), (4, True)):
        A = W.random_dense(40, 33, seed=seed, complex_=cplx)
        res = O.rplu_dense(A, k=12, seed=seed)
        out = O.factorization_check(A, res.L, res.U, res.S)
        s2 = float(np.sum(np.abs(res.S) ** 2))
        assert out["schur_gap_fro2"] <= 1e-24 * out["a_fro2"], out
        assert abs(out["err_fro2"] - s2) <= 1e-10 * s2, (out, s2)


ALL_PINS = [
    pin_stall_rule,
    pin_philox_numpy, pin_inverse_cdf_bruteforce, pin_chi2_first_pivot,
    pin_chi2_second_pivot, pin_one_step_expectation, pin_unitary_dft,
    pin_doubling_enumeration, pin_closed_form_schur, pin_exact_recovery,
    pin_eckart_young_floor, pin_mass_bookkeeping, pin_stop_rules,
    pin_nonfinite, pin_cauchy_vs_dense, pin_cauchy_determinant,
    pin_loewner_entries, pin_c2plu, pin_cplu, pin_cur_form, pin_cauchy_bounds,
    pin_rejection_sampling, pin_cur_aaa, pin_factorization_check,
]
