"""Planted mistakes in the CPU oracle must be caught by its pins.

Each case monkeypatches one oracle routine with a plausible bug (a sign, a
conjugation, a transposed index, a dropped term, an off-by-one edge rule)
and asserts that at least one of the named pins fails.
"""
import numpy as np
import pytest

import pins
from oracle import philox as PH
from oracle import rplu as O

_orig_schur = O.schur_update
_orig_sq = O.squared_magnitude
_orig_gen = O.cauchy_generator_update
_orig_col = O.cauchy_col


def _schur_plus(S, i, j):
    a = S[i, j]
    u = S[i, :].copy()
    l = S[:, j] / a
    l[i] = 1.0
    S += np.outer(l, u)                 # wrong sign
    S[i, :] = 0.0
    S[:, j] = 0.0
    return l, u, a


def _schur_conj(S, i, j):
    a = S[i, j]
    u = S[i, :].conj().copy()           # U conjugated
    l = S[:, j] / a
    l[i] = 1.0
    S -= np.outer(l, u)
    S[i, :] = 0.0
    S[:, j] = 0.0
    return l, u, a


def _schur_noscale(S, i, j):
    a = S[i, j]
    u = S[i, :].copy()
    l = S[:, j].copy()                  # dropped 1/a
    l[i] = 1.0
    S -= np.outer(l, u)
    S[i, :] = 0.0
    S[:, j] = 0.0
    return l, u, a


def _schur_nozero(S, i, j):
    a = S[i, j]
    u = S[i, :].copy()
    l = S[:, j] / a
    l[i] = 1.0
    S -= np.outer(l, u)                 # no exact zeroing of row i / column j
    return l, u, a


def _sq_abs(z):
    return np.abs(z)                    # |z| instead of |z|^2


def _sq_real_only(z):
    return np.real(z) ** 2              # drops the imaginary part


def _first_ge(prefix, target):
    idx = int(np.searchsorted(prefix, target, side="left"))   # >= instead of >
    if idx >= prefix.shape[0]:
        raise ValueError
    return idx


def _gen_conj(x, y, G, B, i, j):
    r = O.cauchy_row(x, y, G, B, i)
    a = r[j]
    c = O.cauchy_col(x, y, G, B, j)
    gi = G[i, :].copy()
    bj = B[:, j].copy()
    G -= np.outer(c, gi) / a
    B -= np.outer(bj, r.conj()) / a     # conjugated row in the B update
    G[i, :] = 0.0
    B[:, j] = 0.0
    return c, r, a


def _gen_swap(x, y, G, B, i, j):
    r = O.cauchy_row(x, y, G, B, i)
    a = r[j]
    c = O.cauchy_col(x, y, G, B, j)
    gi = G[i, :].copy()
    bj = B[:, j].copy()
    G -= np.outer(c, gi) / a
    B -= np.outer(bj, r) / np.conj(a)   # wrong pivot in the B update
    G[i, :] = 0.0
    B[:, j] = 0.0
    return c, r, a


def _col_sign(x, y, G, B, j):
    return (G @ B[:, j]) / (y[j] - x)   # flipped denominator


def _philox_no_bump(counter, key):
    c0, c1, c2, c3 = (int(v) & PH.MASK64 for v in counter)
    k0, k1 = (int(v) & PH.MASK64 for v in key)
    for _ in range(10):                 # key never bumped
        p0 = PH.PHILOX_M0 * c0
        p1 = PH.PHILOX_M1 * c2
        c0, c1, c2, c3 = (p1 >> 64) ^ c1 ^ k0, p1 & PH.MASK64, (p0 >> 64) ^ c3 ^ k1, p0 & PH.MASK64
    return c0, c1, c2, c3


def _stop_tol_linear(t, T, T0, kmax, tol, stall_ref=None):
    if T == 0.0:
        return O.STOP_EXHAUSTED
    if tol > 0.0 and T <= tol * T0:     # tol instead of tol^2
        return O.STOP_TOL
    if stall_ref is not None:
        if t == 0:
            stall_ref[0], stall_ref[1] = T, 0
        elif T < O.STALL_RATIO * stall_ref[0]:
            stall_ref[0], stall_ref[1] = T, t
        if t - stall_ref[1] >= O.STALL_WINDOW:
            return O.STOP_STALL
    if t == kmax:
        return O.STOP_TOL_UNREACHED if tol > 0.0 else O.STOP_RANK
    return 0


def _stop_stall_late(t, T, T0, kmax, tol, stall_ref=None):
    if T == 0.0:
        return O.STOP_EXHAUSTED
    if tol > 0.0 and T <= (tol * tol) * T0:
        return O.STOP_TOL
    if stall_ref is not None:
        if t == 0:
            stall_ref[0], stall_ref[1] = T, 0
        elif T < O.STALL_RATIO * stall_ref[0]:
            stall_ref[0], stall_ref[1] = T, t
        if t - stall_ref[1] > O.STALL_WINDOW:              # > instead of >=
            return O.STOP_STALL
    if t == kmax:
        return O.STOP_TOL_UNREACHED if tol > 0.0 else O.STOP_RANK
    return 0


def _stop_stall_no_update(t, T, T0, kmax, tol, stall_ref=None):
    if T == 0.0:
        return O.STOP_EXHAUSTED
    if tol > 0.0 and T <= (tol * tol) * T0:
        return O.STOP_TOL
    if stall_ref is not None:
        if t == 0:
            stall_ref[0], stall_ref[1] = T, 0                # best never refreshed
        if t - stall_ref[1] >= O.STALL_WINDOW:
            return O.STOP_STALL
    if t == kmax:
        return O.STOP_TOL_UNREACHED if tol > 0.0 else O.STOP_RANK
    return 0


def _rplu_dense_colstage_from_column(A, k=0, tol=0.0, seed=0, stream=0, forced=None,
                                     keep_masses=False):
    # column stage weighted by column i instead of row i (transposed index)
    S = np.array(A, dtype=np.complex128 if np.iscomplexobj(A) else np.float64, copy=True)
    n, m = S.shape
    kmax = O._kmax(n, m, k)
    L = np.zeros((n, kmax), dtype=S.dtype)
    U = np.zeros((kmax, m), dtype=S.dtype)
    piv = np.full((kmax, 2), -1, dtype=np.int64)
    T0 = None
    t = 0
    while True:
        rowmass = np.sum(O.squared_magnitude(S), axis=1)
        T = float(np.cumsum(rowmass)[-1])
        if t == 0:
            T0 = T
        stop = O._stop_reason(t, T, T0, kmax, tol)
        if stop:
            break
        u1, u2 = O.step_uniforms(seed, stream, t)
        fi, fj = O._forced_at(forced, t)
        i = O.inverse_cdf(rowmass, u1, fi).used
        j = O.inverse_cdf(O.squared_magnitude(S[:, i % m]), u2, fj).used % m
        if S[i, j] == 0:
            j = int(np.argmax(np.abs(S[i])))
        l, u, a = O.schur_update(S, i, j)
        L[:, t], U[t, :], piv[t] = l, u, (i, j)
        t += 1
    return O.RPLUResult(L[:, :t], U[:t], piv[:t], t, stop, T0, T, S=S)


def _largest_last(weights, forced=None):
    w = np.asarray(weights, dtype=np.float64)
    drawn = int(len(w) - 1 - np.argmax(w[::-1]))       # ties to the largest index
    used = drawn if forced is None else int(forced)
    return O.Draw(drawn, used, float(np.sum(w)), float("nan"), float("nan"), float("nan"))


def _largest_min(weights, forced=None):
    w = np.asarray(weights, dtype=np.float64)
    drawn = int(np.argmin(w))                           # smallest instead of largest
    used = drawn if forced is None else int(forced)
    return O.Draw(drawn, used, float(np.sum(w)), float("nan"), float("nan"), float("nan"))


def _entry_ties_last(S, forced=(None, None)):
    Wm = O.squared_magnitude(S)
    flat = Wm.size - 1 - int(np.argmax(Wm.ravel()[::-1]))   # ties to the last entry
    i, j = divmod(flat, Wm.shape[1])
    return O._entry_draws(i, j, float(np.sum(Wm)), forced)


def _entry_col_major(S, forced=(None, None)):
    Wm = O.squared_magnitude(S)
    j, i = np.unravel_index(int(np.argmax(Wm.T)), Wm.T.shape)   # first in column-major order
    return O._entry_draws(int(i), int(j), float(np.sum(Wm)), forced)


def _entry_abs_rowmax_of_norm_row(S, forced=(None, None)):
    Wm = O.squared_magnitude(S)
    i = int(np.argmax(np.sum(Wm, axis=1)))                  # C2PLU's row instead
    return O._entry_draws(i, int(np.argmax(Wm[i])), float(np.sum(Wm)), forced)


def _cauchy_entry_later_block(x, y, G, B, rows_per_block=512):
    n = x.shape[0]
    best, bi, bj = -1.0, -1, -1
    for i0 in range(0, n, rows_per_block):
        i1 = min(n, i0 + rows_per_block)
        Wm = O.squared_magnitude((G[i0:i1] @ B) / (x[i0:i1, None] - y[None, :]))
        r, c = np.unravel_index(int(np.argmax(Wm)), Wm.shape)
        if Wm[r, c] >= best:                                 # a later block wins ties
            best, bi, bj = float(Wm[r, c]), i0 + int(r), int(c)
    return bi, bj


def _cur_norm_plus(A, I, J, Uc, nrm, l, chat):
    g = A @ np.conj(l)
    v = A[:, J] @ (Uc @ g[I]) if I else np.zeros_like(g)
    l2 = float(np.sum(O.squared_magnitude(l)))
    return nrm + 2.0 * np.real((g - v) * np.conj(chat)) + l2 * O.squared_magnitude(chat)


def _cur_norm_no_conj(A, I, J, Uc, nrm, l, chat):
    g = A @ l                                            # Alg. 2 as printed, for complex A
    v = A[:, J] @ (Uc @ g[I]) if I else np.zeros_like(g)
    l2 = float(np.sum(O.squared_magnitude(l)))
    return nrm - 2.0 * np.real((g - v) * np.conj(chat)) + l2 * O.squared_magnitude(chat)


def _cur_norm_no_v(A, I, J, Uc, nrm, l, chat):
    g = A @ np.conj(l)                                   # A l instead of A^(k) l
    l2 = float(np.sum(O.squared_magnitude(l)))
    return nrm - 2.0 * np.real(g * np.conj(chat)) + l2 * O.squared_magnitude(chat)


def _core_sign(Uc, z, w, omega):
    Uw, zU = Uc @ w, z @ Uc
    sigma = omega - zU @ w
    k = Uc.shape[0]
    out = np.empty((k + 1, k + 1), dtype=np.result_type(Uc, z, w, omega))
    out[:k, :k] = Uc + np.outer(Uw, zU) / sigma
    out[:k, k] = Uw / sigma                              # sign of the new column
    out[k, :k] = -zU / sigma
    out[k, k] = 1.0 / sigma
    return out, sigma


from oracle import cauchy_bounds as CB  # noqa: E402


def _lists_alpha_dmax(x, y, nu, leaf):
    plan = _REAL_LISTS(x, y, nu, leaf)
    for l in plan.tgt_leaves:                          # 1 / d_max^2 instead of 1 / d_min^2
        plan.A[l] = [(s_, 1.0 / CB.dmax2(plan.src[s_], plan.tgt[l])) for s_, _ in plan.A[l]]
    return plan


def _lists_unsquared(x, y, nu, leaf):
    plan = _REAL_LISTS(x, y, nu * nu, leaf)            # d_max <= nu d_min, unsquared
    plan.nu = nu
    return plan


def _gram_noconj(src, B):
    B = np.asarray(B, dtype=np.complex128)
    return [B[:, nd.idx] @ B[:, nd.idx].T for nd in src]


def _bounds_no_exact(plan, x, y, G, B):
    u = np.zeros(np.asarray(x).shape[0])
    H = CB.gram_matrices(plan.src, B)
    G = np.asarray(G, dtype=np.complex128)
    for l in plan.tgt_leaves:                          # the E lists left out
        rows = plan.tgt[l].idx
        for s_, alpha in plan.A[l]:
            u[rows] += alpha * np.real(np.einsum("ia,ab,ib->i", G[rows], H[s_], np.conj(G[rows])))
    return u


def _reject_inverted(x, y, G, B, u, seed, stream, t):
    for q in range(CB.MAX_TRIALS):
        v_row, v_acc = PH.trial_uniforms(seed, stream, t, q)
        d = O.inverse_cdf(u, v_row)
        rho = float(np.sum(O.squared_magnitude(O.cauchy_row(x, y, G, B, d.used))))
        if v_acc * u[d.used] >= rho:                   # accepts with 1 - rho / u
            return d, q + 1
    raise ValueError("no row accepted")


def _reject_first(x, y, G, B, u, seed, stream, t):
    v_row, _ = PH.trial_uniforms(seed, stream, t, 0)   # no rejection: rows drawn by the bounds
    return O.inverse_cdf(u, v_row), 1


_REAL_LISTS = CB.interaction_lists

from oracle import cur_aaa as AAA  # noqa: E402


def _weights_largest(z, f, support):
    rest = np.setdiff1d(np.arange(z.shape[0]), support)
    t, ft = z[support], f[support]
    Lm = (f[rest, None] - ft[None, :]) / (z[rest, None] - t[None, :])
    _, s_, Vh = np.linalg.svd(Lm, full_matrices=False)
    return np.conj(Vh[0]), s_                      # the largest singular vector


def _gens_sign(fx, fy):
    G, B = _REAL_GENS(fx, fy)
    B[1] = -B[1]                                   # + f^y / alpha in the second row
    return G, B


def _bary_conj(zs, t, ft, w):
    return _REAL_BARY(zs, t, ft, np.conj(w))


_REAL_CHECK = O.factorization_check


def _check_plus(A, L, U, S=None):
    return _REAL_CHECK(A, -np.asarray(L), U, S)    # A + L U


def _check_transposed(A, L, U, S=None):
    out = _REAL_CHECK(A, L, U, None if S is None else np.asarray(S).T.reshape(np.shape(S)))
    return out                                      # S read in the wrong order


_REAL_GENS = AAA.loewner_gens
_REAL_BARY = AAA.bary_eval

MUTATIONS = [
    ("schur_sign", "schur_update", _schur_plus, [pins.pin_closed_form_schur, pins.pin_one_step_expectation]),
    ("schur_conj_u", "schur_update", _schur_conj, [pins.pin_one_step_expectation, pins.pin_unitary_dft, pins.pin_closed_form_schur]),
    ("schur_no_div", "schur_update", _schur_noscale, [pins.pin_closed_form_schur, pins.pin_exact_recovery]),
    ("schur_no_zeroing", "schur_update", _schur_nozero, [pins.pin_doubling_enumeration, pins.pin_closed_form_schur]),
    ("mass_abs", "squared_magnitude", _sq_abs, [pins.pin_chi2_first_pivot, pins.pin_mass_bookkeeping]),
    ("mass_real_only", "squared_magnitude", _sq_real_only, [pins.pin_mass_bookkeeping]),
    ("cdf_ge_edge", "first_exceeding", _first_ge, [pins.pin_inverse_cdf_bruteforce]),
    ("gen_conj_row", "cauchy_generator_update", _gen_conj, [pins.pin_cauchy_vs_dense]),
    ("gen_conj_pivot", "cauchy_generator_update", _gen_swap, [pins.pin_cauchy_vs_dense]),
    ("col_denominator", "cauchy_col", _col_sign, [pins.pin_cauchy_vs_dense, pins.pin_loewner_entries]),
    ("stop_tol_linear", "_stop_reason", _stop_tol_linear, [pins.pin_stop_rules]),
    ("stall_late", "_stop_reason", _stop_stall_late, [pins.pin_stall_rule]),
    ("stall_no_update", "_stop_reason", _stop_stall_no_update, [pins.pin_stall_rule]),
    ("col_stage_transposed", "rplu_dense", _rplu_dense_colstage_from_column, [pins.pin_chi2_first_pivot, pins.pin_mass_bookkeeping]),
    ("c2plu_ties_last", "largest", _largest_last, [pins.pin_c2plu]),
    ("c2plu_argmin", "largest", _largest_min, [pins.pin_c2plu]),
    ("cplu_ties_last", "largest_entry", _entry_ties_last, [pins.pin_cplu]),
    ("cplu_column_major", "largest_entry", _entry_col_major, [pins.pin_cplu]),
    ("cplu_norm_row", "largest_entry", _entry_abs_rowmax_of_norm_row, [pins.pin_cplu]),
    ("cplu_cauchy_later_block", "cauchy_largest_entry", _cauchy_entry_later_block, [pins.pin_cplu]),
    ("cur_norm_sign", "cur_rownorm_update", _cur_norm_plus, [pins.pin_cur_form]),
    ("cur_norm_no_conj", "cur_rownorm_update", _cur_norm_no_conj, [pins.pin_cur_form]),
    ("cur_norm_no_v", "cur_rownorm_update", _cur_norm_no_v, [pins.pin_cur_form]),
    ("cur_core_sign", "block_inverse_update", _core_sign, [pins.pin_cur_form]),
    ("bounds_alpha_dmax", CB, "interaction_lists", _lists_alpha_dmax, [pins.pin_cauchy_bounds]),
    ("bounds_unsquared", CB, "interaction_lists", _lists_unsquared, [pins.pin_cauchy_bounds]),
    ("bounds_gram_noconj", CB, "gram_matrices", _gram_noconj, [pins.pin_cauchy_bounds]),
    ("bounds_no_exact_lists", CB, "row_norm_bounds", _bounds_no_exact, [pins.pin_cauchy_bounds]),
    ("reject_inverted", "_rejection_row", _reject_inverted, [pins.pin_rejection_sampling]),
    ("reject_none", "_rejection_row", _reject_first, [pins.pin_rejection_sampling]),
    ("aaa_largest_vector", AAA, "aaa_weights", _weights_largest, [pins.pin_cur_aaa]),
    ("aaa_generator_sign", AAA, "loewner_gens", _gens_sign, [pins.pin_cur_aaa]),
    ("aaa_conj_weights", AAA, "bary_eval", _bary_conj, [pins.pin_cur_aaa]),
    ("check_sign", "factorization_check", _check_plus, [pins.pin_factorization_check]),
    ("check_schur_order", "factorization_check", _check_transposed, [pins.pin_factorization_check]),
]


def _norm(m):
    """(name, module, attr, impl, catchers); entries without a module patch
    the oracle's rplu module."""
    return m if len(m) == 5 else (m[0], O, m[1], m[2], m[3])


@pytest.mark.parametrize("name,mod,attr,impl,catchers", [_norm(m) for m in MUTATIONS],
                         ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(monkeypatch, name, mod, attr, impl, catchers):
    monkeypatch.setattr(mod, attr, impl)
    caught = []
    for pin in catchers:
        try:
            if pin in (pins.pin_chi2_first_pivot, pins.pin_chi2_second_pivot,
                       pins.pin_rejection_sampling):
                pin(N=8000)
            else:
                pin()
        except (AssertionError, ValueError, IndexError, np.linalg.LinAlgError, O.ZeroPivot):
            caught.append(pin.__name__)
    assert caught, f"mutation {name} slipped past {[p.__name__ for p in catchers]}"


def test_philox_mutation_is_caught(monkeypatch):
    monkeypatch.setattr(PH, "philox4x64_10", _philox_no_bump)
    with pytest.raises(AssertionError):
        pins.pin_philox_numpy()
