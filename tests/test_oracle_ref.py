"""The C++ oracle (oracle/rplu_ref.cpp) against the numpy oracle and against
textbook facts, on the CPU.

Both oracles follow Alg. 1 / Alg. 3 in the same order; they are written
separately (numpy vectorised reductions vs plain loops, numpy's complex
division vs Smith's), so identical pivot sequences and agreement to 1e-13 on
every input below pin each against the other. Independent of the numpy
oracle: the Philox words against numpy.random.Philox, the final Schur
complement against its closed form A - A[:,J] A[I,J]^-1 A[I,:], and the
Cauchy-like generators against the dense matrix they generate.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import ref as R
from oracle import rplu as O
from pins import _numpy_philox_block


@pytest.fixture(scope="module", autouse=True)
def _built():
    R.build()       # always compile the current source for these tests


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _same_run(r, o, tol=1e-13):
    assert r.rank == o.rank and r.stop == o.stop
    assert np.array_equal(r.piv, o.piv)
    assert abs(r.a_fro2 - o.a_fro2) <= tol * o.a_fro2
    assert abs(r.res_fro2 - o.res_fro2) <= tol * o.a_fro2
    assert _rel(r.U, o.U) <= tol
    a = np.array([o.U[t, o.piv[t, 1]] for t in range(o.rank)])
    if o.rank:
        assert _rel(r.L * a, o.L * a) <= tol      # columns of S^(t)


def test_philox_words_match_numpy():
    for seed, stream, t in [(0, 0, 0), (1, 2, 3), (2**63 + 5, 2**40 + 1, 1023), (7, 0, 2**33)]:
        assert list(R.philox(seed, stream, t)) == _numpy_philox_block(seed, stream, t)


@pytest.mark.parametrize("n,m,cplx", [(1, 1, False), (7, 5, False), (64, 97, True),
                                      (130, 60, False), (200, 200, True)])
@pytest.mark.parametrize("seed", [0, 3])
def test_dense_matches_numpy_oracle(n, m, cplx, seed):
    A = W.random_dense(n, m, seed=n * m + seed, complex_=cplx)
    k = min(n, m, 40)
    o = O.rplu_dense(A, k=k, seed=seed, stream=n, keep_masses=True)
    r = R.rplu_dense(A, k=k, seed=seed, stream=n, keep_masses=True)
    _same_run(r, o)
    assert _rel(r.S, o.S) <= 1e-13 or np.linalg.norm(o.S) <= 1e-13 * math.sqrt(o.a_fro2)
    for t in range(o.rank):
        assert np.allclose(r.masses[t], o.masses[t], rtol=1e-13, atol=1e-15 * o.a_fro2)
        tr = r.trace[t]
        assert tr[2] <= tr[1] < tr[3] and tr[6] <= tr[5] < tr[7]   # targets inside their bins


def test_dense_closed_form_and_tolerance():
    A = W.dense_with_spectrum(120, 90, 0.7 ** np.arange(90), seed=4)
    r = R.rplu_dense(A, tol=1e-6, seed=2)
    o = O.rplu_dense(A, tol=1e-6, seed=2)
    _same_run(r, o)
    assert r.stop == O.STOP_TOL
    S_cf = O.schur_closed_form(A, r.piv[:, 0], r.piv[:, 1])
    assert np.linalg.norm(r.S - S_cf) <= 1e-9 * np.linalg.norm(A)
    assert np.linalg.norm(A - r.L @ r.U - r.S) <= 1e-12 * np.linalg.norm(A)


def test_dense_stall_greedy_forced():
    cases = [dict(k=0, tol=1e-30, stall=True), dict(k=25, greedy=True), dict(k=20)]
    for q, kw in enumerate(cases):
        A = W.random_dense(90, 70, seed=40 + q, complex_=(q == 1))
        o = O.rplu_dense(A, seed=5, **kw)
        r = R.rplu_dense(A, seed=5, **kw)
        _same_run(r, o)
    # forced replay: the other oracle's pivots, own draws still traced
    A = W.random_dense(80, 80, seed=9)
    o = O.rplu_dense(A, k=30, seed=1)
    f = [tuple(p) for p in o.piv[::-1]]
    r = R.rplu_dense(A, k=30, seed=1, forced=f)
    o2 = O.rplu_dense(A, k=30, seed=1, forced=f)
    _same_run(r, o2)
    for t in range(30):      # the same draw targets and bins of the used pivots
        ro, co = o2.trace[t].row, o2.trace[t].col
        want = [ro.total, ro.target, ro.lo, ro.hi, co.total, co.target, co.lo, co.hi]
        assert np.allclose(r.trace[t, :8], want, rtol=1e-13, atol=1e-15 * o2.a_fro2), t


def test_nonfinite_and_zero_forced_pivot():
    A = W.random_dense(10, 10, seed=1)
    A[3, 4] = np.nan
    with pytest.raises(R.OracleError):
        R.rplu_dense(A, k=3)
    A = np.eye(5)
    with pytest.raises(R.OracleError):
        R.rplu_dense(A, k=2, forced=[(0, 1)])


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("n,m", [(40, 30), (150, 211)])
def test_cauchy_matches_numpy_oracle(p, n, m):
    x, y, G, B = W.cauchy_like_random(n, m, p, seed=n + m + p)
    k = min(n, m, 20)
    o = O.rplu_cauchy(x, y, G, B, k=k, seed=p, stream=m, keep_masses=True)
    r = R.rplu_cauchy(x, y, G, B, k=k, seed=p, stream=m, keep_masses=True)
    _same_run(r, o)
    scale = np.abs(O.cauchy_entries(x, y, G, B)).max()
    Sr = O.cauchy_entries(x, y, r.G, r.B)
    So = O.cauchy_entries(x, y, o.G, o.B)
    assert np.abs(Sr - So).max() <= 1e-12 * scale
    for t in range(o.rank):
        assert np.allclose(r.masses[t], o.masses[t], rtol=1e-12, atol=1e-14 * o.a_fro2)


def test_cauchy_generators_reproduce_dense_schur():
    """Under the same pivots the C++ generator updates give the dense
    oracle's Schur complement entrywise (eqs. generator_update_g/_b)."""
    x, y, G, B = W.cauchy_like_random(120, 100, 2, seed=3)
    A = O.cauchy_entries(x, y, G, B)
    r = R.rplu_cauchy(x, y, G, B, k=15, seed=4)
    d = O.rplu_dense(A, k=15, forced=[tuple(p) for p in r.piv])
    assert np.abs(O.cauchy_entries(x, y, r.G, r.B) - d.S).max() <= 1e-12 * np.abs(A).max()


def test_cauchy_mass_steps_and_row_masses():
    x, y, G, B = W.cauchy_like_random(200, 180, 1, seed=8)
    assert np.allclose(R.cauchy_row_masses(x, y, G, B), O.cauchy_row_masses(x, y, G, B),
                       rtol=1e-13)
    full = R.rplu_cauchy(x, y, G, B, k=12, seed=3, keep_masses=True)
    part = R.rplu_cauchy(x, y, G, B, k=12, seed=3, forced=[tuple(p) for p in full.piv],
                         mass_steps={0, 5, 11}, keep_masses=True)
    assert np.array_equal(part.piv, full.piv)
    for t in (0, 5, 11):
        assert np.array_equal(part.masses[t], full.masses[t])
    assert np.array_equal(part.U, full.U)


def test_closed_form_masses_streamed():
    """The streamed closed-form masses equal the row masses of
    schur_closed_form (the textbook Schur complement) and the step-by-step
    oracle's masses, with the pivot row of S^(t) equal to U(t,:)."""
    A = W.random_dense(300, 200, seed=3)
    o = O.rplu_dense(A, k=40, seed=1, keep_masses=True)
    I, J = o.piv[:, 0], o.piv[:, 1]
    res = O.schur_closed_form_masses(lambda a, b: A[a:b], 300, I, J, [0, 1, 7, 39], row_block=64)
    for t, (mass, row) in res.items():
        S_cf = O.schur_closed_form(A, I[:t], J[:t])
        assert np.allclose(mass, np.sum(S_cf ** 2, axis=1), rtol=1e-12, atol=1e-14 * o.a_fro2)
        assert np.allclose(mass, o.masses[t], rtol=1e-10, atol=1e-13 * o.a_fro2)
        assert np.allclose(row, o.U[t], rtol=1e-10, atol=1e-12 * np.abs(A).max())
