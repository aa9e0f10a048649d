"""CUR-AAA (rplu_cur_aaa, Alg. 4) and the max-mass stop rule
(RPLU_FLAG_MAXMASS_STOP) on the GPU against the oracle.

The split is the oracle's (the same Philox keys), the CUR run's pivots are
the oracle's own draws, so the support points are identical; the weights
(the smallest right singular vector, found here by one-sided Jacobi
rotations and in the oracle by LAPACK) agree up to a unit factor, and the
interpolants agree on a hold-out circle; the poles of tan(2z) and
tan(2z^2) are found within 1e-10, as in the oracle's pin. With certified
bounds and with C2PLU the same comparisons hold against the oracle run with
the same options.
"""
import numpy as np
import pytest
import torch

import pins
import workloads as W
from oracle import cur_aaa as A
from oracle import rplu as O

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _samples(m, seed=730):
    rng = np.random.default_rng(seed)
    return np.sqrt(rng.random(m)) * np.exp(2j * np.pi * rng.random(m))


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


R0 = np.sqrt(np.pi / 4)
CASES = {"tan2z": (lambda q: np.tan(2 * q), [np.pi / 4, -np.pi / 4]),
         "tan2z2": (lambda q: np.tan(2 * q * q), [R0, -R0, 1j * R0, -1j * R0])}


def _check(r, o, z, f, fn, poles, tag, err_bar=1e-7):
    sup = r.support.cpu().numpy()
    w = r.weights.cpu().numpy()
    assert (r.rank, r.stop) == (o.cur.rank, o.cur.stop), tag
    assert r.which == o.which and np.array_equal(sup, o.support), tag
    ov = abs(np.vdot(o.weights, w))
    assert ov >= 1 - 1e-8, (tag, ov)
    zt = 0.95 * np.exp(2j * np.pi * np.linspace(0, 1, 300))
    rg = A.bary_eval(zt, z[sup], f[sup], w)
    ro = A.bary_eval(zt, z[sup], f[sup], o.weights)
    assert np.abs(rg - ro).max() <= 1e-9 * np.abs(ro).max(), tag
    assert r.max_err <= err_bar and abs(r.max_err - o.max_err) <= 1e-3 * o.max_err + 1e-13, tag
    ev = pins._bary_poles(z[sup], w)
    for p_ in poles:
        assert np.abs(ev - p_).min() <= 1e-10, (tag, p_)
    print(f"{tag}: k {r.rank}, max error {r.max_err:.2e} (oracle {o.max_err:.2e}), "
          f"which {r.which}, trials {r.trials}", flush=True)


@pytest.mark.parametrize("name", list(CASES))
def test_cur_aaa_matches_oracle(rplu_lib, name):
    fn, poles = CASES[name]
    z = _samples(3000)
    f = fn(z)
    r = rplu_lib.rplu_cur_aaa(_t(z), _t(f), 1e-11, seed=3, max_support=60)
    o = A.cur_aaa(z, f, 1e-11, seed=3, kmax=60)
    _check(r, o, z, f, fn, poles, name)


def test_cur_aaa_bounds_and_c2plu(rplu_lib):
    fn, poles = CASES["tan2z2"]
    z = _samples(20000, seed=731)
    f = fn(z)
    r = rplu_lib.rplu_cur_aaa(_t(z), _t(f), 1e-11, seed=5, max_support=60, bounds=(5.0, 32))
    o = A.cur_aaa(z, f, 1e-11, seed=5, kmax=60, bounds=(5.0, 32))
    _check(r, o, z, f, fn, poles, "bounds, 20000 samples", err_bar=1e-6)
    assert r.trials == sum(o.cur.trials)
    r = rplu_lib.rplu_cur_aaa(_t(z), _t(f), 1e-11, seed=5, max_support=60,
                              flags=rplu_lib.RPLU_FLAG_C2PLU)
    o = A.cur_aaa(z, f, 1e-11, seed=5, kmax=60, greedy=True)
    _check(r, o, z, f, fn, poles, "C2PLU, 20000 samples", err_bar=1e-6)


def test_maxmass_stop_rule(rplu_lib):
    """rplu_cauchy with the max-mass rule stops where the oracle does."""
    x, y, G, B = W.cauchy_like_random(500, 400, 2, seed=36)
    for tol in (1e-2, 1e-4):
        r = rplu_lib.rplu_cauchy(_t(x), _t(y), _t(G), _t(B), k=0, tol=tol, seed=1,
                                 flags=rplu_lib.RPLU_FLAG_MAXMASS_STOP)
        o = O.rplu_cauchy(x, y, G, B, tol=tol, seed=1, maxmass=True)
        assert (r.rank, r.stop) == (o.rank, o.stop) and o.stop == O.STOP_TOL
        assert np.array_equal(r.piv.cpu().numpy(), o.piv)


def test_cur_aaa_argument_errors(rplu_lib):
    z = _t(_samples(100))
    with pytest.raises(rplu_lib.RPLUError) as e:
        rplu_lib.rplu_cur_aaa(z, z, 0.0)
    assert e.value.status == -1
    with pytest.raises(rplu_lib.RPLUError) as e:
        rplu_lib.rplu_cur_aaa(z, z, 1e-8, flags=rplu_lib.RPLU_FLAG_CPLU)
    assert e.value.status == -6
