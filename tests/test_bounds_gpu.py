"""Certified row-norm bounds and rejection sampling (RPLU_FLAG_BOUNDS,
App. C and Alg. 3, Step 1) on the GPU against the oracle.

The host plan (quadtrees, interaction lists) and the device bounds follow
the oracle's algorithm; the run is compared draw for draw with the oracle's
run with the same seed, nu and leaf size: at every step the bounds agree
within 1e-12 relative (the same terms summed in another order), the accepted
rows and columns are the oracle's (the trial draws and acceptance tests use
the same Philox words), the total number of trials is the oracle's, and the
regenerated rows U(t,:) and final generators agree within 1e-10. Geometries:
separated sets (p = 1..3), an interleaved cloud (pair-by-pair lists),
spirals against a cluster (aggregated lists only), a leaf of 70 identical
targets (more than a wave). Also: the certified tolerance stop (the exact
residual is within the tolerance), the bound-based C2PLU, the 20000 x 20000
spirals at k = 60, steps of more than four trials, argument errors.
"""
import numpy as np
import pytest
import torch

import parity
import pins
import workloads as W
from oracle import rplu as O

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _run(rplu, x, y, G, B, **kw):
    return rplu.rplu_cauchy(_t(x), _t(y), _t(G), _t(B), want_rowmass=True, want_trace=True, **kw)


def _compare(r, o, tag, u_tol=1e-12):
    assert (r.rank, r.stop) == (o.rank, o.stop), (tag, r.rank, o.rank, r.stop, o.stop)
    assert np.array_equal(r.piv.cpu().numpy(), o.piv), tag
    assert r.trials == sum(o.trials), (tag, r.trials, sum(o.trials))
    um = r.rowmass.cpu().numpy()
    for t in range(o.rank):
        d = np.abs(um[t] - o.masses[t]).max() / np.abs(o.masses[t]).max()
        assert d <= u_tol, (tag, t, d)
    if o.rank:
        assert parity.rel(r.U.cpu().numpy(), o.U) <= 1e-10, tag
    print(f"{tag}: rank {r.rank} stop {r.stop}, {r.trials} trials "
          f"({r.trials / max(1, r.rank):.2f} per step)", flush=True)


@pytest.mark.parametrize("case", range(7))
def test_bounds_match_oracle(rplu_lib, case):
    name, x, y, G, B = pins._bounds_geometries()[case]
    for leaf in (8, 32):
        k = min(30, x.shape[0], y.shape[0])
        r = _run(rplu_lib, x, y, G, B, k=k, seed=5, stream=case, bounds=(5.0, leaf))
        o = O.rplu_cauchy(x, y, G, B, k=k, seed=5, stream=case, bounds=(5.0, leaf),
                          keep_masses=True)
        _compare(r, o, f"{name} leaf {leaf}")


def test_bounds_certified_tolerance_stop(rplu_lib):
    x, y, G, B = W.cauchy_like_random(600, 500, 2, seed=33)
    r = _run(rplu_lib, x, y, G, B, k=0, tol=1e-6, seed=2, bounds=(5.0, 16))
    o = O.rplu_cauchy(x, y, G, B, tol=1e-6, seed=2, bounds=(5.0, 16), keep_masses=True)
    _compare(r, o, "tolerance")
    assert r.stop == rplu_lib.RPLU_STOP_TOL
    A = O.cauchy_entries(x, y, G, B)
    piv = r.piv.cpu().numpy()
    S = O.schur_closed_form(A, piv[:, 0], piv[:, 1])
    res = np.linalg.norm(S) / np.linalg.norm(A)
    print(f"tolerance 1e-6: rank {r.rank}, exact residual {res:.2e}", flush=True)
    assert res <= 1e-6


def test_bounds_c2plu(rplu_lib):
    x, y, G, B = W.cauchy_like_random(400, 350, 1, seed=34)
    r = _run(rplu_lib, x, y, G, B, k=25, flags=rplu_lib.RPLU_FLAG_C2PLU, bounds=(5.0, 16))
    o = O.rplu_cauchy(x, y, G, B, k=25, greedy=True, bounds=(5.0, 16), keep_masses=True)
    assert r.trials == 25
    o.trials = [1] * o.rank
    _compare(r, o, "c2plu with bounds")


def test_bounds_config2_spirals(rplu_lib):
    """The 20000 x 20000 spirals-vs-cluster Cauchy matrix, k = 60."""
    x, y, G, B = W.config2_cauchy_spirals()
    r = _run(rplu_lib, x, y, G, B, k=60, seed=0, bounds=(5.0, 32))
    o = O.rplu_cauchy(x, y, G, B, k=60, seed=0, bounds=(5.0, 32), keep_masses=True)
    _compare(r, o, "spirals 20000^2")


def test_bounds_trials_past_the_first_four(rplu_lib):
    """Steps that need more than four trials: the device tests the first four
    trials of a step at once and then goes on one trial at a time. m = 5000
    columns: each of the first four rows is summed in five column slices."""
    x, y, G, B = W.cauchy_like_random(1500, 5000, 1, seed=36)
    r = _run(rplu_lib, x, y, G, B, k=20, seed=7, stream=1, bounds=(50.0, 16))
    o = O.rplu_cauchy(x, y, G, B, k=20, seed=7, stream=1, bounds=(50.0, 16), keep_masses=True)
    assert max(o.trials) > 4, o.trials
    _compare(r, o, "more than four trials")


def test_bounds_argument_errors(rplu_lib):
    x, y, G, B = W.cauchy_like_random(50, 40, 1, seed=35)
    with pytest.raises(rplu_lib.RPLUError) as e:
        _run(rplu_lib, x, y, G, B, k=3, bounds=(5.0, 65))
    assert e.value.status == -1
    with pytest.raises(rplu_lib.RPLUError) as e:
        _run(rplu_lib, x, y, G, B, k=3, bounds=(0.5, 16))
    assert e.value.status == -1
    with pytest.raises(rplu_lib.RPLUError) as e:
        rplu_lib.rplu_cauchy(_t(x), _t(y), _t(G), _t(B), k=3, bounds=(5.0, 16), want_colmass=True)
    assert e.value.status == -6
