"""CUR-AAA (Alg. 4, Sec. 5.3): rational approximation from samples through a
CUR decomposition of a Loewner matrix, FP64 / complex128.

TEST INFRASTRUCTURE: part of the CPU oracle. Only tests, the smoke check and
the bench's CPU-baseline leg may import it; the product path never does, and
it shares no code with the HIP path.

Steps, in the order of Alg. 4:
  1. split the samples Z into X (ceil(m/2) points) and Y (the rest) at
     random;
  2. form the generators of the Loewner matrix L_ij = (f(x_i) - f(y_j)) /
     (x_i - y_j) (eq. loewner-generators, with the alpha scaling);
  3. run Alg. 3 on them until the largest row mass is at most eps^2 times
     its initial value (the max-mass stop rule; exact masses, or the
     certified bounds);
  4. for the selected rows I (points of X) and columns J (points of Y) as
     support points in turn: the Loewner matrix of eq. Laaa over the other
     samples, the barycentric weights as its right singular vector of the
     smallest singular value (numpy.linalg.svd), and the largest error
     |f(z) - r(z)| over Z of the barycentric interpolant (eq.
     aaa-barycentric; r(t_j) = f(t_j) at a support point);
  5. return the one of the two with the smaller largest error (I on ties).

Readings (also in the design notes):
  * The random split: point q gets the key w0 of Philox4x64-10 with key
    (seed, 1) and counter (q, 0, 0, 0); the ceil(m/2) points of smallest key
    (ties by index) form X; X and Y keep the sample order. The draws of step
    3 use key (seed, 0) as in every run.
  * A sample equal to a support point takes that point's value.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .philox import philox4x64_10
from . import rplu as O


def split_keys(m: int, seed: int) -> np.ndarray:
    return np.array([philox4x64_10((q, 0, 0, 0), (seed, 1))[0] for q in range(m)],
                    dtype=np.uint64)


def random_split(m: int, seed: int):
    """(X indices, Y indices), each in sample order."""
    keys = split_keys(m, seed)
    order = sorted(range(m), key=lambda q: (int(keys[q]), q))
    h = (m + 1) // 2
    return np.array(sorted(order[:h]), dtype=np.int64), np.array(sorted(order[h:]), dtype=np.int64)


def loewner_gens(fx: np.ndarray, fy: np.ndarray):
    """eq. loewner-generators: G = [f^x / alpha, alpha], B = [alpha; -f^y / alpha],
    alpha = sqrt(max(max |f^x|, max |f^y|))."""
    alpha = math.sqrt(max(float(np.max(np.abs(fx))), float(np.max(np.abs(fy)))))
    G = np.stack([fx / alpha, np.full(fx.shape, alpha, dtype=np.complex128)], axis=1)
    B = np.stack([np.full(fy.shape, alpha, dtype=np.complex128), -fy / alpha], axis=0)
    return G, B


def aaa_weights(z, f, support):
    """Weights for the support points z[support]: the right singular vector of
    the smallest singular value of the Loewner matrix of eq. Laaa over the
    other samples. Returns (w, singular values)."""
    rest = np.setdiff1d(np.arange(z.shape[0]), support)
    t, ft = z[support], f[support]
    Lm = (f[rest, None] - ft[None, :]) / (z[rest, None] - t[None, :])
    _, s, Vh = np.linalg.svd(Lm, full_matrices=False)
    return np.conj(Vh[-1]), s


def bary_eval(zs, t, ft, w):
    """r(z) = sum_j w_j f(t_j) / (z - t_j) / sum_j w_j / (z - t_j) (eq.
    aaa-barycentric); r(t_j) = f(t_j)."""
    zs = np.asarray(zs, dtype=np.complex128)
    out = np.empty(zs.shape, dtype=np.complex128)
    for q, zq in enumerate(zs):
        hit = np.nonzero(zq == t)[0]
        if hit.size:
            out[q] = ft[hit[0]]
            continue
        c = w / (zq - t)
        out[q] = np.sum(c * ft) / np.sum(c)
    return out


@dataclass
class AAAResult:
    support: np.ndarray      # indices into z of the support points
    weights: np.ndarray
    which: int               # 0: the selected rows I (points of X), 1: the columns J
    max_err: float           # max over Z of |f - r|
    errs: tuple              # (max error with I, with J)
    X: np.ndarray
    Y: np.ndarray
    cur: object              # the Alg. 3 run


def cur_aaa(z, f, eps: float, seed: int = 0, stream: int = 0, greedy: bool = False,
            bounds=None, kmax: int = 0) -> AAAResult:
    z = np.asarray(z, dtype=np.complex128)
    f = np.asarray(f, dtype=np.complex128)
    X, Y = random_split(z.shape[0], seed)
    G, B = loewner_gens(f[X], f[Y])
    run = O.rplu_cauchy(z[X], z[Y], G, B, k=kmax, tol=eps, seed=seed, stream=stream,
                        greedy=greedy, bounds=bounds, maxmass=True)
    fits = []
    for sup in (X[run.piv[:, 0]], Y[run.piv[:, 1]]):
        w, _ = aaa_weights(z, f, sup)
        r = bary_eval(z, z[sup], f[sup], w)
        fits.append((sup, w, float(np.max(np.abs(f - r)))))
    which = 0 if fits[0][2] <= fits[1][2] else 1
    sup, w, err = fits[which]
    return AAAResult(sup, w, which, err, (fits[0][2], fits[1][2]), X, Y, run)
