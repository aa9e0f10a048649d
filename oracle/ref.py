"""ctypes front end of the C++ FP64 oracle (oracle/rplu_ref.cpp).

TEST INFRASTRUCTURE: only tests, the smoke check and the bench's CPU-baseline
leg use it. It computes what oracle/rplu.py computes (Alg. 1 and Alg. 3 with
exact row masses, C2PLU), with OpenMP over rows for the O(nm) passes, so
that full-size inputs can be replayed and timed on the host cores. The two
oracles are pinned against each other (tests/test_oracle_ref.py).

build() compiles librplu_ref.so next to this file with g++ (-O3, no fused
multiply-add contraction, no fast-math); load() builds it only if it is
missing.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rplu_ref.cpp")
LIB = os.path.join(HERE, "librplu_ref.so")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", "-fopenmp", "-march=x86-64-v3",
         "-ffp-contract=off", "-fno-fast-math", "-Wall"]
TRACE_WORDS = 12

_lib = None


def build() -> str:
    tmp = LIB + ".tmp"
    r = subprocess.run(["g++", *FLAGS, SRC, "-o", tmp], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"oracle build failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        build()
    lib = C.CDLL(LIB)
    P, I64, D = C.c_void_p, C.c_int64, C.c_double
    lib.ref_threads.restype = C.c_int
    lib.ref_philox.argtypes = [C.c_uint64, C.c_uint64, I64, P]
    lib.ref_cauchy_row_masses.argtypes = [I64, I64, C.c_int, P, P, P, P, P]
    lib.ref_rplu_dense.argtypes = [C.c_int, I64, I64, P, I64, D, C.c_uint64, C.c_uint64, C.c_int,
                                   C.c_int, P, P, P, P, P, P, P, P, P, P]
    lib.ref_rplu_dense.restype = C.c_int
    lib.ref_rplu_cauchy.argtypes = [I64, I64, C.c_int, P, P, P, P, I64, D, C.c_uint64, C.c_uint64,
                                    C.c_int, C.c_int, P, P, P, P, P, P, P, P, P, P, P]
    lib.ref_rplu_cauchy.restype = C.c_int
    _lib = lib
    return lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else C.c_void_p(a.ctypes.data)


def threads() -> int:
    return int(load().ref_threads())


def philox(seed: int, stream: int, t: int):
    out = np.zeros(4, dtype=np.uint64)
    load().ref_philox(seed & (2**64 - 1), stream & (2**64 - 1), t, _p(out))
    return tuple(int(v) for v in out)


@dataclass
class RefResult:
    L: np.ndarray        # n x rank
    U: np.ndarray        # rank x m
    piv: np.ndarray      # rank x 2
    rank: int
    stop: int
    a_fro2: float
    res_fro2: float
    trace: Optional[np.ndarray] = None     # rank x 12 (T, u1T, lo, hi, T_i, u2T_i, lo, hi, a.re, a.im, i, j)
    masses: Optional[np.ndarray] = None    # rank x n (steps without masses: zeros)
    S: Optional[np.ndarray] = None
    G: Optional[np.ndarray] = None
    B: Optional[np.ndarray] = None


class OracleError(RuntimeError):
    pass


def _forced_arr(forced, kmax):
    if forced is None:
        return None
    f = np.full(2 * kmax, -1, dtype=np.int32)
    for t, pq in enumerate(forced):
        if t >= kmax:
            break
        if pq is not None:
            f[2 * t], f[2 * t + 1] = int(pq[0]), int(pq[1])
    return f


def rplu_dense(A: np.ndarray, k: int = 0, tol: float = 0.0, seed: int = 0, stream: int = 0,
               forced=None, keep_masses: bool = False, stall: bool = False,
               greedy: bool = False, copy: bool = True) -> RefResult:
    """Alg. 1 (oracle/rplu.py's rplu_dense, same arguments). With copy=False
    a C-contiguous float64/complex128 A is overwritten in place by S."""
    cplx = np.iscomplexobj(A)
    dt = np.complex128 if cplx else np.float64
    S = np.array(A, dtype=dt, copy=True, order="C") if copy else A
    assert S.dtype == dt and S.flags.c_contiguous
    n, m = S.shape
    kmax = min(n, m) if k <= 0 else min(k, n, m)
    L = np.zeros((kmax, n), dtype=dt)
    U = np.zeros((kmax, m), dtype=dt)
    piv = np.full((kmax, 2), -1, dtype=np.int32)
    tr = np.zeros((kmax, TRACE_WORDS))
    rm = np.zeros((kmax, n)) if keep_masses else None
    fa = _forced_arr(forced, kmax)
    rank, stop, T0, T = C.c_int64(), C.c_int32(), C.c_double(), C.c_double()
    st = load().ref_rplu_dense(int(cplx), n, m, _p(S), int(k), float(tol), seed & (2**64 - 1),
                               stream & (2**64 - 1), int(stall), int(greedy), _p(fa), _p(piv),
                               _p(L), _p(U), _p(tr), _p(rm), C.byref(rank), C.byref(stop),
                               C.byref(T0), C.byref(T))
    if st != 0:
        raise OracleError(f"ref_rplu_dense failed: {st}")
    r = rank.value
    return RefResult(L[:r].T.copy(), U[:r].copy(), piv[:r].astype(np.int64), r, stop.value,
                     T0.value, T.value, tr[:r], rm[:r] if rm is not None else None, S=S)


def cauchy_row_masses(x, y, G, B) -> np.ndarray:
    x, y, G, B = (np.ascontiguousarray(v, dtype=np.complex128) for v in (x, y, G, B))
    out = np.empty(x.shape[0])
    load().ref_cauchy_row_masses(x.shape[0], y.shape[0], G.shape[1], _p(x), _p(y), _p(G), _p(B),
                                 _p(out))
    return out


def rplu_cauchy(x, y, G, B, k: int = 0, tol: float = 0.0, seed: int = 0, stream: int = 0,
                forced=None, keep_masses: bool = False, mass_steps=None, stall: bool = False,
                greedy: bool = False) -> RefResult:
    """Alg. 3 with exact row masses (oracle/rplu.py's rplu_cauchy, same
    arguments; mass_steps: the steps at which masses are computed, the rest
    must be forced)."""
    x = np.ascontiguousarray(x, dtype=np.complex128)
    y = np.ascontiguousarray(y, dtype=np.complex128)
    G = np.array(G, dtype=np.complex128, copy=True, order="C")
    B = np.array(B, dtype=np.complex128, copy=True, order="C")
    n, m, p = x.shape[0], y.shape[0], G.shape[1]
    kmax = min(n, m) if k <= 0 else min(k, n, m)
    L = np.zeros((kmax, n), dtype=np.complex128)
    U = np.zeros((kmax, m), dtype=np.complex128)
    piv = np.full((kmax, 2), -1, dtype=np.int32)
    tr = np.zeros((kmax, TRACE_WORDS))
    rm = np.zeros((kmax, n)) if keep_masses else None
    fa = _forced_arr(forced, kmax)
    ms = None
    if mass_steps is not None:
        ms = np.zeros(kmax + 1, dtype=np.uint8)
        for s in mass_steps:
            if 0 <= s <= kmax:
                ms[s] = 1
    rank, stop, T0, T = C.c_int64(), C.c_int32(), C.c_double(), C.c_double()
    st = load().ref_rplu_cauchy(n, m, p, _p(x), _p(y), _p(G), _p(B), int(k), float(tol),
                                seed & (2**64 - 1), stream & (2**64 - 1), int(stall), int(greedy),
                                _p(fa), _p(ms), _p(piv), _p(L), _p(U), _p(tr), _p(rm),
                                C.byref(rank), C.byref(stop), C.byref(T0), C.byref(T))
    if st != 0:
        raise OracleError(f"ref_rplu_cauchy failed: {st}")
    r = rank.value
    return RefResult(L[:r].T.copy(), U[:r].copy(), piv[:r].astype(np.int64), r, stop.value,
                     T0.value, T.value, tr[:r], rm[:r] if rm is not None else None, G=G, B=B)
