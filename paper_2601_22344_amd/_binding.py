"""ctypes binding of librplu.so (the C ABI declared in include/rplu.h).

Argument marshalling only: tensors supply device memory and the current HIP
stream; every step of the method runs in the library's HIP kernels. There is
no fallback: if the library is missing or fails to load, importing this
module raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librplu.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python paper_2601_22344_amd/build.py` "
        "(the RPLU path has no CPU fallback)")
lib = C.CDLL(LIB_PATH)
# the HIP runtime the library links, for copies out of server-owned memory
_hip = C.CDLL("libamdhip64.so.7", mode=C.RTLD_GLOBAL)
_hip.hipMemcpyAsync.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p]
_hip.hipMemcpyAsync.restype = C.c_int
_hip.hipStreamSynchronize.argtypes = [C.c_void_p]
_hip.hipStreamSynchronize.restype = C.c_int


def _hip_check(e: int) -> None:
    if e != 0:
        raise RuntimeError(f"HIP error {e}")

# ------------------------------------------------------------------ constants
RPLU_OK, RPLU_PENDING = 0, 1
RPLU_E_ARG, RPLU_E_NOMEM, RPLU_E_HIP, RPLU_E_NONFINITE = -1, -2, -3, -4
RPLU_E_BUSY, RPLU_E_UNSUPPORTED, RPLU_E_ZERO_PIVOT = -5, -6, -7
RPLU_R32, RPLU_R64, RPLU_C64, RPLU_C128 = 1, 2, 3, 4
RPLU_STOP_RANK, RPLU_STOP_TOL, RPLU_STOP_EXHAUSTED, RPLU_STOP_TOL_UNREACHED = 1, 2, 3, 4
RPLU_STOP_STALL = 5
RPLU_FLAG_COLMASS, RPLU_FLAG_GRAPH, RPLU_FLAG_NO_GRAPH, RPLU_FLAG_STALL_STOP = 1, 2, 4, 8
RPLU_FLAG_SPLIT_SAMPLER = 16
RPLU_FLAG_C2PLU = 32
RPLU_FLAG_REFRESH = 64
RPLU_FLAG_CERTIFY = 128
RPLU_FLAG_KEEP_INPUT = 256
RPLU_FLAG_LAZY_SWEEP = 512
RPLU_FLAG_EAGER_SWEEP = 1024
RPLU_FLAG_CPLU = 2048
RPLU_FLAG_BOUNDS = 4096
RPLU_FLAG_MAXMASS_STOP = 8192
RPLU_E_BOUND = -8
RPLU_CUR_MAX_RANK = 2048
RPLU_LAZY_STEPS = 4
RPLU_MAX_REFRESH = 8
RPLU_REFRESH_DROP2 = 1e-4
RPLU_STOP_REFRESH = 6
RPLU_STALL_WINDOW = 64
RPLU_TRACE_WORDS = 12
RPLU_JOB_DENSE, RPLU_JOB_CAUCHY = 1, 2
RPLU_ORDER_AREA, RPLU_ORDER_CUBE, RPLU_ORDER_GIVEN = 1, 2, 3
RPLU_SERVER_SIMULATE = 1

_DTYPES = {torch.float32: RPLU_R32, torch.float64: RPLU_R64,
           torch.complex64: RPLU_C64, torch.complex128: RPLU_C128}


class rplu_opts(C.Structure):
    _fields_ = [("max_rank", C.c_int64), ("rel_tol", C.c_double), ("seed", C.c_uint64),
                ("stream", C.c_uint64), ("flags", C.c_uint32), ("reserved", C.c_uint32),
                ("forced", C.c_void_p), ("trace", C.c_void_p), ("rowmass_out", C.c_void_p),
                ("colmass_out", C.c_void_p), ("A_orig", C.c_void_p), ("lda_orig", C.c_int64),
                ("bound_nu", C.c_double), ("bound_leaf", C.c_int32), ("reserved2", C.c_uint32)]


class rplu_info(C.Structure):
    _fields_ = [("rank", C.c_int64), ("stop", C.c_int32), ("status", C.c_int32),
                ("a_fro2", C.c_double), ("res_fro2", C.c_double), ("err_fro2", C.c_double),
                ("refreshes", C.c_int32), ("first_refresh", C.c_int32), ("trials", C.c_int64)]


class rplu_aaa_info(C.Structure):
    _fields_ = [("k", C.c_int64), ("rank", C.c_int64), ("trials", C.c_int64),
                ("which", C.c_int32), ("stop", C.c_int32), ("max_err", C.c_double),
                ("err_rows", C.c_double), ("err_cols", C.c_double)]


class rplu_job(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dtype", C.c_int32), ("n", C.c_int64), ("m", C.c_int64),
                ("A", C.c_void_p), ("lda", C.c_int64), ("p", C.c_int32), ("flags", C.c_uint32),
                ("x", C.c_void_p), ("y", C.c_void_p), ("G", C.c_void_p), ("B", C.c_void_p),
                ("piv", C.c_void_p), ("L", C.c_void_p), ("ldl", C.c_int64), ("U", C.c_void_p),
                ("ldu", C.c_int64), ("max_rank", C.c_int64), ("rel_tol", C.c_double),
                ("seed", C.c_uint64), ("stream", C.c_uint64), ("A_orig", C.c_void_p),
                ("lda_orig", C.c_int64), ("ready_event", C.c_void_p)]


class rplu_batch_cfg(C.Structure):
    _fields_ = [("rows_per_pass", C.c_int32), ("wg_per_cu", C.c_int32), ("order", C.c_int32),
                ("reserved", C.c_int32)]


class rplu_verify_out(C.Structure):
    _fields_ = [("a_fro2", C.c_double), ("err_fro2", C.c_double), ("schur_gap_fro2", C.c_double)]


class rplu_server_cfg(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_size_t), ("max_slots", C.c_int32),
                ("queue_capacity", C.c_int32), ("workers", C.c_int32),
                ("batch_max_dim", C.c_int32), ("flags", C.c_uint32), ("tick_steps", C.c_int32)]


class rplu_profile(C.Structure):
    _fields_ = [("launches", C.c_int64 * 4), ("ms", C.c_double * 4)]


class rplu_server_stats_t(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("rejected", C.c_int64),
                ("queued", C.c_int64), ("active", C.c_int64), ("p50_ms", C.c_double),
                ("p99_ms", C.c_double), ("p50_dense_ms", C.c_double),
                ("p99_dense_ms", C.c_double), ("p50_cauchy_ms", C.c_double),
                ("p99_cauchy_ms", C.c_double), ("busy_s", C.c_double),
                ("hbm_in_use", C.c_size_t), ("hbm_peak", C.c_size_t), ("ticks", C.c_int64),
                ("tick_jobs", C.c_int64), ("refreshes", C.c_int64)]


_P = C.c_void_p
_I64 = C.c_int64
lib.rplu_create.argtypes = [C.c_int, C.c_size_t, C.POINTER(_P)]
lib.rplu_destroy.argtypes = [_P]
lib.rplu_dense.argtypes = [_P, C.c_int, _I64, _I64, _P, _I64, C.POINTER(rplu_opts), _P, _P, _I64,
                           _P, _I64, C.POINTER(rplu_info), _P]
lib.rplu_cur.argtypes = [_P, C.c_int, _I64, _I64, _P, _I64, C.POINTER(rplu_opts), _P, _P, _I64,
                         C.POINTER(rplu_info), _P]
lib.rplu_cur_aaa.argtypes = [_P, _I64, _P, _P, C.c_double, C.c_uint64, _I64, C.c_uint32,
                             C.POINTER(rplu_opts), _P, _P, C.POINTER(rplu_aaa_info), _P]
lib.rplu_cauchy.argtypes = [_P, C.c_int, _I64, _I64, C.c_int32, _P, _P, _P, _P,
                            C.POINTER(rplu_opts), _P, _P, _I64, _P, _I64, C.POINTER(rplu_info), _P]
lib.rplu_batched.argtypes = [_P, _I64, C.POINTER(rplu_job), C.POINTER(rplu_info), _P]
lib.rplu_batched_ex.argtypes = [_P, _I64, C.POINTER(rplu_job), C.POINTER(rplu_info),
                                C.POINTER(rplu_batch_cfg), _P]
lib.rplu_batched_tune.argtypes = [_P, _I64, C.POINTER(rplu_job), C.POINTER(rplu_batch_cfg),
                                  C.POINTER(C.c_double), _P]
lib.rplu_verify.argtypes = [_P, C.c_int, _I64, _I64, _I64, _P, _I64, _P, _I64, _P, _I64, _P, _I64,
                            C.POINTER(rplu_verify_out), _P]
lib.rplu_server_create.argtypes = [_P, C.POINTER(rplu_server_cfg), C.POINTER(_P)]
lib.rplu_server_submit.argtypes = [_P, C.POINTER(rplu_job), C.POINTER(C.c_uint64)]
lib.rplu_server_poll.argtypes = [_P, C.c_uint64, C.POINTER(rplu_info)]
lib.rplu_server_stats.argtypes = [_P, C.POINTER(rplu_server_stats_t)]
lib.rplu_server_outputs.argtypes = [_P, C.c_uint64, C.POINTER(_P), C.POINTER(_P),
                                    C.POINTER(_I64), C.POINTER(_P), C.POINTER(_I64)]
lib.rplu_server_release.argtypes = [_P, C.c_uint64]
lib.rplu_server_destroy.argtypes = [_P]
lib.rplu_profile_begin.argtypes = [_P]
lib.rplu_profile_end.argtypes = [_P, C.POINTER(rplu_profile)]
lib.rplu_dense_noalloc.argtypes = [C.c_int, _I64, _I64, _P, _I64, C.POINTER(rplu_opts), _P, _P,
                                   _I64, _P, _I64, C.POINTER(rplu_info), _P]
lib.rplu_dense_noalloc_bytes.argtypes = [C.c_int, _I64, _I64, C.c_uint32, C.c_int]
lib.rplu_dense_noalloc_bytes.restype = C.c_size_t
lib.rplu_status_str.argtypes = [C.c_int32]
lib.rplu_status_str.restype = C.c_char_p
lib.rplu_last_error.restype = C.c_char_p
lib.rplu_last_error.argtypes = []
for _fn in ("rplu_create", "rplu_destroy", "rplu_dense", "rplu_dense_noalloc", "rplu_cauchy",
            "rplu_cur", "rplu_cur_aaa",
            "rplu_batched",
            "rplu_batched_ex", "rplu_batched_tune", "rplu_verify",
            "rplu_server_create", "rplu_server_submit", "rplu_server_poll",
            "rplu_server_stats", "rplu_server_destroy", "rplu_server_outputs",
            "rplu_server_release", "rplu_profile_begin", "rplu_profile_end"):
    getattr(lib, _fn).restype = C.c_int32


class RPLUError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = lib.rplu_last_error().decode(errors="replace")
        super().__init__(f"{where}: {lib.rplu_status_str(status).decode()} ({msg})")


def _check(status: int, where: str) -> int:
    if status < 0:
        raise RPLUError(status, where)
    return status


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _cur_stream(device: torch.device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Context:
    """Owns an rplu_ctx (device workspace) for one device."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        h = C.c_void_p()
        _check(lib.rplu_create(int(device), int(hbm_budget_bytes), C.byref(h)), "rplu_create")
        self.handle = h
        self.device = int(device)

    def close(self):
        if self.handle:
            lib.rplu_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ctx: dict = {}


def rplu_create(device: int = 0, hbm_budget_bytes: int = 0) -> Context:
    return Context(device, hbm_budget_bytes)


def default_context(device: int = 0) -> Context:
    ctx = _default_ctx.get(device)
    if ctx is None:
        ctx = _default_ctx[device] = Context(device)
    return ctx


@dataclass
class Result:
    piv: torch.Tensor              # rank x 2 int32 (device)
    L: Optional[torch.Tensor]      # n x rank (column-major view)
    U: Optional[torch.Tensor]      # rank x m
    rank: int
    stop: int
    a_fro2: float
    res_fro2: float
    trace: Optional[torch.Tensor] = None      # rank x 12 float64
    rowmass: Optional[torch.Tensor] = None    # rank x n float64
    colmass: Optional[torch.Tensor] = None    # rank x m float64
    status: int = 0                           # RPLU_OK or the job's RPLU_E_* code
    refreshes: int = 0                        # residual replacements (RPLU_FLAG_REFRESH)
    first_refresh: int = -1                   # step of the first one, or -1
    err_fro2: float = -1.0                    # certified ||A - L U||^2 (server), or -1
    trials: int = 0                           # rejection trials (RPLU_FLAG_BOUNDS)


def _opts(k, tol, seed, stream, flags, forced, trace, rowmass_out, colmass_out, A_orig=None,
          bound_nu=0.0, bound_leaf=0):
    return rplu_opts(int(k), float(tol), int(seed) & (2**64 - 1), int(stream) & (2**64 - 1),
                     int(flags), 0, _ptr(forced), _ptr(trace), _ptr(rowmass_out),
                     _ptr(colmass_out), _ptr(A_orig),
                     A_orig.stride(0) if A_orig is not None else 0, float(bound_nu),
                     int(bound_leaf), 0)


def rplu_dense(A: torch.Tensor, k: int = 0, tol: float = 0.0, seed: int = 0, stream: int = 0,
               flags: int = 0, forced: Optional[torch.Tensor] = None, want_trace: bool = False,
               want_rowmass: bool = False, want_colmass: bool = False, store_L: bool = True,
               store_U: bool = True, ctx: Optional[Context] = None,
               A_orig: Optional[torch.Tensor] = None) -> Result:
    """Dense RPLU of A (n x m CUDA tensor, row stride >= m, overwritten by the
    final Schur complement). Returns device factors sliced to the rank.
    A_orig: the unmodified input, for RPLU_FLAG_REFRESH (set by default when
    given)."""
    if A_orig is not None:
        if A_orig.shape != A.shape or A_orig.dtype != A.dtype or A_orig.stride(1) != 1:
            raise ValueError("A_orig must have A's shape and dtype, unit column stride")
        flags |= RPLU_FLAG_REFRESH
    if A.dim() != 2 or A.stride(1) != 1 or A.dtype not in _DTYPES or not A.is_cuda:
        raise ValueError("A must be a 2-D CUDA tensor (float32/64, complex64/128), unit column stride")
    n, m = A.shape
    dev = A.device
    ctx = ctx or default_context(dev.index or 0)
    kmax = min(n, m) if k <= 0 else min(k, n, m)
    piv = torch.empty((kmax, 2), dtype=torch.int32, device=dev)
    Lt = torch.empty((kmax, n), dtype=A.dtype, device=dev) if store_L else None
    U = torch.empty((kmax, m), dtype=A.dtype, device=dev) if store_U else None
    trace = torch.empty((kmax, RPLU_TRACE_WORDS), dtype=torch.float64, device=dev) if want_trace else None
    rmo = torch.empty((kmax, n), dtype=torch.float64, device=dev) if want_rowmass else None
    cmo = torch.empty((kmax, m), dtype=torch.float64, device=dev) if want_colmass else None
    if want_colmass:
        flags |= RPLU_FLAG_COLMASS
    if forced is not None:
        forced = forced.to(device=dev, dtype=torch.int32).contiguous()
        if forced.numel() < 2 * kmax:
            raise ValueError("forced needs 2*kmax entries")
    opts = _opts(k, tol, seed, stream, flags, forced, trace, rmo, cmo, A_orig)
    info = rplu_info()
    st = lib.rplu_dense(ctx.handle, _DTYPES[A.dtype], n, m, _ptr(A), A.stride(0), C.byref(opts),
                        _ptr(piv), _ptr(Lt), n, _ptr(U), m, C.byref(info), _cur_stream(dev))
    _check(st, "rplu_dense")
    r = int(info.rank)
    return Result(piv[:r], Lt[:r].T if Lt is not None else None, U[:r] if U is not None else None,
                  r, int(info.stop), float(info.a_fro2), float(info.res_fro2),
                  trace[:r] if trace is not None else None, rmo[:r] if rmo is not None else None,
                  cmo[:r] if cmo is not None else None, refreshes=int(info.refreshes),
                  first_refresh=int(info.first_refresh))


@dataclass
class CURResult:
    """RPLU in CUR form: A ~ A[:, J] Ucore A[I, :] with Ucore = A[I, J]^{-1}."""
    piv: torch.Tensor              # rank x 2 int32 (device): I_t, J_t
    Ucore: torch.Tensor            # rank x rank float64 / complex128 (device)
    rank: int
    stop: int
    a_fro2: float
    res_fro2: float                # sum of the row-norm estimates at the stop test
    trace: Optional[torch.Tensor] = None      # rank x 12 float64
    rowmass: Optional[torch.Tensor] = None    # rank x n float64 (estimates before each draw)

    @property
    def I(self) -> torch.Tensor:   # noqa: E743
        return self.piv[:, 0]

    @property
    def J(self) -> torch.Tensor:
        return self.piv[:, 1]


def rplu_cur(A: torch.Tensor, k: int = 0, tol: float = 0.0, seed: int = 0, stream: int = 0,
             flags: int = 0, forced: Optional[torch.Tensor] = None, want_trace: bool = False,
             want_rowmass: bool = False, ctx: Optional[Context] = None) -> CURResult:
    """RPLU in CUR form (Alg. 2) of A (n x m CUDA tensor, row stride >= m),
    which is only read. Returns the pivot pairs and the core A[I, J]^{-1}."""
    if A.dim() != 2 or A.stride(1) != 1 or A.dtype not in _DTYPES or not A.is_cuda:
        raise ValueError("A must be a 2-D CUDA tensor (float32/64, complex64/128), unit column stride")
    n, m = A.shape
    dev = A.device
    ctx = ctx or default_context(dev.index or 0)
    kmax = min(n, m) if k <= 0 else min(k, n, m)
    cdt = torch.complex128 if A.is_complex() else torch.float64
    piv = torch.empty((kmax, 2), dtype=torch.int32, device=dev)
    Uc = torch.empty((kmax, kmax), dtype=cdt, device=dev)
    trace = torch.empty((kmax, RPLU_TRACE_WORDS), dtype=torch.float64, device=dev) if want_trace else None
    rmo = torch.empty((kmax, n), dtype=torch.float64, device=dev) if want_rowmass else None
    if forced is not None:
        forced = forced.to(device=dev, dtype=torch.int32).contiguous()
        if forced.numel() < 2 * kmax:
            raise ValueError("forced needs 2*kmax entries")
    opts = _opts(k, tol, seed, stream, flags, forced, trace, rmo, None)
    info = rplu_info()
    st = lib.rplu_cur(ctx.handle, _DTYPES[A.dtype], n, m, _ptr(A), A.stride(0), C.byref(opts),
                      _ptr(piv), _ptr(Uc), max(kmax, 1), C.byref(info), _cur_stream(dev))
    _check(st, "rplu_cur")
    r = int(info.rank)
    return CURResult(piv[:r], Uc[:r, :r], r, int(info.stop), float(info.a_fro2),
                     float(info.res_fro2), trace[:r] if trace is not None else None,
                     rmo[:r] if rmo is not None else None)


def rplu_dense_noalloc(A: torch.Tensor, piv: torch.Tensor, L: Optional[torch.Tensor] = None,
                       U: Optional[torch.Tensor] = None, k: int = 0, tol: float = 0.0,
                       seed: int = 0, stream: int = 0, flags: int = 0) -> Result:
    """rplu_dense without a context and without device allocation: the caller
    passes every output (piv: kmax x 2 int32; L: kmax x n, row t = L(:,t);
    U: kmax x m, both of A's dtype, or None). Runs on A's device, on the
    current stream; the library's fixed scratch array holds the step state."""
    if A.dim() != 2 or A.stride(1) != 1 or A.dtype not in _DTYPES or not A.is_cuda:
        raise ValueError("A must be a 2-D CUDA tensor (float32/64, complex64/128), unit column stride")
    n, m = A.shape
    kmax = min(n, m) if k <= 0 else min(k, n, m)
    if piv.dtype != torch.int32 or piv.numel() < 2 * kmax or not piv.is_contiguous():
        raise ValueError("piv must be a contiguous int32 tensor of 2*kmax entries")
    for t_, w in ((L, n), (U, m)):
        if t_ is not None and (t_.dtype != A.dtype or not t_.is_contiguous() or t_.numel() < kmax * w):
            raise ValueError("L (kmax x n) and U (kmax x m) must be contiguous, of A's dtype")
    opts = _opts(k, tol, seed, stream, flags, None, None, None, None)
    info = rplu_info()
    with torch.cuda.device(A.device):
        st = lib.rplu_dense_noalloc(_DTYPES[A.dtype], n, m, _ptr(A), A.stride(0), C.byref(opts),
                                    _ptr(piv), _ptr(L), n, _ptr(U), m, C.byref(info),
                                    _cur_stream(A.device))
    _check(st, "rplu_dense_noalloc")
    r = int(info.rank)
    return Result(piv[:r], L[:r].T if L is not None else None, U[:r] if U is not None else None,
                  r, int(info.stop), float(info.a_fro2), float(info.res_fro2))


def rplu_cauchy(x: torch.Tensor, y: torch.Tensor, G: torch.Tensor, B: torch.Tensor, k: int = 0,
                tol: float = 0.0, seed: int = 0, stream: int = 0, flags: int = 0,
                forced: Optional[torch.Tensor] = None, want_trace: bool = False,
                want_rowmass: bool = False, want_colmass: bool = False, store_L: bool = True,
                store_U: bool = True, ctx: Optional[Context] = None,
                bounds: Optional[tuple] = None) -> Result:
    """Cauchy-like RPLU from nodes x (n), y (m) and generators G (n x p),
    B (p x m), complex128 CUDA tensors; G and B are overwritten by the
    generators of the final Schur complement. bounds = (nu, leaf):
    RPLU_FLAG_BOUNDS (certified row-norm bounds and rejection sampling)."""
    bound_nu, bound_leaf = 0.0, 0
    if bounds is not None:
        flags |= RPLU_FLAG_BOUNDS
        bound_nu, bound_leaf = float(bounds[0]), int(bounds[1])
    for t_ in (x, y, G, B):
        if t_.dtype != torch.complex128 or not t_.is_cuda or not t_.is_contiguous():
            raise ValueError("x, y, G, B must be contiguous complex128 CUDA tensors")
    n, m, p = x.shape[0], y.shape[0], G.shape[1]
    if G.shape != (n, p) or B.shape != (p, m):
        raise ValueError("G must be n x p and B p x m")
    dev = x.device
    ctx = ctx or default_context(dev.index or 0)
    kmax = min(n, m) if k <= 0 else min(k, n, m)
    piv = torch.empty((kmax, 2), dtype=torch.int32, device=dev)
    Lt = torch.empty((kmax, n), dtype=torch.complex128, device=dev) if store_L else None
    U = torch.empty((kmax, m), dtype=torch.complex128, device=dev) if store_U else None
    trace = torch.empty((kmax, RPLU_TRACE_WORDS), dtype=torch.float64, device=dev) if want_trace else None
    rmo = torch.empty((kmax, n), dtype=torch.float64, device=dev) if want_rowmass else None
    cmo = torch.empty((kmax, m), dtype=torch.float64, device=dev) if want_colmass else None
    if want_colmass:
        flags |= RPLU_FLAG_COLMASS
    if forced is not None:
        forced = forced.to(device=dev, dtype=torch.int32).contiguous()
    opts = _opts(k, tol, seed, stream, flags, forced, trace, rmo, cmo, None, bound_nu, bound_leaf)
    info = rplu_info()
    st = lib.rplu_cauchy(ctx.handle, RPLU_C128, n, m, p, _ptr(x), _ptr(y), _ptr(G), _ptr(B),
                         C.byref(opts), _ptr(piv), _ptr(Lt), n, _ptr(U), m, C.byref(info),
                         _cur_stream(dev))
    _check(st, "rplu_cauchy")
    r = int(info.rank)
    return Result(piv[:r], Lt[:r].T if Lt is not None else None, U[:r] if U is not None else None,
                  r, int(info.stop), float(info.a_fro2), float(info.res_fro2),
                  trace[:r] if trace is not None else None, rmo[:r] if rmo is not None else None,
                  cmo[:r] if cmo is not None else None, refreshes=int(info.refreshes),
                  first_refresh=int(info.first_refresh), trials=int(info.trials))


@dataclass
class AAAResult:
    """CUR-AAA: r(z) = sum_j w_j f(t_j) / (z - t_j) / sum_j w_j / (z - t_j)
    with t = z[support]."""
    support: torch.Tensor          # k int32 (device): indices into z
    weights: torch.Tensor          # k complex128 (device)
    which: int                     # 0: rows (points of X), 1: columns (points of Y)
    max_err: float
    err_rows: float
    err_cols: float
    rank: int
    stop: int
    trials: int


def rplu_cur_aaa(z: torch.Tensor, f: torch.Tensor, eps: float, seed: int = 0,
                 max_support: int = 512, flags: int = 0, bounds: Optional[tuple] = None,
                 ctx: Optional[Context] = None) -> AAAResult:
    """CUR-AAA (Alg. 4) on samples z, f (complex128 CUDA vectors)."""
    for t_ in (z, f):
        if t_.dtype != torch.complex128 or not t_.is_cuda or not t_.is_contiguous() or t_.dim() != 1:
            raise ValueError("z and f must be contiguous complex128 CUDA vectors")
    m = z.shape[0]
    dev = z.device
    ctx = ctx or default_context(dev.index or 0)
    ks = min(max_support, m // 2)
    sup = torch.empty(ks, dtype=torch.int32, device=dev)
    w = torch.empty(ks, dtype=torch.complex128, device=dev)
    bo = None
    if bounds is not None:
        flags |= RPLU_FLAG_BOUNDS
        bo = _opts(0, 0.0, 0, 0, 0, None, None, None, None, None, float(bounds[0]), int(bounds[1]))
    info = rplu_aaa_info()
    st = lib.rplu_cur_aaa(ctx.handle, m, _ptr(z), _ptr(f), float(eps), int(seed) & (2**64 - 1),
                          ks, int(flags), C.byref(bo) if bo is not None else None, _ptr(sup),
                          _ptr(w), C.byref(info), _cur_stream(dev))
    _check(st, "rplu_cur_aaa")
    k = int(info.k)
    return AAAResult(sup[:k], w[:k], int(info.which), float(info.max_err), float(info.err_rows),
                     float(info.err_cols), int(info.rank), int(info.stop), int(info.trials))


def rplu_profile_begin(ctx: Context) -> None:
    _check(lib.rplu_profile_begin(ctx.handle), "rplu_profile_begin")


def rplu_profile_end(ctx: Context) -> dict:
    """{'launches': [4 ints], 'ms': [4 floats]}: device time per kernel class
    (0 hot sweep/mass, 1 sampler, 2 update/reduce, 3 initial mass)."""
    out = rplu_profile()
    _check(lib.rplu_profile_end(ctx.handle, C.byref(out)), "rplu_profile_end")
    return {"launches": list(out.launches), "ms": list(out.ms)}


def _per_job(v, count, name):
    if isinstance(v, (list, tuple)):
        if len(v) != count:
            raise ValueError(f"{name}: expected {count} values")
        return list(v)
    return [v] * count


def _batch_jobs(As, k, tol, seed, streams, store_L, store_U, flags=0, A_origs=None):
    count = len(As)
    ks, tols, seeds = _per_job(k, count, "k"), _per_job(tol, count, "tol"), _per_job(seed, count, "seed")
    streams = list(range(count)) if streams is None else _per_job(streams, count, "streams")
    jobs = (rplu_job * max(count, 1))()
    outs = []
    for b, A in enumerate(As):
        if A.dim() != 2 or A.stride(1) != 1 or A.dtype not in (torch.float32, torch.float64) \
                or not A.is_cuda:
            raise ValueError("batched jobs: 2-D float32/float64 CUDA tensors, unit column stride")
        n, m = A.shape
        kk = int(ks[b])
        kmax = min(n, m) if kk <= 0 else min(kk, n, m)
        piv = torch.empty((kmax, 2), dtype=torch.int32, device=A.device)
        Lt = torch.empty((kmax, n), dtype=A.dtype, device=A.device) if store_L else None
        U = torch.empty((kmax, m), dtype=A.dtype, device=A.device) if store_U else None
        j = jobs[b]
        j.kind, j.dtype, j.n, j.m = RPLU_JOB_DENSE, _DTYPES[A.dtype], n, m
        j.A, j.lda = A.data_ptr(), A.stride(0)
        j.piv = piv.data_ptr()
        j.L, j.ldl = (Lt.data_ptr(), n) if Lt is not None else (None, 0)
        j.U, j.ldu = (U.data_ptr(), m) if U is not None else (None, 0)
        j.max_rank, j.rel_tol = kk, float(tols[b])
        j.seed, j.stream = int(seeds[b]) & (2**64 - 1), int(streams[b]) & (2**64 - 1)
        j.flags = int(flags)
        if A_origs is not None:
            Ao = A_origs[b]
            if Ao.shape != A.shape or Ao.dtype != A.dtype or Ao.stride(1) != 1:
                raise ValueError("A_origs[b] must have A's shape and dtype, unit column stride")
            j.A_orig, j.lda_orig = Ao.data_ptr(), Ao.stride(0)
            j.flags |= RPLU_FLAG_REFRESH
        outs.append((piv, Lt, U))
    return jobs, outs


class BatchPlan:
    """A batch of dense jobs with preallocated outputs and a prebuilt job
    table, for repeated launches (the matrices are overwritten by each run)."""

    def __init__(self, As, k=0, tol=0.0, seed=0, streams=None, store_L: bool = True,
                 store_U: bool = True, ctx: Optional[Context] = None, flags: int = 0,
                 A_origs=None):
        self.count = len(As)
        self.device = As[0].device if self.count else torch.device("cuda", 0)
        self.ctx = ctx or default_context(self.device.index or 0)
        self.jobs, self.outs = _batch_jobs(As, k, tol, seed, streams, store_L, store_U, flags,
                                           A_origs)
        self.infos = (rplu_info * max(self.count, 1))()
        self._keep = list(As) + list(A_origs or [])

    def run(self, cfg: Optional[dict] = None, raise_on_error: bool = True) -> int:
        if self.count == 0:
            return 0
        c = None
        if cfg is not None:
            c = rplu_batch_cfg(int(cfg.get("rows_per_pass", 0)), int(cfg.get("wg_per_cu", 0)),
                               int(cfg.get("order", 0)), 0)
        st = lib.rplu_batched_ex(self.ctx.handle, self.count, self.jobs, self.infos,
                                 C.byref(c) if c is not None else None, _cur_stream(self.device))
        if st < 0 and (raise_on_error or all(self.infos[b].status == 0 for b in range(self.count))):
            raise RPLUError(st, "rplu_batched")
        return st

    def ranks(self) -> list:
        return [int(self.infos[b].rank) for b in range(self.count)]

    def results(self) -> list:
        res = []
        for b in range(self.count):
            piv, Lt, U = self.outs[b]
            inf = self.infos[b]
            r = int(inf.rank)
            res.append(Result(piv[:r], Lt[:r].T if Lt is not None else None,
                              U[:r] if U is not None else None, r, int(inf.stop),
                              float(inf.a_fro2), float(inf.res_fro2), status=int(inf.status),
                              refreshes=int(inf.refreshes), first_refresh=int(inf.first_refresh)))
        return res


def rplu_batched(As, k=0, tol=0.0, seed=0, streams=None, store_L: bool = True,
                 store_U: bool = True, cfg: Optional[dict] = None, raise_on_error: bool = True,
                 ctx: Optional[Context] = None, flags: int = 0) -> list:
    """Dense RPLU of every matrix in As (float32 or float64 CUDA tensors, one
    dtype; each overwritten by its final Schur complement) in one persistent
    launch. k, tol, seed may be scalars or per-job lists; streams defaults to
    the job index. cfg: {'rows_per_pass', 'wg_per_cu', 'order'} (missing or 0
    = tuned). Returns one Result per job."""
    if len(As) == 0:
        return []
    plan = BatchPlan(As, k, tol, seed, streams, store_L, store_U, ctx, flags)
    plan.run(cfg, raise_on_error)
    return plan.results()


def rplu_batched_tune(As, k=0, tol=0.0, seed=0, streams=None, store_L: bool = True,
                      store_U: bool = True, ctx: Optional[Context] = None):
    """Runs the autotuner on copies of As (not modified); returns (cfg, ms)."""
    count = len(As)
    dev = As[0].device
    ctx = ctx or default_context(dev.index or 0)
    jobs, _ = _batch_jobs(As, k, tol, seed, streams, store_L, store_U)
    best = rplu_batch_cfg()
    ms = C.c_double()
    _check(lib.rplu_batched_tune(ctx.handle, count, jobs, C.byref(best), C.byref(ms),
                                 _cur_stream(dev)), "rplu_batched_tune")
    return ({"rows_per_pass": best.rows_per_pass, "wg_per_cu": best.wg_per_cu,
             "order": best.order}, float(ms.value))


def rplu_verify(A: torch.Tensor, L: Optional[torch.Tensor], U: Optional[torch.Tensor],
                S: Optional[torch.Tensor] = None, ctx: Optional[Context] = None) -> dict:
    """FP64 norms of a factorisation: ||A||^2, ||A - L U||^2 and (when S is
    given) ||A - L U - S||^2. A, S: n x m row-major; L: n x k (any view whose
    columns are contiguous, e.g. Result.L); U: k x m row-major. float32 or
    float64, one dtype."""
    if A.dtype not in (torch.float32, torch.float64) or A.dim() != 2 or A.stride(1) != 1:
        raise ValueError("A: 2-D float32/float64 CUDA tensor with unit column stride")
    n, m = A.shape
    k = 0 if L is None else L.shape[1]
    dev = A.device
    ctx = ctx or default_context(dev.index or 0)
    ldl = 0
    if k:
        if L.shape[0] != n or L.stride(0) != 1 or U.shape != (k, m) or U.stride(1) != 1:
            raise ValueError("L: n x k with contiguous columns; U: k x m row-major")
        if L.dtype != A.dtype or U.dtype != A.dtype:
            raise ValueError("A, L, U must share one dtype")
        ldl = L.stride(1) if k > 1 else n
    if S is not None and (S.shape != (n, m) or S.stride(1) != 1 or S.dtype != A.dtype):
        raise ValueError("S: n x m row-major, dtype of A")
    out = rplu_verify_out()
    _check(lib.rplu_verify(ctx.handle, _DTYPES[A.dtype], n, m, k, _ptr(A), A.stride(0),
                           _ptr(L) if k else None, ldl, _ptr(U) if k else None,
                           U.stride(0) if k else 0, _ptr(S), S.stride(0) if S is not None else 0,
                           C.byref(out), _cur_stream(dev)), "rplu_verify")
    return {"a_fro2": out.a_fro2, "err_fro2": out.err_fro2, "schur_gap_fro2": out.schur_gap_fro2}


class Server:
    """Continuous-batching server (rplu_server_*). submit_* return a ticket;
    the server owns each job's outputs (allocated in its pool at admission).
    poll returns None while the job is pending, else its Result (raising
    RPLUError if it failed): the outputs are copied into new tensors and the
    job's output block is released."""

    def __init__(self, budget_bytes: int, max_slots: int = 0, queue_capacity: int = 0,
                 workers: int = 0, batch_max_dim: int = 0, simulate: bool = False,
                 ctx: Optional[Context] = None, device: int = 0, tick_steps: int = 0):
        self.ctx = None if simulate else (ctx or default_context(device))
        self.simulate = simulate
        cfg = rplu_server_cfg(int(budget_bytes), int(max_slots), int(queue_capacity), int(workers),
                              int(batch_max_dim), RPLU_SERVER_SIMULATE if simulate else 0,
                              int(tick_steps))
        h = C.c_void_p()
        _check(lib.rplu_server_create(self.ctx.handle if self.ctx else None, C.byref(cfg),
                                      C.byref(h)), "rplu_server_create")
        self.handle = h
        self._pending = {}

    def _submit(self, job, keep, dtype, n, m):
        ev = None
        if not self.simulate:
            # the admission copy waits for the inputs' writes on this stream
            ev = torch.cuda.Event()
            ev.record(torch.cuda.current_stream(keep[0].device))
            job.ready_event = ev.cuda_event
        t = C.c_uint64()
        _check(lib.rplu_server_submit(self.handle, C.byref(job), C.byref(t)), "rplu_server_submit")
        self._pending[t.value] = (keep, ev, dtype, n, m)
        return t.value

    def submit_dense(self, A: torch.Tensor, k: int = 0, tol: float = 0.0, seed: int = 0,
                     stream: int = 0, flags: int = 0) -> int:
        """A is read (never modified); it must stay valid until poll returns.
        flags: RPLU_FLAG_STALL_STOP, RPLU_FLAG_REFRESH, RPLU_FLAG_CERTIFY."""
        if A.dim() != 2 or A.stride(1) != 1 or A.dtype not in _DTYPES:
            raise ValueError("A: 2-D tensor with unit column stride")
        n, m = A.shape
        j = rplu_job()
        j.kind, j.dtype, j.n, j.m, j.A, j.lda = RPLU_JOB_DENSE, _DTYPES[A.dtype], n, m, A.data_ptr(), A.stride(0)
        j.piv, j.L, j.U = None, None, None
        j.max_rank, j.rel_tol = int(k), float(tol)
        j.seed, j.stream = int(seed) & (2**64 - 1), int(stream) & (2**64 - 1)
        j.flags = int(flags)
        return self._submit(j, (A,), A.dtype, n, m)

    def submit_cauchy(self, x, y, G, B, k: int = 0, tol: float = 0.0, seed: int = 0,
                      stream: int = 0, flags: int = 0) -> int:
        """x, y, G, B are read (never modified); they must stay valid until poll returns."""
        n, m, p = x.shape[0], y.shape[0], G.shape[1]
        for t_ in (x, y, G, B):
            if t_.dtype != torch.complex128 or not t_.is_contiguous():
                raise ValueError("x, y, G, B: contiguous complex128 tensors")
        j = rplu_job()
        j.kind, j.dtype, j.n, j.m, j.p = RPLU_JOB_CAUCHY, RPLU_C128, n, m, p
        j.x, j.y, j.G, j.B = x.data_ptr(), y.data_ptr(), G.data_ptr(), B.data_ptr()
        j.piv, j.L, j.U = None, None, None
        j.max_rank, j.rel_tol = int(k), float(tol)
        j.seed, j.stream = int(seed) & (2**64 - 1), int(stream) & (2**64 - 1)
        j.flags = int(flags)
        return self._submit(j, (x, y, G, B), torch.complex128, n, m)

    def poll(self, ticket: int, fetch: bool = True):
        """None while pending; else the Result. fetch=False returns the info
        only (no factors) and releases the job's outputs at once."""
        info = rplu_info()
        st = lib.rplu_server_poll(self.handle, int(ticket), C.byref(info))
        if st == RPLU_PENDING:
            return None
        keep, ev, dtype, n, m = self._pending.pop(ticket, (None, None, None, 0, 0))
        if st < 0:
            raise RPLUError(st, "rplu_server_poll")
        r = int(info.rank)
        res = Result(None, None, None, r, int(info.stop), float(info.a_fro2),
                     float(info.res_fro2), status=int(st))
        res.err_fro2 = float(info.err_fro2)
        res.refreshes = int(info.refreshes)
        res.first_refresh = int(info.first_refresh)
        if self.simulate or not fetch:
            _check(lib.rplu_server_release(self.handle, int(ticket)), "rplu_server_release")
            return res
        piv_p, L_p, U_p = C.c_void_p(), C.c_void_p(), C.c_void_p()
        ldl, ldu = C.c_int64(), C.c_int64()
        _check(lib.rplu_server_outputs(self.handle, int(ticket), C.byref(piv_p), C.byref(L_p),
                                       C.byref(ldl), C.byref(U_p), C.byref(ldu)),
               "rplu_server_outputs")
        dev = keep[0].device
        es = torch.empty((), dtype=dtype).element_size()
        piv = torch.empty((r, 2), dtype=torch.int32, device=dev)
        Lt = torch.empty((r, n), dtype=dtype, device=dev)
        U = torch.empty((r, m), dtype=dtype, device=dev)
        cur = torch.cuda.current_stream(dev).cuda_stream
        if r:
            for dst, src, nbytes in ((piv, piv_p, r * 2 * 4), (Lt, L_p, r * n * es),
                                     (U, U_p, r * m * es)):
                _hip_check(_hip.hipMemcpyAsync(C.c_void_p(dst.data_ptr()), src,
                                               C.c_size_t(nbytes), 3, C.c_void_p(cur)))
            _hip_check(_hip.hipStreamSynchronize(C.c_void_p(cur)))
        _check(lib.rplu_server_release(self.handle, int(ticket)), "rplu_server_release")
        res.piv, res.L, res.U = piv, Lt.T, U
        return res

    def stats(self) -> dict:
        s = rplu_server_stats_t()
        _check(lib.rplu_server_stats(self.handle, C.byref(s)), "rplu_server_stats")
        return {f: getattr(s, f) for f, _ in rplu_server_stats_t._fields_}

    def close(self):
        if self.handle:
            lib.rplu_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
