// One pivot draw (two-stage exact sampling, Sec. 4.1): the stop test, the
// row draw, the pivot row into U(t,:) and the column draw.
//
// Both draws need the chunk totals of a mass vector (cdf.hpp) before the
// single-workgroup chains can run. Two forms, with the same arithmetic and
// so the same pivots and bits:
//   * wide kernels that finish in their last workgroup: every workgroup of
//     CDF_THREADS threads produces WIDE_ELEMS consecutive masses (one per
//     thread, coalesced) and the totals of its WIDE_CHUNKS chunks; the
//     workgroup that arrives last (an atomic counter in the step state,
//     release and acquire fences on either side) runs the draw. One launch
//     per draw, spread over the GPU: the form for long rows and columns and
//     for the Cauchy-like path, whose pivot row is regenerated.
//   * one fused workgroup for both draws (pivot_draw_row + pivot_draw_col)
//     for small dense matrices, where the step is a chain of latencies and
//     one launch per step beats two: the 16 waves walk the chunks with
//     coalesced accesses and keep the totals in LDS.
// In both, a chunk total is cdf_chunk_vals over the lane-consecutive layout
// of the chunk, which LDS staging gives from the coalesced one.
#pragma once

#include "common.hpp"
#include "cdf.hpp"
#include "launch.hpp"

namespace rplu {

constexpr int PIVOT_MAX_CHUNKS = PIVOT_FUSED_MAX / CDF_CHUNK;
constexpr int PIVOT_WAVES = CDF_THREADS / RPLU_WAVE;
constexpr int WIDE_ELEMS = CDF_THREADS;                  // masses per wide workgroup
constexpr int WIDE_CHUNKS = WIDE_ELEMS / CDF_CHUNK;
static_assert(WIDE_CHUNKS * CDF_CHUNK == WIDE_ELEMS, "wide workgroups hold whole chunks");

struct PivotArgs {
    const double* rowmass;
    int n, m;
    StepState* st;
    int32_t* piv;
    uint64_t seed, stream;
    int kmax;
    double tol2;
    int stall;
    const int32_t* forced;
    double* trace;
    double* rowmass_out;
    int greedy;             // 1: C2PLU (Sec. 2.3.3), the largest masses instead of
                            // the draws; 2: CPLU (Sec. 1, complete pivoting), the
                            // first row of largest rowmax, then as C2PLU's column
    const double* rowmax;   // greedy == 2: largest |S_ij|^2 of each row
    int maxmass;            // tolerance stop on the largest row mass (Alg. 4)
};

// What the stop test reads from the state besides t, loaded at the start of
// a draw kernel (only earlier kernels write it), and the step's two Philox
// words: neither depends on the masses, so both are ready before the draw.
struct StopInputs {
    double T0, T_best, T_ref, M0;
    int t_best, refresh_on;
};

__device__ inline StopInputs stop_inputs(const StepState* st) {
    return {st->T0, st->T_best, st->T_ref, st->M0, st->t_best, st->refresh_on};
}

__device__ inline Philox4 step_words(const PivotArgs& a, int t) {
    return philox4x64_10((uint64_t)t, a.stream, 0, 0, a.seed, 0);
}

// Thread 0: stop test at the start of step t on the total T. Returns 1 when
// the run ends here (done, stop or error recorded in the state).
__device__ inline int pivot_stop_test(StepState* st, int t, double T, int kmax, double tol2,
                                      int stall, const StopInputs& in, int maxmass = 0,
                                      double M = 0.0) {
    int stop = 0, err = 0;
    const double T0 = (t == 0) ? T : in.T0;
    const double M0 = (t == 0) ? M : in.M0;     // max-mass rule: the step-0 largest mass
    double T_best = in.T_best;
    int t_best = in.t_best;
    if (stall) {
        if (t == 0) { T_best = T; t_best = 0; }
        else if (T < RPLU_STALL_RATIO * T_best) { T_best = T; t_best = t; }
        st->T_best = T_best;
        st->t_best = t_best;
    }
    double T_ref = in.T_ref;
    if (in.refresh_on && (t == 0 || !(T_ref < __builtin_inf()))) {
        T_ref = T;
        st->T_ref = T;
    }
    if (!isfinite(T)) err = RPLU_E_NONFINITE;
    else if (T == 0.0) stop = RPLU_STOP_EXHAUSTED;
    else if (tol2 > 0.0 && (maxmass ? M <= tol2 * M0 : T <= tol2 * T0)) stop = RPLU_STOP_TOL;
    else if (in.refresh_on && t < kmax && T <= RPLU_REFRESH_DROP2 * T_ref) stop = RPLU_STOP_REFRESH;
    else if (stall && t - t_best >= RPLU_STALL_WINDOW) stop = RPLU_STOP_STALL;
    else if (t >= kmax) stop = tol2 > 0.0 ? RPLU_STOP_TOL_UNREACHED : RPLU_STOP_RANK;
    st->T = T;
    if (t == 0) { st->T0 = T; st->M0 = M; }
    if (err || stop) { st->error = err; st->stop = stop; st->done = 1; }
    return (err || stop) ? 1 : 0;
}

// Thread 0: the column j drawn in U(t,:) (Ti its total, tgt the target, p
// its bin) becomes the pivot: checks it, stores a and 1/a in FP64, copies
// G_i,: and B_:,j for the Cauchy-like generator update (P >= 1), writes the
// pivot pair and the trace words, and advances t.
template <class T, int P>
__device__ inline void pivot_commit_col(StepState* st, int t, int j, int m, const T* Ut, double Ti,
                                        double tgt, const CdfPick& p, int32_t* piv, double* trace,
                                        const cf64* G, const cf64* B) {
    if (j < 0 || j >= m) {
        st->error = RPLU_E_ARG;
        st->done = 1;
        return;
    }
    const T a = Ut[j];
    const double a2 = Sc<T>::mag2(a);
    if (!(a2 > 0.0)) {
        st->error = isfinite(a2) ? RPLU_E_ZERO_PIVOT : RPLU_E_NONFINITE;
        st->done = 1;
        return;
    }
    const typename Sc<T>::W inv = winv(Sc<T>::widen(a));
    const int i = st->i;
    st->j = j;
    st->a_re = Sc<T>::re(a);
    st->a_im = Sc<T>::im(a);
    if constexpr (Sc<T>::cplx) { st->inv_re = inv.re; st->inv_im = inv.im; }
    else { st->inv_re = inv; st->inv_im = 0.0; }
    if constexpr (P > 0) {
        for (int l = 0; l < P; ++l) {
            const cf64 g = G[(int64_t)i * P + l];
            const cf64 b = B[(int64_t)l * m + j];
            st->gi[2 * l] = g.re; st->gi[2 * l + 1] = g.im;
            st->bj[2 * l] = b.re; st->bj[2 * l + 1] = b.im;
        }
    }
    if (piv != nullptr) {               // null: a copy of the step that records nothing
        piv[2 * t] = i;
        piv[2 * t + 1] = j;
    }
    if (trace != nullptr) {
        double* tr = trace + (int64_t)t * RPLU_TRACE_WORDS;
        tr[0] = st->T; tr[1] = st->row_tgt; tr[2] = st->row_lo; tr[3] = st->row_hi;
        tr[4] = Ti; tr[5] = tgt; tr[6] = p.lo; tr[7] = p.hi;
        tr[8] = Sc<T>::re(a); tr[9] = Sc<T>::im(a);
        tr[10] = (double)i; tr[11] = (double)j;
    }
    st->t = t + 1;
}

// ------------------------------------------------ draws from chunk totals

// Whole workgroup (CDF_THREADS): the first index e < len of the largest
// mass(e), the choice of C2PLU (complete 2-norm pivoting, Sec. 2.3.3; ties go
// to the smallest index), in every thread. Masses are finite and >= 0 here
// (the stop test has seen their finite sum).
template <class MassFn>
__device__ inline int wg_argmax(CdfShared& sh, int len, MassFn mass) {
    const int lane = threadIdx.x % RPLU_WAVE, w = threadIdx.x / RPLU_WAVE;
    double bv = -1.0;
    int bi = len;
    constexpr int UG = 8;                            // loads in flight per thread
    int e = threadIdx.x;
    for (; e + (UG - 1) * CDF_THREADS < len; e += UG * CDF_THREADS) {
        double v[UG];
#pragma unroll
        for (int u = 0; u < UG; ++u) v[u] = mass(e + u * CDF_THREADS);
#pragma unroll
        for (int u = 0; u < UG; ++u)
            if (v[u] > bv) { bv = v[u]; bi = e + u * CDF_THREADS; }   // ascending: keeps the first
    }
    for (; e < len; e += CDF_THREADS) {
        const double v = mass(e);
        if (v > bv) { bv = v; bi = e; }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(bv, off, RPLU_WAVE);
        const int oi = __shfl_xor(bi, off, RPLU_WAVE);
        if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
    }
    if (lane == 0) { sh.amax[w] = bv; sh.aidx[w] = bi; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = sh.amax[0];
        int idx = sh.aidx[0];
        for (int q = 1; q < CDF_THREADS / RPLU_WAVE; ++q)
            if (sh.amax[q] > v || (sh.amax[q] == v && sh.aidx[q] < idx)) { v = sh.amax[q]; idx = sh.aidx[q]; }
        sh.ibcast[3] = idx;
    }
    __syncthreads();
    return sh.ibcast[3];
}

// Whole workgroup (CDF_THREADS): stop test and row draw of step t (= st->t)
// from the chunk totals ct of the row masses (global memory or LDS); rnd
// holds the step's Philox words; mass(e) gives the row masses for the walk
// of the drawn chunk (by default from a.rowmass). Returns the row i in every
// thread (recorded in the state with cur = t), or -1 when the run ends here.
struct RowMassGlobal {
    const double* rowmass;
    __device__ double operator()(int e) const { return rowmass[e]; }
};

template <class MassFn>
__device__ inline int pivot_row_draw_ct(CdfShared& sh, int* flag, const PivotArgs& a,
                                        const double* ct, int t, const Philox4& rnd,
                                        const StopInputs& in, MassFn mass) {
    StepState* st = a.st;
    const int K = cdf_chunks(a.n);
    const double T = cdf_levels(sh, ct, K);
    // max-mass rule: the largest mass, when the total is finite (the stop
    // test reports a non-finite one)
    double M = 0.0;
    if (a.maxmass && isfinite(T)) M = mass(wg_argmax(sh, a.n, mass));
    if (threadIdx.x == 0)
        *flag = pivot_stop_test(st, t, T, a.kmax, a.tol2, a.stall, in, a.maxmass, M);
    __syncthreads();
    if (*flag) return -1;
    if (a.rowmass_out != nullptr)
        for (int e = threadIdx.x; e < a.n; e += CDF_THREADS)
            a.rowmass_out[(int64_t)t * a.n + e] = a.rowmass[e];
    const double tgt = unit_from_word(rnd.w[0]) * T;
    // CPLU: the first row holding the largest entry; with C2PLU's column
    // choice in that row this is the first largest entry in row-major order
    const CdfPick p = a.greedy == 2 ? CdfPick{wg_argmax(sh, a.n, RowMassGlobal{a.rowmax}), 0.0, 0.0}
                    : a.greedy     ? CdfPick{wg_argmax(sh, a.n, mass), 0.0, 0.0}
                                   : cdf_draw(sh, ct, K, a.n, mass, tgt);
    const int i = a.forced ? a.forced[2 * t] : p.idx;
    if (i < 0 || i >= a.n) {
        if (threadIdx.x == 0) { st->error = RPLU_E_ARG; st->done = 1; }
        return -1;
    }
    if (threadIdx.x == 0) {
        st->cur = t;
        st->i = i;
        st->row_tgt = tgt;
        st->row_lo = p.lo;
        st->row_hi = p.hi;
        // deferred sweep: a write-back of S^(t) moves the window to start at t
        if (st->flushed == t) st->t_base = t;
    }
    return i;
}

// Whole workgroup: column draw of step t in the pivot row Ut = U(t,:) from
// the chunk totals ct of |U(t,e)|^2 (mass(e) gives |U(t,e)|^2 for the walk of
// the drawn chunk), and the pivot commit.
template <class T>
struct ColMassGlobal {
    const T* Ut;
    __device__ double operator()(int e) const { return Sc<T>::mag2(Ut[e]); }
};

template <class T, int P, class MassFn>
__device__ inline void pivot_col_draw_ct(CdfShared& sh, const PivotArgs& a, int t, const T* Ut,
                                         const double* ct, const cf64* G, const cf64* B,
                                         const Philox4& rnd, MassFn mass) {
    const int K = cdf_chunks(a.m);
    const double Ti = cdf_levels(sh, ct, K);
    const double tgt = unit_from_word(rnd.w[1]) * Ti;
    CdfPick p{0, 0.0, 0.0};
    if (Ti > 0.0 && isfinite(Ti))
        p = a.greedy ? CdfPick{wg_argmax(sh, a.m, mass), 0.0, 0.0}
                     : cdf_draw(sh, ct, K, a.m, mass, tgt);
    if (threadIdx.x == 0) {
        const int j = a.forced ? a.forced[2 * t + 1] : p.idx;
        pivot_commit_col<T, P>(a.st, t, j, a.m, Ut, Ti, tgt, p, a.piv, a.trace, G, B);
    }
}

// -------------------------------------------------------------- wide form

struct WideShared {
    CdfShared cdf;
    double stage[WIDE_ELEMS + WIDE_ELEMS / CDF_E];   // element q at q + q / CDF_E
    double pair[CDF_CHUNK];                          // partial sums handed between threads
    uint64_t words[2];
    int flag;
};

// Stores the step's Philox words in LDS before the workgroup's first barrier,
// so that they are formed while the masses load (left where they are used,
// the compiler would form them after the arrival, on the draw's path); the
// draw takes them back with wide_words.
__device__ inline void wide_keep_words(WideShared& sh, const Philox4& rnd) {
    if (threadIdx.x == 0) { sh.words[0] = rnd.w[0]; sh.words[1] = rnd.w[1]; }
}

__device__ inline Philox4 wide_words(const WideShared& sh) {
    return {{sh.words[0], sh.words[1], 0, 0}};
}

// Whole workgroup: thread q < ELEMS holds the mass of element blockIdx.x *
// ELEMS + q (anything past len is ignored); writes the totals of the
// workgroup's ELEMS / CDF_CHUNK chunks to ct. The staging pads one slot per
// CDF_E elements so that a lane's consecutive reads do not all hit its
// neighbours' banks.
template <int ELEMS = WIDE_ELEMS>
__device__ inline void wide_chunk_totals(WideShared& sh, double mass, int len, double* ct) {
    static_assert(ELEMS % CDF_CHUNK == 0 && ELEMS <= WIDE_ELEMS, "whole chunks per workgroup");
    constexpr int CHUNKS = ELEMS / CDF_CHUNK;
    const int q = threadIdx.x;
    if (q < ELEMS) sh.stage[q + q / CDF_E] = mass;
    __syncthreads();
    const int w = q / RPLU_WAVE, lane = q % RPLU_WAVE;
    const int chunk = blockIdx.x * CHUNKS + w;
    if (w < CHUNKS && chunk < cdf_chunks(len)) {
        const int s0 = w * CDF_CHUNK + lane * CDF_E;      // first of the lane's elements
        double x[CDF_E];
#pragma unroll
        for (int u = 0; u < CDF_E; ++u) x[u] = sh.stage[s0 + s0 / CDF_E + u];
        CdfChunk c;
        cdf_chunk_vals(c, x, chunk, len, lane);
        if (lane == 0) ct[chunk] = c.ct;
    }
}

// Whole workgroup, after its global writes: true (in every thread) in the
// workgroup that arrives last, which then sees every other workgroup's
// writes; that workgroup also clears the counter for the next launch. The
// barrier orders the workgroup's stores before thread 0's device-scope
// release fence and arrival; in the last workgroup, thread 0's acquire fence
// and the barrier after it order every later load after all arrivals. One
// fence per workgroup: on a GPU whose L2 is split between dies a
// device-scope release writes back the L2, too slow to do in every wave.
__device__ inline bool wide_arrive_last(WideShared& sh, uint32_t* counter) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const int last = (atomicAdd(counter, 1u) == gridDim.x - 1) ? 1 : 0;
        if (last) {
            __threadfence();
            *counter = 0u;
        }
        sh.flag = last;
    }
    __syncthreads();
    if (!sh.flag) return false;
    __syncthreads();                    // sh.flag is reused by the draw
    return true;
}

// ------------------------------------------------------ fused workgroup

// Per-wave staging of one chunk's masses (element q at q + q / CDF_E).
constexpr int PIVOT_STAGE = CDF_CHUNK + CDF_CHUNK / CDF_E;

struct PivotShared {
    CdfShared cdf;
    double ctr[PIVOT_MAX_CHUNKS];   // chunk totals of the row masses
    double ctc[PIVOT_MAX_CHUNKS];   // chunk totals of |U(t,e)|^2
    double stage[PIVOT_WAVES][PIVOT_STAGE];
    uint64_t words[2];              // the step's Philox words (as in WideShared)
    int flag;
};

// Chunk totals of a vector of length len into ct (LDS), chunk k by wave
// k mod 16. One workgroup walks the whole vector, so the masses are produced
// with coalesced accesses (lane l takes elements base + 64 u + l, clamped
// into range as in cdf_chunk) and handed to the lane-consecutive layout
// through LDS. load(e) only reads memory and finish(loaded, e) returns the
// mass (and may store), so a lane's loads (all E of them, or as many as fit
// in about 64 registers) are in flight before any is waited for.
template <class LoadFn, class FinishFn>
__device__ inline void pivot_chunk_totals(PivotShared& sh, double* ct, int len, LoadFn load,
                                          FinishFn finish) {
    using L = decltype(load(0));
    constexpr int UG0 = 256 / (int)sizeof(L);
    constexpr int UG = UG0 >= 8 ? 8 : UG0 >= 4 ? 4 : UG0 >= 2 ? 2 : 1;
    const int lane = threadIdx.x % RPLU_WAVE, w = threadIdx.x / RPLU_WAVE;
    double* stage = sh.stage[w];
    const int K = cdf_chunks(len);
    for (int k = w; k < K; k += PIVOT_WAVES) {
        const int base = k * CDF_CHUNK;
#pragma unroll
        for (int u0 = 0; u0 < CDF_E; u0 += UG) {
            L ld[UG];
#pragma unroll
            for (int u = 0; u < UG; ++u)
                ld[u] = load(min(base + (u0 + u) * RPLU_WAVE + lane, len - 1));
#pragma unroll
            for (int u = 0; u < UG; ++u) {
                const int q = (u0 + u) * RPLU_WAVE + lane;
                stage[q + q / CDF_E] = finish(ld[u], min(base + q, len - 1));
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        double x[CDF_E];
#pragma unroll
        for (int u = 0; u < CDF_E; ++u) x[u] = stage[lane * (CDF_E + 1) + u];
        CdfChunk c;
        cdf_chunk_vals(c, x, k, len, lane);
        if (lane == 0) ct[k] = c.ct;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");   // stage reused next chunk
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    __syncthreads();
}

// Whole workgroup: stop test and row draw of step t (= st->t, not done),
// the chunk totals formed here. Returns the row i in every thread, or -1
// when the run ends here. The step's Philox words are formed by the last
// wave, which holds no chunk while the vector has fewer than 16: its chain
// of 64-bit products (some thousand cycles) then runs beside the first
// waves' mass loads instead of before them.
__device__ inline int pivot_draw_row(PivotShared& sh, const PivotArgs& a, int t,
                                     const StopInputs& in) {
    if (threadIdx.x == CDF_THREADS - RPLU_WAVE) {
        const Philox4 rnd = step_words(a, t);
        sh.words[0] = rnd.w[0];
        sh.words[1] = rnd.w[1];
    }
    pivot_chunk_totals(sh, sh.ctr, a.n, [&](int e) { return a.rowmass[e]; },
                       [](double v, int) { return v; });
    const Philox4 w{{sh.words[0], sh.words[1], 0, 0}};
    return pivot_row_draw_ct(sh.cdf, &sh.flag, a, sh.ctr, t, w, in, RowMassGlobal{a.rowmass});
}

// Whole workgroup, after pivot_draw_row returned i >= 0 for step t: writes
// the pivot row into Ut = U(t,:) (element e is value(load(e)); load only
// reads memory), draws the column and commits the pivot. The column draw
// re-reads U(t,:) after the barrier that ends the row pass.
template <class T, int P, class LoadFn, class ValueFn>
__device__ inline void pivot_draw_col(PivotShared& sh, const PivotArgs& a, int t, T* Ut,
                                      const cf64* G, const cf64* B, LoadFn load, ValueFn value) {
    pivot_chunk_totals(sh, sh.ctc, a.m, load, [&](const decltype(load(0))& ld, int e) {
        const T v = value(ld);
        Ut[e] = v;
        return Sc<T>::mag2(v);
    });
    const Philox4 w{{sh.words[0], sh.words[1], 0, 0}};
    pivot_col_draw_ct<T, P>(sh.cdf, a, t, Ut, sh.ctc, G, B, w, ColMassGlobal<T>{Ut});
}

// Host: the pivot kernels' arguments from a sampler descriptor.
inline PivotArgs pivot_args(const SampleArgs& sa) {
    PivotArgs p;
    p.rowmass = sa.rowmass;
    p.n = (int)sa.n;
    p.m = (int)sa.m;
    p.st = sa.st;
    p.piv = sa.piv;
    p.seed = sa.seed;
    p.stream = sa.stream;
    p.kmax = (int)sa.kmax;
    p.tol2 = sa.tol2;
    p.stall = sa.stall;
    p.forced = sa.forced;
    p.trace = sa.trace;
    p.rowmass_out = sa.rowmass_out;
    p.greedy = sa.greedy;
    p.rowmax = sa.rowmax;
    p.maxmass = sa.maxmass;
    return p;
}

inline unsigned wide_blocks(int64_t len) { return (unsigned)((len + WIDE_ELEMS - 1) / WIDE_ELEMS); }

}  // namespace rplu
