// RPLU in CUR form (Alg. 2, Sec. 4.1): the approximation is kept as
// A[:, J] U_k A[I, :] with the core U_k = A[I, J]^{-1}; A is only read. Each
// step reads A once (against one read and one write of S in the dense form)
// and touches O(k^2 + (n + m) k) other data.
//
// Per step t (k = t pivots so far; every kernel returns at once when the
// stop test of the step has fired):
//   k_rows_draw (sample.hip)  stop test on the row-norm estimates and the row
//                    draw i (the estimates are the row masses of the draws)
//   k_cur_zu         z = A[i, J] and z^T U_k (from the transpose of U_k)
//   k_cur_pivrow_draw  the residual's pivot row r^ = A[i, :] - (z^T U_k) A[I, :]
//                    (0 in the selected columns) with the chunk totals of
//                    |r^|^2; the last workgroup draws the column j
//   k_cur_l_gi       l = r^ / r^_j (times the FP64 reciprocal), partial sums of
//                    |l|^2, and for the selected rows g[I] = A[I, :] conj(l)
//                    and w = A[I, j]
//   k_cur_core_mv    y = U_k g[I] and U_k w; the last workgroup forms
//                    sigma = A[i, j] - z^T U_k w and ||l||^2
//   k_cur_sweep      one pass over the live rows of A: g = A conj(l),
//                    v = A[:, J] y, the residual column c^ = A[:, j] - A[:, J] U_k w
//                    and the row-norm update
//                    n <- n - 2 Re((g - v) conj(c^)) + ||l||^2 |c^|^2;
//                    appends A[:, j] to the compact copy of A[:, J]
//   k_cur_core_update  U_{k+1} from U_k (eq. block-inverse-update), and its
//                    transpose
//
// Arithmetic: A in its storage type, everything else in FP64 (complex FP64),
// so single-precision storage loses nothing beyond the rounding of A itself.
// Every reduction has an order fixed by the sizes (deterministic results).
#include <type_traits>

#include "common.hpp"
#include "cdf.hpp"
#include "launch.hpp"
#include "pivot.hpp"

namespace rplu {

// ------------------------------------------------ FP64 scalar helpers

__device__ inline double wzero(double) { return 0.0; }
__device__ inline cf64 wzero(cf64) { return {0.0, 0.0}; }
__device__ inline double wconj(double v) { return v; }
__device__ inline cf64 wconj(cf64 v) { return {v.re, -v.im}; }
__device__ inline double wsubv(double a, double b) { return a - b; }
__device__ inline cf64 wsubv(cf64 a, cf64 b) { return csub(a, b); }
__device__ inline double waddv(double a, double b) { return a + b; }
__device__ inline cf64 waddv(cf64 a, cf64 b) { return cadd(a, b); }
__device__ inline double wneg(double a) { return -a; }
__device__ inline cf64 wneg(cf64 a) { return {-a.re, -a.im}; }
__device__ inline double wdivv(double a, double b) { return a / b; }
__device__ inline cf64 wdivv(cf64 a, cf64 b) { return cdiv(a, b); }
__device__ inline double wre(double a) { return a; }
__device__ inline double wre(cf64 a) { return a.re; }
// c + a b
__device__ inline double wmad(double a, double b, double c) { return fma(a, b, c); }
__device__ inline cf64 wmad(cf64 a, cf64 b, cf64 c) {
    return {fma(a.re, b.re, fma(-a.im, b.im, c.re)), fma(a.re, b.im, fma(a.im, b.re, c.im))};
}
// c - a b
__device__ inline double wmsub(double a, double b, double c) { return fma(-a, b, c); }
__device__ inline cf64 wmsub(cf64 a, cf64 b, cf64 c) {
    return {fma(-a.re, b.re, fma(a.im, b.im, c.re)), fma(-a.re, b.im, fma(-a.im, b.re, c.im))};
}
// Re(a conj(b))
__device__ inline double wre_conj(double a, double b) { return a * b; }
__device__ inline double wre_conj(cf64 a, cf64 b) { return fma(a.re, b.re, a.im * b.im); }
__device__ inline double wmag2(double a) { return a * a; }
__device__ inline double wmag2(cf64 a) { return fma(a.re, a.re, a.im * a.im); }
__device__ inline double wave_sum_w(double v) { return wave_sum(v); }
__device__ inline cf64 wave_sum_w(cf64 v) { return {wave_sum(v.re), wave_sum(v.im)}; }

template <class W>
__device__ inline W w_of_state(double re, double im) {
    if constexpr (std::is_same<W, cf64>::value) return cf64{re, im};
    else return re;
}

// Whole workgroup of BS threads: the sum of v over all threads (wave sums,
// then the waves in order), in every thread. red holds BS / 64 values.
template <int BS, class W>
__device__ inline W wg_sum(W v, W* red) {
    const int lane = threadIdx.x % RPLU_WAVE, wv = threadIdx.x / RPLU_WAVE;
    v = wave_sum_w(v);
    __syncthreads();                       // red may hold an earlier sum
    if (lane == 0) red[wv] = v;
    __syncthreads();
    W s = red[0];
#pragma unroll
    for (int q = 1; q < BS / RPLU_WAVE; ++q) s = waddv(s, red[q]);
    return s;
}

// Whole workgroup, after its global writes: true in the workgroup that
// arrives last (it then sees every other workgroup's writes; see
// wide_arrive_last, whose protocol this repeats with a smaller LDS footprint).
__device__ inline bool cur_arrive_last(int* flag, uint32_t* counter) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const int last = (atomicAdd(counter, 1u) == gridDim.x - 1) ? 1 : 0;
        if (last) {
            __threadfence();
            *counter = 0u;
        }
        *flag = last;
    }
    __syncthreads();
    return *flag != 0;
}

constexpr int CUR_THREADS = 1024;
constexpr int CUR_ZCHUNK = 1024;       // z^T U_k values staged in LDS at a time

// ----------------------------------------------------------- z^T U_k

template <class T>
__global__ __launch_bounds__(CUR_THREADS) void k_cur_zu(CurArgs a) {
    using W = typename Sc<T>::W;
    if (a.st->done) return;
    const int t = a.st->cur, i = a.st->i;
    if (t == 0) return;
    __shared__ W zs[RPLU_CUR_MAX_RANK];
    const T* A = (const T*)a.A;
    for (int q = threadIdx.x; q < t; q += CUR_THREADS) {
        const W z = Sc<T>::widen(A[(int64_t)i * a.lda + a.piv[2 * q + 1]]);
        zs[q] = z;
        if (blockIdx.x == 0) ((W*)a.zv)[q] = z;
    }
    __syncthreads();
    const W* Ut = (const W*)a.Ut;
    const int lane = threadIdx.x % RPLU_WAVE, wv = threadIdx.x / RPLU_WAVE;
    constexpr int NW = CUR_THREADS / RPLU_WAVE;
    for (int b = blockIdx.x * NW + wv; b < t; b += gridDim.x * NW) {
        W acc = wzero(W{});
        for (int q = lane; q < t; q += RPLU_WAVE) acc = wmad(Ut[(int64_t)b * a.kmax + q], zs[q], acc);
        acc = wave_sum_w(acc);
        if (lane == 0) ((W*)a.zU)[b] = acc;       // (z^T U_k)_b = sum_q U_k(q, b) z_q
    }
}

// ------------------------------------------------ pivot row and column draw

template <class T>
__global__ __launch_bounds__(CDF_THREADS) void k_cur_pivrow_draw(CurArgs a, PivotArgs pa) {
    using W = typename Sc<T>::W;
    __shared__ WideShared sh;
    __shared__ W zu[CUR_ZCHUNK];
    __shared__ int ri[CUR_ZCHUNK];
    if (a.st->done) return;
    const int t = a.st->cur, i = a.st->i;
    wide_keep_words(sh, step_words(pa, t));
    const T* A = (const T*)a.A;
    const int e = blockIdx.x * WIDE_ELEMS + threadIdx.x;
    const bool in = e < a.m;
    const int ec = in ? e : (int)a.m - 1;
    W x = Sc<T>::widen(A[(int64_t)i * a.lda + ec]);
    for (int q0 = 0; q0 < t; q0 += CUR_ZCHUNK) {
        const int nq = min(CUR_ZCHUNK, t - q0);
        __syncthreads();
        for (int q = threadIdx.x; q < nq; q += CDF_THREADS) {
            zu[q] = ((const W*)a.zU)[q0 + q];
            ri[q] = a.piv[2 * (q0 + q)];
        }
        __syncthreads();
        // sixteen rows' entries are loaded before any is used (one memory
        // round trip for sixteen rows); the updates stay in order
        constexpr int CUR_U = 16;
        int q = 0;
        for (; q + CUR_U <= nq; q += CUR_U) {
            T v[CUR_U];
#pragma unroll
            for (int u = 0; u < CUR_U; ++u) v[u] = A[(int64_t)ri[q + u] * a.lda + ec];
#pragma unroll
            for (int u = 0; u < CUR_U; ++u) x = wmsub(Sc<T>::widen(v[u]), zu[q + u], x);
        }
        for (; q < nq; ++q) x = wmsub(Sc<T>::widen(A[(int64_t)ri[q] * a.lda + ec]), zu[q], x);
    }
    if (a.selc[ec]) x = wzero(W{});             // selected columns: 0 in the residual
    if (in) ((W*)a.rhat)[e] = x;
    wide_chunk_totals(sh, in ? wmag2(x) : 0.0, (int)a.m, a.ct_col);
    if (!wide_arrive_last(sh, &a.st->arrive)) return;
    pivot_col_draw_ct<W, 0>(sh.cdf, pa, t, (const W*)a.rhat, a.ct_col, nullptr, nullptr,
                            wide_words(sh), ColMassGlobal<W>{(const W*)a.rhat});
    if (threadIdx.x == 0 && !a.st->done) a.selc[a.st->j] = 1;
}

// -------------------------------------- l, ||l||^2 partials, g[I] and w

template <class T>
__global__ __launch_bounds__(CUR_THREADS) void k_cur_l_gi(CurArgs a, int nbl) {
    using W = typename Sc<T>::W;
    __shared__ W red[CUR_THREADS / RPLU_WAVE];
    __shared__ double red2[CUR_THREADS / RPLU_WAVE];
    if (a.st->done) return;
    const int t = a.st->cur, j = a.st->j;
    const W inv = w_of_state<W>(a.st->inv_re, a.st->inv_im);
    const W* rhat = (const W*)a.rhat;
    if ((int)blockIdx.x < nbl) {
        const int e = blockIdx.x * CUR_THREADS + threadIdx.x;
        double v = 0.0;
        if (e < a.m) {
            const W lq = wmul(rhat[e], inv);
            ((W*)a.l)[e] = lq;
            v = wmag2(lq);
        }
        const double s = wg_sum<CUR_THREADS>(v, red2);
        if (threadIdx.x == 0) a.l2part[blockIdx.x] = s;
        return;
    }
    const T* A = (const T*)a.A;
    const int G = gridDim.x - nbl;
    for (int s = blockIdx.x - nbl; s < t; s += G) {
        const int r = a.piv[2 * s];
        const T* Ar = A + (int64_t)r * a.lda;
        W acc = wzero(W{});
        // eight columns' entries are loaded before any is used (one memory
        // round trip for eight); the products are added in column order
        constexpr int CUR_GU = 8;
        int q = threadIdx.x;
        for (; q + (CUR_GU - 1) * CUR_THREADS < a.m; q += CUR_GU * CUR_THREADS) {
            T av[CUR_GU];
            W rv[CUR_GU];
#pragma unroll
            for (int u = 0; u < CUR_GU; ++u) {
                av[u] = Ar[q + u * CUR_THREADS];
                rv[u] = rhat[q + u * CUR_THREADS];
            }
#pragma unroll
            for (int u = 0; u < CUR_GU; ++u)
                acc = wmad(Sc<T>::widen(av[u]), wconj(wmul(rv[u], inv)), acc);
        }
        for (; q < a.m; q += CUR_THREADS)
            acc = wmad(Sc<T>::widen(Ar[q]), wconj(wmul(rhat[q], inv)), acc);
        acc = wg_sum<CUR_THREADS>(acc, red);
        if (threadIdx.x == 0) {
            ((W*)a.gI)[s] = acc;                   // (A conj(l))[I_s]
            ((W*)a.wv)[s] = Sc<T>::widen(Ar[j]);   // A[I_s, j]
        }
    }
}

// --------------------------------------------- U_k g[I], U_k w and sigma

template <class T>
__global__ __launch_bounds__(CUR_THREADS) void k_cur_core_mv(CurArgs a, int nbl) {
    using W = typename Sc<T>::W;
    __shared__ int flag;
    if (a.st->done) return;
    const int t = a.st->cur;
    const W* Uc = (const W*)a.Uc;
    const W* gI = (const W*)a.gI;
    const W* wv = (const W*)a.wv;
    const int lane = threadIdx.x % RPLU_WAVE, wid = threadIdx.x / RPLU_WAVE;
    constexpr int NW = CUR_THREADS / RPLU_WAVE;
    for (int r = blockIdx.x * NW + wid; r < t; r += gridDim.x * NW) {
        W s1 = wzero(W{}), s2 = wzero(W{});
        for (int b = lane; b < t; b += RPLU_WAVE) {
            const W u = Uc[(int64_t)r * a.ldc + b];
            s1 = wmad(u, gI[b], s1);
            s2 = wmad(u, wv[b], s2);
        }
        s1 = wave_sum_w(s1);
        s2 = wave_sum_w(s2);
        if (lane == 0) {
            ((W*)a.y)[r] = s1;
            ((W*)a.Uw)[r] = s2;
        }
    }
    if (!cur_arrive_last(&flag, &a.st->arrive)) return;
    if (wid != 0) return;
    // one wave: sigma = A[i, j] - z^T (U_k w), ||l||^2 = the partials in order
    const W* zv = (const W*)a.zv;
    const W* Uw = (const W*)a.Uw;
    W s = wzero(W{});
    for (int r = lane; r < t; r += RPLU_WAVE) s = wmad(zv[r], Uw[r], s);
    s = wave_sum_w(s);
    double l2 = 0.0;
    for (int b = lane; b < nbl; b += RPLU_WAVE) l2 += a.l2part[b];
    l2 = wave_sum(l2);
    if (lane == 0) {
        const T* A = (const T*)a.A;
        const W omega = Sc<T>::widen(A[(int64_t)a.st->i * a.lda + a.st->j]);
        const W sig = wsubv(omega, s);
        StepState* st = a.st;
        st->sig_re = wre(sig);
        if constexpr (std::is_same<W, cf64>::value) st->sig_im = sig.im;
        else st->sig_im = 0.0;
        st->l2 = l2;
        const double m2 = wmag2(sig);
        if (!(m2 > 0.0) || !isfinite(m2) || !isfinite(l2)) {
            st->error = isfinite(m2) ? RPLU_E_ZERO_PIVOT : RPLU_E_NONFINITE;
            st->done = 1;
        }
    }
}

// ------------------------------------------------------------ main pass

// R rows of A per workgroup, V elements per 16-byte pack (1 when rows are not
// 16-byte aligned). Rows already selected (and the pivot row) are not read:
// their estimates are 0.
template <class T, int R, int BS, int V>
__global__ __launch_bounds__(BS) void k_cur_sweep(CurArgs a) {
    using W = typename Sc<T>::W;
    __shared__ W red[BS / RPLU_WAVE][R][3];
    if (a.st->done) return;
    const int t = a.st->cur, pi = a.st->i, pj = a.st->j;
    const double l2 = a.st->l2;
    const int tid = threadIdx.x, lane = tid % RPLU_WAVE, wv = tid / RPLU_WAVE;
    const int64_t n = a.n, m = a.m;
    const int r0 = blockIdx.x * R;
    const int nr = (int)min((int64_t)R, n - r0);
    bool live[R];
    bool any = false;
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int p = r0 + q;
        live[q] = q < nr && p != pi && a.selr[p] == 0;
        any = any || live[q];
    }
    if (!any) {
        if (tid == 0 && pi >= r0 && pi < r0 + nr) {
            a.nrm[pi] = 0.0;
            a.selr[pi] = 1;
        }
        return;
    }
    const T* A = (const T*)a.A;
    const W* l = (const W*)a.l;
    W rg[R], rv[R], rc[R];
#pragma unroll
    for (int q = 0; q < R; ++q) rg[q] = rv[q] = rc[q] = wzero(W{});

    // g_p = sum_q A[p, q] conj(l_q)
    auto pack = [&](int64_t c, auto full_tag) {
        constexpr bool FULL = decltype(full_tag)::value;
        W lc[V];
#pragma unroll
        for (int v = 0; v < V; ++v) lc[v] = (FULL || c + v < m) ? wconj(l[c + v]) : wzero(W{});
        T x[R][V];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            if (live[q]) {
                const T* p = A + (int64_t)(r0 + q) * a.lda + c;
                if constexpr (FULL && V * sizeof(T) == 16) {
                    // A is re-read every step and does not stay in the caches:
                    // streaming 16-byte loads
                    const uint32_t* w = reinterpret_cast<const uint32_t*>(p);
                    uint32_t u[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) u[k] = __builtin_nontemporal_load(w + k);
                    __builtin_memcpy(&x[q][0], u, 16);
                } else {
#pragma unroll
                    for (int v = 0; v < V; ++v) x[q][v] = (FULL || c + v < m) ? p[v] : Sc<T>::zero();
                }
            }
        }
#pragma unroll
        for (int q = 0; q < R; ++q) {
            if (live[q]) {
#pragma unroll
                for (int v = 0; v < V; ++v) rg[q] = wmad(Sc<T>::widen(x[q][v]), lc[v], rg[q]);
            }
        }
    };
    int64_t c = (int64_t)tid * V;
    for (; c + V <= m; c += (int64_t)BS * V) pack(c, std::true_type{});
    if (c < m) pack(c, std::false_type{});

    // v_p = A[p, J] y and A[p, J] (U_k w) from the compact copy of A[:, J]
    const T* Cm = (const T*)a.C;
    const W* y = (const W*)a.y;
    const W* Uw = (const W*)a.Uw;
    for (int b = tid; b < t; b += BS) {
        const W yb = y[b], ub = Uw[b];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            if (live[q]) {
                const W cb = Sc<T>::widen(Cm[(int64_t)(r0 + q) * a.kmax + b]);
                rv[q] = wmad(cb, yb, rv[q]);
                rc[q] = wmad(cb, ub, rc[q]);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const W s0 = wave_sum_w(rg[q]), s1 = wave_sum_w(rv[q]), s2 = wave_sum_w(rc[q]);
        if (lane == 0) {
            red[wv][q][0] = s0;
            red[wv][q][1] = s1;
            red[wv][q][2] = s2;
        }
    }
    __syncthreads();
    if (tid < nr) {
        const int q = tid, p = r0 + q;
        if (live[q]) {
            W g = red[0][q][0], v = red[0][q][1], cu = red[0][q][2];
#pragma unroll
            for (int w = 1; w < BS / RPLU_WAVE; ++w) {
                g = waddv(g, red[w][q][0]);
                v = waddv(v, red[w][q][1]);
                cu = waddv(cu, red[w][q][2]);
            }
            const T apj = A[(int64_t)p * a.lda + pj];
            const W ch = wsubv(Sc<T>::widen(apj), cu);            // residual column entry
            double nn = a.nrm[p] - 2.0 * wre_conj(wsubv(g, v), ch);
            nn = nn + l2 * wmag2(ch);
            a.nrm[p] = nn < 0.0 ? 0.0 : nn;
            ((T*)a.C)[(int64_t)p * a.kmax + t] = apj;              // A[:, J] gains column j
        } else if (p == pi) {
            a.nrm[p] = 0.0;
            a.selr[p] = 1;
        }
    }
}

// ------------------------------------------------------------ core update

template <class T>
__global__ __launch_bounds__(256) void k_cur_core_update(CurArgs a) {
    using W = typename Sc<T>::W;
    if (a.st->done) return;
    const int t = a.st->cur;
    const W sig = w_of_state<W>(a.st->sig_re, a.st->sig_im);
    const W one = w_of_state<W>(1.0, 0.0);
    W* Uc = (W*)a.Uc;
    W* Ut = (W*)a.Ut;
    const W* Uw = (const W*)a.Uw;
    const W* zU = (const W*)a.zU;
    const int64_t k1 = t + 1;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < k1 * k1;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(e / k1), b = (int)(e % k1);
        W v;
        if (r < t && b < t) v = waddv(Uc[(int64_t)r * a.ldc + b], wdivv(wmul(Uw[r], zU[b]), sig));
        else if (r < t) v = wdivv(wneg(Uw[r]), sig);
        else if (b < t) v = wdivv(wneg(zU[b]), sig);
        else v = wdivv(one, sig);
        Uc[(int64_t)r * a.ldc + b] = v;
        Ut[(int64_t)b * a.kmax + r] = v;
    }
}

// ---------------------------------------------------------------- launchers

constexpr int CUR_ROWS = 8;          // rows per workgroup of the main pass
constexpr int CUR_SWEEP_THREADS = 512;

static unsigned cur_small_grid(int64_t kmax, int per) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((kmax + per - 1) / per, 256));
}

int cur_l_blocks(int64_t m) { return (int)((m + CUR_THREADS - 1) / CUR_THREADS); }

template <class T>
static void cur_part_t(const CurArgs& a, const PivotArgs& pa, int part, hipStream_t s) {
    constexpr int NW = CUR_THREADS / RPLU_WAVE;
    const int nbl = cur_l_blocks(a.m);
    if (part == CUR_PART_PIVOT) {
        hipLaunchKernelGGL((k_cur_zu<T>), dim3(cur_small_grid(a.kmax, NW)), dim3(CUR_THREADS), 0,
                           s, a);
        hipLaunchKernelGGL((k_cur_pivrow_draw<T>), dim3(wide_blocks(a.m)), dim3(CDF_THREADS), 0, s,
                           a, pa);
    } else if (part == CUR_PART_VECTORS) {
        hipLaunchKernelGGL((k_cur_l_gi<T>), dim3(nbl + cur_small_grid(a.kmax, 1)),
                           dim3(CUR_THREADS), 0, s, a, nbl);
        hipLaunchKernelGGL((k_cur_core_mv<T>), dim3(cur_small_grid(a.kmax, NW)), dim3(CUR_THREADS),
                           0, s, a, nbl);
    } else if (part == CUR_PART_SWEEP) {
        const unsigned nb = (unsigned)((a.n + CUR_ROWS - 1) / CUR_ROWS);
        if (a.vec_ok)
            hipLaunchKernelGGL((k_cur_sweep<T, CUR_ROWS, CUR_SWEEP_THREADS, 16 / (int)sizeof(T)>),
                               dim3(nb), dim3(CUR_SWEEP_THREADS), 0, s, a);
        else
            hipLaunchKernelGGL((k_cur_sweep<T, CUR_ROWS, CUR_SWEEP_THREADS, 1>), dim3(nb),
                               dim3(CUR_SWEEP_THREADS), 0, s, a);
    } else {
        const int64_t k1 = a.kmax * a.kmax;
        const unsigned gu = (unsigned)std::max<int64_t>(1, std::min<int64_t>((k1 + 255) / 256, 2048));
        hipLaunchKernelGGL((k_cur_core_update<T>), dim3(gu), dim3(256), 0, s, a);
    }
}

void launch_cur_part(const CurArgs& a, const SampleArgs& sa, int part, hipStream_t s) {
    const PivotArgs pa = pivot_args(sa);
    switch (a.dtype) {
        case RPLU_R32: cur_part_t<float>(a, pa, part, s); break;
        case RPLU_R64: cur_part_t<double>(a, pa, part, s); break;
        case RPLU_C64: cur_part_t<cf32>(a, pa, part, s); break;
        case RPLU_C128: cur_part_t<cf64>(a, pa, part, s); break;
    }
}

}  // namespace rplu
