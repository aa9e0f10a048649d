// Dense RPLU kernels (Alg. 1 with two-stage exact sampling, Sec. 4.1).
//
//   k_dense_sweep   (INIT) row masses ||A_i,:||^2 (and column partials) of A
//   k_dense_pivot   small matrices: the whole pivot draw of a step in one
//                   workgroup (row draw, pivot row i copied into U(t,:),
//                   column draw; pivot.hpp)
//   k_rows_draw, k_dense_pivrow_draw  larger ones: the row draw (sample.hip),
//                   then the pivot row copied by a wide kernel whose last
//                   workgroup draws the column
//   k_dense_sweep   S <- S - L(:,t) U(t,:) with row i and column j set to
//                   exactly 0, L(:,t) formed on the way, and the row masses
//                   of the NEW Schur complement reduced in the same pass
//   k_colmass_reduce  column masses from per-row-block partials
//
// Layout: S row-major (lda), L column-major (ldl), U row-major (ldu).
// The sweep is HBM bound: it reads and writes S once per step. A workgroup
// owns R consecutive rows and walks them in 16-byte packs per thread, so every
// row segment a wave touches is contiguous and each thread keeps R loads in
// flight. The U(t,:) pack is loaded once per column chunk and reused for the R
// rows. A row is reduced by one workgroup only, in an order fixed by (n, m),
// so the masses are deterministic and independent of scheduling.
#include <type_traits>

#include "common.hpp"
#include "cdf.hpp"
#include "launch.hpp"
#include "pivot.hpp"

namespace rplu {

// V consecutive elements moved as one access: 16 bytes when V*sizeof(T) == 16
// (aligned rows), otherwise a single element at its natural alignment, so
// that sizeof(Pack) == V*sizeof(T) and a store never touches a neighbour.
template <class T, int V>
struct alignas(V == 1 ? alignof(T) : 16) Pack { T v[V]; };
static_assert(sizeof(Pack<float, 1>) == 4 && sizeof(Pack<float, 4>) == 16, "pack size");
static_assert(sizeof(Pack<double, 1>) == 8 && sizeof(Pack<cf32, 1>) == 8, "pack size");

// Streaming (non-temporal) 16-byte accesses for S: each element of S is read
// and written once per sweep, so keeping it in the caches only evicts the
// U row and the state that every workgroup shares.
template <class T, int V>
__device__ inline Pack<T, V> ld_s(const T* p) {
    if constexpr (sizeof(Pack<T, V>) == 16) {
        const uint32_t* q = reinterpret_cast<const uint32_t*>(p);
        uint32_t w[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) w[k] = __builtin_nontemporal_load(q + k);
        Pack<T, V> r;
        __builtin_memcpy(&r, w, 16);
        return r;
    } else {
        return *reinterpret_cast<const Pack<T, V>*>(p);
    }
}

template <class T, int V>
__device__ inline void st_s(T* p, const Pack<T, V>& v) {
    if constexpr (sizeof(Pack<T, V>) == 16) {
        uint32_t w[4];
        __builtin_memcpy(w, &v, 16);
        uint32_t* q = reinterpret_cast<uint32_t*>(p);
#pragma unroll
        for (int k = 0; k < 4; ++k) __builtin_nontemporal_store(w[k], q + k);
    } else {
        *reinterpret_cast<Pack<T, V>*>(p) = v;
    }
}

// Whole workgroup: out[q] = the largest of rx[q] over all threads, for the
// nr rows of the block (a maximum is exact, so the order does not matter).
template <int R, int BS>
__device__ inline void row_max_reduce(double (&rx)[R], int nr, double* out) {
    __shared__ double mx[BS / RPLU_WAVE][R];
    const int lane = threadIdx.x % RPLU_WAVE, wv = threadIdx.x / RPLU_WAVE;
#pragma unroll
    for (int q = 0; q < R; ++q) {
        double v = rx[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_xor(v, off, RPLU_WAVE);
            v = o > v ? o : v;
        }
        if (lane == 0) mx[wv][q] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x < nr) {
        double v = mx[0][threadIdx.x];
#pragma unroll
        for (int w = 1; w < BS / RPLU_WAVE; ++w) v = mx[w][threadIdx.x] > v ? mx[w][threadIdx.x] : v;
        out[threadIdx.x] = v;
    }
}

// ----------------------------------------------------------------- sweep

// CMAX (RPLU_FLAG_CPLU): also the largest |S_ij|^2 of every row, into rowmax.
template <class T, int R, int BS, int V, bool INIT, bool COLMASS, bool CMAX>
__global__ __launch_bounds__(BS) void k_dense_sweep(
    T* __restrict__ S, int64_t lda, int n, int m,
    const T* __restrict__ U, int64_t ldu, T* __restrict__ L, int64_t ldl,
    const StepState* __restrict__ st, double* __restrict__ rowmass,
    double* __restrict__ colpart, double* __restrict__ rowmax) {
    using W = typename Sc<T>::W;
    const int tid = threadIdx.x;
    const int lane = tid % RPLU_WAVE, wv = tid / RPLU_WAVE;
    int pi = -1, pj = -1, t = 0;
    W inv{};
    if constexpr (!INIT) {
        if (st->done) return;
        pi = st->i;
        pj = st->j;
        t = st->cur;
        if constexpr (Sc<T>::cplx) inv = W{st->inv_re, st->inv_im};
        else inv = st->inv_re;
    }
    const int r0 = blockIdx.x * R;
    const int nr = min(R, n - r0);
    T lq[R];
    const T* Ut = U + (int64_t)t * ldu;
    if constexpr (!INIT) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int r = r0 + q;
            T l = Sc<T>::zero();
            if (q < nr) {
                if (r == pi) l = Sc<T>::one();
                else l = Sc<T>::narrow(wmul(Sc<T>::widen(S[(int64_t)r * lda + pj]), inv));
            }
            lq[q] = l;
            if (L != nullptr && tid == q && q < nr) L[(int64_t)t * ldl + r] = l;
        }
        __syncthreads();   // every S[r, j] is read before any store to it
    }
    double rp[R], rx[R];
#pragma unroll
    for (int q = 0; q < R; ++q) { rp[q] = 0.0; rx[q] = 0.0; }

    // One pack of V elements at column c for the R rows: update, exact zeros
    // on the pivot row and column, masses. FULL packs use unguarded 16-byte
    // streaming accesses; the single ragged pack at the end of a row (when
    // V does not divide m) is handled element by element.
    auto pack = [&](int64_t c, auto full_tag, auto allrows_tag) {
        constexpr bool FULL = decltype(full_tag)::value;
        constexpr bool ALLR = decltype(allrows_tag)::value;   // nr == R
        double cp[V];
#pragma unroll
        for (int v = 0; v < V; ++v) cp[v] = 0.0;
        Pack<T, V> u;
        if constexpr (!INIT) {
            if constexpr (FULL) u = *reinterpret_cast<const Pack<T, V>*>(Ut + c);
            else {
#pragma unroll
                for (int v = 0; v < V; ++v) u.v[v] = (c + v < m) ? Ut[c + v] : Sc<T>::zero();
            }
        }
        Pack<T, V> s[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            if (ALLR || q < nr) {
                const T* p = S + (int64_t)(r0 + q) * lda + c;
                if constexpr (FULL) s[q] = ld_s<T, V>(p);
                else {
#pragma unroll
                    for (int v = 0; v < V; ++v) s[q].v[v] = (c + v < m) ? p[v] : Sc<T>::zero();
                }
            }
        }
#pragma unroll
        for (int q = 0; q < R; ++q) {
            if (ALLR || q < nr) {
                if constexpr (!INIT) {
                    const bool prow = (r0 + q) == pi;
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        T x = Sc<T>::fms(s[q].v[v], lq[q], u.v[v]);
                        if (prow || c + v == pj) x = Sc<T>::zero();
                        s[q].v[v] = x;
                    }
                }
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    rp[q] = Sc<T>::mag2_add(rp[q], s[q].v[v]);   // 0 for padding
                    if constexpr (COLMASS || CMAX) {
                        const double m2 = Sc<T>::mag2(s[q].v[v]);
                        if constexpr (COLMASS) cp[v] += m2;
                        if constexpr (CMAX) rx[q] = m2 > rx[q] ? m2 : rx[q];
                    }
                }
                if constexpr (!INIT) {
                    T* p = S + (int64_t)(r0 + q) * lda + c;
                    if constexpr (FULL) st_s<T, V>(p, s[q]);
                    else {
#pragma unroll
                        for (int v = 0; v < V; ++v) if (c + v < m) p[v] = s[q].v[v];
                    }
                }
            }
        }
        if constexpr (COLMASS) {
            double* cpo = colpart + (int64_t)blockIdx.x * m + c;
#pragma unroll
            for (int v = 0; v < V; ++v) if (FULL || c + v < m) cpo[v] = cp[v];
        }
    };

    int64_t c = (int64_t)tid * V;
    if (nr == R) {                               // every block but maybe the last
        for (; c + V <= m; c += (int64_t)BS * V) pack(c, std::true_type{}, std::true_type{});
        if (c < m) pack(c, std::false_type{}, std::true_type{});   // ragged (m % V != 0)
    } else {
        for (; c + V <= m; c += (int64_t)BS * V) pack(c, std::true_type{}, std::false_type{});
        if (c < m) pack(c, std::false_type{}, std::false_type{});
    }

    // row masses: wave sums, then a fixed-order sum over the 4 waves
    __shared__ double red[BS / RPLU_WAVE][R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        double v = wave_sum(rp[q]);
        if (lane == 0) red[wv][q] = v;
    }
    if constexpr (CMAX) row_max_reduce<R, BS>(rx, nr, rowmax + r0);
    __syncthreads();
    if (tid < nr) {
        double v = red[0][tid];
#pragma unroll
        for (int w = 1; w < BS / RPLU_WAVE; ++w) v += red[w][tid];
        rowmass[r0 + tid] = v;
    }
}

// ---------------------------------------------------------- deferred sweep
//
// The eager sweep reads and writes all of S at every step. The deferred sweep
// keeps S^(tb) in memory and, at step t, reads it and applies the updates of
// steps tb..t in registers, in the eager sweep's order and with its
// operations (x <- fms(x, L(r,s), U(s,c)), and the exact zeros of row i_s and
// column j_s, which later steps leave 0), so every value, multiplier and mass
// is the eager sweep's bit for bit; it writes S^(t+1) back only when the window is full (LAZY_B steps)
// or at the last step kmax - 1, and the next draw moves tb there. Per step it
// reads S once and writes it every LAZY_B steps. The window's U rows come
// from U (L2-resident: LAZY_B rows), its multipliers from L.

// The window of step t as the workgroup sees it (uniform values).
template <class T>
struct LazyWin {
    int tb, w;                   // steps tb .. tb + w - 1
    int wi[LAZY_B], wj[LAZY_B];  // their pivots
};

template <class T>
__device__ inline LazyWin<T> lazy_window(const int32_t* __restrict__ piv, int tb, int t) {
    LazyWin<T> W;
    W.tb = tb;
    W.w = t - tb;
#pragma unroll
    for (int s = 0; s < LAZY_B; ++s) {
        W.wi[s] = s < W.w ? piv[2 * (tb + s)] : -1;
        W.wj[s] = s < W.w ? piv[2 * (tb + s) + 1] : -1;
    }
    return W;
}

// Row i of S^(t) from S^(tb) (the eager sweep's value): the pivot row of the
// draw kernels when the sweep is deferred.
template <class T>
struct LazyRowAcc {
    const T* Si;                 // row i of S^(tb)
    const T* U;
    int64_t ldu;
    int i;
    LazyWin<T> W;
    T l[LAZY_B];                 // L(i, tb + s)
    bool zr[LAZY_B];             // row i was the pivot row of step tb + s
    __host__ __device__ T operator()(int e) const {
        T x = Si[e];
#pragma unroll
        for (int s = 0; s < LAZY_B; ++s) {
            if (s < W.w) {
                const T y = Sc<T>::fms(x, l[s], U[(int64_t)(W.tb + s) * ldu + e]);
                x = (zr[s] || e == W.wj[s]) ? Sc<T>::zero() : y;
            }
        }
        return x;
    }
};

template <class T>
__device__ inline LazyRowAcc<T> lazy_row(const T* S, int64_t lda, const T* U, int64_t ldu,
                                         const T* L, int64_t ldl, const int32_t* piv, int i,
                                         int tb, int t) {
    LazyRowAcc<T> a;
    a.Si = S + (int64_t)i * lda;
    a.U = U;
    a.ldu = ldu;
    a.i = i;
    a.W = lazy_window<T>(piv, tb, t);
#pragma unroll
    for (int s = 0; s < LAZY_B; ++s) {
        a.l[s] = s < a.W.w ? L[(int64_t)(tb + s) * ldl + i] : Sc<T>::zero();
        a.zr[s] = a.W.wi[s] == i;
    }
    return a;
}

// FINAL = false: the sweep of step t = st->cur (the pending updates of steps
// tb..t-1 plus step t, whose multipliers L(:,t) are formed here); row masses
// (and column partials) of S^(t+1). FINAL = true: after the run, S^(st->t)
// written back if the last write-back is older; no masses.
template <class T, int R, int BS, int V, bool COLMASS, bool FINAL, bool CMAX>
__global__ __launch_bounds__(BS) void k_dense_lazy(
    T* __restrict__ S, int64_t lda, int n, int m,
    const T* __restrict__ U, int64_t ldu, T* __restrict__ L, int64_t ldl,
    const int32_t* __restrict__ piv, StepState* __restrict__ st, double* __restrict__ rowmass,
    double* __restrict__ colpart, int kmax, double* __restrict__ rowmax) {
    using W = typename Sc<T>::W;
    const int tid = threadIdx.x;
    const int lane = tid % RPLU_WAVE, wv = tid / RPLU_WAVE;
    int t, pi = -1, pj = -1;
    W inv{};
    if constexpr (FINAL) {
        if (st->error != 0) return;
        t = st->t;
        if (st->flushed == t) return;            // S^(t) is in memory already
    } else {
        if (st->done) return;
        t = st->cur;
        pi = st->i;
        pj = st->j;
        if constexpr (Sc<T>::cplx) inv = W{st->inv_re, st->inv_im};
        else inv = st->inv_re;
    }
    const int tb = st->t_base;
    // window steps tb .. tb + w - 1 (FINAL: up to t - 1; else up to t)
    const int w = FINAL ? t - tb : t - tb + 1;
    const bool flush = FINAL || w == LAZY_B || t + 1 == kmax;
    int wi[LAZY_B], wj[LAZY_B];
#pragma unroll
    for (int s = 0; s < LAZY_B; ++s) {
        const bool cur = !FINAL && s == w - 1;
        wi[s] = s < w ? (cur ? pi : piv[2 * (tb + s)]) : -1;
        wj[s] = s < w ? (cur ? pj : piv[2 * (tb + s) + 1]) : -1;
    }
    const int r0 = blockIdx.x * R;
    const int nr = min(R, n - r0);
    T lw[R][LAZY_B];
    bool zrow[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = r0 + min(q, nr - 1);
        bool z = false;
#pragma unroll
        for (int s = 0; s < LAZY_B; ++s) z = z || (s < w && wi[s] == r);
        zrow[q] = z;
#pragma unroll
        for (int s = 0; s < LAZY_B; ++s) {
            const bool older = FINAL ? s < w : s < w - 1;
            lw[q][s] = older ? L[(int64_t)(tb + s) * ldl + r] : Sc<T>::zero();
        }
        if constexpr (!FINAL) {
            // L(r, t) = S^(t)(r, j) / a: the window's updates on the stored
            // S(r, j), as the eager sweep reads it from memory
            T x = S[(int64_t)r * lda + pj];
#pragma unroll
            for (int s = 0; s < LAZY_B; ++s) {
                if (s < w - 1) {
                    const T y = Sc<T>::fms(x, lw[q][s], U[(int64_t)(tb + s) * ldu + pj]);
                    x = (wi[s] == r || wj[s] == pj) ? Sc<T>::zero() : y;
                }
            }
            const T l = (r == pi) ? Sc<T>::one() : Sc<T>::narrow(wmul(Sc<T>::widen(x), inv));
#pragma unroll
            for (int s = 0; s < LAZY_B; ++s)
                if (s == w - 1) lw[q][s] = l;
            if (tid == q && q < nr) L[(int64_t)t * ldl + r] = l;
        }
    }
    // every S[r, j] is read before any store to it; a sweep that writes
    // nothing back needs no barrier, and its first loads go out at once
    if (!FINAL && flush) __syncthreads();
    if (!flush) {
        // nothing is written: a block whose rows are all pivoted in the
        // window has masses 0 and need not read S
        bool all = true;
#pragma unroll
        for (int q = 0; q < R; ++q) all = all && (q >= nr || zrow[q]);
        if (all && !COLMASS) {
            if (tid < nr) {
                rowmass[r0 + tid] = 0.0;
                if constexpr (CMAX) rowmax[r0 + tid] = 0.0;
            }
            return;
        }
    }
    double rp[R], rx[R];
#pragma unroll
    for (int q = 0; q < R; ++q) { rp[q] = 0.0; rx[q] = 0.0; }

    // The column loop for a window of WW steps (a compile-time length: no
    // per-step branches, only the live multipliers in registers).
    auto cols = [&](auto wtag) {
        constexpr int WW = decltype(wtag)::value;
        auto pack = [&](int64_t c, auto full_tag, auto allrows_tag) {
            constexpr bool FULL = decltype(full_tag)::value;
            constexpr bool ALLR = decltype(allrows_tag)::value;
            double cp[V];
#pragma unroll
            for (int v = 0; v < V; ++v) cp[v] = 0.0;
            // The eager sweep sets column j_s to 0 at step s, and the later
            // steps leave it 0 (U(s', j_s) = 0 there), so zeroing the window's
            // pivot columns once, after the chain, gives the same values; the
            // mask is shared by the R rows.
            Pack<T, V> u[WW];
            bool zc[V];
#pragma unroll
            for (int v = 0; v < V; ++v) zc[v] = false;
#pragma unroll
            for (int s = 0; s < WW; ++s) {
                const int pv = wj[s] - (int)c;
#pragma unroll
                for (int v = 0; v < V; ++v) zc[v] = zc[v] || v == pv;
                const T* Us = U + (int64_t)(tb + s) * ldu + c;
                if constexpr (FULL) u[s] = *reinterpret_cast<const Pack<T, V>*>(Us);
                else {
#pragma unroll
                    for (int v = 0; v < V; ++v) u[s].v[v] = (c + v < m) ? Us[v] : Sc<T>::zero();
                }
            }
            Pack<T, V> x[R];
#pragma unroll
            for (int q = 0; q < R; ++q) {
                if ((ALLR || q < nr) && !zrow[q]) {
                    const T* p = S + (int64_t)(r0 + q) * lda + c;
                    if constexpr (FULL) x[q] = ld_s<T, V>(p);
                    else {
#pragma unroll
                        for (int v = 0; v < V; ++v) x[q].v[v] = (c + v < m) ? p[v] : Sc<T>::zero();
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < R; ++q) {
                if (ALLR || q < nr) {
                    if (zrow[q]) {
#pragma unroll
                        for (int v = 0; v < V; ++v) x[q].v[v] = Sc<T>::zero();
                    } else {
#pragma unroll
                        for (int s = 0; s < WW; ++s) {
#pragma unroll
                            for (int v = 0; v < V; ++v)
                                x[q].v[v] = Sc<T>::fms(x[q].v[v], lw[q][s], u[s].v[v]);
                        }
#pragma unroll
                        for (int v = 0; v < V; ++v)
                            if (zc[v]) x[q].v[v] = Sc<T>::zero();
                        if constexpr (!FINAL) {
#pragma unroll
                            for (int v = 0; v < V; ++v) {
                                rp[q] = Sc<T>::mag2_add(rp[q], x[q].v[v]);   // 0 for padding
                                if constexpr (COLMASS || CMAX) {
                                    const double m2 = Sc<T>::mag2(x[q].v[v]);
                                    if constexpr (COLMASS) cp[v] += m2;
                                    if constexpr (CMAX) rx[q] = m2 > rx[q] ? m2 : rx[q];
                                }
                            }
                        }
                    }
                    if (flush) {
                        T* p = S + (int64_t)(r0 + q) * lda + c;
                        if constexpr (FULL) st_s<T, V>(p, x[q]);
                        else {
#pragma unroll
                            for (int v = 0; v < V; ++v) if (c + v < m) p[v] = x[q].v[v];
                        }
                    }
                }
            }
            if constexpr (COLMASS && !FINAL) {
                double* cpo = colpart + (int64_t)blockIdx.x * m + c;
#pragma unroll
                for (int v = 0; v < V; ++v) if (FULL || c + v < m) cpo[v] = cp[v];
            }
        };
        int64_t c = (int64_t)tid * V;
        if (nr == R) {
            for (; c + V <= m; c += (int64_t)BS * V) pack(c, std::true_type{}, std::true_type{});
            if (c < m) pack(c, std::false_type{}, std::true_type{});
        } else {
            for (; c + V <= m; c += (int64_t)BS * V) pack(c, std::true_type{}, std::false_type{});
            if (c < m) pack(c, std::false_type{}, std::false_type{});
        }
    };
    static_assert(LAZY_B <= 8, "one case per window length");
    switch (w) {
        case 1: cols(std::integral_constant<int, 1>{}); break;
        case 2: cols(std::integral_constant<int, 2>{}); break;
        case 3: cols(std::integral_constant<int, 3>{}); break;
        case 4: cols(std::integral_constant<int, 4>{}); break;
        case 5: if constexpr (LAZY_B >= 5) cols(std::integral_constant<int, 5 <= LAZY_B ? 5 : 1>{}); break;
        case 6: if constexpr (LAZY_B >= 6) cols(std::integral_constant<int, 6 <= LAZY_B ? 6 : 1>{}); break;
        case 7: if constexpr (LAZY_B >= 7) cols(std::integral_constant<int, 7 <= LAZY_B ? 7 : 1>{}); break;
        case 8: if constexpr (LAZY_B >= 8) cols(std::integral_constant<int, 8 <= LAZY_B ? 8 : 1>{}); break;
        default: break;
    }
    if constexpr (FINAL) return;
    if (flush && blockIdx.x == 0 && tid == 0) st->flushed = t + 1;

    // row masses: wave sums, then a fixed-order sum over the waves (as eager)
    __shared__ double red[BS / RPLU_WAVE][R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        double v = wave_sum(rp[q]);
        if (lane == 0) red[wv][q] = v;
    }
    if constexpr (CMAX) row_max_reduce<R, BS>(rx, nr, rowmax + r0);
    __syncthreads();
    if (tid < nr) {
        double v = red[0][tid];
#pragma unroll
        for (int wq = 1; wq < BS / RPLU_WAVE; ++wq) v += red[wq][tid];
        rowmass[r0 + tid] = v;
    }
}

// Column masses: colmass[c] = sum over row blocks b (in order) of colpart[b][c].
// Row `st->t` of colmass_out (the masses the next draw sees) is written;
// rows at or beyond rows_cap are not stored.
__global__ void k_colmass_reduce(const double* __restrict__ colpart, int nb, int m,
                                 const StepState* __restrict__ st, int after_step,
                                 double* __restrict__ colmass_out, int64_t ld_out,
                                 int rows_cap) {
    if (after_step && st->done) return;
    const int row = after_step ? st->t : 0;
    if (row >= rows_cap) return;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= m) return;
    double v = 0.0;
    for (int b = 0; b < nb; ++b) v += colpart[(int64_t)b * m + c];
    colmass_out[(int64_t)row * ld_out + c] = v;
}

// ----------------------------------------------------------- pivot row

// Wide: copies row i of S into U(t,:) (one element per thread, coalesced)
// with the chunk totals of |S_i,e|^2; the last workgroup draws the column
// and commits the pivot (pivot.hpp).
template <class T, bool LAZY>
__global__ __launch_bounds__(CDF_THREADS) void k_dense_pivrow_draw(
    const T* __restrict__ S, int64_t lda, T* __restrict__ U, int64_t ldu, const T* __restrict__ L,
    int64_t ldl, PivotArgs pa, double* __restrict__ ct) {
    __shared__ WideShared sh;
    if (pa.st->done) return;
    const int t = pa.st->cur;
    wide_keep_words(sh, step_words(pa, t));
    const int i = pa.st->i;
    const T* Si = S + (int64_t)i * lda;
    T* Ut = U + (int64_t)t * ldu;
    const int e = blockIdx.x * WIDE_ELEMS + threadIdx.x;
    double v = 0.0;
    if (e < pa.m) {
        T x;
        if constexpr (LAZY) x = lazy_row<T>(S, lda, U, ldu, L, ldl, pa.piv, i, pa.st->t_base, t)(e);
        else x = Si[e];
        Ut[e] = x;
        v = Sc<T>::mag2(x);
    }
    wide_chunk_totals(sh, v, pa.m, ct);
    if (!wide_arrive_last(sh, &pa.st->arrive)) return;
    pivot_col_draw_ct<T, 0>(sh.cdf, pa, t, Ut, ct, nullptr, nullptr, wide_words(sh),
                            ColMassGlobal<T>{Ut});
}

// One workgroup: the whole pivot draw of a step (pivot.hpp), the pivot row
// copied from S into U(t,:); the same results as k_rows_draw followed by
// k_dense_pivrow_draw, in one launch.
template <class T, bool LAZY>
__global__ __launch_bounds__(CDF_THREADS) void k_dense_pivot(const T* __restrict__ S, int64_t lda,
                                                             T* __restrict__ U, int64_t ldu,
                                                             const T* __restrict__ L, int64_t ldl,
                                                             PivotArgs pa) {
    __shared__ PivotShared sh;
    if (pa.st->done) return;
    const int t = pa.st->t;
    const StopInputs in = stop_inputs(pa.st);
    // the window start this step will have (the draw moves it in the state)
    const int tb = (pa.st->flushed == t) ? t : pa.st->t_base;
    const int i = pivot_draw_row(sh, pa, t, in);
    if (i < 0) return;
    const T* Si = S + (int64_t)i * lda;
    if constexpr (LAZY) {
        const LazyRowAcc<T> row = lazy_row<T>(S, lda, U, ldu, L, ldl, pa.piv, i, tb, t);
        pivot_draw_col<T, 0>(sh, pa, t, U + (int64_t)t * ldu, nullptr, nullptr, row,
                             [](const T& v) { return v; });
    } else {
        pivot_draw_col<T, 0>(sh, pa, t, U + (int64_t)t * ldu, nullptr, nullptr,
                             [&](int e) { return Si[e]; }, [](const T& v) { return v; });
    }
}

// ------------------------------------------------- one launch per step
//
// Small matrices (n, m <= DENSE_STEP_MAX): the draws of a step and its sweep
// in one launch of ceil(n / DENSE_STEP_ROWS) workgroups. A step has two
// grid-wide dependencies (every row mass before the row draw, the pivot row
// before the column draw and the update), and in the two-kernel form each
// costs a launch. Here every workgroup makes both draws itself, on the same
// inputs with the same arithmetic (pivot_draw_row and pivot_draw_col), so
// each reaches the same pivot, and then sweeps its own rows: no workgroup
// waits for another. What keeps it free of races:
//   * each workgroup has its own copy of the step state (it reads and writes
//     only that one; slot 0, which workgroup 0 keeps, is read back);
//   * the row masses alternate between two buffers: step t reads slot t mod 2
//     and writes slot (t + 1) mod 2;
//   * the pivot row i is read by every workgroup during step t, so its owner
//     does not overwrite it: a pivoted row is marked dead, swept no more (its
//     entries would be exact zeros, its mass 0 and its multipliers +-0, which
//     is what the owner records), and zeroed in S after the run;
//   * workgroup 0 writes U(t,:), piv, the trace and the row-mass output; the
//     others keep their copy of the pivot row in a row of their own.
// The draws, multipliers, updates and row masses are those of k_dense_pivot
// and k_dense_sweep bit for bit: the same functions for the draws, and per
// row the sweep's 512-thread pack mapping, wave sums and wave order.
constexpr int STEP_HALF = DENSE_THREADS;                 // threads per row (the sweep's)

template <class T, int V>
__global__ __launch_bounds__(CDF_THREADS) void k_dense_step(
    T* __restrict__ S, int64_t lda, T* __restrict__ U, int64_t ldu, T* __restrict__ L,
    int64_t ldl, PivotArgs pa, StepState* __restrict__ states, double* __restrict__ masses,
    T* __restrict__ urows, int64_t ldur, uint8_t* __restrict__ dead) {
    using W = typename Sc<T>::W;
    __shared__ PivotShared sh;
    __shared__ double red[CDF_THREADS / RPLU_WAVE];
    __shared__ double pv[3];
    __shared__ int pvi[2];
    StepState* st = states + blockIdx.x;
    if (st->done) return;
    const int t = st->t;
    const int n = pa.n, m = pa.m;
    pa.st = st;
    pa.rowmass = masses + (int64_t)(t & 1) * n;
    if (blockIdx.x != 0) {
        pa.piv = nullptr;
        pa.trace = nullptr;
        pa.rowmass_out = nullptr;
    }
    T* Ut = blockIdx.x == 0 ? U + (int64_t)t * ldu : urows + (int64_t)blockIdx.x * ldur;
    const StopInputs in = stop_inputs(st);

    // This workgroup's rows do not depend on the draws: their packs are
    // loaded first, so that the loads run under the draws. Thread ht of half
    // h holds the packs at columns (ht + k STEP_HALF) V of rows r0 + 2q + h.
    constexpr int NQ = DENSE_STEP_ROWS / 2;
    constexpr int PK = (DENSE_STEP_MAX + STEP_HALF * V - 1) / (STEP_HALF * V);
    const int h = threadIdx.x / STEP_HALF, ht = threadIdx.x % STEP_HALF;
    const int r0 = blockIdx.x * DENSE_STEP_ROWS;
    Pack<T, V> pre[NQ][PK];
    bool live[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int r = r0 + 2 * q + h;
        live[q] = r < n && dead[r] == 0;
        const T* Sr = S + (int64_t)(live[q] ? r : 0) * lda;
#pragma unroll
        for (int k = 0; k < PK; ++k) {
            const int64_t c = (int64_t)(ht + k * STEP_HALF) * V;
            if (live[q] && c + V <= m) pre[q][k] = ld_s<T, V>(Sr + c);
            else {
#pragma unroll
                for (int v = 0; v < V; ++v)
                    pre[q][k].v[v] = (live[q] && c + v < m) ? Sr[c + v] : Sc<T>::zero();
            }
        }
    }

    const int i = pivot_draw_row(sh, pa, t, in);
    if (i < 0) return;
    const T* Si = S + (int64_t)i * lda;
    pivot_draw_col<T, 0>(sh, pa, t, Ut, nullptr, nullptr, [&](int e) { return Si[e]; },
                         [](const T& v) { return v; });
    // thread 0 committed the pivot (or recorded an error) in this state
    if (threadIdx.x == 0) {
        pvi[0] = st->done;
        pvi[1] = st->j;
        pv[0] = st->inv_re;
        pv[1] = st->inv_im;
    }
    __syncthreads();
    if (pvi[0]) return;
    const int pj = pvi[1];
    W inv;
    if constexpr (Sc<T>::cplx) inv = W{pv[0], pv[1]};
    else inv = pv[0];

    // the sweep of this workgroup's rows, two at a time (one per half), in
    // k_dense_sweep's order: packs by increasing column, the ragged pack of
    // a row (m mod V columns) element by element
    const int lane = threadIdx.x % RPLU_WAVE, wv = threadIdx.x / RPLU_WAVE;
    double* mnext = masses + (int64_t)((t + 1) & 1) * n;
    // the multipliers of all the workgroup's rows first: a row's S[r, j] is
    // read by every wave of its half, and one wave's store of the row's
    // packs (column j set to 0) must not overtake another wave's read
    T lq[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int r = r0 + 2 * q + h;
        lq[q] = Sc<T>::zero();
        if (r < n) {
            if (r == i) lq[q] = Sc<T>::one();
            else lq[q] = Sc<T>::narrow(wmul(Sc<T>::widen(live[q] ? S[(int64_t)r * lda + pj]
                                                                 : Sc<T>::zero()), inv));
            if (L != nullptr && ht == 0) L[(int64_t)t * ldl + r] = lq[q];
        }
    }
    __syncthreads();                                  // every S[r, j] read before any store
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int r = r0 + 2 * q + h;
        const bool valid = r < n;
        const bool prow = r == i;
        const bool gone = valid && !prow && !live[q];
        const T l = lq[q];
        double rp = 0.0;
        if (valid && !prow && !gone) {
            T* Sr = S + (int64_t)r * lda;
#pragma unroll
            for (int k = 0; k < PK; ++k) {
                const int64_t c = (int64_t)(ht + k * STEP_HALF) * V;
                if (c >= m) break;
                const bool full = c + V <= m;
                Pack<T, V> u, x = pre[q][k];
                if (full) u = *reinterpret_cast<const Pack<T, V>*>(Ut + c);
                else {
#pragma unroll
                    for (int v = 0; v < V; ++v) u.v[v] = (c + v < m) ? Ut[c + v] : Sc<T>::zero();
                }
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    T y = Sc<T>::fms(x.v[v], l, u.v[v]);
                    if (c + v == pj) y = Sc<T>::zero();
                    x.v[v] = y;
                    rp = Sc<T>::mag2_add(rp, y);
                }
                if (full) st_s<T, V>(Sr + c, x);
                else {
#pragma unroll
                    for (int v = 0; v < V; ++v) if (c + v < m) Sr[c + v] = x.v[v];
                }
            }
        }
        const double ws = wave_sum(rp);
        if (lane == 0) red[wv] = ws;
        __syncthreads();
        if (valid && ht == 0) {
            double v = red[h * (STEP_HALF / RPLU_WAVE)];
#pragma unroll
            for (int w = 1; w < STEP_HALF / RPLU_WAVE; ++w) v += red[h * (STEP_HALF / RPLU_WAVE) + w];
            mnext[r] = v;
            if (prow) dead[r] = 1;
        }
        __syncthreads();
    }
}

// Before the first step: every workgroup's state zeroed, no row dead.
__global__ void k_dense_step_init(StepState* __restrict__ states, int groups,
                                  uint8_t* __restrict__ dead, int n) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < groups) states[g] = StepState{};
    for (int r = g; r < n; r += gridDim.x * blockDim.x) dead[r] = 0;
}

// After the run: the pivoted rows of S set to exact zeros (the sweep leaves
// them as they were at their pivot step).
template <class T>
__global__ void k_dense_step_finish(T* __restrict__ S, int64_t lda, int n, int m,
                                    const uint8_t* __restrict__ dead) {
    const int r = blockIdx.x;
    if (r >= n || dead[r] == 0) return;
    for (int c = threadIdx.x; c < m; c += blockDim.x) S[(int64_t)r * lda + c] = Sc<T>::zero();
}

// ---------------------------------------------------------------- launchers

template <class T, int R, int V, bool INIT, bool COLMASS, bool CMAX>
static void launch_sweep_v(const DenseArgs& a, hipStream_t s) {
    constexpr int BS = COLMASS ? DENSE_THREADS_COLMASS : DENSE_THREADS;
    const int nb = (int)((a.n + R - 1) / R);
    hipLaunchKernelGGL((k_dense_sweep<T, R, BS, V, INIT, COLMASS, CMAX>), dim3(nb), dim3(BS), 0, s,
                       (T*)a.S, a.lda, (int)a.n, (int)a.m, (const T*)a.U, a.ldu, (T*)a.L, a.ldl,
                       a.st, a.rowmass, a.colpart, a.rowmax);
}

template <class T, int R, bool INIT, bool COLMASS, bool CMAX = false>
static void launch_sweep_t(const DenseArgs& a, hipStream_t s) {
    constexpr int VV = 16 / (int)sizeof(T);
    if (a.vec_ok) launch_sweep_v<T, R, VV, INIT, COLMASS, CMAX>(a, s);
    else launch_sweep_v<T, R, 1, INIT, COLMASS, CMAX>(a, s);
}

// (the host never asks for column masses with CPLU's row maxima)
template <class T>
static void launch_sweep_dt(const DenseArgs& a, bool init, hipStream_t s) {
    if (a.rowmax) {
        if (init) launch_sweep_t<T, DENSE_ROWS, true, false, true>(a, s);
        else launch_sweep_t<T, DENSE_ROWS, false, false, true>(a, s);
    } else if (a.colmass) {
        if (init) launch_sweep_t<T, DENSE_ROWS_COLMASS, true, true>(a, s);
        else launch_sweep_t<T, DENSE_ROWS_COLMASS, false, true>(a, s);
    } else {
        if (init) launch_sweep_t<T, DENSE_ROWS, true, false>(a, s);
        else launch_sweep_t<T, DENSE_ROWS, false, false>(a, s);
    }
}

template <class T, int R, int V, bool COLMASS, bool FINAL, bool CMAX>
static void launch_lazy_v(const DenseArgs& a, hipStream_t s) {
    constexpr int BS = COLMASS ? DENSE_THREADS_COLMASS : DENSE_THREADS;
    const int nb = (int)((a.n + R - 1) / R);
    hipLaunchKernelGGL((k_dense_lazy<T, R, BS, V, COLMASS, FINAL, CMAX>), dim3(nb), dim3(BS), 0, s,
                       (T*)a.S, a.lda, (int)a.n, (int)a.m, (const T*)a.U, a.ldu, (T*)a.L, a.ldl,
                       a.piv, a.st, a.rowmass, a.colpart, (int)a.kmax, a.rowmax);
}

// (column masses take the eager sweep: the host never sets lazy with them;
// the final write-back forms no masses)
template <class T, bool FINAL>
static void launch_lazy_dt(const DenseArgs& a, hipStream_t s) {
    constexpr int VV = 16 / (int)sizeof(T);
    constexpr int R = Sc<T>::cplx ? DENSE_LAZY_ROWS / 2 : DENSE_LAZY_ROWS;
    if (!FINAL && a.rowmax) {
        if (a.vec_ok) launch_lazy_v<T, R, VV, false, FINAL, true>(a, s);
        else launch_lazy_v<T, R, 1, false, FINAL, true>(a, s);
    } else {
        if (a.vec_ok) launch_lazy_v<T, R, VV, false, FINAL, false>(a, s);
        else launch_lazy_v<T, R, 1, false, FINAL, false>(a, s);
    }
}

template <bool FINAL>
static void launch_lazy(const DenseArgs& a, hipStream_t s) {
    switch (a.dtype) {
        case RPLU_R32: launch_lazy_dt<float, FINAL>(a, s); break;
        case RPLU_R64: launch_lazy_dt<double, FINAL>(a, s); break;
        case RPLU_C64: launch_lazy_dt<cf32, FINAL>(a, s); break;
        case RPLU_C128: launch_lazy_dt<cf64, FINAL>(a, s); break;
    }
}

void launch_dense_sweep(const DenseArgs& a, bool init, hipStream_t s) {
    if (!init && a.lazy) { launch_lazy<false>(a, s); return; }
    switch (a.dtype) {
        case RPLU_R32: launch_sweep_dt<float>(a, init, s); break;
        case RPLU_R64: launch_sweep_dt<double>(a, init, s); break;
        case RPLU_C64: launch_sweep_dt<cf32>(a, init, s); break;
        case RPLU_C128: launch_sweep_dt<cf64>(a, init, s); break;
    }
}

void launch_dense_flush(const DenseArgs& a, hipStream_t s) {
    if (a.lazy) launch_lazy<true>(a, s);
}

int dense_row_block(bool colmass) { return colmass ? DENSE_ROWS_COLMASS : DENSE_ROWS; }

void launch_dense_step_init(const DenseArgs& a, const DenseStepArgs& d, hipStream_t s) {
    const int nthr = 256;
    const int64_t work = a.n > d.groups ? a.n : d.groups;
    hipLaunchKernelGGL(k_dense_step_init, dim3((unsigned)((work + nthr - 1) / nthr)), dim3(nthr), 0, s,
                       d.states, d.groups, d.dead, (int)a.n);
}

template <class T>
static void step_t(const DenseArgs& a, const SampleArgs& sa, const DenseStepArgs& d, hipStream_t s) {
    constexpr int VV = 16 / (int)sizeof(T);
    PivotArgs pa = pivot_args(sa);
    if (a.vec_ok)
        hipLaunchKernelGGL((k_dense_step<T, VV>), dim3((unsigned)d.groups), dim3(CDF_THREADS), 0, s,
                           (T*)a.S, a.lda, (T*)a.U, a.ldu, (T*)a.L, a.ldl, pa, d.states, d.masses,
                           (T*)d.urows, d.ldur, d.dead);
    else
        hipLaunchKernelGGL((k_dense_step<T, 1>), dim3((unsigned)d.groups), dim3(CDF_THREADS), 0, s,
                           (T*)a.S, a.lda, (T*)a.U, a.ldu, (T*)a.L, a.ldl, pa, d.states, d.masses,
                           (T*)d.urows, d.ldur, d.dead);
}

void launch_dense_step(const DenseArgs& a, const SampleArgs& sa, const DenseStepArgs& d,
                       hipStream_t s) {
    switch (a.dtype) {
        case RPLU_R32: step_t<float>(a, sa, d, s); break;
        case RPLU_R64: step_t<double>(a, sa, d, s); break;
        case RPLU_C64: step_t<cf32>(a, sa, d, s); break;
        case RPLU_C128: step_t<cf64>(a, sa, d, s); break;
    }
}

template <class T>
static void step_finish_t(const DenseArgs& a, const DenseStepArgs& d, hipStream_t s) {
    hipLaunchKernelGGL((k_dense_step_finish<T>), dim3((unsigned)a.n), dim3(256), 0, s, (T*)a.S,
                       a.lda, (int)a.n, (int)a.m, d.dead);
}

void launch_dense_step_finish(const DenseArgs& a, const DenseStepArgs& d, hipStream_t s) {
    switch (a.dtype) {
        case RPLU_R32: step_finish_t<float>(a, d, s); break;
        case RPLU_R64: step_finish_t<double>(a, d, s); break;
        case RPLU_C64: step_finish_t<cf32>(a, d, s); break;
        case RPLU_C128: step_finish_t<cf64>(a, d, s); break;
    }
}


void launch_colmass_sum(const double* part, int nb, int64_t m, StepState* st, double* out,
                        int64_t ld_out, int64_t rows_cap, hipStream_t s) {
    hipLaunchKernelGGL(k_colmass_reduce, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, part,
                       nb, (int)m, st, 1, out, ld_out, (int)rows_cap);
}

void launch_colmass_reduce(const DenseArgs& a, bool after_step, hipStream_t s) {
    const int nb = (int)((a.n + DENSE_ROWS_COLMASS - 1) / DENSE_ROWS_COLMASS);
    const int threads = 256;
    hipLaunchKernelGGL(k_colmass_reduce, dim3((unsigned)((a.m + threads - 1) / threads)),
                       dim3(threads), 0, s, a.colpart, nb, (int)a.m, a.st, after_step ? 1 : 0,
                       a.colmass_out, a.m, (int)a.kmax);
}

template <class T>
static void pivot_t(const DenseArgs& a, const SampleArgs& sa, hipStream_t s) {
    if (a.lazy)
        hipLaunchKernelGGL((k_dense_pivot<T, true>), dim3(1), dim3(CDF_THREADS), 0, s,
                           (const T*)a.S, a.lda, (T*)a.U, a.ldu, (const T*)a.L, a.ldl,
                           pivot_args(sa));
    else
        hipLaunchKernelGGL((k_dense_pivot<T, false>), dim3(1), dim3(CDF_THREADS), 0, s,
                           (const T*)a.S, a.lda, (T*)a.U, a.ldu, (const T*)a.L, a.ldl,
                           pivot_args(sa));
}

void launch_dense_pivot(const DenseArgs& a, const SampleArgs& sa, hipStream_t s) {
    switch (a.dtype) {
        case RPLU_R32: pivot_t<float>(a, sa, s); break;
        case RPLU_R64: pivot_t<double>(a, sa, s); break;
        case RPLU_C64: pivot_t<cf32>(a, sa, s); break;
        case RPLU_C128: pivot_t<cf64>(a, sa, s); break;
    }
}

template <class T>
static void pivrow_draw_t(const DenseArgs& a, const SampleArgs& sa, hipStream_t s) {
    if (a.lazy)
        hipLaunchKernelGGL((k_dense_pivrow_draw<T, true>), dim3(wide_blocks(a.m)), dim3(CDF_THREADS),
                           0, s, (const T*)a.S, a.lda, (T*)a.U, a.ldu, (const T*)a.L, a.ldl,
                           pivot_args(sa), a.ct_col);
    else
        hipLaunchKernelGGL((k_dense_pivrow_draw<T, false>), dim3(wide_blocks(a.m)), dim3(CDF_THREADS),
                           0, s, (const T*)a.S, a.lda, (T*)a.U, a.ldu, (const T*)a.L, a.ldl,
                           pivot_args(sa), a.ct_col);
}

void launch_dense_pivrow_draw(const DenseArgs& a, const SampleArgs& sa, hipStream_t s) {
    switch (a.dtype) {
        case RPLU_R32: pivrow_draw_t<float>(a, sa, s); break;
        case RPLU_R64: pivrow_draw_t<double>(a, sa, s); break;
        case RPLU_C64: pivrow_draw_t<cf32>(a, sa, s); break;
        case RPLU_C128: pivrow_draw_t<cf64>(a, sa, s); break;
    }
}

}  // namespace rplu
