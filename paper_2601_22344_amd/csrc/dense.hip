// Dense RPLU kernels (Alg. 1 with two-stage exact sampling, Sec. 4.1).
//
//   k_dense_init    row masses ||A_i,:||^2 (and column partials) of A
//   k_dense_sample  stop test, row draw, column draw of the pivot row,
//                   copy of the pivot row into U(t,:), pivot reciprocal
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
#include "common.hpp"
#include "cdf.hpp"
#include "launch.hpp"

namespace rplu {

// V consecutive elements moved as one access: 16 bytes when V*sizeof(T) == 16
// (aligned rows), otherwise a single element at its natural alignment, so
// that sizeof(Pack) == V*sizeof(T) and a store never touches a neighbour.
template <class T, int V>
struct alignas(V == 1 ? alignof(T) : 16) Pack { T v[V]; };
static_assert(sizeof(Pack<float, 1>) == 4 && sizeof(Pack<float, 4>) == 16, "pack size");
static_assert(sizeof(Pack<double, 1>) == 8 && sizeof(Pack<cf32, 1>) == 8, "pack size");

// ----------------------------------------------------------------- sweep

template <class T, int R, int V, bool INIT, bool COLMASS>
__global__ __launch_bounds__(256) void k_dense_sweep(
    T* __restrict__ S, int64_t lda, int n, int m,
    const T* __restrict__ U, int64_t ldu, T* __restrict__ L, int64_t ldl,
    const StepState* __restrict__ st, double* __restrict__ rowmass,
    double* __restrict__ colpart) {
    using W = typename Sc<T>::W;
    constexpr int BS = 256;
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
    double rp[R];
#pragma unroll
    for (int q = 0; q < R; ++q) rp[q] = 0.0;

    for (int64_t c = (int64_t)tid * V; c < m; c += (int64_t)BS * V) {
        double cp[V];
#pragma unroll
        for (int v = 0; v < V; ++v) cp[v] = 0.0;
        const bool full = c + V <= m;
        Pack<T, V> u;
        if constexpr (!INIT) {
            if (full) u = *reinterpret_cast<const Pack<T, V>*>(Ut + c);
            else {
#pragma unroll
                for (int v = 0; v < V; ++v) u.v[v] = (c + v < m) ? Ut[c + v] : Sc<T>::zero();
            }
        }
        Pack<T, V> s[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            if (q < nr) {
                const T* p = S + (int64_t)(r0 + q) * lda + c;
                if (full) s[q] = *reinterpret_cast<const Pack<T, V>*>(p);
                else {
#pragma unroll
                    for (int v = 0; v < V; ++v) s[q].v[v] = (c + v < m) ? p[v] : Sc<T>::zero();
                }
            }
        }
#pragma unroll
        for (int q = 0; q < R; ++q) {
            if (q < nr) {
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
                    const double m2 = (c + v < m) ? Sc<T>::mag2(s[q].v[v]) : 0.0;
                    rp[q] += m2;
                    if constexpr (COLMASS) cp[v] += m2;
                }
                if constexpr (!INIT) {
                    T* p = S + (int64_t)(r0 + q) * lda + c;
                    if (full) *reinterpret_cast<Pack<T, V>*>(p) = s[q];
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
            for (int v = 0; v < V; ++v) if (c + v < m) cpo[v] = cp[v];
        }
    }
    // row masses: wave sums, then a fixed-order sum over the 4 waves
    __shared__ double red[BS / RPLU_WAVE][R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        double v = wave_sum(rp[q]);
        if (lane == 0) red[wv][q] = v;
    }
    __syncthreads();
    if (tid < nr) {
        double v = red[0][tid];
#pragma unroll
        for (int w = 1; w < BS / RPLU_WAVE; ++w) v += red[w][tid];
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

// ---------------------------------------------------------------- sampler

template <class T>
__global__ __launch_bounds__(CDF_THREADS) void k_dense_sample(
    const T* __restrict__ S, int64_t lda, int n, int m,
    const double* __restrict__ rowmass, StepState* __restrict__ st,
    int32_t* __restrict__ piv, T* __restrict__ U, int64_t ldu,
    uint64_t seed, uint64_t stream, int kmax, double tol2,
    const int32_t* __restrict__ forced, double* __restrict__ trace,
    double* __restrict__ rowmass_out) {
    __shared__ CdfShared sh;
    __shared__ int s_flag;
    if (st->done) return;
    const int t = st->t;
    const int tid = threadIdx.x;

    const double Ttot = cdf_total(sh, n, [&](int e) { return rowmass[e]; });
    if (tid == 0) {
        int stop = 0, err = 0;
        double T0 = (t == 0) ? Ttot : st->T0;
        if (!isfinite(Ttot)) err = RPLU_E_NONFINITE;
        else if (Ttot == 0.0) stop = RPLU_STOP_EXHAUSTED;
        else if (tol2 > 0.0 && Ttot <= tol2 * T0) stop = RPLU_STOP_TOL;
        else if (t >= kmax) stop = tol2 > 0.0 ? RPLU_STOP_TOL_UNREACHED : RPLU_STOP_RANK;
        st->T = Ttot;
        if (t == 0) st->T0 = Ttot;
        if (err || stop) {
            st->error = err;
            st->stop = stop;
            st->done = 1;
        }
        s_flag = (err || stop) ? 1 : 0;
    }
    __syncthreads();
    if (s_flag) return;
    if (rowmass_out != nullptr)
        for (int e = tid; e < n; e += CDF_THREADS) rowmass_out[(int64_t)t * n + e] = rowmass[e];

    const Philox4 rnd = philox4x64_10((uint64_t)t, stream, 0, 0, seed, 0);
    const double u1 = unit_from_word(rnd.w[0]), u2 = unit_from_word(rnd.w[1]);

    const double tgt_i = u1 * Ttot;
    CdfPick pr = cdf_select(sh, n, [&](int e) { return rowmass[e]; }, tgt_i);
    const int i = forced ? forced[2 * t] : pr.idx;
    const int j_forced = forced ? forced[2 * t + 1] : 0;
    if (i < 0 || i >= n || j_forced < 0 || j_forced >= m) {   // bad forced pivot
        if (tid == 0) { st->error = RPLU_E_ARG; st->done = 1; }
        return;
    }
    const T* Si = S + (int64_t)i * lda;
    auto cm = [&](int e) { return Sc<T>::mag2(Si[e]); };
    const double Ti = cdf_total(sh, m, cm);
    const double tgt_j = u2 * Ti;
    CdfPick pc{0, 0.0, 0.0};
    if (Ti > 0.0 && isfinite(Ti)) pc = cdf_select(sh, m, cm, tgt_j);
    const int j = forced ? j_forced : pc.idx;

    const T a = Si[j];
    T* Ut = U + (int64_t)t * ldu;
    for (int e = tid; e < m; e += CDF_THREADS) Ut[e] = Si[e];
    if (tid == 0) {
        const double a2 = Sc<T>::mag2(a);
        int err = 0;
        if (!(a2 > 0.0)) err = isfinite(a2) ? RPLU_E_ZERO_PIVOT : RPLU_E_NONFINITE;
        if (err) {
            st->error = err;
            st->done = 1;
        } else {
            typename Sc<T>::W inv = winv(Sc<T>::widen(a));
            st->i = i;
            st->j = j;
            st->a_re = Sc<T>::re(a);
            st->a_im = Sc<T>::im(a);
            if constexpr (Sc<T>::cplx) { st->inv_re = inv.re; st->inv_im = inv.im; }
            else { st->inv_re = inv; st->inv_im = 0.0; }
            st->cur = t;
            st->t = t + 1;
            piv[2 * t] = i;
            piv[2 * t + 1] = j;
            if (trace != nullptr) {
                double* tr = trace + (int64_t)t * RPLU_TRACE_WORDS;
                tr[0] = Ttot; tr[1] = tgt_i; tr[2] = pr.lo; tr[3] = pr.hi;
                tr[4] = Ti; tr[5] = tgt_j; tr[6] = pc.lo; tr[7] = pc.hi;
                tr[8] = Sc<T>::re(a); tr[9] = Sc<T>::im(a);
                tr[10] = (double)i; tr[11] = (double)j;
            }
        }
    }
}

__global__ void k_state_init(StepState* st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        StepState z{};
        *st = z;
    }
}

// ---------------------------------------------------------------- launchers

template <class T, int R, int V, bool INIT, bool COLMASS>
static void launch_sweep_v(const DenseArgs& a, hipStream_t s) {
    const int nb = (int)((a.n + R - 1) / R);
    hipLaunchKernelGGL((k_dense_sweep<T, R, V, INIT, COLMASS>), dim3(nb), dim3(256), 0, s,
                       (T*)a.S, a.lda, (int)a.n, (int)a.m, (const T*)a.U, a.ldu, (T*)a.L, a.ldl,
                       a.st, a.rowmass, a.colpart);
}

template <class T, int R, bool INIT, bool COLMASS>
static void launch_sweep_t(const DenseArgs& a, hipStream_t s) {
    constexpr int VV = 16 / (int)sizeof(T);
    if (a.vec_ok) launch_sweep_v<T, R, VV, INIT, COLMASS>(a, s);
    else launch_sweep_v<T, R, 1, INIT, COLMASS>(a, s);
}

template <class T>
static void launch_sweep_dt(const DenseArgs& a, bool init, hipStream_t s) {
    if (a.colmass) {
        if (init) launch_sweep_t<T, DENSE_ROWS_COLMASS, true, true>(a, s);
        else launch_sweep_t<T, DENSE_ROWS_COLMASS, false, true>(a, s);
    } else {
        if (init) launch_sweep_t<T, DENSE_ROWS, true, false>(a, s);
        else launch_sweep_t<T, DENSE_ROWS, false, false>(a, s);
    }
}

void launch_dense_sweep(const DenseArgs& a, bool init, hipStream_t s) {
    switch (a.dtype) {
        case RPLU_R32: launch_sweep_dt<float>(a, init, s); break;
        case RPLU_R64: launch_sweep_dt<double>(a, init, s); break;
        case RPLU_C64: launch_sweep_dt<cf32>(a, init, s); break;
        case RPLU_C128: launch_sweep_dt<cf64>(a, init, s); break;
    }
}

int dense_row_block(bool colmass) { return colmass ? DENSE_ROWS_COLMASS : DENSE_ROWS; }

void launch_colmass_reduce(const DenseArgs& a, bool after_step, hipStream_t s) {
    const int nb = (int)((a.n + DENSE_ROWS_COLMASS - 1) / DENSE_ROWS_COLMASS);
    const int threads = 256;
    hipLaunchKernelGGL(k_colmass_reduce, dim3((unsigned)((a.m + threads - 1) / threads)),
                       dim3(threads), 0, s, a.colpart, nb, (int)a.m, a.st, after_step ? 1 : 0,
                       a.colmass_out, a.m, (int)a.kmax);
}

template <class T>
static void launch_sample_t(const DenseArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_dense_sample<T>, dim3(1), dim3(CDF_THREADS), 0, s, (const T*)a.S,
                       a.lda, (int)a.n, (int)a.m, a.rowmass, a.st, a.piv, (T*)a.U, a.ldu,
                       a.seed, a.stream, (int)a.kmax, a.tol2, a.forced, a.trace, a.rowmass_out);
}

void launch_dense_sample(const DenseArgs& a, hipStream_t s) {
    switch (a.dtype) {
        case RPLU_R32: launch_sample_t<float>(a, s); break;
        case RPLU_R64: launch_sample_t<double>(a, s); break;
        case RPLU_C64: launch_sample_t<cf32>(a, s); break;
        case RPLU_C128: launch_sample_t<cf64>(a, s); break;
    }
}

void launch_state_init(StepState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, s, st);
}

}  // namespace rplu
