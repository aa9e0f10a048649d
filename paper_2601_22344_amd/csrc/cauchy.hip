// Cauchy-like RPLU kernels (Alg. 3 with exact row masses, Sec. 5.1).
//
// S is never stored: s_ij = (G_i,: B_:,j) / (x_i - y_j) (eq. cauchy-like).
//
//   k_cauchy_mass    row masses sum_j |s_ij|^2 (Sec. 5.1, row-norm formula),
//                    all pairs, exact. Compute bound on FP64 vector ALUs:
//                    per pair a complex difference, |d|^2, the p-term product
//                    G_i,: B_:,j, its |.|^2 and one reciprocal. Each thread
//                    keeps RT target rows (x_i, G_i,:) in registers; the
//                    workgroup stages tiles of source columns (y_j, B_:,j) in
//                    LDS and every lane reads them as broadcasts. Columns are
//                    split over `splits` workgroup columns; the partial sums
//                    are added in split order by the sampler (deterministic).
//   k_cauchy_sample  stop test; row draw; regenerate the pivot row
//                    r = (G_i,: B) ./ (x_i - y) into U(t,:); column draw over
//                    |r|^2; pivot a = r_j and its reciprocal.
//   k_cauchy_update  column c = (G B_:,j) ./ (x - y_j), L(:,t) = c / a with
//                    L(i,t) = 1; G <- G - (1/a) c G_i,: and
//                    B <- B - (1/a) B_:,j r (eqs. generator_update_g/_b),
//                    G_i,: and B_:,j set to exactly 0. O((n + m) p).
#include "common.hpp"
#include "cdf.hpp"
#include "launch.hpp"

namespace rplu {

constexpr int CM_THREADS = 256;
constexpr int CM_RT = 2;                       // target rows per thread
constexpr int CM_ROWS = CM_THREADS * CM_RT;    // target rows per workgroup
constexpr int CM_TILE = 256;                   // source columns per LDS tile

// 1/d for d > 0 in FP64: hardware reciprocal estimate refined by two Newton
// steps r <- r + r (1 - d r), each of which roughly doubles the correct bits.
__device__ inline double rcp_refined(double d) {
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    return fma(r, e, r);
}

template <int P>
__global__ __launch_bounds__(CM_THREADS) void k_cauchy_mass(
    const cf64* __restrict__ x, const cf64* __restrict__ y, const cf64* __restrict__ G,
    const cf64* __restrict__ B, int n, int m, int cols_per_split,
    const StepState* __restrict__ st, double* __restrict__ partial) {
    if (st->done) return;
    __shared__ double sy_re[CM_TILE], sy_im[CM_TILE];
    __shared__ double sw[P == 1 ? CM_TILE : 1];                 // |b_j|^2 (p = 1)
    __shared__ cf64 sb[P == 1 ? 1 : P][P == 1 ? 1 : CM_TILE];   // b_lj (p > 1)
    const int tid = threadIdx.x;
    const int split = blockIdx.y;
    const int c_beg = split * cols_per_split;
    const int c_end = min(m, c_beg + cols_per_split);

    double xr[CM_RT], xi[CM_RT], acc[CM_RT], gscale[CM_RT];
    cf64 g[CM_RT][P];
#pragma unroll
    for (int q = 0; q < CM_RT; ++q) {
        const int r = blockIdx.x * CM_ROWS + q * CM_THREADS + tid;
        const bool ok = r < n;
        cf64 xv = ok ? x[r] : cf64{0.0, 0.0};
        xr[q] = xv.re;
        xi[q] = xv.im;
        acc[q] = 0.0;
        double gg = 0.0;
#pragma unroll
        for (int l = 0; l < P; ++l) {
            g[q][l] = ok ? G[(int64_t)r * P + l] : cf64{0.0, 0.0};
            gg += g[q][l].re * g[q][l].re + g[q][l].im * g[q][l].im;
        }
        gscale[q] = gg;
    }

    for (int c0 = c_beg; c0 < c_end; c0 += CM_TILE) {
        const int nt = min(CM_TILE, c_end - c0);
        __syncthreads();
        for (int e = tid; e < nt; e += CM_THREADS) {
            const cf64 yv = y[c0 + e];
            sy_re[e] = yv.re;
            sy_im[e] = yv.im;
            if constexpr (P == 1) {
                const cf64 b = B[c0 + e];
                sw[e] = b.re * b.re + b.im * b.im;
            } else {
#pragma unroll
                for (int l = 0; l < P; ++l) sb[l][e] = B[(int64_t)l * m + c0 + e];
            }
        }
        __syncthreads();
        for (int e = 0; e < nt; ++e) {
            const double yr = sy_re[e], yi = sy_im[e];
#pragma unroll
            for (int q = 0; q < CM_RT; ++q) {
                const double dr = xr[q] - yr, di = xi[q] - yi;
                const double d2 = fma(dr, dr, di * di);
                const double rinv = rcp_refined(d2);
                if constexpr (P == 1) {
                    acc[q] = fma(sw[e], rinv, acc[q]);
                } else {
                    double sr = 0.0, si = 0.0;
#pragma unroll
                    for (int l = 0; l < P; ++l) {
                        const cf64 b = sb[l][e];
                        sr = fma(g[q][l].re, b.re, sr);
                        sr = fma(-g[q][l].im, b.im, sr);
                        si = fma(g[q][l].re, b.im, si);
                        si = fma(g[q][l].im, b.re, si);
                    }
                    acc[q] = fma(fma(sr, sr, si * si), rinv, acc[q]);
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < CM_RT; ++q) {
        const int r = blockIdx.x * CM_ROWS + q * CM_THREADS + tid;
        if (r < n) partial[(int64_t)split * n + r] = (P == 1) ? gscale[q] * acc[q] : acc[q];
    }
}

template <int P>
__device__ inline cf64 gen_dot(const cf64* g, const cf64* __restrict__ B, int m, int c) {
    cf64 s{0.0, 0.0};
#pragma unroll
    for (int l = 0; l < P; ++l) {
        const cf64 b = B[(int64_t)l * m + c];
        s.re = fma(g[l].re, b.re, s.re);
        s.re = fma(-g[l].im, b.im, s.re);
        s.im = fma(g[l].re, b.im, s.im);
        s.im = fma(g[l].im, b.re, s.im);
    }
    return s;
}

// rowmass[e] = sum over splits s, in order, of partial[s][e].
__global__ __launch_bounds__(256) void k_cauchy_reduce(
    const double* __restrict__ partial, int splits, int n, const StepState* __restrict__ st,
    int kmax, double* __restrict__ rowmass, double* __restrict__ rowmass_out) {
    if (st->done) return;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    double v = 0.0;
    for (int s = 0; s < splits; ++s) v += partial[(int64_t)s * n + e];
    rowmass[e] = v;
    const int t = st->t;
    if (rowmass_out != nullptr && t < kmax) rowmass_out[(int64_t)t * n + e] = v;
}

template <int P>
__global__ __launch_bounds__(CDF_THREADS) void k_cauchy_sample(
    const cf64* __restrict__ x, const cf64* __restrict__ y, const cf64* __restrict__ G,
    const cf64* __restrict__ B, int n, int m, const double* __restrict__ rowmass,
    StepState* __restrict__ st, int32_t* __restrict__ piv,
    cf64* __restrict__ U, int64_t ldu, uint64_t seed, uint64_t stream, int kmax, double tol2,
    const int32_t* __restrict__ forced, double* __restrict__ trace) {
    __shared__ CdfShared sh;
    __shared__ int s_flag;
    __shared__ cf64 s_gi[P];
    if (st->done) return;
    const int t = st->t;
    const int tid = threadIdx.x;
    const double T = cdf_total(sh, n, [&](int e) { return rowmass[e]; });
    if (tid == 0) {
        int stop = 0, err = 0;
        const double T0 = (t == 0) ? T : st->T0;
        if (!isfinite(T)) err = RPLU_E_NONFINITE;
        else if (T == 0.0) stop = RPLU_STOP_EXHAUSTED;
        else if (tol2 > 0.0 && T <= tol2 * T0) stop = RPLU_STOP_TOL;
        else if (t >= kmax) stop = tol2 > 0.0 ? RPLU_STOP_TOL_UNREACHED : RPLU_STOP_RANK;
        st->T = T;
        if (t == 0) st->T0 = T;
        if (err || stop) { st->error = err; st->stop = stop; st->done = 1; }
        s_flag = (err || stop) ? 1 : 0;
    }
    __syncthreads();
    if (s_flag) return;
    const Philox4 rnd = philox4x64_10((uint64_t)t, stream, 0, 0, seed, 0);
    const double u1 = unit_from_word(rnd.w[0]), u2 = unit_from_word(rnd.w[1]);
    const double tgt_i = u1 * T;
    const CdfPick pr = cdf_select(sh, n, [&](int e) { return rowmass[e]; }, tgt_i);
    const int i = forced ? forced[2 * t] : pr.idx;
    const int j_forced = forced ? forced[2 * t + 1] : 0;
    if (i < 0 || i >= n || j_forced < 0 || j_forced >= m) {
        if (tid == 0) { st->error = RPLU_E_ARG; st->done = 1; }
        return;
    }
    if (tid < P) s_gi[tid] = G[(int64_t)i * P + tid];
    __syncthreads();
    cf64 gi[P];
#pragma unroll
    for (int l = 0; l < P; ++l) gi[l] = s_gi[l];
    const cf64 xi = x[i];
    cf64* Ut = U + (int64_t)t * ldu;
    for (int c = tid; c < m; c += CDF_THREADS) Ut[c] = cdiv(gen_dot<P>(gi, B, m, c), csub(xi, y[c]));
    __syncthreads();
    auto cm = [&](int e) { const cf64 v = Ut[e]; return v.re * v.re + v.im * v.im; };
    const double Ti = cdf_total(sh, m, cm);
    const double tgt_j = u2 * Ti;
    CdfPick pc{0, 0.0, 0.0};
    if (Ti > 0.0 && isfinite(Ti)) pc = cdf_select(sh, m, cm, tgt_j);
    const int j = forced ? j_forced : pc.idx;
    if (tid == 0) {
        const cf64 a = Ut[j];
        const double a2 = a.re * a.re + a.im * a.im;
        if (!(a2 > 0.0)) {
            st->error = isfinite(a2) ? RPLU_E_ZERO_PIVOT : RPLU_E_NONFINITE;
            st->done = 1;
        } else {
            const cf64 inv = winv(a);
            st->i = i; st->j = j;
            st->a_re = a.re; st->a_im = a.im;
            st->inv_re = inv.re; st->inv_im = inv.im;
            for (int l = 0; l < P; ++l) {
                st->gi[2 * l] = gi[l].re; st->gi[2 * l + 1] = gi[l].im;
                const cf64 b = B[(int64_t)l * m + j];
                st->bj[2 * l] = b.re; st->bj[2 * l + 1] = b.im;
            }
            st->cur = t;
            st->t = t + 1;
            piv[2 * t] = i;
            piv[2 * t + 1] = j;
            if (trace != nullptr) {
                double* tr = trace + (int64_t)t * RPLU_TRACE_WORDS;
                tr[0] = T; tr[1] = tgt_i; tr[2] = pr.lo; tr[3] = pr.hi;
                tr[4] = Ti; tr[5] = tgt_j; tr[6] = pc.lo; tr[7] = pc.hi;
                tr[8] = a.re; tr[9] = a.im; tr[10] = (double)i; tr[11] = (double)j;
            }
        }
    }
}

template <int P>
__global__ __launch_bounds__(256) void k_cauchy_update(
    const cf64* __restrict__ x, const cf64* __restrict__ y, cf64* __restrict__ G,
    cf64* __restrict__ B, int n, int m, const StepState* __restrict__ st,
    const cf64* __restrict__ U, int64_t ldu, cf64* __restrict__ L, int64_t ldl) {
    if (st->done) return;
    const int pi = st->i, pj = st->j, t = st->cur;
    const cf64 inv{st->inv_re, st->inv_im};
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < n) {
        const int r = (int)idx;
        cf64 g[P], bj[P], gi[P];
#pragma unroll
        for (int l = 0; l < P; ++l) {
            g[l] = G[(int64_t)r * P + l];
            bj[l] = cf64{st->bj[2 * l], st->bj[2 * l + 1]};
            gi[l] = cf64{st->gi[2 * l], st->gi[2 * l + 1]};
        }
        cf64 s{0.0, 0.0};
#pragma unroll
        for (int l = 0; l < P; ++l) s = cadd(s, wmul(g[l], bj[l]));
        const cf64 c = cdiv(s, csub(x[r], y[pj]));
        const cf64 l_r = wmul(c, inv);
        if (L != nullptr) L[(int64_t)t * ldl + r] = (r == pi) ? cf64{1.0, 0.0} : l_r;
#pragma unroll
        for (int l = 0; l < P; ++l) {
            cf64 v = (r == pi) ? cf64{0.0, 0.0} : csub(g[l], wmul(l_r, gi[l]));
            G[(int64_t)r * P + l] = v;
        }
    }
    if (idx < m) {
        const int c = (int)idx;
        const cf64 rc = U[(int64_t)t * ldu + c];
        const cf64 f = wmul(rc, inv);
#pragma unroll
        for (int l = 0; l < P; ++l) {
            const cf64 bjl{st->bj[2 * l], st->bj[2 * l + 1]};
            const cf64 b = B[(int64_t)l * m + c];
            B[(int64_t)l * m + c] = (c == pj) ? cf64{0.0, 0.0} : csub(b, wmul(bjl, f));
        }
    }
}

// ---------------------------------------------------------------- launchers

int cauchy_rows_per_block() { return CM_ROWS; }

template <int P>
static void mass_p(const CauchyArgs& a, hipStream_t s) {
    const int cps = (int)((a.m + a.splits - 1) / a.splits);
    dim3 grid((unsigned)((a.n + CM_ROWS - 1) / CM_ROWS), (unsigned)a.splits);
    hipLaunchKernelGGL(k_cauchy_mass<P>, grid, dim3(CM_THREADS), 0, s, (const cf64*)a.x,
                       (const cf64*)a.y, (const cf64*)a.G, (const cf64*)a.B, (int)a.n, (int)a.m,
                       cps, a.st, a.partial);
}

template <int P>
static void sample_p(const CauchyArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_cauchy_reduce, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s,
                       a.partial, a.splits, (int)a.n, a.st, (int)a.kmax, a.rowmass,
                       a.rowmass_out);
    hipLaunchKernelGGL(k_cauchy_sample<P>, dim3(1), dim3(CDF_THREADS), 0, s, (const cf64*)a.x,
                       (const cf64*)a.y, (const cf64*)a.G, (const cf64*)a.B, (int)a.n, (int)a.m,
                       a.rowmass, a.st, a.piv, (cf64*)a.U, a.ldu, a.seed,
                       a.stream, (int)a.kmax, a.tol2, a.forced, a.trace);
}

template <int P>
static void update_p(const CauchyArgs& a, hipStream_t s) {
    const int64_t work = a.n > a.m ? a.n : a.m;
    hipLaunchKernelGGL(k_cauchy_update<P>, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, s,
                       (const cf64*)a.x, (const cf64*)a.y, (cf64*)a.G, (cf64*)a.B, (int)a.n,
                       (int)a.m, a.st, (const cf64*)a.U, a.ldu, (cf64*)a.L, a.ldl);
}

#define RPLU_DISPATCH_P(fn)                         \
    switch (a.p) {                                  \
        case 1: fn<1>(a, s); break;                 \
        case 2: fn<2>(a, s); break;                 \
        case 3: fn<3>(a, s); break;                 \
        case 4: fn<4>(a, s); break;                 \
    }

void launch_cauchy_mass(const CauchyArgs& a, hipStream_t s) { RPLU_DISPATCH_P(mass_p) }
void launch_cauchy_sample(const CauchyArgs& a, hipStream_t s) { RPLU_DISPATCH_P(sample_p) }
void launch_cauchy_update(const CauchyArgs& a, hipStream_t s) { RPLU_DISPATCH_P(update_p) }

}  // namespace rplu
