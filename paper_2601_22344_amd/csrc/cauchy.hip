// Cauchy-like RPLU kernels (Alg. 3 with exact row masses, Sec. 5.1).
//
// S is never stored: s_ij = (G_i,: B_:,j) / (x_i - y_j) (eq. cauchy-like).
//
//   k_cauchy_mass1, k_cauchy_mass  row masses sum_j |s_ij|^2 (Sec. 5.1,
//                    row-norm formula), all pairs, exact. Compute bound on
//                    FP64 vector ALUs: per pair |x_i - y_j|^2, the p-term
//                    product G_i,: B_:,j, its |.|^2 and one reciprocal. Each
//                    thread keeps 2 target rows (x_i, G_i,:) in registers;
//                    source columns come as uniform loads (p = 1, with a
//                    centred short form of |x - y|^2 where it is accurate)
//                    or LDS broadcasts (p > 1); eight columns share one
//                    reciprocal. Columns are split over `splits` workgroup
//                    columns; the partial sums are added in a fixed order by
//                    k_cauchy_reduce_draw (deterministic).
//   k_cauchy_reduce_draw  row masses from the split partials (two halves of
//                    the splits per row, each in order) and their chunk
//                    totals; the last workgroup runs the stop test and draws
//                    the row (pivot.hpp)
//   k_cauchy_rowgen_draw  regenerates the pivot row
//                    r = (G_i,: B) ./ (x_i - y) into U(t,:) with the chunk
//                    totals of |r|^2; the last workgroup draws the column
//   k_cauchy_transpose  optional column masses (the same all-pairs sums with
//                    rows and columns exchanged, in k_cauchy_mass): G^T, B^T
//   k_cauchy_frame   once per run (p = 1): the box of y, its centre and the
//                    per-column data of k_cauchy_mass1
//   k_cauchy_update  column c = (G B_:,j) ./ (x - y_j), L(:,t) = c / a with
//                    L(i,t) = 1; G <- G - (1/a) c G_i,: and
//                    B <- B - (1/a) B_:,j r (eqs. generator_update_g/_b),
//                    G_i,: and B_:,j set to exactly 0. O((n + m) p).
#include "common.hpp"
#include "cdf.hpp"
#include "launch.hpp"
#include "pivot.hpp"
#include "runtime.hpp"

namespace rplu {

constexpr int CM_THREADS = 512;
constexpr int CM_RT = 2;                       // target rows per thread
constexpr int CM_ROWS = CM_THREADS * CM_RT;    // target rows per workgroup
constexpr int CM_TILE = 256;                   // columns per tile (LDS staging for p > 1;
                                               // the unit of the exactness check)
constexpr int CM_GRP = 8;                      // columns sharing one reciprocal

// 1/d for d > 0 to about 2^-48 relative: the hardware estimate (~24 bits)
// refined by one Newton step. Enough for masses, which only feed the draws.
__device__ inline double rcp_1nr(double d) {
    const double r = __builtin_amdgcn_rcp(d);
    return fma(r, fma(-d, r, 1.0), r);
}

// |G_i,: B_:,j|^2 for one target row (registers) and one source column (LDS).
template <int P>
__device__ inline double gb_mag2(const cf64* g, const cf64 (*sb)[CM_TILE], int e) {
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int l = 0; l < P; ++l) {
        const cf64 b = sb[l][e];
        sr = fma(g[l].re, b.re, sr);
        sr = fma(-g[l].im, b.im, sr);
        si = fma(g[l].re, b.im, si);
        si = fma(g[l].im, b.re, si);
    }
    return fma(sr, sr, si * si);
}

// Row masses sum_j w_ij / d_ij with d_ij = |x_i - y_j|^2 and w_ij =
// |G_i,: B_:,j|^2 (for p = 1, |g_i|^2 |b_j|^2: the factor |g_i|^2 is taken
// out of the sum).
//
// Eight columns share one reciprocal: sum_u w_u / d_u = N / D with
// D = prod_u d_u and N = sum_u w_u prod_{v != u} d_v, formed as a pairwise
// tree (N01 = w0 d1 + w1 d0, D01 = d0 d1, and so on up the tree). This takes
// the per-pair cost from one reciprocal and its Newton step to an eighth of
// that. A tile is first summed this way while recording, without branching,
// whether any group had D outside [2^-1000, 2^1000] or a non-finite N
// (extreme magnitudes, or x_i == y_j); only then is that thread's tile sum
// for the row recomputed term by term, so the result is the plain sum for
// every input.
__device__ inline void mass_group(const double (&d)[CM_GRP], const double (&w)[CM_GRP], bool& ok,
                                  double& acc) {
    const double d01 = d[0] * d[1], d23 = d[2] * d[3];
    const double d45 = d[4] * d[5], d67 = d[6] * d[7];
    const double D03 = d01 * d23, D47 = d45 * d67;
    const double D = D03 * D47;
    const double N03 = fma(fma(w[0], d[1], w[1] * d[0]), d23, fma(w[2], d[3], w[3] * d[2]) * d01);
    const double N47 = fma(fma(w[4], d[5], w[5] * d[4]), d67, fma(w[6], d[7], w[7] * d[6]) * d45);
    const double N = fma(N03, D47, N47 * D03);
    ok = ok & (D >= 0x1p-1000) & (D <= 0x1p+1000) & (fabs(N) <= 0x1p+1000);
    acc = fma(N, rcp_1nr(D), acc);
}

// ------------------------------------------------------- LDS-staged form

// Each thread keeps CM_RT target rows (x_i, G_i,:) in registers; the
// workgroup stages tiles of source columns (y_j, B_:,j) in LDS and every
// lane reads them as broadcasts. The row masses for p >= 2, and the column
// masses for every p (the same sums with the roles of (x, G) and (y, B^T)
// exchanged).
template <int P>
__device__ inline void mass_tile_exact(double& acc_t, double xr, double xi, const cf64* sy,
                                       const cf64* g, const cf64 (*sb)[CM_TILE], int nt) {
    double s = 0.0;
    for (int e = 0; e < nt; ++e) {
        const double w = gb_mag2<P>(g, sb, e);
        const double a = xr - sy[e].re, b = xi - sy[e].im;
        s = fma(w, rcp_refined(fma(a, a, b * b)), s);
    }
    acc_t = s;
}

template <int P>
__global__ __launch_bounds__(CM_THREADS) void k_cauchy_mass(
    const cf64* __restrict__ x, const cf64* __restrict__ y, const cf64* __restrict__ G,
    const cf64* __restrict__ B, int n, int m, int cols_per_split,
    const StepState* __restrict__ st, double* __restrict__ partial) {
    if (st->done) return;
    __shared__ cf64 sy[CM_TILE];
    __shared__ cf64 sb[P][CM_TILE];
    const int tid = threadIdx.x;
    const int split = blockIdx.y;
    const int c_beg = split * cols_per_split;
    const int c_end = min(m, c_beg + cols_per_split);

    double xr[CM_RT], xi[CM_RT], acc[CM_RT];
    cf64 g[CM_RT][P];
#pragma unroll
    for (int q = 0; q < CM_RT; ++q) {
        const int r = blockIdx.x * CM_ROWS + q * CM_THREADS + tid;
        const bool ok = r < n;
        const cf64 xv = ok ? x[r] : cf64{0.0, 0.0};
        xr[q] = xv.re;
        xi[q] = xv.im;
        acc[q] = 0.0;
#pragma unroll
        for (int l = 0; l < P; ++l) g[q][l] = ok ? G[(int64_t)r * P + l] : cf64{0.0, 0.0};
    }

    for (int c0 = c_beg; c0 < c_end; c0 += CM_TILE) {
        const int nt = min(CM_TILE, c_end - c0);
        __syncthreads();
        for (int e = tid; e < nt; e += CM_THREADS) {
            sy[e] = y[c0 + e];
#pragma unroll
            for (int l = 0; l < P; ++l) sb[l][e] = B[(int64_t)l * m + c0 + e];
        }
        __syncthreads();
        double acc_t[CM_RT];
        bool ok[CM_RT];
#pragma unroll
        for (int q = 0; q < CM_RT; ++q) { acc_t[q] = 0.0; ok[q] = true; }
        const int ng = nt / CM_GRP * CM_GRP;
        for (int e = 0; e < ng; e += CM_GRP) {
            cf64 yy[CM_GRP];
#pragma unroll
            for (int u = 0; u < CM_GRP; ++u) yy[u] = sy[e + u];
#pragma unroll
            for (int q = 0; q < CM_RT; ++q) {
                double d[CM_GRP], w[CM_GRP];
#pragma unroll
                for (int u = 0; u < CM_GRP; ++u) {
                    const double a = xr[q] - yy[u].re, b = xi[q] - yy[u].im;
                    d[u] = fma(a, a, b * b);
                    w[u] = gb_mag2<P>(g[q], sb, e + u);
                }
                mass_group(d, w, ok[q], acc_t[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < CM_RT; ++q) {
            if (__builtin_expect(!ok[q], 0))      // rare: recompute this tile term by term
                mass_tile_exact<P>(acc_t[q], xr[q], xi[q], sy, g[q], sb, ng);
            for (int e = ng; e < nt; ++e) {       // ragged tail of the tile
                const double w = gb_mag2<P>(g[q], sb, e);
                const double a = xr[q] - sy[e].re, b = xi[q] - sy[e].im;
                acc_t[q] = fma(w, rcp_refined(fma(a, a, b * b)), acc_t[q]);
            }
            acc[q] += acc_t[q];
        }
    }
#pragma unroll
    for (int q = 0; q < CM_RT; ++q) {
        const int r = blockIdx.x * CM_ROWS + q * CM_THREADS + tid;
        if (r < n) partial[(int64_t)split * n + r] = acc[q];
    }
}

// --------------------------------------------------------------- p = 1

// For p = 1 the source column j is three numbers besides w_j = |b_j|^2, the
// same for every lane: the kernel reads them straight from memory with
// uniform (scalar) loads into scalar registers, which FP64 instructions take
// as operands, so no LDS staging or broadcast reads remain and the vector
// ALUs do only the pair arithmetic. With c the centre of the bounding box of
// y, |x - y|^2 = |x - c|^2 + |y - c|^2 - 2 Re((x - c) conj(y - c)); with
// -2(x - c) and |x - c|^2 per row in registers and y - c, |y - c|^2 per
// column precomputed (MassCol), a pair costs an add and two FMAs instead of
// two subtractions, a multiply and an FMA. The rounding error of that form is
// a few units of 2^-53 of |x - c|^2 + |y - c|^2 rather than of |x - y|^2, so
// a wave takes it only when, for each of its rows x, the distance from x to
// the bounding box of y proves |x - c|^2 + max_j |y_j - c|^2 <= 64 min_j
// |x - y_j|^2: the relative error of each |x - y|^2 then stays under 400
// units of 2^-53 (4.4e-14, the draws being compared at 1e-12). Other waves,
// and the exact recomputation of a flagged tile, use the plain form from y
// itself.
struct MassCol {
    double yr, yi;      // y_j - c
    double sy;          // |y_j - c|^2
    double w;           // |b_j|^2, rewritten by the generator update
};

struct MassFrame {
    double cr, ci;                  // c: centre of the bounding box of y
    double yr0, yr1, yi0, yi1;      // the box
    double R2;                      // max_j |y_j - c|^2
    double pad;
};

constexpr double CM_SHORT_RATIO = 0x1p-6;

// Ranges under which the 16-column form of k_cauchy_mass1 can neither
// overflow nor underflow: with every |x - y|^2 in [2^-28, 2^28] and every
// w_j = |b_j|^2 zero or in [2^-500, 2^500], each product of up to 16
// distances lies in [2^-449, 2^449] and each term w_u prod_{v != u} d_v in
// [2^-921, 2^921].
constexpr double CM_D_LO = 0x1p-28, CM_D_HI = 0x1p+28;
constexpr double CM_W_LO = 0x1p-500, CM_W_HI = 0x1p+500;

__device__ inline bool w_in_range(double w) { return w == 0.0 || (w >= CM_W_LO && w <= CM_W_HI); }

__device__ inline double wave_min(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, RPLU_WAVE));
    return v;
}

__device__ inline double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, RPLU_WAVE));
    return v;
}

// One workgroup, once per run: the box of y, its centre, R2 and MassCol.
__global__ __launch_bounds__(1024) void k_cauchy_frame(const cf64* __restrict__ y,
                                                       const cf64* __restrict__ B, int m,
                                                       MassFrame* __restrict__ fr,
                                                       MassCol* __restrict__ col,
                                                       StepState* __restrict__ st) {
    __shared__ double red[5][16];
    __shared__ double cen[2];
    const int tid = threadIdx.x, lane = tid % RPLU_WAVE, w = tid / RPLU_WAVE;
    double r0 = INFINITY, r1 = -INFINITY, i0 = INFINITY, i1 = -INFINITY;
    for (int j = tid; j < m; j += 1024) {
        const cf64 v = y[j];
        r0 = fmin(r0, v.re); r1 = fmax(r1, v.re);
        i0 = fmin(i0, v.im); i1 = fmax(i1, v.im);
    }
    r0 = wave_min(r0); r1 = wave_max(r1); i0 = wave_min(i0); i1 = wave_max(i1);
    if (lane == 0) { red[0][w] = r0; red[1][w] = r1; red[2][w] = i0; red[3][w] = i1; }
    __syncthreads();
    if (tid == 0) {
        for (int q = 1; q < 16; ++q) {
            r0 = fmin(r0, red[0][q]); r1 = fmax(r1, red[1][q]);
            i0 = fmin(i0, red[2][q]); i1 = fmax(i1, red[3][q]);
        }
        cen[0] = 0.5 * (r0 + r1);
        cen[1] = 0.5 * (i0 + i1);
        fr->cr = cen[0]; fr->ci = cen[1];
        fr->yr0 = r0; fr->yr1 = r1; fr->yi0 = i0; fr->yi1 = i1;
        fr->pad = 0.0;
    }
    __syncthreads();
    const double cr = cen[0], ci = cen[1];
    double smax = 0.0;
    bool bad = false;
    for (int j = tid; j < m; j += 1024) {
        const cf64 v = y[j], b = B[j];
        const double yr = v.re - cr, yi = v.im - ci;
        const double sy = fma(yr, yr, yi * yi);
        const double w = b.re * b.re + b.im * b.im;
        col[j] = MassCol{yr, yi, sy, w};
        smax = fmax(smax, sy);
        bad = bad | !w_in_range(w);
    }
    if (__any(bad) && lane == 0) atomicOr(&st->wbad, 1);
    smax = wave_max(smax);
    if (lane == 0) red[4][w] = smax;
    __syncthreads();
    if (tid == 0) {
        for (int q = 1; q < 16; ++q) smax = fmax(smax, red[4][q]);
        fr->R2 = smax;
    }
}

// Level-1 pairs (D_k = d_2k d_2k+1, N_k = w_2k d_2k+1 + w_2k+1 d_2k) of K
// column pairs merged pairwise, (N, D) of one pair of halves at a time, into
// one fraction N / D = sum_u w_u / d_u; the result is left in N[0], D[0].
template <int K>
__device__ __forceinline__ void pair_tree(double (&N)[K], double (&D)[K]) {
#pragma unroll
    for (int h = K; h > 1; h /= 2) {
#pragma unroll
        for (int k = 0; k < h / 2; ++k) {
            const double nk = fma(N[2 * k], D[2 * k + 1], N[2 * k + 1] * D[2 * k]);
            D[k] = D[2 * k] * D[2 * k + 1];
            N[k] = nk;
        }
    }
}

// The masses of k_cauchy_mass1 over the columns [c_beg, c_end) in the short
// form, for waves whose distances and weights keep every product of the
// reciprocal tree inside the FP64 range (CM_D_*, CM_W_*): sixteen columns
// share one reciprocal, with no range checks and no recomputation; the last
// columns of the range go in a group of eight, then one by one.
template <int K>
__device__ __forceinline__ void mass1_groups(const MassCol* __restrict__ col, int e,
                                             const double (&a2)[CM_RT], const double (&b2)[CM_RT],
                                             const double (&sx)[CM_RT], double (&acc)[CM_RT]) {
    double N[CM_RT][K], D[CM_RT][K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const MassCol u0 = col[e + 2 * k], u1 = col[e + 2 * k + 1];
#pragma unroll
        for (int q = 0; q < CM_RT; ++q) {
            const double d0 = fma(a2[q], u0.yr, fma(b2[q], u0.yi, sx[q] + u0.sy));
            const double d1 = fma(a2[q], u1.yr, fma(b2[q], u1.yi, sx[q] + u1.sy));
            D[q][k] = d0 * d1;
            N[q][k] = fma(u0.w, d1, u1.w * d0);
        }
    }
#pragma unroll
    for (int q = 0; q < CM_RT; ++q) {
        pair_tree<K>(N[q], D[q]);
        acc[q] = fma(N[q][0], rcp_1nr(D[q][0]), acc[q]);
    }
}

__device__ __forceinline__ void mass1_fast(const MassCol* __restrict__ col, int c_beg, int c_end,
                                           const double (&a2)[CM_RT], const double (&b2)[CM_RT],
                                           const double (&sx)[CM_RT], double (&acc)[CM_RT]) {
    int e = c_beg;
#pragma unroll 1
    for (; e + 16 <= c_end; e += 16) mass1_groups<8>(col, e, a2, b2, sx, acc);
    if (e + 8 <= c_end) {
        mass1_groups<4>(col, e, a2, b2, sx, acc);
        e += 8;
    }
    for (; e < c_end; ++e) {
        const MassCol u = col[e];
#pragma unroll
        for (int q = 0; q < CM_RT; ++q) {
            const double d = fma(a2[q], u.yr, fma(b2[q], u.yi, sx[q] + u.sy));
            acc[q] = fma(u.w, rcp_refined(d), acc[q]);
        }
    }
}

__global__ __launch_bounds__(CM_THREADS) void k_cauchy_mass1(
    const cf64* __restrict__ x, const cf64* __restrict__ y, const cf64* __restrict__ G,
    const MassCol* __restrict__ col, const MassFrame* __restrict__ frame, int n, int m,
    int cols_per_split, const StepState* __restrict__ st, double* __restrict__ partial) {
    if (st->done) return;
    const int tid = threadIdx.x;
    const int split = blockIdx.y;
    const int c_beg = split * cols_per_split;
    const int c_end = min(m, c_beg + cols_per_split);
    const double cr = frame->cr, ci = frame->ci;

    double xr[CM_RT], xi[CM_RT], a2[CM_RT], b2[CM_RT], sx[CM_RT], gscale[CM_RT], acc[CM_RT];
    bool safe = true;     // the short form is accurate for this lane's rows
    bool inrange = true;  // and every |x - y_j|^2 of them lies in [CM_D_LO, CM_D_HI]
#pragma unroll
    for (int q = 0; q < CM_RT; ++q) {
        const int r = blockIdx.x * CM_ROWS + q * CM_THREADS + tid;
        const bool valid = r < n;
        const cf64 xv = valid ? x[r] : cf64{0.0, 0.0};
        const cf64 g = valid ? G[r] : cf64{0.0, 0.0};
        xr[q] = xv.re;
        xi[q] = xv.im;
        const double ar = xv.re - cr, ai = xv.im - ci;
        a2[q] = -2.0 * ar;
        b2[q] = -2.0 * ai;
        sx[q] = fma(ar, ar, ai * ai);
        gscale[q] = g.re * g.re + g.im * g.im;
        acc[q] = 0.0;
        // min_j |x - y_j|^2 >= the squared distance from x to the box of y,
        // and max_j (|x - c|^2 + |y_j - c|^2) <= |x - c|^2 + R2
        const double dx = fmax(0.0, fmax(frame->yr0 - xv.re, xv.re - frame->yr1));
        const double dy = fmax(0.0, fmax(frame->yi0 - xv.im, xv.im - frame->yi1));
        // and |x - y_j|^2 <= (|x - c| + |y_j - c|)^2 <= 2 (|x - c|^2 + R2)
        if (valid) {
            const double dist2 = fma(dx, dx, dy * dy);
            safe = safe & (dist2 >= CM_SHORT_RATIO * (sx[q] + frame->R2));
            inrange = inrange & (dist2 >= CM_D_LO) & (2.0 * (sx[q] + frame->R2) <= CM_D_HI);
        }
    }
    const int shortf = __all(safe) ? 1 : 0;     // the same in every lane of the wave
    const int fastf = (shortf && __all(inrange) && st->wbad == 0) ? 1 : 0;

    if (fastf) mass1_fast(col, c_beg, c_end, a2, b2, sx, acc);
    else
    for (int c0 = c_beg; c0 < c_end; c0 += CM_TILE) {
        const int nt = min(CM_TILE, c_end - c0);
        const int ng = nt / CM_GRP * CM_GRP;
        double acc_t[CM_RT];
        bool ok[CM_RT];
#pragma unroll
        for (int q = 0; q < CM_RT; ++q) { acc_t[q] = 0.0; ok[q] = true; }
        if (shortf) {
#pragma unroll 2
            for (int e = c0; e < c0 + ng; e += CM_GRP) {
                MassCol cc[CM_GRP];
                double w[CM_GRP];
#pragma unroll
                for (int u = 0; u < CM_GRP; ++u) { cc[u] = col[e + u]; w[u] = cc[u].w; }
#pragma unroll
                for (int q = 0; q < CM_RT; ++q) {
                    double d[CM_GRP];
#pragma unroll
                    for (int u = 0; u < CM_GRP; ++u)
                        d[u] = fma(a2[q], cc[u].yr, fma(b2[q], cc[u].yi, sx[q] + cc[u].sy));
                    mass_group(d, w, ok[q], acc_t[q]);
                }
            }
        } else {
            for (int e = c0; e < c0 + ng; e += CM_GRP) {
                cf64 yy[CM_GRP];
                double w[CM_GRP];
#pragma unroll
                for (int u = 0; u < CM_GRP; ++u) { yy[u] = y[e + u]; w[u] = col[e + u].w; }
#pragma unroll
                for (int q = 0; q < CM_RT; ++q) {
                    double d[CM_GRP];
#pragma unroll
                    for (int u = 0; u < CM_GRP; ++u) {
                        const double a = xr[q] - yy[u].re, b = xi[q] - yy[u].im;
                        d[u] = fma(a, a, b * b);
                    }
                    mass_group(d, w, ok[q], acc_t[q]);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < CM_RT; ++q) {
            if (__builtin_expect(!ok[q], 0)) {    // rare: recompute this tile term by term
                double s = 0.0;
                for (int e = c0; e < c0 + ng; ++e) {
                    const double a = xr[q] - y[e].re, b = xi[q] - y[e].im;
                    s = fma(col[e].w, rcp_refined(fma(a, a, b * b)), s);
                }
                acc_t[q] = s;
            }
            for (int e = c0 + ng; e < c0 + nt; ++e) {   // ragged tail of the tile
                const double a = xr[q] - y[e].re, b = xi[q] - y[e].im;
                acc_t[q] = fma(col[e].w, rcp_refined(fma(a, a, b * b)), acc_t[q]);
            }
            acc[q] += acc_t[q];
        }
    }
#pragma unroll
    for (int q = 0; q < CM_RT; ++q) {
        const int r = blockIdx.x * CM_ROWS + q * CM_THREADS + tid;
        if (r < n) partial[(int64_t)split * n + r] = gscale[q] * acc[q];
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

// Wide: rowmass[e] = sum over splits s of partial[s][e] for one chunk of
// rows per workgroup, two threads per row: each adds one half of the splits
// in order and the row's mass is (first half) + (second half); with the
// chunk totals. The last workgroup runs the stop test and draws the pivot
// row (pivot.hpp).
__global__ __launch_bounds__(CDF_THREADS) void k_cauchy_reduce_draw(
    const double* __restrict__ partial, int splits, double* __restrict__ rowmass, PivotArgs pa,
    double* __restrict__ ct) {
    __shared__ WideShared sh;
    if (pa.st->done) return;
    const int t = pa.st->t;
    const StopInputs in = stop_inputs(pa.st);
    wide_keep_words(sh, step_words(pa, t));
    const int n = pa.n;
    const int q = threadIdx.x % CDF_CHUNK, h = threadIdx.x / CDF_CHUNK;
    const int e = blockIdx.x * CDF_CHUNK + q;
    const int mid = (splits + 1) / 2;
    double v = 0.0;
    if (e < n) {
        const int s0 = h ? mid : 0, s1 = h ? splits : mid;
#pragma unroll 16
        for (int s = s0; s < s1; ++s) v += partial[(int64_t)s * n + e];
    }
    if (h == 1) sh.pair[q] = v;
    __syncthreads();
    if (h == 0) {
        v = v + sh.pair[q];
        if (e < n) rowmass[e] = v;
    }
    wide_chunk_totals<CDF_CHUNK>(sh, v, n, ct);
    if (!wide_arrive_last(sh, &pa.st->arrive)) return;
    if (threadIdx.x == 0) pa.st->wbad = 0;      // this step's mass pass has read it
    pivot_row_draw_ct(sh.cdf, &sh.flag, pa, ct, t, wide_words(sh), in, RowMassGlobal{rowmass});
}

// Wide: regenerates the pivot row r = (G_i,: B) ./ (x_i - y) into U(t,:)
// (Alg. 3, row of A^(k)), one column per thread, with the chunk totals of
// |r|^2; the last workgroup draws the column and commits the pivot, copying
// G_i,: and B_:,j for the generator update.
template <int P>
__global__ __launch_bounds__(CDF_THREADS) void k_cauchy_rowgen_draw(
    const cf64* __restrict__ x, const cf64* __restrict__ y, const cf64* __restrict__ G,
    const cf64* __restrict__ B, cf64* __restrict__ U, int64_t ldu, PivotArgs pa,
    double* __restrict__ ct) {
    __shared__ WideShared sh;
    if (pa.st->done) return;
    const int m = pa.m;
    const int t = pa.st->cur, i = pa.st->i;
    wide_keep_words(sh, step_words(pa, t));
    cf64* Ut = U + (int64_t)t * ldu;
    const int c = blockIdx.x * WIDE_ELEMS + threadIdx.x;
    double v = 0.0;
    if (c < m) {
        cf64 gi[P];
#pragma unroll
        for (int l = 0; l < P; ++l) gi[l] = G[(int64_t)i * P + l];
        const cf64 r = cdiv_fast(gen_dot<P>(gi, B, m, c), csub(x[i], y[c]));
        Ut[c] = r;
        v = Sc<cf64>::mag2(r);
    }
    wide_chunk_totals(sh, v, m, ct);
    if (!wide_arrive_last(sh, &pa.st->arrive)) return;
    pivot_col_draw_ct<cf64, P>(sh.cdf, pa, t, Ut, ct, G, B, wide_words(sh), ColMassGlobal<cf64>{Ut});
}

// For p = 1 it also rewrites w_j = |b_j|^2 of the mass kernel's column data
// and flags a w_j outside the range of the 16-column form (StepState::wbad).
template <int P>
__global__ __launch_bounds__(256) void k_cauchy_update(
    const cf64* __restrict__ x, const cf64* __restrict__ y, cf64* __restrict__ G,
    cf64* __restrict__ B, int n, int m, StepState* __restrict__ st,
    const cf64* __restrict__ U, int64_t ldu, cf64* __restrict__ L, int64_t ldl,
    MassCol* __restrict__ col) {
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
        const cf64 c = cdiv_fast(s, csub(x[r], y[pj]));
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
            const cf64 nb = (c == pj) ? cf64{0.0, 0.0} : csub(b, wmul(bjl, f));
            B[(int64_t)l * m + c] = nb;
            if constexpr (P == 1) {
                const double w = nb.re * nb.re + nb.im * nb.im;
                col[c].w = w;
                if (!w_in_range(w)) atomicOr(&st->wbad, 1);
            }
        }
    }
}

// Column-mass pass, p > 1: G^T (p x n) and B^T (m x p), row-major.
__global__ __launch_bounds__(256) void k_cauchy_transpose(const cf64* __restrict__ G,
                                                          const cf64* __restrict__ B, int n,
                                                          int m, int p, const StepState* st,
                                                          cf64* __restrict__ Gt,
                                                          cf64* __restrict__ Bt) {
    if (st->done) return;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < (int64_t)n * p) {
        const int64_t i = idx / p, l = idx % p;
        Gt[l * n + i] = G[idx];
    }
    if (idx < (int64_t)m * p) {
        const int64_t j = idx / p, l = idx % p;
        Bt[idx] = B[l * m + j];
    }
}

// ---------------------------------------------------------------- launchers

int cauchy_rows_per_block() { return CM_ROWS; }

static int mass_wg_per_cu(const void* f) {
    int nb = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, CM_THREADS, 0);
    return (e == hipSuccess && nb > 0) ? nb : 2;
}

MassSlots cauchy_mass_slots(int cu_count) {
    MassSlots sl;
    sl.cu_count = cu_count;
    sl.row_wg[1] = mass_wg_per_cu(reinterpret_cast<const void*>(&k_cauchy_mass1));
    sl.col_wg[1] = mass_wg_per_cu(reinterpret_cast<const void*>(&k_cauchy_mass<1>));
    sl.row_wg[2] = sl.col_wg[2] = mass_wg_per_cu(reinterpret_cast<const void*>(&k_cauchy_mass<2>));
    sl.row_wg[3] = sl.col_wg[3] = mass_wg_per_cu(reinterpret_cast<const void*>(&k_cauchy_mass<3>));
    sl.row_wg[4] = sl.col_wg[4] = mass_wg_per_cu(reinterpret_cast<const void*>(&k_cauchy_mass<4>));
    sl.row_wg[0] = sl.row_wg[1];
    sl.col_wg[0] = sl.col_wg[1];
    return sl;
}

template <int P>
static void mass_p(const CauchyArgs& a, hipStream_t s) {
    const int cps = a.cols_per_split;
    dim3 grid((unsigned)((a.n + CM_ROWS - 1) / CM_ROWS), (unsigned)a.splits);
    if (P == 1 && a.mcol != nullptr)
        hipLaunchKernelGGL(k_cauchy_mass1, grid, dim3(CM_THREADS), 0, s, (const cf64*)a.x,
                           (const cf64*)a.y, (const cf64*)a.G, (const MassCol*)a.mcol,
                           (const MassFrame*)a.mframe, (int)a.n, (int)a.m, cps, a.st, a.partial);
    else
        hipLaunchKernelGGL(k_cauchy_mass<P>, grid, dim3(CM_THREADS), 0, s, (const cf64*)a.x,
                           (const cf64*)a.y, (const cf64*)a.G, (const cf64*)a.B, (int)a.n,
                           (int)a.m, cps, a.st, a.partial);
}

size_t cauchy_mass_col_bytes(int p, int64_t m) { return p == 1 ? (size_t)m * sizeof(MassCol) : 0; }
size_t cauchy_mass_frame_bytes(int p) { return p == 1 ? sizeof(MassFrame) : 0; }

void launch_cauchy_transpose(const CauchyArgs& a, void* Gt, void* Bt, hipStream_t s) {
    const int64_t work = (a.n > a.m ? a.n : a.m) * a.p;
    hipLaunchKernelGGL(k_cauchy_transpose, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, s,
                       (const cf64*)a.G, (const cf64*)a.B, (int)a.n, (int)a.m, a.p, a.st,
                       (cf64*)Gt, (cf64*)Bt);
}

void launch_cauchy_frame(const CauchyArgs& a, hipStream_t s) {
    if (a.p != 1) return;
    hipLaunchKernelGGL(k_cauchy_frame, dim3(1), dim3(1024), 0, s, (const cf64*)a.y,
                       (const cf64*)a.B, (int)a.m, (MassFrame*)a.mframe, (MassCol*)a.mcol, a.st);
}

void launch_cauchy_reduce_draw(const CauchyArgs& a, const SampleArgs& sa, hipStream_t s) {
    hipLaunchKernelGGL(k_cauchy_reduce_draw, dim3((unsigned)cdf_chunks((int)a.n)), dim3(CDF_THREADS), 0, s,
                       a.partial, a.splits, a.rowmass, pivot_args(sa), sa.ct_row);
}

template <int P>
static void rowgen_draw_p(const CauchyArgs& a, const SampleArgs& sa, hipStream_t s) {
    hipLaunchKernelGGL(k_cauchy_rowgen_draw<P>, dim3(wide_blocks(a.m)), dim3(CDF_THREADS), 0, s,
                       (const cf64*)a.x, (const cf64*)a.y, (const cf64*)a.G, (const cf64*)a.B,
                       (cf64*)a.U, a.ldu, pivot_args(sa), a.ct_col);
}

template <int P>
static void update_p(const CauchyArgs& a, hipStream_t s) {
    const int64_t work = a.n > a.m ? a.n : a.m;
    hipLaunchKernelGGL(k_cauchy_update<P>, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, s,
                       (const cf64*)a.x, (const cf64*)a.y, (cf64*)a.G, (cf64*)a.B, (int)a.n,
                       (int)a.m, a.st, (const cf64*)a.U, a.ldu, (cf64*)a.L, a.ldl,
                       (MassCol*)a.mcol);
}

#define RPLU_DISPATCH_P(fn)                         \
    switch (a.p) {                                  \
        case 1: fn<1>(a, s); break;                 \
        case 2: fn<2>(a, s); break;                 \
        case 3: fn<3>(a, s); break;                 \
        case 4: fn<4>(a, s); break;                 \
    }

void launch_cauchy_mass(const CauchyArgs& a, hipStream_t s) { RPLU_DISPATCH_P(mass_p) }
void launch_cauchy_update(const CauchyArgs& a, hipStream_t s) { RPLU_DISPATCH_P(update_p) }

void launch_cauchy_rowgen_draw(const CauchyArgs& a, const SampleArgs& sa, hipStream_t s) {
    switch (a.p) {
        case 1: rowgen_draw_p<1>(a, sa, s); break;
        case 2: rowgen_draw_p<2>(a, sa, s); break;
        case 3: rowgen_draw_p<3>(a, sa, s); break;
        case 4: rowgen_draw_p<4>(a, sa, s); break;
    }
}

}  // namespace rplu
