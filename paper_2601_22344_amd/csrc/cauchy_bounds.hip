// Certified row-norm upper bounds for the Cauchy-like form (App. C, Alg.
// C.2) and the rejection-sampled row draw (Alg. 3, Step 1).
//
// Per step, on the plan built once per run (bounds_plan.cpp):
//   k_bh_gram_leaves  H_s = sum_{j in s} B_:,j B_:,j^* for every source leaf
//                     (one wave per leaf, fixed-order wave sums)
//   k_bh_gram_tree    inner source nodes, deepest level first: H_s = the sum
//                     of its children's (one workgroup, a barrier per level)
//   k_bh_bounds       u_i = sum over the aggregated entries (s, alpha) of the
//                     target leaf of alpha G_i,: H_s G_i,:^* plus the exact
//                     terms |G_i,: B_:,j|^2 / |x_i - y_j|^2 of its exact source
//                     leaves; one wave per target leaf, a lane per target
//                     point, the source data as wave-uniform loads
//   k_rows_draw (sample.hip)  the stop test on sum(u) and the row draw of
//                     trial 0 (the bounds are the row masses of the draw)
//   k_bh_reject       rho_i = ||S_i,:||^2 of the drawn row, accepted when
//                     v u_i < rho_i (v from word w2 of the trial's Philox
//                     block); otherwise the next trial q draws a row from the
//                     same CDF with word w0 of counter (t, stream, q, 0). The
//                     first BH_REJ_CAND trials are evaluated at once, each
//                     row's mass by S workgroups over a slice of its columns;
//                     the workgroup that arrives last takes the first trial
//                     that passes, or goes on with the trials after them
//                     alone (one workgroup per row)
// The accepted row then takes the exact form's kernels: regeneration with
// the column draw, and the generator update.
#include <algorithm>
#include <cstring>

#include "common.hpp"
#include "cdf.hpp"
#include "launch.hpp"
#include "pivot.hpp"
#include "bounds_plan.hpp"

namespace rplu {

constexpr int BH_TREE_THREADS = 256;

// c + a conj(b)
__device__ inline cf64 cmad_conj(cf64 a, cf64 b, cf64 c) {
    return {fma(a.re, b.re, fma(a.im, b.im, c.re)), fma(a.im, b.re, fma(-a.re, b.im, c.im))};
}

template <int P>
__global__ __launch_bounds__(RPLU_WAVE) void k_bh_gram_leaves(BoundsPlan bp,
                                                              const cf64* __restrict__ B, int m,
                                                              const StepState* __restrict__ st) {
    if (st->done) return;
    const int s = bp.src_leaves[blockIdx.x];
    const int lane = threadIdx.x;
    cf64 h[P][P];
#pragma unroll
    for (int a = 0; a < P; ++a)
#pragma unroll
        for (int c = 0; c < P; ++c) h[a][c] = cf64{0.0, 0.0};
    for (int q = bp.node_beg[s] + lane; q < bp.node_end[s]; q += RPLU_WAVE) {
        const int j = bp.src_perm[q];
        cf64 b[P];
#pragma unroll
        for (int l = 0; l < P; ++l) b[l] = B[(int64_t)l * m + j];
#pragma unroll
        for (int a = 0; a < P; ++a)
#pragma unroll
            for (int c = 0; c < P; ++c) h[a][c] = cmad_conj(b[a], b[c], h[a][c]);
    }
    cf64* H = (cf64*)bp.H + (int64_t)s * P * P;
#pragma unroll
    for (int a = 0; a < P; ++a)
#pragma unroll
        for (int c = 0; c < P; ++c) {
            const double re = wave_sum(h[a][c].re), im = wave_sum(h[a][c].im);
            if (lane == 0) H[a * P + c] = cf64{re, im};
        }
}

template <int P>
__global__ __launch_bounds__(BH_TREE_THREADS) void k_bh_gram_tree(BoundsPlan bp,
                                                                  const StepState* __restrict__ st) {
    if (st->done) return;
    cf64* H = (cf64*)bp.H;
    for (int d = bp.max_depth; d >= 0; --d) {
        for (int q = bp.level_off[d] + threadIdx.x; q < bp.level_off[d + 1]; q += BH_TREE_THREADS) {
            const int s = bp.inner[q];
            cf64 acc[P * P];
#pragma unroll
            for (int e = 0; e < P * P; ++e) acc[e] = cf64{0.0, 0.0};
            for (int c = 0; c < 4; ++c) {
                const int ch = bp.node_child[4 * s + c];
                if (ch < 0) break;
#pragma unroll
                for (int e = 0; e < P * P; ++e) acc[e] = cadd(acc[e], H[(int64_t)ch * P * P + e]);
            }
#pragma unroll
            for (int e = 0; e < P * P; ++e) H[(int64_t)s * P * P + e] = acc[e];
        }
        __syncthreads();
    }
}

// The same bottom-up pass with the matrices, the inner-node list and the
// child lists in LDS (one load of each from the plan at the start), so that
// a level costs no memory round trip: the tree pass had spent one per level.
// Sums and their order are those of k_bh_gram_tree. For plans whose data fit
// in BH_TREE_LDS bytes.
constexpr size_t BH_TREE_LDS = 64 * 1024;

template <int P>
__host__ __device__ inline size_t bh_tree_lds_bytes(int n_nodes, int n_inner, int max_depth) {
    return (size_t)n_nodes * P * P * sizeof(cf64) + (size_t)n_inner * 5 * sizeof(int32_t) +
           (size_t)(max_depth + 2) * sizeof(int32_t);
}

template <int P>
__global__ __launch_bounds__(BH_TREE_THREADS) void k_bh_gram_tree_lds(BoundsPlan bp,
                                                                      const StepState* __restrict__ st) {
    extern __shared__ double lds_raw[];
    if (st->done) return;
    const int n_inner = bp.n_inner;
    cf64* hs = reinterpret_cast<cf64*>(lds_raw);
    int32_t* node = reinterpret_cast<int32_t*>(hs + (size_t)bp.n_src_nodes * P * P);
    int32_t* kids = node + n_inner;                   // 4 per inner node, in list order
    int32_t* loff = kids + 4 * n_inner;
    cf64* H = (cf64*)bp.H;
#pragma unroll 4
    for (int q = threadIdx.x; q < bp.n_src_leaves * P * P; q += BH_TREE_THREADS) {
        const int s = bp.src_leaves[q / (P * P)];
        hs[(int64_t)s * P * P + q % (P * P)] = H[(int64_t)s * P * P + q % (P * P)];
    }
    for (int q = threadIdx.x; q < n_inner; q += BH_TREE_THREADS) {
        const int s = bp.inner[q];
        node[q] = s;
#pragma unroll
        for (int c = 0; c < 4; ++c) kids[4 * q + c] = bp.node_child[4 * s + c];
    }
    for (int q = threadIdx.x; q < bp.max_depth + 2; q += BH_TREE_THREADS) loff[q] = bp.level_off[q];
    __syncthreads();
    for (int d = bp.max_depth; d >= 0; --d) {
        for (int q = loff[d] + threadIdx.x; q < loff[d + 1]; q += BH_TREE_THREADS) {
            const int s = node[q];
            cf64 acc[P * P];
#pragma unroll
            for (int e = 0; e < P * P; ++e) acc[e] = cf64{0.0, 0.0};
            for (int c = 0; c < 4; ++c) {
                const int ch = kids[4 * q + c];
                if (ch < 0) break;
#pragma unroll
                for (int e = 0; e < P * P; ++e) acc[e] = cadd(acc[e], hs[(int64_t)ch * P * P + e]);
            }
#pragma unroll
            for (int e = 0; e < P * P; ++e) {
                hs[(int64_t)s * P * P + e] = acc[e];
                H[(int64_t)s * P * P + e] = acc[e];
            }
        }
        __syncthreads();
    }
}

template <int P>
__device__ inline void bh_point(const BoundsPlan& bp, const cf64* __restrict__ x,
                                const cf64* __restrict__ y, const cf64* __restrict__ G,
                                const cf64* __restrict__ B, int m, int l, bool act, int i) {
    const cf64 xi = x[i];
    cf64 g[P];
#pragma unroll
    for (int a = 0; a < P; ++a) g[a] = G[(int64_t)i * P + a];
    double acc = 0.0;
    const cf64* H = (const cf64*)bp.H;
    // G_i H_s G_i^* = sum_a g_a (sum_c H_ac conj(g_c)), real
    auto form = [&](const cf64* h) {
        double q = 0.0;
#pragma unroll
        for (int a = 0; a < P; ++a) {
            cf64 w{0.0, 0.0};
#pragma unroll
            for (int c = 0; c < P; ++c) w = cmad_conj(h[a * P + c], g[c], w);
            q = fma(g[a].re, w.re, fma(-g[a].im, w.im, q));
        }
        return q;
    };
    // the list's entries in batches: their node indices and weights, then
    // their matrices, are loaded before any is used (two dependent loads per
    // entry had each waited a round trip); the terms are added in list order
    constexpr int BH_E = P == 1 ? 8 : (P == 2 ? 2 : 1);
    int e = bp.A_off[l];
    const int e1 = bp.A_off[l + 1];
    for (; e + BH_E <= e1; e += BH_E) {
        int nd[BH_E];
        double al[BH_E];
#pragma unroll
        for (int u = 0; u < BH_E; ++u) {
            nd[u] = bp.A_node[e + u];
            al[u] = bp.A_alpha[e + u];
        }
        cf64 h[BH_E][P * P];
#pragma unroll
        for (int u = 0; u < BH_E; ++u)
#pragma unroll
            for (int k = 0; k < P * P; ++k) h[u][k] = H[(int64_t)nd[u] * P * P + k];
#pragma unroll
        for (int u = 0; u < BH_E; ++u) acc = fma(al[u], form(h[u]), acc);
    }
    for (; e < e1; ++e) acc = fma(bp.A_alpha[e], form(H + (int64_t)bp.A_node[e] * P * P), acc);
    for (int e = bp.E_off[l]; e < bp.E_off[l + 1]; ++e) {
        const int s = bp.E_node[e];
        for (int q = bp.node_beg[s]; q < bp.node_end[s]; ++q) {
            const int j = bp.src_perm[q];
            cf64 dot{0.0, 0.0};
#pragma unroll
            for (int a = 0; a < P; ++a) dot = cadd(dot, wmul(g[a], B[(int64_t)a * m + j]));
            const cf64 d = csub(xi, y[j]);
            acc += Sc<cf64>::mag2(dot) / Sc<cf64>::mag2(d);
        }
    }
    if (act) bp.u[i] = acc;
}

template <int P>
__global__ __launch_bounds__(RPLU_WAVE) void k_bh_bounds(BoundsPlan bp, const cf64* __restrict__ x,
                                                         const cf64* __restrict__ y,
                                                         const cf64* __restrict__ G,
                                                         const cf64* __restrict__ B, int m,
                                                         const StepState* __restrict__ st) {
    if (st->done) return;
    const int l = blockIdx.x, lane = threadIdx.x;
    const int beg = bp.tl_beg[l], end = bp.tl_end[l];
    // a lane per target point (a leaf of identical points may hold more than
    // a wave: chunks of 64)
    for (int q0 = beg; q0 < end; q0 += RPLU_WAVE)
        bh_point<P>(bp, x, y, G, B, m, l, q0 + lane < end, bp.tgt_perm[min(q0 + lane, end - 1)]);
}

// sum over the columns j0 <= j < j1 of |S_ij|^2 of the Cauchy-like matrix,
// the row regenerated as in k_cauchy_rowgen_draw; whole workgroup,
// fixed-order sum, in every thread.
template <int P>
__device__ inline double bh_row_mass(const cf64* __restrict__ x, const cf64* __restrict__ y,
                                     const cf64* __restrict__ G, const cf64* __restrict__ B,
                                     int m, int i, int j0, int j1, double* red) {
    cf64 gi[P];
#pragma unroll
    for (int l = 0; l < P; ++l) gi[l] = G[(int64_t)i * P + l];
    const cf64 xi = x[i];
    double v = 0.0;
    // each thread takes columns threadIdx.x + 1024 k, added in order; eight
    // columns' data are loaded before any is used, so one memory round trip
    // serves eight columns (a loop of single columns waited on each)
    auto term = [&](const cf64 (&b)[P], cf64 yc) {
        cf64 s{0.0, 0.0};
#pragma unroll
        for (int l = 0; l < P; ++l) {
            s.re = fma(gi[l].re, b[l].re, s.re);
            s.re = fma(-gi[l].im, b[l].im, s.re);
            s.im = fma(gi[l].re, b[l].im, s.im);
            s.im = fma(gi[l].im, b[l].re, s.im);
        }
        return Sc<cf64>::mag2(cdiv_fast(s, csub(xi, yc)));
    };
    constexpr int BH_U = 8;
    int c = j0 + (int)threadIdx.x;
    for (; c + (BH_U - 1) * CDF_THREADS < j1; c += BH_U * CDF_THREADS) {
        cf64 bb[BH_U][P], yy[BH_U];
#pragma unroll
        for (int u = 0; u < BH_U; ++u) {
#pragma unroll
            for (int l = 0; l < P; ++l) bb[u][l] = B[(int64_t)l * m + c + u * CDF_THREADS];
            yy[u] = y[c + u * CDF_THREADS];
        }
#pragma unroll
        for (int u = 0; u < BH_U; ++u) v += term(bb[u], yy[u]);
    }
    for (; c < j1; c += CDF_THREADS) {
        cf64 b1[P];
#pragma unroll
        for (int l = 0; l < P; ++l) b1[l] = B[(int64_t)l * m + c];
        v += term(b1, y[c]);
    }
    v = wave_sum(v);
    const int lane = threadIdx.x % RPLU_WAVE, w = threadIdx.x / RPLU_WAVE;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double r = red[0];
    for (int q = 1; q < CDF_THREADS / RPLU_WAVE; ++q) r += red[q];
    return r;
}

// Grid: BH_REJ_CAND x S workgroups (S = gridDim.x / BH_REJ_CAND); workgroup
// (c, s) draws trial c's row (trial 0's row is the draw kernel's) and sums
// its masses over the s-th of S equal column slices. The workgroup that
// arrives last adds each trial's S slices in order and tests the trials in
// order; past them, it goes on alone as one trial per row sweep. The
// accepted row, the trial count and the error are those of testing the
// trials one at a time.
template <int P>
__global__ __launch_bounds__(CDF_THREADS) void k_bh_reject(BoundsPlan bp, const cf64* __restrict__ x,
                                                           const cf64* __restrict__ y,
                                                           const cf64* __restrict__ G,
                                                           const cf64* __restrict__ B, PivotArgs pa,
                                                           const double* __restrict__ ct_row) {
    __shared__ CdfShared sh;
    __shared__ double red[CDF_THREADS / RPLU_WAVE];
    __shared__ int last;
    StepState* st = pa.st;
    if (st->done) return;
    const int t = st->cur;
    if (pa.greedy || pa.forced) {                 // the draw kernel's row stands
        if (blockIdx.x == 0 && threadIdx.x == 0) { st->trials = 1; st->trials_total += 1; }
        return;
    }
    const int S = gridDim.x / BH_REJ_CAND;
    const int c = blockIdx.x / S, s = blockIdx.x % S;
    const int K = cdf_chunks(pa.n);
    int i = st->i;
    double tgt = st->row_tgt, lo = st->row_lo, hi = st->row_hi;
    if (c > 0) {
        const double T = cdf_levels(sh, ct_row, K);
        const Philox4 w = philox4x64_10((uint64_t)t, pa.stream, (uint64_t)c, 0, pa.seed, 0);
        tgt = unit_from_word(w.w[0]) * T;
        const CdfPick p = cdf_draw(sh, ct_row, K, pa.n, RowMassGlobal{bp.u}, tgt);
        i = p.idx;
        lo = p.lo;
        hi = p.hi;
    }
    const int j0 = (int)((int64_t)pa.m * s / S), j1 = (int)((int64_t)pa.m * (s + 1) / S);
    const double part = bh_row_mass<P>(x, y, G, B, pa.m, i, j0, j1, red);
    if (threadIdx.x == 0) {
        bp.rej_part[blockIdx.x] = part;
        if (s == 0) {
            double* cd = bp.rej_cand + 4 * c;
            cd[0] = (double)i;
            cd[1] = tgt;
            cd[2] = lo;
            cd[3] = hi;
        }
    }
    // arrival (bh_row_mass ended on a barrier after the stores' values were
    // formed; the barrier here orders thread 0's stores): thread 0's
    // device-scope release fence before its arrival, and in the last
    // workgroup its acquire fence and the barrier after it order every
    // later load after all arrivals; the last workgroup clears the counter
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const int l = (atomicAdd(&st->arrive, 1u) == gridDim.x - 1) ? 1 : 0;
        if (l) {
            __threadfence();
            st->arrive = 0u;
        }
        last = l;
    }
    __syncthreads();
    if (!last) return;
    for (int q = 0; q < BH_REJ_CAND; ++q) {
        double rho = 0.0;
        for (int r = 0; r < S; ++r) rho += bp.rej_part[q * S + r];
        const double* cd = bp.rej_cand + 4 * q;
        const int iq = (int)cd[0];
        const Philox4 w = philox4x64_10((uint64_t)t, pa.stream, (uint64_t)q, 0, pa.seed, 0);
        if (unit_from_word(w.w[2]) * bp.u[iq] < rho) {
            if (threadIdx.x == 0) {
                st->i = iq;
                st->row_tgt = cd[1];
                st->row_lo = cd[2];
                st->row_hi = cd[3];
                st->trials = q + 1;
                st->trials_total += q + 1;
            }
            return;
        }
    }
    const double T = cdf_levels(sh, ct_row, K);
    for (int q = BH_REJ_CAND; q < RPLU_BOUND_MAX_TRIALS; ++q) {
        const Philox4 w = philox4x64_10((uint64_t)t, pa.stream, (uint64_t)q, 0, pa.seed, 0);
        tgt = unit_from_word(w.w[0]) * T;
        const CdfPick p = cdf_draw(sh, ct_row, K, pa.n, RowMassGlobal{bp.u}, tgt);
        const double rho = bh_row_mass<P>(x, y, G, B, pa.m, p.idx, 0, pa.m, red);
        if (unit_from_word(w.w[2]) * bp.u[p.idx] < rho) {
            if (threadIdx.x == 0) {
                st->i = p.idx;
                st->row_tgt = tgt;
                st->row_lo = p.lo;
                st->row_hi = p.hi;
                st->trials = q + 1;
                st->trials_total += q + 1;
            }
            return;
        }
    }
    if (threadIdx.x == 0) {
        st->error = RPLU_E_BOUND;
        st->done = 1;
    }
}

// ---------------------------------------------------------------- launchers

size_t bounds_plan_bytes(const HostBoundsPlan& P, int64_t n, int p) {
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t ns = P.src.size();
    return up(P.tgt_perm.size() * 4) + up(P.src_perm.size() * 4) + 3 * up(ns * 4) + up(ns * 16) +
           up(P.src_leaves.size() * 4) + up(P.inner.size() * 4) + up(P.level_off.size() * 4) +
           2 * up(P.tl_beg.size() * 4) + up(P.A_off.size() * 4) + up(P.A_node.size() * 4) +
           up(P.A_alpha.size() * 8) + up(P.E_off.size() * 4) + up(P.E_node.size() * 4) +
           up(ns * (size_t)p * p * 16) + up((size_t)n * 8) + up(BH_REJ_CAND * BH_REJ_MAX_SPLIT * 8) +
           up(BH_REJ_CAND * 4 * 8);
}

// Copies the host plan into `dev` (bounds_plan_bytes bytes) on stream s and
// fills the device descriptor; the host vectors must live until the copies
// have run (the caller synchronises).
hipError_t upload_bounds_plan(const HostBoundsPlan& P, int64_t n, int p, char* dev, hipStream_t s,
                              std::vector<int32_t>* staging, BoundsPlan* out) {
    size_t off = 0;
    auto take = [&](size_t b) {
        char* r = dev + off;
        off += (b + 255) / 256 * 256;
        return r;
    };
    hipError_t e = hipSuccess;
    auto put = [&](const void* src, size_t b) -> void* {
        char* d = take(b);
        if (b && e == hipSuccess) e = hipMemcpyAsync(d, src, b, hipMemcpyHostToDevice, s);
        return d;
    };
    const int ns = (int)P.src.size();
    staging->assign((size_t)ns * 7, -1);      // node_beg, node_end, node_child (4)
    for (int v = 0; v < ns; ++v) {
        (*staging)[v] = P.src[v].beg;
        (*staging)[ns + v] = P.src[v].end;
        for (int c = 0; c < 4; ++c) (*staging)[2 * ns + 4 * v + c] = P.src[v].child[c];
    }
    BoundsPlan b;
    std::memset(&b, 0, sizeof b);        // padding too: the plan keys the graph cache
    b.n_src_nodes = ns;
    b.n_src_leaves = (int)P.src_leaves.size();
    b.n_tgt_leaves = (int)P.tl_beg.size();
    b.max_depth = P.max_depth;
    b.n_inner = (int)P.inner.size();
    b.pad = 0;
    b.nu = P.nu;
    b.tgt_perm = (const int32_t*)put(P.tgt_perm.data(), P.tgt_perm.size() * 4);
    b.src_perm = (const int32_t*)put(P.src_perm.data(), P.src_perm.size() * 4);
    b.node_beg = (const int32_t*)put(staging->data(), (size_t)ns * 4);
    b.node_end = (const int32_t*)put(staging->data() + ns, (size_t)ns * 4);
    (void)take((size_t)ns * 4);              // (spare, keeps bounds_plan_bytes' count)
    b.node_child = (const int32_t*)put(staging->data() + 2 * ns, (size_t)ns * 16);
    b.src_leaves = (const int32_t*)put(P.src_leaves.data(), P.src_leaves.size() * 4);
    b.inner = (const int32_t*)put(P.inner.data(), P.inner.size() * 4);
    b.level_off = (const int32_t*)put(P.level_off.data(), P.level_off.size() * 4);
    b.tl_beg = (const int32_t*)put(P.tl_beg.data(), P.tl_beg.size() * 4);
    b.tl_end = (const int32_t*)put(P.tl_end.data(), P.tl_end.size() * 4);
    b.A_off = (const int32_t*)put(P.A_off.data(), P.A_off.size() * 4);
    b.A_node = (const int32_t*)put(P.A_node.data(), P.A_node.size() * 4);
    b.A_alpha = (const double*)put(P.A_alpha.data(), P.A_alpha.size() * 8);
    b.E_off = (const int32_t*)put(P.E_off.data(), P.E_off.size() * 4);
    b.E_node = (const int32_t*)put(P.E_node.data(), P.E_node.size() * 4);
    b.H = take((size_t)ns * p * p * 16);
    b.u = (double*)take((size_t)n * 8);
    b.rej_part = (double*)take((size_t)BH_REJ_CAND * BH_REJ_MAX_SPLIT * 8);
    b.rej_cand = (double*)take((size_t)BH_REJ_CAND * 4 * 8);
    *out = b;
    return e;
}

template <int P>
static void bounds_p(const BoundsPlan& bp, const CauchyArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_bh_gram_leaves<P>, dim3((unsigned)bp.n_src_leaves), dim3(RPLU_WAVE), 0, s,
                       bp, (const cf64*)a.B, (int)a.m, a.st);
    const int n_inner = bp.n_inner;
    const size_t lds = bh_tree_lds_bytes<P>(bp.n_src_nodes, n_inner, bp.max_depth);
    if (lds <= BH_TREE_LDS)
        hipLaunchKernelGGL(k_bh_gram_tree_lds<P>, dim3(1), dim3(BH_TREE_THREADS), lds, s, bp, a.st);
    else
        hipLaunchKernelGGL(k_bh_gram_tree<P>, dim3(1), dim3(BH_TREE_THREADS), 0, s, bp, a.st);
    hipLaunchKernelGGL(k_bh_bounds<P>, dim3((unsigned)bp.n_tgt_leaves), dim3(RPLU_WAVE), 0, s, bp,
                       (const cf64*)a.x, (const cf64*)a.y, (const cf64*)a.G, (const cf64*)a.B,
                       (int)a.m, a.st);
}

template <int P>
static void reject_p(const BoundsPlan& bp, const CauchyArgs& a, const SampleArgs& sa,
                     hipStream_t s) {
    // slices of at least 1024 columns, at most BH_REJ_MAX_SPLIT per row
    const int S = (int)std::min<int64_t>(BH_REJ_MAX_SPLIT, std::max<int64_t>(1, (a.m + 1023) / 1024));
    hipLaunchKernelGGL(k_bh_reject<P>, dim3(BH_REJ_CAND * S), dim3(CDF_THREADS), 0, s, bp, (const cf64*)a.x,
                       (const cf64*)a.y, (const cf64*)a.G, (const cf64*)a.B, pivot_args(sa),
                       (const double*)sa.ct_row);
}

void launch_bh_bounds(const BoundsPlan& bp, const CauchyArgs& a, hipStream_t s) {
    switch (a.p) {
        case 1: bounds_p<1>(bp, a, s); break;
        case 2: bounds_p<2>(bp, a, s); break;
        case 3: bounds_p<3>(bp, a, s); break;
        case 4: bounds_p<4>(bp, a, s); break;
    }
}

void launch_bh_reject(const BoundsPlan& bp, const CauchyArgs& a, const SampleArgs& sa,
                      hipStream_t s) {
    switch (a.p) {
        case 1: reject_p<1>(bp, a, sa, s); break;
        case 2: reject_p<2>(bp, a, sa, s); break;
        case 3: reject_p<3>(bp, a, sa, s); break;
        case 4: reject_p<4>(bp, a, sa, s); break;
    }
}

}  // namespace rplu
