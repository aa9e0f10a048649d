// Two-level inverse-CDF sampling over a mass vector.
//
// The index drawn for a target u*T is the first index e whose inclusive
// prefix P(e) of the masses exceeds u*T (two-stage exact sampling draws a row
// by its mass, then a column of that row by |S_ij|^2; Sec. 4.1).
//
// The vector (length len) is cut into chunks of CDF_CHUNK = 64 lanes x E
// consecutive elements. Prefix structure, deterministic for a given len:
//   * inside chunk k, lane l sums its E elements in order (local prefix loc,
//     lane total lt); the lane totals are scanned across the wave
//     (Hillis-Steele) and the exclusive scan ex gives each lane's offset;
//     the chunk total is ct_k = ex_L + lt_L (L = last lane holding data);
//   * chunks are grouped by CDF_GROUP; inside group g the chunk offsets are
//     a sequential chain io_k (io = 0 at the group start, io += ct_k), the
//     group total gt_g is the chain's end;
//   * the group offsets are a sequential chain goff_0 = 0,
//     goff_{g+1} = goff_g + gt_g, and the total is T := goff_G.
// The prefix of element e in chunk k of group g is
//     P(e) = goff_g + (io_k + (ex_l + loc_l(e))),
// so the last element of chunk k has P = goff_g + io_{k+1} and the last of
// group g has P = goff_{g+1}, bit for bit: the chunk and group intervals
// tile [0, T) with no gap, and the first group (then chunk) whose upper end
// exceeds u*T always holds a hit. A hit must also have positive mass; if
// rounding at a lane boundary leaves only zero-mass hits in the chunk, its
// last positive-mass element is taken (the chunk has one, as its total is
// positive). A zero-mass index is never drawn.
//
// The chunk totals are computed by wide kernels (one wave per chunk, spread
// over the whole GPU, fused with whatever produces the masses); the chains,
// the stop test and the draw run in one workgroup, and one wave of it
// re-walks the selected chunk.
#pragma once

#include "common.hpp"

namespace rplu {

constexpr int CDF_E = 8;                           // consecutive elements per lane
constexpr int CDF_CHUNK = RPLU_WAVE * CDF_E;       // elements per chunk (one wave)
constexpr int CDF_GROUP = 32;                      // chunks per group
constexpr int CDF_THREADS = 1024;                  // sampler workgroup
constexpr int CDF_MAX_GROUPS = CDF_THREADS;        // => len <= 2^24 elements

__device__ __host__ inline int cdf_chunks(int len) { return (len + CDF_CHUNK - 1) / CDF_CHUNK; }

// One chunk as seen by one wave: the lane's E masses (0 beyond len), its
// exclusive offset ex, its total lt and the chunk total ct (same in every
// lane). Indices are clamped into range and the values masked afterwards, so
// every mass() call is unconditional and the loads issue back to back; a
// callback that also stores (a row copy) rewrites element len-1 with the
// value it already holds.
struct CdfChunk {
    double v[CDF_E];
    double ex, lt, ct;
};

// The chunk structure from the lane's E masses x (elements s0 .. s0 + E - 1,
// s0 = chunk * CDF_CHUNK + lane * E; entries at or past len are ignored).
__device__ inline void cdf_chunk_vals(CdfChunk& c, const double (&x)[CDF_E], int chunk, int len,
                                      int lane) {
    const int s0 = chunk * CDF_CHUNK + lane * CDF_E;
    double l = 0.0;
#pragma unroll
    for (int u = 0; u < CDF_E; ++u) {
        c.v[u] = (s0 + u < len) ? x[u] : 0.0;
        l += c.v[u];
    }
    const double incl = wave_incl_scan(l, lane);
    double ex = __shfl_up(incl, 1, RPLU_WAVE);
    if (lane == 0) ex = 0.0;
    c.ex = ex;
    c.lt = l;
    const int L = min(RPLU_WAVE - 1, (len - 1 - chunk * CDF_CHUNK) / CDF_E);
    c.ct = __shfl(ex + l, L, RPLU_WAVE);
}

template <class MassFn>
__device__ inline void cdf_chunk(CdfChunk& c, int chunk, int len, int lane, MassFn& mass) {
    const int s0 = chunk * CDF_CHUNK + lane * CDF_E;
    double x[CDF_E];
#pragma unroll
    for (int u = 0; u < CDF_E; ++u) x[u] = mass(min(s0 + u, len - 1));
    cdf_chunk_vals(c, x, chunk, len, lane);
}

struct CdfPick {
    int idx;        // drawn index
    double lo, hi;  // CDF edges of the drawn bin: P(idx-1), P(idx)
};

// Within chunk `chunk` (whole wave): the first element with positive mass
// whose prefix goff + (io + (ex + loc)) exceeds target; `before` is the prefix
// just before the chunk's first element.
template <class MassFn>
__device__ inline CdfPick cdf_chunk_select(int chunk, int len, int lane, MassFn& mass, double goff,
                                           double io, double before, double target) {
    CdfChunk c;
    cdf_chunk(c, chunk, len, lane, mass);
    double prev = __shfl_up(goff + (io + (c.ex + c.lt)), 1, RPLU_WAVE);
    if (lane == 0) prev = before;
    int hit_u = -1, pos_u = -1;
    double hlo = 0.0, hhi = 0.0, plo = 0.0, phi = 0.0, loc = 0.0;
#pragma unroll
    for (int u = 0; u < CDF_E; ++u) {
        loc += c.v[u];                          // the same sequence as c.lt
        const double P = goff + (io + (c.ex + loc));
        if (c.v[u] > 0.0) {
            if (hit_u < 0 && P > target) { hit_u = u; hlo = prev; hhi = P; }
            pos_u = u; plo = prev; phi = P;
        }
        prev = P;
    }
    const unsigned long long bal = __ballot(hit_u >= 0);
    CdfPick r{-1, 0.0, 0.0};
    if (bal) {
        const int fl = __ffsll(bal) - 1;
        r.idx = chunk * CDF_CHUNK + fl * CDF_E + __shfl(hit_u, fl, RPLU_WAVE);
        r.lo = __shfl(hlo, fl, RPLU_WAVE);
        r.hi = __shfl(hhi, fl, RPLU_WAVE);
    } else {
        const unsigned long long pos = __ballot(pos_u >= 0);
        if (pos) {
            const int lp = 63 - __clzll(pos);
            r.idx = chunk * CDF_CHUNK + lp * CDF_E + __shfl(pos_u, lp, RPLU_WAVE);
            r.lo = __shfl(plo, lp, RPLU_WAVE);
            r.hi = __shfl(phi, lp, RPLU_WAVE);
        }
    }
    return r;
}

// Wide kernel body: wave w of the grid computes chunk w's total.
template <class MassFn>
__device__ inline void cdf_chunk_totals_wave(int len, double* __restrict__ ct, MassFn mass) {
    const int lane = threadIdx.x % RPLU_WAVE;
    const int chunk = (int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / RPLU_WAVE);
    if (chunk >= cdf_chunks(len)) return;
    CdfChunk c;
    cdf_chunk(c, chunk, len, lane, mass);
    if (lane == 0) ct[chunk] = c.ct;
}

// ------------------------------------------------------ sampler workgroup

struct CdfShared {
    double goff[CDF_MAX_GROUPS + 1];
    int flag[CDF_THREADS / RPLU_WAVE];
    double bcast[4];
    int ibcast[4];
    double amax[CDF_THREADS / RPLU_WAVE];   // wg_argmax: per-wave best value
    int aidx[CDF_THREADS / RPLU_WAVE];      // and its index
};

// Group totals and offsets from the chunk totals ct[0..K); returns T in every
// thread. Thread g sums group g's chunks in order; thread 0 chains groups.
__device__ inline double cdf_levels(CdfShared& sh, const double* __restrict__ ct, int K) {
    const int G = (K + CDF_GROUP - 1) / CDF_GROUP;
    const int g = threadIdx.x;
    if (g < G) {
        const int cnt = min(CDF_GROUP, K - g * CDF_GROUP);   // chunks of the group
        double x[CDF_GROUP];                       // loads issued together
#pragma unroll
        for (int q = 0; q < CDF_GROUP; ++q) x[q] = ct[min(g * CDF_GROUP + q, K - 1)];
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < CDF_GROUP; ++q) {      // in order; no pass past the last chunk
            if (q >= cnt) break;
            s = s + x[q];
        }
        sh.goff[g + 1] = s;                        // group total, for now
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double o = 0.0;
        sh.goff[0] = 0.0;
        for (int q = 0; q < G; ++q) { o = o + sh.goff[q + 1]; sh.goff[q + 1] = o; }
    }
    __syncthreads();
    return sh.goff[G];
}

// After cdf_levels: the drawn index for target (0 <= target < T), same in
// every thread. MassFn gives the masses of the vector (re-walks one chunk).
template <class MassFn>
__device__ CdfPick cdf_draw(CdfShared& sh, const double* __restrict__ ct, int K, int len,
                            MassFn mass, double target) {
    const int G = (K + CDF_GROUP - 1) / CDF_GROUP;
    const int lane = threadIdx.x % RPLU_WAVE, w = threadIdx.x / RPLU_WAVE;
    // first group whose upper end exceeds the target
    const bool above = threadIdx.x < G && sh.goff[threadIdx.x + 1] > target;
    const unsigned long long b = __ballot(above);
    if (lane == 0) sh.flag[w] = b ? w * RPLU_WAVE + (__ffsll(b) - 1) : 0x7fffffff;
    __syncthreads();
    if (w == 0) {
        int g = lane < CDF_THREADS / RPLU_WAVE ? sh.flag[lane] : 0x7fffffff;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) g = min(g, __shfl_xor(g, off, RPLU_WAVE));
        g = min(g, G - 1);                         // T > target: always found
        // chunk inside the group: the first k whose upper end goff + io_{k+1}
        // exceeds the target (the last chunk of the group if none), with the
        // chain io_{k0} = 0, io_{k+1} = io_k + ct_k added left to right as in
        // cdf_levels. Lane q forms io_{k0+q} itself (the same additions in
        // the same order), so every chunk is tested at once.
        const double goff = sh.goff[g];
        const int k0 = g * CDF_GROUP, k1 = min(K, k0 + CDF_GROUP);
        const double myct = ct[min(k0 + lane, K - 1)];   // lane q holds ct[k0 + q]
        double io = 0.0;
        // only lanes below k1 - k0 are read below, and lane q's sum needs
        // the chunks before it: the chain stops at the group's last chunk
#pragma unroll
        for (int q = 0; q < CDF_GROUP - 1; ++q) {
            if (q >= k1 - k0 - 1) break;
            const double c = uniform_lane(myct, q);
            if (q < lane) io = io + c;
        }
        const bool hit = lane < k1 - 1 - k0 && goff + (io + myct) > target;
        const unsigned long long hb = __ballot(hit);
        const int kl = hb ? __ffsll(hb) - 1 : k1 - 1 - k0;
        const int k = k0 + kl;
        io = uniform_lane(io, kl);
        const double before = (k == k0) ? goff : goff + io;
        const CdfPick p = cdf_chunk_select(k, len, lane, mass, goff, io, before, target);
        if (lane == 0) { sh.ibcast[0] = p.idx; sh.bcast[0] = p.lo; sh.bcast[1] = p.hi; }
    }
    __syncthreads();
    const CdfPick r{sh.ibcast[0], sh.bcast[0], sh.bcast[1]};
    __syncthreads();
    return r;
}

}  // namespace rplu
