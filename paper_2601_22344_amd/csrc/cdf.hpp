// Inverse-CDF sampling over a mass vector inside one 1024-thread workgroup.
//
// The index drawn for a target u*T is the first index e whose inclusive
// prefix P(e) of the masses exceeds u*T (two-stage exact sampling draws a row
// by its mass, then a column of that row by |S_ij|^2; Sec. 4.1).
//
// Prefix structure (two levels, deterministic for a given length):
//   * wave w of the 16 waves owns the contiguous range [w*Rw, (w+1)*Rw),
//     Rw a multiple of 64, walked in 64-element chunks; inside a chunk the
//     lanes form an inclusive Hillis-Steele scan with shuffles and a running
//     carry links the chunks, giving the wave-local prefix p(e) and the wave
//     total tot_w = p(last);
//   * the wave offsets are chained sequentially: off_0 = 0,
//     off_{w+1} = off_w + tot_w, and the total is T := off_16. The wave
//     intervals [off_w, off_{w+1}) therefore tile [0, T) with no gap.
// The drawn index lies in the first wave with off_{w+1} > u*T; in that wave
// the global prefix is P(e) = off_w + p(e), and P(last) == off_{w+1}
// bit for bit, so a hit always exists. A hit must also have positive mass;
// if rounding in off_w + p(e) leaves only zero-mass hits, the last
// positive-mass index of the wave is taken (the wave has one, as its total
// is positive). This keeps a zero-mass index from ever being drawn.
#pragma once

#include "common.hpp"

namespace rplu {

constexpr int CDF_THREADS = 1024;
constexpr int CDF_WAVES = CDF_THREADS / RPLU_WAVE;

struct CdfShared {
    double tot[CDF_WAVES];
    double off[CDF_WAVES + 1];
    double bcast[4];
    int ibcast[4];
};

struct CdfPick {
    int idx;        // drawn index
    double lo, hi;  // CDF edges of the drawn bin: P(idx-1), P(idx)
};

__device__ inline int cdf_wave_range(int len) {
    int r = (len + CDF_WAVES - 1) / CDF_WAVES;
    return (r + RPLU_WAVE - 1) / RPLU_WAVE * RPLU_WAVE;
}

// Pass 1: returns T (same value in every thread). MassFn: double(int e),
// called only for 0 <= e < len.
template <class MassFn>
__device__ double cdf_total(CdfShared& sh, int len, MassFn mass) {
    const int lane = threadIdx.x % RPLU_WAVE, w = threadIdx.x / RPLU_WAVE;
    const int Rw = cdf_wave_range(len);
    const int b = w * Rw, e_end = min(len, b + Rw);
    double carry = 0.0;
    for (int c = b; c < e_end; c += RPLU_WAVE) {
        int e = c + lane;
        double v = e < e_end ? mass(e) : 0.0;
        double s = wave_incl_scan(v, lane);
        // link chunks through the last VALID lane, so that p(last) == tot_w
        carry += __shfl(s, min(RPLU_WAVE, e_end - c) - 1, RPLU_WAVE);
    }
    if (lane == 0) sh.tot[w] = carry;
    __syncthreads();
    if (threadIdx.x == 0) {
        double o = 0.0;
        sh.off[0] = 0.0;
        for (int q = 0; q < CDF_WAVES; ++q) { o = o + sh.tot[q]; sh.off[q + 1] = o; }
    }
    __syncthreads();
    return sh.off[CDF_WAVES];
}

// Pass 2, after cdf_total on the same data: the drawn index for `target`
// (0 <= target < T), its bin edges, same result in every thread.
template <class MassFn>
__device__ CdfPick cdf_select(CdfShared& sh, int len, MassFn mass, double target) {
    const int lane = threadIdx.x % RPLU_WAVE, w = threadIdx.x / RPLU_WAVE;
    int ww = 0;
    while (ww < CDF_WAVES - 1 && !(sh.off[ww + 1] > target)) ++ww;
    if (w == ww) {
        const int Rw = cdf_wave_range(len);
        const int b = w * Rw, e_end = min(len, b + Rw);
        const double base = sh.off[w];
        double carry = 0.0;
        int found = -1, last_pos = -1;
        double flo = 0.0, fhi = 0.0, plo = base, phi = base;
        for (int c = b; c < e_end; c += RPLU_WAVE) {
            int e = c + lane;
            double v = e < e_end ? mass(e) : 0.0;
            double s = wave_incl_scan(v, lane);
            double P = base + (carry + s);
            double Pprev = __shfl_up(P, 1, RPLU_WAVE);
            if (lane == 0) Pprev = (c == b) ? base : base + carry;
            bool hit = (e < e_end) && (v > 0.0) && (P > target);
            unsigned long long bal = __ballot(hit);
            unsigned long long pos = __ballot((e < e_end) && (v > 0.0));
            if (pos) {
                int lp = 63 - __clzll(pos);
                int cand = c + lp;
                double lo = __shfl(Pprev, lp, RPLU_WAVE), hi = __shfl(P, lp, RPLU_WAVE);
                last_pos = cand; plo = lo; phi = hi;
            }
            if (bal) {
                int fl = __ffsll(bal) - 1;
                found = c + fl;
                flo = __shfl(Pprev, fl, RPLU_WAVE);
                fhi = __shfl(P, fl, RPLU_WAVE);
                break;
            }
            carry += __shfl(s, min(RPLU_WAVE, e_end - c) - 1, RPLU_WAVE);
        }
        if (found < 0) { found = last_pos; flo = plo; fhi = phi; }
        if (lane == 0) { sh.ibcast[0] = found; sh.bcast[0] = flo; sh.bcast[1] = fhi; }
    }
    __syncthreads();
    CdfPick r{sh.ibcast[0], sh.bcast[0], sh.bcast[1]};
    __syncthreads();
    return r;
}

}  // namespace rplu
