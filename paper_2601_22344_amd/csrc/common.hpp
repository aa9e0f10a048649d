// Device-side building blocks shared by the RPLU kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rplu.h"

#define RPLU_WAVE 64

namespace rplu {

// ---------------------------------------------------------------- complex

struct cf32 { float re, im; };
struct cf64 { double re, im; };

// Scalar traits: storage type T, its FP64 "wide" form W (double or cf64),
// |z|^2 in FP64, and the FMA-form update s - l*u in the storage precision.
template <class T> struct Sc;

template <> struct Sc<float> {
    using W = double;
    static constexpr bool cplx = false;
    __device__ __host__ static inline double mag2(float v) { double d = v; return d * d; }
    // acc + |v|^2 with one rounding (the square of a float is exact in FP64);
    // every row-mass sum uses it, so that no kernel's sum depends on where
    // the compiler contracts a multiply and an add
    __device__ static inline double mag2_add(double acc, float v) { double d = v; return fma(d, d, acc); }
    __device__ static inline W widen(float v) { return (double)v; }
    __device__ static inline float narrow(W v) { return (float)v; }
    __device__ static inline float zero() { return 0.f; }
    __device__ static inline float one() { return 1.f; }
    __device__ static inline float fms(float s, float l, float u) { return fmaf(-l, u, s); }
    __device__ static inline double re(float v) { return v; }
    __device__ static inline double im(float) { return 0.0; }
};

template <> struct Sc<double> {
    using W = double;
    static constexpr bool cplx = false;
    __device__ __host__ static inline double mag2(double v) { return v * v; }
    __device__ static inline double mag2_add(double acc, double v) { return fma(v, v, acc); }
    __device__ static inline W widen(double v) { return v; }
    __device__ static inline double narrow(W v) { return v; }
    __device__ static inline double zero() { return 0.0; }
    __device__ static inline double one() { return 1.0; }
    __device__ static inline double fms(double s, double l, double u) { return fma(-l, u, s); }
    __device__ static inline double re(double v) { return v; }
    __device__ static inline double im(double) { return 0.0; }
};

template <> struct Sc<cf32> {
    using W = cf64;
    static constexpr bool cplx = true;
    // explicit fma: every call site rounds |z|^2 the same way
    __device__ __host__ static inline double mag2(cf32 v) {
        double a = v.re, b = v.im;
        return fma(a, a, b * b);
    }
    __device__ static inline double mag2_add(double acc, cf32 v) { return acc + mag2(v); }
    __device__ static inline W widen(cf32 v) { return {(double)v.re, (double)v.im}; }
    __device__ static inline cf32 narrow(W v) { return {(float)v.re, (float)v.im}; }
    __device__ static inline cf32 zero() { return {0.f, 0.f}; }
    __device__ static inline cf32 one() { return {1.f, 0.f}; }
    // s - l*u = (s.re - l.re u.re + l.im u.im, s.im - l.re u.im - l.im u.re)
    __device__ static inline cf32 fms(cf32 s, cf32 l, cf32 u) {
        float r = fmaf(-l.re, u.re, s.re);
        r = fmaf(l.im, u.im, r);
        float i = fmaf(-l.re, u.im, s.im);
        i = fmaf(-l.im, u.re, i);
        return {r, i};
    }
    __device__ static inline double re(cf32 v) { return v.re; }
    __device__ static inline double im(cf32 v) { return v.im; }
};

template <> struct Sc<cf64> {
    using W = cf64;
    static constexpr bool cplx = true;
    __device__ __host__ static inline double mag2(cf64 v) { return fma(v.re, v.re, v.im * v.im); }
    __device__ static inline double mag2_add(double acc, cf64 v) { return acc + mag2(v); }
    __device__ static inline W widen(cf64 v) { return v; }
    __device__ static inline cf64 narrow(W v) { return v; }
    __device__ static inline cf64 zero() { return {0.0, 0.0}; }
    __device__ static inline cf64 one() { return {1.0, 0.0}; }
    __device__ static inline cf64 fms(cf64 s, cf64 l, cf64 u) {
        double r = fma(-l.re, u.re, s.re);
        r = fma(l.im, u.im, r);
        double i = fma(-l.re, u.im, s.im);
        i = fma(-l.im, u.re, i);
        return {r, i};
    }
    __device__ static inline double re(cf64 v) { return v.re; }
    __device__ static inline double im(cf64 v) { return v.im; }
};

__device__ inline double wmul(double a, double b) { return a * b; }
__device__ inline cf64 wmul(cf64 a, cf64 b) {
    return {fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}
__device__ inline cf64 cadd(cf64 a, cf64 b) { return {a.re + b.re, a.im + b.im}; }
__device__ inline cf64 csub(cf64 a, cf64 b) { return {a.re - b.re, a.im - b.im}; }

// 1/a in FP64. Complex: Smith's scaling avoids overflow/underflow of |a|^2.
__device__ inline double winv(double a) { return 1.0 / a; }
__device__ inline cf64 winv(cf64 a) {
    if (fabs(a.re) >= fabs(a.im)) {
        double r = a.im / a.re, d = a.re + a.im * r;
        return {1.0 / d, -r / d};
    } else {
        double r = a.re / a.im, d = a.re * r + a.im;
        return {r / d, -1.0 / d};
    }
}
// a / b, complex, Smith's algorithm.
__device__ inline cf64 cdiv(cf64 a, cf64 b) {
    if (fabs(b.re) >= fabs(b.im)) {
        double r = b.im / b.re, d = b.re + b.im * r;
        return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
    } else {
        double r = b.re / b.im, d = b.re * r + b.im;
        return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
    }
}

// 1/d for d > 0 in FP64: hardware reciprocal estimate refined by two Newton
// steps r <- r + r (1 - d r), each of which roughly doubles the correct bits.
__device__ inline double rcp_refined(double d) {
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    return fma(r, e, r);
}

// a / b as a conj(b) / |b|^2 with one refined reciprocal when |b|^2 lies well
// inside the FP64 range; Smith's algorithm otherwise.
__device__ inline cf64 cdiv_fast(cf64 a, cf64 b) {
    const double d2 = fma(b.re, b.re, b.im * b.im);
    if (d2 >= 0x1p-1000 && d2 <= 0x1p+1000) {
        const double r = rcp_refined(d2);
        return {fma(a.re, b.re, a.im * b.im) * r, fma(a.im, b.re, -a.re * b.im) * r};
    }
    return cdiv(a, b);
}

// ------------------------------------------------------------------ Philox

// Philox4x64-10 (Salmon et al., SC'11): ten rounds of two 64x64->128-bit
// multiplications with key bumps by 64-bit Weyl constants between rounds.
struct Philox4 { uint64_t w[4]; };

__device__ inline Philox4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                        uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += W0; k1 += W1; }
        uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    return {{c0, c1, c2, c3}};
}

__device__ inline double unit_from_word(uint64_t w) {
    return (double)(w >> 11) * 0x1.0p-53;
}

// ------------------------------------------------------------ reductions

// Cross-lane moves of a double as two 32-bit halves, all 64 lanes active.
// dpp_d: the value of the lane that the DPP control CTRL selects (within a
// row of 16 lanes). swap_sum32 / swap_sum16: v + v(lane ^ 32) / v + v(lane ^
// 16), from the gfx950 lane swaps (the first result holds the lower half-wave
// or the even rows in both places, the second the upper half or the odd rows,
// so each lane adds its own value and its partner's).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_update_dpp(0u, (uint32_t)b, CTRL, 0xf, 0xf, false);
    const uint32_t hi = __builtin_amdgcn_update_dpp(0u, (uint32_t)(b >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ double swap_sum32(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)b, (uint32_t)b, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(b >> 32), (uint32_t)(b >> 32), false, false);
    return __builtin_bit_cast(double, ((uint64_t)hi[0] << 32) | lo[0]) +
           __builtin_bit_cast(double, ((uint64_t)hi[1] << 32) | lo[1]);
}

__device__ __forceinline__ double swap_sum16(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const auto lo = __builtin_amdgcn_permlane16_swap((uint32_t)b, (uint32_t)b, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((uint32_t)(b >> 32), (uint32_t)(b >> 32), false, false);
    return __builtin_bit_cast(double, ((uint64_t)hi[0] << 32) | lo[0]) +
           __builtin_bit_cast(double, ((uint64_t)hi[1] << 32) | lo[1]);
}

// Sum over the 64 lanes, the same in every lane: the butterfly
// v <- v + v(lane ^ d) for d = 32, 16, 8, 4, 2, 1, without LDS. Within a row
// of 16 lanes a rotation by 8 is lane ^ 8; after the steps d' > d a lane's
// value depends only on lane mod 2d, where a rotation by d and lane ^ d pick
// equal values. Every step adds the butterfly's two operands (addition
// commutes), so each lane gets the butterfly's bits. Call with every lane of
// the wave active.
__device__ inline double wave_sum(double v) {
    v = swap_sum32(v);
    v = swap_sum16(v);
    v = v + dpp_d<0x128>(v);     // row_ror:8
    v = v + dpp_d<0x124>(v);     // row_ror:4
    v = v + dpp_d<0x122>(v);     // row_ror:2
    v = v + dpp_d<0x121>(v);     // row_ror:1
    return v;
}

// The value v of lane q (q the same in every lane), for every lane.
__device__ inline double uniform_lane(double v, int q) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)b, q);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(b >> 32), q);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Inclusive scan across the 64 lanes of a wave (Hillis-Steele).
__device__ inline double wave_incl_scan(double v, int lane) {
#pragma unroll
    for (int off = 1; off < RPLU_WAVE; off <<= 1) {
        double o = __shfl_up(v, off, RPLU_WAVE);
        if (lane >= off) v += o;
    }
    return v;
}

// --------------------------------------------------------------- state

constexpr double RPLU_STALL_RATIO = 63.0 / 64.0;   // see RPLU_FLAG_STALL_STOP

// Per-run device state. The row draw of step t reads t, runs the stop test,
// and records cur = t and the row i; the column draw records j, the pivot
// and its reciprocal and sets t = t + 1; the other kernels of the step read
// cur, i, j. Only the workgroup running a draw writes the state (besides the
// arrival counter of the wide draw kernels).
struct StepState {
    int32_t t;          // pivots taken so far
    int32_t cur;        // step the current sweep/update applies
    int32_t done;       // 1 once the stop test fired or an error occurred
    int32_t stop;       // RPLU_STOP_*
    int32_t error;      // 0 or an RPLU_E_* code raised on the device
    int32_t i, j;       // current pivot
    int32_t pad;
    double T0, T;       // ||A||_F^2 and the latest total
    double T_best;      // stall rule: best total so far and the step it was
    int32_t t_best;     // reached (an improvement is a fall below 63/64 of it)
    int32_t pad2;
    double a_re, a_im;  // pivot entry
    double inv_re, inv_im;  // 1/a in FP64
    double row_tgt, row_lo, row_hi;   // row draw: target u1*T and its bin edges
    double gi[8];       // Cauchy: copy of G_i,: (p <= 4 complex)
    double bj[8];       // Cauchy: copy of B_:,j
    uint32_t arrive;    // workgroups of the running wide draw kernel that
                        // are done (0 between launches)
    uint32_t pad3;
    double T_ref;       // RPLU_FLAG_REFRESH: the total at the start or at the
                        // last residual replacement (inf: take the next one)
    int32_t refresh_on; // replacements left to trigger (0 or 1)
    int32_t t_base;     // deferred sweep: S in memory holds S^(t_base); the
                        // updates of steps t_base.. are applied on the fly
    int32_t flushed;    // deferred sweep: the step whose S^(flushed) the last
                        // write-back stored (the next draw moves t_base there)
    int32_t pad4;
    double sig_re, sig_im;  // CUR form: sigma = A[i, j] - z^T U_k w of the step
    double l2;              // CUR form: ||l||^2 of the step
    int32_t trials;         // RPLU_FLAG_BOUNDS: trials of the step's row draw
    int32_t wbad;           // Cauchy, p = 1: some w_j = |b_j|^2 of the mass
                            // kernel's column data lies outside {0} and
                            // [2^-500, 2^500] (set by the generator update,
                            // cleared by the row draw of every step)
    int64_t trials_total;   // and over the run
    double M0;              // max-mass stop rule: the largest row mass at step 0
};

}  // namespace rplu
