// CUR-AAA (Alg. 4, Sec. 5.3): rational approximation from samples (z_q, f_q)
// through a CUR decomposition of a Loewner matrix.
//
//   1. split the samples at random: sample q gets the key w0 of Philox with
//      key (seed, 1) and counter (q, 0, 0, 0) (k_aaa_keys); the ceil(m/2)
//      smallest keys (ties by index) form X, the rest Y, each in sample order;
//   2. the Loewner generators G = [f^x / alpha, alpha], B = [alpha; -f^y /
//      alpha] (eq. loewner-generators);
//   3. Alg. 3 (rplu_cauchy) with the max-mass stop: until the largest row
//      mass (or bound) is at most eps^2 times its initial value;
//   4. for the selected rows I (points of X) and columns J (points of Y) in
//      turn: the Loewner matrix of eq. Laaa over the other samples
//      (k_aaa_loewner), its right singular vector of the smallest singular
//      value by one-sided Jacobi rotations on the device (k_jacobi_round, a
//      round-robin schedule of disjoint column pairs per launch, sweeps until
//      no pair rotates), and the largest error of the barycentric
//      interpolant over all samples (k_aaa_eval; eq. aaa-barycentric);
//   5. the fit with the smaller largest error (I on ties).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "common.hpp"
#include "launch.hpp"
#include "runtime.hpp"

namespace rplu {
namespace {

constexpr int AAA_THREADS = 256;
constexpr int AAA_MAX_SWEEPS = 40;

__global__ void k_aaa_keys(int m, uint64_t seed, uint64_t* __restrict__ keys) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < m) keys[q] = philox4x64_10((uint64_t)q, 0, 0, 0, seed, 1).w[0];
}

// L(r, c) = (f(z_rest[r]) - f(t_c)) / (z_rest[r] - t_c), column-major with
// leading dimension M (the rows), kp columns (a zero column pads an odd k).
__global__ void k_aaa_loewner(const cf64* __restrict__ z, const cf64* __restrict__ f,
                              const int32_t* __restrict__ rest, int M,
                              const int32_t* __restrict__ sup, int k, int kp,
                              cf64* __restrict__ L) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)M * kp) return;
    const int c = (int)(e / M), r = (int)(e % M);
    cf64 v{0.0, 0.0};
    if (c < k) {
        const int i = rest[r], j = sup[c];
        v = cdiv(csub(f[i], f[j]), csub(z[i], z[j]));
    }
    L[e] = v;
}

__device__ inline double block_sum(double v, double* red) {
    const int lane = threadIdx.x % RPLU_WAVE, w = threadIdx.x / RPLU_WAVE;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = red[0];
    for (int q = 1; q < AAA_THREADS / RPLU_WAVE; ++q) s += red[q];
    return s;
}

// One round of one-sided (Hestenes) Jacobi on the columns of A (M rows) and
// V (kp rows): workgroup b takes the pair (P[b], Q[b]), forms
// alpha = |a_p|^2, beta = |a_q|^2, gamma = a_p^* a_q, and when
// |gamma| > 1e-15 sqrt(alpha beta) rotates the pair so that it becomes
// orthogonal: with a_q' = conj(gamma) / |gamma| a_q (then a_p^* a_q' is real),
// a_p <- c a_p - s a_q', a_q <- s a_p + c a_q', t = s / c the root of smaller
// magnitude of t^2 + 2 zeta t - 1 = 0, zeta = (beta - alpha) / (2 |gamma|).
__global__ __launch_bounds__(AAA_THREADS) void k_jacobi_round(cf64* __restrict__ A, int M,
                                                              cf64* __restrict__ V, int kp,
                                                              const int32_t* __restrict__ P,
                                                              const int32_t* __restrict__ Q,
                                                              int* __restrict__ rotated) {
    __shared__ double red[AAA_THREADS / RPLU_WAVE];
    __shared__ double rot[5];
    const int p = P[blockIdx.x], q = Q[blockIdx.x];
    cf64* ap = A + (int64_t)p * M;
    cf64* aq = A + (int64_t)q * M;
    double a = 0.0, b = 0.0, gr = 0.0, gi = 0.0;
    for (int i = threadIdx.x; i < M; i += AAA_THREADS) {
        const cf64 x = ap[i], y = aq[i];
        a = fma(x.re, x.re, fma(x.im, x.im, a));
        b = fma(y.re, y.re, fma(y.im, y.im, b));
        gr = fma(x.re, y.re, fma(x.im, y.im, gr));       // conj(x) y
        gi = fma(x.re, y.im, fma(-x.im, y.re, gi));
    }
    a = block_sum(a, red);
    b = block_sum(b, red);
    gr = block_sum(gr, red);
    gi = block_sum(gi, red);
    if (threadIdx.x == 0) {
        const double g = hypot(gr, gi);
        rot[0] = 0.0;
        if (g > 0.0 && g > 1e-15 * sqrt(a * b)) {
            const double zeta = (b - a) / (2.0 * g);
            const double az = fabs(zeta);
            const double t = (zeta >= 0.0 ? 1.0 : -1.0) /
                             (az > 1e150 ? 2.0 * az : az + sqrt(1.0 + zeta * zeta));
            const double c = 1.0 / sqrt(1.0 + t * t);
            rot[0] = 1.0;
            rot[1] = c;
            rot[2] = c * t;
            rot[3] = gr / g;           // conj(gamma) / |gamma|
            rot[4] = -gi / g;
            *rotated = 1;
        }
    }
    __syncthreads();
    if (rot[0] == 0.0) return;
    const double c = rot[1], s = rot[2];
    const cf64 ph{rot[3], rot[4]};
    auto apply = [&](cf64* u, cf64* v, int len) {
        for (int i = threadIdx.x; i < len; i += AAA_THREADS) {
            const cf64 x = u[i];
            const cf64 y = wmul(ph, v[i]);
            u[i] = cf64{c * x.re - s * y.re, c * x.im - s * y.im};
            v[i] = cf64{s * x.re + c * y.re, s * x.im + c * y.im};
        }
    };
    apply(ap, aq, M);
    apply(V + (int64_t)p * kp, V + (int64_t)q * kp, kp);
}

__global__ __launch_bounds__(AAA_THREADS) void k_col_norms(const cf64* __restrict__ A, int M,
                                                           double* __restrict__ out) {
    __shared__ double red[AAA_THREADS / RPLU_WAVE];
    const cf64* a = A + (int64_t)blockIdx.x * M;
    double s = 0.0;
    for (int i = threadIdx.x; i < M; i += AAA_THREADS) s = fma(a[i].re, a[i].re, fma(a[i].im, a[i].im, s));
    s = block_sum(s, red);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// |f(z_i) - r(z_i)| for every sample, r the barycentric form with support
// sup[0..k) and weights w; the largest of each block into bmax.
__global__ __launch_bounds__(AAA_THREADS) void k_aaa_eval(const cf64* __restrict__ z,
                                                          const cf64* __restrict__ f, int m,
                                                          const int32_t* __restrict__ sup,
                                                          const cf64* __restrict__ w, int k,
                                                          double* __restrict__ bmax) {
    __shared__ double red[AAA_THREADS / RPLU_WAVE];
    const int i = blockIdx.x * AAA_THREADS + threadIdx.x;
    double err = 0.0;
    if (i < m) {
        const cf64 zi = z[i];
        cf64 num{0.0, 0.0}, den{0.0, 0.0};
        int hit = -1;
        for (int j = 0; j < k; ++j) {
            const cf64 tj = z[sup[j]];
            if (tj.re == zi.re && tj.im == zi.im) { hit = j; break; }
            const cf64 cw = cdiv(w[j], csub(zi, tj));
            num = cadd(num, wmul(cw, f[sup[j]]));
            den = cadd(den, cw);
        }
        const cf64 r = hit >= 0 ? f[sup[hit]] : cdiv(num, den);
        const cf64 d = csub(f[i], r);
        err = hypot(d.re, d.im);
        if (!(err == err)) err = __builtin_inf();
    }
    const int lane = threadIdx.x % RPLU_WAVE, wv = threadIdx.x / RPLU_WAVE;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) err = fmax(err, __shfl_xor(err, off, RPLU_WAVE));
    if (lane == 0) red[wv] = err;
    __syncthreads();
    if (threadIdx.x == 0) {
        double mx = red[0];
        for (int q = 1; q < AAA_THREADS / RPLU_WAVE; ++q) mx = fmax(mx, red[q]);
        bmax[blockIdx.x] = mx;
    }
}

// Device buffers of one call, freed on every return path.
struct DevBuf {
    std::vector<void*> ptrs;
    ~DevBuf() { for (void* p : ptrs) (void)hipFree(p); }
    hipError_t get(void** out, size_t bytes) {
        hipError_t e = hipMalloc(out, std::max<size_t>(bytes, 256));
        if (e == hipSuccess) ptrs.push_back(*out);
        return e;
    }
};

#define AAA_TRY(expr, what)                              \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

// Support points sup (indices into z, k of them): weights into w_out (k
// complex), the largest error over the samples into *err.
rplu_status aaa_fit(const cf64* z, const cf64* f, int m, const std::vector<int32_t>& sup,
                    cf64* w_dev_out, std::vector<cf64>* w_host, double* err, hipStream_t s) {
    const int k = (int)sup.size();
    const int kp = k + (k & 1);
    std::vector<char> is_sup((size_t)m, 0);
    for (int32_t j : sup) is_sup[(size_t)j] = 1;
    std::vector<int32_t> rest;
    rest.reserve((size_t)(m - k));
    for (int q = 0; q < m; ++q) if (!is_sup[(size_t)q]) rest.push_back(q);
    const int M = (int)rest.size();
    // round-robin schedule of kp players: player 0 fixed, the others rotate
    const int R = kp - 1, H = kp / 2;
    std::vector<int32_t> Ps((size_t)R * H), Qs((size_t)R * H);
    std::vector<int> pos((size_t)kp);
    std::iota(pos.begin(), pos.end(), 0);
    for (int r = 0; r < R; ++r) {
        for (int j = 0; j < H; ++j) {
            Ps[(size_t)r * H + j] = pos[(size_t)j];
            Qs[(size_t)r * H + j] = pos[(size_t)(kp - 1 - j)];
        }
        std::rotate(pos.begin() + 1, pos.end() - 1, pos.end());
    }
    std::vector<cf64> Vh((size_t)kp * kp, cf64{0.0, 0.0});
    for (int q = 0; q < kp; ++q) Vh[(size_t)q * kp + q] = cf64{1.0, 0.0};

    DevBuf db;
    void *dsup, *drest, *dL, *dV, *dP, *dQ, *dflag, *dnorm, *dmax;
    const int nb = (m + AAA_THREADS - 1) / AAA_THREADS;
    AAA_TRY(db.get(&dsup, (size_t)k * 4), "hipMalloc");
    AAA_TRY(db.get(&drest, (size_t)M * 4), "hipMalloc");
    AAA_TRY(db.get(&dL, (size_t)M * kp * 16), "hipMalloc");
    AAA_TRY(db.get(&dV, (size_t)kp * kp * 16), "hipMalloc");
    AAA_TRY(db.get(&dP, Ps.size() * 4), "hipMalloc");
    AAA_TRY(db.get(&dQ, Qs.size() * 4), "hipMalloc");
    AAA_TRY(db.get(&dflag, 4), "hipMalloc");
    AAA_TRY(db.get(&dnorm, (size_t)kp * 8), "hipMalloc");
    AAA_TRY(db.get(&dmax, (size_t)nb * 8), "hipMalloc");
    AAA_TRY(hipMemcpyAsync(dsup, sup.data(), (size_t)k * 4, hipMemcpyHostToDevice, s), "copy");
    AAA_TRY(hipMemcpyAsync(drest, rest.data(), (size_t)M * 4, hipMemcpyHostToDevice, s), "copy");
    AAA_TRY(hipMemcpyAsync(dV, Vh.data(), Vh.size() * 16, hipMemcpyHostToDevice, s), "copy");
    AAA_TRY(hipMemcpyAsync(dP, Ps.data(), Ps.size() * 4, hipMemcpyHostToDevice, s), "copy");
    AAA_TRY(hipMemcpyAsync(dQ, Qs.data(), Qs.size() * 4, hipMemcpyHostToDevice, s), "copy");
    const int64_t ne = (int64_t)M * kp;
    hipLaunchKernelGGL(k_aaa_loewner, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, z, f,
                       (const int32_t*)drest, M, (const int32_t*)dsup, k, kp, (cf64*)dL);
    for (int sweep = 0; sweep < AAA_MAX_SWEEPS && R > 0; ++sweep) {
        AAA_TRY(hipMemsetAsync(dflag, 0, 4, s), "hipMemsetAsync");
        for (int r = 0; r < R; ++r)
            hipLaunchKernelGGL(k_jacobi_round, dim3((unsigned)H), dim3(AAA_THREADS), 0, s,
                               (cf64*)dL, M, (cf64*)dV, kp, (const int32_t*)dP + (size_t)r * H,
                               (const int32_t*)dQ + (size_t)r * H, (int*)dflag);
        int flag = 0;
        AAA_TRY(hipMemcpyAsync(&flag, dflag, 4, hipMemcpyDeviceToHost, s), "copy");
        AAA_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
        if (!flag) break;
    }
    hipLaunchKernelGGL(k_col_norms, dim3((unsigned)kp), dim3(AAA_THREADS), 0, s,
                       (const cf64*)dL, M, (double*)dnorm);
    std::vector<double> nrm((size_t)kp);
    AAA_TRY(hipMemcpyAsync(nrm.data(), dnorm, (size_t)kp * 8, hipMemcpyDeviceToHost, s), "copy");
    AAA_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
    // the smallest singular value among the k real columns (not the pad)
    int pmin = 0;
    for (int q = 1; q < k; ++q) if (nrm[(size_t)q] < nrm[(size_t)pmin]) pmin = q;
    // its right singular vector: column pmin of V (the first k entries)
    cf64* vcol = (cf64*)dV + (size_t)pmin * kp;
    AAA_TRY(hipMemcpyAsync(w_dev_out, vcol, (size_t)k * 16, hipMemcpyDeviceToDevice, s), "copy");
    w_host->resize((size_t)k);
    AAA_TRY(hipMemcpyAsync(w_host->data(), vcol, (size_t)k * 16, hipMemcpyDeviceToHost, s), "copy");
    hipLaunchKernelGGL(k_aaa_eval, dim3((unsigned)nb), dim3(AAA_THREADS), 0, s, z, f, m,
                       (const int32_t*)dsup, (const cf64*)w_dev_out, k, (double*)dmax);
    std::vector<double> bm((size_t)nb);
    AAA_TRY(hipMemcpyAsync(bm.data(), dmax, (size_t)nb * 8, hipMemcpyDeviceToHost, s), "copy");
    AAA_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
    AAA_TRY(hipGetLastError(), "CUR-AAA kernels");
    *err = *std::max_element(bm.begin(), bm.end());
    return RPLU_OK;
}

}  // namespace
}  // namespace rplu

using namespace rplu;

extern "C" rplu_status rplu_cur_aaa(rplu_ctx ctx, int64_t m, const void* z, const void* f,
                                    double eps, uint64_t seed, int64_t max_support,
                                    uint32_t flags, const rplu_opts* bound_opts,
                                    int32_t* support, void* weights, rplu_aaa_info* info,
                                    void* hip_stream) {
    if (ctx == nullptr || info == nullptr || z == nullptr || f == nullptr || support == nullptr ||
        weights == nullptr)
        return fail(RPLU_E_ARG, "rplu_cur_aaa: ctx, z, f, support, weights and info are required");
    if (m < 4 || m > INT32_MAX) return fail(RPLU_E_ARG, "rplu_cur_aaa: m must be in [4, 2^31)");
    if (!(eps > 0.0) || !std::isfinite(eps)) return fail(RPLU_E_ARG, "rplu_cur_aaa: eps must be > 0");
    if (max_support < 1) return fail(RPLU_E_ARG, "rplu_cur_aaa: max_support must be >= 1");
    if (flags & ~(uint32_t)(RPLU_FLAG_C2PLU | RPLU_FLAG_BOUNDS | RPLU_FLAG_NO_GRAPH))
        return fail(RPLU_E_UNSUPPORTED, "rplu_cur_aaa: flags other than C2PLU, BOUNDS, NO_GRAPH");
    std::memset(info, 0, sizeof *info);
    hipError_t e0 = hipSetDevice(ctx->device);
    if (e0 != hipSuccess) return hip_fail(e0, "hipSetDevice");
    hipStream_t s = (hipStream_t)hip_stream;
    const int mi = (int)m;
    DevBuf db;
    void* dkeys;
    AAA_TRY(db.get(&dkeys, (size_t)m * 8), "hipMalloc");
    hipLaunchKernelGGL(k_aaa_keys, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, mi, seed,
                       (uint64_t*)dkeys);
    std::vector<uint64_t> keys((size_t)m);
    std::vector<cf64> hz((size_t)m), hf((size_t)m);
    AAA_TRY(hipMemcpyAsync(keys.data(), dkeys, (size_t)m * 8, hipMemcpyDeviceToHost, s), "copy");
    AAA_TRY(hipMemcpyAsync(hz.data(), z, (size_t)m * 16, hipMemcpyDeviceToHost, s), "copy");
    AAA_TRY(hipMemcpyAsync(hf.data(), f, (size_t)m * 16, hipMemcpyDeviceToHost, s), "copy");
    AAA_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
    // 1. the split: the ceil(m/2) smallest keys (ties by index) form X
    std::vector<int32_t> order((size_t)m);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return keys[(size_t)a] < keys[(size_t)b]; });
    const int nx = (mi + 1) / 2, ny = mi - nx;
    std::vector<int32_t> X(order.begin(), order.begin() + nx), Y(order.begin() + nx, order.end());
    std::sort(X.begin(), X.end());
    std::sort(Y.begin(), Y.end());
    // 2. Loewner generators (eq. loewner-generators)
    double fmax = 0.0;
    for (const cf64& v : hf) fmax = std::max(fmax, std::hypot(v.re, v.im));
    const double alpha = std::sqrt(fmax);
    if (!(alpha > 0.0) || !std::isfinite(alpha))
        return fail(RPLU_E_NONFINITE, "rplu_cur_aaa: the values are all zero or not finite");
    std::vector<cf64> hx((size_t)nx), hy((size_t)ny), hG((size_t)nx * 2), hB((size_t)2 * ny);
    for (int q = 0; q < nx; ++q) {
        const cf64 v = hf[(size_t)X[(size_t)q]];
        hx[(size_t)q] = hz[(size_t)X[(size_t)q]];
        hG[(size_t)2 * q] = cf64{v.re / alpha, v.im / alpha};
        hG[(size_t)2 * q + 1] = cf64{alpha, 0.0};
    }
    for (int q = 0; q < ny; ++q) {
        const cf64 v = hf[(size_t)Y[(size_t)q]];
        hy[(size_t)q] = hz[(size_t)Y[(size_t)q]];
        hB[(size_t)q] = cf64{alpha, 0.0};
        hB[(size_t)ny + q] = cf64{-v.re / alpha, -v.im / alpha};
    }
    void *dx, *dy, *dG, *dB, *dpiv;
    const int64_t kmax = std::min<int64_t>(max_support, std::min(nx, ny));
    AAA_TRY(db.get(&dx, (size_t)nx * 16), "hipMalloc");
    AAA_TRY(db.get(&dy, (size_t)ny * 16), "hipMalloc");
    AAA_TRY(db.get(&dG, (size_t)nx * 32), "hipMalloc");
    AAA_TRY(db.get(&dB, (size_t)ny * 32), "hipMalloc");
    AAA_TRY(db.get(&dpiv, (size_t)kmax * 8), "hipMalloc");
    AAA_TRY(hipMemcpyAsync(dx, hx.data(), (size_t)nx * 16, hipMemcpyHostToDevice, s), "copy");
    AAA_TRY(hipMemcpyAsync(dy, hy.data(), (size_t)ny * 16, hipMemcpyHostToDevice, s), "copy");
    AAA_TRY(hipMemcpyAsync(dG, hG.data(), (size_t)nx * 32, hipMemcpyHostToDevice, s), "copy");
    AAA_TRY(hipMemcpyAsync(dB, hB.data(), (size_t)ny * 32, hipMemcpyHostToDevice, s), "copy");
    // 3. Alg. 3 with the max-mass stop
    rplu_opts o;
    std::memset(&o, 0, sizeof o);
    if (bound_opts) o = *bound_opts;
    o.max_rank = kmax;
    o.rel_tol = eps;
    o.seed = seed;
    o.flags = flags | RPLU_FLAG_MAXMASS_STOP;
    o.forced = nullptr;
    o.trace = nullptr;
    o.rowmass_out = nullptr;
    o.colmass_out = nullptr;
    rplu_info ri;
    rplu_status rc = rplu_cauchy(ctx, RPLU_C128, nx, ny, 2, dx, dy, dG, dB, &o, (int32_t*)dpiv,
                                 nullptr, 0, nullptr, 0, &ri, hip_stream);
    if (rc) return rc;
    info->rank = ri.rank;
    info->stop = ri.stop;
    info->trials = ri.trials;
    const int k = (int)ri.rank;
    if (k < 1) return fail(RPLU_E_ARG, "rplu_cur_aaa: no pivot was taken");
    std::vector<int32_t> piv((size_t)2 * k);
    AAA_TRY(hipMemcpyAsync(piv.data(), dpiv, (size_t)k * 8, hipMemcpyDeviceToHost, s), "copy");
    AAA_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
    // 4. the two fits
    std::vector<int32_t> supI((size_t)k), supJ((size_t)k);
    for (int t = 0; t < k; ++t) {
        supI[(size_t)t] = X[(size_t)piv[(size_t)2 * t]];
        supJ[(size_t)t] = Y[(size_t)piv[(size_t)2 * t + 1]];
    }
    void *dwI, *dwJ;
    AAA_TRY(db.get(&dwI, (size_t)k * 16), "hipMalloc");
    AAA_TRY(db.get(&dwJ, (size_t)k * 16), "hipMalloc");
    std::vector<cf64> wI, wJ;
    double eI = 0.0, eJ = 0.0;
    rc = aaa_fit((const cf64*)z, (const cf64*)f, mi, supI, (cf64*)dwI, &wI, &eI, s);
    if (rc) return rc;
    rc = aaa_fit((const cf64*)z, (const cf64*)f, mi, supJ, (cf64*)dwJ, &wJ, &eJ, s);
    if (rc) return rc;
    // 5. the better fit
    const bool useI = !(eJ < eI);
    const std::vector<int32_t>& sup = useI ? supI : supJ;
    AAA_TRY(hipMemcpyAsync(support, sup.data(), (size_t)k * 4, hipMemcpyHostToDevice, s), "copy");
    AAA_TRY(hipMemcpyAsync(weights, useI ? dwI : dwJ, (size_t)k * 16, hipMemcpyDeviceToDevice, s),
            "copy");
    AAA_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
    info->k = k;
    info->which = useI ? 0 : 1;
    info->max_err = useI ? eI : eJ;
    info->err_rows = eI;
    info->err_cols = eJ;
    return RPLU_OK;
}
