// Verification of a rank-k factorisation with FP64 matrix cores, and the
// residual replacement S := A - L U of a single-precision run.
//
// The residual after k steps is A^(k) = A - A_hat^(k) with A_hat^(k) = L U
// (eqs. residual_update and approximation_update; Alg. 1 builds L(:,t) and
// U(t,:) so that the sum of their outer products is A_hat^(k)). This pass
// forms E = A - L U tile by tile and reduces, in FP64,
//   ||A||_F^2,  ||A - L U||_F^2  and  ||A - L U - S||_F^2
// where S is the Schur complement the factorisation left behind (optional).
// The first gives the approximation error of the method; the second is zero
// up to rounding when L, U and S are consistent.
//
// L U is a dense contraction over k: each workgroup owns a 128 x 128 tile of
// E, stages 16-wide slices of L and U (converted to FP64) in LDS and runs
// v_mfma_f64_16x16x4f64; each of its 4 waves accumulates a 64 x 64 quarter
// as 4 x 4 MFMA blocks. Operand layout of one 16x16x4 step (lane l):
//   A operand: L(row0 + l % 16, k0 + l / 16);  B operand: U(k0 + l / 16, col0 + l % 16)
//   result:    register r holds block entry (4 r + l / 16, l % 16).
// Per-tile sums are reduced by wave sums and a fixed-order combine; the tile
// partials are then summed by one workgroup in a fixed order, so the result
// does not depend on scheduling.
#include "common.hpp"
#include "launch.hpp"

namespace rplu {

constexpr int VF_TILE = 128;
constexpr int VF_KC = 16;
constexpr int VF_THREADS = 256;
constexpr int VF_PAD = 4;                 // LDS row padding (doubles)

typedef double vf_d4 __attribute__((ext_vector_type(4)));

template <class T>
__device__ inline double vf_load(const T* p) { return (double)*p; }

// MODE 0: norms of A and E; 1: also ||E - S||; 2 (refresh): no norms, E
// rounded to T is written to S (the residual replacement of a run that has
// stalled in single precision).
// The k loop is software pipelined: the slice k0 + 16 is loaded from global
// memory into registers while the matrix cores work on slice k0 from one of
// two LDS buffers, so one barrier per slice suffices (a buffer is written
// again only after every wave has passed the barrier that follows its last
// read). Two workgroups fit on a CU (waves_per_eu 2).
template <class T, int MODE>
__global__ __launch_bounds__(VF_THREADS) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_verify(
    int n, int m, int k, const T* __restrict__ A, int64_t lda, const T* __restrict__ L,
    int64_t ldl, const T* __restrict__ U, int64_t ldu, const T* S, int64_t lds,
    double* __restrict__ partial) {
    constexpr bool WITH_S = MODE == 1;
    __shared__ double sL[2][VF_KC][VF_TILE + VF_PAD];
    __shared__ double sU[2][VF_KC][VF_TILE + VF_PAD];
    __shared__ double sred[VF_THREADS / RPLU_WAVE][3];
    const int tid = threadIdx.x, lane = tid % RPLU_WAVE, wv = tid / RPLU_WAVE;
    const int wy = wv / 2, wx = wv % 2;
    const int r0 = blockIdx.y * VF_TILE, c0 = blockIdx.x * VF_TILE;
    vf_d4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = vf_d4{0.0, 0.0, 0.0, 0.0};

    const int lr = tid % VF_TILE;        // row (of L) / column (of U) this thread stages
    const int lk = tid / VF_TILE;        // 0 or 1: first slice column it stages
    const bool rin = r0 + lr < n, cin = c0 + lr < m;
    const T* Lp = L + r0 + lr;
    const T* Up = U + c0 + lr;
    T pl[VF_KC / 2], pu[VF_KC / 2];
    // L(r0.., k0..k0+15) and U(k0..k0+15, c0..) into registers, zero outside
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < VF_KC / 2; ++q) {
            const int kk = k0 + lk + 2 * q;
            const bool kin = kk < k;
            pl[q] = (kin && rin) ? Lp[(int64_t)kk * ldl] : (T)0;
            pu[q] = (kin && cin) ? Up[(int64_t)kk * ldu] : (T)0;
        }
    };
    fetch(0);
    int buf = 0;
    for (int k0 = 0; k0 < k; k0 += VF_KC) {
#pragma unroll
        for (int q = 0; q < VF_KC / 2; ++q) {
            sL[buf][lk + 2 * q][lr] = (double)pl[q];
            sU[buf][lk + 2 * q][lr] = (double)pu[q];
        }
        __syncthreads();
        if (k0 + VF_KC < k) fetch(k0 + VF_KC);
#pragma unroll
        for (int kq = 0; kq < VF_KC / 4; ++kq) {
            const int kr = kq * 4 + lane / 16;
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = sL[buf][kr][wy * 64 + i * 16 + lane % 16];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = sU[buf][kr][wx * 64 + j * 16 + lane % 16];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        buf ^= 1;
    }

    double sa = 0.0, se = 0.0, ss = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = r0 + wy * 64 + i * 16 + 4 * r + lane / 16;
                const int col = c0 + wx * 64 + j * 16 + lane % 16;
                if (row < n && col < m) {
                    const double av = vf_load(A + (int64_t)row * lda + col);
                    const double e = av - acc[i][j][r];
                    if constexpr (MODE == 2) {
                        const_cast<T*>(S)[(int64_t)row * lds + col] = (T)e;
                        continue;
                    }
                    sa = fma(av, av, sa);
                    se = fma(e, e, se);
                    if constexpr (WITH_S) {
                        const double e2 = e - vf_load(S + (int64_t)row * lds + col);
                        ss = fma(e2, e2, ss);
                    }
                }
            }
    if constexpr (MODE == 2) return;
    sa = wave_sum(sa);
    se = wave_sum(se);
    ss = wave_sum(ss);
    if (lane == 0) { sred[wv][0] = sa; sred[wv][1] = se; sred[wv][2] = ss; }
    __syncthreads();
    if (tid < 3) {
        double v = sred[0][tid];
        for (int w = 1; w < VF_THREADS / RPLU_WAVE; ++w) v += sred[w][tid];
        partial[((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * 3 + tid] = v;
    }
}

// One workgroup: out[q] = sum over tiles of partial[tile][q], in a fixed
// order (per-thread strided sums, then a fixed tree).
__global__ __launch_bounds__(256) void k_verify_reduce(const double* __restrict__ partial,
                                                       int64_t tiles, double* __restrict__ out) {
    __shared__ double red[256][3];
    double v[3] = {0.0, 0.0, 0.0};
    for (int64_t t = threadIdx.x; t < tiles; t += 256)
#pragma unroll
        for (int q = 0; q < 3; ++q) v[q] += partial[t * 3 + q];
#pragma unroll
    for (int q = 0; q < 3; ++q) red[threadIdx.x][q] = v[q];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
#pragma unroll
            for (int q = 0; q < 3; ++q) red[threadIdx.x][q] += red[threadIdx.x + h][q];
        __syncthreads();
    }
    if (threadIdx.x < 3) out[threadIdx.x] = red[0][threadIdx.x];
}

int64_t verify_tiles(int64_t n, int64_t m) {
    return ((n + VF_TILE - 1) / VF_TILE) * ((m + VF_TILE - 1) / VF_TILE);
}

template <class T>
static void verify_t(const VerifyArgs& a, hipStream_t s) {
    const dim3 grid((unsigned)((a.m + VF_TILE - 1) / VF_TILE), (unsigned)((a.n + VF_TILE - 1) / VF_TILE));
    if (a.S)
        hipLaunchKernelGGL((k_verify<T, 1>), grid, dim3(VF_THREADS), 0, s, (int)a.n, (int)a.m,
                           (int)a.k, (const T*)a.A, a.lda, (const T*)a.L, a.ldl, (const T*)a.U,
                           a.ldu, (const T*)a.S, a.lds, a.partial);
    else
        hipLaunchKernelGGL((k_verify<T, 0>), grid, dim3(VF_THREADS), 0, s, (int)a.n, (int)a.m,
                           (int)a.k, (const T*)a.A, a.lda, (const T*)a.L, a.ldl, (const T*)a.U,
                           a.ldu, (const T*)nullptr, (int64_t)0, a.partial);
    hipLaunchKernelGGL(k_verify_reduce, dim3(1), dim3(256), 0, s, a.partial,
                       verify_tiles(a.n, a.m), a.out);
}

void launch_verify(const VerifyArgs& a, hipStream_t s) {
    if (a.dtype == RPLU_R64) verify_t<double>(a, s);
    else verify_t<float>(a, s);
}

template <class T>
static void refresh_t(const RefreshArgs& a, hipStream_t s) {
    const dim3 grid((unsigned)((a.m + VF_TILE - 1) / VF_TILE), (unsigned)((a.n + VF_TILE - 1) / VF_TILE));
    hipLaunchKernelGGL((k_verify<T, 2>), grid, dim3(VF_THREADS), 0, s, (int)a.n, (int)a.m, (int)a.t,
                       (const T*)a.A, a.lda, (const T*)a.L, a.ldl, (const T*)a.U, a.ldu,
                       (const T*)a.S, a.lds, (double*)nullptr);
}

void launch_refresh(const RefreshArgs& a, hipStream_t s) {
    if (a.dtype == RPLU_R64) refresh_t<double>(a, s);
    else refresh_t<float>(a, s);
}

}  // namespace rplu
