// Batched dense RPLU: many independent instances in one persistent launch.
//
// Each workgroup (512 threads) takes instances from a device work queue (an
// atomic counter over a host-ordered table, largest estimated cost first)
// and runs an instance's whole step loop (Alg. 1 with two-stage sampling,
// Sec. 4.1) with workgroup barriers only. Row masses and the scaled pivot
// column live in LDS; the pivot row goes to U(t,:) (or a per-workgroup row).
//
// Every reduction uses the thread-to-element mapping and order of the
// single-instance path (the sweep's 512 threads x 16-byte packs, its wave
// sums and fixed-order sum over the 8 waves; the chunk totals, the chain and
// the in-chunk select of cdf.hpp), so an instance's pivots and factors are
// bitwise those of rplu_dense on the same buffer. Two schedule knobs leave
// the arithmetic unchanged and are left to the autotuner:
//   * R, the rows a lane group sweeps per pass (each row keeps its own
//     partial sums, so R changes only how many rows are in flight);
//   * the number of resident workgroups per CU.
// When a row needs only 1, 2 or 4 of the 8 waves, the workgroup splits into
// 8, 4 or 2 lane groups that sweep different rows at once: the idle waves of
// the single-instance kernel add exact zeros after the active ones.
#include <type_traits>

#include "common.hpp"
#include "cdf.hpp"
#include "launch.hpp"

namespace rplu {

constexpr int BT_THREADS = 512;
constexpr int BT_WAVES = BT_THREADS / RPLU_WAVE;
constexpr int BT_MAXK = RPLU_BATCH_MAX_DIM / CDF_CHUNK;   // chunks of a mass vector
constexpr int BT_MAXR = 8;

static_assert(BT_THREADS == DENSE_THREADS, "same sweep mapping as rplu_dense");
static_assert(BT_MAXK <= CDF_GROUP, "one CDF group: the chain is a single sequential sum");

template <class T, int V>
struct alignas(V == 1 ? alignof(T) : 16) BPack { T v[V]; };
static_assert(sizeof(BPack<float, 1>) == 4 && sizeof(BPack<double, 2>) == 16, "pack size");

struct BtShared {
    double ctr[BT_MAXK];                  // chunk totals: row masses
    double ctc[BT_MAXK];                  // chunk totals: pivot row
    double red[2][BT_WAVES][BT_MAXR];     // per-wave row sums, double-buffered
    double bc[4];
    int bi[2];
    int job;
};

// Values every lane of the workgroup holds alike (read from LDS after a
// barrier), moved to scalar registers so that everything derived from them
// (the job's pointers and sizes, the pivot) stays out of vector registers.
__device__ __forceinline__ int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double uniform_d(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// One pass over the instance: S <- S - l u^T with row pi and column pj set
// to exactly 0 (unless INIT), and the row masses of the result into s_rm.
template <class T, int R, int V, bool INIT>
__device__ __forceinline__ void bt_sweep(T* __restrict__ S, int64_t lda, int n, int m, int pi, int pj,
                         const T* __restrict__ s_l, const T* __restrict__ Ut,
                         double* __restrict__ s_rm, BtShared& sh) {
    const int tid = threadIdx.x, lane = tid % RPLU_WAVE, wv = tid / RPLU_WAVE;
    const int aw = (m + RPLU_WAVE * V - 1) / (RPLU_WAVE * V);   // waves a row needs
    const int gw = aw > 4 ? 8 : (aw > 2 ? 4 : (aw > 1 ? 2 : 1));
    const int groups = BT_WAVES / gw;
    const int grp = wv / gw;
    const int gt = tid - grp * gw * RPLU_WAVE;                   // thread index in its group
    const int nblk = (n + R - 1) / R;
    int par = 0;
    for (int b0 = 0; b0 < nblk; b0 += groups, par ^= 1) {
        const int blk = b0 + grp;
        const int r0 = blk * R;
        const int nr = blk < nblk ? min(R, n - r0) : 0;
        double rp[R];
#pragma unroll
        for (int q = 0; q < R; ++q) rp[q] = 0.0;
        T lq[R];
#pragma unroll
        for (int q = 0; q < R; ++q) lq[q] = (!INIT && q < nr) ? s_l[r0 + q] : Sc<T>::zero();

        auto pack = [&](int64_t c, auto full_tag, auto allrows_tag) {
            constexpr bool FULL = decltype(full_tag)::value;
            constexpr bool ALLR = decltype(allrows_tag)::value;
            BPack<T, V> u;
            if constexpr (!INIT) {
                if constexpr (FULL) u = *reinterpret_cast<const BPack<T, V>*>(Ut + c);
                else {
#pragma unroll
                    for (int v = 0; v < V; ++v) u.v[v] = (c + v < m) ? Ut[c + v] : Sc<T>::zero();
                }
            }
            BPack<T, V> s[R];
#pragma unroll
            for (int q = 0; q < R; ++q) {
                if (ALLR || q < nr) {
                    const T* p = S + (int64_t)(r0 + q) * lda + c;
                    if constexpr (FULL) s[q] = *reinterpret_cast<const BPack<T, V>*>(p);
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
                    for (int v = 0; v < V; ++v) rp[q] += Sc<T>::mag2(s[q].v[v]);
                    if constexpr (!INIT) {
                        T* p = S + (int64_t)(r0 + q) * lda + c;
                        if constexpr (FULL) *reinterpret_cast<BPack<T, V>*>(p) = s[q];
                        else {
#pragma unroll
                            for (int v = 0; v < V; ++v) if (c + v < m) p[v] = s[q].v[v];
                        }
                    }
                }
            }
        };

        if (nr > 0) {
            // With gw < 8 the group covers the row in one pass (gw*64*V >= m).
            int64_t c = (int64_t)gt * V;
            // (not unrolled: the R rows already keep R loads in flight, and
            // registers decide how many workgroups share a CU)
            if (nr == R) {
#pragma unroll 1
                for (; c + V <= m; c += (int64_t)BT_THREADS * V) pack(c, std::true_type{}, std::true_type{});
                if (c < m) pack(c, std::false_type{}, std::true_type{});
            } else {
#pragma unroll 1
                for (; c + V <= m; c += (int64_t)BT_THREADS * V) pack(c, std::true_type{}, std::false_type{});
                if (c < m) pack(c, std::false_type{}, std::false_type{});
            }
        }

        if (gw == 1) {
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const double v = wave_sum(rp[q]);
                if (lane == 0 && q < nr) s_rm[r0 + q] = v;
            }
        } else {
            // gw is uniform over the workgroup, so is this barrier. The two
            // red buffers alternate: the reads of pass k and the writes of
            // pass k+2 are separated by the barrier of pass k+1.
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const double v = wave_sum(rp[q]);
                if (lane == 0) sh.red[par][wv][q] = v;
            }
            __syncthreads();
            if (gt < nr) {
                double v = sh.red[par][grp * gw][gt];
                for (int w = 1; w < gw; ++w) v += sh.red[par][grp * gw + w][gt];
                s_rm[r0 + gt] = v;
            }
        }
    }
}

// Chunk totals of `len` masses into ct (the waves take chunks in turn) and
// the total T = 0 + sum_k ct_k in order, as the one-group chain of cdf.hpp.
template <class MassFn>
__device__ __forceinline__ double bt_levels(int len, double* ct, MassFn& mass, BtShared& sh) {
    const int lane = threadIdx.x % RPLU_WAVE, wv = threadIdx.x / RPLU_WAVE;
    const int K = cdf_chunks(len);
    for (int k = wv; k < K; k += BT_WAVES) {
        CdfChunk c;
        cdf_chunk(c, k, len, lane, mass);
        if (lane == 0) ct[k] = c.ct;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int k = 0; k < K; ++k) s = s + ct[k];
        sh.bc[0] = 0.0 + s;
    }
    __syncthreads();
    return uniform_d(sh.bc[0]);
}

// The draw of cdf_draw for one group (goff = 0): wave 0 chains the chunk
// totals and re-walks the selected chunk.
template <class MassFn>
__device__ __forceinline__ CdfPick bt_draw(int len, const double* ct, MassFn& mass, double target,
                                  BtShared& sh) {
    const int lane = threadIdx.x % RPLU_WAVE, wv = threadIdx.x / RPLU_WAVE;
    // bi and bc[1..2] were last read before the barriers of bt_levels
    if (wv == 0) {
        const int K = cdf_chunks(len);
        const double goff = 0.0;
        double io = 0.0;
        int k = 0;
        for (; k < K - 1; ++k) {
            const double nio = io + ct[k];
            if (goff + nio > target) break;
            io = nio;
        }
        const double before = (k == 0) ? goff : goff + io;
        const CdfPick p = cdf_chunk_select(k, len, lane, mass, goff, io, before, target);
        if (lane == 0) { sh.bi[0] = p.idx; sh.bc[1] = p.lo; sh.bc[2] = p.hi; }
    }
    __syncthreads();
    const CdfPick r{uniform_i(sh.bi[0]), sh.bc[1], sh.bc[2]};
    return r;
}

template <class T, int R, int V>
__device__ __forceinline__ void bt_run(const BatchJob& jb, T* __restrict__ uscr, BatchInfo* __restrict__ info,
                       double* __restrict__ s_rm, T* __restrict__ s_l, BtShared& sh) {
    using W = typename Sc<T>::W;
    T* __restrict__ S = (T*)jb.A;
    T* __restrict__ L = (T*)jb.L;
    const int n = jb.n, m = jb.m;
    const int64_t lda = jb.lda;
    T* Ubase = jb.U ? (T*)jb.U : uscr;
    const int64_t ldu = jb.U ? jb.ldu : 0;
    bt_sweep<T, R, V, true>(S, lda, n, m, -1, -1, s_l, nullptr, s_rm, sh);
    __syncthreads();
    double T0 = 0.0, Tc = 0.0;
    int t = 0, stop = 0, err = 0;
    for (;; ++t) {
        auto rmass = [&](int e) { return s_rm[e]; };
        Tc = bt_levels(n, sh.ctr, rmass, sh);
        if (t == 0) T0 = Tc;
        if (!isfinite(Tc)) err = RPLU_E_NONFINITE;
        else if (Tc == 0.0) stop = RPLU_STOP_EXHAUSTED;
        else if (jb.tol2 > 0.0 && Tc <= jb.tol2 * T0) stop = RPLU_STOP_TOL;
        else if (t >= jb.kmax) stop = jb.tol2 > 0.0 ? RPLU_STOP_TOL_UNREACHED : RPLU_STOP_RANK;
        if (err || stop) break;
        const Philox4 rnd = philox4x64_10((uint64_t)t, jb.stream, 0, 0, jb.seed, 0);
        const CdfPick pr = bt_draw(n, sh.ctr, rmass, unit_from_word(rnd.w[0]) * Tc, sh);
        const int i = pr.idx;
        if (i < 0 || i >= n) { err = RPLU_E_ARG; break; }
        const T* Si = S + (int64_t)i * lda;
        T* Ut = Ubase + (int64_t)t * ldu;
        auto rcopy = [&](int e) { const T v = Si[e]; Ut[e] = v; return Sc<T>::mag2(v); };
        const double Ti = bt_levels(m, sh.ctc, rcopy, sh);
        auto smass = [&](int e) { return Sc<T>::mag2(Si[e]); };
        CdfPick pc{0, 0.0, 0.0};
        if (Ti > 0.0 && isfinite(Ti)) pc = bt_draw(m, sh.ctc, smass, unit_from_word(rnd.w[1]) * Ti, sh);
        const int j = pc.idx;
        if (j < 0 || j >= m) { err = RPLU_E_ARG; break; }
        const T a = Si[j];
        const double a2 = Sc<T>::mag2(a);
        if (!(a2 > 0.0)) { err = isfinite(a2) ? RPLU_E_ZERO_PIVOT : RPLU_E_NONFINITE; break; }
        const W inv = winv(Sc<T>::widen(a));
        if (threadIdx.x == 0 && jb.piv != nullptr) { jb.piv[2 * t] = i; jb.piv[2 * t + 1] = j; }
        // scaled pivot column: L(:,t) and the multipliers of the sweep
        for (int r = threadIdx.x; r < n; r += BT_THREADS) {
            const T l = (r == i) ? Sc<T>::one()
                                 : Sc<T>::narrow(wmul(Sc<T>::widen(S[(int64_t)r * lda + j]), inv));
            s_l[r] = l;
            if (L != nullptr) L[(int64_t)t * jb.ldl + r] = l;
        }
        __syncthreads();                  // column j read before any store to it
        bt_sweep<T, R, V, false>(S, lda, n, m, i, j, s_l, Ut, s_rm, sh);
        __syncthreads();                  // new masses and S visible to every wave
    }
    if (threadIdx.x == 0) {
        info->rank = t;
        info->stop = stop;
        info->error = err;
        info->a_fro2 = T0;
        info->res_fro2 = Tc;
    }
}

// Persistent kernel. Every workgroup leaves once the queue index passes
// `count`, so the grid drains after the last instance.
template <class T, int R>
__global__ __launch_bounds__(BT_THREADS) void k_batched(const BatchJob* __restrict__ jobs,
                                                         const int32_t* __restrict__ order,
                                                         int count, int* __restrict__ queue,
                                                         T* __restrict__ uscratch, int64_t uscr_ld,
                                                         int maxn, BatchInfo* __restrict__ infos) {
    extern __shared__ double bt_dyn[];
    __shared__ BtShared sh;
    double* s_rm = bt_dyn;
    T* s_l = reinterpret_cast<T*>(bt_dyn + maxn);
    T* myscr = uscratch + (int64_t)blockIdx.x * uscr_ld;
    constexpr int VV = 16 / (int)sizeof(T);
    for (;;) {
        if (threadIdx.x == 0) sh.job = atomicAdd(queue, 1);
        __syncthreads();
        const int q = uniform_i(sh.job);
        __syncthreads();
        if (q >= count) break;
        const int b = order[q];
        const BatchJob jb = jobs[b];
        if (jb.vec) bt_run<T, R, VV>(jb, myscr, &infos[b], s_rm, s_l, sh);
        else bt_run<T, R, 1>(jb, myscr, &infos[b], s_rm, s_l, sh);
        __syncthreads();
    }
}

__global__ void k_queue_reset(int* q) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *q = 0;
}

template <class T, int R>
static const void* batched_fn() { return reinterpret_cast<const void*>(&k_batched<T, R>); }

static const void* batched_kernel(int dtype, int rows) {
    const bool d = dtype == RPLU_R64;
    switch (rows) {
        case 1: return d ? batched_fn<double, 1>() : batched_fn<float, 1>();
        case 2: return d ? batched_fn<double, 2>() : batched_fn<float, 2>();
        case 4: return d ? batched_fn<double, 4>() : batched_fn<float, 4>();
        case 8: return d ? batched_fn<double, 8>() : batched_fn<float, 8>();
        default: return nullptr;
    }
}

size_t batched_lds_bytes(int dtype, int maxn) {
    return (size_t)maxn * (8 + (dtype == RPLU_R64 ? 8 : 4));
}

int batched_max_resident(int dtype, int rows, int maxn) {
    const void* fn = batched_kernel(dtype, rows);
    if (fn == nullptr) return 0;
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn, BT_THREADS,
                                                     batched_lds_bytes(dtype, maxn)) != hipSuccess)
        return 0;
    return blocks;
}

template <class T, int R>
static void launch_t(const BatchLaunch& a, hipStream_t s) {
    hipLaunchKernelGGL((k_batched<T, R>), dim3(a.grid), dim3(BT_THREADS),
                       batched_lds_bytes(a.dtype, a.maxn), s, a.jobs, a.order, a.count, a.queue,
                       (T*)a.uscratch, a.uscr_ld, a.maxn, a.infos);
}

template <class T>
static void launch_dt(const BatchLaunch& a, hipStream_t s) {
    switch (a.rows) {
        case 1: launch_t<T, 1>(a, s); break;
        case 2: launch_t<T, 2>(a, s); break;
        case 4: launch_t<T, 4>(a, s); break;
        case 8: launch_t<T, 8>(a, s); break;
    }
}

void launch_batched(const BatchLaunch& a, hipStream_t s) {
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, s, a.queue);
    if (a.dtype == RPLU_R64) launch_dt<double>(a, s);
    else launch_dt<float>(a, s);
}

}  // namespace rplu
