// Batched dense RPLU: many independent instances in one persistent launch.
//
// Each workgroup (1024 threads) takes instances from a device work queue (an
// atomic counter over a host-ordered table, largest estimated cost first)
// and runs an instance's whole step loop (Alg. 1 with two-stage sampling,
// Sec. 4.1) with workgroup barriers only. Row masses, the scaled pivot
// column and the list of rows not yet pivoted live in LDS; the pivot row goes
// to U(t,:) (or a per-workgroup row) and, for rows of up to four virtual
// waves, to LDS as well.
//
// Every reduction uses the thread-to-element mapping and order of the
// single-instance path (the sweep's 512-thread x 16-byte-pack layout, its wave
// sums and fixed-order sum over the 8 waves; the chunk totals, the chain and
// the in-chunk select of cdf.hpp), so an instance's pivots and factors are
// bitwise those of rplu_dense on the same buffer. Two schedule knobs leave
// the arithmetic unchanged and are left to the autotuner:
//   * R: the rows a wave sweeps at once in the general pass (each row keeps
//     its own partial sums, so R changes only how many rows are in flight)
//     and the packs a wave loads at once in the block pass (bt_packs);
//   * the number of resident workgroups per CU.
#include <type_traits>

#include "common.hpp"
#include "cdf.hpp"
#include "launch.hpp"

namespace rplu {

constexpr int BT_THREADS = 1024;                   // physical workgroup
constexpr int BT_WAVES = BT_THREADS / RPLU_WAVE;
constexpr int VT_THREADS = DENSE_THREADS;          // the single-instance sweep's mapping
constexpr int VT_WAVES = VT_THREADS / RPLU_WAVE;
constexpr int BT_MAXK = RPLU_BATCH_MAX_DIM / CDF_CHUNK;   // chunks of a mass vector

static_assert(BT_MAXK <= CDF_GROUP, "one CDF group: the chain is a single sequential sum");

template <class T, int V>
struct alignas(V == 1 ? alignof(T) : 16) BPack { T v[V]; };

// Instance buffers come from the job table, so the compiler cannot tell that
// they are global memory: through plain pointers it emits flat accesses,
// which also count against the LDS counter, and every LDS wait of the sweep
// then waits for the row loads and stores in flight as well. Pointers into
// instance memory carry the global address space instead.
template <class T> using gmem = __attribute__((address_space(1))) T;

// A whole pack from / to instance memory as one 16-byte access: a native
// vector value (the pack's own copy operations take generic references, and
// element-wise copies let the compiler split the store).
template <class T, int V> struct PackVec { typedef T type __attribute__((ext_vector_type(V))); };
template <class T> struct PackVec<T, 1> { typedef T type; };

template <class T, int V>
__device__ __forceinline__ BPack<T, V> ld_pack(const gmem<T>* p) {
    using VT = typename PackVec<T, V>::type;
    const VT w = *reinterpret_cast<const gmem<VT>*>(p);
    BPack<T, V> x;
    if constexpr (V == 1) x.v[0] = w;
    else {
#pragma unroll
        for (int v = 0; v < V; ++v) x.v[v] = w[v];
    }
    return x;
}

template <class T, int V>
__device__ __forceinline__ void st_pack(gmem<T>* p, const BPack<T, V>& x) {
    using VT = typename PackVec<T, V>::type;
    VT w;
    if constexpr (V == 1) w = x.v[0];
    else {
#pragma unroll
        for (int v = 0; v < V; ++v) w[v] = x.v[v];
    }
    *reinterpret_cast<gmem<VT>*>(p) = w;
}

static_assert(sizeof(BPack<float, 1>) == 4 && sizeof(BPack<double, 2>) == 16, "pack size");

struct BtShared {
    double ctr[BT_MAXK];                  // chunk totals: row masses
    double ctc[BT_MAXK];                  // chunk totals: pivot row
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

// One pass over the live rows of the instance: S <- S - l u^T with row pi
// and column pj set to exactly 0 (unless INIT), and the row masses of the
// result into s_rm. rows[0..nalive) lists the rows not yet pivoted; a
// pivoted row is exactly +0 and would stay +0 under every later update (its
// multiplier is +-0 and its entries +0), so leaving it out changes no bit.
//
// Blocks of R live rows go to the waves in turn, and a wave sweeps its block
// on its own, with no barrier. The single-instance kernel reduces a row with
// 8 waves: wave w holds columns (64 w + lane) V + 512 V k, each lane sums its
// packs in order, each wave sums its lanes (wave_sum), and the 8 wave sums
// are added in wave order. Here one wave walks those 8 virtual waves in turn
// with the same lane mapping, so it forms the same per-lane sums, the same
// wave sums and the same ordered total; a virtual wave that holds no column
// would add an exact 0 and is skipped.
template <class T, int R, int V, bool INIT>
__device__ __forceinline__ void bt_sweep(gmem<T>* __restrict__ S, int64_t lda, int m, int pi, int pj,
                                         const T* __restrict__ s_l, const gmem<T>* __restrict__ Ut,
                                         double* __restrict__ s_rm,
                                         const uint16_t* __restrict__ rows, int nalive) {
    const int lane = threadIdx.x % RPLU_WAVE, wv = threadIdx.x / RPLU_WAVE;
    const int vws = min(VT_WAVES, (m + RPLU_WAVE * V - 1) / (RPLU_WAVE * V));
    const int nblk = (nalive + R - 1) / R;
#pragma unroll 1
    for (int blk = wv; blk < nblk; blk += BT_WAVES) {
        const int b0 = blk * R;
        const int nr = min(R, nalive - b0);
        int ri[R];
#pragma unroll
        for (int q = 0; q < R; ++q) ri[q] = rows[b0 + min(q, nr - 1)];
        T lq[R];
#pragma unroll
        for (int q = 0; q < R; ++q) lq[q] = (!INIT && q < nr) ? s_l[ri[q]] : Sc<T>::zero();
        double tot[R];
#pragma unroll
        for (int q = 0; q < R; ++q) tot[q] = 0.0;
        double rp[R];

        gmem<T>* rowp[R];
#pragma unroll
        for (int q = 0; q < R; ++q) rowp[q] = S + (int64_t)ri[q] * lda;

        // Pivot row and column become exact zeros by a select (pv = offset
        // of column pj inside the pack), so every load is unconditional.
        auto pack = [&](int c, auto full_tag, auto allrows_tag) {
            constexpr bool FULL = decltype(full_tag)::value;
            constexpr bool ALLR = decltype(allrows_tag)::value;
            BPack<T, V> u;
            if constexpr (!INIT) {
                if constexpr (FULL) u = ld_pack<T, V>(Ut + c);
                else {
#pragma unroll
                    for (int v = 0; v < V; ++v) u.v[v] = (c + v < m) ? Ut[c + v] : Sc<T>::zero();
                }
            }
            BPack<T, V> s[R];
#pragma unroll
            for (int q = 0; q < R; ++q) {
                if (ALLR || q < nr) {
                    const gmem<T>* p = rowp[q] + c;
                    if constexpr (FULL) s[q] = ld_pack<T, V>(p);
                    else {
#pragma unroll
                        for (int v = 0; v < V; ++v) s[q].v[v] = (c + v < m) ? p[v] : Sc<T>::zero();
                    }
                }
            }
            const int pv = pj - c;
#pragma unroll
            for (int q = 0; q < R; ++q) {
                if (ALLR || q < nr) {
                    if constexpr (!INIT) {
                        const bool zr = ri[q] == pi;
#pragma unroll
                        for (int v = 0; v < V; ++v) {
                            const T x = Sc<T>::fms(s[q].v[v], lq[q], u.v[v]);
                            s[q].v[v] = ((v == pv) | zr) ? Sc<T>::zero() : x;
                        }
                    }
#pragma unroll
                    for (int v = 0; v < V; ++v) rp[q] = Sc<T>::mag2_add(rp[q], s[q].v[v]);
                    if constexpr (!INIT) {
                        gmem<T>* p = rowp[q] + c;
                        if constexpr (FULL) st_pack<T, V>(p, s[q]);
                        else {
#pragma unroll
                            for (int v = 0; v < V; ++v) if (c + v < m) p[v] = s[q].v[v];
                        }
                    }
                }
            }
        };

#pragma unroll 1
        for (int vw = 0; vw < vws; ++vw) {
#pragma unroll
            for (int q = 0; q < R; ++q) rp[q] = 0.0;
            int c = (vw * RPLU_WAVE + lane) * V;      // virtual thread vw*64 + lane
            // (not unrolled: the R rows already keep R loads in flight)
            if (nr == R) {
#pragma unroll 1
                for (; c + V <= m; c += VT_THREADS * V) pack(c, std::true_type{}, std::true_type{});
                if (c < m) pack(c, std::false_type{}, std::true_type{});
            } else {
#pragma unroll 1
                for (; c + V <= m; c += VT_THREADS * V) pack(c, std::true_type{}, std::false_type{});
                if (c < m) pack(c, std::false_type{}, std::false_type{});
            }
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const double w = wave_sum(rp[q]);
                tot[q] = (vw == 0) ? w : tot[q] + w;
            }
        }
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < R; ++q)
                if (q < nr) s_rm[ri[q]] = tot[q];
        }
    }
}

// The pack of V elements at p when `rem` = m - c elements remain in the row:
// a 16-byte store when the pack is whole, element stores up to m at the row's
// end, nothing past it.
template <class T, int V>
__device__ __forceinline__ void bt_store(gmem<T>* p, int rem, const BPack<T, V>& x) {
    if (rem >= V) st_pack<T, V>(p, x);
    else {
#pragma unroll
        for (int v = 0; v < V; ++v) if (v < rem) p[v] = x.v[v];
    }
}

// Branch-free pieces of the block pass. A branch between loads into the same
// registers (a whole-pack load on one side, element loads or zeros on the
// other) makes the compiler wait for every load in flight before it, which
// serialises a block's loads. So every lane loads a whole pack inside the row
// (its own when its pack is whole, else the row's first: rows of at least V
// columns), the one partial pack of a row (m mod V columns from cp = m - m mod
// V on) comes from V element loads at clamped addresses into registers of its
// own, and bt_pick selects what the lane's pack holds: the whole pack, the
// partial pack's first rem columns then zeros, or zeros.
template <class T, int V>
__device__ __forceinline__ BPack<T, V> bt_tail(const gmem<T>* row, int cp, int mt) {
    BPack<T, V> x;
#pragma unroll
    for (int v = 0; v < V; ++v) x.v[v] = row[cp + min(v, mt - 1)];
    return x;
}

template <class T, int V>
__device__ __forceinline__ BPack<T, V> bt_pick(const BPack<T, V>& whole, const BPack<T, V>& tail,
                                               int rem) {
    BPack<T, V> x;
#pragma unroll
    for (int v = 0; v < V; ++v)
        x.v[v] = rem >= V ? whole.v[v] : (v < rem ? tail.v[v] : Sc<T>::zero());
    return x;
}

constexpr int BT_NV = 4;   // virtual waves of 16-byte packs a row may span in the block pass

// Elements of the pivot row's LDS copy s_u: a row of BT_NV x 64 16-byte
// packs (1024 FP32, 512 FP64 columns).
template <class T> constexpr int bt_su() { return BT_NV * RPLU_WAVE * (16 / (int)sizeof(T)); }

// The value of lane 0 (every lane holds the same), in scalar registers.
__device__ __forceinline__ float uniform_v(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double uniform_v(double v) { return uniform_d(v); }

// Four wave sums at once, each with wave_sum's butterfly (v + v(lane ^ 32),
// then ^ 16, then the rotations inside rows of 16 lanes), so each sum has
// wave_sum's bits. The first step pairs a with b and c with d through the
// half-wave swap (its first result holds the two operands' lower halves,
// the second their upper halves: lanes 0-31 then hold a(l) + a(l + 32),
// lanes 32-63 b's pair sums); the second step pairs the two results through
// the row swap (even rows of both operands, then odd rows). The sums end up
// in rows of 16 lanes: a in lanes 0-15, c in 16-31, b in 32-47, d in 48-63.
__device__ __forceinline__ double pair_swap32(double a, double b) {
    const uint64_t x = __builtin_bit_cast(uint64_t, a), y = __builtin_bit_cast(uint64_t, b);
    const auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)x, (uint32_t)y, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(x >> 32), (uint32_t)(y >> 32), false, false);
    return __builtin_bit_cast(double, ((uint64_t)hi[0] << 32) | lo[0]) +
           __builtin_bit_cast(double, ((uint64_t)hi[1] << 32) | lo[1]);
}
__device__ __forceinline__ double pair_swap16(double a, double b) {
    const uint64_t x = __builtin_bit_cast(uint64_t, a), y = __builtin_bit_cast(uint64_t, b);
    const auto lo = __builtin_amdgcn_permlane16_swap((uint32_t)x, (uint32_t)y, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((uint32_t)(x >> 32), (uint32_t)(y >> 32), false, false);
    return __builtin_bit_cast(double, ((uint64_t)hi[0] << 32) | lo[0]) +
           __builtin_bit_cast(double, ((uint64_t)hi[1] << 32) | lo[1]);
}
__device__ __forceinline__ double wave_sum4(double a, double b, double c, double d) {
    double v = pair_swap16(pair_swap32(a, b), pair_swap32(c, d));
    v = v + dpp_d<0x128>(v);     // row_ror:8
    v = v + dpp_d<0x124>(v);     // row_ror:4
    v = v + dpp_d<0x122>(v);     // row_ror:2
    v = v + dpp_d<0x121>(v);     // row_ror:1
    return v;
}
// lanes of the four sums of wave_sum4, in argument order
constexpr int BT_SUM4_LANE[4] = {0, 32, 16, 48};

// The pass of bt_sweep for rows the pivot row's LDS copy s_u holds (V <= m
// <= bt_su elements), whose lanes hold at most KP packs per virtual wave: NVW
// virtual waves of KP = 1 pack (m <= NVW x 64 V), or for single-element
// packs (V = 1, rows not 16-byte aligned) all 8 virtual waves of KP = 1 or
// 2 packs (m <= 512 KP). A wave takes blocks of RB rows and loads a whole
// block (RB rows by NVW x KP packs) before any arithmetic, so one memory
// round trip serves the block instead of one per virtual wave; the pivot
// row's packs come from s_u. Each row keeps the per-lane sums (0 + |x_0|^2
// + ... in pack order, exactly 0 for a lane with no column), the wave sums
// and their sum in virtual-wave order of bt_sweep (a virtual wave past the
// row's last adds an exact 0 to a total >= +0), so S and the masses are the
// same bits; lane q holds the running total of row q (the wave sums are the
// same in every lane).
template <class T, int RB, int NVW, int KP, int V, bool INIT>
__device__ __forceinline__ void bt_sweep_block(gmem<T>* __restrict__ S, int64_t lda, int m, int pi, int pj,
                                               const T* __restrict__ s_l, const T* __restrict__ s_u,
                                               double* __restrict__ s_rm,
                                               const uint16_t* __restrict__ rows, int nalive) {
    static_assert(KP == 1 || V == 1, "several packs per virtual wave: single-element packs");
    const int lane = threadIdx.x % RPLU_WAVE, wv = threadIdx.x / RPLU_WAVE;
    const int nblk = (nalive + RB - 1) / RB;
    // columns of the row from this lane's pack (k, kp) on, and a whole pack
    // inside the row to load for it (formed where used: as arrays they took
    // a register each)
    const int m0 = m - lane * V;
    auto rem = [&](int k, int kp) { return m0 - (k * RPLU_WAVE + kp * VT_THREADS) * V; };
    auto cl = [&](int k, int kp) { const int r = rem(k, kp); return r >= V ? m - r : 0; };
    const int mt = m % V, cp = m - mt;
#pragma unroll 1
    for (int blk = wv; blk < nblk; blk += BT_WAVES) {
        const int b0 = blk * RB;
        const int nr = min(RB, nalive - b0);
        int ri[RB];
        T lq[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            ri[q] = uniform_i(rows[b0 + min(q, nr - 1)]);
            lq[q] = INIT ? Sc<T>::zero() : uniform_v(s_l[ri[q]]);
        }
        BPack<T, V> x[RB][NVW][KP], xt[RB];
#pragma unroll
        for (int v = 0; v < V; ++v) {
#pragma unroll
            for (int q = 0; q < RB; ++q) xt[q].v[v] = Sc<T>::zero();
        }
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const gmem<T>* rp = S + (int64_t)ri[q] * lda;
#pragma unroll
            for (int k = 0; k < NVW; ++k)
#pragma unroll
                for (int kp = 0; kp < KP; ++kp) x[q][k][kp] = ld_pack<T, V>(rp + cl(k, kp));
        }
        if (mt != 0) {
#pragma unroll
            for (int q = 0; q < RB; ++q) xt[q] = bt_tail<T, V>(S + (int64_t)ri[q] * lda, cp, mt);
        }
        // the block's wave sums, virtual wave k of row q as sum k RB + q,
        // are formed four at a time (wave_sum4); each row's total adds its
        // virtual waves' sums in order, as bt_sweep does
        constexpr int NS = NVW * RB;
        double tot[RB];
        double pend[4];
        auto flush = [&](int i_last, int cnt) {
            const double v = wave_sum4(pend[0], cnt > 1 ? pend[1] : 0.0, cnt > 2 ? pend[2] : 0.0,
                                       cnt > 3 ? pend[3] : 0.0);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (u < cnt) {
                    const int i = i_last - (cnt - 1) + u;
                    const int kk = i / RB, qq = i % RB;
                    const double w = uniform_lane(v, BT_SUM4_LANE[u]);
                    tot[qq] = (kk == 0) ? w : tot[qq] + w;
                }
            }
        };
#pragma unroll
        for (int k = 0; k < NVW; ++k) {
            int c[KP], pv[KP];
            BPack<T, V> uk[KP];
#pragma unroll
            for (int kp = 0; kp < KP; ++kp) {
                c[kp] = m - rem(k, kp);
                pv[kp] = pj - c[kp];
                // (c < bt_su for every lane: s_u is read in bounds, and past m
                // the value goes unused)
                if constexpr (!INIT) uk[kp] = *reinterpret_cast<const BPack<T, V>*>(s_u + c[kp]);
            }
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                double part = 0.0;
                if (q < nr) {
                    double acc = 0.0;
#pragma unroll
                    for (int kp = 0; kp < KP; ++kp) {
                        const int rk = m - c[kp];
                        BPack<T, V> xk = bt_pick<T, V>(x[q][k][kp], xt[q], rk);
                        if constexpr (!INIT) {
                            const bool zr = ri[q] == pi;
#pragma unroll
                            for (int v = 0; v < V; ++v) {
                                const T y = Sc<T>::fms(xk.v[v], lq[q], uk[kp].v[v]);
                                xk.v[v] = ((v == pv[kp]) | zr) ? Sc<T>::zero() : y;
                            }
                        }
                        // a lane past the row's end holds exact zeros here
                        // (its pack picked as 0, s_u zero past m, so the
                        // update leaves +0), and adding 0 to a sum >= +0
                        // changes no bit: no select needed
#pragma unroll
                        for (int v = 0; v < V; ++v) acc = Sc<T>::mag2_add(acc, xk.v[v]);
                        if constexpr (!INIT) {
                            if (rk > 0) bt_store<T, V>(S + (int64_t)ri[q] * lda + c[kp], rk, xk);
                        }
                    }
                    part = acc;
                }
                const int i = k * RB + q;
                pend[i % 4] = part;
                if (i % 4 == 3 || i == NS - 1) flush(i, i % 4 + 1);
            }
        }
        double mine = tot[0];
#pragma unroll
        for (int q = 1; q < RB; ++q) mine = (lane == q) ? tot[q] : mine;
        if (lane < nr) s_rm[rows[b0 + lane]] = mine;
    }
}

// Packs a wave holds at once in the block pass for the row knob R (more than
// 8 spill registers at 1024 threads).
template <int R> constexpr int bt_packs() { return R == 1 ? 4 : 8; }

// One pass of the sweep: the block pass when the row fits s_u (m <= bt_su),
// with RB = packs / (virtual waves) rows per block for rows of up to four
// virtual waves, one row per block for single-element packs over all eight
// (8 or 16 loads in flight per lane: two or four rows per block spilled
// registers and ran slower); else bt_sweep with R rows in flight.
template <class T, int R, int V, bool INIT>
__device__ __forceinline__ void bt_pass(gmem<T>* __restrict__ S, int64_t lda, int m, int pi, int pj,
                                        const T* __restrict__ s_l, const gmem<T>* __restrict__ Ut,
                                        const T* __restrict__ s_u,
                                        double* __restrict__ s_rm, const uint16_t* __restrict__ rows,
                                        int nalive) {
    constexpr int P = bt_packs<R>();
    constexpr int SUC = bt_su<T>();
    static_assert(BT_NV == 4, "one case per virtual-wave count");
    const int g = m < V ? 0 : (m + RPLU_WAVE * V - 1) / (RPLU_WAVE * V);   // 64-lane groups
    if (g >= 1 && g <= BT_NV) {
        switch (g) {
            case 1: bt_sweep_block<T, P, 1, 1, V, INIT>(S, lda, m, pi, pj, s_l, s_u, s_rm, rows, nalive); break;
            case 2: bt_sweep_block<T, P / 2, 2, 1, V, INIT>(S, lda, m, pi, pj, s_l, s_u, s_rm, rows, nalive); break;
            case 3: bt_sweep_block<T, P / 3, 3, 1, V, INIT>(S, lda, m, pi, pj, s_l, s_u, s_rm, rows, nalive); break;
            default: bt_sweep_block<T, P / 4, 4, 1, V, INIT>(S, lda, m, pi, pj, s_l, s_u, s_rm, rows, nalive); break;
        }
        return;
    }
    if constexpr (V == 1) {
        // all 8 virtual waves, one or two columns each per lane
        if (m <= VT_THREADS && m <= SUC) {
            bt_sweep_block<T, 1, VT_WAVES, 1, 1, INIT>(S, lda, m, pi, pj, s_l, s_u, s_rm, rows, nalive);
            return;
        }
        if constexpr (2 * VT_THREADS <= SUC) {
            if (m <= 2 * VT_THREADS) {
                bt_sweep_block<T, 1, VT_WAVES, 2, 1, INIT>(S, lda, m, pi, pj, s_l, s_u, s_rm, rows, nalive);
                return;
            }
        }
    }
    bt_sweep<T, R, V, INIT>(S, lda, m, pi, pj, s_l, Ut, s_rm, rows, nalive);
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

// s_u: the pivot row in LDS for rows that take the block pass (V <= m <=
// bt_su), zero past m, so the column draw, the pivot entry and the sweep's
// multiplier packs read LDS instead of the row in memory.
template <class T, int R, int V>
__device__ __forceinline__ void bt_run(const BatchJob& jb, T* __restrict__ uscr, BatchInfo* __restrict__ info,
                       double* __restrict__ s_rm, T* __restrict__ s_l, uint16_t* __restrict__ s_alive,
                       uint16_t* __restrict__ s_pos, T* __restrict__ s_u, BtShared& sh) {
    using W = typename Sc<T>::W;
    gmem<T>* __restrict__ S = (gmem<T>*)jb.A;
    gmem<T>* __restrict__ L = (gmem<T>*)jb.L;
    const int n = jb.n, m = jb.m;
    const int64_t lda = jb.lda;
    gmem<T>* Ubase = (gmem<T>*)(jb.U ? (T*)jb.U : uscr);
    const int64_t ldu = jb.U ? jb.ldu : 0;
    constexpr int SU = bt_su<T>();
    const bool lds_row = m >= V && m <= SU;
    for (int r = threadIdx.x; r < n; r += BT_THREADS) {
        s_alive[r] = (uint16_t)r;
        s_pos[r] = (uint16_t)r;
    }
    for (int e = m + threadIdx.x; e < SU; e += BT_THREADS) s_u[e] = Sc<T>::zero();
    __syncthreads();
    int nalive = n;
    const int t0 = jb.t0;
    // A resumed run (t0 > 0) starts with every row live: rows pivoted since
    // the last residual replacement are exactly +0, get mass 0 from this
    // pass and stay +0 under later updates (multiplier +-0, entries +0), so
    // sweeping them changes no bit, while rows pivoted before a replacement
    // hold the residual of the stored factors and must be swept.
    bt_pass<T, R, V, true>(S, lda, m, -1, -1, s_l, nullptr, s_u, s_rm, s_alive, nalive);
    __syncthreads();
    double T0 = 0.0, Tc = 0.0, Tbest = 0.0, Tref = 0.0;
    int t = t0, stop = 0, err = 0, prev_i = -1, tbest = 0;
    for (;; ++t) {
        if (prev_i >= 0) {
            // the previous pivot row leaves the live list (the barriers of
            // the sampling below order this before the next sweep)
            if (threadIdx.x == 0) {
                const int p = s_pos[prev_i];
                const int last = s_alive[nalive - 1];
                s_alive[p] = (uint16_t)last;
                s_pos[last] = (uint16_t)p;
            }
            nalive -= 1;
        }
        auto rmass = [&](int e) { return s_rm[e]; };
        Tc = bt_levels(n, sh.ctr, rmass, sh);
        if (t == 0) { T0 = Tc; Tbest = Tc; tbest = 0; Tref = Tc; }
        else if (t == t0) {
            T0 = jb.T0_in;
            Tref = jb.Tref_in < 0.0 ? Tc : jb.Tref_in;
            if (jb.Tbest_in < 0.0) { Tbest = Tc; tbest = t; }
            else {
                Tbest = jb.Tbest_in;
                tbest = jb.tbest_in;
                if (Tc < RPLU_STALL_RATIO * Tbest) { Tbest = Tc; tbest = t; }
            }
        }
        else if (Tc < RPLU_STALL_RATIO * Tbest) { Tbest = Tc; tbest = t; }
        if (!isfinite(Tc)) err = RPLU_E_NONFINITE;
        else if (Tc == 0.0) stop = RPLU_STOP_EXHAUSTED;
        else if (jb.tol2 > 0.0 && Tc <= jb.tol2 * T0) stop = RPLU_STOP_TOL;
        else if (jb.refresh_on && t < jb.kmax && Tc <= RPLU_REFRESH_DROP2 * Tref)
            stop = RPLU_STOP_REFRESH;
        else if (jb.stall && t - tbest >= RPLU_STALL_WINDOW) stop = RPLU_STOP_STALL;
        else if (t >= jb.kmax) stop = jb.tol2 > 0.0 ? RPLU_STOP_TOL_UNREACHED : RPLU_STOP_RANK;
        if (err || stop) break;
        if (jb.t_end > t0 && t >= jb.t_end) break;      // paused: resumed by a later launch
        const Philox4 rnd = philox4x64_10((uint64_t)t, jb.stream, 0, 0, jb.seed, 0);
        const CdfPick pr = bt_draw(n, sh.ctr, rmass, unit_from_word(rnd.w[0]) * Tc, sh);
        const int i = pr.idx;
        if (i < 0 || i >= n) { err = RPLU_E_ARG; break; }
        const gmem<T>* Si = S + (int64_t)i * lda;
        gmem<T>* Ut = Ubase + (int64_t)t * ldu;
        auto rcopy = [&](int e) {
            const T v = Si[e];
            Ut[e] = v;
            if (lds_row) s_u[e] = v;
            return Sc<T>::mag2(v);
        };
        const double Ti = bt_levels(m, sh.ctc, rcopy, sh);
        auto smass = [&](int e) { return Sc<T>::mag2(lds_row ? s_u[e] : Si[e]); };
        CdfPick pc{0, 0.0, 0.0};
        if (Ti > 0.0 && isfinite(Ti)) pc = bt_draw(m, sh.ctc, smass, unit_from_word(rnd.w[1]) * Ti, sh);
        const int j = pc.idx;
        if (j < 0 || j >= m) { err = RPLU_E_ARG; break; }
        const T a = lds_row ? s_u[j] : Si[j];
        const double a2 = Sc<T>::mag2(a);
        if (!(a2 > 0.0)) { err = isfinite(a2) ? RPLU_E_ZERO_PIVOT : RPLU_E_NONFINITE; break; }
        const W inv = winv(Sc<T>::widen(a));
        if (threadIdx.x == 0 && jb.piv != nullptr) {
            gmem<int32_t>* piv = (gmem<int32_t>*)jb.piv;
            piv[2 * t] = i;
            piv[2 * t + 1] = j;
        }
        // scaled pivot column: L(:,t) and the multipliers of the sweep
        for (int r = threadIdx.x; r < n; r += BT_THREADS) {
            const T l = (r == i) ? Sc<T>::one()
                                 : Sc<T>::narrow(wmul(Sc<T>::widen(S[(int64_t)r * lda + j]), inv));
            s_l[r] = l;
            if (L != nullptr) L[(int64_t)t * jb.ldl + r] = l;
        }
        __syncthreads();                  // column j read before any store to it
        bt_pass<T, R, V, false>(S, lda, m, i, j, s_l, Ut, s_u, s_rm, s_alive, nalive);
        __syncthreads();                  // new masses and S visible to every wave
        prev_i = i;
    }
    if (threadIdx.x == 0) {
        info->rank = t;
        info->stop = stop;
        info->error = err;
        info->a_fro2 = T0;
        info->res_fro2 = Tc;
        info->T_best = Tbest;
        info->T_ref = Tref;
        info->t_best = tbest;
    }
}

// Persistent kernel. Every workgroup leaves once the queue index passes
// `count` (or after `count` iterations), so the grid drains after the last
// instance. Keep a barrier between
// any thread-0-only work at the end of an iteration and the thread-0 queue
// fetch at the top: with the two adjacent, the compiler can give the loop a
// second back edge that bypasses the fetch for the other lanes, and since a
// barrier counts whole waves those lanes then re-run a stale job index.
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
    uint16_t* s_alive = reinterpret_cast<uint16_t*>(s_l + maxn);
    uint16_t* s_pos = s_alive + maxn;
    T* myscr = uscratch + (int64_t)blockIdx.x * uscr_ld;
    constexpr int VV = 16 / (int)sizeof(T);
    __shared__ __align__(16) T s_u[bt_su<T>()];
    static_assert(sizeof(BtShared) + sizeof(s_u) <= BT_STATIC_LDS, "static LDS bound of the host check");
    // At most `count` iterations per workgroup (the queue holds count jobs),
    // so the loop ends even if a fetch were ever skipped.
    for (int iter = 0; iter < count; ++iter) {
        if (threadIdx.x == 0) sh.job = atomicAdd(queue, 1);
        __syncthreads();
        const int q = uniform_i(sh.job);
        __syncthreads();
        if (q >= count) break;
        const int b = order[q];
        const BatchJob jb = jobs[b];
        if (jb.vec) bt_run<T, R, VV>(jb, myscr, &infos[b], s_rm, s_l, s_alive, s_pos, s_u, sh);
        else bt_run<T, R, 1>(jb, myscr, &infos[b], s_rm, s_l, s_alive, s_pos, s_u, sh);
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
    // row masses, multipliers, live-row list and positions
    return (size_t)maxn * (8 + (dtype == RPLU_R64 ? 8 : 4) + 2 * sizeof(uint16_t));
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
