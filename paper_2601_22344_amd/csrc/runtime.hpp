// Host-side runtime state shared by the C-ABI translation units (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "rplu.h"

namespace rplu {
struct StepState;

// Workgroup slots of the all-pairs mass kernels (Cauchy-like form): the CUs
// and, per generator width p = 1..4, how many workgroups of the row pass and
// of the column pass one CU holds at once (the kernels' occupancy). They size
// the column splits so that the grid fills whole rounds of the chip.
struct MassSlots {
    int cu_count = 256;
    int row_wg[5] = {2, 2, 2, 2, 2};
    int col_wg[5] = {2, 2, 2, 2, 2};
};
// Queries the occupancy of the mass kernels on the current device (2 per CU
// for a kernel whose query fails).
MassSlots cauchy_mass_slots(int cu_count);
}

struct rplu_prof_rec {
    int cls;
    hipEvent_t a, b;
};

// An instantiated step-loop graph: a chunk of `ch` steps replayed `reps`
// times, then a tail graph of the remaining steps. `key` fingerprints every
// launch argument, so a call with the same buffers and sizes reuses it.
struct rplu_graph_entry {
    uint64_t key = 0;
    bool valid = false;
    uint64_t last_use = 0;
    int64_t ch = 0, reps = 0, tail = 0;
    hipGraphExec_t main = nullptr, rest = nullptr;
};

constexpr int RPLU_GRAPH_CACHE = 6;

// A tuned batched-launch configuration and the batch signature it was
// measured for.
struct rplu_tune_entry {
    uint64_t key;
    rplu_batch_cfg cfg;
    double ms;
};

struct rplu_ctx_s {
    int device = 0;
    int cu_count = 0;
    size_t hbm_budget = 0;          // cap on ws + batch_ws (0: none)
    size_t lds_per_block = 0;       // bytes of LDS one workgroup may use
    void* ws = nullptr;             // grow-only device workspace
    size_t ws_cap = 0;
    void* batch_ws = nullptr;       // batched-launch descriptors and queue
    size_t batch_ws_cap = 0;
    rplu::StepState* host_state = nullptr;   // pinned staging for state read-back
    hipStream_t cap_stream = nullptr;        // stream the step loop is captured on
    // profiling
    bool prof_on = false;                    // record events around launches
    std::vector<hipEvent_t> ev_pool;         // reusable events (plain launches)
    size_t ev_used = 0;
    std::vector<rplu_prof_rec> prof;         // pending event records
    rplu_graph_entry graphs[RPLU_GRAPH_CACHE];
    uint64_t use_clock = 0;
    std::vector<rplu_tune_entry> tune;       // batched-launch tuning table
    rplu::MassSlots mass_slots;              // occupancy of the Cauchy mass kernels
};

namespace rplu {
rplu_status fail(rplu_status code, const char* fmt, ...);
rplu_status hip_fail(hipError_t e, const char* what);
size_t dtype_size(int dt);
rplu_status ws_reserve(rplu_ctx_s* ctx, size_t bytes, hipStream_t s);
void graph_cache_clear(rplu_ctx_s* ctx);

// Enqueues `launch` on stream s; while profiling is on (which also selects
// plain launches over graph replay), brackets it with two events and
// remembers them under class `cls`.
template <class F>
inline void timed(rplu_ctx_s* ctx, int cls, hipStream_t s, F&& launch) {
    if (ctx == nullptr || !ctx->prof_on) { launch(); return; }
    while (ctx->ev_pool.size() < ctx->ev_used + 2) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) { launch(); return; }
        ctx->ev_pool.push_back(e);
    }
    hipEvent_t a = ctx->ev_pool[ctx->ev_used++], b = ctx->ev_pool[ctx->ev_used++];
    (void)hipEventRecord(a, s);
    launch();
    (void)hipEventRecord(b, s);
    ctx->prof.push_back({cls, a, b});
}

// Dense-run workspace layout and the shared dense step loop (api.hip); the
// context-free caller (rplu_dense_noalloc) passes ctx == nullptr.
struct DenseWs {
    size_t o_st, o_rm, o_rx, o_ctr, o_ctc, o_cp, o_u, total;
    // the one-launch step (k_dense_step): per-workgroup states, the
    // workgroups' pivot-row copies, the dead-row flags
    bool step = false;
    int groups = 0;
    int64_t ldur = 0;
    size_t o_sts = 0, o_ur = 0, o_dead = 0;   // (o_rm then holds two buffers)
};
// Whether a dense run may take the one-launch step (small, and no option
// that needs the separate kernels).
bool dense_step_eligible(int64_t n, int64_t m, uint32_t flags);
// allow_step = false: the layout of the separate kernels only (the
// context-free entry point).
DenseWs dense_ws_layout(int dtype, int64_t n, int64_t m, uint32_t flags, bool need_u,
                        bool allow_step = true);
rplu_status dense_check(const char* who, int dtype, int64_t n, int64_t m, const void* A,
                        int64_t lda, const rplu_opts* opts, const int32_t* piv, const void* L,
                        int64_t ldl, const void* U, int64_t ldu, const rplu_info* info);
rplu_status dense_run(rplu_ctx_s* ctx, char* ws, int dtype, int64_t n, int64_t m, void* A,
                      int64_t lda, const rplu_opts* opts, int32_t* piv, void* L, int64_t ldl,
                      void* U, int64_t ldu, rplu_info* info, hipStream_t s);

struct CauchyWs {
    int64_t splits = 0, cps = 0, splits_c = 0, cps_c = 0;
    size_t o_st, o_rm, o_pa, o_ctr, o_ctc, o_u, o_mc, o_mf, o_pc, o_gt, o_bt, total;
};
rplu_status cauchy_check(const char* who, int dtype, int64_t n, int64_t m, int p, const void* x,
                         const void* y, const void* G, const void* B, const rplu_opts* opts,
                         const int32_t* piv, const void* L, int64_t ldl, const void* U,
                         int64_t ldu, const rplu_info* info);
CauchyWs cauchy_ws_layout(const MassSlots& slots, int64_t n, int64_t m, int p, uint32_t flags,
                          bool colmass, bool need_u);
struct BoundsPlan;
// bp: the device plan of RPLU_FLAG_BOUNDS, or null (exact masses).
rplu_status cauchy_run(rplu_ctx_s* ctx, char* ws, int64_t n, int64_t m, int p, const void* x,
                       const void* y, void* G, void* B, const rplu_opts* opts, int32_t* piv,
                       void* L, int64_t ldl, void* U, int64_t ldu, rplu_info* info,
                       hipStream_t s, const BoundsPlan* bp = nullptr);

struct BatchJob;
struct BatchInfo;
rplu_status batch_job_of(const rplu_job& j, BatchJob* out);
rplu_status batch_launch_jobs(rplu_ctx_s* ctx, int dtype, const std::vector<BatchJob>& jobs,
                              const rplu_batch_cfg& c, hipStream_t s, std::vector<BatchInfo>* out);

// FNV-1a over raw bytes, for graph cache keys.
inline uint64_t fnv1a(const void* p, size_t n, uint64_t h = 1469598103934665603ull) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) { h ^= c[i]; h *= 1099511628211ull; }
    return h;
}
}  // namespace rplu
