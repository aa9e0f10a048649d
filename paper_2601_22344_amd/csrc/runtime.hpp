// Host-side runtime state shared by the C-ABI translation units (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "rplu.h"

namespace rplu {
struct StepState;
}

#include <vector>

struct rplu_prof_rec {
    int cls;
    hipEvent_t a, b;
};

struct rplu_ctx_s {
    int device = 0;
    int cu_count = 0;
    void* ws = nullptr;             // grow-only device workspace
    size_t ws_cap = 0;
    void* batch_ws = nullptr;       // batched-launch descriptors and queue
    size_t batch_ws_cap = 0;
    rplu::StepState* host_state = nullptr;   // pinned staging for state read-back
    bool prof_on = false;                    // record events around launches
    std::vector<hipEvent_t> ev_pool;         // reusable events
    size_t ev_used = 0;
    std::vector<rplu_prof_rec> prof;
};

namespace rplu {
rplu_status fail(rplu_status code, const char* fmt, ...);
rplu_status hip_fail(hipError_t e, const char* what);
size_t dtype_size(int dt);
rplu_status ws_reserve(rplu_ctx_s* ctx, size_t bytes, hipStream_t s);

// Enqueues `launch` on stream s; while profiling is on, brackets it with two
// events and remembers them under class `cls`.
template <class F>
inline void timed(rplu_ctx_s* ctx, int cls, hipStream_t s, F&& launch) {
    if (!ctx->prof_on) { launch(); return; }
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
}  // namespace rplu
