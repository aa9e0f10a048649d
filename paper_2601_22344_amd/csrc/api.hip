// C ABI of the RPLU library: argument checks, device workspace, and the host
// step loop that enqueues the per-step kernels.
//
// Step loop. Every kernel reads the step index from the device-side
// StepState, so a chunk of steps is the same sequence of launches whatever t
// is. The host enqueues chunks of CH steps and reads the state's `done` word
// back once per chunk; after the stop test fires on the device, the kernels
// that remain in the chunk return at once. With RPLU_FLAG_GRAPH the chunk is
// captured once into a hipGraph and replayed. One synchronisation with the
// caller's stream per chunk is the only host/device round trip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "cdf.hpp"
#include "common.hpp"
#include "launch.hpp"
#include "runtime.hpp"
#include "bounds_plan.hpp"

namespace rplu {

static thread_local std::string g_last_error;

rplu_status fail(rplu_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

rplu_status hip_fail(hipError_t e, const char* what) {
    return fail(RPLU_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

size_t dtype_size(int dt) {
    switch (dt) {
        case RPLU_R32: return 4;
        case RPLU_R64: return 8;
        case RPLU_C64: return 8;
        case RPLU_C128: return 16;
        default: return 0;
    }
}

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Largest n or m: the sampler chains at most CDF_MAX_GROUPS groups of
// CDF_GROUP chunks of CDF_CHUNK elements.
constexpr int64_t RPLU_MAX_DIM = (int64_t)CDF_MAX_GROUPS * CDF_GROUP * CDF_CHUNK;

rplu_status ws_reserve(rplu_ctx_s* ctx, size_t bytes, hipStream_t s) {
    if (bytes <= ctx->ws_cap) return RPLU_OK;
    if (ctx->hbm_budget && bytes + ctx->batch_ws_cap > ctx->hbm_budget)
        return fail(RPLU_E_NOMEM, "workspace of %zu bytes exceeds the context budget of %zu",
                    bytes + ctx->batch_ws_cap, ctx->hbm_budget);
    if (ctx->ws) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
        graph_cache_clear(ctx);           // captured graphs point into the old workspace
        (void)hipFree(ctx->ws);
        ctx->ws = nullptr;
        ctx->ws_cap = 0;
    }
    size_t cap = std::max(bytes, (size_t)1 << 20);
    hipError_t e = hipMalloc(&ctx->ws, cap);
    if (e != hipSuccess) {
        ctx->ws = nullptr;
        return fail(RPLU_E_NOMEM, "workspace of %zu bytes: %s", cap, hipGetErrorString(e));
    }
    ctx->ws_cap = cap;
    return RPLU_OK;
}

// Carves consecutive 256-byte aligned regions out of the context workspace.
struct Carver {
    size_t off = 0;
    size_t take(size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    }
};

// Without a context the copy goes straight to the caller's (pageable) stack.
static rplu_status read_state(rplu_ctx_s* ctx, const StepState* st, hipStream_t s,
                              StepState* out) {
    StepState* dst = ctx ? ctx->host_state : out;
    hipError_t e = hipMemcpyAsync(dst, st, sizeof(StepState), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(state)");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (ctx) std::memcpy(out, ctx->host_state, sizeof(StepState));
    return RPLU_OK;
}

static rplu_status finish(const StepState& hs, rplu_info* info, int refreshes = 0,
                          int first_refresh = -1) {
    info->rank = hs.t;
    info->stop = hs.stop;
    info->status = hs.error;
    info->a_fro2 = hs.T0;
    info->res_fro2 = hs.T;
    info->err_fro2 = -1.0;
    info->refreshes = refreshes;
    info->first_refresh = first_refresh;
    info->trials = hs.trials_total;
    switch (hs.error) {
        case 0: return RPLU_OK;
        case RPLU_E_NONFINITE: return fail(RPLU_E_NONFINITE, "non-finite mass or pivot at step %d", hs.t);
        case RPLU_E_ZERO_PIVOT: return fail(RPLU_E_ZERO_PIVOT, "forced pivot is zero at step %d", hs.t);
        case RPLU_E_ARG: return fail(RPLU_E_ARG, "forced pivot out of range at step %d", hs.t);
        case RPLU_E_BOUND:
            return fail(RPLU_E_BOUND, "no row accepted in %d trials at step %d",
                        RPLU_BOUND_MAX_TRIALS, hs.t);
        default: return fail(hs.error, "device error %d at step %d", hs.error, hs.t);
    }
}

static void destroy_entry(rplu_graph_entry& g) {
    if (g.main) (void)hipGraphExecDestroy(g.main);
    if (g.rest) (void)hipGraphExecDestroy(g.rest);
    g = rplu_graph_entry{};
}

void graph_cache_clear(rplu_ctx_s* ctx) {
    for (rplu_graph_entry& g : ctx->graphs) destroy_entry(g);
}

template <class F>
static rplu_status capture(rplu_ctx_s* ctx, int64_t steps, F& enqueue_step, hipGraphExec_t* out) {
    hipStream_t cs = ctx->cap_stream;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    for (int64_t q = 0; q < steps; ++q) enqueue_step(cs);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) { *out = nullptr; return hip_fail(e, "hipGraphInstantiate"); }
    return RPLU_OK;
}

// Runs `steps_total` steps of `enqueue_step(stream)`.
//
// Graph path (default): the loop is captured once as a chunk of CH steps and
// a tail of the remaining steps, on the context's capture stream, and the
// instantiated graphs are replayed on the caller's stream; `key` identifies
// the launch arguments, so repeated calls on the same buffers reuse them.
// Plain path (RPLU_FLAG_NO_GRAPH, or while profiling, whose events time
// individual launches): the same launches issued directly. Either way the host reads
// the device `done` word after each chunk and stops early once the stop test
// has fired; the kernels left in a chunk return at once.
template <class F>
static rplu_status run_loop(rplu_ctx_s* ctx, StepState* st, int64_t steps_total, bool use_graph,
                            uint64_t key, hipStream_t s, F&& enqueue_step) {
    if (steps_total <= 0) return RPLU_OK;
    const int64_t CH = steps_total <= 64 ? steps_total : 32;
    int32_t done_word = 0;             // pageable landing word when there is no context
    auto done_after_sync = [&](bool& done) -> rplu_status {
        int32_t* dst = ctx ? &ctx->host_state->done : &done_word;
        hipError_t e = hipMemcpyAsync(dst, &st->done, sizeof(int32_t), hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(done)");
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        done = *dst != 0;
        return RPLU_OK;
    };

    rplu_graph_entry* g = nullptr;
    if (use_graph && ctx != nullptr && !ctx->prof_on && ctx->cap_stream != nullptr) {
        key = fnv1a(&steps_total, sizeof steps_total, key);
        for (rplu_graph_entry& c : ctx->graphs)
            if (c.valid && c.key == key) g = &c;
        if (g == nullptr) {
            rplu_graph_entry* victim = &ctx->graphs[0];
            for (rplu_graph_entry& c : ctx->graphs)
                if (!c.valid || c.last_use < victim->last_use) victim = &c;
            destroy_entry(*victim);
            victim->ch = CH;
            victim->reps = steps_total / CH;
            victim->tail = steps_total - victim->reps * CH;
            rplu_status rc = capture(ctx, CH, enqueue_step, &victim->main);
            if (rc == RPLU_OK && victim->tail > 0)
                rc = capture(ctx, victim->tail, enqueue_step, &victim->rest);
            if (rc == RPLU_OK) {
                victim->key = key;
                victim->valid = true;
                g = victim;
            } else {
                destroy_entry(*victim);    // fall back to plain launches
            }
        }
        if (g != nullptr) g->last_use = ++ctx->use_clock;
    }

    if (g != nullptr) {
        for (int64_t r = 0; r < g->reps; ++r) {
            hipError_t e = hipGraphLaunch(g->main, s);
            if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
            if ((r == g->reps - 1) && g->tail == 0) return RPLU_OK;
            bool done = false;
            rplu_status rc = done_after_sync(done);
            if (rc) return rc;
            if (done) return RPLU_OK;
        }
        if (g->tail > 0) {
            hipError_t e = hipGraphLaunch(g->rest, s);
            if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
        }
        return RPLU_OK;
    }

    for (int64_t done_steps = 0; done_steps < steps_total; done_steps += CH) {
        const int64_t todo = std::min(CH, steps_total - done_steps);
        for (int64_t q = 0; q < todo; ++q) enqueue_step(s);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
        if (done_steps + CH >= steps_total) break;
        bool done = false;
        rplu_status rc = done_after_sync(done);
        if (rc) return rc;
        if (done) break;
    }
    return RPLU_OK;
}

// Work split of an all-pairs mass pass with `rows` targets and `cols`
// sources over a grid of (row blocks) x (splits) workgroups: two workgroups
// per slot of the chip (`wg` workgroups of the kernel per CU at once), at
// least 256 columns per split. Two rounds rather than one let the
// dispatcher refill the slots that the ragged last row block frees early
// (measured at 20000 x 20000: 90 us per pass against 97 us for one round).
// Columns per split are a multiple of the 8-column reciprocal group.
static void cauchy_mass_layout(int cu_count, int wg, int64_t rows, int64_t cols,
                               int64_t* splits_out, int64_t* cps_out) {
    const int64_t nbr = (rows + cauchy_rows_per_block() - 1) / cauchy_rows_per_block();
    const int64_t slots = std::max<int64_t>(1, (int64_t)cu_count * std::max(1, wg));
    int64_t splits = (2 * slots + nbr - 1) / nbr;
    splits = std::max<int64_t>(1, std::min<int64_t>(splits, std::max<int64_t>(1, cols / 256)));
    int64_t cps = (cols + splits - 1) / splits;
    cps = (cps + 7) / 8 * 8;
    *splits_out = (cols + cps - 1) / cps;
    *cps_out = cps;
}

// Dense path: the fused one-workgroup pivot draw (one launch per step
// instead of two) unless a side exceeds its limit or the caller asks for
// the wide form.
static int use_fused_pivot(int64_t n, int64_t m, uint32_t flags) {
    return (n <= PIVOT_FUSED_MAX && m <= PIVOT_FUSED_MAX && !(flags & RPLU_FLAG_SPLIT_SAMPLER))
               ? 1 : 0;
}

static int64_t kmax_of(int64_t n, int64_t m, int64_t k) {
    const int64_t mn = std::min(n, m);
    return k <= 0 ? mn : std::min(k, mn);
}

bool dense_step_eligible(int64_t n, int64_t m, uint32_t flags) {
    return n <= DENSE_STEP_MAX && m <= DENSE_STEP_MAX &&
           !(flags & (RPLU_FLAG_COLMASS | RPLU_FLAG_CPLU | RPLU_FLAG_REFRESH |
                      RPLU_FLAG_SPLIT_SAMPLER | RPLU_FLAG_LAZY_SWEEP));
}

// Workspace of one dense run, carved from a 256-byte aligned base.
DenseWs dense_ws_layout(int dtype, int64_t n, int64_t m, uint32_t flags, bool need_u,
                        bool allow_step) {
    const size_t es = dtype_size(dtype);
    const bool colmass = (flags & RPLU_FLAG_COLMASS) != 0;
    Carver cv;
    DenseWs w;
    w.step = allow_step && dense_step_eligible(n, m, flags);
    w.o_st = cv.take(sizeof(StepState));
    w.o_rm = cv.take((size_t)n * 8 * (w.step ? 2 : 1));   // step form: two buffers
    w.o_rx = (flags & RPLU_FLAG_CPLU) ? cv.take((size_t)n * 8) : 0;
    w.o_ctr = cv.take((size_t)cdf_chunks((int)n) * 8);
    w.o_ctc = cv.take((size_t)cdf_chunks((int)m) * 8);
    const int64_t nbc = (n + DENSE_ROWS_COLMASS - 1) / DENSE_ROWS_COLMASS;
    w.o_cp = colmass ? cv.take((size_t)nbc * m * 8) : 0;
    w.o_u = need_u ? cv.take((size_t)m * es) : 0;
    if (w.step) {
        w.groups = (int)((n + DENSE_STEP_ROWS - 1) / DENSE_STEP_ROWS);
        w.ldur = (m + 3) / 4 * 4;                     // 16-byte aligned rows
        w.o_sts = cv.take((size_t)w.groups * sizeof(StepState));
        w.o_ur = cv.take((size_t)w.groups * (size_t)w.ldur * es);
        w.o_dead = cv.take((size_t)n);
    }
    w.total = cv.off;
    return w;
}

rplu_status dense_check(const char* who, int dtype, int64_t n, int64_t m, const void* A,
                        int64_t lda, const rplu_opts* opts, const int32_t* piv, const void* L,
                        int64_t ldl, const void* U, int64_t ldu, const rplu_info* info) {
    if (opts == nullptr || info == nullptr)
        return fail(RPLU_E_ARG, "%s: opts and info are required", who);
    if (dtype_size(dtype) == 0) return fail(RPLU_E_ARG, "%s: unknown dtype %d", who, dtype);
    if (n < 1 || m < 1 || n > INT32_MAX || m > INT32_MAX)
        return fail(RPLU_E_ARG, "%s: shape %lld x %lld out of range", who, (long long)n,
                    (long long)m);
    if (A == nullptr || lda < m) return fail(RPLU_E_ARG, "%s: A NULL or lda < m", who);
    if (piv == nullptr) return fail(RPLU_E_ARG, "%s: piv is required", who);
    if (L != nullptr && ldl < n) return fail(RPLU_E_ARG, "%s: ldl < n", who);
    if (U != nullptr && ldu < m) return fail(RPLU_E_ARG, "%s: ldu < m", who);
    if (opts->rel_tol < 0 || !(opts->rel_tol == opts->rel_tol))
        return fail(RPLU_E_ARG, "%s: rel_tol must be >= 0", who);
    if (opts->colmass_out != nullptr && !(opts->flags & RPLU_FLAG_COLMASS))
        return fail(RPLU_E_ARG, "%s: colmass_out needs RPLU_FLAG_COLMASS", who);
    if (n > RPLU_MAX_DIM || m > RPLU_MAX_DIM)
        return fail(RPLU_E_UNSUPPORTED, "%s: n and m must be <= %lld", who,
                    (long long)RPLU_MAX_DIM);
    if (opts->flags & RPLU_FLAG_CPLU) {
        if (opts->flags & RPLU_FLAG_C2PLU)
            return fail(RPLU_E_ARG, "%s: RPLU_FLAG_CPLU with RPLU_FLAG_C2PLU", who);
        if (opts->flags & RPLU_FLAG_COLMASS)
            return fail(RPLU_E_UNSUPPORTED, "%s: RPLU_FLAG_CPLU with RPLU_FLAG_COLMASS", who);
    }
    if (opts->flags & RPLU_FLAG_REFRESH) {
        if (dtype != RPLU_R32 && dtype != RPLU_R64)
            return fail(RPLU_E_UNSUPPORTED, "%s: RPLU_FLAG_REFRESH needs R32 or R64", who);
        if (opts->flags & RPLU_FLAG_COLMASS)
            return fail(RPLU_E_UNSUPPORTED, "%s: RPLU_FLAG_REFRESH with RPLU_FLAG_COLMASS", who);
        const bool orig = (opts->A_orig != nullptr && opts->lda_orig >= m) ||
                          (opts->A_orig == nullptr && (opts->flags & RPLU_FLAG_KEEP_INPUT));
        if (!orig || L == nullptr || U == nullptr)
            return fail(RPLU_E_ARG, "%s: RPLU_FLAG_REFRESH needs A_orig (lda_orig >= m) or "
                        "RPLU_FLAG_KEEP_INPUT, and L and U", who);
    }
    return RPLU_OK;
}

// The dense step loop on a workspace laid out by dense_ws_layout at `ws`.
// With a context: graph replay (unless RPLU_FLAG_NO_GRAPH), profiling, pinned
// read-back. Without (ctx == nullptr): plain launches and pageable read-back
// only, so nothing is allocated.
rplu_status dense_run(rplu_ctx_s* ctx, char* ws, int dtype, int64_t n, int64_t m, void* A,
                      int64_t lda, const rplu_opts* opts, int32_t* piv, void* L, int64_t ldl,
                      void* U, int64_t ldu, rplu_info* info, hipStream_t s) {
    const size_t es = dtype_size(dtype);
    const int64_t kmax = kmax_of(n, m, opts->max_rank);
    const bool colmass = (opts->flags & RPLU_FLAG_COLMASS) != 0;
    const DenseWs w = dense_ws_layout(dtype, n, m, opts->flags, U == nullptr, ctx != nullptr);

    DenseArgs a;
    std::memset(&a, 0, sizeof a);        // padding too: the struct keys the graph cache
    a.dtype = dtype;
    // deferred sweep (the same results bit for bit): for matrices that do not
    // stay in the caches, when L and U are stored and no column masses asked
    const bool can_lazy = L != nullptr && U != nullptr && !colmass;
    const bool big = (size_t)n * (size_t)lda * es >= RPLU_LAZY_MIN_BYTES;
    a.lazy = can_lazy && !(opts->flags & RPLU_FLAG_EAGER_SWEEP) &&
             (big || (opts->flags & RPLU_FLAG_LAZY_SWEEP)) ? 1 : 0;
    a.n = n;
    a.m = m;
    a.S = A;
    a.lda = lda;
    a.U = U ? U : (void*)(ws + w.o_u);
    a.ldu = U ? ldu : 0;          // a single workspace row, reused every step
    a.L = L;
    a.ldl = ldl;
    a.piv = piv;
    a.st = (StepState*)(ws + w.o_st);
    a.rowmass = (double*)(ws + w.o_rm);
    a.rowmax = (opts->flags & RPLU_FLAG_CPLU) ? (double*)(ws + w.o_rx) : nullptr;
    a.ct_col = (double*)(ws + w.o_ctc);
    a.colpart = colmass ? (double*)(ws + w.o_cp) : nullptr;
    a.colmass = colmass;
    a.vec_ok = ((uintptr_t)A % 16 == 0) && ((lda * (int64_t)es) % 16 == 0) &&
               ((uintptr_t)a.U % 16 == 0) && ((a.ldu * (int64_t)es) % 16 == 0);
    a.colmass_out = opts->colmass_out;
    a.rowmass_out = opts->rowmass_out;
    a.trace = opts->trace;
    a.forced = opts->forced;
    a.seed = opts->seed;
    a.stream = opts->stream;
    a.kmax = kmax;
    a.tol2 = opts->rel_tol * opts->rel_tol;

    const bool refresh = (opts->flags & RPLU_FLAG_REFRESH) != 0;
    // small runs: draws and sweep of a step in one launch (k_dense_step), the
    // same results bit for bit; workgroup 0's state is the run's
    DenseStepArgs d;
    std::memset(&d, 0, sizeof d);
    if (w.step) {
        d.states = (StepState*)(ws + w.o_sts);
        d.masses = a.rowmass;
        d.urows = ws + w.o_ur;
        d.ldur = w.ldur;
        d.dead = (uint8_t*)(ws + w.o_dead);
        d.groups = w.groups;
        a.st = d.states;
        launch_dense_step_init(a, d, s);
    } else {
        launch_state_init(a.st, s, refresh ? 1 : 0);
    }
    timed(ctx, 3, s, [&] { launch_dense_sweep(a, /*init=*/true, s); });
    if (colmass && a.colmass_out) launch_colmass_reduce(a, false, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "initial mass launch");

    SampleArgs sa;
    std::memset(&sa, 0, sizeof sa);
    sa.dtype = dtype;
    sa.p = 0;
    sa.n = n;
    sa.m = m;
    sa.rowmass = a.rowmass;
    sa.ct_row = (double*)(ws + w.o_ctr);
    sa.ct_col = a.ct_col;
    sa.st = a.st;
    sa.piv = piv;
    sa.U = a.U;
    sa.ldu = a.ldu;
    sa.seed = opts->seed;
    sa.stream = opts->stream;
    sa.kmax = kmax;
    sa.tol2 = a.tol2;
    sa.stall = (opts->flags & RPLU_FLAG_STALL_STOP) ? 1 : 0;
    sa.greedy = (opts->flags & RPLU_FLAG_C2PLU) ? 1 : (opts->flags & RPLU_FLAG_CPLU) ? 2 : 0;
    sa.maxmass = (opts->flags & RPLU_FLAG_MAXMASS_STOP) ? 1 : 0;
    sa.rowmax = a.rowmax;
    sa.forced = opts->forced;
    sa.trace = opts->trace;
    sa.rowmass_out = opts->rowmass_out;
    sa.fused = use_fused_pivot(n, m, opts->flags);

    const bool graph = ctx != nullptr && !(opts->flags & RPLU_FLAG_NO_GRAPH);
    uint64_t key = fnv1a(&sa, sizeof sa, fnv1a(&a, sizeof a, 0x64656e7365ull));
    if (w.step) {
        key = fnv1a(&d, sizeof d, key);
        rplu_status rc = run_loop(ctx, a.st, kmax + 1, graph, key, s, [&](hipStream_t q) {
            timed(ctx, 0, q, [&] { launch_dense_step(a, sa, d, q); });
        });
        if (rc) return rc;
        launch_dense_step_finish(a, d, s);
        StepState hs;
        rc = read_state(ctx, a.st, s, &hs);
        if (rc) return rc;
        return finish(hs, info, 0, -1);
    }
    auto step = [&](hipStream_t q) {
        timed(ctx, 1, q, [&] {
            if (sa.fused) {
                launch_dense_pivot(a, sa, q);
            } else {
                launch_rows_draw(sa, q);
                launch_dense_pivrow_draw(a, sa, q);
            }
        });
        timed(ctx, 0, q, [&] { launch_dense_sweep(a, /*init=*/false, q); });
        if (colmass && a.colmass_out)
            timed(ctx, 2, q, [&] { launch_colmass_reduce(a, true, q); });
    };
    rplu_status rc = run_loop(ctx, a.st, kmax + 1, graph, key, s, step);
    if (rc) return rc;
    launch_dense_flush(a, s);            // deferred sweep: S^(rank) into A
    StepState hs;
    rc = read_state(ctx, a.st, s, &hs);
    if (rc) return rc;
    // RPLU_FLAG_REFRESH: when a replacement is due (the device stopped with
    // RPLU_STOP_REFRESH) or the stall rule fired above the tolerance, the run
    // goes on from the true residual A_orig - L U (formed in FP64)
    // A tolerance stop reached on a swept (not replaced) S is checked the same
    // way: the replaced residual's total is the true error of the factors, so
    // the run stops at once when that is within the tolerance, else goes on.
    int r = 0, first = -1, t_last = -1;
    for (; refresh && r < RPLU_MAX_REFRESH && hs.error == 0 && hs.t < kmax &&
           (hs.stop == RPLU_STOP_REFRESH || hs.stop == RPLU_STOP_STALL ||
            (hs.stop == RPLU_STOP_TOL && hs.t > t_last));
         ++r) {
        if (r == 0) first = hs.t;
        t_last = hs.t;
        RefreshArgs ra;
        std::memset(&ra, 0, sizeof ra);
        ra.dtype = dtype;
        ra.n = n;
        ra.m = m;
        ra.t = hs.t;
        ra.A = opts->A_orig;
        ra.lda = opts->lda_orig;
        ra.L = L;
        ra.ldl = ldl;
        ra.U = U;
        ra.ldu = ldu;
        ra.S = A;
        ra.lds = lda;
        ra.piv = piv;
        launch_refresh(ra, s);
        timed(ctx, 3, s, [&] { launch_dense_sweep(a, /*init=*/true, s); });
        launch_state_resume(a.st, r + 1 < RPLU_MAX_REFRESH ? 1 : 0, s);
        hipError_t e2 = hipGetLastError();
        if (e2 != hipSuccess) return hip_fail(e2, "residual replacement launch");
        rc = run_loop(ctx, a.st, kmax + 1 - hs.t, graph, key, s, step);
        if (rc) return rc;
        launch_dense_flush(a, s);
        rc = read_state(ctx, a.st, s, &hs);
        if (rc) return rc;
    }
    return finish(hs, info, r, first);
}


// Cauchy-like run: argument checks, workspace layout and the step loop on a
// given workspace (the server places it in a job's slot).
rplu_status cauchy_check(const char* who, int dtype, int64_t n, int64_t m, int p, const void* x,
                         const void* y, const void* G, const void* B, const rplu_opts* opts,
                         const int32_t* piv, const void* L, int64_t ldl, const void* U,
                         int64_t ldu, const rplu_info* info) {
    if (opts == nullptr || info == nullptr)
        return fail(RPLU_E_ARG, "%s: opts and info are required", who);
    if (dtype != RPLU_C128) return fail(RPLU_E_UNSUPPORTED, "%s: only RPLU_C128", who);
    if (opts->flags & RPLU_FLAG_CPLU)
        return fail(RPLU_E_UNSUPPORTED, "%s: RPLU_FLAG_CPLU is for dense matrices", who);
    if (n < 1 || m < 1 || n > INT32_MAX || m > INT32_MAX)
        return fail(RPLU_E_ARG, "%s: shape out of range", who);
    if (p < 1 || p > 4) return fail(RPLU_E_UNSUPPORTED, "%s: p must be in [1, 4]", who);
    if (!x || !y || !G || !B || !piv)
        return fail(RPLU_E_ARG, "%s: x, y, G, B and piv are required", who);
    if (L != nullptr && ldl < n) return fail(RPLU_E_ARG, "%s: ldl < n", who);
    if (U != nullptr && ldu < m) return fail(RPLU_E_ARG, "%s: ldu < m", who);
    if (opts->rel_tol < 0 || !(opts->rel_tol == opts->rel_tol))
        return fail(RPLU_E_ARG, "%s: rel_tol must be >= 0", who);
    if (opts->colmass_out != nullptr && !(opts->flags & RPLU_FLAG_COLMASS))
        return fail(RPLU_E_ARG, "%s: colmass_out needs RPLU_FLAG_COLMASS", who);
    if (opts->flags & RPLU_FLAG_REFRESH)
        return fail(RPLU_E_UNSUPPORTED, "%s: RPLU_FLAG_REFRESH is for dense runs", who);
    if (opts->flags & RPLU_FLAG_BOUNDS) {
        if (opts->flags & RPLU_FLAG_COLMASS)
            return fail(RPLU_E_UNSUPPORTED, "%s: RPLU_FLAG_BOUNDS with RPLU_FLAG_COLMASS", who);
        if (!(opts->bound_nu == 0.0 || opts->bound_nu >= 1.0) || !std::isfinite(opts->bound_nu))
            return fail(RPLU_E_ARG, "%s: bound_nu must be 0 (default) or >= 1", who);
        if (opts->bound_leaf < 0 || opts->bound_leaf > RPLU_BOUND_LEAF_MAX)
            return fail(RPLU_E_ARG, "%s: bound_leaf must be in [0, %d]", who, RPLU_BOUND_LEAF_MAX);
    }
    if (n > RPLU_MAX_DIM || m > RPLU_MAX_DIM)
        return fail(RPLU_E_UNSUPPORTED, "%s: n and m must be <= %lld", who,
                    (long long)RPLU_MAX_DIM);
    return RPLU_OK;
}

CauchyWs cauchy_ws_layout(const MassSlots& sl, int64_t n, int64_t m, int p, uint32_t flags,
                          bool colmass, bool need_u) {
    (void)flags;
    CauchyWs w;
    const int pc = (p >= 1 && p <= 4) ? p : 1;
    cauchy_mass_layout(sl.cu_count, sl.row_wg[pc], n, m, &w.splits, &w.cps);
    if (colmass) cauchy_mass_layout(sl.cu_count, sl.col_wg[pc], m, n, &w.splits_c, &w.cps_c);
    Carver cv;
    w.o_st = cv.take(sizeof(StepState));
    w.o_rm = cv.take((size_t)n * 8);
    w.o_pa = cv.take((size_t)n * w.splits * 8);
    w.o_ctr = cv.take((size_t)cdf_chunks((int)n) * 8);
    w.o_ctc = cv.take((size_t)cdf_chunks((int)m) * 8);
    w.o_u = need_u ? cv.take((size_t)m * 16) : 0;
    w.o_mc = cv.take(cauchy_mass_col_bytes(p, m));
    w.o_mf = cv.take(cauchy_mass_frame_bytes(p));
    w.o_pc = colmass ? cv.take((size_t)m * w.splits_c * 8) : 0;
    w.o_gt = (colmass && p > 1) ? cv.take((size_t)n * p * 16) : 0;
    w.o_bt = (colmass && p > 1) ? cv.take((size_t)m * p * 16) : 0;
    w.total = cv.off;
    return w;
}

rplu_status cauchy_run(rplu_ctx_s* ctx, char* ws, int64_t n, int64_t m, int p, const void* x,
                       const void* y, void* G, void* B, const rplu_opts* opts, int32_t* piv,
                       void* L, int64_t ldl, void* U, int64_t ldu, rplu_info* info,
                       hipStream_t s, const BoundsPlan* bp) {
    const bool colmass = opts->colmass_out != nullptr;
    const int64_t kmax = kmax_of(n, m, opts->max_rank);
    const CauchyWs w = cauchy_ws_layout(ctx->mass_slots, n, m, p, opts->flags, colmass, U == nullptr);
    CauchyArgs a;
    std::memset(&a, 0, sizeof a);        // padding too: the struct keys the graph cache
    a.splits = (int)w.splits;
    a.cols_per_split = (int)w.cps;
    char* wsb = ws;
    a.n = n;
    a.m = m;
    a.p = p;
    a.mcol = (p == 1) ? (void*)(wsb + w.o_mc) : nullptr;
    a.mframe = (p == 1) ? (void*)(wsb + w.o_mf) : nullptr;
    a.x = x;
    a.y = y;
    a.G = G;
    a.B = B;
    a.U = U ? U : (void*)(wsb + w.o_u);
    a.ldu = U ? ldu : 0;
    a.L = L;
    a.ldl = ldl;
    a.piv = piv;
    a.st = (StepState*)(wsb + w.o_st);
    a.partial = (double*)(wsb + w.o_pa);
    a.rowmass = (double*)(wsb + w.o_rm);
    a.ct_col = (double*)(wsb + w.o_ctc);
    a.colmass_out = opts->colmass_out;
    a.trace = opts->trace;
    a.forced = opts->forced;
    a.seed = opts->seed;
    a.stream = opts->stream;
    a.kmax = kmax;
    // with bounds the stop test runs on sum(u), with tol^2 / nu (certified);
    // the max-mass rule takes tol^2 as it is
    const bool maxmass = (opts->flags & RPLU_FLAG_MAXMASS_STOP) != 0;
    a.tol2 = opts->rel_tol * opts->rel_tol / (bp && !maxmass ? bp->nu : 1.0);

    CauchyArgs ac;                       // the column pass
    std::memset(&ac, 0, sizeof ac);
    if (colmass) {
        ac.n = m;
        ac.m = n;
        ac.p = p;
        ac.x = y;
        ac.y = x;
        // for p = 1, B (1 x m) read as m x 1 is B^T and G (n x 1) read as 1 x n is G^T
        ac.G = (p > 1) ? (void*)(wsb + w.o_bt) : B;     // B^T, m x p
        ac.B = (p > 1) ? (void*)(wsb + w.o_gt) : G;     // G^T, p x n
        ac.st = a.st;
        ac.partial = (double*)(wsb + w.o_pc);
        ac.splits = (int)w.splits_c;
        ac.cols_per_split = (int)w.cps_c;
    }

    launch_state_init(a.st, s);
    launch_cauchy_frame(a, s);
    SampleArgs sa;
    std::memset(&sa, 0, sizeof sa);
    sa.dtype = RPLU_C128;
    sa.p = p;
    sa.n = n;
    sa.m = m;
    sa.rowmass = bp ? bp->u : a.rowmass;
    sa.ct_row = (double*)(wsb + w.o_ctr);
    sa.ct_col = a.ct_col;
    sa.st = a.st;
    sa.piv = piv;
    sa.U = a.U;
    sa.ldu = a.ldu;
    sa.G = G;
    sa.B = B;
    sa.seed = opts->seed;
    sa.stream = opts->stream;
    sa.kmax = kmax;
    sa.tol2 = a.tol2;
    sa.stall = (opts->flags & RPLU_FLAG_STALL_STOP) ? 1 : 0;
    sa.greedy = (opts->flags & RPLU_FLAG_C2PLU) ? 1 : 0;
    sa.maxmass = maxmass ? 1 : 0;
    sa.forced = opts->forced;
    sa.trace = opts->trace;
    sa.rowmass_out = opts->rowmass_out;
    const bool graph = !(opts->flags & RPLU_FLAG_NO_GRAPH);
    uint64_t key = fnv1a(&ac, sizeof ac, fnv1a(&sa, sizeof sa,
                                              fnv1a(&a, sizeof a, 0x636175636879ull)));
    if (bp) key = fnv1a(bp, sizeof *bp, key);
    rplu_status rc;
    if (bp) {
        rc = run_loop(ctx, a.st, kmax + 1, graph, key, s, [&](hipStream_t q) {
            timed(ctx, 0, q, [&] { launch_bh_bounds(*bp, a, q); });
            timed(ctx, 1, q, [&] {
                launch_rows_draw(sa, q);
                launch_bh_reject(*bp, a, sa, q);
                launch_cauchy_rowgen_draw(a, sa, q);
            });
            timed(ctx, 2, q, [&] { launch_cauchy_update(a, q); });
        });
        if (rc) return rc;
        StepState hs;
        rc = read_state(ctx, a.st, s, &hs);
        if (rc) return rc;
        return finish(hs, info);
    }
    rc = run_loop(ctx, a.st, kmax + 1, graph, key, s, [&](hipStream_t q) {
        timed(ctx, 0, q, [&] { launch_cauchy_mass(a, q); });
        if (colmass)
            timed(ctx, 2, q, [&] {
                if (p > 1) launch_cauchy_transpose(a, ac.B, ac.G, q);
                launch_cauchy_mass(ac, q);
                launch_colmass_sum(ac.partial, ac.splits, m, a.st, a.colmass_out, m, kmax, q);
            });
        timed(ctx, 1, q, [&] {
            launch_cauchy_reduce_draw(a, sa, q);
            launch_cauchy_rowgen_draw(a, sa, q);
        });
        timed(ctx, 2, q, [&] { launch_cauchy_update(a, q); });
    });
    if (rc) return rc;
    StepState hs;
    rc = read_state(ctx, a.st, s, &hs);
    if (rc) return rc;
    return finish(hs, info);
}


// RPLU in CUR form (Alg. 2): argument checks, workspace and the step loop.
static rplu_status cur_run(rplu_ctx_s* ctx, int dtype, int64_t n, int64_t m, const void* A,
                           int64_t lda, const rplu_opts* opts, int32_t* piv, void* Ucore,
                           int64_t ldc, rplu_info* info, hipStream_t s) {
    const char* who = "rplu_cur";
    if (opts == nullptr || info == nullptr)
        return fail(RPLU_E_ARG, "%s: opts and info are required", who);
    if (dtype_size(dtype) == 0) return fail(RPLU_E_ARG, "%s: unknown dtype %d", who, dtype);
    if (n < 1 || m < 1 || n > INT32_MAX || m > INT32_MAX)
        return fail(RPLU_E_ARG, "%s: shape %lld x %lld out of range", who, (long long)n,
                    (long long)m);
    if (n > RPLU_MAX_DIM || m > RPLU_MAX_DIM)
        return fail(RPLU_E_UNSUPPORTED, "%s: n and m must be <= %lld", who,
                    (long long)RPLU_MAX_DIM);
    if (A == nullptr || lda < m) return fail(RPLU_E_ARG, "%s: A NULL or lda < m", who);
    if (piv == nullptr || Ucore == nullptr)
        return fail(RPLU_E_ARG, "%s: piv and Ucore are required", who);
    const int64_t kmax = kmax_of(n, m, opts->max_rank);
    if (kmax > RPLU_CUR_MAX_RANK)
        return fail(RPLU_E_UNSUPPORTED, "%s: rank %lld above RPLU_CUR_MAX_RANK (%d)", who,
                    (long long)kmax, RPLU_CUR_MAX_RANK);
    if (ldc < kmax) return fail(RPLU_E_ARG, "%s: ldc < kmax", who);
    if (opts->rel_tol < 0 || !(opts->rel_tol == opts->rel_tol))
        return fail(RPLU_E_ARG, "%s: rel_tol must be >= 0", who);
    if (opts->flags & (RPLU_FLAG_COLMASS | RPLU_FLAG_REFRESH | RPLU_FLAG_CPLU) ||
        opts->colmass_out != nullptr)
        return fail(RPLU_E_UNSUPPORTED, "%s: column masses, residual replacement and CPLU "
                    "are not available in CUR form", who);

    const size_t es = dtype_size(dtype);
    const size_t ws_ = (dtype == RPLU_C64 || dtype == RPLU_C128) ? 16 : 8;   // FP64 form
    const int nbl = cur_l_blocks(m);
    Carver cv;
    const size_t o_st = cv.take(sizeof(StepState));
    const size_t o_nrm = cv.take((size_t)n * 8);
    const size_t o_selr = cv.take((size_t)n);
    const size_t o_selc = cv.take((size_t)m);
    const size_t o_ctr = cv.take((size_t)cdf_chunks((int)n) * 8);
    const size_t o_ctc = cv.take((size_t)cdf_chunks((int)m) * 8);
    const size_t o_rh = cv.take((size_t)m * ws_);
    const size_t o_l = cv.take((size_t)m * ws_);
    const size_t o_vec = cv.take((size_t)6 * kmax * ws_);
    const size_t o_l2 = cv.take((size_t)nbl * 8);
    const size_t o_ut = cv.take((size_t)kmax * kmax * ws_);
    const size_t o_c = cv.take((size_t)n * kmax * es);
    rplu_status rc = ws_reserve(ctx, cv.off, s);
    if (rc) return rc;
    char* ws = (char*)ctx->ws;

    CurArgs c;
    std::memset(&c, 0, sizeof c);        // padding too: the struct keys the graph cache
    c.dtype = dtype;
    c.vec_ok = ((uintptr_t)A % 16 == 0) && ((lda * (int64_t)es) % 16 == 0);
    c.n = n;
    c.m = m;
    c.kmax = kmax;
    c.A = A;
    c.lda = lda;
    c.Uc = Ucore;
    c.ldc = ldc;
    c.Ut = ws + o_ut;
    c.C = ws + o_c;
    c.nrm = (double*)(ws + o_nrm);
    c.selr = (uint8_t*)(ws + o_selr);
    c.selc = (uint8_t*)(ws + o_selc);
    c.rhat = ws + o_rh;
    c.l = ws + o_l;
    char* vec = ws + o_vec;
    c.zv = vec;
    c.zU = vec + 1 * kmax * ws_;
    c.gI = vec + 2 * kmax * ws_;
    c.wv = vec + 3 * kmax * ws_;
    c.y = vec + 4 * kmax * ws_;
    c.Uw = vec + 5 * kmax * ws_;
    c.l2part = (double*)(ws + o_l2);
    c.ct_col = (double*)(ws + o_ctc);
    c.piv = piv;
    c.st = (StepState*)(ws + o_st);

    // initial row norms ||A_i,:||^2: the dense path's first mass pass (it
    // only reads A)
    DenseArgs d;
    std::memset(&d, 0, sizeof d);
    d.dtype = dtype;
    d.n = n;
    d.m = m;
    d.S = const_cast<void*>(A);
    d.lda = lda;
    d.st = c.st;
    d.rowmass = c.nrm;
    d.vec_ok = c.vec_ok != 0;
    launch_state_init(c.st, s);
    hipError_t e = hipMemsetAsync(c.selr, 0, (size_t)n, s);
    if (e == hipSuccess) e = hipMemsetAsync(c.selc, 0, (size_t)m, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync(selection masks)");
    timed(ctx, 3, s, [&] { launch_dense_sweep(d, /*init=*/true, s); });
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "initial row-norm launch");

    SampleArgs sa;
    std::memset(&sa, 0, sizeof sa);
    sa.dtype = dtype;
    sa.n = n;
    sa.m = m;
    sa.rowmass = c.nrm;
    sa.ct_row = (double*)(ws + o_ctr);
    sa.ct_col = c.ct_col;
    sa.st = c.st;
    sa.piv = piv;
    sa.seed = opts->seed;
    sa.stream = opts->stream;
    sa.kmax = kmax;
    sa.tol2 = opts->rel_tol * opts->rel_tol;
    sa.stall = (opts->flags & RPLU_FLAG_STALL_STOP) ? 1 : 0;
    sa.greedy = (opts->flags & RPLU_FLAG_C2PLU) ? 1 : 0;
    sa.forced = opts->forced;
    sa.trace = opts->trace;
    sa.rowmass_out = opts->rowmass_out;
    (void)nbl;

    const bool graph = !(opts->flags & RPLU_FLAG_NO_GRAPH);
    const uint64_t key = fnv1a(&sa, sizeof sa, fnv1a(&c, sizeof c, 0x637572ull));
    // profile classes: 0 the pass over A, 1 the draws, 2 the O(k m + k^2) rest
    auto step = [&](hipStream_t q) {
        timed(ctx, 1, q, [&] {
            launch_rows_draw(sa, q);
            launch_cur_part(c, sa, CUR_PART_PIVOT, q);
        });
        timed(ctx, 2, q, [&] { launch_cur_part(c, sa, CUR_PART_VECTORS, q); });
        timed(ctx, 0, q, [&] { launch_cur_part(c, sa, CUR_PART_SWEEP, q); });
        timed(ctx, 2, q, [&] { launch_cur_part(c, sa, CUR_PART_CORE, q); });
    };
    rc = run_loop(ctx, c.st, kmax + 1, graph, key, s, step);
    if (rc) return rc;
    StepState hs;
    rc = read_state(ctx, c.st, s, &hs);
    if (rc) return rc;
    return finish(hs, info);
}

}  // namespace rplu

using namespace rplu;

extern "C" {

const char* rplu_last_error(void) { return g_last_error.c_str(); }

const char* rplu_status_str(rplu_status s) {
    switch (s) {
        case RPLU_OK: return "RPLU_OK";
        case RPLU_PENDING: return "RPLU_PENDING";
        case RPLU_E_ARG: return "RPLU_E_ARG";
        case RPLU_E_NOMEM: return "RPLU_E_NOMEM";
        case RPLU_E_HIP: return "RPLU_E_HIP";
        case RPLU_E_NONFINITE: return "RPLU_E_NONFINITE";
        case RPLU_E_BUSY: return "RPLU_E_BUSY";
        case RPLU_E_UNSUPPORTED: return "RPLU_E_UNSUPPORTED";
        case RPLU_E_ZERO_PIVOT: return "RPLU_E_ZERO_PIVOT";
        case RPLU_E_BOUND: return "RPLU_E_BOUND";
        default: return "RPLU_E_UNKNOWN";
    }
}

rplu_status rplu_create(int device, size_t hbm_budget_bytes, rplu_ctx* out) {
    if (out == nullptr) return fail(RPLU_E_ARG, "rplu_create: out is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= count)
        return fail(RPLU_E_ARG, "rplu_create: device %d not in [0, %d)", device, count);
    e = hipSetDevice(device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    rplu_ctx_s* c = new rplu_ctx_s();
    c->device = device;
    c->hbm_budget = hbm_budget_bytes;
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) { delete c; return hip_fail(e, "hipGetDeviceProperties"); }
    c->cu_count = prop.multiProcessorCount;
    c->lds_per_block = prop.sharedMemPerBlock;
    c->mass_slots = cauchy_mass_slots(c->cu_count);
    e = hipHostMalloc((void**)&c->host_state, sizeof(StepState), hipHostMallocDefault);
    if (e != hipSuccess) { delete c; return hip_fail(e, "hipHostMalloc"); }
    // capture only (never executes work); default priority
    e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) c->cap_stream = nullptr;   // graphs disabled, plain launches
    *out = c;
    return RPLU_OK;
}

rplu_status rplu_verify(rplu_ctx ctx, rplu_dtype dtype, int64_t n, int64_t m, int64_t k,
                        const void* A, int64_t lda, const void* L, int64_t ldl, const void* U,
                        int64_t ldu, const void* S, int64_t lds, rplu_verify_out* out,
                        void* hip_stream) {
    if (ctx == nullptr || out == nullptr) return fail(RPLU_E_ARG, "rplu_verify: ctx and out are required");
    if (dtype != RPLU_R32 && dtype != RPLU_R64)
        return fail(RPLU_E_UNSUPPORTED, "rplu_verify: real dtypes (R32, R64) only");
    if (n < 1 || m < 1 || k < 0 || n > INT32_MAX || m > INT32_MAX || k > INT32_MAX)
        return fail(RPLU_E_ARG, "rplu_verify: shape out of range");
    if (A == nullptr || lda < m) return fail(RPLU_E_ARG, "rplu_verify: A NULL or lda < m");
    if (k > 0 && (L == nullptr || U == nullptr || ldl < n || ldu < m))
        return fail(RPLU_E_ARG, "rplu_verify: L (ldl >= n) and U (ldu >= m) are required when k > 0");
    if (S != nullptr && lds < m) return fail(RPLU_E_ARG, "rplu_verify: lds < m");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t s = (hipStream_t)hip_stream;
    Carver cv;
    const size_t o_p = cv.take((size_t)verify_tiles(n, m) * 3 * sizeof(double));
    const size_t o_o = cv.take(3 * sizeof(double));
    rplu_status rc = ws_reserve(ctx, cv.off, s);
    if (rc) return rc;
    char* ws = (char*)ctx->ws;
    VerifyArgs a;
    std::memset(&a, 0, sizeof a);
    a.dtype = dtype;
    a.n = n;
    a.m = m;
    a.k = k;
    a.A = A;
    a.lda = lda;
    a.L = L;
    a.ldl = ldl;
    a.U = U;
    a.ldu = ldu;
    a.S = S;
    a.lds = lds;
    a.partial = (double*)(ws + o_p);
    a.out = (double*)(ws + o_o);
    launch_verify(a, s);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "verify launch");
    double h[3];
    e = hipMemcpyAsync(h, a.out, sizeof h, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "rplu_verify read-back");
    out->a_fro2 = h[0];
    out->err_fro2 = h[1];
    out->schur_gap_fro2 = S ? h[2] : 0.0;
    return RPLU_OK;
}

rplu_status rplu_profile_begin(rplu_ctx ctx) {
    if (ctx == nullptr) return fail(RPLU_E_ARG, "rplu_profile_begin: ctx is NULL");
    ctx->prof.clear();
    ctx->ev_used = 0;
    ctx->prof_on = true;
    return RPLU_OK;
}

rplu_status rplu_profile_end(rplu_ctx ctx, rplu_profile* out) {
    if (ctx == nullptr || out == nullptr) return fail(RPLU_E_ARG, "rplu_profile_end: NULL argument");
    std::memset(out, 0, sizeof *out);
    ctx->prof_on = false;
    rplu_status rc = RPLU_OK;
    for (const rplu_prof_rec& r : ctx->prof) {
        hipError_t e = hipEventSynchronize(r.b);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess) { rc = hip_fail(e, "hipEventElapsedTime"); break; }
        out->launches[r.cls] += 1;
        out->ms[r.cls] += ms;
    }
    ctx->prof.clear();
    ctx->ev_used = 0;
    return rc;
}

rplu_status rplu_destroy(rplu_ctx ctx) {
    if (ctx == nullptr) return RPLU_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (hipEvent_t ev : ctx->ev_pool) (void)hipEventDestroy(ev);
    graph_cache_clear(ctx);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->batch_ws) (void)hipFree(ctx->batch_ws);
    if (ctx->host_state) (void)hipHostFree(ctx->host_state);
    delete ctx;
    return RPLU_OK;
}

rplu_status rplu_dense(rplu_ctx ctx, rplu_dtype dtype, int64_t n, int64_t m, void* A,
                       int64_t lda, const rplu_opts* opts, int32_t* piv, void* L, int64_t ldl,
                       void* U, int64_t ldu, rplu_info* info, void* hip_stream) {
    if (ctx == nullptr) return fail(RPLU_E_ARG, "rplu_dense: ctx is required");
    rplu_status rc = dense_check("rplu_dense", dtype, n, m, A, lda, opts, piv, L, ldl, U, ldu, info);
    if (rc) return rc;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t s = (hipStream_t)hip_stream;
    const DenseWs w = dense_ws_layout(dtype, n, m, opts->flags, U == nullptr);
    const bool keep = (opts->flags & RPLU_FLAG_KEEP_INPUT) != 0;
    const size_t es = dtype_size(dtype);
    const size_t copy = keep ? align_up((size_t)n * lda * es + 16, 256) : 0;
    rc = ws_reserve(ctx, w.total + copy, s);
    if (rc) return rc;
    if (!keep)
        return dense_run(ctx, (char*)ctx->ws, dtype, n, m, A, lda, opts, piv, L, ldl, U, ldu,
                         info, s);
    // the working copy keeps A's 16-byte offset and pitch: the same kernels
    // and vector widths as a run on A itself
    char* Ak = (char*)ctx->ws + w.total + (uintptr_t)A % 16;
    e = hipMemcpy2DAsync(Ak, (size_t)lda * es, A, (size_t)lda * es, (size_t)m * es, (size_t)n,
                         hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy2DAsync(KEEP_INPUT copy)");
    rplu_opts o = *opts;
    if ((o.flags & RPLU_FLAG_REFRESH) && o.A_orig == nullptr) {
        o.A_orig = A;
        o.lda_orig = lda;
    }
    return dense_run(ctx, (char*)ctx->ws, dtype, n, m, Ak, lda, &o, piv, L, ldl, U, ldu, info, s);
}

rplu_status rplu_cur(rplu_ctx ctx, rplu_dtype dtype, int64_t n, int64_t m, const void* A,
                     int64_t lda, const rplu_opts* opts, int32_t* piv, void* Ucore, int64_t ldc,
                     rplu_info* info, void* hip_stream) {
    if (ctx == nullptr) return fail(RPLU_E_ARG, "rplu_cur: ctx is required");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    return cur_run(ctx, dtype, n, m, A, lda, opts, piv, Ucore, ldc, info,
                   (hipStream_t)hip_stream);
}

rplu_status rplu_cauchy(rplu_ctx ctx, rplu_dtype dtype, int64_t n, int64_t m, int32_t p,
                        const void* x, const void* y, void* G, void* B, const rplu_opts* opts,
                        int32_t* piv, void* L, int64_t ldl, void* U, int64_t ldu,
                        rplu_info* info, void* hip_stream) {
    if (ctx == nullptr) return fail(RPLU_E_ARG, "rplu_cauchy: ctx is required");
    rplu_status rc = cauchy_check("rplu_cauchy", dtype, n, m, p, x, y, G, B, opts, piv, L, ldl, U,
                                  ldu, info);
    if (rc) return rc;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t s = (hipStream_t)hip_stream;
    const CauchyWs w = cauchy_ws_layout(ctx->mass_slots, n, m, p, opts->flags,
                                        opts->colmass_out != nullptr, U == nullptr);
    const bool keep = (opts->flags & RPLU_FLAG_KEEP_INPUT) != 0;
    const size_t gb = align_up((size_t)n * p * 16, 256), bb = align_up((size_t)p * m * 16, 256);
    // RPLU_FLAG_BOUNDS: the plan (quadtrees and interaction lists) is built
    // on the host from the nodes and placed after the run's workspace
    HostBoundsPlan hp;
    size_t plan_bytes = 0;
    if (opts->flags & RPLU_FLAG_BOUNDS) {
        std::vector<CPoint> hx((size_t)n), hy((size_t)m);
        e = hipMemcpyAsync(hx.data(), x, (size_t)n * 16, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(hy.data(), y, (size_t)m * 16, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "reading the nodes for the bound plan");
        const double nu = opts->bound_nu > 0.0 ? opts->bound_nu : RPLU_BOUND_NU_DEFAULT;
        const int leaf = opts->bound_leaf > 0 ? opts->bound_leaf : RPLU_BOUND_LEAF_DEFAULT;
        build_bounds_plan(hx.data(), n, hy.data(), m, nu, leaf, &hp);
        plan_bytes = align_up(bounds_plan_bytes(hp, n, p), 256);
    }
    rc = ws_reserve(ctx, w.total + plan_bytes + (keep ? gb + bb : 0), s);
    if (rc) return rc;
    BoundsPlan bp;
    std::vector<int32_t> staging;
    if (plan_bytes) {
        e = upload_bounds_plan(hp, n, p, (char*)ctx->ws + w.total, s, &staging, &bp);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "bound plan upload");
    }
    if (keep) {
        char* Gk = (char*)ctx->ws + w.total + plan_bytes;
        char* Bk = Gk + gb;
        e = hipMemcpyAsync(Gk, G, (size_t)n * p * 16, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(Bk, B, (size_t)p * m * 16, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(KEEP_INPUT copy)");
        G = Gk;
        B = Bk;
    }
    return cauchy_run(ctx, (char*)ctx->ws, n, m, p, x, y, G, B, opts, piv, L, ldl, U, ldu, info, s,
                      plan_bytes ? &bp : nullptr);
}

}  // extern "C"
