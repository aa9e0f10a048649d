// C ABI of the batched launch: job checks, queue order, the autotuner and its
// table. The kernel is in batched.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "launch.hpp"
#include "runtime.hpp"

namespace rplu {
namespace {

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Prepared {
    int dtype = RPLU_R32;
    int maxn = 0, maxm = 0;
    double mean_area = 0.0;
    std::vector<BatchJob> jobs;
};

rplu_status prepare(int64_t count, const rplu_job* jobs, Prepared& P, const char* who) {
    if (count < 0 || count > INT32_MAX) return fail(RPLU_E_ARG, "%s: count %lld out of range", who, (long long)count);
    if (count > 0 && jobs == nullptr) return fail(RPLU_E_ARG, "%s: jobs is NULL", who);
    P.jobs.resize((size_t)count);
    P.dtype = count > 0 ? jobs[0].dtype : RPLU_R32;
    double area = 0.0;
    for (int64_t b = 0; b < count; ++b) {
        const rplu_job& j = jobs[b];
        const long long lb = (long long)b;
        if (j.kind != RPLU_JOB_DENSE) return fail(RPLU_E_UNSUPPORTED, "%s: job %lld: dense jobs only", who, lb);
        if (j.dtype != RPLU_R32 && j.dtype != RPLU_R64)
            return fail(RPLU_E_UNSUPPORTED, "%s: job %lld: dtype must be R32 or R64", who, lb);
        if (j.dtype != P.dtype) return fail(RPLU_E_ARG, "%s: job %lld: all jobs must share one dtype", who, lb);
        if (j.n < 1 || j.m < 1) return fail(RPLU_E_ARG, "%s: job %lld: empty shape", who, lb);
        if (j.n > RPLU_BATCH_MAX_DIM || j.m > RPLU_BATCH_MAX_DIM)
            return fail(RPLU_E_UNSUPPORTED, "%s: job %lld: n and m must be <= %d", who, lb, RPLU_BATCH_MAX_DIM);
        if (j.A == nullptr || j.lda < j.m) return fail(RPLU_E_ARG, "%s: job %lld: A NULL or lda < m", who, lb);
        if (j.piv == nullptr) return fail(RPLU_E_ARG, "%s: job %lld: piv is required", who, lb);
        if (j.L != nullptr && j.ldl < j.n) return fail(RPLU_E_ARG, "%s: job %lld: ldl < n", who, lb);
        if (j.U != nullptr && j.ldu < j.m) return fail(RPLU_E_ARG, "%s: job %lld: ldu < m", who, lb);
        if (!(j.rel_tol >= 0.0)) return fail(RPLU_E_ARG, "%s: job %lld: rel_tol must be >= 0", who, lb);
        if (j.flags & (RPLU_FLAG_C2PLU | RPLU_FLAG_CPLU))
            return fail(RPLU_E_ARG, "%s: job %lld: RPLU_FLAG_C2PLU and RPLU_FLAG_CPLU are not "
                        "available in batches", who, lb);
        if ((j.flags & RPLU_FLAG_REFRESH) &&
            (j.A_orig == nullptr || j.lda_orig < j.m || j.L == nullptr || j.U == nullptr))
            return fail(RPLU_E_ARG, "%s: job %lld: RPLU_FLAG_REFRESH needs A_orig (lda_orig >= m), "
                        "L and U", who, lb);
        const int64_t es = (int64_t)dtype_size(j.dtype);
        const int64_t mn = std::min(j.n, j.m);
        BatchJob& q = P.jobs[(size_t)b];
        std::memset(&q, 0, sizeof q);
        q.A = j.A;
        q.L = j.L;
        q.U = j.U;
        q.piv = j.piv;
        q.lda = j.lda;
        q.ldl = j.L ? j.ldl : 0;
        q.ldu = j.U ? j.ldu : 0;
        q.n = (int32_t)j.n;
        q.m = (int32_t)j.m;
        q.kmax = (int32_t)(j.max_rank <= 0 ? mn : std::min(j.max_rank, mn));
        // the same rule as rplu_dense (a workspace row when U is NULL is aligned)
        q.vec = ((uintptr_t)j.A % 16 == 0) && ((j.lda * es) % 16 == 0) &&
                (j.U == nullptr || (((uintptr_t)j.U % 16 == 0) && ((j.ldu * es) % 16 == 0)));
        q.tol2 = j.rel_tol * j.rel_tol;
        q.stall = (j.flags & RPLU_FLAG_STALL_STOP) ? 1 : 0;
        q.refresh_on = (j.flags & RPLU_FLAG_REFRESH) ? 1 : 0;
        q.seed = j.seed;
        q.stream = j.stream;
        P.maxn = std::max(P.maxn, q.n);
        P.maxm = std::max(P.maxm, q.m);
        area += (double)q.n * (double)q.m;
    }
    P.mean_area = count > 0 ? area / (double)count : 0.0;
    return RPLU_OK;
}

std::vector<int32_t> make_order(const std::vector<BatchJob>& J, int order) {
    std::vector<int32_t> o(J.size());
    std::iota(o.begin(), o.end(), 0);
    if (order == RPLU_ORDER_GIVEN) return o;
    auto cost = [&](int32_t b) {
        const double a = (double)J[b].n * (double)J[b].m;
        return order == RPLU_ORDER_CUBE ? a * (double)J[b].kmax : a;
    };
    // longest (estimated) first; ties keep job order
    std::stable_sort(o.begin(), o.end(), [&](int32_t x, int32_t y) { return cost(x) > cost(y); });
    return o;
}

int ilog2(double v) {
    int e = 0;
    while (v >= 2.0 && e < 62) { v *= 0.5; ++e; }
    return e;
}

uint64_t signature(const Prepared& P) {
    const int64_t w[5] = {P.dtype, ilog2((double)P.jobs.size()), ilog2(2.0 * P.maxn - 1),
                          ilog2(2.0 * P.maxm - 1), ilog2(P.mean_area)};
    return fnv1a(w, sizeof w, 0x6261746368ull);
}

rplu_status batch_reserve(rplu_ctx_s* ctx, size_t bytes, hipStream_t s) {
    if (bytes <= ctx->batch_ws_cap) return RPLU_OK;
    if (ctx->hbm_budget && bytes + ctx->ws_cap > ctx->hbm_budget)
        return fail(RPLU_E_NOMEM, "batched workspace of %zu bytes exceeds the context budget of %zu",
                    bytes + ctx->ws_cap, ctx->hbm_budget);
    if (ctx->batch_ws) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        (void)hipFree(ctx->batch_ws);
        ctx->batch_ws = nullptr;
        ctx->batch_ws_cap = 0;
    }
    const size_t cap = std::max(bytes, (size_t)1 << 20);
    hipError_t e = hipMalloc(&ctx->batch_ws, cap);
    if (e != hipSuccess) {
        ctx->batch_ws = nullptr;
        return fail(RPLU_E_NOMEM, "batched workspace of %zu bytes: %s", cap, hipGetErrorString(e));
    }
    ctx->batch_ws_cap = cap;
    return RPLU_OK;
}

rplu_status check_cfg(const rplu_batch_cfg& c) {
    if (c.rows_per_pass != 1 && c.rows_per_pass != 2 && c.rows_per_pass != 4 && c.rows_per_pass != 8)
        return fail(RPLU_E_ARG, "rplu_batched: rows_per_pass must be 1, 2, 4 or 8");
    if (c.wg_per_cu < 1 || c.wg_per_cu > 8) return fail(RPLU_E_ARG, "rplu_batched: wg_per_cu must be in [1, 8]");
    if (c.order < RPLU_ORDER_AREA || c.order > RPLU_ORDER_GIVEN)
        return fail(RPLU_E_ARG, "rplu_batched: unknown order %d", c.order);
    return RPLU_OK;
}

// One launch over P.jobs with configuration c; optionally the device time
// (events around the launch) and the per-job results.
rplu_status run_batch(rplu_ctx_s* ctx, const Prepared& P, const rplu_batch_cfg& c, hipStream_t s,
                      std::vector<BatchInfo>* infos, float* ms) {
    const int count = (int)P.jobs.size();
    if (count == 0) return RPLU_OK;
    const size_t es = dtype_size(P.dtype);
    if (batched_lds_bytes(P.dtype, P.maxn) + BT_STATIC_LDS > ctx->lds_per_block)
        return fail(RPLU_E_UNSUPPORTED, "rplu_batched: n = %d needs %zu bytes of LDS per workgroup",
                    P.maxn, batched_lds_bytes(P.dtype, P.maxn) + BT_STATIC_LDS);
    const int resident = batched_max_resident(P.dtype, c.rows_per_pass, P.maxn);
    if (resident < 1) return fail(RPLU_E_UNSUPPORTED, "rplu_batched: kernel does not fit on a CU");
    const int per_cu = std::min(c.wg_per_cu, resident);
    const int grid = std::max(1, std::min(count, ctx->cu_count * per_cu));
    const int64_t uscr_ld = (int64_t)round_up((size_t)P.maxm, 64);
    const std::vector<int32_t> order = make_order(P.jobs, c.order);

    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t o = off; off = round_up(off + bytes, 256); return o; };
    const size_t o_jobs = take(sizeof(BatchJob) * count);
    const size_t o_ord = take(sizeof(int32_t) * count);
    const size_t o_inf = take(sizeof(BatchInfo) * count);
    const size_t o_q = take(sizeof(int32_t));
    const size_t o_u = take((size_t)grid * uscr_ld * es);
    rplu_status rc = batch_reserve(ctx, off, s);
    if (rc) return rc;
    char* ws = (char*)ctx->batch_ws;
    hipError_t e = hipMemcpyAsync(ws + o_jobs, P.jobs.data(), sizeof(BatchJob) * count,
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ws + o_ord, order.data(), sizeof(int32_t) * count, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(jobs)");

    BatchLaunch a;
    std::memset(&a, 0, sizeof a);
    a.dtype = P.dtype;
    a.rows = c.rows_per_pass;
    a.grid = grid;
    a.maxn = P.maxn;
    a.count = count;
    a.jobs = (const BatchJob*)(ws + o_jobs);
    a.order = (const int32_t*)(ws + o_ord);
    a.queue = (int*)(ws + o_q);
    a.uscratch = ws + o_u;
    a.uscr_ld = uscr_ld;
    a.infos = (BatchInfo*)(ws + o_inf);

    hipEvent_t ev[2] = {nullptr, nullptr};
    if (ms) {
        if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess)
            return fail(RPLU_E_HIP, "rplu_batched: hipEventCreate failed");
        (void)hipEventRecord(ev[0], s);
    }
    if (ms) launch_batched(a, s);
    else timed(ctx, 0, s, [&] { launch_batched(a, s); });   // profiling: class 0
    e = hipGetLastError();
    if (ms) (void)hipEventRecord(ev[1], s);
    if (e != hipSuccess) {
        if (ms) { (void)hipEventDestroy(ev[0]); (void)hipEventDestroy(ev[1]); }
        return hip_fail(e, "batched launch");
    }
    if (infos) {
        infos->resize(count);
        e = hipMemcpyAsync(infos->data(), a.infos, sizeof(BatchInfo) * count, hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(infos)");
    }
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (ms) {
        e = hipEventElapsedTime(ms, ev[0], ev[1]);
        (void)hipEventDestroy(ev[0]);
        (void)hipEventDestroy(ev[1]);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    }
    return RPLU_OK;
}

// Times candidate configurations on device copies of (a cost-stratified
// subset of) the jobs. The copies keep each input's offset modulo 16 and its
// lda, so the vector-width decision is the one of the real run; L columns go
// to one scratch column per job (ldl = 0) and U rows to the per-workgroup
// row, which moves the same bytes as the real outputs.
rplu_status tune(rplu_ctx_s* ctx, const Prepared& P, hipStream_t s, rplu_batch_cfg* best,
                 double* best_ms) {
    const size_t es = dtype_size(P.dtype);
    const size_t count = P.jobs.size();
    std::vector<size_t> bytes(count);
    size_t total = 0;
    for (size_t b = 0; b < count; ++b) {
        bytes[b] = round_up((size_t)P.jobs[b].n * P.jobs[b].lda * es + 16, 256) +
                   round_up((size_t)P.jobs[b].n * es, 256);
        total += bytes[b];
    }
    size_t freeb = 0, totalb = 0;
    if (hipMemGetInfo(&freeb, &totalb) != hipSuccess) freeb = (size_t)8 << 30;
    const size_t cap = std::min<size_t>((size_t)8 << 30, freeb / 4);
    std::vector<int32_t> pick;
    if (total <= cap) {
        pick.resize(count);
        std::iota(pick.begin(), pick.end(), 0);
    } else {
        const std::vector<int32_t> o = make_order(P.jobs, RPLU_ORDER_AREA);
        const size_t stride = (total + cap - 1) / cap;
        size_t used = 0;
        for (size_t q = 0; q < count; q += stride) {
            if (used + bytes[o[q]] > cap) break;
            pick.push_back(o[q]);
            used += bytes[o[q]];
        }
        if (pick.empty()) return fail(RPLU_E_NOMEM, "rplu_batched_tune: no room for a tuning copy");
    }
    size_t need = 0;
    for (int32_t b : pick) need += bytes[b];
    char* buf = nullptr;
    hipError_t e = hipMalloc((void**)&buf, need);
    if (e != hipSuccess) return fail(RPLU_E_NOMEM, "rplu_batched_tune: %zu bytes: %s", need, hipGetErrorString(e));

    Prepared Q;
    Q.dtype = P.dtype;
    Q.jobs.resize(pick.size());
    double area = 0.0;
    size_t off = 0;
    for (size_t q = 0; q < pick.size(); ++q) {
        const BatchJob& src = P.jobs[pick[q]];
        BatchJob& d = Q.jobs[q];
        d = src;
        d.A = buf + off + (uintptr_t)src.A % 16;
        off += round_up((size_t)src.n * src.lda * es + 16, 256);
        d.L = src.L ? (void*)(buf + off) : nullptr;
        d.ldl = 0;
        off += round_up((size_t)src.n * es, 256);
        d.U = nullptr;
        d.ldu = 0;
        d.piv = nullptr;
        Q.maxn = std::max(Q.maxn, d.n);
        Q.maxm = std::max(Q.maxm, d.m);
        area += (double)d.n * d.m;
    }
    Q.mean_area = area / (double)pick.size();

    auto restore = [&]() -> hipError_t {
        for (size_t q = 0; q < pick.size(); ++q) {
            const BatchJob& src = P.jobs[pick[q]];
            const size_t pitch = (size_t)src.lda * es;
            hipError_t r = hipMemcpy2DAsync(Q.jobs[q].A, pitch, src.A, pitch, (size_t)src.m * es,
                                            (size_t)src.n, hipMemcpyDeviceToDevice, s);
            if (r != hipSuccess) return r;
        }
        return hipSuccess;
    };

    std::vector<rplu_batch_cfg> cands;
    for (int rows : {1, 2, 4}) {        // (8 rows spill registers at 1024 threads)
        const int res = batched_max_resident(P.dtype, rows, Q.maxn);
        for (int wg = 1; wg <= std::min(4, res); ++wg) cands.push_back({rows, wg, RPLU_ORDER_AREA, 0});
    }
    rplu_status rc = RPLU_OK;
    rplu_batch_cfg win{4, 2, RPLU_ORDER_AREA, 0};
    float win_ms = -1.f;
    auto trial = [&](const rplu_batch_cfg& c) -> rplu_status {
        hipError_t r = restore();
        if (r != hipSuccess) return hip_fail(r, "hipMemcpy2DAsync(tuning copy)");
        float ms = 0.f;
        rplu_status st = run_batch(ctx, Q, c, s, nullptr, &ms);
        if (st) return st;
        if (win_ms < 0.f || ms < win_ms) { win_ms = ms; win = c; }
        return RPLU_OK;
    };
    // first launch of each kernel loads its code object: warm every variant
    // on one job (any data: every run ends within kmax steps)
    {
        hipError_t r = restore();
        if (r != hipSuccess) rc = hip_fail(r, "hipMemcpy2DAsync(tuning copy)");
        Prepared W = Q;
        W.jobs.resize(1);
        for (int rows : {1, 2, 4})
            if (rc == RPLU_OK) rc = run_batch(ctx, W, {rows, 1, RPLU_ORDER_GIVEN, 0}, s, nullptr, nullptr);
    }
    for (size_t q = 0; q < cands.size() && rc == RPLU_OK; ++q) rc = trial(cands[q]);
    for (int ord : {RPLU_ORDER_CUBE, RPLU_ORDER_GIVEN}) {
        if (rc) break;
        rplu_batch_cfg c = win;
        c.order = ord;
        rc = trial(c);
    }
    (void)hipStreamSynchronize(s);
    (void)hipFree(buf);
    if (rc) return rc;
    *best = win;
    if (best_ms) *best_ms = win_ms;
    const uint64_t key = signature(P);
    for (rplu_tune_entry& t : ctx->tune)
        if (t.key == key) { t.cfg = win; t.ms = win_ms; return RPLU_OK; }
    ctx->tune.push_back({key, win, win_ms});
    return RPLU_OK;
}

const rplu_tune_entry* lookup(const rplu_ctx_s* ctx, const Prepared& P) {
    const uint64_t key = signature(P);
    for (const rplu_tune_entry& t : ctx->tune)
        if (t.key == key) return &t;
    return nullptr;
}

}  // namespace

// Internal, for the server's step ticks: the BatchJob of one rplu_job (the
// checks and decisions of rplu_batched), and one launch over given jobs.
rplu_status batch_job_of(const rplu_job& j, BatchJob* out) {
    Prepared P;
    rplu_status rc = prepare(1, &j, P, "rplu_server");
    if (rc) return rc;
    *out = P.jobs[0];
    return RPLU_OK;
}

rplu_status batch_launch_jobs(rplu_ctx_s* ctx, int dtype, const std::vector<BatchJob>& jobs,
                              const rplu_batch_cfg& c, hipStream_t s, std::vector<BatchInfo>* out) {
    Prepared P;
    P.dtype = dtype;
    P.jobs = jobs;
    for (const BatchJob& q : jobs) {
        P.maxn = std::max(P.maxn, q.n);
        P.maxm = std::max(P.maxm, q.m);
    }
    return run_batch(ctx, P, c, s, out, nullptr);
}

}  // namespace rplu

using namespace rplu;

extern "C" {

rplu_status rplu_batched_tune(rplu_ctx ctx, int64_t count, const rplu_job* jobs,
                              rplu_batch_cfg* best_out, double* best_ms_out, void* hip_stream) {
    if (ctx == nullptr || best_out == nullptr)
        return fail(RPLU_E_ARG, "rplu_batched_tune: ctx and best_out are required");
    Prepared P;
    rplu_status rc = prepare(count, jobs, P, "rplu_batched_tune");
    if (rc) return rc;
    if (count == 0) return fail(RPLU_E_ARG, "rplu_batched_tune: no jobs");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    return tune(ctx, P, (hipStream_t)hip_stream, best_out, best_ms_out);
}

rplu_status rplu_batched_ex(rplu_ctx ctx, int64_t count, const rplu_job* jobs,
                            rplu_info* infos_host, const rplu_batch_cfg* cfg, void* hip_stream) {
    if (ctx == nullptr || (count > 0 && infos_host == nullptr))
        return fail(RPLU_E_ARG, "rplu_batched: ctx and infos_host are required");
    Prepared P;
    rplu_status rc = prepare(count, jobs, P, "rplu_batched");
    if (rc) return rc;
    if (count == 0) return RPLU_OK;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t s = (hipStream_t)hip_stream;

    rplu_batch_cfg c{0, 0, 0, 0};
    if (cfg) c = *cfg;
    if (c.rows_per_pass == 0 || c.wg_per_cu == 0 || c.order == 0) {
        rplu_batch_cfg base{4, 2, RPLU_ORDER_AREA, 0};
        const rplu_tune_entry* t = lookup(ctx, P);
        if (t) base = t->cfg;
        else if (cfg == nullptr) {
            rc = tune(ctx, P, s, &base, nullptr);
            if (rc) return rc;
        }
        if (c.rows_per_pass == 0) c.rows_per_pass = base.rows_per_pass;
        if (c.wg_per_cu == 0) c.wg_per_cu = base.wg_per_cu;
        if (c.order == 0) c.order = base.order;
    }
    rc = check_cfg(c);
    if (rc) return rc;
    std::vector<BatchInfo> out;
    rc = run_batch(ctx, P, c, s, &out, nullptr);
    if (rc) return rc;
    // RPLU_FLAG_REFRESH: jobs the stall rule stopped above their tolerance
    // go on from the true residual, as in rplu_dense (a resumed launch over
    // just those jobs, at most RPLU_MAX_REFRESH rounds)
    std::vector<int32_t> refreshes((size_t)count, 0), first_ref((size_t)count, -1);
    std::vector<int64_t> last_ref((size_t)count, -1);
    for (int round = 0; round < RPLU_MAX_REFRESH; ++round) {
        Prepared R;
        R.dtype = P.dtype;
        std::vector<int64_t> idx;
        for (int64_t b = 0; b < count; ++b) {
            const BatchInfo& o = out[(size_t)b];
            const BatchJob& q = P.jobs[(size_t)b];
            // a tolerance stop on a swept S (steps taken since the start or the
            // last replacement) is checked on the replaced residual too
            const bool tol_check = o.stop == RPLU_STOP_TOL && o.rank > last_ref[(size_t)b];
            if (!(jobs[b].flags & RPLU_FLAG_REFRESH) || o.error != 0 || o.rank >= q.kmax ||
                (o.stop != RPLU_STOP_STALL && o.stop != RPLU_STOP_REFRESH && !tol_check))
                continue;
            last_ref[(size_t)b] = o.rank;
            RefreshArgs ra;
            std::memset(&ra, 0, sizeof ra);
            ra.dtype = P.dtype;
            ra.n = q.n;
            ra.m = q.m;
            ra.t = o.rank;
            ra.A = jobs[b].A_orig;
            ra.lda = jobs[b].lda_orig;
            ra.L = q.L;
            ra.ldl = q.ldl;
            ra.U = q.U;
            ra.ldu = q.ldu;
            ra.S = q.A;
            ra.lds = q.lda;
            ra.piv = q.piv;
            launch_refresh(ra, s);
            BatchJob r = q;
            r.t0 = (int32_t)o.rank;
            r.t_end = 0;
            r.T0_in = o.a_fro2;
            r.Tbest_in = -1.0;
            r.Tref_in = -1.0;
            r.refresh_on = refreshes[(size_t)b] + 1 < RPLU_MAX_REFRESH ? 1 : 0;
            R.jobs.push_back(r);
            R.maxn = std::max(R.maxn, r.n);
            R.maxm = std::max(R.maxm, r.m);
            idx.push_back(b);
        }
        if (idx.empty()) break;
        hipError_t e2 = hipGetLastError();
        if (e2 != hipSuccess) return hip_fail(e2, "residual replacement launch");
        std::vector<BatchInfo> o2;
        rplu_batch_cfg c2 = c;
        c2.order = RPLU_ORDER_GIVEN;
        rc = run_batch(ctx, R, c2, s, &o2, nullptr);
        if (rc) return rc;
        for (size_t q = 0; q < idx.size(); ++q) {
            if (refreshes[(size_t)idx[q]] == 0) first_ref[(size_t)idx[q]] = R.jobs[q].t0;
            out[(size_t)idx[q]] = o2[q];
            refreshes[(size_t)idx[q]] += 1;
        }
    }
    rplu_status first = RPLU_OK;
    int64_t first_b = -1;
    for (int64_t b = 0; b < count; ++b) {
        rplu_info& inf = infos_host[b];
        inf.rank = out[b].rank;
        inf.stop = out[b].stop;
        inf.status = out[b].error;
        inf.a_fro2 = out[b].a_fro2;
        inf.res_fro2 = out[b].res_fro2;
        inf.err_fro2 = -1.0;
        inf.refreshes = refreshes[(size_t)b];
        inf.first_refresh = first_ref[(size_t)b];
        inf.trials = 0;
        if (out[b].error != 0 && first_b < 0) { first = out[b].error; first_b = b; }
    }
    if (first_b >= 0)
        return fail(first, "rplu_batched: job %lld failed with status %d at step %lld",
                    (long long)first_b, (int)first, (long long)out[first_b].rank);
    return RPLU_OK;
}

rplu_status rplu_batched(rplu_ctx ctx, int64_t count, const rplu_job* jobs, rplu_info* infos_host,
                         void* hip_stream) {
    return rplu_batched_ex(ctx, count, jobs, infos_host, nullptr, hip_stream);
}

}  // extern "C"
