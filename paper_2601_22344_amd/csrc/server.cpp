// Continuous-batching server behind rplu_server_* (semantics in rplu.h).
//
// State: a FIFO of submitted jobs, a list of admitted jobs that no worker has
// started, and a first-fit slot pool over one device allocation. Admission
// runs under the lock whenever a job is submitted or finishes. Workers take
// admitted work as soon as they are free: all ready small dense jobs of one
// dtype form one batched launch, anything else runs alone. HIP calls are made
// only by workers, outside the lock, on their own streams.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rplu.h"
#include "runtime.hpp"

namespace rplu {
namespace {

using Clock = std::chrono::steady_clock;

size_t rup(size_t v, size_t a) { return (v + a - 1) / a * a; }

// First-fit sub-allocator over [0, cap): free blocks keyed by offset, merged
// with their neighbours on release.
class SlotPool {
public:
    void reset(size_t cap) {
        free_.clear();
        if (cap) free_[0] = cap;
    }
    bool take(size_t bytes, size_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, o = it->first + bytes;
            free_.erase(it);
            if (rest) free_[o] = rest;
            return true;
        }
        return false;
    }
    void give(size_t off, size_t bytes) {
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

private:
    std::map<size_t, size_t> free_;
};

enum { CLS_DENSE = 0, CLS_CAUCHY = 1 };

struct SJob {
    uint64_t ticket = 0;
    rplu_job d{};
    int cls = CLS_DENSE;
    bool batchable = false;
    size_t bytes = 0, off = 0;
    Clock::time_point t_submit, t_done;
    bool done = false;
    rplu_status status = RPLU_PENDING;
    rplu_info info{};
};

struct Worker {
    std::thread th;
    rplu_ctx ctx = nullptr;
    hipStream_t stream = nullptr;
};

double pct(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    const size_t i = std::min(v.size() - 1, (size_t)(q * (double)(v.size() - 1) + 0.5));
    std::nth_element(v.begin(), v.begin() + (ptrdiff_t)i, v.end());
    return v[i];
}

}  // namespace
}  // namespace rplu

using namespace rplu;

struct rplu_server_s {
    rplu_server_cfg cfg{};
    bool simulate = false;
    int device = 0;
    char* pool_base = nullptr;
    size_t pool_cap = 0;
    SlotPool pool;
    std::mutex mu;
    std::condition_variable cv_work;
    std::condition_variable cv_idle;
    std::deque<SJob*> waiting;
    std::deque<SJob*> ready;
    std::unordered_map<uint64_t, SJob*> jobs;
    uint64_t next_ticket = 1;
    int64_t submitted = 0, completed = 0, rejected = 0, active = 0, running = 0;
    int64_t batches = 0, batched_jobs = 0;
    size_t in_use = 0;
    std::vector<double> lat[2];
    double busy_s = 0.0;
    Clock::time_point busy_since;
    bool stopping = false;
    std::vector<Worker> workers;
};

namespace rplu {
namespace {

// With the lock held: admit waiting jobs in FIFO order while they fit.
void admit_locked(rplu_server_s* S) {
    bool any = false;
    while (!S->waiting.empty()) {
        SJob* j = S->waiting.front();
        if (S->cfg.max_slots > 0 && S->active >= S->cfg.max_slots) break;
        size_t off = 0;
        if (!S->pool.take(j->bytes, &off)) break;
        j->off = off;
        S->in_use += j->bytes;
        if (S->active == 0) S->busy_since = Clock::now();
        ++S->active;
        S->waiting.pop_front();
        S->ready.push_back(j);
        any = true;
    }
    if (any) S->cv_work.notify_all();
}

// With the lock held: a job finished (status/info already set).
void finish_locked(rplu_server_s* S, SJob* j) {
    j->t_done = Clock::now();
    j->done = true;
    S->pool.give(j->off, j->bytes);
    S->in_use -= j->bytes;
    --S->active;
    ++S->completed;
    S->lat[j->cls].push_back(std::chrono::duration<double, std::milli>(j->t_done - j->t_submit).count());
    if (S->active == 0)
        S->busy_s += std::chrono::duration<double>(j->t_done - S->busy_since).count();
}

void simulate_run(const std::vector<SJob*>& js) {
    size_t bytes = 0;
    for (SJob* j : js) bytes += j->bytes;
    std::this_thread::sleep_for(std::chrono::duration<double>((double)bytes / 1e10));
    for (SJob* j : js) {
        j->info = rplu_info{};
        j->info.stop = RPLU_STOP_RANK;
        j->status = RPLU_OK;
    }
}

// The job's overwritten inputs in its slot, keeping the caller's pitch and
// 16-byte alignment offset (the vector width the kernels pick depends on it).
void* dense_slot(rplu_server_s* S, const SJob* j) {
    return S->pool_base + j->off + ((uintptr_t)j->d.A % 16);
}

void run_single(rplu_server_s* S, Worker& W, SJob* j) {
    const rplu_job& d = j->d;
    rplu_opts o;
    std::memset(&o, 0, sizeof o);
    o.max_rank = d.max_rank;
    o.rel_tol = d.rel_tol;
    o.seed = d.seed;
    o.stream = d.stream;
    // every job has new buffers: no graph to reuse
    o.flags = RPLU_FLAG_NO_GRAPH | (d.flags & RPLU_FLAG_STALL_STOP);
    hipStream_t s = W.stream;
    if (j->cls == CLS_DENSE) {
        const size_t es = dtype_size(d.dtype), pitch = (size_t)d.lda * es;
        void* A = dense_slot(S, j);
        hipError_t e = hipMemcpy2DAsync(A, pitch, d.A, pitch, (size_t)d.m * es, (size_t)d.n,
                                        hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) { j->status = hip_fail(e, "server: input copy"); return; }
        j->status = rplu_dense(W.ctx, (rplu_dtype)d.dtype, d.n, d.m, A, d.lda, &o, d.piv, d.L,
                               d.ldl, d.U, d.ldu, &j->info, s);
    } else {
        char* G = S->pool_base + j->off;
        char* B = G + rup((size_t)d.n * d.p * 16, 256);
        hipError_t e = hipMemcpyAsync(G, d.G, (size_t)d.n * d.p * 16, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(B, d.B, (size_t)d.p * d.m * 16, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) { j->status = hip_fail(e, "server: input copy"); return; }
        j->status = rplu_cauchy(W.ctx, (rplu_dtype)d.dtype, d.n, d.m, d.p, d.x, d.y, G, B, &o,
                                d.piv, d.L, d.ldl, d.U, d.ldu, &j->info, s);
    }
    j->info.status = j->status;
}

void run_batch(rplu_server_s* S, Worker& W, const std::vector<SJob*>& js) {
    hipStream_t s = W.stream;
    std::vector<rplu_job> dj(js.size());
    std::vector<rplu_info> inf(js.size());
    for (size_t q = 0; q < js.size(); ++q) {
        const rplu_job& d = js[q]->d;
        const size_t es = dtype_size(d.dtype), pitch = (size_t)d.lda * es;
        void* A = dense_slot(S, js[q]);
        hipError_t e = hipMemcpy2DAsync(A, pitch, d.A, pitch, (size_t)d.m * es, (size_t)d.n,
                                        hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) {
            const rplu_status st = hip_fail(e, "server: input copy");
            for (SJob* j : js) { j->status = st; j->info.status = st; }
            return;
        }
        dj[q] = d;
        dj[q].A = A;
    }
    const rplu_batch_cfg cfg{4, 1, RPLU_ORDER_AREA, 0};
    const rplu_status st = rplu_batched_ex(W.ctx, (int64_t)js.size(), dj.data(), inf.data(), &cfg, s);
    const bool per_job = st == RPLU_OK ||
                         std::any_of(inf.begin(), inf.end(), [](const rplu_info& i) { return i.status != 0; });
    for (size_t q = 0; q < js.size(); ++q) {
        js[q]->info = inf[q];
        js[q]->status = per_job ? inf[q].status : st;
        js[q]->info.status = js[q]->status;
    }
}

void worker_main(rplu_server_s* S, int w) {
    Worker& W = S->workers[w];
    if (!S->simulate) (void)hipSetDevice(S->device);
    for (;;) {
        std::vector<SJob*> batch;
        SJob* single = nullptr;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_work.wait(lk, [&] { return S->stopping || !S->ready.empty(); });
            if (S->ready.empty()) return;      // stopping, and nothing left
            SJob* h = S->ready.front();
            if (h->batchable) {
                for (auto it = S->ready.begin(); it != S->ready.end();) {
                    if ((*it)->batchable && (*it)->d.dtype == h->d.dtype) {
                        batch.push_back(*it);
                        it = S->ready.erase(it);
                    } else {
                        ++it;
                    }
                }
                ++S->batches;
                S->batched_jobs += (int64_t)batch.size();
            } else {
                single = h;
                S->ready.pop_front();
            }
            ++S->running;
        }
        if (S->simulate) simulate_run(single ? std::vector<SJob*>{single} : batch);
        else if (single) run_single(S, W, single);
        else run_batch(S, W, batch);
        {
            std::lock_guard<std::mutex> lk(S->mu);
            if (single) finish_locked(S, single);
            for (SJob* j : batch) finish_locked(S, j);
            --S->running;
            admit_locked(S);
        }
        S->cv_idle.notify_all();
    }
}

rplu_status check_job(const rplu_server_s* S, const rplu_job& d, size_t* bytes, int* cls,
                      bool* batchable) {
    if (d.kind == RPLU_JOB_DENSE) {
        const size_t es = dtype_size(d.dtype);
        if (es == 0) return fail(RPLU_E_ARG, "rplu_server_submit: unknown dtype %d", d.dtype);
        if (d.n < 1 || d.m < 1 || d.n > INT32_MAX || d.m > INT32_MAX)
            return fail(RPLU_E_ARG, "rplu_server_submit: shape out of range");
        if (d.A == nullptr || d.lda < d.m || d.piv == nullptr)
            return fail(RPLU_E_ARG, "rplu_server_submit: A, lda >= m and piv are required");
        if ((d.L && d.ldl < d.n) || (d.U && d.ldu < d.m))
            return fail(RPLU_E_ARG, "rplu_server_submit: ldl < n or ldu < m");
        *bytes = rup((size_t)d.n * d.lda * es + 16, 256);
        *cls = CLS_DENSE;
        const int64_t bmax = S->cfg.batch_max_dim;
        *batchable = (d.dtype == RPLU_R32 || d.dtype == RPLU_R64) && d.n <= bmax && d.m <= bmax;
    } else if (d.kind == RPLU_JOB_CAUCHY) {
        if (d.dtype != RPLU_C128) return fail(RPLU_E_UNSUPPORTED, "rplu_server_submit: Cauchy jobs are C128");
        if (d.n < 1 || d.m < 1 || d.n > INT32_MAX || d.m > INT32_MAX || d.p < 1 || d.p > 4)
            return fail(RPLU_E_ARG, "rplu_server_submit: Cauchy shape or p out of range");
        if (!d.x || !d.y || !d.G || !d.B || !d.piv)
            return fail(RPLU_E_ARG, "rplu_server_submit: x, y, G, B and piv are required");
        if ((d.L && d.ldl < d.n) || (d.U && d.ldu < d.m))
            return fail(RPLU_E_ARG, "rplu_server_submit: ldl < n or ldu < m");
        *bytes = rup((size_t)d.n * d.p * 16, 256) + rup((size_t)d.p * d.m * 16 + 16, 256);
        *cls = CLS_CAUCHY;
        *batchable = false;
    } else {
        return fail(RPLU_E_ARG, "rplu_server_submit: unknown job kind %d", d.kind);
    }
    if (!(d.rel_tol >= 0.0)) return fail(RPLU_E_ARG, "rplu_server_submit: rel_tol must be >= 0");
    if (d.flags & RPLU_FLAG_C2PLU) return fail(RPLU_E_ARG, "rplu_server_submit: RPLU_FLAG_C2PLU is not served");
    if (*bytes > S->pool_cap)
        return fail(RPLU_E_ARG, "rplu_server_submit: footprint %zu exceeds the pool (%zu bytes)",
                    *bytes, S->pool_cap);
    return RPLU_OK;
}

void teardown(rplu_server_s* S) {
    for (Worker& W : S->workers) {
        if (W.stream) (void)hipStreamDestroy(W.stream);
        if (W.ctx) (void)rplu_destroy(W.ctx);
    }
    if (S->pool_base) {
        if (S->simulate) std::free(S->pool_base);
        else (void)hipFree(S->pool_base);
    }
    for (auto& kv : S->jobs) delete kv.second;
    delete S;
}

}  // namespace
}  // namespace rplu

extern "C" {

rplu_status rplu_server_create(rplu_ctx ctx, const rplu_server_cfg* cfg, rplu_server* out) {
    if (out == nullptr || cfg == nullptr) return fail(RPLU_E_ARG, "rplu_server_create: cfg and out are required");
    *out = nullptr;
    const bool sim = (cfg->flags & RPLU_SERVER_SIMULATE) != 0;
    if (!sim && ctx == nullptr) return fail(RPLU_E_ARG, "rplu_server_create: ctx is required");
    if (cfg->hbm_budget_bytes < 4096) return fail(RPLU_E_ARG, "rplu_server_create: budget too small");
    rplu_server_s* S = new rplu_server_s();
    S->cfg = *cfg;
    if (S->cfg.workers <= 0) S->cfg.workers = 3;
    if (S->cfg.workers > 16) S->cfg.workers = 16;
    if (S->cfg.batch_max_dim <= 0) S->cfg.batch_max_dim = 2048;
    if (S->cfg.batch_max_dim > 8192) S->cfg.batch_max_dim = 8192;
    S->simulate = sim;
    S->device = ctx ? ctx->device : 0;
    S->pool_cap = rup(cfg->hbm_budget_bytes, 256);
    if (sim) {
        S->pool_base = (char*)std::malloc(256);   // offsets only; never dereferenced
        if (!S->pool_base) { delete S; return fail(RPLU_E_NOMEM, "rplu_server_create: host memory"); }
    } else {
        hipError_t e = hipSetDevice(S->device);
        if (e == hipSuccess) e = hipMalloc((void**)&S->pool_base, S->pool_cap);
        if (e != hipSuccess) {
            S->pool_base = nullptr;
            teardown(S);
            return fail(RPLU_E_NOMEM, "rplu_server_create: slot pool of %zu bytes: %s", S->pool_cap,
                        hipGetErrorString(e));
        }
    }
    S->pool.reset(S->pool_cap);
    S->workers.resize((size_t)S->cfg.workers);
    if (!sim) {
        for (Worker& W : S->workers) {
            rplu_status rc = rplu_create(S->device, &W.ctx);
            if (rc) { teardown(S); return rc; }
            hipError_t e = hipStreamCreateWithFlags(&W.stream, hipStreamNonBlocking);
            if (e != hipSuccess) { W.stream = nullptr; teardown(S); return hip_fail(e, "hipStreamCreateWithFlags"); }
        }
    }
    for (int w = 0; w < S->cfg.workers; ++w) S->workers[(size_t)w].th = std::thread(worker_main, S, w);
    *out = S;
    return RPLU_OK;
}

rplu_status rplu_server_submit(rplu_server S, const rplu_job* job, uint64_t* ticket) {
    if (S == nullptr || job == nullptr || ticket == nullptr)
        return fail(RPLU_E_ARG, "rplu_server_submit: NULL argument");
    size_t bytes = 0;
    int cls = 0;
    bool batchable = false;
    rplu_status rc = check_job(S, *job, &bytes, &cls, &batchable);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stopping) return fail(RPLU_E_ARG, "rplu_server_submit: server is shutting down");
    if (S->cfg.queue_capacity > 0 && (int64_t)S->waiting.size() >= S->cfg.queue_capacity) {
        ++S->rejected;
        return fail(RPLU_E_BUSY, "rplu_server_submit: %zu jobs waiting", S->waiting.size());
    }
    SJob* j = new SJob();
    j->ticket = S->next_ticket++;
    j->d = *job;
    j->cls = cls;
    j->batchable = batchable;
    j->bytes = bytes;
    j->t_submit = Clock::now();
    S->jobs[j->ticket] = j;
    S->waiting.push_back(j);
    ++S->submitted;
    *ticket = j->ticket;
    admit_locked(S);
    return RPLU_OK;
}

rplu_status rplu_server_poll(rplu_server S, uint64_t ticket, rplu_info* info) {
    if (S == nullptr || info == nullptr) return fail(RPLU_E_ARG, "rplu_server_poll: NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) return fail(RPLU_E_ARG, "rplu_server_poll: unknown ticket %llu", (unsigned long long)ticket);
    SJob* j = it->second;
    if (!j->done) return RPLU_PENDING;
    *info = j->info;
    const rplu_status st = j->status;
    S->jobs.erase(it);
    delete j;
    if (st < 0) return fail(st, "rplu_server_poll: job %llu failed", (unsigned long long)ticket);
    return st;
}

rplu_status rplu_server_stats(rplu_server S, rplu_server_stats_t* out) {
    if (S == nullptr || out == nullptr) return fail(RPLU_E_ARG, "rplu_server_stats: NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    std::memset(out, 0, sizeof *out);
    out->submitted = S->submitted;
    out->completed = S->completed;
    out->rejected = S->rejected;
    out->queued = (int64_t)S->waiting.size();
    out->active = S->active;
    std::vector<double> all = S->lat[CLS_DENSE];
    all.insert(all.end(), S->lat[CLS_CAUCHY].begin(), S->lat[CLS_CAUCHY].end());
    out->p50_ms = pct(all, 0.50);
    out->p99_ms = pct(all, 0.99);
    out->p50_dense_ms = pct(S->lat[CLS_DENSE], 0.50);
    out->p99_dense_ms = pct(S->lat[CLS_DENSE], 0.99);
    out->p50_cauchy_ms = pct(S->lat[CLS_CAUCHY], 0.50);
    out->p99_cauchy_ms = pct(S->lat[CLS_CAUCHY], 0.99);
    out->busy_s = S->busy_s + (S->active > 0 ? std::chrono::duration<double>(Clock::now() - S->busy_since).count() : 0.0);
    out->hbm_in_use = S->in_use;
    out->batches = S->batches;
    out->batched_jobs = S->batched_jobs;
    return RPLU_OK;
}

rplu_status rplu_server_destroy(rplu_server S) {
    if (S == nullptr) return RPLU_OK;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        S->cv_idle.wait(lk, [&] { return S->waiting.empty() && S->ready.empty() && S->active == 0; });
        S->stopping = true;
    }
    S->cv_work.notify_all();
    for (Worker& W : S->workers)
        if (W.th.joinable()) W.th.join();
    teardown(S);
    return RPLU_OK;
}

}  // extern "C"
