// Continuous-batching server behind rplu_server_* (semantics in rplu.h).
//
// A submitted job waits in FIFO order until its footprint fits in the slot
// pool (one device allocation, sub-allocated first-fit): a work block (the
// copy of the inputs the run overwrites, the run's workspace, the
// certification partials) and, when the server owns the outputs, an output
// block (piv, L, U). Everything a job touches on the device is inside these
// blocks, so device use stays within the pool. Admitted jobs go to one of two
// executors, whose streams run side by side on the device:
//   * the tick thread (step-level continuous batching): every admitted small
//     dense job (R32/R64, n, m <= batch_max_dim) joins the resident set; one
//     launch of the batched kernel per tick advances every resident job by up
//     to tick_steps steps. A job pauses at the step boundary and resumes in
//     the next tick (the kernel recomputes its row masses from S, the same
//     bits it would have carried), so a job admitted during a tick starts at
//     the next one, and finished jobs leave at once.
//   * worker threads: larger dense jobs and Cauchy-like jobs, one per worker,
//     each run alone on the worker's stream with plain launches.
// A job's results are those of the same run alone: the batched kernel is
// bitwise rplu_dense, pauses do not change a bit, and slots keep each input's
// row pitch and 16-byte offset. HIP calls are made only by the executors,
// outside the lock.
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

#include "launch.hpp"
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
constexpr int DEFAULT_TICK = 32;

struct SJob {
    uint64_t ticket = 0;
    rplu_job d{};
    int cls = CLS_DENSE;
    bool tick = false;           // executor: the tick thread (else a worker)
    bool own_out = false;        // outputs live in the server's output block
    bool certify = false;
    int64_t kmax = 0;
    size_t es = 0;
    size_t work_bytes = 0, out_bytes = 0, work_off = 0, out_off = 0;
    bool work_held = false, out_held = false;
    size_t o_S = 0, o_B = 0, o_ws = 0, o_vf = 0;       // in the work block
    size_t o_piv = 0, o_L = 0, o_U = 0;                 // in the output block
    // device pointers of the run (set at admission)
    void* S = nullptr;           // dense working copy (or Cauchy G), B below
    void* Bw = nullptr;
    int32_t* piv = nullptr;
    void* L = nullptr;
    void* U = nullptr;
    int64_t ldl = 0, ldu = 0;
    // tick jobs between ticks
    bool started = false;
    int32_t t = 0, tbest = 0, refreshes = 0, first_refresh = -1, t_refresh = -1;
    double T0 = 0.0, Tbest = -1.0, Tref = -1.0;
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
    MassSlots mass_slots;                // occupancy of the Cauchy mass kernels
    char* pool_base = nullptr;
    size_t pool_cap = 0;
    SlotPool pool;
    std::mutex mu;
    std::condition_variable cv_work;     // workers
    std::condition_variable cv_tick;     // the tick thread
    std::condition_variable cv_idle;
    std::deque<SJob*> waiting;
    std::deque<SJob*> ready_big;         // admitted, for a worker
    std::deque<SJob*> ready_tick;        // admitted, joining the next tick
    std::unordered_map<uint64_t, SJob*> jobs;
    uint64_t next_ticket = 1;
    int64_t submitted = 0, completed = 0, rejected = 0, active = 0;
    int64_t ticks = 0, tick_jobs = 0, refreshes = 0;
    size_t in_use = 0, peak = 0;
    std::vector<double> lat[2];
    double busy_s = 0.0;
    Clock::time_point busy_since;
    bool stopping = false;
    std::vector<Worker> workers;
    std::thread tick_th;
    rplu_ctx tick_ctx = nullptr;
    hipStream_t tick_stream = nullptr;
};

namespace rplu {
namespace {

// With the lock held: admit waiting jobs in FIFO order while their blocks fit.
void admit_locked(rplu_server_s* S) {
    bool any_tick = false, any_big = false;
    while (!S->waiting.empty()) {
        SJob* j = S->waiting.front();
        if (S->cfg.max_slots > 0 && S->active >= S->cfg.max_slots) break;
        size_t wo = 0, oo = 0;
        if (!S->pool.take(j->work_bytes, &wo)) break;
        if (j->out_bytes && !S->pool.take(j->out_bytes, &oo)) {
            S->pool.give(wo, j->work_bytes);
            break;
        }
        j->work_off = wo;
        j->out_off = oo;
        j->work_held = true;
        j->out_held = j->out_bytes > 0;
        S->in_use += j->work_bytes + j->out_bytes;
        S->peak = std::max(S->peak, S->in_use);
        if (S->active == 0) S->busy_since = Clock::now();
        ++S->active;
        S->waiting.pop_front();
        if (j->tick) { S->ready_tick.push_back(j); any_tick = true; }
        else { S->ready_big.push_back(j); any_big = true; }
    }
    if (any_big) S->cv_work.notify_all();
    if (any_tick) S->cv_tick.notify_all();
}

void release_out_locked(rplu_server_s* S, SJob* j) {
    if (j->out_held) {
        S->pool.give(j->out_off, j->out_bytes);
        S->in_use -= j->out_bytes;
        j->out_held = false;
    }
}

// With the lock held: a job finished (status and info set). Its work block
// goes back to the pool; its output block stays until rplu_server_release
// (or goes now when the run failed).
void finish_locked(rplu_server_s* S, SJob* j) {
    j->t_done = Clock::now();
    j->done = true;
    if (j->work_held) {
        S->pool.give(j->work_off, j->work_bytes);
        S->in_use -= j->work_bytes;
        j->work_held = false;
    }
    if (j->status < 0) release_out_locked(S, j);
    --S->active;
    ++S->completed;
    S->lat[j->cls].push_back(std::chrono::duration<double, std::milli>(j->t_done - j->t_submit).count());
    if (S->active == 0)
        S->busy_s += std::chrono::duration<double>(j->t_done - S->busy_since).count();
}

void set_info_done(SJob* j, int64_t rank, int stop, double a2, double r2) {
    j->info = rplu_info{};
    j->info.rank = rank;
    j->info.stop = stop;
    j->info.status = j->status;
    j->info.a_fro2 = a2;
    j->info.res_fro2 = r2;
    j->info.err_fro2 = -1.0;
    j->info.refreshes = j->refreshes;
    j->info.first_refresh = j->first_refresh;
}

// Device pointers of an admitted job inside its blocks.
void bind_job(rplu_server_s* S, SJob* j) {
    char* w = S->pool_base + j->work_off;
    const rplu_job& d = j->d;
    if (j->cls == CLS_DENSE) {
        j->S = w + j->o_S + ((uintptr_t)d.A % 16);
    } else {
        j->S = w + j->o_S;
        j->Bw = w + j->o_B;
    }
    if (j->own_out) {
        char* o = S->pool_base + j->out_off;
        j->piv = (int32_t*)(o + j->o_piv);
        j->L = o + j->o_L;
        j->U = o + j->o_U;
        j->ldl = d.n;
        j->ldu = d.m;
    } else {
        j->piv = d.piv;
        j->L = d.L;
        j->U = d.U;
        j->ldl = d.ldl;
        j->ldu = d.ldu;
    }
}

// The job's inputs into its work block on stream s, after the submitter's
// ready event (if any).
hipError_t copy_inputs(const SJob* j, hipStream_t s) {
    const rplu_job& d = j->d;
    hipError_t e = hipSuccess;
    if (d.ready_event) e = hipStreamWaitEvent(s, (hipEvent_t)d.ready_event, 0);
    if (e != hipSuccess) return e;
    if (j->cls == CLS_DENSE) {
        const size_t pitch = (size_t)d.lda * j->es;
        return hipMemcpy2DAsync(j->S, pitch, d.A, pitch, (size_t)d.m * j->es, (size_t)d.n,
                                hipMemcpyDeviceToDevice, s);
    }
    e = hipMemcpyAsync(j->S, d.G, (size_t)d.n * d.p * 16, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(j->Bw, d.B, (size_t)d.p * d.m * 16, hipMemcpyDeviceToDevice, s);
    return e;
}

// ||A - L U||^2 of a finished dense job into info.err_fro2 (enqueued on s;
// the caller synchronises and reads `host` afterwards).
hipError_t enqueue_certify(rplu_server_s* S, SJob* j, double* out_dev, hipStream_t s) {
    const rplu_job& d = j->d;
    VerifyArgs a;
    std::memset(&a, 0, sizeof a);
    a.dtype = d.dtype;
    a.n = d.n;
    a.m = d.m;
    a.k = j->info.rank;
    a.A = d.A;
    a.lda = d.lda;
    a.L = j->L;
    a.ldl = j->ldl;
    a.U = j->U;
    a.ldu = j->ldu;
    a.partial = (double*)(S->pool_base + j->work_off + j->o_vf);
    a.out = out_dev;
    launch_verify(a, s);
    return hipGetLastError();
}

// -------------------------------------------------------------- workers

void run_single(rplu_server_s* S, Worker& W, SJob* j) {
    const rplu_job& d = j->d;
    hipStream_t s = W.stream;
    hipError_t e = copy_inputs(j, s);
    if (e != hipSuccess) { j->status = hip_fail(e, "server: input copy"); return; }
    rplu_opts o;
    std::memset(&o, 0, sizeof o);
    o.max_rank = d.max_rank;
    o.rel_tol = d.rel_tol;
    o.seed = d.seed;
    o.stream = d.stream;
    o.flags = RPLU_FLAG_NO_GRAPH | (d.flags & (RPLU_FLAG_STALL_STOP | RPLU_FLAG_REFRESH));
    char* ws = S->pool_base + j->work_off + j->o_ws;
    if (j->cls == CLS_DENSE) {
        o.A_orig = d.A;
        o.lda_orig = d.lda;
        j->status = dense_run(W.ctx, ws, d.dtype, d.n, d.m, j->S, d.lda, &o, j->piv, j->L, j->ldl,
                              j->U, j->ldu, &j->info, s);
    } else {
        j->status = cauchy_run(W.ctx, ws, d.n, d.m, d.p, d.x, d.y, j->S, j->Bw, &o, j->piv, j->L,
                               j->ldl, j->U, j->ldu, &j->info, s);
    }
    j->info.status = j->status;
    j->refreshes = j->info.refreshes;
    j->first_refresh = j->info.first_refresh;
    if (j->status == RPLU_OK && j->certify) {
        double* od = (double*)(S->pool_base + j->work_off + j->o_vf) +
                     verify_tiles(d.n, d.m) * 3;
        double h[3] = {0, 0, 0};
        e = enqueue_certify(S, j, od, s);
        if (e == hipSuccess) e = hipMemcpyAsync(h, od, sizeof h, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) { j->status = hip_fail(e, "server: certification"); j->info.status = j->status; }
        else j->info.err_fro2 = h[1];
    }
}

void simulate_sleep(double bytes) {
    std::this_thread::sleep_for(std::chrono::duration<double>(bytes / 1e10));
}

void worker_main(rplu_server_s* S, int w) {
    Worker& W = S->workers[(size_t)w];
    if (!S->simulate) (void)hipSetDevice(S->device);
    for (;;) {
        SJob* j = nullptr;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_work.wait(lk, [&] { return S->stopping || !S->ready_big.empty(); });
            if (S->ready_big.empty()) return;      // stopping, and nothing left
            j = S->ready_big.front();
            S->ready_big.pop_front();
            bind_job(S, j);
        }
        if (S->simulate) {
            simulate_sleep((double)(j->work_bytes + j->out_bytes));
            j->status = RPLU_OK;
            set_info_done(j, j->kmax, RPLU_STOP_RANK, 0.0, 0.0);
        } else {
            run_single(S, W, j);
        }
        {
            std::lock_guard<std::mutex> lk(S->mu);
            finish_locked(S, j);
            admit_locked(S);
        }
        S->cv_idle.notify_all();
    }
}

// ----------------------------------------------------------- tick thread

// One tick over the resident jobs of one dtype: each runs from its step t
// until it stops or reaches t + tick_steps. Returns the jobs that finished.
void run_tick(rplu_server_s* S, int dtype, std::vector<SJob*>& res, std::vector<SJob*>& fin) {
    const int tick = S->cfg.tick_steps;
    std::vector<BatchJob> bj;
    std::vector<SJob*> who;
    for (SJob* j : res) {
        if (j->d.dtype != dtype) continue;
        rplu_job d = j->d;
        d.A_orig = j->d.A;                 // the caller's input is the original
        d.lda_orig = j->d.lda;
        d.A = j->S;
        d.piv = j->piv;
        d.L = j->L;
        d.ldl = j->ldl;
        d.U = j->U;
        d.ldu = j->ldu;
        BatchJob q;
        const rplu_status rc = batch_job_of(d, &q);
        if (rc) {
            j->status = rc;
            set_info_done(j, j->t, 0, j->T0, 0.0);
            fin.push_back(j);
            continue;
        }
        q.t0 = j->t;
        q.t_end = j->t + tick;
        q.T0_in = j->T0;
        q.Tbest_in = j->Tbest;
        q.tbest_in = j->tbest;
        q.Tref_in = j->Tref;
        q.refresh_on = (q.refresh_on && j->refreshes < RPLU_MAX_REFRESH) ? 1 : 0;
        bj.push_back(q);
        who.push_back(j);
    }
    if (bj.empty()) return;
    std::vector<BatchInfo> out;
    const rplu_batch_cfg cfg{4, 1, RPLU_ORDER_AREA, 0};
    const rplu_status rc = batch_launch_jobs(S->tick_ctx, dtype, bj, cfg, S->tick_stream, &out);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        ++S->ticks;
    }
    for (size_t q = 0; q < who.size(); ++q) {
        SJob* j = who[q];
        if (rc != RPLU_OK) {
            j->status = rc;
            set_info_done(j, j->t, 0, j->T0, 0.0);
            fin.push_back(j);
            continue;
        }
        const BatchInfo& o = out[q];
        if (o.error != 0) {
            j->status = o.error;
            set_info_done(j, o.rank, o.stop, o.a_fro2, o.res_fro2);
            fin.push_back(j);
        } else if ((o.stop == RPLU_STOP_STALL || o.stop == RPLU_STOP_REFRESH ||
                    (o.stop == RPLU_STOP_TOL && o.rank > j->t_refresh)) &&
                   (j->d.flags & RPLU_FLAG_REFRESH) && j->refreshes < RPLU_MAX_REFRESH &&
                   o.rank < bj[q].kmax) {
            // residual replacement, as rplu_dense does; the job stays resident
            RefreshArgs ra;
            std::memset(&ra, 0, sizeof ra);
            ra.dtype = dtype;
            ra.n = j->d.n;
            ra.m = j->d.m;
            ra.t = o.rank;
            ra.A = j->d.A;
            ra.lda = j->d.lda;
            ra.L = j->L;
            ra.ldl = j->ldl;
            ra.U = j->U;
            ra.ldu = j->ldu;
            ra.S = j->S;
            ra.lds = j->d.lda;
            ra.piv = j->piv;
            launch_refresh(ra, S->tick_stream);
            if (j->refreshes == 0) j->first_refresh = (int32_t)o.rank;
            j->t_refresh = (int32_t)o.rank;
            j->t = (int32_t)o.rank;
            j->T0 = o.a_fro2;
            j->Tbest = -1.0;
            j->tbest = j->t;
            j->Tref = -1.0;
            j->refreshes += 1;
            std::lock_guard<std::mutex> lk(S->mu);
            ++S->refreshes;
        } else if (o.stop != 0) {
            j->status = RPLU_OK;
            set_info_done(j, o.rank, o.stop, o.a_fro2, o.res_fro2);
            fin.push_back(j);
        } else {                                        // paused at t + tick
            j->t = (int32_t)o.rank;
            j->T0 = o.a_fro2;
            j->Tbest = o.T_best;
            j->tbest = o.t_best;
            j->Tref = o.T_ref;
        }
    }
}

void simulate_tick(rplu_server_s* S, std::vector<SJob*>& res, std::vector<SJob*>& fin) {
    double bytes = 0.0;
    for (SJob* j : res) {
        const int64_t steps = std::min<int64_t>(S->cfg.tick_steps, j->kmax - j->t);
        bytes += (double)(j->work_bytes + j->out_bytes) * (double)std::max<int64_t>(steps, 1) /
                 (double)std::max<int64_t>(j->kmax, 1);
        j->t += (int32_t)steps;
        if (j->t >= j->kmax) {
            j->status = RPLU_OK;
            set_info_done(j, j->kmax, RPLU_STOP_RANK, 0.0, 0.0);
            fin.push_back(j);
        }
    }
    simulate_sleep(bytes);
    std::lock_guard<std::mutex> lk(S->mu);
    ++S->ticks;
}

void tick_main(rplu_server_s* S) {
    if (!S->simulate) (void)hipSetDevice(S->device);
    std::vector<SJob*> res;
    for (;;) {
        std::vector<SJob*> incoming;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_tick.wait(lk, [&] {
                return S->stopping || !S->ready_tick.empty() || !res.empty();
            });
            if (S->ready_tick.empty() && res.empty()) return;   // stopping, nothing left
            incoming.assign(S->ready_tick.begin(), S->ready_tick.end());
            S->ready_tick.clear();
            for (SJob* j : incoming) bind_job(S, j);
        }
        std::vector<SJob*> fin;
        for (SJob* j : incoming) {
            if (!S->simulate) {
                const hipError_t e = copy_inputs(j, S->tick_stream);
                if (e != hipSuccess) {
                    j->status = hip_fail(e, "server: input copy");
                    set_info_done(j, 0, 0, 0.0, 0.0);
                    fin.push_back(j);
                    continue;
                }
            }
            j->started = true;
            res.push_back(j);
        }
        if (S->simulate) {
            simulate_tick(S, res, fin);
        } else {
            run_tick(S, RPLU_R32, res, fin);
            run_tick(S, RPLU_R64, res, fin);
            // certification of the finished jobs (one synchronisation)
            std::vector<double> h(fin.size() * 3, 0.0);
            hipError_t e = hipSuccess;
            for (size_t q = 0; q < fin.size() && e == hipSuccess; ++q) {
                SJob* j = fin[q];
                if (j->status != RPLU_OK || !j->certify) continue;
                double* od = (double*)(S->pool_base + j->work_off + j->o_vf) +
                             verify_tiles(j->d.n, j->d.m) * 3;
                e = enqueue_certify(S, j, od, S->tick_stream);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(&h[q * 3], od, 3 * sizeof(double), hipMemcpyDeviceToHost,
                                       S->tick_stream);
            }
            if (e == hipSuccess) e = hipStreamSynchronize(S->tick_stream);
            for (size_t q = 0; q < fin.size(); ++q) {
                SJob* j = fin[q];
                if (j->status != RPLU_OK || !j->certify) continue;
                if (e != hipSuccess) {
                    j->status = hip_fail(e, "server: certification");
                    j->info.status = j->status;
                } else {
                    j->info.err_fro2 = h[q * 3 + 1];
                }
            }
        }
        if (!fin.empty()) {
            std::lock_guard<std::mutex> lk(S->mu);
            for (SJob* j : fin) {
                auto it = std::find(res.begin(), res.end(), j);
                if (it != res.end()) res.erase(it);
                ++S->tick_jobs;
                finish_locked(S, j);
            }
            admit_locked(S);
        }
        if (!fin.empty()) S->cv_idle.notify_all();
    }
}

// ------------------------------------------------------------ submission

// Checks a job and lays out its blocks (footprint = work + output block).
rplu_status plan_job(const rplu_server_s* S, const rplu_job& d, SJob* j) {
    const bool own = d.piv == nullptr;
    if (own && (d.L != nullptr || d.U != nullptr))
        return fail(RPLU_E_ARG, "rplu_server_submit: with piv NULL (server-owned outputs) L and U "
                    "must be NULL too");
    j->own_out = own;
    const int64_t mn = std::min(d.n, d.m);
    if (d.kind == RPLU_JOB_DENSE) {
        const size_t es = dtype_size(d.dtype);
        if (es == 0) return fail(RPLU_E_ARG, "rplu_server_submit: unknown dtype %d", d.dtype);
        if (d.n < 1 || d.m < 1 || d.n > INT32_MAX || d.m > INT32_MAX)
            return fail(RPLU_E_ARG, "rplu_server_submit: shape out of range");
        if (d.A == nullptr || d.lda < d.m)
            return fail(RPLU_E_ARG, "rplu_server_submit: A and lda >= m are required");
        if (!own && ((d.L && d.ldl < d.n) || (d.U && d.ldu < d.m)))
            return fail(RPLU_E_ARG, "rplu_server_submit: ldl < n or ldu < m");
        j->es = es;
        j->cls = CLS_DENSE;
        const int64_t bmax = S->cfg.batch_max_dim;
        j->tick = (d.dtype == RPLU_R32 || d.dtype == RPLU_R64) && d.n <= bmax && d.m <= bmax;
        const bool real = d.dtype == RPLU_R32 || d.dtype == RPLU_R64;
        const bool has_lu = own || (d.L != nullptr && d.U != nullptr);
        if ((d.flags & (RPLU_FLAG_REFRESH | RPLU_FLAG_CERTIFY)) && (!real || !has_lu))
            return fail(RPLU_E_ARG, "rplu_server_submit: RPLU_FLAG_REFRESH and RPLU_FLAG_CERTIFY "
                        "need a real dtype (R32, R64) and L and U");
        j->certify = (d.flags & RPLU_FLAG_CERTIFY) != 0;
        size_t off = 0;
        j->o_S = off;
        off = rup(off + (size_t)d.n * d.lda * es + 16, 256);
        if (!j->tick) {
            j->o_ws = off;
            const bool need_u = !own && d.U == nullptr;
            off = rup(off + dense_ws_layout(d.dtype, d.n, d.m, d.flags, need_u).total, 256);
        }
        if (j->certify) {
            j->o_vf = off;
            off = rup(off + ((size_t)verify_tiles(d.n, d.m) * 3 + 3) * 8, 256);
        }
        j->work_bytes = off;
    } else if (d.kind == RPLU_JOB_CAUCHY) {
        if (d.dtype != RPLU_C128) return fail(RPLU_E_UNSUPPORTED, "rplu_server_submit: Cauchy jobs are C128");
        if (d.n < 1 || d.m < 1 || d.n > INT32_MAX || d.m > INT32_MAX || d.p < 1 || d.p > 4)
            return fail(RPLU_E_ARG, "rplu_server_submit: Cauchy shape or p out of range");
        if (!d.x || !d.y || !d.G || !d.B)
            return fail(RPLU_E_ARG, "rplu_server_submit: x, y, G and B are required");
        if (!own && ((d.L && d.ldl < d.n) || (d.U && d.ldu < d.m)))
            return fail(RPLU_E_ARG, "rplu_server_submit: ldl < n or ldu < m");
        if (d.flags & (RPLU_FLAG_REFRESH | RPLU_FLAG_CERTIFY))
            return fail(RPLU_E_ARG, "rplu_server_submit: RPLU_FLAG_REFRESH and RPLU_FLAG_CERTIFY "
                        "are for dense jobs");
        j->es = 16;
        j->cls = CLS_CAUCHY;
        j->tick = false;
        size_t off = 0;
        j->o_S = off;
        off = rup(off + (size_t)d.n * d.p * 16, 256);
        j->o_B = off;
        off = rup(off + (size_t)d.p * d.m * 16, 256);
        j->o_ws = off;
        const bool need_u = !own && d.U == nullptr;
        off = rup(off + cauchy_ws_layout(S->mass_slots, d.n, d.m, d.p, d.flags, false, need_u).total, 256);
        j->work_bytes = off;
    } else {
        return fail(RPLU_E_ARG, "rplu_server_submit: unknown job kind %d", d.kind);
    }
    j->kmax = d.max_rank <= 0 ? mn : std::min<int64_t>(d.max_rank, mn);
    if (own) {
        size_t off = 0;
        j->o_piv = off;
        off = rup(off + (size_t)j->kmax * 2 * 4, 256);
        j->o_L = off;
        off = rup(off + (size_t)d.n * j->kmax * j->es, 256);
        j->o_U = off;
        off = rup(off + (size_t)j->kmax * d.m * j->es, 256);
        j->out_bytes = off;
    }
    if (!(d.rel_tol >= 0.0)) return fail(RPLU_E_ARG, "rplu_server_submit: rel_tol must be >= 0");
    if (d.flags & (RPLU_FLAG_C2PLU | RPLU_FLAG_CPLU))
        return fail(RPLU_E_ARG, "rplu_server_submit: RPLU_FLAG_C2PLU and RPLU_FLAG_CPLU are not served");
    if (j->work_bytes + j->out_bytes > S->pool_cap)
        return fail(RPLU_E_ARG, "rplu_server_submit: footprint %zu exceeds the pool (%zu bytes)",
                    j->work_bytes + j->out_bytes, S->pool_cap);
    return RPLU_OK;
}

void teardown(rplu_server_s* S) {
    for (Worker& W : S->workers) {
        if (W.stream) (void)hipStreamDestroy(W.stream);
        if (W.ctx) (void)rplu_destroy(W.ctx);
    }
    if (S->tick_stream) (void)hipStreamDestroy(S->tick_stream);
    if (S->tick_ctx) (void)rplu_destroy(S->tick_ctx);
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
    if (S->cfg.batch_max_dim > RPLU_BATCH_MAX_DIM) S->cfg.batch_max_dim = RPLU_BATCH_MAX_DIM;
    if (S->cfg.tick_steps <= 0) S->cfg.tick_steps = DEFAULT_TICK;
    S->simulate = sim;
    S->device = ctx ? ctx->device : 0;
    if (ctx) S->mass_slots = ctx->mass_slots;
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
            rplu_status rc = rplu_create(S->device, 0, &W.ctx);
            if (rc) { teardown(S); return rc; }
            hipError_t e = hipStreamCreateWithFlags(&W.stream, hipStreamNonBlocking);
            if (e != hipSuccess) { W.stream = nullptr; teardown(S); return hip_fail(e, "hipStreamCreateWithFlags"); }
        }
        rplu_status rc = rplu_create(S->device, 0, &S->tick_ctx);
        if (rc) { teardown(S); return rc; }
        hipError_t e = hipStreamCreateWithFlags(&S->tick_stream, hipStreamNonBlocking);
        if (e != hipSuccess) { S->tick_stream = nullptr; teardown(S); return hip_fail(e, "hipStreamCreateWithFlags"); }
    }
    for (int w = 0; w < S->cfg.workers; ++w) S->workers[(size_t)w].th = std::thread(worker_main, S, w);
    S->tick_th = std::thread(tick_main, S);
    *out = S;
    return RPLU_OK;
}

rplu_status rplu_server_submit(rplu_server S, const rplu_job* job, uint64_t* ticket) {
    if (S == nullptr || job == nullptr || ticket == nullptr)
        return fail(RPLU_E_ARG, "rplu_server_submit: NULL argument");
    SJob* j = new SJob();
    j->d = *job;
    rplu_status rc = plan_job(S, *job, j);
    if (rc) { delete j; return rc; }
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stopping) { delete j; return fail(RPLU_E_ARG, "rplu_server_submit: server is shutting down"); }
    if (S->cfg.queue_capacity > 0 && (int64_t)S->waiting.size() >= S->cfg.queue_capacity) {
        ++S->rejected;
        delete j;
        return fail(RPLU_E_BUSY, "rplu_server_submit: %zu jobs waiting", S->waiting.size());
    }
    j->ticket = S->next_ticket++;
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
    if (!j->own_out || st < 0) {
        release_out_locked(S, j);
        S->jobs.erase(it);
        delete j;
    }
    if (st < 0) return fail(st, "rplu_server_poll: job %llu failed", (unsigned long long)ticket);
    return st;
}

rplu_status rplu_server_outputs(rplu_server S, uint64_t ticket, int32_t** piv, void** L,
                                int64_t* ldl, void** U, int64_t* ldu) {
    if (S == nullptr) return fail(RPLU_E_ARG, "rplu_server_outputs: NULL server");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end())
        return fail(RPLU_E_ARG, "rplu_server_outputs: unknown ticket %llu", (unsigned long long)ticket);
    SJob* j = it->second;
    if (!j->done) return RPLU_PENDING;
    if (!j->own_out || !j->out_held)
        return fail(RPLU_E_ARG, "rplu_server_outputs: ticket %llu has no server-owned outputs",
                    (unsigned long long)ticket);
    if (piv) *piv = j->piv;
    if (L) *L = j->L;
    if (ldl) *ldl = j->ldl;
    if (U) *U = j->U;
    if (ldu) *ldu = j->ldu;
    return RPLU_OK;
}

rplu_status rplu_server_release(rplu_server S, uint64_t ticket) {
    if (S == nullptr) return fail(RPLU_E_ARG, "rplu_server_release: NULL server");
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->jobs.find(ticket);
        if (it == S->jobs.end())
            return fail(RPLU_E_ARG, "rplu_server_release: unknown ticket %llu", (unsigned long long)ticket);
        SJob* j = it->second;
        if (!j->done) return fail(RPLU_E_ARG, "rplu_server_release: ticket %llu is not done",
                                  (unsigned long long)ticket);
        release_out_locked(S, j);
        S->jobs.erase(it);
        delete j;
        admit_locked(S);
    }
    return RPLU_OK;
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
    out->hbm_peak = S->peak;
    out->ticks = S->ticks;
    out->tick_jobs = S->tick_jobs;
    out->refreshes = S->refreshes;
    return RPLU_OK;
}

rplu_status rplu_server_destroy(rplu_server S) {
    if (S == nullptr) return RPLU_OK;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        S->cv_idle.wait(lk, [&] {
            return S->waiting.empty() && S->ready_big.empty() && S->ready_tick.empty() &&
                   S->active == 0;
        });
        S->stopping = true;
    }
    S->cv_work.notify_all();
    S->cv_tick.notify_all();
    for (Worker& W : S->workers)
        if (W.th.joinable()) W.th.join();
    if (S->tick_th.joinable()) S->tick_th.join();
    teardown(S);
    return RPLU_OK;
}

}  // extern "C"
