// Serving loop of libmcdose: requests from any thread, admitted against the
// HBM budget, transported in epochs of the regrouped engine by one worker
// thread per context, finalised one by one as they complete.
//
// An epoch is one regrouped launch sequence over the admitted requests of one
// phantom (phantoms taken in turn).  Request r advances by a slice of its
// histories, [done_r, done_r + q_r), with its own seed, key and persistent
// batch-statistics tally; the histories it has already run are carried in the
// per-sub-tally counts.  Because every history draws from streams keyed by
// (seed, request key, history), a request's result does not depend on how its
// histories were sliced or which requests shared its epochs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "engine.h"
#include "mcdose.h"
#include "runtime.h"

using namespace mcd;
using Clock = std::chrono::steady_clock;

namespace {

struct Request {
    uint64_t ticket = 0;
    int32_t phantom = -1;
    mcd_source src{};
    uint64_t n = 0, done = 0;          // n: histories to run (adaptive: at most)
    double target = 0.0;               // adaptive: sigma-bar to reach (0: run all n)
    uint64_t next_check = 0;           // adaptive: finalise once done reaches it
    uint32_t seed = 0, key = 0;
    int state = MCD_QUEUED;
    int status = MCD_OK;
    std::string msg;
    bool cancel = false;
    bool admitting = false;          // the worker is allocating its memory
    // device memory (owned while admitted; dose and sigma until collected)
    void* tally = nullptr;
    size_t tally_bytes = 0;
    double* dose = nullptr;
    double* sigma = nullptr;
    size_t out_bytes = 0;
    double nb[kBatches] = {};        // histories already in each sub-tally
    double dmax = 0, sigma_bar = 0, kernel_ms = 0;
    Clock::time_point t_submit, t_done;
};

constexpr uint64_t kAdaptiveMin = 1000;   // histories before an adaptive request may stop

// Next checkpoint of an adaptive request that has run d histories with
// sigma-bar sb (Dmax > 0 when have_dose).  sigma-bar falls as N^-1/2, so the
// target is due near N* = d (sb / target)^2; the next finalisation comes at
// 95% of that, at most four times d, so a request is finalised a handful of
// times instead of after every epoch, and stops within one epoch slice of
// where a finalisation after every epoch would stop it.
uint64_t next_checkpoint(uint64_t d, double sb, double target, bool have_dose)
{
    if (d < kAdaptiveMin) return kAdaptiveMin;
    if (!have_dose || !(sb > 0.0)) return 2 * d;
    const double due = 0.95 * (double)d * (sb / target) * (sb / target);
    const double next = std::min(due, 4.0 * (double)d);
    return std::max<uint64_t>(d + 1, (uint64_t)next);
}

double ms_between(Clock::time_point a, Clock::time_point b)
{
    return std::chrono::duration<double, std::milli>(b - a).count();
}

}  // namespace

// An epoch on another phantom's requests passes a phantom over; after this
// many in a row its requests run next (shortest-remaining order).
constexpr int kMaxPassOver = 3;

struct mcd_server {
    std::mutex mu;
    std::condition_variable cv_work;  // worker: something to do
    std::condition_variable cv_done;  // waiters: a request ended
    std::thread worker;
    bool running = false, stop = false;
    hipStream_t stream = nullptr;
    mcd_serve_config cfg{};
    uint64_t next_ticket = 1;
    std::map<uint64_t, std::unique_ptr<Request>> reqs;  // every ticket not yet collected
    std::deque<Request*> pending;                        // QUEUED, in arrival order
    std::vector<Request*> active;                        // ADMITTED or RUNNING
    int last_phantom = -1;
    std::vector<int> passed;                             // epochs each phantom was passed over
    uint64_t req_bytes = 0;                              // memory held by requests
    bool mem_blocked = false;                            // the queue head waits for memory to be freed
    mcd_serve_stats stats{};
};

// ------------------------------------------------------------------ worker

static void free_request_memory(mcd_ctx* c, Request* r, bool outputs_too)
{
    mcd_server* S = c->server;
    {
        std::lock_guard<std::mutex> g(S->mu);
        S->req_bytes -= std::min<uint64_t>(S->req_bytes, r->tally_bytes + (outputs_too ? 2 * r->out_bytes : 0));
    }
    c->release(r->tally, r->tally_bytes);
    r->tally = nullptr;
    r->tally_bytes = 0;
    if (outputs_too) {
        c->release(r->dose, r->out_bytes);
        c->release(r->sigma, r->out_bytes);
        r->dose = r->sigma = nullptr;
        r->out_bytes = 0;
    }
    // a queued request may fit now
    std::lock_guard<std::mutex> g(S->mu);
    S->mem_blocked = false;
    S->cv_work.notify_one();
}

// Ends a request (under the server mutex).
static void end_request(mcd_server* S, Request* r, int state, int status, const std::string& msg)
{
    r->state = state;
    r->status = status;
    r->msg = msg;
    r->t_done = Clock::now();
    if (state == MCD_DONE) ++S->stats.completed;
    else if (state == MCD_FAILED) ++S->stats.failed;
    else if (state == MCD_CANCELED) ++S->stats.canceled;
    S->cv_done.notify_all();
}

// Admits queued requests in arrival order while their memory fits (run_mu held).
static void admit(mcd_ctx* c, mcd_server* S)
{
    const int max_active = S->cfg.max_active ? S->cfg.max_active : kMaxBatch;
    const int fp32 = S->cfg.opts.tally_fp32 ? 1 : 0;
    for (;;) {
        Request* r;
        {
            std::lock_guard<std::mutex> g(S->mu);
            while (!S->pending.empty() && S->pending.front()->cancel) {
                Request* x = S->pending.front();
                S->pending.pop_front();
                end_request(S, x, MCD_CANCELED, MCD_E_CANCELED, "request cancelled");
            }
            if (S->pending.empty() || (int)S->active.size() >= max_active) return;
            r = S->pending.front();
            r->admitting = true;         // from here a cancel only sets r->cancel
        }
        const PhantomRec& ph = c->phantoms[r->phantom];
        const size_t tb = (size_t)kBatches * (size_t)ph.nv * (fp32 ? sizeof(float) : sizeof(double));
        const size_t ob = (size_t)ph.nv * sizeof(double);
        // keep room for the lane stacks the epoch launches may still need
        int blocks = 0, threads = 0;
        const int depth = S->cfg.opts.stack_depth ? S->cfg.opts.stack_depth : kDefaultDepth;
        size_t reserve = (size_t)1 << 20;
        if (c->launch_shape(&S->cfg.opts, c->tables[ph.tables].n_mat, &blocks, &threads) == MCD_OK) {
            const uint64_t lanes = (uint64_t)blocks * threads;
            const size_t lanes_b =
                stack_scratch_bytes(lanes, depth, S->cfg.opts.regroup == 0 || S->cfg.opts.regroup == 3);
            if (lanes_b > c->rb.scratch_bytes) reserve += lanes_b - c->rb.scratch_bytes;
            if (S->cfg.opts.regroup == 1) {
                const int cpl = S->cfg.opts.chunk_per_lane ? S->cfg.opts.chunk_per_lane : kDefaultChunkPerLane;
                const unsigned int cap = queue_capacity(lanes * (uint64_t)cpl);
                if (cap > c->rb.cap) reserve += (size_t)4 * (cap - c->rb.cap) * kRec;
            }
        }
        // fits now, or only once other requests free their memory (the ones
        // running, and finished ones whose results are not collected yet)
        bool fits, never;
        {
            std::lock_guard<std::mutex> g(c->mu_alloc);
            std::lock_guard<std::mutex> g2(S->mu);
            const uint64_t need = tb + 2 * ob;
            const uint64_t others = c->used - std::min<uint64_t>(c->used, S->req_bytes);
            fits = c->used + need + reserve <= c->budget &&
                   (!S->cfg.memory_limit || S->req_bytes + need <= S->cfg.memory_limit);
            never = others + need + reserve > c->budget || (S->cfg.memory_limit && need > S->cfg.memory_limit);
        }
        int rc = MCD_E_NOMEM;
        std::string why = "request needs more device memory than the HBM budget or the serving memory limit";
        if (fits) {
            rc = c->alloc(&r->tally, tb, "request tally");
            if (rc == MCD_OK) r->tally_bytes = tb;
            if (rc == MCD_OK) rc = c->alloc((void**)&r->dose, ob, "request dose");
            if (rc == MCD_OK) rc = c->alloc((void**)&r->sigma, ob, "request sigma");
            if (rc == MCD_OK) {
                r->out_bytes = ob;
                hipError_t e = launch_fill_u32(r->tally, tb / 4, 0u, S->stream);
                if (e != hipSuccess) rc = c->hip_fail(e, "tally clear");
            }
            if (rc != MCD_OK) {
                why = c->last_error();
                c->release(r->tally, tb);
                c->release(r->dose, ob);
                c->release(r->sigma, ob);
                r->tally = r->dose = r->sigma = nullptr;
                r->tally_bytes = 0;
            }
        }
        bool cancelled;
        {
            std::lock_guard<std::mutex> g(S->mu);
            r->admitting = false;
            cancelled = r->cancel;
            if (rc == MCD_OK) S->req_bytes += tb + 2 * ob;
            if (rc == MCD_OK && !cancelled) {
                S->pending.pop_front();
                r->state = MCD_ADMITTED;
                r->out_bytes = ob;
                S->active.push_back(r);
                continue;
            }
            if (!cancelled && !never && rc == MCD_E_NOMEM && !fits) {
                // wait for memory: epochs of the active requests free theirs,
                // collecting finished requests frees theirs
                if (S->active.empty()) S->mem_blocked = true;
                return;
            }
            S->pending.pop_front();
            if (!cancelled) {                                // can never fit
                end_request(S, r, MCD_FAILED, MCD_E_NOMEM, why);
                continue;
            }
        }
        r->out_bytes = ob;
        free_request_memory(c, r, true);
        std::lock_guard<std::mutex> g(S->mu);
        end_request(S, r, MCD_CANCELED, MCD_E_CANCELED, "request cancelled");
    }
}

// Runs one epoch over the admitted requests of the next phantom (run_mu held).
static void run_epoch(mcd_ctx* c, mcd_server* S)
{
    std::vector<Request*> batch;
    std::vector<Request*> dropped;
    {
        std::lock_guard<std::mutex> g(S->mu);
        std::vector<Request*> keep;
        for (Request* r : S->active) (r->cancel ? dropped : keep).push_back(r);
        S->active.swap(keep);
        if (!S->active.empty()) {
            int pick = -1;
            if (S->cfg.phantom_order == MCD_PHANTOMS_IN_TURN) {
                // next phantom in turn that has admitted requests
                for (Request* r : S->active)
                    if (r->phantom > S->last_phantom && (pick < 0 || r->phantom < pick)) pick = r->phantom;
                if (pick < 0)
                    for (Request* r : S->active)
                        if (pick < 0 || r->phantom < pick) pick = r->phantom;
            } else {
                // the phantom passed over longest once that reaches kMaxPassOver
                // epochs, else the one holding the request with the fewest
                // histories left (ties: the lower handle)
                if (S->passed.size() < c->phantoms.size()) S->passed.resize(c->phantoms.size(), 0);
                int starved = -1;
                uint64_t fewest = 0;
                for (Request* r : S->active) {
                    const int p = r->phantom;
                    if (S->passed[p] >= kMaxPassOver &&
                        (starved < 0 || S->passed[p] > S->passed[starved] ||
                         (S->passed[p] == S->passed[starved] && p < starved)))
                        starved = p;
                    const uint64_t left = r->n - r->done;
                    if (pick < 0 || left < fewest || (left == fewest && p < pick)) {
                        pick = p;
                        fewest = left;
                    }
                }
                if (starved >= 0) pick = starved;
                // every other phantom with admitted requests waits one more epoch
                std::vector<char> waits(S->passed.size(), 0);
                for (Request* r : S->active) waits[r->phantom] = r->phantom != pick;
                for (size_t p = 0; p < waits.size(); ++p) S->passed[p] = waits[p] ? S->passed[p] + 1 : 0;
            }
            S->last_phantom = pick;
            for (Request* r : S->active)
                if (r->phantom == pick && (int)batch.size() < kMaxBatch) batch.push_back(r);
            for (Request* r : batch) r->state = MCD_RUNNING;
        }
    }
    // dropped requests left the active list but have not ended, so no waiter
    // can collect them while their memory is freed
    for (Request* r : dropped) free_request_memory(c, r, true);
    if (!dropped.empty()) {
        std::lock_guard<std::mutex> g(S->mu);
        for (Request* r : dropped) end_request(S, r, MCD_CANCELED, MCD_E_CANCELED, "request cancelled");
    }
    if (batch.empty()) return;

    // Slices: the requests closest to completion finish first, the rest share
    // what is left of the epoch evenly (water filling).
    const PhantomRec& ph = c->phantoms[batch[0]->phantom];
    uint64_t budget = S->cfg.epoch_histories;
    if (!budget) {
        int blocks = 0, threads = 0;
        if (c->launch_shape(&S->cfg.opts, c->tables[ph.tables].n_mat, &blocks, &threads) != MCD_OK)
            blocks = threads = 1;
        const int cpl = S->cfg.opts.chunk_per_lane ? S->cfg.opts.chunk_per_lane : kDefaultChunkPerLane;
        // four cycles' worth: each epoch ends with a tail in which few waves
        // are busy, so short epochs pay more tails, and long ones hold small
        // requests back (on the 20 req/s mixed stream half this size raised
        // p50 by 8% and p99 by 10%, twice this size p99 by 4%)
        budget = 4 * (uint64_t)blocks * threads * (uint64_t)cpl;
    }
    std::sort(batch.begin(), batch.end(),
              [](const Request* a, const Request* b) { return a->n - a->done < b->n - b->done; });
    const size_t n = batch.size();
    std::vector<uint64_t> slice(n);
    uint64_t left = std::max<uint64_t>(budget, n);
    for (size_t i = 0; i < n; ++i) {
        const uint64_t share = std::max<uint64_t>(left / (n - i), 1);
        slice[i] = std::min(batch[i]->n - batch[i]->done, share);
        left -= std::min(left, slice[i]);
    }
    // requests finalised after the epoch first: those that finish, and the
    // adaptive ones (their sigma-bar decides whether they finish)
    std::vector<size_t> order(n);
    for (size_t i = 0; i < n; ++i) order[i] = i;
    auto finalised = [&](size_t i) {
        const Request* r = batch[i];
        return r->done + slice[i] == r->n || (r->target > 0.0 && r->done + slice[i] >= r->next_check);
    };
    std::stable_partition(order.begin(), order.end(), finalised);
    std::vector<const mcd_source*> srcs(n);
    std::vector<uint64_t> ns(n);
    std::vector<uint32_t> keys(n);
    std::vector<ReqExtra> extra(n);
    std::vector<Request*> rq(n);
    int n_fin = 0;
    for (size_t j = 0; j < n; ++j) {
        Request* r = batch[order[j]];
        rq[j] = r;
        srcs[j] = &r->src;
        ns[j] = slice[order[j]];
        keys[j] = r->key;
        extra[j].first = r->done;
        extra[j].seed = r->seed;
        extra[j].tally = r->tally;
        extra[j].dose = r->dose;
        extra[j].sigma = r->sigma;
        extra[j].nb_prior = r->nb;
        if (finalised(order[j])) ++n_fin;
    }
    mcd_opts o = S->cfg.opts;
    RegroupPlan plan;
    int rc = c->plan_regroup(rq[0]->phantom, srcs.data(), ns.data(), keys.data(), (int)n, 0, &o, false,
                             plan, extra.data());
    std::vector<double> red;
    unsigned char small[kSmallBytes];
    float kms = 0.f, tms = 0.f;
    if (rc == MCD_OK) {
        plan.n_fin = n_fin;
        for (auto& f : plan.fin) f.S = nullptr;
        rc = run_regroup(c, plan, false, false, S->stream);
    }
    if (rc == MCD_OK) {
        red.resize((size_t)3 * std::max(n_fin, 1));
        hipError_t e = hipMemcpyAsync(small, c->small, kSmallBytes, hipMemcpyDeviceToHost, S->stream);
        if (e == hipSuccess && n_fin)
            e = hipMemcpyAsync(red.data(), c->rb.red, (size_t)3 * n_fin * sizeof(double),
                               hipMemcpyDeviceToHost, S->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(S->stream);
        if (e != hipSuccess) rc = c->hip_fail(e, "epoch results");
        (void)hipEventElapsedTime(&kms, c->ev[1], c->ev[2]);
        (void)hipEventElapsedTime(&tms, c->ev[0], c->ev[3]);
    }
    if (rc != MCD_OK) {
        const std::string why = c->last_error();
        for (Request* r : rq) free_request_memory(c, r, true);
        std::lock_guard<std::mutex> g(S->mu);
        std::vector<Request*> keep;
        for (Request* r : S->active)
            if (std::find(rq.begin(), rq.end(), r) == rq.end()) keep.push_back(r);
        S->active.swap(keep);
        for (Request* r : rq) end_request(S, r, MCD_FAILED, rc, "serving epoch: " + why);
        return;
    }
    // which requests end with this epoch: all their histories ran, or the
    // adaptive ones reached their sigma-bar (only the worker writes done and n)
    std::vector<char> ends(n, 0);
    for (int j = 0; j < n_fin; ++j) {
        const Request* r = rq[j];
        const uint64_t d = r->done + ns[j];
        const double dmax = red[3 * j];
        const double sb = red[3 * j + 2] > 0 ? red[3 * j + 1] / red[3 * j + 2] : 0.0;
        ends[j] = d == r->n || (r->target > 0.0 && d >= kAdaptiveMin && dmax > 0.0 && sb <= r->target);
    }
    for (int j = 0; j < n_fin; ++j)
        if (ends[j]) free_request_memory(c, rq[j], false);
    std::lock_guard<std::mutex> g(S->mu);
    double bal[kBal];
    std::memcpy(bal, small + kOffBal, sizeof bal);
    mcd_energy_balance& eb = S->stats.eb;
    eb.e_src += bal[0];
    eb.e_csda += bal[1];
    eb.e_local += bal[2];
    eb.e_esc += bal[3];
    eb.e_miss += bal[4];
    eb.track_e += bal[5];
    uint64_t cnt[MCD_NCOUNT];
    std::memcpy(cnt, small + kOffCnt, sizeof cnt);
    for (int i = 0; i < MCD_NCOUNT; ++i)
        S->stats.counters[i] = i == MCD_C_MAX_STACK ? std::max(S->stats.counters[i], cnt[i])
                                                    : S->stats.counters[i] + cnt[i];
    ++S->stats.epochs;
    S->stats.busy_ms += tms;
    S->stats.kernel_ms += kms;
    for (size_t j = 0; j < n; ++j) {
        Request* r = rq[j];
        for (int b = 0; b < kBatches; ++b) r->nb[b] = plan.fin[j].nb[b];
        r->done += ns[j];
        r->kernel_ms += kms;
        S->stats.histories += ns[j];
        if ((int)j < n_fin) {
            r->dmax = red[3 * j];
            r->sigma_bar = red[3 * j + 2] > 0 ? red[3 * j + 1] / red[3 * j + 2] : 0.0;
            if (r->target > 0.0)
                r->next_check = next_checkpoint(r->done, r->sigma_bar, r->target, r->dmax > 0.0);
        }
        if (ends[j]) end_request(S, r, MCD_DONE, MCD_OK, "");
        else r->state = MCD_ADMITTED;
    }
    std::vector<Request*> keep;
    for (Request* r : S->active)
        if (r->state != MCD_DONE) keep.push_back(r);
    S->active.swap(keep);
}

static void serve_loop(mcd_ctx* c)
{
    mcd_server* S = c->server;
    (void)hipSetDevice(c->device);
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_work.wait(lk, [S] {
                return S->stop || !S->active.empty() || (!S->pending.empty() && !S->mem_blocked);
            });
            if (S->stop) return;
        }
        std::lock_guard<mcd::FairMutex> run(c->run_mu);
        admit(c, S);
        run_epoch(c, S);
    }
}

// ------------------------------------------------------------------ public

static mcd_server* server_of(mcd_ctx* c)
{
    std::lock_guard<std::mutex> g(c->mu);
    if (!c->server) c->server = new (std::nothrow) mcd_server();
    return c->server;
}

static int check_config(mcd_ctx* c, const mcd_serve_config* cfg)
{
    const mcd_opts& o = cfg->opts;
    if (o.first_history || o.accumulate || o.history_records || o.lockstep || o.use_graph ||
        o.kernel != MCD_KERNEL_REGROUPED || o.tally_slots)
        return c->fail(MCD_E_INVAL, "serve config: first_history, accumulate, history_records, lockstep, "
                                    "use_graph and tally_slots must be 0 and kernel regrouped");
    if (o.regroup < 0 || o.regroup > 3) return c->fail(MCD_E_INVAL, "serve config: regroup must be 0 to 3");
    if (o.stack_depth && (o.stack_depth < 4 || o.stack_depth > 4096))
        return c->fail(MCD_E_INVAL, "serve config: stack_depth in [4, 4096]");
    if (o.chunk_per_lane < 0 || o.chunk_per_lane > 4096)
        return c->fail(MCD_E_INVAL, "serve config: chunk_per_lane in [0, 4096]");
    if (cfg->max_active < 0 || cfg->max_active > kMaxBatch)
        return c->fail(MCD_E_INVAL, "serve config: max_active in [0, 4096]");
    if (cfg->epoch_histories >= ((uint64_t)1 << 40))
        return c->fail(MCD_E_INVAL, "serve config: epoch_histories < 2^40");
    if (cfg->phantom_order != MCD_PHANTOMS_SHORTEST && cfg->phantom_order != MCD_PHANTOMS_IN_TURN)
        return c->fail(MCD_E_INVAL, "serve config: phantom_order must be MCD_PHANTOMS_SHORTEST or _IN_TURN");
    mcd::Sched sc;
    int rc = c->wave_schedule(&o, &sc, mcd::kSchedWavePhotonSources);   // thresholds in range
    if (rc) return rc;
    int b = 0, t = 0;
    return c->launch_shape(&o, 1, &b, &t);
}

int mcd_serve_configure(mcd_ctx* c, const mcd_serve_config* cfg)
{
    if (!c) return MCD_E_INVAL;
    mcd_serve_config z{};
    if (!cfg) cfg = &z;
    int rc = check_config(c, cfg);
    if (rc) return rc;
    mcd_server* S = server_of(c);
    if (!S) return c->fail(MCD_E_NOMEM, "server state");
    std::lock_guard<std::mutex> g(S->mu);
    if (!S->reqs.empty())
        return c->fail(MCD_E_BUSY, "submitted requests are not all collected");
    S->cfg = *cfg;
    return MCD_OK;
}

static int submit(mcd_ctx* c, int32_t phantom, const mcd_source* src, uint64_t n_histories, double target,
                  uint64_t seed, uint32_t request_key, uint64_t* out_ticket)
{
    DevSource ds;
    int rc = c->validate_source(src, &ds);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> g(c->mu);
        if (phantom < 0 || phantom >= (int32_t)c->phantoms.size() || !c->phantoms[phantom].live)
            return c->fail(MCD_E_NOTFOUND, "unknown phantom handle");
    }
    mcd_server* S = server_of(c);
    if (!S) return c->fail(MCD_E_NOMEM, "server state");
    auto r = std::unique_ptr<Request>(new (std::nothrow) Request());
    if (!r) return c->fail(MCD_E_NOMEM, "request record");
    r->phantom = phantom;
    r->src = *src;
    r->n = n_histories;
    r->target = target;
    r->seed = (uint32_t)seed;
    r->key = request_key;
    r->t_submit = Clock::now();
    std::lock_guard<std::mutex> g(S->mu);
    if (S->stop) return c->fail(MCD_E_INVAL, "context is shutting down");
    if (!S->running) {
        mcd::DeviceGuard dg(c->device);
        if (hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess)
            return c->fail(MCD_E_DEVICE, "serving stream");
        try {
            S->worker = std::thread(serve_loop, c);
        } catch (...) {
            (void)hipStreamDestroy(S->stream);
            S->stream = nullptr;
            return c->fail(MCD_E_NOMEM, "serving thread");
        }
        S->running = true;
    }
    r->ticket = S->next_ticket++;
    *out_ticket = r->ticket;
    S->pending.push_back(r.get());
    S->reqs.emplace(r->ticket, std::move(r));
    ++S->stats.submitted;
    S->cv_work.notify_one();
    return MCD_OK;
}

int mcd_submit(mcd_ctx* c, int32_t phantom, const mcd_source* src, uint64_t n_histories,
               uint64_t seed, uint32_t request_key, uint64_t* out_ticket)
{
    if (!c || !src || !out_ticket) return MCD_E_INVAL;
    if (n_histories < 2 || n_histories >= ((uint64_t)1 << 32) || seed >= ((uint64_t)1 << 32))
        return c->fail(MCD_E_INVAL, "need 2 <= n_histories < 2^32 and seed < 2^32");
    return submit(c, phantom, src, n_histories, 0.0, seed, request_key, out_ticket);
}

int mcd_submit_adaptive(mcd_ctx* c, int32_t phantom, const mcd_source* src, double sigma_bar_target,
                        uint64_t n_max, uint64_t seed, uint32_t request_key, uint64_t* out_ticket)
{
    if (!c || !src || !out_ticket) return MCD_E_INVAL;
    if (!(sigma_bar_target > 0.0 && sigma_bar_target < 1.0))
        return c->fail(MCD_E_INVAL, "need 0 < sigma_bar_target < 1");
    if (n_max < kAdaptiveMin || n_max >= ((uint64_t)1 << 32) || seed >= ((uint64_t)1 << 32))
        return c->fail(MCD_E_INVAL, "need 1000 <= n_max < 2^32 and seed < 2^32");
    return submit(c, phantom, src, n_max, sigma_bar_target, seed, request_key, out_ticket);
}

int mcd_poll(mcd_ctx* c, uint64_t ticket, int32_t* state, uint64_t* histories_done)
{
    if (!c) return MCD_E_INVAL;
    mcd_server* S = server_of(c);
    if (!S) return c->fail(MCD_E_NOMEM, "server state");
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return c->fail(MCD_E_NOTFOUND, "unknown or collected ticket");
    if (state) *state = it->second->state;
    if (histories_done) *histories_done = it->second->done;
    return MCD_OK;
}

int mcd_cancel(mcd_ctx* c, uint64_t ticket)
{
    if (!c) return MCD_E_INVAL;
    mcd_server* S = server_of(c);
    if (!S) return c->fail(MCD_E_NOMEM, "server state");
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return c->fail(MCD_E_NOTFOUND, "unknown or collected ticket");
    Request* r = it->second.get();
    if (r->state == MCD_QUEUED && !r->admitting) {
        S->pending.erase(std::find(S->pending.begin(), S->pending.end(), r));
        end_request(S, r, MCD_CANCELED, MCD_E_CANCELED, "request cancelled");
        S->mem_blocked = false;              // the next request may fit
        S->cv_work.notify_one();
    } else if (r->state == MCD_QUEUED || r->state == MCD_ADMITTED || r->state == MCD_RUNNING) {
        r->cancel = true;
        S->cv_work.notify_one();
    }
    return MCD_OK;
}

int mcd_wait(mcd_ctx* c, uint64_t ticket, mcd_result* out, int64_t timeout_ms)
{
    if (!c) return MCD_E_INVAL;
    mcd_server* S = server_of(c);
    if (!S) return c->fail(MCD_E_NOMEM, "server state");
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->reqs.find(ticket) == S->reqs.end()) return c->fail(MCD_E_NOTFOUND, "unknown or collected ticket");
    // the predicate looks the ticket up again: another waiter may collect it
    auto ended = [S, ticket] {
        auto i = S->reqs.find(ticket);
        if (i == S->reqs.end()) return true;
        const int st = i->second->state;
        return st == MCD_DONE || st == MCD_FAILED || st == MCD_CANCELED;
    };
    if (timeout_ms < 0) {
        S->cv_done.wait(lk, ended);
    } else if (!S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ended)) {
        return c->fail(MCD_E_BUSY, "request not finished");
    }
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return c->fail(MCD_E_NOTFOUND, "ticket collected by another waiter");
    Request* r = it->second.get();
    std::unique_ptr<Request> own = std::move(it->second);
    S->reqs.erase(it);
    lk.unlock();
    int rc = r->status;
    if (r->state == MCD_DONE && out) {
        const hipMemcpyKind k = out->on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        mcd::DeviceGuard dg(c->device);
        hipError_t e = hipSuccess;
        if (out->dose) e = hipMemcpy(out->dose, r->dose, r->out_bytes, k);
        if (e == hipSuccess && out->sigma) e = hipMemcpy(out->sigma, r->sigma, r->out_bytes, k);
        if (e != hipSuccess) rc = c->hip_fail(e, "result copy");
        out->dmax = r->dmax;
        out->sigma_bar = r->sigma_bar;
        out->kernel_ms = r->kernel_ms;
        out->total_ms = ms_between(r->t_submit, r->t_done);
        out->n_histories = r->done;
    } else if (rc != MCD_OK) {
        c->fail(rc, r->msg);
    }
    free_request_memory(c, r, true);
    return rc;
}

int mcd_serve_stats_get(mcd_ctx* c, mcd_serve_stats* out)
{
    if (!c || !out) return MCD_E_INVAL;
    mcd_server* S = server_of(c);
    if (!S) return c->fail(MCD_E_NOMEM, "server state");
    std::lock_guard<std::mutex> g(S->mu);
    *out = S->stats;
    out->queued = S->pending.size();
    out->active = S->active.size();
    out->request_bytes = S->req_bytes;
    std::lock_guard<std::mutex> ga(c->mu_alloc);
    out->hbm_used = c->used;
    out->hbm_budget = c->budget;
    return MCD_OK;
}

bool mcd_ctx::serving_uses(int32_t phantom)
{
    if (!server) return false;
    std::lock_guard<std::mutex> g(server->mu);
    // every request on the phantom counts until mcd_wait collects it, so that
    // whether an unload is refused does not depend on how far the device got
    for (auto& kv : server->reqs)
        if (kv.second->phantom == phantom) return true;
    return false;
}

void mcd_ctx::shutdown_serving()
{
    mcd_server* S = server;
    if (!S) return;
    {
        std::lock_guard<std::mutex> g(S->mu);
        S->stop = true;
        S->cv_work.notify_all();
    }
    if (S->worker.joinable()) S->worker.join();
    for (auto& kv : S->reqs) free_request_memory(this, kv.second.get(), true);
    if (S->stream) (void)hipStreamDestroy(S->stream);
    delete S;
    server = nullptr;
}
