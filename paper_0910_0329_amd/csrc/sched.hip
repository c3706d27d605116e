// Launch scheduling of libmcdose: the plain per-history path and the
// regrouped photon/electron cycle engine shared by mcd_simulate,
// mcd_simulate_batch and the serving loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "engine.h"
#include "mcdose.h"
#include "runtime.h"

using namespace mcd;

// ------------------------------------------------------------------ common

int mcd_ctx::launch_shape(const mcd_opts* o, int n_mat, int* blocks, int* threads, bool* gtab_out,
                          int* resident_out)
{
    int t = o && o->block_size ? o->block_size : kDefaultBlock;
    if (t < 64 || t > 512 || (t & 63))
        return fail(MCD_E_INVAL, "opts: block_size must be a multiple of 64 in [64, 512]");
    int b = o && o->grid_blocks ? o->grid_blocks : 0;
    if (b < 0 || b > 1 << 20) return fail(MCD_E_INVAL, "opts: grid_blocks must be in [0, 2^20]");
    const int place = o ? o->table_placement : MCD_TABLES_AUTO;
    if (place < MCD_TABLES_AUTO || place > MCD_TABLES_GLOBAL)
        return fail(MCD_E_INVAL, "opts: table_placement must be MCD_TABLES_AUTO, _LDS or _GLOBAL");
    // the wave-stack schedule of the regrouped kernel (regroup 0 or 3)
    const bool wave = (!o || o->kernel == MCD_KERNEL_REGROUPED) && (!o || o->regroup == 0 || o->regroup == 3);
    if (place == MCD_TABLES_GLOBAL && !wave)
        return fail(MCD_E_INVAL, "opts: table_placement MCD_TABLES_GLOBAL needs the wave-stack schedule "
                                 "(regrouped kernel, regroup 0 or 3)");
    bool gtab = place == MCD_TABLES_GLOBAL;
    // workgroups a CU holds at once: for the wave-stack kernel from its
    // registers and LDS (either table placement), else from the LDS alone
    int per_cu = 0;
    if (wave) {
        mcd::DeviceGuard dg(device);
        const int in_lds = transport_lds_bytes(n_mat) <= max_lds ? wave_blocks_per_cu(t, n_mat, false) : 0;
        const int in_mem = wave_blocks_per_cu(t, n_mat, true);
        // automatic: device-memory tables only where the LDS copy costs workgroups
        if (place == MCD_TABLES_AUTO) gtab = in_mem > in_lds;
        per_cu = gtab ? in_mem : in_lds;
    }
    const int lds = wave ? wave_lds_bytes(n_mat, gtab) : transport_lds_bytes(n_mat);
    if (lds > max_lds)
        return fail(MCD_E_INVAL, "tables need " + std::to_string(lds) +
                                     " bytes of LDS per workgroup; the device allows " +
                                     std::to_string(max_lds));
    if (b == 0) b = cu_count * (per_cu > 0 ? per_cu : std::max(1, std::min(kLdsPerCu / lds, 2048 / t)));
    *blocks = b;
    *threads = t;
    if (gtab_out) *gtab_out = gtab;
    if (resident_out) *resident_out = per_cu;
    return MCD_OK;
}

int mcd_launch_shape(mcd_ctx* c, int32_t phantom, const mcd_opts* opts, int32_t* grid_blocks,
                     int32_t* block_size, int32_t* cu_count, int32_t* resident_per_cu,
                     int32_t* table_placement)
{
    if (!c) return MCD_E_INVAL;
    if (!grid_blocks || !block_size || !cu_count || !resident_per_cu || !table_placement)
        return c->fail(MCD_E_INVAL, "launch_shape: null output");
    std::lock_guard<mcd::FairMutex> run_lock(c->run_mu);
    if (phantom < 0 || phantom >= (int32_t)c->phantoms.size() || !c->phantoms[phantom].live)
        return c->fail(MCD_E_NOTFOUND, "unknown phantom handle");
    int b = 0, t = 0, per_cu = 0;
    bool gtab = false;
    const int rc = c->launch_shape(opts, c->tables[c->phantoms[phantom].tables].n_mat, &b, &t, &gtab, &per_cu);
    if (rc) return rc;
    *grid_blocks = b;
    *block_size = t;
    *cu_count = c->cu_count;
    *resident_per_cu = per_cu;
    *table_placement = gtab ? MCD_TABLES_GLOBAL : MCD_TABLES_LDS;
    return MCD_OK;
}

int mcd_ctx::wave_schedule(const mcd_opts* o, Sched* sc, SchedDefaults d)
{
    sc->fetch_div = o && o->sched_fetch_div ? o->sched_fetch_div : d.fetch_div;
    sc->hard_div = o && o->sched_hard_div ? o->sched_hard_div : d.hard_div;
    sc->photon_div = o && o->sched_photon_div ? o->sched_photon_div : d.photon_div;
    sc->fetch_photon_div = o && o->sched_fetch_photon_div ? o->sched_fetch_photon_div : d.fetch_photon_div;
    sc->segments = o && o->sched_segments ? o->sched_segments : d.segments;
    if (sc->fetch_div < 1 || sc->fetch_div > 64 || sc->hard_div < 1 || sc->hard_div > 64 ||
        sc->photon_div < 1 || sc->photon_div > 64 || sc->fetch_photon_div < 1 || sc->fetch_photon_div > 64 ||
        sc->segments < 1 || sc->segments > 64)
        return fail(MCD_E_INVAL, "opts: sched_fetch_div, sched_hard_div, sched_photon_div, "
                                 "sched_fetch_photon_div, sched_segments in [0, 64]");
    return MCD_OK;
}

void mcd_ctx::fill_geom(KGeom& g, const PhantomRec& ph)
{
    std::memset(&g, 0, sizeof g);
    g.t = tables[ph.tables].dev;
    g.maj = ph.maj;
    g.vox = ph.vox;
    g.nx = ph.g.nx;
    g.ny = ph.g.ny;
    g.nz = ph.g.nz;
    g.dx = (float)ph.g.dx;
    g.dy = (float)ph.g.dy;
    g.dz = (float)ph.g.dz;
    g.x0 = (float)ph.g.x0;
    g.y0 = (float)ph.g.y0;
    g.z0 = (float)ph.g.z0;
    g.x1 = (float)(ph.g.x0 + ph.g.nx * ph.g.dx);
    g.y1 = (float)(ph.g.y0 + ph.g.ny * ph.g.dy);
    g.z1 = (float)(ph.g.z0 + ph.g.nz * ph.g.dz);
    g.idx = (float)(1.0 / ph.g.dx);
    g.idy = (float)(1.0 / ph.g.dy);
    g.idz = (float)(1.0 / ph.g.dz);
}

static bool phantom_ok(mcd_ctx* c, int32_t phantom)
{
    return phantom >= 0 && phantom < (int32_t)c->phantoms.size() && c->phantoms[phantom].live;
}

// ------------------------------------------------------------ plain kernel

int mcd_ctx::simulate_plain(int32_t phantom, const mcd_source* src, uint64_t n_histories,
                            uint64_t seed, uint32_t request_key, const mcd_opts* opts,
                            mcd_result* out, hipStream_t s)
{
    const PhantomRec& ph = phantoms[phantom];
    const uint64_t first = opts ? opts->first_history : 0;
    DevSource ds;
    int rc = validate_source(src, &ds);
    if (rc) return rc;
    const int depth = opts && opts->stack_depth ? opts->stack_depth : kDefaultDepth;
    const int slots = opts && opts->tally_slots ? opts->tally_slots : kDefaultSlots;
    if (depth < 4 || depth > 4096) return fail(MCD_E_INVAL, "opts: stack_depth in [4, 4096]");
    if (slots < 16 || slots > 32768 || (slots & (slots - 1)))
        return fail(MCD_E_INVAL, "opts: tally_slots must be a power of two in [16, 32768]");
    int blocks, threads;
    rc = launch_shape(opts, tables[ph.tables].n_mat, &blocks, &threads);
    if (rc) return rc;
    Sched sc;
    if ((rc = wave_schedule(opts, &sc, kSchedPlain))) return rc;
    const bool diag = opts && opts->diagnostics;
    const bool accumulate = opts && opts->accumulate;
    if (opts && opts->history_records && !diag)
        return fail(MCD_E_INVAL, "history records need diagnostics");
    if (accumulate && tally_owner != phantom)
        return fail(MCD_E_INVAL, "opts.accumulate: the previous run used another phantom");

    if ((rc = ensure_scratch((size_t)blocks * threads, depth, slots, s))) return rc;
    if ((rc = ensure_tallies(ph.nv, s))) return rc;
    const bool want_final = out->dose || out->sigma;
    if (want_final && (!out->on_device || !out->dose || !out->sigma))
        if ((rc = ensure_stage(ph.nv, s))) return rc;

    if (opts && (opts->refined_build < 0 || opts->refined_build > 1))
        return fail(MCD_E_INVAL, "opts: refined_build must be 0 or 1");
    KPlain p;
    std::memset(&p, 0, sizeof p);
    fill_geom(p.g, ph);
    if (opts && opts->refined_build) p.g.t.refined = 1;
    p.src = ds;
    p.seed = (uint32_t)seed;
    p.key = request_key;
    p.first = (uint32_t)first;
    p.n = (uint32_t)n_histories;
    p.S = S;
    p.Q = Q;
    p.bal = (double*)(small + kOffBal);
    p.cnt = (unsigned long long*)(small + kOffCnt);
    p.err = (int*)(small + kOffErr);
    p.next = (unsigned long long*)(small + kOffNext);
    p.scratch = scratch;
    p.stack_depth = depth;
    p.slots = slots;
    p.lane_bytes = lane_bytes;
    p.hist = diag && opts ? opts->history_records : nullptr;
    p.lockstep = opts && opts->lockstep ? 1 : 0;
    p.sched = sc;
    double* red = (double*)(small + kOffRed);

    hipError_t e = hipEventRecord(ev[0], s);
    if (e == hipSuccess && !accumulate) {
        e = launch_fill_u32(S, (size_t)ph.nv * 2, 0u, s);
        if (e == hipSuccess) e = launch_fill_u32(Q, (size_t)ph.nv * 2, 0u, s);
    }
    if (e == hipSuccess && p.hist) e = launch_fill_u32(p.hist, (size_t)n_histories * 8, 0u, s);
    if (e == hipSuccess) e = launch_fill_u32(small, kSmallBytes / 4, 0u, s);
    if (e == hipSuccess) e = hipEventRecord(ev[1], s);
    if (e == hipSuccess) e = launch_plain(p, blocks, threads, diag, s);
    if (e == hipSuccess) e = hipEventRecord(ev[2], s);
    double* d_dose = nullptr;
    double* d_sigma = nullptr;
    const uint64_t n_total = n_histories + (accumulate ? tally_hist : 0);
    if (e == hipSuccess && want_final) {
        const bool direct = out->on_device && out->dose && out->sigma;
        d_dose = direct ? out->dose : dose;
        d_sigma = direct ? out->sigma : sigma;
        e = launch_finalize(S, Q, ph.vox, ph.nv, ph.g.dx * ph.g.dy * ph.g.dz, n_total, d_dose,
                            d_sigma, red, s);
    }
    if (e == hipSuccess) e = hipEventRecord(ev[3], s);
    unsigned char host_small[kSmallBytes];
    if (e == hipSuccess) e = hipMemcpyAsync(host_small, small, kSmallBytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "plain transport launch");
    int err;
    std::memcpy(&err, host_small + kOffErr, 4);
    if (err) {
        keys_clean = false;          // lanes stopped mid-history
        tally_owner = -1;
        return fail(err, err == MCD_E_OVERFLOW
                             ? "particle stack or local counter overflow: raise stack_depth or tally_slots"
                             : "device error");
    }
    tally_owner = phantom;
    tally_hist = n_total;

    const size_t vb = (size_t)ph.nv * sizeof(double);
    const hipMemcpyKind k_out = out->on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (out->dose && d_dose != out->dose) e = hipMemcpyAsync(out->dose, d_dose, vb, k_out, s);
    if (e == hipSuccess && out->sigma && d_sigma != out->sigma)
        e = hipMemcpyAsync(out->sigma, d_sigma, vb, k_out, s);
    if (e == hipSuccess && out->S) e = hipMemcpyAsync(out->S, S, vb, k_out, s);
    if (e == hipSuccess && out->Q) e = hipMemcpyAsync(out->Q, Q, vb, k_out, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "result copy");

    double bal[kBal];
    std::memcpy(bal, host_small + kOffBal, sizeof bal);
    out->eb = {bal[0], bal[1], bal[2], bal[3], bal[4], bal[5]};
    std::memcpy(out->counters, host_small + kOffCnt, sizeof out->counters);
    double r3[3];
    std::memcpy(r3, host_small + kOffRed, sizeof r3);
    out->dmax = want_final ? r3[0] : 0.0;
    out->sigma_bar = want_final && r3[2] > 0 ? r3[1] / r3[2] : 0.0;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ev[1], ev[2]);
    out->kernel_ms = ms;
    out->launches = 1;
    out->n_histories = n_total;
    (void)hipEventElapsedTime(&ms, ev[0], ev[3]);
    out->total_ms = ms;
    return MCD_OK;
}

// --------------------------------------------------------- regrouped engine

// Records per particle queue for cycles of `chunk` new histories.  A full
// queue is not an error (the particle stays on its lane's stack), so the
// capacity is bounded: 2^26 records of 48 B, 3.2 GB per buffer.
unsigned int mcd::queue_capacity(uint64_t chunk)
{
    return (unsigned int)std::min<uint64_t>(std::max<uint64_t>(2 * chunk, 1 << 16), (uint64_t)1 << 26);
}

size_t mcd::stack_scratch_bytes(uint64_t lanes, int depth, bool wave_stacks)
{
    if (wave_stacks) return (size_t)((lanes + 63) / 64) * wave_stack_bytes(16 * depth);
    return (size_t)lanes * phase_lane_bytes(depth);
}

// Histories h in [first, first + n) with h mod kBatches == b.
static double batch_count(uint64_t first, uint64_t n, int b)
{
    auto upto = [b](uint64_t x) -> uint64_t {      // count of h < x with h mod B == b
        return x / kBatches + ((x % kBatches) > (uint64_t)b ? 1 : 0);
    };
    return (double)(upto(first + n) - upto(first));
}

// Validates the requests and options of a regrouped run and fills the plan's
// host side (request and finaliser tables, launch shape, schedule); touches no
// device memory.
int mcd_ctx::prepare_regroup(int32_t phantom, const mcd_source* const* srcs, const uint64_t* ns,
                             const uint32_t* keys, int n_req, uint64_t seed, const mcd_opts* opts,
                             RegroupPlan& plan, const ReqExtra* extra)
{
    const PhantomRec& ph = phantoms[phantom];
    if (n_req < 1 || n_req > kMaxBatch) return fail(MCD_E_INVAL, "1 to 4096 requests per launch");
    if (seed >= ((uint64_t)1 << 32)) return fail(MCD_E_INVAL, "seed must be < 2^32");
    const uint64_t first = opts ? opts->first_history : 0;
    if (first >= ((uint64_t)1 << 32)) return fail(MCD_E_INVAL, "first_history must be < 2^32");
    if (opts && opts->lockstep) return fail(MCD_E_INVAL, "lockstep is a plain-kernel mode");
    if (opts && opts->stack_depth && (opts->stack_depth < 4 || opts->stack_depth > 4096))
        return fail(MCD_E_INVAL, "opts: stack_depth in [4, 4096]");
    const int cpl = opts && opts->chunk_per_lane ? opts->chunk_per_lane : kDefaultChunkPerLane;
    if (cpl < 1 || cpl > 4096) return fail(MCD_E_INVAL, "opts: chunk_per_lane in [1, 4096]");
    plan = RegroupPlan();
    plan.phantom = phantom;
    plan.n_req = n_req;
    plan.n_fin = n_req;
    plan.depth = opts && opts->stack_depth ? opts->stack_depth : kDefaultDepth;
    if (opts && (opts->regroup < 0 || opts->regroup > 3)) return fail(MCD_E_INVAL, "opts: regroup must be 0 to 3");
    plan.use_queues = opts && opts->regroup == 1;
    plan.wave_stacks = !opts || opts->regroup == 0 || opts->regroup == 3;
    plan.fp32 = opts && opts->tally_fp32 ? 1 : 0;
    plan.diag = opts && opts->diagnostics;
    if (opts && (opts->refined_build < 0 || opts->refined_build > 1))
        return fail(MCD_E_INVAL, "opts: refined_build must be 0 or 1");
    plan.refined_build = opts && opts->refined_build;
    if (opts && opts->history_records && (!plan.diag || n_req != 1))
        return fail(MCD_E_INVAL, "history records need diagnostics and a single request");
    int rc = launch_shape(opts, tables[ph.tables].n_mat, &plan.blocks, &plan.threads, &plan.global_tables);
    if (rc) return rc;
    bool photons_only = true;
    for (int r = 0; r < n_req; ++r) photons_only = photons_only && srcs[r] && srcs[r]->particle == MCD_PHOTON;
    const SchedDefaults sd = plan.wave_stacks ? (photons_only ? kSchedWavePhotonSources : kSchedWaveChargedSources)
                                              : (photons_only ? kSchedPhotonSources : kSchedChargedSources);
    if ((rc = wave_schedule(opts, &plan.sched, sd))) return rc;
    plan.req.resize(n_req);
    plan.fin.resize(n_req);
    plan.nb.assign((size_t)n_req * kBatches, 0.0);
    uint64_t lo = 0;
    for (int r = 0; r < n_req; ++r) {
        const uint64_t f = extra ? extra[r].first : first;
        if (ns[r] == 0 || ns[r] >= ((uint64_t)1 << 32) || f + ns[r] > ((uint64_t)1 << 32))
            return fail(MCD_E_INVAL, "need 1 <= n_histories < 2^32 and first + n <= 2^32 (request " +
                                         std::to_string(r) + ")");
        ReqDev& q = plan.req[r];
        std::memset(&q, 0, sizeof q);
        if ((rc = validate_source(srcs[r], &q.src))) return rc;
        q.seed = extra ? extra[r].seed : (uint32_t)seed;
        q.key = keys[r];
        q.first = (uint32_t)f;
        q.n = (uint32_t)ns[r];
        q.lo = lo;
        q.hist = plan.diag && opts ? opts->history_records : nullptr;
        lo += ns[r];
        for (int b = 0; b < kBatches; ++b) plan.nb[(size_t)r * kBatches + b] = batch_count(f, ns[r], b);
    }
    if (lo >= ((uint64_t)1 << 40)) return fail(MCD_E_INVAL, "at most 2^40 histories per launch");
    plan.total = lo;
    const uint64_t lanes = (uint64_t)plan.blocks * plan.threads;
    // With queues a cycle hands the other phase its particles, so new histories
    // come in chunks; with lane stacks one launch takes every history (each
    // launch ends with a tail of lanes finishing their last history).
    plan.chunk = plan.use_queues ? std::min<uint64_t>(lanes * (uint64_t)cpl, plan.total)
                                 : std::min<uint64_t>(plan.total, (uint64_t)1 << 31);
    // the electron phase of the last cycle keeps its photons on the lane stacks,
    // so no cycle is needed after the last new history
    plan.cycles = (int)((plan.total + plan.chunk - 1) / plan.chunk);
    return MCD_OK;
}

int mcd_ctx::plan_regroup(int32_t phantom, const mcd_source* const* srcs, const uint64_t* ns,
                          const uint32_t* keys, int n_req, uint64_t seed, const mcd_opts* opts,
                          bool keep_tally, RegroupPlan& plan, const ReqExtra* extra)
{
    int rc = prepare_regroup(phantom, srcs, ns, keys, n_req, seed, opts, plan, extra);
    if (rc) return rc;
    const PhantomRec& ph = phantoms[phantom];
    const uint64_t lanes = (uint64_t)plan.blocks * plan.threads;
    plan.bufs = &rb;
    plan.small = small;

    // device buffers
    const size_t elem = plan.fp32 ? sizeof(float) : sizeof(double);
    const size_t tally_bytes = extra ? 0 : (size_t)n_req * kBatches * (size_t)ph.nv * elem;
    const size_t stage_bytes = (size_t)n_req * (size_t)ph.nv * sizeof(double);
    const unsigned int cap = plan.use_queues ? queue_capacity(plan.chunk) : (1u << 12);
    if (keep_tally && (rb.tally_bytes < tally_bytes || rg_owner != phantom || rg_fp32 != plan.fp32 ||
                       n_req != 1))
        return fail(MCD_E_INVAL, "opts.accumulate: no matching regrouped tally to add to");
    size_t have;
    if (rb.cap < cap) {
        have = (size_t)4 * rb.cap * kRec;
        if ((rc = grow((void**)&rb.queues, &have, (size_t)4 * cap * kRec, "particle queues"))) return rc;
        rb.cap = cap;
    }
    if (!rb.ctl) {
        have = 0;
        if ((rc = grow((void**)&rb.ctl, &have, 4 * sizeof(QCtl), "queue control"))) return rc;
    }
    if (rb.claim_cap < plan.cycles + 4 * kExtraCycles) {
        have = (size_t)rb.claim_cap * 4;
        const int want = plan.cycles + 64 * kExtraCycles;
        if ((rc = grow((void**)&rb.claim, &have, (size_t)want * 4, "claim counters"))) return rc;
        rb.claim_cap = want;
    }
    if (rb.req_cap < n_req) {
        have = (size_t)rb.req_cap * sizeof(ReqDev);
        if ((rc = grow((void**)&rb.req, &have, (size_t)n_req * sizeof(ReqDev), "request table"))) return rc;
        have = (size_t)rb.req_cap * sizeof(FinalReq);
        if ((rc = grow((void**)&rb.fin, &have, (size_t)n_req * sizeof(FinalReq), "request table"))) return rc;
        have = (size_t)rb.req_cap * 3 * sizeof(double);
        if ((rc = grow((void**)&rb.red, &have, (size_t)n_req * 3 * sizeof(double), "request table"))) return rc;
        rb.req_cap = n_req;
    }
    if (!keep_tally && tally_bytes) {
        if ((rc = grow(&rb.tally, &rb.tally_bytes, tally_bytes, "tallies"))) return rc;
    }
    if (!extra && rb.stage_bytes < stage_bytes) {
        (void)hipDeviceSynchronize();
        release(rb.dose, rb.stage_bytes);
        release(rb.sigma, rb.stage_bytes);
        rb.dose = rb.sigma = nullptr;
        rb.stage_bytes = 0;
        if ((rc = alloc((void**)&rb.dose, stage_bytes, "dose staging"))) return rc;
        if ((rc = alloc((void**)&rb.sigma, stage_bytes, "dose staging"))) {
            release(rb.dose, stage_bytes);
            rb.dose = nullptr;
            return rc;
        }
        rb.stage_bytes = stage_bytes;
    }
    if ((rc = grow((void**)&rb.scratch, &rb.scratch_bytes, stack_scratch_bytes(lanes, plan.depth, plan.wave_stacks),
                   "particle stacks")))
        return rc;

    for (int r = 0; r < n_req; ++r) {
        plan.req[r].tally = extra ? extra[r].tally : (char*)rb.tally + (size_t)r * kBatches * ph.nv * elem;
        FinalReq& f = plan.fin[r];
        std::memset(&f, 0, sizeof f);
        f.tally = plan.req[r].tally;
        f.dose = extra ? extra[r].dose : rb.dose + (size_t)r * ph.nv;
        f.sigma = extra ? extra[r].sigma : rb.sigma + (size_t)r * ph.nv;
        f.red = rb.red + 3 * r;
        for (int b = 0; b < kBatches; ++b) {
            f.nb[b] = plan.nb[(size_t)r * kBatches + b];
            if (keep_tally) f.nb[b] += rg_nb[b];
            if (extra && extra[r].nb_prior) f.nb[b] += extra[r].nb_prior[b];
        }
    }
    return MCD_OK;
}

int mcd_ctx::enqueue_cycles(const RegroupPlan& plan, int c0, int c1, hipStream_t s)
{
    const PhantomRec& ph = phantoms[plan.phantom];
    const RegroupBufs& B = *plan.bufs;
    KPhase k;
    std::memset(&k, 0, sizeof k);
    fill_geom(k.g, ph);
    if (plan.refined_build) k.g.t.refined = 1;
    k.req = B.req;
    k.n_req = plan.n_req;
    k.tally_fp32 = plan.fp32;
    k.total = plan.total;
    k.chunk = plan.chunk;
    k.claim = B.claim;
    k.q_cap = B.cap;
    k.use_queues = plan.use_queues;
    k.nv = ph.nv;
    k.bal = (double*)(plan.small + kOffBal);
    k.cnt = (unsigned long long*)(plan.small + kOffCnt);
    k.err = (int*)(plan.small + kOffErr);
    k.scratch = B.scratch;
    k.stack_depth = plan.depth;
    k.lane_bytes = phase_lane_bytes(plan.depth);
    k.sched = plan.sched;
    char* Qg[2] = {B.queues, B.queues + (size_t)B.cap * kRec};
    char* Qe[2] = {B.queues + (size_t)2 * B.cap * kRec, B.queues + (size_t)3 * B.cap * kRec};
    QCtl* Cg[2] = {B.ctl + 0, B.ctl + 1};
    QCtl* Ce[2] = {B.ctl + 2, B.ctl + 3};
    for (int c = c0; c < c1; ++c) {
        if (c >= B.claim_cap) return fail(MCD_E_OVERFLOW, "too many transport cycles");
        const int a = c & 1, b = (c + 1) & 1;
        k.cycle = (uint32_t)c;
        // photon phase: photons of the previous electron phase and new histories
        k.q_in = Qg[a];
        k.q_in_ctl = Cg[a];
        k.q_out = Qe[a];
        k.q_out_ctl = Ce[a];
        k.q_reset_ctl = Cg[b];
        k.use_queues = plan.use_queues;
        if (plan.wave_stacks) {
            // one launch takes every history; its waves pool their stacks
            k.stack_depth = 16 * plan.depth;
            k.lane_bytes = wave_stack_bytes(k.stack_depth);
            hipError_t e = launch_wave(k, plan.blocks, plan.threads, plan.diag, plan.global_tables, s);
            if (e != hipSuccess) return hip_fail(e, "wave-stack transport launch");
            continue;
        }
        hipError_t e = launch_phase(k, true, plan.blocks, plan.threads, plan.diag, s);
        if (e != hipSuccess) return hip_fail(e, "photon phase launch");
        if (!plan.use_queues) continue;       // nothing is ever queued for it
        // electron phase: electrons of this photon phase; the last cycle keeps
        // the photons it creates on the lane stacks
        k.use_queues = c + 1 < c1 ? 1 : 0;
        k.q_in = Qe[a];
        k.q_in_ctl = Ce[a];
        k.q_out = Qg[b];
        k.q_out_ctl = Cg[b];
        k.q_reset_ctl = Ce[b];
        e = launch_phase(k, false, plan.blocks, plan.threads, plan.diag, s);
        if (e != hipSuccess) return hip_fail(e, "electron phase launch");
    }
    return MCD_OK;
}

// Clears the run state, then schedules every cycle and the finalisation.
// Safe to capture in a graph: fills are kernels, copies happen beforehand.
// Under capture (`captured`) no timing event is recorded (an event recorded
// into a graph does not time its replays; the caller times the launch) and the
// history records are not cleared (their buffer changes from call to call, so
// the caller clears them before each launch).
int mcd_ctx::enqueue_regroup(const RegroupPlan& plan, bool clear_tally, bool captured, hipStream_t s)
{
    const PhantomRec& ph = phantoms[plan.phantom];
    const RegroupBufs& B = *plan.bufs;
    hipError_t e = captured ? hipSuccess : hipEventRecord(ev[0], s);
    if (e == hipSuccess && clear_tally)
        e = launch_fill_u32(B.tally, (size_t)plan.n_req * kBatches * ph.nv * (plan.fp32 ? 1 : 2), 0u, s);
    if (e == hipSuccess) e = launch_fill_u32(B.ctl, 4 * sizeof(QCtl) / 4, 0u, s);
    if (e == hipSuccess) e = launch_fill_u32(B.claim, (size_t)B.claim_cap, 0u, s);
    if (e == hipSuccess) e = launch_fill_u32(plan.small, kSmallBytes / 4, 0u, s);
    if (e == hipSuccess) e = launch_fill_u32(B.red, (size_t)plan.n_req * 6, 0u, s);
    if (e == hipSuccess && plan.req[0].hist && !captured)
        e = launch_fill_u32(plan.req[0].hist, (size_t)plan.req[0].n * 8, 0u, s);
    if (e == hipSuccess && !captured) e = hipEventRecord(ev[1], s);
    if (e != hipSuccess) return hip_fail(e, "regrouped set-up");
    int rc = enqueue_cycles(plan, 0, plan.cycles, s);
    if (rc) return rc;
    e = captured ? hipSuccess : hipEventRecord(ev[2], s);
    if (e == hipSuccess)
        e = launch_finalize_batches(B.fin, plan.n_fin, ph.vox, ph.nv, ph.g.dx * ph.g.dy * ph.g.dz,
                                    plan.fp32, s);
    if (e == hipSuccess && !captured) e = hipEventRecord(ev[3], s);
    if (e != hipSuccess) return hip_fail(e, "finalisation launch");
    return MCD_OK;
}

// Waits for the scheduled cycles.  The last electron phase keeps its photons
// on the lane stacks, so no photon should remain queued; if one does, more
// cycles run and the finalisation is repeated.
int mcd_ctx::finish_regroup(RegroupPlan& plan, hipStream_t s, int* cycles_run)
{
    const PhantomRec& ph = phantoms[plan.phantom];
    const RegroupBufs& B = *plan.bufs;
    int done = plan.cycles;
    for (;;) {
        QCtl ctl[4];
        int err = 0;
        hipError_t e = hipMemcpyAsync(ctl, B.ctl, sizeof ctl, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(&err, plan.small + kOffErr, 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "regrouped run");
        if (err)
            return fail(err, err == MCD_E_OVERFLOW ? "particle stack overflow: raise stack_depth"
                                                   : "device error in a transport phase");
        if (ctl[done & 1].count == 0) break;      // photons waiting for cycle `done`
        int rc = enqueue_cycles(plan, done, done + 1, s);
        if (rc) return rc;
        done += 1;
        e = launch_fill_u32(B.red, (size_t)plan.n_req * 6, 0u, s);
        if (e == hipSuccess) e = hipEventRecord(ev[2], s);
        if (e == hipSuccess)
            e = launch_finalize_batches(B.fin, plan.n_fin, ph.vox, ph.nv,
                                        ph.g.dx * ph.g.dy * ph.g.dz, plan.fp32, s);
        if (e == hipSuccess) e = hipEventRecord(ev[3], s);
        if (e != hipSuccess) return hip_fail(e, "extra cycles");
    }
    if (cycles_run) *cycles_run = done;
    return MCD_OK;
}

int mcd_ctx::collect_regroup(const RegroupPlan& plan, mcd_result* const* outs, mcd_result* total,
                             hipStream_t s)
{
    const PhantomRec& ph = phantoms[plan.phantom];
    const RegroupBufs& B = *plan.bufs;
    const size_t vb = (size_t)ph.nv * sizeof(double);
    unsigned char host_small[kSmallBytes];
    std::vector<double> red((size_t)plan.n_req * 3);
    hipError_t e = hipMemcpyAsync(host_small, plan.small, kSmallBytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(red.data(), B.red, red.size() * sizeof(double), hipMemcpyDeviceToHost, s);
    for (int r = 0; r < plan.n_req && e == hipSuccess; ++r) {
        mcd_result* o = outs[r];
        if (!o) continue;
        const hipMemcpyKind k = o->on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        if (o->dose && o->dose != plan.fin[r].dose) e = hipMemcpyAsync(o->dose, plan.fin[r].dose, vb, k, s);
        if (e == hipSuccess && o->sigma && o->sigma != plan.fin[r].sigma)
            e = hipMemcpyAsync(o->sigma, plan.fin[r].sigma, vb, k, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "result copy");
    float kms = 0.f, tms = 0.f;
    (void)hipEventElapsedTime(&kms, ev[1], ev[2]);
    (void)hipEventElapsedTime(&tms, ev[0], ev[3]);
    double bal[kBal];
    std::memcpy(bal, host_small + kOffBal, sizeof bal);
    for (int r = 0; r < plan.n_req; ++r) {
        mcd_result* o = outs[r];
        if (!o) continue;
        o->dmax = red[3 * r];
        o->sigma_bar = red[3 * r + 2] > 0 ? red[3 * r + 1] / red[3 * r + 2] : 0.0;
        o->kernel_ms = kms;
        o->launches = plan.launches;
        double nh = 0.0;
        for (int b = 0; b < kBatches; ++b) nh += plan.fin[r].nb[b];
        o->n_histories = (uint64_t)nh;
        o->total_ms = tms;
    }
    if (total) {
        total->eb = {bal[0], bal[1], bal[2], bal[3], bal[4], bal[5]};
        std::memcpy(total->counters, host_small + kOffCnt, sizeof total->counters);
        total->kernel_ms = kms;
        total->launches = plan.launches;
        total->n_histories = plan.total;
        total->total_ms = tms;
    }
    return MCD_OK;
}

void mcd_ctx::release_graph()
{
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    graph_exec = nullptr;
    graph = nullptr;
    graph_key.clear();
}

// Uploads the request and finaliser tables, then runs the plan (captured
// into a graph and replayed when `use_graph` is set).
int mcd::run_regroup(mcd_ctx* c, RegroupPlan& plan, bool clear_tally, bool use_graph, hipStream_t s)
{
    // S outputs are written by the finaliser straight from the sub-tallies
    hipError_t e = hipMemcpy(plan.bufs->req, plan.req.data(), plan.n_req * sizeof(ReqDev), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(plan.bufs->fin, plan.fin.data(), plan.n_req * sizeof(FinalReq), hipMemcpyHostToDevice);
    if (e != hipSuccess) return c->hip_fail(e, "request table upload");
    int rc;
    if (!use_graph) {
        if ((rc = c->enqueue_regroup(plan, clear_tally, false, s))) return rc;
    } else {
        // key: the launch configuration and every device pointer the graph bakes in
        std::vector<unsigned char> key;
        auto add = [&key](const void* p, size_t n) {
            const unsigned char* b = (const unsigned char*)p;
            key.insert(key.end(), b, b + n);
        };
        add(&plan.phantom, sizeof plan.phantom);
        add(&plan.n_req, sizeof plan.n_req);
        add(&plan.n_fin, sizeof plan.n_fin);
        add(&plan.total, sizeof plan.total);
        add(&plan.chunk, sizeof plan.chunk);
        add(&plan.cycles, sizeof plan.cycles);
        add(&plan.blocks, sizeof plan.blocks);
        add(&plan.threads, sizeof plan.threads);
        add(&plan.depth, sizeof plan.depth);
        add(&plan.fp32, sizeof plan.fp32);
        add(&plan.diag, sizeof plan.diag);
        add(&plan.refined_build, sizeof plan.refined_build);
        add(&plan.use_queues, sizeof plan.use_queues);
        add(&plan.wave_stacks, sizeof plan.wave_stacks);
        add(&plan.global_tables, sizeof plan.global_tables);
        add(&plan.sched, sizeof plan.sched);
        add(&clear_tally, sizeof clear_tally);
        add(&c->rb, sizeof c->rb);
        add(&c->small, sizeof c->small);
        add(&c->phantoms[plan.phantom].vox, sizeof(void*));
        if (!c->graph_exec || key != c->graph_key) {
            c->release_graph();
            e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return c->hip_fail(e, "graph capture");
            rc = c->enqueue_regroup(plan, clear_tally, true, s);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(s, &g);
            if (rc) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (e2 != hipSuccess) return c->hip_fail(e2, "graph capture");
            e = hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                (void)hipGraphDestroy(g);
                return c->hip_fail(e, "graph instantiation");
            }
            c->graph = g;
            c->graph_key = key;
        }
        // the replay is timed as a whole: set-up fills, transport and
        // finalisation (the fills and the finaliser take microseconds)
        e = hipEventRecord(c->ev[0], s);
        if (e == hipSuccess && plan.req[0].hist)
            e = launch_fill_u32(plan.req[0].hist, (size_t)plan.req[0].n * 8, 0u, s);
        if (e == hipSuccess) e = hipEventRecord(c->ev[1], s);
        if (e == hipSuccess) e = hipGraphLaunch(c->graph_exec, s);
        if (e == hipSuccess) e = hipEventRecord(c->ev[2], s);
        if (e == hipSuccess) e = hipEventRecord(c->ev[3], s);
        if (e != hipSuccess) return c->hip_fail(e, "graph launch");
    }
    int cycles_run = 0;
    int rc2 = c->finish_regroup(plan, s, &cycles_run);
    plan.launches = cycles_run * (plan.use_queues ? 2 : 1);
    return rc2;
}

// ------------------------------------------------------------------ public

int mcd_simulate(mcd_ctx* c, int32_t phantom, const mcd_source* src, uint64_t n_histories,
                 uint64_t seed, uint32_t request_key, const mcd_opts* opts, mcd_result* out,
                 void* hip_stream)
{
    if (!c || !out) return MCD_E_INVAL;
    std::lock_guard<mcd::FairMutex> run_lock(c->run_mu);
    if (!phantom_ok(c, phantom)) return c->fail(MCD_E_NOTFOUND, "unknown phantom handle");
    const uint64_t first = opts ? opts->first_history : 0;
    if (n_histories == 0 || n_histories >= ((uint64_t)1 << 32) || seed >= ((uint64_t)1 << 32) ||
        first >= ((uint64_t)1 << 32) || first + n_histories > ((uint64_t)1 << 32))
        return c->fail(MCD_E_INVAL, "need 1 <= n_histories < 2^32, seed < 2^32, first + n <= 2^32");
    if (n_histories < 2 && (out->dose || out->sigma))
        return c->fail(MCD_E_INVAL, "an uncertainty needs at least 2 histories");
    const int kernel = opts ? opts->kernel : MCD_KERNEL_REGROUPED;
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : c->stream;
    mcd::DeviceGuard dg(c->device);
    if (kernel == MCD_KERNEL_PLAIN)
        return c->simulate_plain(phantom, src, n_histories, seed, request_key, opts, out, s);
    if (kernel != MCD_KERNEL_REGROUPED) return c->fail(MCD_E_INVAL, "opts: unknown kernel");
    if (out->Q) return c->fail(MCD_E_INVAL, "Q needs history-by-history statistics (plain kernel)");
    const bool accumulate = opts && opts->accumulate;
    RegroupPlan plan;
    int rc = c->plan_regroup(phantom, &src, &n_histories, &request_key, 1, seed, opts, accumulate, plan);
    if (rc) return rc;
    plan.fin[0].S = nullptr;
    if (out->S) {
        if (out->on_device) plan.fin[0].S = out->S;
        else if ((rc = c->ensure_stage(c->phantoms[phantom].nv, s))) return rc;
        if (!out->on_device) plan.fin[0].S = c->dose;
    }
    const bool use_graph = opts && opts->use_graph;
    if (use_graph && hip_stream) s = c->stream;       // capture needs a non-legacy stream
    if ((rc = run_regroup(c, plan, !accumulate, use_graph, s))) {
        c->rg_owner = -1;
        return rc;
    }
    if (!accumulate) c->rg_nb.assign(kBatches, 0.0);
    for (int b = 0; b < kBatches; ++b) c->rg_nb[b] += plan.nb[b];
    c->rg_owner = phantom;
    c->rg_fp32 = plan.fp32;
    mcd_result* outs[1] = {out};
    if ((rc = c->collect_regroup(plan, outs, out, s))) return rc;
    if (out->S && !out->on_device) {
        hipError_t e = hipMemcpy(out->S, c->dose, (size_t)c->phantoms[phantom].nv * sizeof(double),
                                 hipMemcpyDeviceToHost);
        if (e != hipSuccess) return c->hip_fail(e, "S copy");
    }
    return MCD_OK;
}

int mcd_simulate_batch(mcd_ctx* c, int32_t phantom, const mcd_batch_item* items, int32_t n_items,
                       uint64_t seed, const mcd_opts* opts, mcd_result* total, void* hip_stream)
{
    if (!c || !items || n_items < 1 || n_items > kMaxBatch) return MCD_E_INVAL;
    std::lock_guard<mcd::FairMutex> run_lock(c->run_mu);
    if (!phantom_ok(c, phantom)) return c->fail(MCD_E_NOTFOUND, "unknown phantom handle");
    if (opts && (opts->kernel != MCD_KERNEL_REGROUPED || opts->accumulate))
        return c->fail(MCD_E_INVAL, "batches run on the regrouped kernel without accumulation");
    std::vector<const mcd_source*> srcs(n_items);
    std::vector<uint64_t> ns(n_items);
    std::vector<uint32_t> keys(n_items);
    std::vector<mcd_result*> outs(n_items);
    for (int i = 0; i < n_items; ++i) {
        srcs[i] = &items[i].src;
        ns[i] = items[i].n_histories;
        keys[i] = items[i].request_key;
        outs[i] = items[i].out;
        if (outs[i] && outs[i]->Q) return c->fail(MCD_E_INVAL, "Q needs the plain kernel");
        if (ns[i] < 2 && outs[i] && (outs[i]->dose || outs[i]->sigma))
            return c->fail(MCD_E_INVAL, "an uncertainty needs at least 2 histories");
    }
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : c->stream;
    mcd::DeviceGuard dg(c->device);
    RegroupPlan plan;
    int rc = c->plan_regroup(phantom, srcs.data(), ns.data(), keys.data(), n_items, seed, opts, false, plan);
    if (rc) return rc;
    for (int i = 0; i < n_items; ++i)
        plan.fin[i].S = outs[i] && outs[i]->S && outs[i]->on_device ? outs[i]->S : nullptr;
    const bool use_graph = opts && opts->use_graph;
    if (use_graph) s = c->stream;
    if ((rc = run_regroup(c, plan, true, use_graph, s))) return rc;
    c->rg_owner = -1;
    return c->collect_regroup(plan, outs.data(), total, s);
}
