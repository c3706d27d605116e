// Host-side state of an mcdose context (internal to libmcdose).
#pragma once

#include <hip/hip_runtime.h>

#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "engine.h"
#include "mcdose.h"

namespace mcd {

constexpr int kDefaultBlock = 512;
constexpr int kDefaultDepth = 64;
constexpr int kDefaultSlots = 512;
constexpr int kDefaultChunkPerLane = 16;
constexpr int kLdsPerCu = 160 * 1024;
constexpr int kExtraCycles = 8;     // claim counters kept beyond the planned cycles
constexpr int kMaxBatch = 4096;
// Wave-schedule defaults (fetch_div, hard_div, photon_div), swept on the 6 MV
// and 20 MeV workloads.  The regrouped kernel's depend on the kind of its
// sources: photon-only launches fetch at 1/3 (their histories end often, and
// fuller fetch steps pay off), sample hard events at 1/24 and fly photons
// once they are half the electrons; launches with electron or positron
// sources fetch at 1/4, sample hard events at 1/8 and fly photons at a sixth
// of the electrons.  The plain kernel does best at (3, 24, 2) for both.
struct SchedDefaults {
    int fetch_div, hard_div, photon_div, fetch_photon_div, segments;
};
constexpr SchedDefaults kSchedPhotonSources{3, 24, 2, 3, 1};
constexpr SchedDefaults kSchedChargedSources{4, 8, 6, 4, 1};
constexpr SchedDefaults kSchedPlain{3, 24, 2, 3, 1};
// Wave-stack schedule (the default regrouped one).  In electron mode a wave
// fetches once 1/16 of its lanes are idle (an electron step runs many
// segments, so idle lanes are expensive there); in photon mode once half of
// them are (fuller fetch steps between short photon steps).  Hard events at
// 1/24 of the lanes for photon sources and as soon as one lane waits for
// charged sources.  photon_div there sets when the wave leaves its photon or
// electron mode (work of the mode's kind below 64 / photon_div lanes): 1, as
// soon as it cannot fill the wave.  An electron step runs up to 12 segments
// before the wave decides again.
constexpr SchedDefaults kSchedWavePhotonSources{16, 24, 1, 2, 12};
constexpr SchedDefaults kSchedWaveChargedSources{16, 64, 1, 2, 12};

// Small per-run device block: energy balance, counters, error flag, work
// counter and finalisation reductions of the plain kernel.
constexpr size_t kOffBal = 0;                            // kBal doubles
constexpr size_t kOffCnt = 64;                           // kCounters u64
constexpr size_t kOffErr = kOffCnt + 8 * kCounters;      // int
constexpr size_t kOffNext = kOffErr + 8;                 // u64
constexpr size_t kOffRed = kOffNext + 8;                 // 3 doubles: Dmax bits, sum sigma/D, count
constexpr size_t kSmallBytes = (kOffRed + 24 + 63) / 64 * 64;
static_assert(kOffCnt >= 8 * kBal, "energy balance overlaps the counters");
static_assert(kSmallBytes % 64 == 0 && kOffRed + 24 <= kSmallBytes, "small block layout");

constexpr int kNQ = 13;           // tabulated quantities per material in a table blob

struct TableSet {
    DevTables dev{};
    std::vector<double> q;           // FP64 nodes [n_mat][kNQ][512] (ranges, majorants)
    int n_mat = 0;
    double emin = 0, emax = 0, e_abs_e = 0, e_abs_g = 0, w_cc = 0, w_cr = 0;
    double kappa_step = 0, f_e = 0, a_hinge = 0;
    size_t bytes = 0;                // each of phot, elec, hinge (posi: half as many)
    bool live = false;
    const double* range(int m) const { return &q[((size_t)m * kNQ + 3) * kNE]; }
    const double* range_pos(int m) const { return &q[((size_t)m * kNQ + 10) * kNE]; }
};

struct PhantomRec {
    mcd_grid g{};
    int tables = -1;
    int64_t nv = 0;
    uint2* vox = nullptr;
    float* maj = nullptr;
    bool live = false;
};

// Device buffers of one regrouped launch sequence (queues, requests, tallies).
struct RegroupBufs {
    char* queues = nullptr;          // 4 buffers of cap records: Qg[0], Qg[1], Qe[0], Qe[1]
    unsigned int cap = 0;
    QCtl* ctl = nullptr;             // 4 control blocks
    unsigned int* claim = nullptr;   // per-cycle claim counters
    int claim_cap = 0;
    ReqDev* req = nullptr;
    int req_cap = 0;
    FinalReq* fin = nullptr;
    double* red = nullptr;           // 3 doubles per request
    void* tally = nullptr;           // n_req * kBatches * nv accumulators
    size_t tally_bytes = 0;
    double* dose = nullptr;          // staging: n_req * nv
    double* sigma = nullptr;
    size_t stage_bytes = 0;
    char* scratch = nullptr;         // lane stacks
    size_t scratch_bytes = 0;
};

// Per-request overrides of a regrouped run (serving): history offset, seed,
// persistent tally and dose buffers, and histories already in the tally.
struct ReqExtra {
    uint64_t first = 0;
    uint32_t seed = 0;
    void* tally = nullptr;
    double* dose = nullptr;
    double* sigma = nullptr;
    const double* nb_prior = nullptr;
};

// A prepared regrouped run: everything the kernels and the finaliser need.
struct RegroupPlan {
    int phantom = -1;
    int n_req = 0;
    int n_fin = 0;                   // requests 0 .. n_fin-1 are finalised after the run
    uint64_t total = 0, chunk = 0;
    int cycles = 0;                  // scheduled cycles
    int launches = 0;                // transport launches actually run
    int blocks = 0, threads = 0;
    int depth = 0;
    int fp32 = 0;
    bool diag = false;
    bool refined_build = false;      // force the kernels built with the refinement code
    bool use_queues = false;
    bool wave_stacks = false;        // secondaries on per-wave photon and electron stacks
    bool global_tables = false;      // wave-stack kernel reads its tables from device memory
    Sched sched{};
    RegroupBufs* bufs = nullptr;     // device buffers the run uses (the context's, or a
    unsigned char* small = nullptr;  // carve-out of the no-allocation scratch)
    std::vector<ReqDev> req;
    std::vector<FinalReq> fin;
    std::vector<double> nb;          // n_req * kBatches histories per sub-tally
};

}  // namespace mcd

struct mcd_server;
struct mcd_ctx;

namespace mcd {
// Uploads the request tables of a plan and runs it on stream s (captured in a
// graph and replayed when use_graph); returns when the device is done.
int run_regroup(mcd_ctx* c, RegroupPlan& plan, bool clear_tally, bool use_graph, hipStream_t s);
// Records per particle queue for cycles of `chunk` new histories.
unsigned int queue_capacity(uint64_t chunk);
// Device bytes of the particle stacks of `lanes` lanes at stack depth `depth`:
// per-lane stacks, or (wave_stacks) per-wave photon and electron stacks of
// 16 x depth records each, the same number of records per wave.
size_t stack_scratch_bytes(uint64_t lanes, int depth, bool wave_stacks);
// Looks up the calling thread's current device's copy of the no-allocation
// scratch array (once per device; later calls return the first outcome).
hipError_t noalloc_setup(int device);

// Makes `dev` the calling thread's current HIP device for the guard's scope
// and gives the caller back its own device afterwards, so that no entry point
// changes the caller's HIP state.
class DeviceGuard {
public:
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
        ok_ = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        if (prev_ >= 0) (void)hipSetDevice(prev_);
    }
    DeviceGuard(const DeviceGuard&) = delete;
    DeviceGuard& operator=(const DeviceGuard&) = delete;
    bool ok() const { return ok_; }

private:
    int prev_ = -1;
    bool ok_ = false;
};

// Mutex that hands itself over in request order (a ticket lock).  The serving
// worker takes the device lock once per epoch and asks for it again at once;
// with a plain mutex it can win every time and hold off a blocking call for
// the whole backlog.  Usable with std::lock_guard.
class FairMutex {
public:
    void lock()
    {
        std::unique_lock<std::mutex> lk(m_);
        const uint64_t t = next_++;
        cv_.wait(lk, [&] { return serving_ == t; });
    }
    void unlock()
    {
        {
            std::lock_guard<std::mutex> lk(m_);
            ++serving_;
        }
        cv_.notify_all();
    }

private:
    std::mutex m_;
    std::condition_variable cv_;
    uint64_t next_ = 0, serving_ = 0;
};
}  // namespace mcd

struct mcd_ctx {
    int device = 0;
    int cu_count = 0;
    int clock_khz = 0;        // peak engine clock
    int max_lds = 0;     // dynamic LDS bytes a workgroup may use
    hipStream_t stream = nullptr;
    uint64_t budget = 0, used = 0;
    // Lock order: run_mu, then mu, then the server's mutex.
    std::mutex mu;        // tables / phantoms vectors (changed under run_mu and mu)
    mcd::FairMutex run_mu;  // one device run (blocking call or serving epoch) at a time, FIFO
    std::mutex mu_alloc;  // budget accounting
    std::vector<mcd::TableSet> tables;
    std::vector<mcd::PhantomRec> phantoms;

    // plain kernel: lane scratch (stacks and local counters) and tallies
    char* scratch = nullptr;
    size_t scratch_bytes = 0, scratch_lanes = 0, lane_bytes = 0;
    int stack_depth = 0, slot_count = 0;
    bool keys_clean = false;
    double* S = nullptr;
    double* Q = nullptr;
    int64_t tally_cap = 0;
    int tally_owner = -1;
    uint64_t tally_hist = 0;
    double* dose = nullptr;
    double* sigma = nullptr;
    int64_t stage_cap = 0;
    unsigned char* small = nullptr;
    hipEvent_t ev[4] = {};

    // regrouped kernel
    mcd::RegroupBufs rb;
    int rg_owner = -1;                // phantom of the accumulated regrouped tally
    std::vector<double> rg_nb;        // accumulated histories per sub-tally
    int rg_fp32 = -1;
    // graph cache for repeated batched calls
    hipGraphExec_t graph_exec = nullptr;
    hipGraph_t graph = nullptr;
    std::vector<unsigned char> graph_key;

    // serving
    mcd_server* server = nullptr;

    int fail(int status, const std::string& msg);
    int hip_fail(hipError_t e, const char* what);
    int alloc(void** p, size_t bytes, const char* what);
    void release(void* p, size_t bytes);
    int grow(void** p, size_t* have, size_t need, const char* what);
    int validate_source(const mcd_source* s, mcd::DevSource* d);
    int ensure_scratch(size_t lanes, int depth, int slots, hipStream_t s);
    int ensure_tallies(int64_t nv, hipStream_t s);
    int ensure_stage(int64_t nv, hipStream_t s);
    // Validates the launch options and resolves the default grid; gtab: the
    // wave-stack kernel reads its tables from device memory; resident: the
    // workgroups a CU holds at once (wave-stack kernel only, else 0).
    int launch_shape(const mcd_opts* o, int n_mat, int* blocks, int* threads, bool* gtab = nullptr,
                     int* resident = nullptr);
    int wave_schedule(const mcd_opts* o, mcd::Sched* sc, mcd::SchedDefaults d);
    void fill_geom(mcd::KGeom& g, const mcd::PhantomRec& ph);
    int simulate_plain(int32_t phantom, const mcd_source* src, uint64_t n, uint64_t seed,
                       uint32_t key, const mcd_opts* opts, mcd_result* out, hipStream_t s);
    // regrouped engine
    int prepare_regroup(int32_t phantom, const mcd_source* const* srcs, const uint64_t* ns,
                        const uint32_t* keys, int n_req, uint64_t seed, const mcd_opts* opts,
                        mcd::RegroupPlan& plan, const mcd::ReqExtra* extra = nullptr);
    int plan_regroup(int32_t phantom, const mcd_source* const* srcs, const uint64_t* ns,
                     const uint32_t* keys, int n_req, uint64_t seed, const mcd_opts* opts,
                     bool keep_tally, mcd::RegroupPlan& plan, const mcd::ReqExtra* extra = nullptr);
    int enqueue_regroup(const mcd::RegroupPlan& plan, bool clear_tally, bool captured, hipStream_t s);
    int enqueue_cycles(const mcd::RegroupPlan& plan, int c0, int c1, hipStream_t s);
    int finish_regroup(mcd::RegroupPlan& plan, hipStream_t s, int* cycles_run);
    int collect_regroup(const mcd::RegroupPlan& plan, mcd_result* const* outs, mcd_result* total,
                        hipStream_t s);
    void release_graph();
    void shutdown_serving();
    bool serving_uses(int32_t phantom);
    const std::string& last_error() const;
};
