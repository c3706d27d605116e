// Host-side state of an mcdose context (internal to libmcdose).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "engine.h"
#include "mcdose.h"

namespace mcd {

constexpr int kDefaultBlock = 512;
constexpr int kDefaultDepth = 64;
constexpr int kDefaultSlots = 512;
constexpr int kLdsPerCu = 160 * 1024;

// Small per-run device block: energy balance, counters, error flag, work
// counter and finalisation reductions.
constexpr size_t kOffBal = 0;       // kBal doubles
constexpr size_t kOffCnt = 64;      // kCounters u64
constexpr size_t kOffErr = 320;     // int
constexpr size_t kOffNext = 328;    // u64
constexpr size_t kOffRed = 336;     // 3 doubles: Dmax bits, sum sigma/D, count
constexpr size_t kSmallBytes = 384;

struct TableSet {
    DevTables dev{};
    std::vector<double> q;           // FP64 nodes [n_mat][8][512] (for majorants)
    int n_mat = 0;
    double emin = 0, emax = 0, e_abs_e = 0, e_abs_g = 0, w_cc = 0, w_cr = 0;
    double kappa_step = 0, f_e = 0, a_hinge = 0;
    size_t bytes = 0;
    bool live = false;
    const double* range(int m) const { return &q[((size_t)m * 8 + 3) * kNE]; }
};

struct PhantomRec {
    mcd_grid g{};
    int tables = -1;
    int64_t nv = 0;
    uint2* vox = nullptr;
    float* maj = nullptr;
    bool live = false;
};

}  // namespace mcd

struct mcd_ctx {
    int device = 0;
    int cu_count = 0;
    int max_lds = 0;     // dynamic LDS bytes a workgroup may use
    hipStream_t stream = nullptr;
    uint64_t budget = 0, used = 0;
    std::mutex mu;        // tables / phantoms vectors
    std::mutex run_mu;    // one blocking run at a time
    std::vector<mcd::TableSet> tables;
    std::vector<mcd::PhantomRec> phantoms;

    // lane scratch (particle stacks and local counters)
    char* scratch = nullptr;
    size_t scratch_bytes = 0, scratch_lanes = 0, lane_bytes = 0;
    int stack_depth = 0, slot_count = 0;
    bool keys_clean = false;

    // tallies of the blocking path and host-output staging
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

    std::string last_error;

    int fail(int status, const std::string& msg);
    int hip_fail(hipError_t e, const char* what);
    int alloc(void** p, size_t bytes, const char* what);
    void release(void* p, size_t bytes);
    int validate_source(const mcd_source* s, mcd::DevSource* d);
    int ensure_scratch(size_t lanes, int depth, int slots, hipStream_t s);
    int ensure_tallies(int64_t nv, hipStream_t s);
    int ensure_stage(int64_t nv, hipStream_t s);
    int launch_shape(const mcd_opts* o, int n_mat, int* blocks, int* threads);
    void fill_params(mcd::KParams& p, const mcd::PhantomRec& ph, const mcd::DevSource& ds,
                     uint64_t seed, uint32_t key, uint64_t first, uint64_t n);
    void shutdown_serving() {}
};
