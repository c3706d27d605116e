// Internal interface between the host runtime and the device kernels of
// libmcdose.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcd {

constexpr int kNE = 512;          // energy nodes of every table
constexpr int kMaxMat = 8;        // materials per table set on the device
constexpr int kCounters = 40;
constexpr int kBal = 6;           // e_src, e_csda, e_local, e_esc, e_miss, track_e
constexpr int kRec = 48;          // bytes per stacked or queued particle
constexpr int kBatches = 16;      // sub-tallies of the batch-statistics tally (power of two)

// Device-side tables of one material set (FP32, converted from the FP64 blob).
//   phot[m*512 + i] = (mu_C/rho, mu_pe/rho, mu_pp/rho, mu_R/rho)   cm^2/g
//   (mu_R, coherent scattering, is zero unless the tables carry it)
//   elec[m*512 + i] = (R, 1/(lambda1 rho), Sigma_M/rho, Sigma_B/rho)
struct DevTables {
    float4* phot;
    float4* elec;
    float r_abs[kMaxMat];   // R(E_abs,e) per material
    int n_mat;
    float l2_emin;          // log2(E_0)
    float inv_dl2;          // 1 / (log2 step of the grid)
    float dl2;              // log2 step of the grid
    float emin, emax;
    float e_abs_e, e_abs_g, w_cc, w_cr, kappa_step, f_e, a_hinge;
    float f_shift;          // log2(1 - f_e) / (log2 step): (1 - f_e) E is this many nodes below E
    int angular;            // 1: emission angles for photoelectrons, brems photons, pair leptons
    float ray_b[kMaxMat];   // Rayleigh form-factor scale: b = ray_b[m] E^2 (1/MeV^2)
    const float4* hinge;    // [m*512 + i] = (A, B, S, 0) of the second-moment hinge law
    int hinge2;             // 1: hinge angles from the second-moment law
    const float2* posi;     // [m*512 + i] = (R+, Sigma_Bh/rho): positron range and hard Bhabha
    float r_abs_pos[kMaxMat];  // R+(E_abs,e) per material
    int bhabha;             // 1: positrons take posi and Bhabha events
    int refined;            // any of angular, hinge2, bhabha or mu_R > 0: the kernels
                            // built with the refinement code must run
};

// Source descriptor as the kernels see it.
struct DevSource {
    int particle, energy_kind, beam_kind, n_bins;
    float e0;
    float pos[3];
    float field[4];
    float edges[65];
    float cdf[64];
    double extra;           // 2 m c^2 for positron primaries, else 0
};

// Wave schedule of the transport loop (thresholds, see Transport::run).
struct Sched {
    int fetch_div;           // fetch when >= 1/fetch_div of the live lanes need a particle
    int hard_div;            // sample hard events when >= 1/hard_div of the live lanes wait
    int photon_div;          // photon flights when photons >= electrons / photon_div
    int fetch_photon_div;    // wave stacks: fetch_div while the wave is in photon mode
    int segments;            // wave stacks: segments an electron step may run
};

// Tables and phantom of a launch.
struct KGeom {
    DevTables t;
    const float* maj;        // [512] majorant attenuation of the phantom, 1/cm
    const uint2* vox;        // per voxel: (float bits of rho, material index)
    int nx, ny, nz;
    float dx, dy, dz, x0, y0, z0, x1, y1, z1, idx, idy, idz;
};

// Plain per-history kernel: one lane follows one history at a time with an
// exact history-by-history local counter.
struct KPlain {
    KGeom g;
    DevSource src;
    uint32_t seed, key;
    uint32_t first, n;       // history range [first, first + n)
    double* S;               // per-voxel sum of per-history energy, MeV
    double* Q;               // per-voxel sum of its square, MeV^2
    double* bal;             // [kBal]
    unsigned long long* cnt; // [kCounters]
    int* err;                // 0 ok, else an mcd_status
    unsigned long long* next;// work counter: next history offset
    char* scratch;           // per-lane stack and local counter
    int stack_depth;
    int slots;               // local counter slots, power of two
    size_t lane_bytes;
    void* hist;              // mcd_history_record[n] or null
    int lockstep;            // 1: all lanes of a wave run the same history
    Sched sched;
};

// One request of a regrouped launch (device copy).
struct ReqDev {
    DevSource src;
    uint32_t seed, key;
    uint32_t first, n;       // history range
    uint64_t lo;             // index of its first history in the launch's work list
    void* tally;             // kBatches sub-tallies of nv voxels (double or float)
    void* hist;              // mcd_history_record[n] or null (diagnostics)
};

// Queue control words: count (particles appended), head (particles taken).
struct QCtl {
    unsigned int count, head, pad0, pad1;
};

// One phase of a regrouped cycle: the photon phase takes photons queued by the
// previous electron phase plus new histories; the electron phase takes the
// electrons the photon phase queued.  Cross-type secondaries go to the other
// type's queue (or, when it is full, stay on the lane's own stack).
struct KPhase {
    KGeom g;
    const ReqDev* req;
    int n_req;
    int tally_fp32;
    uint64_t total;          // histories in the launch
    uint64_t chunk;          // new histories per cycle
    uint32_t cycle;
    unsigned int* claim;     // per-cycle claim counters
    const char* q_in;        // queue consumed by this phase
    QCtl* q_in_ctl;
    char* q_out;             // queue of the other particle type, appended to
    QCtl* q_out_ctl;
    QCtl* q_reset_ctl;       // control block zeroed at the start of this phase
    unsigned int q_cap;      // capacity of every queue buffer (particles)
    int use_queues;          // 0: cross-type secondaries stay on the lane stack
    int64_t nv;
    double* bal;
    unsigned long long* cnt;
    int* err;
    char* scratch;           // per-lane particle stacks
    int stack_depth;
    size_t lane_bytes;
    Sched sched;
};

size_t plain_lane_bytes(int stack_depth, int slots);
size_t phase_lane_bytes(int stack_depth);
size_t wave_stack_bytes(int cap);
int transport_lds_bytes(int n_mat);

// Launchers.
// Both launchers pick the kernel built for the tables' refinements (p.g.t.refined).
hipError_t launch_plain(const KPlain& p, int blocks, int threads, bool diag, hipStream_t s);
hipError_t launch_phase(const KPhase& p, bool photons, int blocks, int threads, bool diag,
                        hipStream_t s);
// gtab: photon and electron tables read from device memory, not LDS.
hipError_t launch_wave(const KPhase& p, int blocks, int threads, bool diag, bool gtab, hipStream_t s);
// LDS bytes per workgroup of the wave-stack kernel, and the workgroups of
// `threads` threads one CU holds at once (registers and LDS; 0 on error).
int wave_lds_bytes(int n_mat, bool gtab);
int wave_blocks_per_cu(int threads, int n_mat, bool gtab);
hipError_t launch_finalize(const double* S, const double* Q, const uint2* vox, int64_t nv,
                           double vol, uint64_t n, double* dose, double* sigma, double* red,
                           hipStream_t s);
// Batch-statistics finalisation of n_req tallies (kBatches sub-tallies each).
struct FinalReq {
    const void* tally;
    double* S;               // sum of the sub-tallies, or null
    double* dose;
    double* sigma;
    double* red;             // [3]: Dmax bits, sum sigma/D, count
    double nb[kBatches];     // histories per sub-tally
};
hipError_t launch_finalize_batches(const FinalReq* reqs, int n_req, const uint2* vox,
                                   int64_t nv, double vol, int fp32, hipStream_t s);
hipError_t launch_clear_lane_keys(char* scratch, size_t lanes, size_t lane_bytes, int stack_depth,
                                  int slots, hipStream_t s);
hipError_t launch_fill_u32(void* p, size_t n_words, uint32_t v, hipStream_t s);
// Sets the dynamic-LDS limit of the transport kernels (once, before any launch
// or graph capture).
hipError_t init_kernels(int max_lds);
hipError_t init_plain_kernels(int max_lds);
hipError_t init_phase_kernels(int max_lds);
hipError_t init_check_kernels(int max_lds);
hipError_t init_wave_kernels(int max_lds);

}  // namespace mcd
