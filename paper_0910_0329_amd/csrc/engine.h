// Internal interface between the host runtime and the device kernels of
// libmcdose.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcd {

constexpr int kNE = 512;          // energy nodes of every table
constexpr int kMaxMat = 8;        // materials per table set on the device
constexpr int kCounters = 32;
constexpr int kBal = 6;           // e_src, e_csda, e_local, e_esc, e_miss, track_e
constexpr int kStackRec = 48;     // bytes per stacked particle

// Device-side tables of one material set (FP32, converted from the FP64 blob).
//   phot[m*512 + i] = (mu_C/rho, mu_pe/rho, mu_pp/rho, 0)   cm^2/g
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
};

// Source descriptor as the kernel sees it.
struct DevSource {
    int particle, energy_kind, beam_kind, n_bins;
    float e0;
    float pos[3];
    float field[4];
    float edges[65];
    float cdf[64];
    double extra;           // 2 m c^2 for positron primaries, else 0
};

// Everything one transport launch needs.
struct KParams {
    DevTables t;
    const float* maj;        // [512] majorant attenuation of the phantom, 1/cm
    const uint2* vox;        // per voxel: (float bits of rho, material index)
    int nx, ny, nz;
    float dx, dy, dz, x0, y0, z0, x1, y1, z1, idx, idy, idz;
    DevSource src;
    uint32_t seed, key;
    uint32_t first, n;       // history range [first, first + n)
    double* S;               // per-voxel sum of per-history energy, MeV
    double* Q;               // per-voxel sum of its square, MeV^2
    double* bal;             // [kBal]
    unsigned long long* cnt; // [kCounters]
    int* err;                // 0 ok, else an mcd_status
    unsigned long long* next; // work counter: next history offset
    char* scratch;           // per-lane stack and local counter
    int stack_depth;
    int slots;               // local counter slots, power of two
    int lockstep;            // 1: all lanes of a wave run the same history
    size_t lane_bytes;
    void* hist;              // mcd_history_record[n] or null
};

size_t lane_scratch_bytes(int stack_depth, int slots);

// Launchers (kernels.hip).
hipError_t launch_transport(const KParams& p, int blocks, int threads, bool diag, hipStream_t s);
hipError_t launch_finalize(const double* S, const double* Q, const uint2* vox, int64_t nv,
                           double vol, uint64_t n, double* dose, double* sigma, double* red,
                           hipStream_t s);
hipError_t launch_clear_lane_keys(char* scratch, size_t lanes, size_t lane_bytes, int stack_depth,
                                  int slots, hipStream_t s);
hipError_t launch_fill_u32(void* p, size_t n_words, uint32_t v, hipStream_t s);
int transport_lds_bytes(int n_mat);

}  // namespace mcd
