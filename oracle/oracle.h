/*
 * FP64 reference ("oracle") for the coupled electron-photon Monte Carlo dose
 * computation of Jia et al., "Development of a GPU-based Monte Carlo dose
 * calculation code for coupled electron-photon transport" (DPM scheme, Sec. 2.1;
 * per-history flow of Fig. 1 / Sec. 2.2; local counter and dose collection,
 * Sec. 2.4; uncertainty estimate, Sec. 3).
 *
 * TEST INFRASTRUCTURE ONLY.  This code is plain, slow and single-threaded on
 * purpose.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it; the product path never does.  It shares no source
 * with the GPU library: it parses the table blob, interpolates, builds the
 * majorant, draws Philox numbers and transports particles with its own code.
 *
 * Conventions: cm, MeV, g, g/cm^3.  Arrays over voxels are x-fastest
 * (index = (k*ny + j)*nx + i).  All functions return 0 on success and a
 * negative code on invalid input (-1); outputs are then left untouched.
 */
#ifndef MCD_ORACLE_H
#define MCD_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t nx, ny, nz;
    double dx, dy, dz;
    double x0, y0, z0;  /* corner of the box; the top face is z = z0 */
} orc_grid;

typedef struct {
    int32_t particle;      /* 0 photon, 1 electron, 2 positron */
    int32_t energy_kind;   /* 0 mono, 1 histogram */
    int32_t beam_kind;     /* 0 pencil along +z, 1 point source with a field */
    int32_t n_bins;        /* histogram bins, <= 64 */
    double e0;             /* MeV, mono */
    double pos[3];         /* pencil: entry (x, y) on the top face; point: source point */
    double field[4];       /* centre x, centre y, half-width x, half-width y on z = z0 */
    double edges[65];
    double weights[64];
} orc_source;

/* Energy-balance channels (MeV), accumulated (+=) by orc_simulate. */
enum { ORC_E_SRC, ORC_E_CSDA, ORC_E_LOCAL, ORC_E_ESC, ORC_E_MISS, ORC_TRACK_E, ORC_NBAL };

/* Event counters, accumulated (+=) by orc_simulate. */
enum {
    ORC_C_HISTORIES, ORC_C_FLIGHTS, ORC_C_VIRTUAL, ORC_C_COMPTON, ORC_C_PHOTO, ORC_C_PAIR,
    ORC_C_SEGMENTS, ORC_C_SEG_E, ORC_C_SEG_H, ORC_C_SEG_K, ORC_C_SEG_B, ORC_C_SEG_F,
    ORC_C_HINGES, ORC_C_MOLLER, ORC_C_BREMS, ORC_C_SPAWNS, ORC_C_PHILOX, ORC_C_FLUSHES,
    ORC_C_ESCAPES, ORC_C_MISSES, ORC_C_LOCAL, ORC_C_VOID, ORC_C_COMPTON_TRIES,
    ORC_C_MOLLER_TRIES, ORC_C_MAX_STACK, ORC_C_RAYLEIGH, ORC_C_BHABHA, ORC_NCOUNT = 32
};

/* Optional per-history record: total deposited energy, total electron track
 * length, and an order-independent hash of every particle's event sequence. */
typedef struct {
    double edep;
    double track_e;
    uint64_t hash;
    uint32_t n_particles;
    uint32_t escaped;     /* 1 if any particle of the history left the box */
} orc_history;

/* Philox4x32-10 (Salmon et al., SC'11): out = bijection(ctr) under key (k0, k1). */
void orc_philox(uint32_t k0, uint32_t k1, const uint32_t ctr[4], uint32_t out[4]);

/* u = ((x >> 9) + 0.5) * 2^-23, in (0, 1) and exact in FP32 and FP64. */
double orc_uniform(uint32_t x);

/* Validates a table blob; returns the number of materials or -1. */
int orc_blob_check(const void* blob, size_t nbytes);

/* Linear-in-ln(E) interpolation of quantity q of material m (clamped grid). */
int orc_interp(const void* blob, size_t nbytes, int m, int q, double e, double* out);

/* Inverse of the interpolated range of material m: T with R(T) = r. */
int orc_range_inverse(const void* blob, size_t nbytes, int m, double r, double* out);

/* Array forms of the three functions above, for tests that compare many
 * points: n counters (4 words each, out likewise); n energies; n ranges, with
 * q the range quantity to invert (3: electron range R, 10: positron range). */
void orc_philox_n(uint32_t k0, uint32_t k1, const uint32_t* ctr, size_t n, uint32_t* out);
int orc_interp_n(const void* blob, size_t nbytes, int m, int q, const double* e, size_t n, double* out);
int orc_range_inverse_n(const void* blob, size_t nbytes, int m, int q, const double* r, size_t n,
                        double* out);

/* Majorant attenuation mu_max(E_i) (1/cm) at the 512 grid nodes. */
int orc_majorant(const void* blob, size_t nbytes, const orc_grid* g, const uint8_t* mat,
                 const float* rho, double* out512);

/* Transport histories [first, first + n) and accumulate the dose tallies
 * S[v] += sum_h e_{h,v}, Q[v] += sum_h e_{h,v}^2 (MeV, MeV^2).  `bal` has
 * ORC_NBAL entries, `cnt` ORC_NCOUNT; `hist` (n entries) may be NULL; `Sb`
 * (16 x nv, or NULL) accumulates the group tallies, history h into group
 * h mod 16. */
int orc_simulate(const void* blob, size_t nbytes, const orc_grid* g, const uint8_t* mat,
                 const float* rho, const orc_source* src, uint64_t first, uint64_t n,
                 uint32_t seed, uint32_t request_key, double* S, double* Q, double* bal,
                 uint64_t* cnt, orc_history* hist, double* Sb);

/* Depth z of the primary photon's first real interaction for each history of a
 * photon source (+inf when it escapes first, NaN when it misses the phantom),
 * and (if kind_out) its kind: 2 Compton, 3 photoelectric, 4 pair, 6 escape.
 * For transmission and branching checks. */
int orc_first_interaction(const void* blob, size_t nbytes, const orc_grid* g,
                          const uint8_t* mat, const float* rho, const orc_source* src,
                          uint64_t n, uint32_t seed, uint32_t request_key, double* z_out,
                          int32_t* kind_out);

/* Sampler checks: n independent samples, sample i drawn from stream (seed, 0, i)
 * with the transport's own draw order, written as 8 doubles out[8 i ..]:
 *   which 0  Compton at photon energy e: cos(theta), E'/E, photon direction,
 *            electron direction (both rotated from a fixed oblique direction)
 *   which 1  hard Moller at kinetic energy e: W/T, cos(theta_delta), primary
 *            direction, delta-ray direction
 *   which 2  hard bremsstrahlung at kinetic energy e: W
 *   which 3  random hinge: cos(theta), 0, new direction
 *   which 4  Sauter photoelectron angle at kinetic energy e: cos(theta)
 *   which 5  forward emission angle (bremsstrahlung photon, pair lepton) for
 *            an emitter of kinetic energy e: cos(theta)
 *   which 6+m  Rayleigh angle at photon energy e in material m: cos(theta)
 *   which 256+m  second-moment hinge at electron energy e in material m:
 *            cos(theta), lambda1/lambda2
 *   which 512  Bhabha event of a positron of kinetic energy e: fraction of e
 *            given to the electron                                            */
int orc_sample(const void* blob, size_t nbytes, int which, double e, uint64_t n, uint32_t seed,
               double* out);

/* Finalisation (Sec. 3): dose and standard deviation per voxel in Gy per
 * source history, Dmax and sigma-bar (mean sigma/D over voxels with D > Dmax/2). */
int orc_finalize(const orc_grid* g, const float* rho, const double* S, const double* Q,
                 uint64_t n, double* dose, double* sigma, double* dmax, double* sigma_bar);

/* Finalisation with group statistics: dose from the summed group tallies and
 * sigma from the spread of the 16 group means (nb[b] histories in group b). */
int orc_finalize_groups(const orc_grid* g, const float* rho, const double* Sb, const double* nb,
                        double* dose, double* sigma, double* dmax, double* sigma_bar);

#ifdef __cplusplus
}
#endif
#endif
