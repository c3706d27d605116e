/*
 * mcdose: coupled electron-photon Monte Carlo dose engine for AMD Instinct
 * MI355X (gfx950).  C ABI of libmcdose.so.
 *
 * The engine computes what Jia et al. (arXiv:0910.0329) move to a GPU: the DPM
 * transport scheme of Sec. 2.1 (Woodcock photon tracking; condensed-history
 * electrons with continuous slowing down below the production thresholds and
 * detailed hard Moller/bremsstrahlung events above them) run history by
 * history as in the flow of Fig. 1 / Sec. 2.2, with a per-history local
 * counter collected into a global dose counter (Sec. 2.4) and the uncertainty
 * estimate of Sec. 3.
 *
 * Conventions
 *   - Units: cm, MeV, g, g/cm^3; dose in Gy per source history.
 *   - Voxel arrays are x-fastest: v = (k * ny + j) * nx + i.
 *   - Every function returns an mcd_status (0 = OK, negative = error) and
 *     mcd_last_error() explains an error.  On error no handle (mcd_create
 *     sets its handle to NULL), host result field or host array is written,
 *     except that a HIP failure during the copy of results (MCD_E_DEVICE) may
 *     leave output arrays partly written; device buffers the caller passed as
 *     outputs (dose and sigma written in place, history records) may hold
 *     partial data after any error.  No C++ exception or abort crosses this
 *     interface.
 *   - Host pointers are read during the call and may be freed on return.
 *   - Device pointers are HIP device addresses on the context's device.
 *     Entry points make that device current while they run and give the
 *     calling thread back its own current device before returning.
 *   - Calls on one context may come from several threads: blocking runs and
 *     serving epochs take turns on the device; table and phantom loads wait
 *     for the run in progress.  mcd_destroy must not overlap other calls.
 */
#ifndef MCDOSE_H
#define MCDOSE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MCD_OK = 0,
    MCD_E_INVAL = -1,     /* invalid argument (sizes, ranges, table or phantom content) */
    MCD_E_NOMEM = -2,     /* device allocation failed or would exceed the HBM budget */
    MCD_E_NOTFOUND = -3,  /* unknown table, phantom or ticket handle */
    MCD_E_OVERFLOW = -4,  /* particle stack or per-history local counter overflowed */
    MCD_E_DEVICE = -5,    /* HIP runtime error (message in mcd_last_error) */
    MCD_E_BUSY = -6,      /* request not finished yet */
    MCD_E_CANCELED = -7   /* request was cancelled */
} mcd_status;

typedef struct mcd_ctx mcd_ctx;

/* Voxel grid: nx*ny*nz voxels of dx*dy*dz cm; the box spans
 * [x0, x0 + nx dx) x [y0, y0 + ny dy) x [z0, z0 + nz dz); its top face z = z0
 * faces the source. */
typedef struct {
    int32_t nx, ny, nz;
    double dx, dy, dz;
    double x0, y0, z0;
} mcd_grid;

enum { MCD_PHOTON = 0, MCD_ELECTRON = 1, MCD_POSITRON = 2 };
enum { MCD_MONO = 0, MCD_HISTOGRAM = 1 };
enum { MCD_PENCIL = 0, MCD_POINT_FIELD = 1 };
#define MCD_MAX_BINS 64

/* Source model (Sec. 3: point sources with a rectangular field, a
 * monoenergetic electron beam or a photon spectrum).
 *   pencil      enters the top face at (pos[0], pos[1]) along +z;
 *   point-field from the point pos towards a point drawn uniformly on the
 *               rectangle centred at (field[0], field[1]) with half-widths
 *               (field[2], field[3]) on the plane z = z0; primaries whose
 *               entry point is outside the top face miss the phantom.
 * Energies: mono e0, or a histogram of n_bins bins (edges[0..n_bins],
 * weights[0..n_bins-1], any positive scale); 0 < E <= 20 MeV. */
typedef struct {
    int32_t particle;      /* MCD_PHOTON, MCD_ELECTRON, MCD_POSITRON */
    int32_t energy_kind;   /* MCD_MONO, MCD_HISTOGRAM */
    int32_t beam_kind;     /* MCD_PENCIL, MCD_POINT_FIELD */
    int32_t n_bins;
    double e0;
    double pos[3];
    double field[4];
    double edges[MCD_MAX_BINS + 1];
    double weights[MCD_MAX_BINS];
} mcd_source;

/* Energy bookkeeping of a run, MeV (FP64 sums on the device). */
typedef struct {
    double e_src;    /* source energy (a positron counts T + 2 m c^2) */
    double e_csda;   /* continuous-slowing-down deposits */
    double e_local;  /* below-cutoff deposits on the spot */
    double e_esc;    /* energy carried out of the box */
    double e_miss;   /* primaries that missed the phantom */
    double track_e;  /* total electron path length, cm */
} mcd_energy_balance;

/* Event counters (filled when mcd_opts.diagnostics != 0). */
enum {
    MCD_C_HISTORIES, MCD_C_FLIGHTS, MCD_C_VIRTUAL, MCD_C_COMPTON, MCD_C_PHOTO, MCD_C_PAIR,
    MCD_C_SEGMENTS, MCD_C_SEG_E, MCD_C_SEG_H, MCD_C_SEG_K, MCD_C_SEG_B, MCD_C_SEG_F,
    MCD_C_HINGES, MCD_C_MOLLER, MCD_C_BREMS, MCD_C_SPAWNS, MCD_C_PHILOX, MCD_C_FLUSHES,
    MCD_C_ESCAPES, MCD_C_MISSES, MCD_C_LOCAL, MCD_C_VOID, MCD_C_COMPTON_TRIES,
    MCD_C_MOLLER_TRIES, MCD_C_MAX_STACK,
    /* wave schedule: iterations of the transport loop (summed over waves),
     * live lanes summed over them, and per kind of work (fetch, photon flight,
     * electron segment, hard event) the iterations that ran it and the lanes
     * that took part */
    MCD_C_ITERS, MCD_C_LIVE, MCD_C_IT_FETCH, MCD_C_IT_PHOTON, MCD_C_IT_ELECTRON, MCD_C_IT_HARD,
    MCD_C_LN_FETCH, MCD_C_LN_PHOTON, MCD_C_LN_ELECTRON, MCD_C_LN_HARD,
    MCD_C_RAYLEIGH,  /* coherent scatterings (tables with the Rayleigh flag) */
    MCD_C_BHABHA,    /* hard Bhabha events (tables with the Bhabha flag) */
    MCD_NCOUNT = 40
};

/* Per-history diagnostic record (mcd_opts.history_records). */
typedef struct {
    double edep;          /* energy deposited by the history, MeV */
    double track_e;       /* electron path length of the history, cm */
    uint64_t hash;        /* order-independent hash of its particles' event sequences */
    uint32_t n_particles;
    uint32_t escaped;
} mcd_history_record;

/* Transport kernels.
 *   MCD_KERNEL_REGROUPED  particles regrouped by type into photon and electron
 *                         phases with device queues; batch statistics (the
 *                         histories form 16 groups, history mod 16, and sigma
 *                         comes from the spread of the group means).
 *   MCD_KERNEL_PLAIN      one lane per history with its own secondary stack
 *                         and an exact history-by-history local counter
 *                         (sigma from the per-history second moment).      */
enum { MCD_KERNEL_REGROUPED = 0, MCD_KERNEL_PLAIN = 1 };
/* mcd_opts.table_placement */
enum { MCD_TABLES_AUTO = 0, MCD_TABLES_LDS = 1, MCD_TABLES_GLOBAL = 2 };

/* Run options; NULL means defaults.  None of them changes which histories are
 * simulated or how: the histories depend only on (tables, phantom, source,
 * history range, seed, request key); the kernel choice selects the
 * uncertainty estimator and the tally precision selects FP64 or FP32 sums. */
typedef struct {
    uint64_t first_history;   /* histories [first_history, first_history + n) */
    int32_t block_size;       /* threads per block, 0 = tuned default */
    int32_t grid_blocks;      /* blocks, 0 = enough to fill the device (with the wave-stack
                                 schedule: the number of workgroups the device holds at
                                 once, from the kernel's registers and LDS) */
    int32_t stack_depth;      /* particle stack per lane, 0 = default (64) */
    int32_t tally_slots;      /* plain kernel: local counter slots (power of 2), 0 = 512 */
    int32_t diagnostics;      /* 1: fill counters (slower kernel variant) */
    int32_t accumulate;       /* 1: add to the tallies of the previous call instead of clearing */
    void* history_records;    /* device array of n mcd_history_record, or NULL */
    int32_t lockstep;         /* plain kernel, measurement mode: all 64 lanes of a wave replay the
                                 same history, so the wave executes that history's instruction
                                 path without divergence; tallies then count each history 64 times */
    int32_t kernel;           /* MCD_KERNEL_REGROUPED (default) or MCD_KERNEL_PLAIN */
    int32_t tally_fp32;       /* regrouped kernel: FP32 instead of FP64 dose accumulators */
    int32_t chunk_per_lane;   /* regrouped kernel with queues (regroup 1): new histories per lane
                                 and cycle, 0 = 16; with lane stacks one launch takes them all */
    int32_t use_graph;        /* regrouped kernel: capture the launch sequence in a hipGraph
                                 and replay it when the same call is repeated */
    int32_t regroup;          /* regrouped kernel schedule: 0 = default (3), 1 = cross-type
                                 secondaries go through the photon/electron queues, 2 = they
                                 stay on the lane's own stack (one lane transports a whole
                                 history; the phases then only split new histories), 3 = the
                                 secondaries of a wave's 64 lanes go on two stacks of the wave,
                                 one per particle type; the wave runs in a photon or an
                                 electron mode, and lanes holding the other kind park their
                                 particle mid-flight and take a waiting one of the mode's kind
                                 (stacks of 16 x stack_depth records per wave) */
    /* Wave schedule of both kernels: each iteration a wave runs one kind of
     * step for the lanes that need it.  Fetching a particle runs when at
     * least 1/fetch_div of the wave's live lanes need one, sampling hard
     * events when 1/hard_div wait for it, photon flights when photons are at
     * least electrons/photon_div; else electron segments.  1..64, 0 = default:
     * plain kernel (3, 24, 2); regrouped kernel with lane stacks or queues
     * (3, 24, 2) when every source is a photon source, else (4, 8, 6); with
     * wave stacks (regroup 0 or 3) (16, 24, 1) or (16, 64, 1), where
     * photon_div instead sets the mode switch (the mode's work below
     * 64 / photon_div lanes) and fetch_div holds in electron mode only. */
    int32_t sched_fetch_div;
    int32_t sched_hard_div;
    int32_t sched_photon_div;
    int32_t refined_build;    /* 1: run the transport kernels built with the refinement code
                                 even when the tables use none of it (the same histories;
                                 a check of the lean build).  0 = pick by the tables */
    int32_t table_placement;  /* where the transport reads the photon and electron tables
                                 (32 B per material and energy node, Sec. 2.3):
                                 MCD_TABLES_LDS = a copy in each workgroup's LDS;
                                 MCD_TABLES_GLOBAL = device memory, through the L1 and L2
                                 caches, which leaves the LDS free (wave-stack schedule,
                                 regroup 0 or 3, only; other schedules return MCD_E_INVAL);
                                 MCD_TABLES_AUTO (0, default) = the LDS unless its copy lets
                                 a CU hold fewer workgroups than device-memory tables do
                                 (large table sets), then device memory; the other
                                 schedules always use the LDS.  The histories are the same
                                 either way. */
    int32_t sched_fetch_photon_div; /* wave stacks (regroup 0 or 3): the fetch threshold
                                 while the wave is in photon mode (1/this of its live
                                 lanes need a particle); 1..64, 0 = default 2.  Ignored
                                 by the other schedules. */
    int32_t sched_segments;   /* wave stacks (regroup 0 or 3): condensed-history segments
                                 an electron step may run before the wave's next schedule
                                 decision (a lane stops early at a hard event or at its
                                 particle's end); 1..64, 0 = default 12.  Ignored by the
                                 other schedules.  The histories do not depend on it. */
} mcd_opts;

/* Output of a run.  dose and sigma (nx*ny*nz doubles each, Gy per source
 * history) and S, Q (raw tallies: sum over histories of the per-history
 * energy in a voxel and of its square, MeV and MeV^2; Q only with the plain
 * kernel) are caller-allocated and optional (NULL to skip); they are device
 * pointers when on_device != 0, host pointers otherwise.  The scalars are
 * filled on return. */
typedef struct {
    double* dose;
    double* sigma;
    double* S;
    double* Q;
    int32_t on_device;
    mcd_energy_balance eb;
    uint64_t counters[MCD_NCOUNT];
    double dmax;          /* maximum dose, Gy per history */
    double sigma_bar;     /* mean sigma/D over voxels with D > dmax / 2 (Sec. 3) */
    double kernel_ms;     /* device time of the transport kernel(s) */
    double total_ms;      /* device time from tally clear to finalisation */
    int32_t launches;     /* transport kernel launches of the run */
    int32_t reserved;
    uint64_t n_histories; /* histories behind dose and sigma */
} mcd_result;

/* Creates a context on HIP device `device`.  hbm_budget_bytes caps what the
 * context allocates (0: 90% of the free device memory at creation). */
int mcd_create(int device, uint64_t hbm_budget_bytes, mcd_ctx** out);
int mcd_destroy(mcd_ctx* ctx);

/* Loads a physics table blob (cross sections per interaction, material and
 * energy, Sec. 2.2; format: magic "MCDTAB\0\1", version 4, 512-node log grid
 * from 1 keV to 20 MeV, 13 quantities per material, at most 8 materials).
 * Header flags select physics refinements beyond the paper's scheme:
 *   4  emission angles (Sauter photoelectrons, forward-peaked bremsstrahlung
 *      photons and pair leptons),  8  density effect (tables only),
 *   16 Rayleigh scattering (mu_R tabulated),
 *   32 hinge angles matching the second Lewis moment (from lambda2),
 *   64 positrons with their own range and hard Bhabha events;
 * 1 and 2 mark test tables.  Other bits are rejected.  The blob is validated
 * (sizes, monotone ranges, non-negative finite values, scalar ranges) and
 * converted to FP32 device tables.  *out_tables receives a handle; the blob
 * stays the caller's.  Errors: MCD_E_INVAL for a malformed blob, MCD_E_NOMEM
 * past the HBM budget. */
int mcd_load_materials(mcd_ctx* ctx, const void* blob, size_t nbytes, int32_t* out_tables);
int mcd_unload_materials(mcd_ctx* ctx, int32_t tables);

/* Uploads a voxel phantom (the slab phantoms of Sec. 3 are voxel grids of
 * materials and densities; the Woodcock tracking of Sec. 2.1 needs the
 * majorant attenuation over them): material index per voxel, u8, < number of
 * materials; density per voxel, f32 > 0; both host arrays of nx*ny*nz, read
 * during the call.  The phantom is bound to a table set and its Woodcock
 * majorant is built (max over materials present of rho mu(E), rounded up to
 * FP32).  It stays resident until unloaded.  *out_phantom receives a handle.
 * Errors: MCD_E_INVAL (grid sizes or spacings, material index out of range,
 * density not finite and > 0), MCD_E_NOTFOUND (tables), MCD_E_NOMEM. */
int mcd_load_phantom(mcd_ctx* ctx, const mcd_grid* grid, const uint8_t* mat, const float* rho,
                     int32_t tables, int32_t* out_phantom);
/* Frees a phantom.  MCD_E_BUSY while served requests on it are not all
 * collected by mcd_wait (whatever their state), MCD_E_NOTFOUND for an unknown
 * handle.  Waits for the device run in progress. */
int mcd_unload_phantom(mcd_ctx* ctx, int32_t phantom);

/* Transports n_histories source histories through a phantom and returns the
 * dose and its uncertainty (Fig. 1 flow: source particle, transport, secondary
 * stack, dose collection).  seed and request_key key the Philox4x32-10 streams
 * (seed < 2^32, request_key < 2^32, first_history + n_histories <= 2^32).
 * Blocking: returns when the results are in `out`.  hip_stream may be a
 * hipStream_t (e.g. torch's current stream) or NULL for the context's stream.
 * The caller owns every buffer in `out` (host or device per out->on_device).
 * Errors: MCD_E_INVAL (arguments, options), MCD_E_NOTFOUND (handle),
 * MCD_E_NOMEM (HBM budget), MCD_E_OVERFLOW (particle stack or local counter:
 * raise stack_depth / tally_slots), MCD_E_DEVICE (HIP error); mcd_last_error
 * gives the message.  On error the scalar fields of `out` are untouched;
 * device-resident dose and sigma buffers may hold partial values. */
int mcd_simulate(mcd_ctx* ctx, int32_t phantom, const mcd_source* src, uint64_t n_histories,
                 uint64_t seed, uint32_t request_key, const mcd_opts* opts, mcd_result* out,
                 void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * regrouped run of mcd_simulate with lane stacks, calling no hipMalloc or
 * hipFree.  Every buffer beyond the inputs and outputs (run scalars, counters,
 * request tables, the 16 sub-tallies, the lane stacks) lives in a device array
 * of 512 MiB that the library holds on each device it runs on until the
 * process ends.  The run must fit in it: 16 x nv tally words (8 bytes, or 4
 * with tally_fp32) plus grid lanes x stack_depth x 48 bytes (each lane's
 * share rounded up to 256 bytes; stack_depth 0 means 26 here) plus a few KB;
 * otherwise MCD_E_INVAL names the size needed.  With the default launch shape
 * of a 256-CU device (262144 lanes, 320 MiB of stacks) that leaves room for
 * 1.5e6 voxels with FP64 sums or 3.1e6 with FP32 sums; fewer grid_blocks or a
 * smaller stack_depth leave more.  A particle stack that
 * overflows ends the run with MCD_E_OVERFLOW (raise stack_depth).
 * out->dose and out->sigma must be device buffers (out->on_device = 1); S is
 * optional and Q is refused.  opts as for mcd_simulate, except that kernel
 * must be MCD_KERNEL_REGROUPED, regroup 0 or 2, use_graph and accumulate 0.
 * The histories and results equal mcd_simulate's with the same arguments and
 * regroup 2 (its lane-stack run), up to FP64 summation order; its default
 * wave-stack run follows the same histories, with deposits that can differ in
 * the last bits.  Calls on one device share the array: the library
 * runs them one at a time (calls that overlap from several threads or
 * contexts wait for each other). */
int mcd_simulate_noalloc(mcd_ctx* ctx, int32_t phantom, const mcd_source* src, uint64_t n_histories,
                         uint64_t seed, uint32_t request_key, const mcd_opts* opts, mcd_result* out,
                         void* hip_stream);

/* One beam or beamlet of a batched call. */
typedef struct {
    mcd_source src;
    uint64_t n_histories;
    uint32_t request_key;
    uint32_t reserved;
    mcd_result* out;          /* per-item dose/sigma/S outputs and dmax, sigma_bar (eb and
                                 counters are reported for the whole batch in `total`) */
} mcd_batch_item;

/* Runs many sources with uneven history counts on one phantom in one
 * regrouped launch sequence (one hipGraph launch when opts->use_graph), in
 * place of the batch-by-batch kernel relaunches of Sec. 2.2:
 * their histories share the photon and electron phases, each item keeps its
 * own tally.  Every item's result equals what mcd_simulate returns for it
 * alone with the same seed and request key (up to FP64 summation order).
 * n_items <= 4096; the sum of n_histories < 2^40. */
int mcd_simulate_batch(mcd_ctx* ctx, int32_t phantom, const mcd_batch_item* items, int32_t n_items,
                       uint64_t seed, const mcd_opts* opts, mcd_result* total, void* hip_stream);

/* The launch shape a run on `phantom` with `opts` (NULL = defaults) takes:
 * workgroups (`*grid_blocks`, the default when opts->grid_blocks is 0) of
 * `*block_size` threads, the device's compute units (`*cu_count`), the
 * workgroups one CU holds at once for that kernel (`*resident_per_cu`, from
 * its registers and LDS; the wave-stack kernel only, else 0) and the table
 * placement MCD_TABLES_AUTO resolves to (`*table_placement`, LDS or GLOBAL).
 * Options are validated as mcd_simulate does; nothing runs.  For tuning the
 * occupancy (waves per CU) of a persistent launch. */
int mcd_launch_shape(mcd_ctx* ctx, int32_t phantom, const mcd_opts* opts, int32_t* grid_blocks,
                     int32_t* block_size, int32_t* cu_count, int32_t* resident_per_cu,
                     int32_t* table_placement);

/* ------------------------------------------------------------------ serving
 *
 * Requests submitted from any thread are transported by a worker thread of
 * the context.  Arriving requests wait in a queue (QUEUED) until their device
 * memory fits the HBM budget (ADMITTED): a batch-statistics tally of 16 x nv
 * accumulators plus dose and sigma (nv doubles each), so a 256^3 phantom
 * costs 2.4 GB per request with FP64 sums and 1.3 GB with FP32 sums.  The
 * worker then runs epochs (RUNNING): one regrouped launch sequence over the
 * admitted requests of one phantom (chosen by mcd_serve_config.phantom_order), in which every
 * request advances by a slice of its histories.  Slices are handed out so
 * that the requests closest to completion finish first and the rest share
 * the epoch evenly.  A request's histories are the same whatever the slices:
 * history h always draws from the streams keyed by (seed, request_key, h), so
 * the result equals mcd_simulate of the same request with the regrouped
 * kernel up to FP64 summation order.  A request is finalised (dose, sigma,
 * Dmax, sigma-bar) in the epoch that completes it (DONE) and stays until
 * mcd_wait collects it.  Not part of the paper, which runs one plan at a time. */
enum { MCD_QUEUED = 0, MCD_ADMITTED = 1, MCD_RUNNING = 2, MCD_DONE = 3, MCD_FAILED = 4,
       MCD_CANCELED = 5 };
/* mcd_serve_config.phantom_order */
enum { MCD_PHANTOMS_SHORTEST = 0, MCD_PHANTOMS_IN_TURN = 1 };

typedef struct {
    mcd_opts opts;              /* launch options of the epochs (block_size, grid_blocks,
                                   stack_depth, chunk_per_lane, regroup, tally_fp32,
                                   diagnostics, sched_*, refined_build); first_history,
                                   accumulate, history_records, lockstep, use_graph and
                                   tally_slots must be 0, kernel MCD_KERNEL_REGROUPED */
    uint64_t epoch_histories;   /* histories per epoch over all its requests, 0 = four cycles'
                                   worth (4 x lanes x chunk_per_lane) */
    int32_t max_active;         /* admitted requests at most, 0 = 4096 */
    int32_t phantom_order;      /* which phantom's requests the next epoch runs:
                                   MCD_PHANTOMS_SHORTEST (0) = the phantom holding the request
                                   with the fewest histories left, unless a phantom with
                                   admitted requests has been passed over for 3 epochs in a
                                   row (then the one passed over longest);
                                   MCD_PHANTOMS_IN_TURN = phantoms in turn */
    uint64_t memory_limit;      /* bytes of request memory (tallies, dose, sigma) held at once,
                                   0 = only the context's HBM budget limits it */
} mcd_serve_config;

/* Serving counters since the first submit. */
typedef struct {
    uint64_t submitted, completed, failed, canceled;
    uint64_t queued, active;             /* now */
    uint64_t request_bytes;              /* device memory held by requests now */
    uint64_t hbm_used, hbm_budget;       /* the context's device memory now, and its cap */
    uint64_t histories;                  /* histories transported */
    uint64_t epochs;
    double busy_ms;                      /* device time of the epochs (set-up to finalisation) */
    double kernel_ms;                    /* device time of their transport phases */
    mcd_energy_balance eb;               /* summed over all epochs */
    uint64_t counters[MCD_NCOUNT];       /* filled when opts.diagnostics */
} mcd_serve_stats;

/* Sets the serving configuration.  Allowed before the first submit or once
 * every submitted request is collected by mcd_wait; else MCD_E_BUSY.  NULL
 * restores the defaults. */
int mcd_serve_configure(mcd_ctx* ctx, const mcd_serve_config* cfg);

/* Queues a request (2 <= n_histories < 2^32, seed < 2^32) and returns its
 * ticket at once; the source is copied.  Never waits for the device.  Starts
 * the worker thread on first use. */
int mcd_submit(mcd_ctx* ctx, int32_t phantom, const mcd_source* src, uint64_t n_histories,
               uint64_t seed, uint32_t request_key, uint64_t* out_ticket);

/* Queues a request that stops at a target uncertainty: its histories run in
 * epochs as for mcd_submit, and the request is finalised at checkpoints
 * (after the epoch that reaches 95% of the histories its last sigma-bar
 * projects for the target by the N^-1/2 law, at most four times the
 * histories it has); it completes once sigma-bar <= sigma_bar_target (and
 * Dmax > 0, at least 1000 histories) at a checkpoint, or when n_max
 * histories have run.  The
 * result equals mcd_simulate of the same request with N = the histories it
 * ran (mcd_result.n_histories), up to FP64 summation order.
 * 0 < sigma_bar_target < 1, 1000 <= n_max < 2^32. */
int mcd_submit_adaptive(mcd_ctx* ctx, int32_t phantom, const mcd_source* src, double sigma_bar_target,
                        uint64_t n_max, uint64_t seed, uint32_t request_key, uint64_t* out_ticket);

/* State of a ticket (MCD_QUEUED ... MCD_CANCELED) and histories transported
 * so far (either pointer may be NULL).  MCD_E_NOTFOUND for an unknown or
 * already collected ticket. */
int mcd_poll(mcd_ctx* ctx, uint64_t ticket, int32_t* state, uint64_t* histories_done);

/* Waits up to timeout_ms (< 0: forever) for the request to end.  DONE:
 * copies dose and sigma into out (as in mcd_simulate; NULL pointers skip),
 * fills dmax, sigma_bar, kernel_ms (device time of the epochs the request
 * took part in) and total_ms (submit to completion, wall clock), frees the
 * request and returns MCD_OK.  FAILED: returns the request's status (the
 * message in mcd_last_error) and frees it.  CANCELED: MCD_E_CANCELED, freed.
 * Timeout: MCD_E_BUSY, nothing freed.  eb and counters of a served request
 * are not kept separately (see mcd_serve_stats). */
int mcd_wait(mcd_ctx* ctx, uint64_t ticket, mcd_result* out, int64_t timeout_ms);

/* Cancels a request.  A queued request is cancelled at once; an admitted or
 * running one at the end of the current epoch, when its memory is freed.  A
 * request that already ended is left as it is.  The ticket is still collected
 * with mcd_wait. */
int mcd_cancel(mcd_ctx* ctx, uint64_t ticket);

int mcd_serve_stats_get(mcd_ctx* ctx, mcd_serve_stats* out);

/* ------------------------------------------------------------ verification
 *
 * These calls run the device functions of the transport kernels on caller
 * data, so that a test can hold them against independent implementations:
 * the Philox4x32-10 generator that replaces the paper's RANECU streams
 * (Sec. 2.4), and the lookups in the FP32 cross-section tables that the
 * paper keeps in texture memory (Sec. 2.3) and this engine stages into LDS.
 * Both are blocking; every pointer is a device pointer on the context's
 * device, owned by the caller. */

/* Philox4x32-10 (Salmon et al., SC'11) under the key (seed, key) applied to
 * n_blocks counters of four u32 words each (counters[4 i .. 4 i + 3] = c0..c3);
 * the four output words of block i go to out[4 i .. 4 i + 3].  Both arrays
 * 16-byte aligned; 1 <= n_blocks <= 2^32.  MCD_E_INVAL otherwise. */
int mcd_check_philox(mcd_ctx* ctx, uint32_t seed, uint32_t key, const uint32_t* counters,
                     uint64_t n_blocks, uint32_t* out, void* hip_stream);

/* Table quantities (per mass, as in the table blob; the values are those
 * indices of the blob's quantity list), the phantom's Woodcock majorant
 * (1/cm), and the inverse of the CSDA range (electron or positron: x is a
 * range in g/cm^2 and the result an energy in MeV). */
enum {
    MCD_Q_MU_C = 0, MCD_Q_MU_PE = 1, MCD_Q_MU_PP = 2, MCD_Q_RANGE = 3, MCD_Q_LAMBDA1_INV = 4,
    MCD_Q_SIGMA_M = 5, MCD_Q_SIGMA_B = 6, MCD_Q_MU_R = 8, MCD_Q_RANGE_POS = 10, MCD_Q_SIGMA_BH = 11,
    MCD_Q_MAJORANT = 100, MCD_Q_RANGE_INV = 101, MCD_Q_RANGE_POS_INV = 102
};

/* Evaluates `quantity` of `material` (ignored for the majorant) at n points
 * x (energies in MeV, or ranges for the inverses) with the tables of
 * `phantom` as the transport kernels do: FP32 nodes staged in LDS,
 * interpolation linear in log E (clamped to the grid), range inversion on
 * the same interpolant.  1 <= n <= 2^32.  MCD_E_NOTFOUND for an unknown
 * phantom, MCD_E_INVAL for a bad material, quantity or size. */
int mcd_check_tables(mcd_ctx* ctx, int32_t phantom, int32_t material, int32_t quantity, const float* x,
                     uint64_t n, float* out, void* hip_stream);

/* Measurement of the ceiling of the tally's operation (the dose collection by
 * atomic floating-point addition of Sec. 2.4, here FP64): adds 1.0 at
 * target[idx[i]] for i < n, reps times over, with the same atomic
 * instruction the tally flushes use, and returns the device time in *ms
 * (host).  target (n_target doubles) and idx (n u32) are device arrays of the
 * caller; indices >= n_target are skipped.  The rate for an address stream
 * drawn like the tally's flushes bounds how fast a kernel can flush. */
int mcd_measure_atomics(mcd_ctx* ctx, double* target, uint64_t n_target, const uint32_t* idx, uint64_t n,
                        int32_t reps, double* ms, void* hip_stream);

/* Issue rate of one kind of VALU instruction: every lane of eight waves per
 * SIMD runs `iters` x 128 operations in eight independent chains (no loads
 * or stores in the loop), and *cycles_per_op (host) receives the SIMD cycles
 * per wave-wide operation at the device's peak engine clock.  Kinds:
 *   MCD_VALU_FMA_F32  one v_fma_f32
 *   MCD_VALU_ADD_F32  one v_add_f32
 *   MCD_VALU_MUL_F32  one v_mul_f32
 *   MCD_VALU_XAD_U32  one 32-bit xor-add (v_xad_u32)
 *   MCD_VALU_MAD_U64  a 32 x 32 -> 64-bit multiply (v_mad_u64_u32) and an xor,
 *                     the Philox round's product
 *   MCD_VALU_FMAMK_F32 one FMA with literal constants (v_fmamk_f32)
 *   MCD_VALU_RCP_F32  one reciprocal (v_rcp_f32), a transcendental-unit op
 *   MCD_VALU_EXP_F32  one base-2 exponential (v_exp_f32), likewise.
 * A wave64 instruction on a 16-lane SIMD takes 4 cycles; fewer means the
 * hardware issues it on wider datapaths.  sink: one device float the kernel
 * never writes in practice.  For the transport's ALU roofline. */
enum { MCD_VALU_FMA_F32 = 0, MCD_VALU_ADD_F32 = 1, MCD_VALU_MUL_F32 = 2, MCD_VALU_XAD_U32 = 3,
       MCD_VALU_MAD_U64 = 4, MCD_VALU_FMAMK_F32 = 5, MCD_VALU_RCP_F32 = 6, MCD_VALU_EXP_F32 = 7 };
int mcd_measure_valu(mcd_ctx* ctx, int32_t kind, int32_t iters, float* sink, double* cycles_per_op,
                     void* hip_stream);

/* Status and error text.  mcd_last_error reports the last failure of a call
 * made on this context by the calling thread. */
const char* mcd_status_string(int status);
const char* mcd_last_error(mcd_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
