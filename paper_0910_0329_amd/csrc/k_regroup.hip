// Regrouped transport: particles are sorted by type into queues so that every
// wave runs one kind of step (photon flights or electron segments) and the
// wavefront does not serialise the two code paths.
//
// A cycle is a photon phase followed by an electron phase.  The photon phase
// transports the photons queued by the previous electron phase and up to
// `chunk` new histories (photon primaries in place; electron and positron
// primaries are queued); electrons and positrons it creates are queued for the
// electron phase.  The electron phase transports them; the photons it creates
// (bremsstrahlung, annihilation) are queued for the next photon phase.
// Same-type secondaries stay on the lane's own stack, and so does a
// cross-type secondary when the other queue is full, so no particle is lost
// and the result does not depend on the queue capacity.  Every lane loops
// until its phase has no work left; the host (or a captured graph) runs
// cycles until all histories are claimed, and the electron phase of the last
// cycle keeps the photons it creates on the lane stacks, so nothing is left
// queued at the end.
//
// Histories of several requests (beams, beamlets, served requests) share a
// launch: each particle carries its request slot, which selects the Philox key
// and the request's tally.  The tally is batch-statistical: history h adds to
// sub-tally h mod 16, and the uncertainty comes from the spread of the 16
// sub-tally means.  Consecutive deposits of a particle into one voxel are
// summed in registers and added with one atomic per voxel visit.
#include "transport.h"

namespace mcd {

template <bool DIAG, bool PHOTONS, bool REF>
struct PhaseLane : Transport<PhaseLane<DIAG, PHOTONS, REF>, DIAG, REF> {
    const KPhase& p;
    char* stack;
    int sp;
    int cur_v;
    float cur_e;
    // request context of the particle in flight
    int slot;
    void* tally;
    mcd_history_record* hist;
    uint32_t first;
    // per-particle diagnostics
    double p_edep, p_track;
    // work sources of this phase
    unsigned int n_in;
    bool more_new;

    DEV PhaseLane(const KPhase& pp, char* base) : Transport<PhaseLane<DIAG, PHOTONS, REF>, DIAG, REF>(pp.g),
                                                   p(pp), stack(base), sp(0), cur_v(-1), cur_e(0.f),
                                                   slot(-1), tally(nullptr), hist(nullptr), first(0),
                                                   p_edep(0.0), p_track(0.0) {}

    DEV void fail(int status)
    {
        this->failed = 1;
        atomicCAS(p.err, 0, status);
    }

    DEV void use_request(uint32_t s)
    {
        if ((int)s == slot) return;
        const ReqDev& r = p.req[s];
        slot = (int)s;
        this->env.seed = r.seed;
        this->env.key = r.key;
        tally = r.tally;
        hist = (mcd_history_record*)r.hist;
        first = r.first;
    }

    DEV void flush_visit(const Part& q)
    {
        if (cur_v < 0) return;
        const size_t idx = (size_t)(q.h & (kBatches - 1)) * (size_t)p.nv + (size_t)cur_v;
        if (p.tally_fp32) unsafeAtomicAdd((float*)tally + idx, cur_e);
        else unsafeAtomicAdd((double*)tally + idx, (double)cur_e);
        if (DIAG) ++this->c[MCD_C_FLUSHES];
        cur_v = -1;
    }

    DEV void deposit(const Part& q, int v, float e)
    {
        if (e == 0.f) return;
        if (DIAG) p_edep += (double)e;
        if (v == cur_v) {
            cur_e += e;
        } else {
            flush_visit(q);
            cur_v = v;
            cur_e = e;
        }
    }

    DEV void flush_particle(const Part& q)
    {
        flush_visit(q);
        if (DIAG && hist && p_edep != 0.0) unsafeAtomicAdd(&hist[q.h - first].edep, p_edep);
        p_edep = 0.0;
    }

    DEV void add_track(const Part&, float l) { if (DIAG) p_track += (double)l; }

    DEV void escaped(const Part& q)
    {
        if (DIAG && hist) atomicMax(&hist[q.h - first].escaped, 1u);
    }

    DEV void particle_done(const Part& q, uint64_t ph)
    {
        flush_visit(q);
        if (DIAG && hist) {
            mcd_history_record* r = &hist[q.h - first];
            if (p_edep != 0.0) unsafeAtomicAdd(&r->edep, p_edep);
            if (p_track != 0.0) unsafeAtomicAdd(&r->track_e, p_track);
            atomicAdd((unsigned long long*)&r->hash, (unsigned long long)ph);
            atomicAdd(&r->n_particles, 1u);
        }
        p_edep = p_track = 0.0;
    }

    DEV void push_stack(const Part& s)
    {
        if (sp >= p.stack_depth) {
            fail(MCD_E_OVERFLOW);
            return;
        }
        store_rec(stack + (size_t)sp * kRec, s);
        ++sp;
        if (DIAG && (uint32_t)sp > this->c[MCD_C_MAX_STACK]) this->c[MCD_C_MAX_STACK] = (uint32_t)sp;
    }

    DEV void spawn(const Part& s)
    {
        const bool cross = PHOTONS ? s.type != PHOTON : s.type == PHOTON;
        if (cross && p.use_queues) {
            const unsigned int i = wave_fetch_add(&p.q_out_ctl->count);
            if (i < p.q_cap) {
                store_rec(p.q_out + (size_t)i * kRec, s);
                return;
            }
        }
        push_stack(s);
    }

    // Starts transport of a particle read from a stack or queue.
    DEV bool begin(Part& q)
    {
        if (q.type < PHOTON || q.type > POSITRON || (int)q.slot >= p.n_req) {
            fail(MCD_E_DEVICE);
            return false;
        }
        use_request(q.slot);
        this->start_particle(q);
        return true;
    }

    // Next particle of the lane: its own stack, else the input queue, else a
    // new history of this cycle (photon phase).  False when no work is left.
    DEV bool fetch(Part& q)
    {
        if (sp > 0) {
            --sp;
            load_rec(stack + (size_t)sp * kRec, q);
            return begin(q);
        }
        if (n_in) {
            const unsigned int i = wave_fetch_add(&p.q_in_ctl->head);
            if (i < n_in) {
                load_rec(p.q_in + (size_t)i * kRec, q);
                return begin(q);
            }
            n_in = 0;
        }
        if (more_new && !this->failed) {
            more_new = claim(q);
            return more_new;
        }
        return false;
    }

    // Claims the next new history of this cycle.  Returns false when none is left.
    DEV bool claim(Part& q)
    {
        const unsigned int j = wave_fetch_add(&p.claim[p.cycle]);
        const uint64_t gi = (uint64_t)p.cycle * p.chunk + j;
        if ((uint64_t)j >= p.chunk || gi >= p.total) return false;
        int lo = 0, hi = p.n_req - 1;          // last request whose first index <= gi
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (p.req[mid].lo <= gi) lo = mid; else hi = mid - 1;
        }
        const ReqDev& r = p.req[lo];
        use_request((uint32_t)lo);
        q.slot = (uint32_t)lo;
        q.h = r.first + (uint32_t)(gi - r.lo);
        this->start_history(q, r.src, r.src.edges, r.src.cdf);
        if (q.type == DEAD) {
            flush_particle(q);
        } else if (q.type == PHOTON) {
            this->start_particle(q);
        } else {
            spawn(q);               // electron or positron primary: to the electron phase
            q.type = DEAD;
        }
        return true;
    }
};

template <bool DIAG, bool PHOTONS, bool REF>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_phase(KPhase p)
{
    extern __shared__ float4 lds[];
    Env env;
    float* extra;
    stage_tables(p.g, lds, env, &extra);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        p.q_reset_ctl->count = 0u;
        p.q_reset_ctl->head = 0u;
    }
    __syncthreads();

    const size_t lane_id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    PhaseLane<DIAG, PHOTONS, REF> L(p, p.scratch + lane_id * p.lane_bytes);
    L.env = env;
    L.init_base();
    L.n_in = min(p.q_in_ctl->count, p.q_cap);
    L.more_new = PHOTONS;
    Part q;
    q.type = DEAD;
    q.pend = 0;
    L.run(q, p.sched);
    L.reduce_out(p.bal, p.cnt);
}

size_t phase_lane_bytes(int stack_depth)
{
    size_t b = (size_t)stack_depth * kRec;
    return (b + 255) & ~(size_t)255;
}

// The instance for (diagnostics, photon phase, refinements) = bits 4, 2, 1 of which.
static void (*phase_kernel(int which))(KPhase)
{
    switch (which) {
    case 0: return k_phase<false, false, false>;
    case 1: return k_phase<false, false, true>;
    case 2: return k_phase<false, true, false>;
    case 3: return k_phase<false, true, true>;
    case 4: return k_phase<true, false, false>;
    case 5: return k_phase<true, false, true>;
    case 6: return k_phase<true, true, false>;
    default: return k_phase<true, true, true>;
    }
}

hipError_t launch_phase(const KPhase& p, bool photons, int blocks, int threads, bool diag,
                        hipStream_t s)
{
    const size_t lds = transport_lds_bytes(p.g.t.n_mat);
    const int which = (diag ? 4 : 0) | (photons ? 2 : 0) | (p.g.t.refined ? 1 : 0);
    hipLaunchKernelGGL(phase_kernel(which), dim3(blocks), dim3(threads), lds, s, p);
    return hipGetLastError();
}

hipError_t init_phase_kernels(int max_lds)
{
    for (int which = 0; which < 8; ++which) {
        const hipError_t e = hipFuncSetAttribute((const void*)phase_kernel(which),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t init_kernels(int max_lds)
{
    hipError_t e = init_plain_kernels(max_lds);
    if (e == hipSuccess) e = init_phase_kernels(max_lds);
    if (e == hipSuccess) e = init_wave_kernels(max_lds);
    return e == hipSuccess ? init_check_kernels(max_lds) : e;
}

}  // namespace mcd
