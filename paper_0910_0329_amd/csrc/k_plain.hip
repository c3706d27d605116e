// The plain per-history kernel: one lane follows one source history and every
// secondary it creates, as in the paper's kernel (Fig. 1, Sec. 2.2).  The
// source particle is sampled, transported, its secondaries go on the lane's own
// stack and are popped until the stack is empty, then the history's deposits
// are collected (Sec. 2.4).  The lane takes one transport step per loop
// iteration, so a wave re-converges after every step, and takes a new history
// from a global work counter when its history is finished.
//
// Local counter (exact history-by-history statistics): consecutive deposits
// into one voxel are summed in registers, then kept in the lane's
// open-addressing table (voxel -> energy of the current history); at history
// end every entry e is added to S[v] (e) and Q[v] (e^2) with FP64 atomics.
#include "transport.h"

namespace mcd {

template <bool DIAG, bool REF>
struct PlainLane : Transport<PlainLane<DIAG, REF>, DIAG, REF> {
    using Base = Transport<PlainLane<DIAG, REF>, DIAG, REF>;
    const KPlain& p;
    char* stack;
    uint32_t* keys;
    float* vals;
    uint16_t* list;
    int sp, nused, lgslots;
    int cur_v;
    float cur_e;
    // history assignment
    const float* s_edges;
    const float* s_cdf;
    size_t lane_id, n_lanes;
    uint32_t off, rounds;
    bool have;
    // per-history diagnostics
    double h_edep, h_track;
    uint64_t h_hash;
    uint32_t h_parts, h_esc;

    DEV PlainLane(const KPlain& pp, char* base) : Base(pp.g), p(pp)
    {
        stack = base;
        keys = (uint32_t*)(base + (size_t)p.stack_depth * kRec);
        vals = (float*)(keys + p.slots);
        list = (uint16_t*)(vals + p.slots);
        sp = nused = 0;
        lgslots = 31 - __builtin_clz((unsigned)p.slots);
        cur_v = -1;
        cur_e = 0.f;
        off = rounds = 0;
        have = false;
        h_edep = h_track = 0.0;
        h_hash = 0;
        h_parts = h_esc = 0;
    }

    DEV void fail(int status)
    {
        this->failed = 1;
        atomicCAS(p.err, 0, status);
    }

    DEV void table_add(int v, float e)
    {
        const uint32_t key = (uint32_t)v + 1u;
        const uint32_t mask = (uint32_t)p.slots - 1u;
        uint32_t s = ((uint32_t)v * 0x9E3779B1u) >> (32 - lgslots);
        for (;;) {
            const uint32_t k = keys[s];
            if (k == key) {
                vals[s] += e;
                return;
            }
            if (k == 0u) {
                if (nused >= (p.slots >> 1) + (p.slots >> 2)) {
                    fail(MCD_E_OVERFLOW);
                    return;
                }
                keys[s] = key;
                vals[s] = e;
                list[nused++] = (uint16_t)s;
                return;
            }
            s = (s + 1u) & mask;
        }
    }

    DEV void deposit(const Part&, int v, float e)
    {
        if (e == 0.f) return;
        if (DIAG) h_edep += (double)e;
        if (v == cur_v) {
            cur_e += e;
        } else {
            if (cur_v >= 0) table_add(cur_v, cur_e);
            cur_v = v;
            cur_e = e;
        }
    }

    DEV void flush_particle(const Part&) {}
    DEV void add_track(const Part&, float l) { if (DIAG) h_track += (double)l; }
    DEV void escaped(const Part&) { if (DIAG) h_esc = 1; }
    DEV void particle_done(const Part&, uint64_t ph)
    {
        if (DIAG) {
            h_hash += ph;
            ++h_parts;
        }
    }

    DEV void spawn(const Part& s)
    {
        if (sp >= p.stack_depth) {
            fail(MCD_E_OVERFLOW);
            return;
        }
        store_rec(stack + (size_t)sp * kRec, s);
        ++sp;
        if (DIAG && (uint32_t)sp > this->c[MCD_C_MAX_STACK]) this->c[MCD_C_MAX_STACK] = (uint32_t)sp;
    }

    DEV void pop(Part& q)
    {
        --sp;
        load_rec(stack + (size_t)sp * kRec, q);
    }

    // Next particle of the lane: the top of its stack, else (after closing
    // the history it has finished) the source particle of a new history.
    // False when no work is left.
    DEV bool fetch(Part& q)
    {
        if (sp > 0) {
            pop(q);
            this->start_particle(q);
            return true;
        }
        if (have) {
            finish_history(off);
            have = false;
        }
        // Only the lane's own failure stops it: polling the shared error flag
        // here costs a system-scope load per history on the critical path
        // (measured 4x slower); other lanes finish their work and the host
        // reports the error.
        if (this->failed) return false;
        unsigned long long o;
        if (p.lockstep) {
            // every lane of a wave takes the same history (a static round-robin
            // over waves): the wave then runs that history's instruction path
            // without divergence
            o = (unsigned long long)(lane_id >> 6) + (unsigned long long)rounds * (n_lanes >> 6);
            ++rounds;
        } else {
            o = wave_fetch_add(p.next);
        }
        if (o >= (unsigned long long)p.n) return false;
        off = (uint32_t)o;
        have = true;
        q.h = p.first + off;
        this->start_history(q, p.src, s_edges, s_cdf);
        if (q.type != DEAD) this->start_particle(q);
        return true;
    }

    // Dose collection at history end: S += e_{h,v}, Q += e_{h,v}^2 (FP64).
    DEV void finish_history(uint32_t off)
    {
        if (cur_v >= 0) table_add(cur_v, cur_e);
        cur_v = -1;
        for (int i = 0; i < nused; ++i) {
            const uint32_t s = list[i];
            const int v = (int)keys[s] - 1;
            const double e = (double)vals[s];
            unsafeAtomicAdd(&p.S[v], e);
            unsafeAtomicAdd(&p.Q[v], e * e);
            keys[s] = 0u;
        }
        if (DIAG) {
            this->c[MCD_C_FLUSHES] += (uint32_t)nused;
            if (p.hist) {
                mcd_history_record* r = (mcd_history_record*)p.hist + off;
                r->edep = h_edep;
                r->track_e = h_track;
                r->hash = h_hash;
                r->n_particles = h_parts;
                r->escaped = h_esc;
            }
            h_edep = h_track = 0.0;
            h_hash = 0;
            h_parts = h_esc = 0;
        }
        nused = 0;
    }
};

template <bool DIAG, bool REF>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_plain(KPlain p)
{
    extern __shared__ float4 lds[];
    Env env;
    float* extra;
    stage_tables(p.g, lds, env, &extra);
    float* s_edges = extra;
    float* s_cdf = extra + 68;
    for (int i = threadIdx.x; i < 65; i += blockDim.x) s_edges[i] = p.src.edges[i];
    for (int i = threadIdx.x; i < 64; i += blockDim.x) s_cdf[i] = p.src.cdf[i];
    __syncthreads();
    env.seed = p.seed;
    env.key = p.key;

    const size_t lane_id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    PlainLane<DIAG, REF> L(p, p.scratch + lane_id * p.lane_bytes);
    L.env = env;
    L.init_base();
    L.s_edges = s_edges;
    L.s_cdf = s_cdf;
    L.lane_id = lane_id;
    L.n_lanes = (size_t)gridDim.x * blockDim.x;
    Part q;
    q.type = DEAD;
    q.slot = 0;
    q.pend = 0;
    L.run(q, p.sched);
    L.reduce_out(p.bal, p.cnt);
}

size_t plain_lane_bytes(int stack_depth, int slots)
{
    size_t b = (size_t)stack_depth * kRec + (size_t)slots * 10;
    return (b + 255) & ~(size_t)255;
}

int transport_lds_bytes(int n_mat)
{
    return 2 * n_mat * kNE * (int)sizeof(float4) + (kNE + 3 * kMaxMat + 68 + 64) * (int)sizeof(float);
}

hipError_t launch_plain(const KPlain& p, int blocks, int threads, bool diag, hipStream_t s)
{
    const size_t lds = transport_lds_bytes(p.g.t.n_mat);
    const bool ref = p.g.t.refined != 0;
    if (diag && ref) hipLaunchKernelGGL((k_plain<true, true>), dim3(blocks), dim3(threads), lds, s, p);
    else if (diag) hipLaunchKernelGGL((k_plain<true, false>), dim3(blocks), dim3(threads), lds, s, p);
    else if (ref) hipLaunchKernelGGL((k_plain<false, true>), dim3(blocks), dim3(threads), lds, s, p);
    else hipLaunchKernelGGL((k_plain<false, false>), dim3(blocks), dim3(threads), lds, s, p);
    return hipGetLastError();
}

hipError_t init_plain_kernels(int max_lds)
{
    const void* fns[4] = {(const void*)k_plain<true, true>, (const void*)k_plain<true, false>,
                          (const void*)k_plain<false, true>, (const void*)k_plain<false, false>};
    for (const void* f : fns) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace mcd
