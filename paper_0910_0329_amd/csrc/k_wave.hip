// Wave-stack transport: the regrouped engine with the secondary stacks of a
// wave's 64 lanes pooled by particle type.
//
// Each wave owns two stacks in global memory, one of photons and one of
// electrons and positrons.  A secondary goes on the stack of its type, and any
// lane of the wave can carry on any of the wave's particles.  A particle can
// also be parked mid-flight: its record keeps the position, direction,
// energy, stream counter and the random block in use, and for an electron its
// voxel, hinge and hard-event state.  The wave works in a photon or an
// electron mode: lanes that need a particle take one of the mode's kind, and
// lanes that hold the other kind park it and take a waiting particle of the
// mode's kind, so the mode's steps run with the whole wave.  The mode changes
// when its kind no longer has work for a good part of the wave (lanes plus
// stacked particles below 64 / photon_div) and the other kind has more.  A
// new history starts only while the two stacks together hold fewer than a
// quarter of their capacity, which bounds the particles a wave holds.
//
// A particle's stream and tally depend only on its own lineage and history
// index, so which lane carries a particle, and when, does not change any
// result: the histories are those of every other kernel (their deposits can
// differ in the last bits where the compiler fuses multiply-adds differently
// in the two kernels' code).  The stack counts
// live in LDS (one pair per wave, touched only by that wave), the records in
// global memory; the wave's own instruction stream orders every push before
// the pops that follow it.
#include "transport.h"

namespace mcd {

constexpr int kWaveRec = 80;         // bytes per photon-stack record
// An electron step runs up to Sched::segments condensed-history segments (12
// by default) before the wave returns to its schedule: a lane goes on with its
// next segment while its particle stays a charged particle without a pending
// hard event (lanes that stop wait for the others).  The schedule's
// bookkeeping at the loop top costs more than the lanes that idle through the
// remaining segments; a fixed count did better than stopping once half the
// lanes had stopped.
constexpr int kWaveERec = 112;       // bytes per electron-stack record (with the electron state)
enum { WS_PHOTON = 0, WS_ELECTRON = 1 };

// Record of a wave stack, four float4:
//   f0 = (x, y, z, E), f1 = (u, v, w, bits(type | slot << 4 | nsp << 16)),
//   f2 = bits(l0, l1, h, d | ring << 31 | parked << 30), f3 = words of random
// block d >> 2 (a parked photon that had drawn from it; ring = 1).  A fresh
// secondary holds its parent's lineage, d = kLineagePending | spawn index and
// nsp = 0 (its own spawn count starts at start_particle), and leaves f3
// unwritten.  A parked particle also keeps its open tally visit (the voxel
// and the FP32 sum of its deposits there so far), so that its deposits are
// grouped as if it had never stopped: f4 = (bits(cur_v), cur_e, flags, 0), and
// an electron f5 = bits(ix, iy, iz, 0), f6 = (nh, xi, kap, 0), flags = before
// | pend << 1.
DEV void store_wave_rec(char* base, const Part& q, bool parked)
{
    float4* r = (float4*)base;
    const bool ring = parked && (q.d >> 2) < q.g;
    const uint32_t nsp = parked ? q.nsp : 0u;
    r[0] = make_float4(q.x, q.y, q.z, q.e);
    r[1] = make_float4(q.u, q.v, q.w, __uint_as_float((uint32_t)q.type | (q.slot << 4) | (nsp << 16)));
    r[2] = make_float4(__uint_as_float(q.l0), __uint_as_float(q.l1), __uint_as_float(q.h),
                       __uint_as_float(q.d | (ring ? 0x80000000u : 0u) | (parked ? 0x40000000u : 0u)));
    if (ring) {
        const bool hi = ((q.d >> 2) & 1u) != 0;
        r[3] = hi ? make_float4(__uint_as_float(q.r4), __uint_as_float(q.r5), __uint_as_float(q.r6),
                                __uint_as_float(q.r7))
                  : make_float4(__uint_as_float(q.r0), __uint_as_float(q.r1), __uint_as_float(q.r2),
                                __uint_as_float(q.r3));
    }
}

DEV void store_parked_state(char* base, const Part& q, int cur_v, float cur_e, bool electron)
{
    float4* r = (float4*)base;
    const uint32_t flags = electron ? ((uint32_t)q.before | ((uint32_t)q.pend << 1)) : 0u;
    r[4] = make_float4(__int_as_float(cur_v), cur_e, __uint_as_float(flags), 0.f);
    if (electron) {
        r[5] = make_float4(__int_as_float(q.ix), __int_as_float(q.iy), __int_as_float(q.iz), 0.f);
        r[6] = make_float4(q.nh, q.xi, q.kap, 0.f);
    }
}

DEV void load_parked_state(const char* base, Part& q, int& cur_v, float& cur_e, bool electron)
{
    const float4* r = (const float4*)base;
    const float4 a = r[4];
    cur_v = __float_as_int(a.x);
    cur_e = a.y;
    if (electron) {
        const uint32_t f = __float_as_uint(a.z);
        q.before = (int)(f & 1u);
        q.pend = (int)((f >> 1) & 1u);
        const float4 b = r[5], c = r[6];
        q.ix = __float_as_int(b.x);
        q.iy = __float_as_int(b.y);
        q.iz = __float_as_int(b.z);
        q.nh = c.x;
        q.xi = c.y;
        q.kap = c.z;
    }
}

// Returns true when the record was parked mid-flight (its random block, if it
// had drawn from one, restored).
DEV bool load_wave_rec(const char* base, Part& q)
{
    const float4* r = (const float4*)base;
    const float4 a = r[0], b = r[1], c = r[2];
    q.x = a.x; q.y = a.y; q.z = a.z; q.e = a.w;
    q.u = b.x; q.v = b.y; q.w = b.z;
    const uint32_t ts = __float_as_uint(b.w);
    q.type = (int)(ts & 15u);
    q.slot = (ts >> 4) & 0xFFFu;
    q.nsp = ts >> 16;
    q.l0 = __float_as_uint(c.x);
    q.l1 = __float_as_uint(c.y);
    q.h = __float_as_uint(c.z);
    const uint32_t dw = __float_as_uint(c.w);
    q.d = dw & 0x3FFFFFFFu;
    q.pend = 0;
    q.g = q.d >> 2;
    if (dw >> 31) {
        const float4 w = r[3];
        const uint32_t w0 = __float_as_uint(w.x), w1 = __float_as_uint(w.y), w2 = __float_as_uint(w.z),
                       w3 = __float_as_uint(w.w);
        if (q.g & 1u) {
            q.r4 = w0; q.r5 = w1; q.r6 = w2; q.r7 = w3;
        } else {
            q.r0 = w0; q.r1 = w1; q.r2 = w2; q.r3 = w3;
        }
        ++q.g;
    }
    return ((dw >> 30) & 1u) != 0;
}

template <bool DIAG, bool REF>
struct WaveLane : Transport<WaveLane<DIAG, REF>, DIAG, REF> {
    using Base = Transport<WaveLane<DIAG, REF>, DIAG, REF>;
    const KPhase& p;
    char* base;                    // this wave's stacks: photon records, their diagnostic
                                   // event hashes, electron records (wave-uniform)
    volatile unsigned int* cnt;    // LDS: records on the photon and electron stacks
    int cur_v;
    float cur_e;
    int slot;
    void* tally;
    mcd_history_record* hist;
    uint32_t first;
    double p_edep, p_track;
    bool more_new;                 // wave-uniform: new histories may remain

    DEV WaveLane(const KPhase& pp, char* b, volatile unsigned int* c)
        : Base(pp.g), p(pp), base(b), cnt(c), cur_v(-1), cur_e(0.f), slot(-1), tally(nullptr), hist(nullptr),
          first(0), p_edep(0.0), p_track(0.0), more_new(true) {}

    // layout: photon records | their hashes | electron records | their hashes
    DEV unsigned cap() const { return (unsigned)p.stack_depth; }
    DEV char* rec(int k, unsigned i) const
    {
        if (k == WS_PHOTON) return base + (size_t)i * kWaveRec;
        return base + (size_t)cap() * (kWaveRec + sizeof(uint64_t)) + (size_t)i * kWaveERec;
    }
    DEV uint64_t* hashes(int k) const
    {
        if (k == WS_PHOTON) return (uint64_t*)(base + (size_t)cap() * kWaveRec);
        return (uint64_t*)(base + (size_t)cap() * (kWaveRec + sizeof(uint64_t) + kWaveERec));
    }

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

    // ------------------------------------------------------------- tally
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

    // ------------------------------------------------------- wave stacks
    // Pushes the calling lanes' particles onto stack k.  The active lanes may
    // be any subset of the wave: they read the count from LDS, place their
    // records after it by rank and all write back the same new count.
    DEV void push(int k, const Part& s, bool parked, uint64_t hash)
    {
        const uint64_t m = __builtin_amdgcn_ballot_w64(true);
        const unsigned rank =
            __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        // the first active lane reserves the slots with one LDS atomic (an
        // LDS access, so only the LDS counter is waited for)
        const unsigned n_push = (unsigned)__popcll(m);
        unsigned base = 0u;
        if (rank == 0)
            base = __hip_atomic_fetch_add((__attribute__((address_space(3))) unsigned int*)(cnt + k), n_push,
                                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        const unsigned top0 = __builtin_amdgcn_readfirstlane(base);
        const unsigned i = top0 + rank;
        if (i < cap()) {
            store_wave_rec(rec(k, i), s, parked);
            if (parked) store_parked_state(rec(k, i), s, cur_v, cur_e, k == WS_ELECTRON);
            if (DIAG) hashes(k)[i] = hash;
        } else {
            fail(MCD_E_OVERFLOW);
        }
        const unsigned top = min(top0 + n_push, cap());
        if (top0 + n_push > cap()) cnt[k] = top;      // overflow (failed above): keep the count in range
        if (DIAG && top > this->c[MCD_C_MAX_STACK]) this->c[MCD_C_MAX_STACK] = top;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    }

    DEV void spawn(const Part& s) { push(s.type == PHOTON ? WS_PHOTON : WS_ELECTRON, s, false, 0ull); }

    // Sets the count of stack k with an LDS store (no wait for the wave's
    // outstanding global stores).
    DEV void lds_set_count(int k, unsigned v)
    {
        __hip_atomic_store((__attribute__((address_space(3))) unsigned int*)(cnt + k), v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WAVEFRONT);
    }

    // Takes record i of stack k into q and starts it (a parked particle
    // resumes where it stopped, with its event hash; a fresh one starts anew).
    DEV bool take(int k, unsigned i, Part& q)
    {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const bool parked = load_wave_rec(rec(k, i), q);
        if (q.type < PHOTON || q.type > POSITRON || (int)q.slot >= p.n_req) {
            fail(MCD_E_DEVICE);
            q.type = DEAD;
            return false;
        }
        use_request(q.slot);
        if (parked) {
            load_parked_state(rec(k, i), q, cur_v, cur_e, k == WS_ELECTRON);
            if (k == WS_ELECTRON) this->enter_voxel(q);
            if (DIAG) this->p_hash = hashes(k)[i];
        } else {
            this->start_particle(q);
        }
        return true;
    }

    // Parks the lane's particle (mid-flight) on the stack of its kind with its
    // open tally visit; the lane starts its next particle with none.
    DEV void park(Part& q)
    {
        if (DIAG && hist) {
            mcd_history_record* r = &hist[q.h - first];
            if (p_edep != 0.0) unsafeAtomicAdd(&r->edep, p_edep);
            if (p_track != 0.0) unsafeAtomicAdd(&r->track_e, p_track);
        }
        p_edep = p_track = 0.0;
        push(q.type == PHOTON ? WS_PHOTON : WS_ELECTRON, q, true, DIAG ? this->p_hash : 0ull);
        cur_v = -1;
        q.type = DEAD;
    }

    // Claims the next new history; false when none is left.  Its primary
    // starts on this lane, whatever its kind.
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
        if (q.type == DEAD) flush_particle(q);
        else this->start_particle(q);
        return true;
    }

    // Fetch step of the lanes that need a particle: first the stack of the
    // wave's mode, then new histories while they may start, else the other
    // stack.  sg and se are the stacks' current counts (the caller's copies
    // of the LDS words).  Returns false only for a lane whose claim found the
    // histories exhausted (claims held back by full stacks are not
    // exhaustion).
    DEV bool fetch_wave(Part& q, bool prefer_photons, bool can_claim, unsigned sg, unsigned se)
    {
        const uint64_t m = __builtin_amdgcn_ballot_w64(true);
        const unsigned rank =
            __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        const unsigned nfl = (unsigned)__popcll(m);
        const int ka = prefer_photons ? WS_PHOTON : WS_ELECTRON, kb = 1 - ka;
        const unsigned ca = prefer_photons ? sg : se, cb = prefer_photons ? se : sg;
        const unsigned ta = min(nfl, ca), tb = can_claim ? 0u : min(nfl - ta, cb);
        lds_set_count(ka, ca - ta);
        lds_set_count(kb, cb - tb);
        // one take for both stacks (lanes of a fetch may take from either)
        if (rank < ta + tb) {
            const bool a = rank < ta;
            take(a ? ka : kb, a ? ca - 1 - rank : cb - 1 - (rank - ta), q);
        }
        // every record taken above is read before a new history below can
        // push onto the slots just freed (a positron primary below its
        // cutoff annihilates at once)
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        if (rank < ta + tb || !can_claim || this->failed) return true;
        return claim(q);
    }

    // ---------------------------------------------------- wave schedule
    // As Transport::run, with the wave stacks and the wave's mode (photon or
    // electron): lanes holding the other kind park and take waiting particles
    // of the mode's kind; fetching lanes count only while something can be
    // fetched; steps of the mode's kind run unless fetch or hard-event
    // thresholds call (an electron step runs up to sc.segments segments, a
    // photon step up to two flights); the wave ends when no lane
    // holds a particle and nothing is left to fetch.
    enum { ST_FETCH, ST_PHOTON, ST_ELECTRON, ST_HARD };

    DEV int state(const Part& q) const
    {
        return q.type == DEAD ? ST_FETCH : (q.type == PHOTON ? ST_PHOTON : (q.pend ? ST_HARD : ST_ELECTRON));
    }

    // Lanes in state from1 or from2 (the first `top` of them) park their
    // particle on its own kind's stack and take record top - 1 - rank of
    // stack `to`, which holds the other kind; that stack keeps top - k.
    DEV void swap_in(Part& q, int st, int from1, int from2, int to, unsigned top)
    {
        if (st == from1 || st == from2) {
            const uint64_t m = __builtin_amdgcn_ballot_w64(true);
            const unsigned rank =
                __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            const unsigned k = min((unsigned)__popcll(m), top);
            if (rank < k) {
                park(q);
                take(to, top - 1 - rank, q);
            }
            lds_set_count(to, top - k);
        }
    }

    DEV void run_wave(Part& q, const Sched sc)
    {
        const unsigned claim_cap = min(cap() / 4u, 384u);
        const int low = max(64 / sc.photon_div, 1);
        const bool claim_photon = p.req[0].src.particle == PHOTON;
        int mode = claim_photon ? ST_PHOTON : ST_ELECTRON;      // wave-uniform
        for (;;) {
            int st = state(q);
            const uint64_t live = __builtin_amdgcn_ballot_w64(true);
            const int n = __popcll(live);
            int nf = __popcll(__builtin_amdgcn_ballot_w64(st == ST_FETCH));
            int np = __popcll(__builtin_amdgcn_ballot_w64(st == ST_PHOTON));
            int nh = __popcll(__builtin_amdgcn_ballot_w64(st == ST_HARD));
            int ne = n - nf - np - nh;
            const unsigned sg = cnt[WS_PHOTON], se = cnt[WS_ELECTRON];
            if (nf == n && sg + se == 0 && !more_new) break;
            const bool can_claim = more_new && sg + se < claim_cap;
            // work of each kind: lanes, stacked particles, and fetching lanes
            // when new histories (of the first source's kind) may start
            const int wp = np + (int)min(sg, 64u) + (can_claim && claim_photon ? nf : 0);
            const int we = ne + nh + (int)min(se, 64u) + (can_claim && !claim_photon ? nf : 0);
            if (mode == ST_PHOTON ? (wp < low && we > wp) : (we < low && wp > we))
                mode = ST_PHOTON + ST_ELECTRON - mode;
            // a swap parks k particles on their own kind's stack and takes k
            // from the other: the counts move by k and their sum stays
            unsigned sgn = sg, sen = se;
            const bool swap_e = mode == ST_ELECTRON && np && se;
            const bool swap_p = mode == ST_PHOTON && ne + nh && sg;
            if (swap_e || swap_p) {
                if (swap_e) {
                    swap_in(q, st, ST_PHOTON, ST_PHOTON, WS_ELECTRON, se);
                    const unsigned k = min((unsigned)np, se);
                    sgn = sg + k;
                    sen = se - k;
                } else {
                    swap_in(q, st, ST_ELECTRON, ST_HARD, WS_PHOTON, sg);
                    const unsigned k = min((unsigned)(ne + nh), sg);
                    sen = se + k;
                    sgn = sg - k;
                }
                // the swapped lanes changed state
                st = state(q);
                nf = __popcll(__builtin_amdgcn_ballot_w64(st == ST_FETCH));
                np = __popcll(__builtin_amdgcn_ballot_w64(st == ST_PHOTON));
                nh = __popcll(__builtin_amdgcn_ballot_w64(st == ST_HARD));
                ne = n - nf - np - nh;
            }
            const bool fetchable = sg + se > 0 || can_claim;
            const int nfe = fetchable ? nf : 0;
            int act;
            const int fdiv = mode == ST_PHOTON ? sc.fetch_photon_div : sc.fetch_div;
            if (nfe && (nfe * fdiv >= n || nfe == n)) act = ST_FETCH;
            else if (nh && (nh * sc.hard_div >= n || nh + nf == n)) act = ST_HARD;
            else if (mode == ST_PHOTON ? np : ne) act = mode;
            else if (np) act = ST_PHOTON;
            else if (ne) act = ST_ELECTRON;
            else act = nh ? ST_HARD : ST_FETCH;
            const int na = DIAG ? __popcll(__builtin_amdgcn_ballot_w64(st == act)) : 0;
            if (DIAG && __builtin_amdgcn_mbcnt_hi((uint32_t)(live >> 32),
                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)live, 0u)) == 0) {
                ++this->c[MCD_C_ITERS];
                this->c[MCD_C_LIVE] += (uint32_t)n;
                ++this->c[MCD_C_IT_FETCH + act];
                this->c[MCD_C_LN_FETCH + act] += (uint32_t)na;
            }
            bool exhausted = false;
            if (st == act) {
                if (act == ST_FETCH) {
                    exhausted = !fetch_wave(q, mode == ST_PHOTON, can_claim, sgn, sen);
                } else if (act == ST_PHOTON) {
                    this->template photon_step<2>(q);
                } else {
                    if (act == ST_ELECTRON) {
#pragma nounroll
                        for (int t = 0;;) {
                            this->electron_step(q);
                            if (++t == sc.segments || q.type == DEAD || q.pend) break;
                        }
                    }
                    // with photon sources, lanes whose electron step stopped at
                    // a hard event sample it at once, without a schedule
                    // decision in between (+0.3-1.2% on the photon workloads;
                    // with electron sources waiting for the next decision,
                    // which may fetch first, did 3-6% better)
                    if (q.type != DEAD && q.pend && (act == ST_HARD || claim_photon)) this->hard_event(q);
                }
            }
            if (__builtin_amdgcn_ballot_w64(exhausted) != 0) more_new = false;
            if (this->failed) break;
        }
    }
};

// GTAB: photon and electron tables read from device memory instead of LDS.
template <bool DIAG, bool REF, bool GTAB>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_wave(KPhase p)
{
    extern __shared__ float4 lds[];
    Env env;
    float* extra;
    stage_tables<GTAB>(p.g, lds, env, &extra);
    // wave-uniform: the wave's index, its LDS counters and its stacks
    const uint32_t w_in_block = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    volatile unsigned int* wc = (volatile unsigned int*)extra + 2 * w_in_block;
    if ((threadIdx.x & 63) == 0) {
        wc[0] = 0u;
        wc[1] = 0u;
    }
    __syncthreads();
    const size_t wave = (size_t)blockIdx.x * (blockDim.x >> 6) + w_in_block;
    WaveLane<DIAG, REF> L(p, p.scratch + wave * p.lane_bytes, wc);
    L.env = env;
    L.init_base();
    Part q;
    q.type = DEAD;
    q.pend = 0;
    L.run_wave(q, p.sched);
    L.reduce_out(p.bal, p.cnt);
}

// Bytes of one wave's stacks for `cap` records per stack (photon and electron
// records and their diagnostic event hashes).
size_t wave_stack_bytes(int cap)
{
    const size_t b = (size_t)cap * (kWaveRec + kWaveERec + 2 * sizeof(uint64_t));
    return (b + 255) & ~(size_t)255;
}

static void (*wave_kernel(int which))(KPhase)
{
    switch (which) {
    case 0: return k_wave<false, false, false>;
    case 1: return k_wave<false, true, false>;
    case 2: return k_wave<true, false, false>;
    case 3: return k_wave<true, true, false>;
    case 4: return k_wave<false, false, true>;
    case 5: return k_wave<false, true, true>;
    case 6: return k_wave<true, false, true>;
    default: return k_wave<true, true, true>;
    }
}

static int wave_which(bool diag, bool refined, bool gtab)
{
    return (gtab ? 4 : 0) | (diag ? 2 : 0) | (refined ? 1 : 0);
}

int wave_lds_bytes(int n_mat, bool gtab)
{
    return gtab ? transport_lds_bytes(0) : transport_lds_bytes(n_mat);
}

hipError_t launch_wave(const KPhase& p, int blocks, int threads, bool diag, bool gtab, hipStream_t s)
{
    const size_t lds = wave_lds_bytes(p.g.t.n_mat, gtab);
    hipLaunchKernelGGL(wave_kernel(wave_which(diag, p.g.t.refined != 0, gtab)), dim3(blocks), dim3(threads),
                       lds, s, p);
    return hipGetLastError();
}

int wave_blocks_per_cu(int threads, int n_mat, bool gtab)
{
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &n, wave_kernel(wave_which(false, false, gtab)), threads, (size_t)wave_lds_bytes(n_mat, gtab));
    return e == hipSuccess ? n : 0;
}

hipError_t init_wave_kernels(int max_lds)
{
    for (int which = 0; which < 8; ++which) {
        const hipError_t e = hipFuncSetAttribute((const void*)wave_kernel(which),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace mcd
