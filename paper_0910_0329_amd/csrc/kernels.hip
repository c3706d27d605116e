// Device side of libmcdose: the per-history transport kernel, the dose
// finalisation and small fill kernels, for gfx950 (wave64).
//
// One lane follows one source history and every secondary it creates, as in
// the paper's kernel (Fig. 1, Sec. 2.2): the source particle is sampled,
// transported, secondaries go on the lane's own stack and are popped until it
// is empty, then the history's deposits are collected.  The lane's loop takes
// one transport step per iteration (one Woodcock flight of a photon or one
// condensed-history segment of an electron), so that a wave re-converges after
// every step instead of after every particle.  Lanes take new histories from a
// global work counter when theirs is finished.
//
// Physics (Sec. 2.1): Woodcock tracking against a phantom majorant; Compton,
// photoelectric and pair interactions; electron steps limited by the
// absorption energy, the next hard event, the random-hinge budget, the voxel
// face and the energy-loss fraction; CSDA loss by inversion of the range table;
// hard Moller and bremsstrahlung events spawning secondaries.  Transport is
// FP32; dose tallies and the energy balance are FP64.
//
// Memory: cross-section tables (FP32, float4 per energy node) are staged in
// LDS by every workgroup; the phantom is one 8-byte record per voxel in HBM;
// each lane owns a slice of scratch with its particle stack and its local
// counter (an open-addressing table voxel -> energy of the current history,
// Sec. 2.4), flushed with hardware FP64 atomics at history end.
#include "engine.h"

#include "mcdose.h"

namespace mcd {

#define DEV __device__ __forceinline__

constexpr float kMC2 = 0.51099895f;
constexpr float kLn2 = 0.693147180559945309f;
constexpr float kInf = __builtin_huge_valf();

enum { PHOTON = 0, ELECTRON = 1, POSITRON = 2, DEAD = -1 };
enum { LIM_E, LIM_H, LIM_K, LIM_B, LIM_F };
// Event codes of the per-particle hash (diagnostics).
enum { EV_VIRTUAL = 1, EV_COMPTON, EV_PHOTO, EV_PAIR, EV_PAIR_VOID, EV_G_ESCAPE, EV_G_ABSORB,
       EV_SEG = 10, EV_MOLLER = 20, EV_BREMS, EV_MOLLER_VOID, EV_E_ESCAPE };

DEV float fdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
DEV float neg_ln(float u) { return -__log2f(u) * kLn2; }

// Philox4x32-10 (Salmon et al., SC'11), in place on the counter.
DEV void philox10(uint32_t k0, uint32_t k1, uint32_t& c0, uint32_t& c1, uint32_t& c2,
                  uint32_t& c3)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
}

// One particle in flight, with its random stream: the draw counter and the
// cached Philox block of (history, lineage, draw / 4).
struct Part {
    float x, y, z, u, v, w, e;
    int type;
    uint32_t l0, l1, draw, nsp;
    uint32_t b0, b1, b2, b3;
    int ix, iy, iz;          // electron voxel (state, advanced across faces)
    float nh, xi, kap;       // hard-event mfps to go, hinge fraction, hinge budget
    int before;              // 1 before the hinge of the current step
};

template <bool DIAG>
struct Lane {
    const KParams& p;
    const float4* phot;      // LDS
    const float4* elec;      // LDS
    const float* maj;        // LDS
    const float* edges;      // LDS
    const float* cdf;        // LDS
    const float* r_abs;      // LDS: R(E_abs,e) per material
    uint32_t h;              // current history
    char* stack;
    uint32_t* keys;
    float* vals;
    uint16_t* list;
    int sp, nused, lgslots, failed;
    int cur_v;
    float cur_e;
    double e_src, e_csda, e_local, e_esc, e_miss, track;
    // diagnostics
    uint32_t c[kCounters];
    double h_edep, h_track;
    uint64_t h_hash, p_hash;
    uint32_t h_parts, h_esc;

    DEV Lane(const KParams& pp, const float4* ph, const float4* el, const float* mj,
             const float* ed, const float* cd, const float* ra, char* base)
        : p(pp), phot(ph), elec(el), maj(mj), edges(ed), cdf(cd), r_abs(ra), h(0)
    {
        stack = base;
        keys = (uint32_t*)(base + (size_t)p.stack_depth * kStackRec);
        vals = (float*)(keys + p.slots);
        list = (uint16_t*)(vals + p.slots);
        sp = nused = failed = 0;
        lgslots = 31 - __builtin_clz((unsigned)p.slots);
        cur_v = -1;
        cur_e = 0.f;
        e_src = e_csda = e_local = e_esc = e_miss = track = 0.0;
        if (DIAG) {
            for (int i = 0; i < kCounters; ++i) c[i] = 0;
            h_edep = h_track = 0.0;
            h_hash = p_hash = 0;
            h_parts = h_esc = 0;
        }
    }

    DEV void count(int i) { if (DIAG) ++c[i]; }
    DEV void ev(uint32_t code) { if (DIAG) p_hash = (p_hash ^ code) * 0x100000001b3ull; }

    DEV void fail(int status)
    {
        failed = 1;
        atomicCAS(p.err, 0, status);
    }

    // ------------------------------------------------------------- random
    DEV float uni(Part& q)
    {
        const uint32_t wd = q.draw & 3u;
        if (wd == 0) {
            uint32_t c0 = h, c1 = q.l0, c2 = q.l1, c3 = q.draw >> 2;
            philox10(p.seed, p.key, c0, c1, c2, c3);
            q.b0 = c0; q.b1 = c1; q.b2 = c2; q.b3 = c3;
            count(MCD_C_PHILOX);
        }
        const uint32_t x = wd == 0 ? q.b0 : (wd == 1 ? q.b1 : (wd == 2 ? q.b2 : q.b3));
        ++q.draw;
        return ((float)(x >> 9) + 0.5f) * 0x1p-23f;
    }

    DEV void child_lineage(Part& q, uint32_t& o0, uint32_t& o1)
    {
        uint32_t c0 = h, c1 = q.l0, c2 = q.l1, c3 = 0x80000000u | q.nsp;
        philox10(p.seed, p.key, c0, c1, c2, c3);
        o0 = c0;
        o1 = c1;
        ++q.nsp;
        count(MCD_C_PHILOX);
    }

    // ------------------------------------------------------------ tables
    DEV void eidx(float e, int& i, float& fr) const
    {
        e = fminf(fmaxf(e, p.t.emin), p.t.emax);
        const float x = (__log2f(e) - p.t.l2_emin) * p.t.inv_dl2;
        i = min(max((int)x, 0), kNE - 2);
        fr = x - (float)i;
    }

    DEV float range_at(int m, float e) const
    {
        int i;
        float fr;
        eidx(e, i, fr);
        const float a = elec[m * kNE + i].x, b = elec[m * kNE + i + 1].x;
        return a + (b - a) * fr;
    }

    // Inverse of the interpolated range of material m: the node interval holding
    // r is found by walking down from interval i0 (r never exceeds the range at
    // the start of the segment), then that linear piece is solved for log E.
    DEV float range_inverse(int m, float r, int i0) const
    {
        const float4* el = elec + m * kNE;
        int j = i0;
        while (j > 0 && el[j].x > r) --j;
        if (el[j].x > r) return p.t.emin;
        while (j < kNE - 2 && el[j + 1].x <= r) ++j;
        const float r0 = el[j].x, r1 = el[j + 1].x;
        const float fr = fminf(fdiv(r - r0, r1 - r0), 1.0f);
        return exp2f(p.t.l2_emin + ((float)j + fr) * p.t.dl2);
    }

    // --------------------------------------------------------- geometry
    DEV bool inside(float x, float y, float z) const
    {
        return x >= p.x0 && x < p.x1 && y >= p.y0 && y < p.y1 && z >= p.z0 && z < p.z1;
    }

    DEV void floor_voxel(float x, float y, float z, int& ix, int& iy, int& iz) const
    {
        ix = min(max((int)floorf((x - p.x0) * p.idx), 0), p.nx - 1);
        iy = min(max((int)floorf((y - p.y0) * p.idy), 0), p.ny - 1);
        iz = min(max((int)floorf((z - p.z0) * p.idz), 0), p.nz - 1);
    }

    DEV int lin(int ix, int iy, int iz) const { return (iz * p.ny + iy) * p.nx + ix; }

    // ------------------------------------------------------------- tally
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

    // Local counter: consecutive deposits into one voxel are summed in
    // registers before they reach the lane's table.
    DEV void deposit(int v, float e)
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

    DEV void local(int v, float e)
    {
        count(MCD_C_LOCAL);
        e_local += (double)e;
        deposit(v, e);
    }

    // Dose collection at history end: S += e_{h,v}, Q += e_{h,v}^2 (FP64).
    DEV void flush_history()
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
        if (DIAG) c[MCD_C_FLUSHES] += (uint32_t)nused;
        nused = 0;
    }

    // ------------------------------------------------------------ stack
    DEV void push(int type, float e, float x, float y, float z, float u, float v, float w,
                  uint32_t l0, uint32_t l1)
    {
        if (sp >= p.stack_depth) {
            fail(MCD_E_OVERFLOW);
            return;
        }
        float4* r = (float4*)(stack + (size_t)sp * kStackRec);
        r[0] = make_float4(x, y, z, e);
        r[1] = make_float4(u, v, w, 0.f);
        r[2] = make_float4(__uint_as_float(l0), __uint_as_float(l1), __int_as_float(type), 0.f);
        ++sp;
        if (DIAG && (uint32_t)sp > c[MCD_C_MAX_STACK]) c[MCD_C_MAX_STACK] = (uint32_t)sp;
    }

    DEV void pop(Part& q)
    {
        --sp;
        const float4* r = (const float4*)(stack + (size_t)sp * kStackRec);
        const float4 a = r[0], b = r[1], c2 = r[2];
        q.x = a.x; q.y = a.y; q.z = a.z; q.e = a.w;
        q.u = b.x; q.v = b.y; q.w = b.z;
        q.l0 = __float_as_uint(c2.x);
        q.l1 = __float_as_uint(c2.y);
        q.type = __float_as_int(c2.z);
        q.draw = 0;
        q.nsp = 0;
    }

    // ------------------------------------------------------ secondaries
    // A secondary below its absorption energy is deposited on the spot (a
    // positron then annihilates with uniforms of the stream q); above it, it
    // is pushed with q's next child lineage.
    DEV void emit_photon(Part& q, float e, float x, float y, float z, float u, float v, float w,
                         int vox)
    {
        if (e <= p.t.e_abs_g) {
            local(vox, e);
            return;
        }
        uint32_t l0, l1;
        child_lineage(q, l0, l1);
        count(MCD_C_SPAWNS);
        push(PHOTON, e, x, y, z, u, v, w, l0, l1);
    }

    DEV void annihilate(Part& q, float x, float y, float z, int vox)
    {
        const float cost = 2.f * uni(q) - 1.f;
        const float ph = uni(q);
        const float sint = sqrtf(fmaxf(0.f, 1.f - cost * cost));
        const float cp = __builtin_amdgcn_cosf(ph), sph = __builtin_amdgcn_sinf(ph);
        const float dx = sint * cp, dy = sint * sph;
        emit_photon(q, kMC2, x, y, z, dx, dy, cost, vox);
        emit_photon(q, kMC2, x, y, z, -dx, -dy, -cost, vox);
    }

    DEV void emit_charged(Part& q, int type, float e, float x, float y, float z, float u,
                          float v, float w, int vox)
    {
        if (e <= p.t.e_abs_e) {
            local(vox, e);
            if (type == POSITRON) annihilate(q, x, y, z, vox);
            return;
        }
        uint32_t l0, l1;
        child_lineage(q, l0, l1);
        count(MCD_C_SPAWNS);
        push(type, e, x, y, z, u, v, w, l0, l1);
    }

    // ---------------------------------------------------------- rotation
    // Rotates (u, v, w) by polar cosine cost and azimuth (cos, sin) = (cp, sp).
    DEV static void rotate(float& u, float& v, float& w, float cost, float cp, float sph)
    {
        const float sint = sqrtf(fmaxf(0.f, 1.f - cost * cost));
        const float s = sqrtf(u * u + v * v);
        float nu, nv, nw;
        if (s < 1e-7f) {
            nu = sint * cp;
            nv = sint * sph;
            nw = (w > 0.f ? 1.f : -1.f) * cost;
        } else {
            const float is = __builtin_amdgcn_rcpf(s);
            nu = u * cost + sint * (u * w * cp - v * sph) * is;
            nv = v * cost + sint * (v * w * cp + u * sph) * is;
            nw = w * cost - s * sint * cp;
        }
        const float n = __builtin_amdgcn_rsqf(nu * nu + nv * nv + nw * nw);
        u = nu * n;
        v = nv * n;
        w = nw * n;
    }

    // ---------------------------------------------------------- particles
    DEV void start_particle(Part& q)
    {
        if (DIAG) p_hash = (0xcbf29ce484222325ull ^ ((uint64_t)q.l1 << 32 | q.l0)) * 0x100000001b3ull;
        if (q.type != PHOTON) {
            // electron birth: mfps to the first hard event, first hinge position
            floor_voxel(q.x, q.y, q.z, q.ix, q.iy, q.iz);
            q.nh = neg_ln(uni(q));
            q.xi = uni(q);
            q.kap = q.xi * p.t.kappa_step;
            q.before = 1;
        }
    }

    DEV void end_particle(Part& q)
    {
        q.type = DEAD;
        if (DIAG) {
            h_hash += p_hash;
            ++h_parts;
        }
    }

    // Source particle of history h from block 0 of the primary stream.
    DEV void start_history(Part& q)
    {
        q.l0 = q.l1 = 0;
        q.draw = 0;
        q.nsp = 0;
        const float u0 = uni(q), u1 = uni(q), u2 = uni(q), u3 = uni(q);
        const DevSource& s = p.src;
        float e;
        if (s.energy_kind == MCD_MONO) {
            e = s.e0;
        } else {
            int lo = 0, hi = s.n_bins - 1;      // first bin whose CDF exceeds u2
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (cdf[mid] > u2) hi = mid; else lo = mid + 1;
            }
            e = edges[lo] + u3 * (edges[lo + 1] - edges[lo]);
        }
        float x, y, u = 0.f, v = 0.f, w = 1.f;
        if (s.beam_kind == MCD_PENCIL) {
            x = s.pos[0];
            y = s.pos[1];
        } else {
            x = s.field[0] - s.field[2] + 2.f * s.field[2] * u0;
            y = s.field[1] - s.field[3] + 2.f * s.field[3] * u1;
            const float dx = x - s.pos[0], dy = y - s.pos[1], dz = p.z0 - s.pos[2];
            const float n = __builtin_amdgcn_rsqf(dx * dx + dy * dy + dz * dz);
            u = dx * n;
            v = dy * n;
            w = dz * n;
        }
        count(MCD_C_HISTORIES);
        e_src += (double)e + s.extra;
        q.type = DEAD;
        if (!(x >= p.x0 && x < p.x1 && y >= p.y0 && y < p.y1 && w > 0.f)) {
            e_miss += (double)e + s.extra;
            count(MCD_C_MISSES);
            return;
        }
        q.x = x; q.y = y; q.z = p.z0;
        q.u = u; q.v = v; q.w = w;
        q.e = e;
        q.draw = 4;                              // transport starts at block 1
        const float cut = s.particle == PHOTON ? p.t.e_abs_g : p.t.e_abs_e;
        if (e <= cut) {
            int ix, iy, iz;
            floor_voxel(q.x, q.y, q.z, ix, iy, iz);
            const int vx = lin(ix, iy, iz);
            local(vx, e);
            if (s.particle == POSITRON) annihilate(q, q.x, q.y, q.z, vx);
            return;
        }
        q.type = s.particle;
        start_particle(q);
    }

    DEV void finish_history(uint32_t off)
    {
        flush_history();
        if (DIAG) {
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
    }

    // One Woodcock flight and, if the stop is real, its interaction.
    DEV void photon_step(Part& q)
    {
        int i;
        float fr;
        eidx(q.e, i, fr);
        const float mu_max = maj[i] + (maj[i + 1] - maj[i]) * fr;
        const float s = fdiv(neg_ln(uni(q)), mu_max);
        count(MCD_C_FLIGHTS);
        q.x += s * q.u;
        q.y += s * q.v;
        q.z += s * q.w;
        if (!inside(q.x, q.y, q.z)) {
            ev(EV_G_ESCAPE);
            e_esc += (double)q.e;
            count(MCD_C_ESCAPES);
            if (DIAG) h_esc = 1;
            end_particle(q);
            return;
        }
        int ix, iy, iz;
        floor_voxel(q.x, q.y, q.z, ix, iy, iz);
        const int vx = lin(ix, iy, iz);
        const uint2 vd = p.vox[vx];
        const float rho = __uint_as_float(vd.x);
        const int m = (int)vd.y;
        const float4 a = phot[m * kNE + i], b = phot[m * kNE + i + 1];
        const float mu_c = rho * (a.x + (b.x - a.x) * fr);
        const float mu_pe = rho * (a.y + (b.y - a.y) * fr);
        const float mu_pp = rho * (a.z + (b.z - a.z) * fr);
        const float xs = uni(q) * mu_max;
        if (xs < mu_c) {
            ev(EV_COMPTON);
            count(MCD_C_COMPTON);
            compton(q, vx);
        } else if (xs < mu_c + mu_pe) {
            ev(EV_PHOTO);
            count(MCD_C_PHOTO);
            emit_charged(q, ELECTRON, q.e, q.x, q.y, q.z, q.u, q.v, q.w, vx);
            end_particle(q);
        } else if (xs < mu_c + mu_pe + mu_pp) {
            if (q.e > 2.f * kMC2) {
                ev(EV_PAIR);
                count(MCD_C_PAIR);
                const float ttot = q.e - 2.f * kMC2;
                const float tm = uni(q) * ttot;
                const float tp = ttot - tm;
                emit_charged(q, ELECTRON, tm, q.x, q.y, q.z, q.u, q.v, q.w, vx);
                emit_charged(q, POSITRON, tp, q.x, q.y, q.z, q.u, q.v, q.w, vx);
                end_particle(q);
            } else {
                ev(EV_PAIR_VOID);
                count(MCD_C_VOID);
            }
        } else {
            ev(EV_VIRTUAL);
            count(MCD_C_VIRTUAL);
        }
    }

    // Klein-Nishina by composition and rejection (three uniforms per try).
    DEV void compton(Part& q, int vx)
    {
        const float e = q.e;
        const float k = fdiv(e, kMC2);
        const float tmin = __builtin_amdgcn_rcpf(1.f + 2.f * k);
        const float a1 = __log2f(1.f + 2.f * k) * kLn2;
        const float a2 = 2.f * k * (1.f + k) * tmin * tmin;
        const float l2tmin = __log2f(tmin);
        float tau, cost;
        for (;;) {
            const float ua = uni(q), ub = uni(q), uc = uni(q);
            count(MCD_C_COMPTON_TRIES);
            if (ua * (a1 + a2) < a1) tau = exp2f(ub * l2tmin);
            else tau = sqrtf(tmin * tmin + ub * (1.f - tmin * tmin));
            cost = 1.f - fdiv(1.f - tau, k * tau);
            const float sin2 = 1.f - cost * cost;
            if (uc <= 1.f - fdiv(tau * sin2, 1.f + tau * tau)) break;
        }
        const float ph = uni(q);
        const float cp = __builtin_amdgcn_cosf(ph), sph = __builtin_amdgcn_sinf(ph);
        const float te = e - tau * e;          // electron energy; the photon keeps
        const float e1 = e - te;               // exactly the rest (e1 + te == e)
        const float pe2 = e * e + e1 * e1 - 2.f * e * e1 * cost;
        float cose = pe2 > 0.f ? (e - e1 * cost) * __builtin_amdgcn_rsqf(pe2) : 1.f;
        cose = fminf(fmaxf(cose, -1.f), 1.f);
        float du = q.u, dv = q.v, dw = q.w;
        rotate(du, dv, dw, cose, -cp, -sph);   // azimuth phi + pi
        emit_charged(q, ELECTRON, te, q.x, q.y, q.z, du, dv, dw, vx);
        rotate(q.u, q.v, q.w, cost, cp, sph);
        q.e = e1;
        if (e1 <= p.t.e_abs_g) {
            ev(EV_G_ABSORB);
            local(vx, e1);
            end_particle(q);
        }
    }

    // Distance along the direction to the exit face of the electron's voxel.
    DEV float boundary(const Part& q, int& axis) const
    {
        float best = kInf;
        axis = 0;
        if (q.u != 0.f) {
            const float f = p.x0 + (float)(q.u > 0.f ? q.ix + 1 : q.ix) * p.dx;
            best = fmaxf(0.f, fdiv(f - q.x, q.u));
        }
        if (q.v != 0.f) {
            const float f = p.y0 + (float)(q.v > 0.f ? q.iy + 1 : q.iy) * p.dy;
            const float d = fmaxf(0.f, fdiv(f - q.y, q.v));
            if (d < best) { best = d; axis = 1; }
        }
        if (q.w != 0.f) {
            const float f = p.z0 + (float)(q.w > 0.f ? q.iz + 1 : q.iz) * p.dz;
            const float d = fmaxf(0.f, fdiv(f - q.z, q.w));
            if (d < best) { best = d; axis = 2; }
        }
        return best;
    }

    // One condensed-history segment inside the current voxel.
    DEV void electron_step(Part& q)
    {
        const int vx = lin(q.ix, q.iy, q.iz);
        const uint2 vd = p.vox[vx];
        const float rho = __uint_as_float(vd.x);
        const float irho = __builtin_amdgcn_rcpf(rho);
        const int m = (int)vd.y;
        const float T = q.e;
        int i;
        float fr;
        eidx(T, i, fr);
        const float4 a = elec[m * kNE + i], b = elec[m * kNE + i + 1];
        const float rt = a.x + (b.x - a.x) * fr;
        const float lam = a.y + (b.y - a.y) * fr;
        const float sh = (a.z + (b.z - a.z) * fr) + (a.w + (b.w - a.w) * fr);
        // the five limits, ties resolved in the order E, h, kappa, b, f
        float l = fmaxf(0.f, (rt - r_abs[m]) * irho);
        int lim = LIM_E;
        const float l_h = sh > 0.f ? fmaxf(0.f, fdiv(q.nh, rho * sh)) : kInf;
        if (l_h < l) { l = l_h; lim = LIM_H; }
        const float l_k = fmaxf(0.f, fdiv(q.kap, rho * lam));
        if (l_k < l) { l = l_k; lim = LIM_K; }
        int axis;
        const float l_b = boundary(q, axis);
        if (l_b < l) { l = l_b; lim = LIM_B; }
        const float l_f = (rt - range_at(m, (1.f - p.t.f_e) * T)) * irho;
        if (l_f < l) { l = l_f; lim = LIM_F; }
        // move and lose energy continuously
        q.x += l * q.u;
        q.y += l * q.v;
        q.z += l * q.w;
        float tn;
        if (lim == LIM_E) tn = T > p.t.e_abs_e ? p.t.e_abs_e : T;
        else tn = fminf(T, range_inverse(m, rt - rho * l, i));
        const float dep = T - tn;
        e_csda += (double)dep;
        deposit(vx, dep);
        track += (double)l;
        if (DIAG) h_track += (double)l;
        q.nh -= l * rho * sh;
        q.kap -= l * rho * lam;
        q.e = tn;
        count(MCD_C_SEGMENTS);
        count(MCD_C_SEG_E + lim);
        ev(EV_SEG + (uint32_t)lim);

        if (lim == LIM_E) {
            local(vx, tn);
            if (q.type == POSITRON) annihilate(q, q.x, q.y, q.z, vx);
            end_particle(q);
        } else if (lim == LIM_H) {
            hard_event(q, m, vx);
        } else if (lim == LIM_K) {
            if (q.before) {
                count(MCD_C_HINGES);
                const float u = uni(q);
                const float A = p.t.a_hinge;
                const float mu = fdiv(A * u, 1.f + A - u);
                const float ph = uni(q);
                rotate(q.u, q.v, q.w, 1.f - 2.f * mu, __builtin_amdgcn_cosf(ph),
                       __builtin_amdgcn_sinf(ph));
                q.kap = (1.f - q.xi) * p.t.kappa_step;
                q.before = 0;
            } else {
                q.xi = uni(q);
                q.kap = q.xi * p.t.kappa_step;
                q.before = 1;
            }
        } else if (lim == LIM_B) {
            bool out;
            if (axis == 0) {
                q.ix += q.u > 0.f ? 1 : -1;
                out = q.ix < 0 || q.ix >= p.nx;
            } else if (axis == 1) {
                q.iy += q.v > 0.f ? 1 : -1;
                out = q.iy < 0 || q.iy >= p.ny;
            } else {
                q.iz += q.w > 0.f ? 1 : -1;
                out = q.iz < 0 || q.iz >= p.nz;
            }
            if (out) {
                ev(EV_E_ESCAPE);
                e_esc += (double)q.e + (q.type == POSITRON ? 2.0 * (double)kMC2 : 0.0);
                count(MCD_C_ESCAPES);
                if (DIAG) h_esc = 1;
                end_particle(q);
            }
        }
    }

    DEV void hard_event(Part& q, int m, int vx)
    {
        float T = q.e;
        int i;
        float fr;
        eidx(T, i, fr);
        const float4 a = elec[m * kNE + i], b = elec[m * kNE + i + 1];
        const float sm = a.z + (b.z - a.z) * fr;
        const float sb = a.w + (b.w - a.w) * fr;
        if (uni(q) * (sm + sb) < sm) {
            if (T <= 2.f * p.t.w_cc) {
                ev(EV_MOLLER_VOID);
                count(MCD_C_VOID);
            } else {
                ev(EV_MOLLER);
                count(MCD_C_MOLLER);
                const float e0 = fdiv(p.t.w_cc, T);
                const float tau = fdiv(T, kMC2);
                const float gg = fdiv(tau, tau + 1.f);
                const float c = fdiv(2.f * tau + 1.f, (tau + 1.f) * (tau + 1.f));
                float eps;
                for (;;) {
                    eps = fdiv(e0, 1.f - uni(q) * (1.f - 2.f * e0));
                    const float ua = uni(q);
                    count(MCD_C_MOLLER_TRIES);
                    const float r = fdiv(eps, 1.f - eps);
                    const float g = 1.f + r * r + gg * gg * eps * eps - c * r;
                    if (ua * 2.25f <= g) break;
                }
                const float ph = uni(q);
                const float cp = __builtin_amdgcn_cosf(ph), sph = __builtin_amdgcn_sinf(ph);
                const float tn = T - eps * T;      // primary keeps exactly T - W
                const float wd = T - tn;
                const float cs = sqrtf(fdiv(wd * (T + 2.f * kMC2), T * (wd + 2.f * kMC2)));
                const float cpr = sqrtf(fdiv(tn * (T + 2.f * kMC2), T * (tn + 2.f * kMC2)));
                float du = q.u, dv = q.v, dw = q.w;
                rotate(du, dv, dw, fminf(cs, 1.f), -cp, -sph);
                emit_charged(q, ELECTRON, wd, q.x, q.y, q.z, du, dv, dw, vx);
                rotate(q.u, q.v, q.w, fminf(cpr, 1.f), cp, sph);
                T = tn;
            }
        } else {
            ev(EV_BREMS);
            count(MCD_C_BREMS);
            const float w = fminf(p.t.w_cr * exp2f(uni(q) * __log2f(fdiv(T, p.t.w_cr))), T);
            (void)uni(q);                          // azimuth, drawn for the draw order
            const float tn = T - w;
            emit_photon(q, T - tn, q.x, q.y, q.z, q.u, q.v, q.w, vx);
            T = tn;
        }
        q.e = T;
        if (T <= p.t.e_abs_e) {
            local(vx, T);
            if (q.type == POSITRON) annihilate(q, q.x, q.y, q.z, vx);
            end_particle(q);
            return;
        }
        q.nh = neg_ln(uni(q));
    }
};

size_t lane_scratch_bytes(int stack_depth, int slots)
{
    size_t b = (size_t)stack_depth * kStackRec + (size_t)slots * 10;
    return (b + 255) & ~(size_t)255;
}

int transport_lds_bytes(int n_mat)
{
    return 2 * n_mat * kNE * (int)sizeof(float4) + (kNE + 68 + 64 + kMaxMat) * (int)sizeof(float);
}

template <bool DIAG>
__global__ __launch_bounds__(512) void k_transport(KParams p)
{
    extern __shared__ float4 lds[];
    const int nt = p.t.n_mat * kNE;
    float4* s_phot = lds;
    float4* s_elec = lds + nt;
    float* s_maj = (float*)(lds + 2 * nt);
    float* s_edges = s_maj + kNE;
    float* s_cdf = s_edges + 68;
    float* s_rabs = s_cdf + 64;
    for (int i = threadIdx.x; i < nt; i += blockDim.x) {
        s_phot[i] = p.t.phot[i];
        s_elec[i] = p.t.elec[i];
    }
    for (int i = threadIdx.x; i < kNE; i += blockDim.x) s_maj[i] = p.maj[i];
    for (int i = threadIdx.x; i < 65; i += blockDim.x) s_edges[i] = p.src.edges[i];
    for (int i = threadIdx.x; i < 64; i += blockDim.x) s_cdf[i] = p.src.cdf[i];
    for (int i = threadIdx.x; i < kMaxMat; i += blockDim.x) s_rabs[i] = p.t.r_abs[i];
    __syncthreads();

    const size_t lane_id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    Lane<DIAG> L(p, s_phot, s_elec, s_maj, s_edges, s_cdf, s_rabs,
                 p.scratch + lane_id * p.lane_bytes);
    Part q;
    q.type = DEAD;
    bool have = false;
    uint32_t off = 0, rounds = 0;
    const size_t n_lanes = (size_t)gridDim.x * blockDim.x;
    for (;;) {
        if (q.type == DEAD) {
            if (L.sp > 0) {
                L.pop(q);
                L.start_particle(q);
            } else {
                if (have) {
                    L.finish_history(off);
                    have = false;
                }
                if (L.failed || __atomic_load_n(p.err, __ATOMIC_RELAXED)) break;
                unsigned long long o;
                if (p.lockstep) {
                    // every lane of a wave takes the same history (a static
                    // round-robin over waves): the wave then runs that
                    // history's instruction path without divergence
                    o = (unsigned long long)(lane_id >> 6) + (unsigned long long)rounds * (n_lanes >> 6);
                    ++rounds;
                } else {
                    o = atomicAdd(p.next, 1ull);
                }
                if (o >= (unsigned long long)p.n) break;
                off = (uint32_t)o;
                have = true;
                L.h = p.first + off;
                L.start_history(q);
                continue;
            }
        }
        if (q.type == PHOTON) L.photon_step(q);
        else L.electron_step(q);
        if (L.failed) break;
    }

    // wave-level reduction of the energy balance, then one atomic per wave
    double b[kBal] = {L.e_src, L.e_csda, L.e_local, L.e_esc, L.e_miss, L.track};
#pragma unroll
    for (int k = 0; k < kBal; ++k)
        for (int o = 32; o > 0; o >>= 1) b[k] += __shfl_xor(b[k], o, 64);
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < kBal; ++k) unsafeAtomicAdd(&p.bal[k], b[k]);
    if (DIAG) {
        for (int k = 0; k < kCounters; ++k) {
            if (k == MCD_C_MAX_STACK) {
                uint32_t v = L.c[k];
                for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, 64));
                if ((threadIdx.x & 63) == 0) atomicMax(&p.cnt[k], (unsigned long long)v);
            } else {
                unsigned long long v = L.c[k];
                for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
                if ((threadIdx.x & 63) == 0 && v) atomicAdd(&p.cnt[k], v);
            }
        }
    }
}

hipError_t launch_transport(const KParams& p, int blocks, int threads, bool diag, hipStream_t s)
{
    const size_t lds = transport_lds_bytes(p.t.n_mat);
    const void* fn = diag ? (const void*)k_transport<true> : (const void*)k_transport<false>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (diag) hipLaunchKernelGGL(k_transport<true>, dim3(blocks), dim3(threads), lds, s, p);
    else hipLaunchKernelGGL(k_transport<false>, dim3(blocks), dim3(threads), lds, s, p);
    return hipGetLastError();
}

// ------------------------------------------------------------- finalise

// dose = S / (N rho V) and sigma from the history-by-history second moment,
// in Gy per source history; red[0] collects Dmax (as bits: doses are >= 0).
__global__ void k_dose(const double* S, const double* Q, const uint2* vox, int64_t nv,
                       double vol, double N, double* dose, double* sigma, double* red)
{
    __shared__ double smax[4];
    double mx = 0.0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv;
         v += (int64_t)gridDim.x * blockDim.x) {
        const double scale = 1.602176634e-10 / ((double)__uint_as_float(vox[v].x) * vol);
        const double mean = S[v] / N;
        const double var = (Q[v] / N - mean * mean) / (N - 1.0);
        const double d = mean * scale;
        dose[v] = d;
        sigma[v] = sqrt(var > 0.0 ? var : 0.0) * scale;
        mx = fmax(mx, d);
    }
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if ((threadIdx.x & 63) == 0) smax[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < (int)(blockDim.x >> 6); ++i) mx = fmax(mx, smax[i]);
        atomicMax((unsigned long long*)&red[0], (unsigned long long)__double_as_longlong(mx));
    }
}

// sigma-bar: mean of sigma/D over voxels with D > Dmax / 2 (red[1] sum, red[2] count).
__global__ void k_sigma_bar(const double* dose, const double* sigma, int64_t nv, double* red)
{
    const double half = 0.5 * red[0];
    double acc = 0.0, cnt = 0.0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv;
         v += (int64_t)gridDim.x * blockDim.x) {
        const double d = dose[v];
        if (d > half) {
            acc += sigma[v] / d;
            cnt += 1.0;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        acc += __shfl_xor(acc, o, 64);
        cnt += __shfl_xor(cnt, o, 64);
    }
    if ((threadIdx.x & 63) == 0 && cnt > 0.0) {
        unsafeAtomicAdd(&red[1], acc);
        unsafeAtomicAdd(&red[2], cnt);
    }
}

hipError_t launch_finalize(const double* S, const double* Q, const uint2* vox, int64_t nv,
                           double vol, uint64_t n, double* dose, double* sigma, double* red,
                           hipStream_t s)
{
    const int threads = 256;
    int blocks = (int)((nv + threads - 1) / threads);
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_dose, dim3(blocks), dim3(threads), 0, s, S, Q, vox, nv, vol, (double)n,
                       dose, sigma, red);
    hipLaunchKernelGGL(k_sigma_bar, dim3(blocks), dim3(threads), 0, s, dose, sigma, nv, red);
    return hipGetLastError();
}

// Zeroes the local-counter keys of every lane (needed once after allocation
// and after a run that stopped on an error with keys still set).
__global__ void k_clear_keys(char* scratch, size_t lanes, size_t lane_bytes, size_t key_off,
                             int slots)
{
    const size_t total = lanes * (size_t)slots;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (size_t)gridDim.x * blockDim.x) {
        const size_t lane = t / (size_t)slots, k = t % (size_t)slots;
        ((uint32_t*)(scratch + lane * lane_bytes + key_off))[k] = 0u;
    }
}

__global__ void k_fill_u32(uint32_t* p, size_t n, uint32_t v)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Fills with a kernel rather than a memset node, so that the sequence can be
// captured into a graph and replayed.
hipError_t launch_fill_u32(void* p, size_t n_words, uint32_t v, hipStream_t s)
{
    if (n_words == 0) return hipSuccess;
    size_t blocks = (n_words + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t*)p, n_words, v);
    return hipGetLastError();
}

hipError_t launch_clear_lane_keys(char* scratch, size_t lanes, size_t lane_bytes, int stack_depth,
                                  int slots, hipStream_t s)
{
    hipLaunchKernelGGL(k_clear_keys, dim3(4096), dim3(256), 0, s, scratch, lanes, lane_bytes,
                       (size_t)stack_depth * kStackRec, slots);
    return hipGetLastError();
}

}  // namespace mcd
