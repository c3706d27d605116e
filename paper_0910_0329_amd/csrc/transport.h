// Device transport machine shared by every kernel of libmcdose (gfx950, wave64).
//
// The physics follows the DPM scheme the paper ports (Sec. 2.1): photons by
// Woodcock tracking against a phantom majorant with Compton, photoelectric and
// pair interactions; electrons and positrons by condensed-history segments
// limited by the absorption energy, the next hard event, the random-hinge
// budget, the voxel face and the energy-loss fraction, with CSDA loss from the
// range table and hard Moller / bremsstrahlung events spawning secondaries.
// Transport arithmetic is FP32.
//
// Random numbers: Philox4x32-10 keyed by (seed, request key); a particle's
// counter is (history, lineage lo, lineage hi, block) and its i-th uniform is
// word i mod 4 of block i / 4, as u = ((x >> 9) + 0.5) 2^-23 (exact in FP32).
// Each particle keeps a ring of its two most recent blocks; a step refills the
// ring once at its start, so the Philox rounds run at one place per step.
//
// The machine is written once and specialised by the kernels through CRTP:
// a derived lane supplies deposit(), spawn() and the per-history bookkeeping.
#pragma once

#include "engine.h"
#include "mcdose.h"

namespace mcd {

#define DEV __device__ __forceinline__

constexpr float kMC2 = 0.51099895f;
constexpr float kLn2 = 0.693147180559945309f;
constexpr float kInf = __builtin_huge_valf();
// Draw-index flag of a secondary whose lineage is not computed yet (the
// index bits then hold its parent's spawn index).
constexpr uint32_t kLineagePending = 1u << 29;

enum { PHOTON = 0, ELECTRON = 1, POSITRON = 2, DEAD = -1 };
enum { LIM_E, LIM_H, LIM_K, LIM_B, LIM_F };
// Event codes of the per-particle hash (diagnostics).
enum { EV_VIRTUAL = 1, EV_COMPTON, EV_PHOTO, EV_PAIR, EV_PAIR_VOID, EV_G_ESCAPE, EV_G_ABSORB, EV_RAYLEIGH,
       EV_SEG = 10, EV_MOLLER = 20, EV_BREMS, EV_MOLLER_VOID, EV_E_ESCAPE, EV_BHABHA, EV_BHABHA_VOID };

DEV float fdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
// Hardware square root and base-2 exponential (v_sqrt_f32, v_exp_f32, about
// 1 ulp) in place of the correctly rounded library forms, which add up to a
// dozen instructions each for denormal scaling and rounding fix-up.  The
// transport's square roots take normal numbers or zero, and its exponentials
// give normal numbers, except the Rayleigh screening factor (1 + 2b)^-3,
// which is subtracted from 1 and vanishes there either way.
DEV float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
DEV float fexp2(float x) { return __builtin_amdgcn_exp2f(x); }

// Linear interpolation between two table nodes (fr in [0, 1)); every table
// lookup of the transport goes through it.
DEV float lerp(float a, float b, float fr) { return a + (b - a) * fr; }

// Wave-aggregated counter increment: the active lanes that reach it share one
// atomic add of their count on *ctr; each gets old + (its rank among them).
DEV unsigned int wave_fetch_add(unsigned int* ctr)
{
    const uint64_t m = __builtin_amdgcn_ballot_w64(true);
    const unsigned int rank =
        __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    unsigned int base = 0;
    if (rank == 0) base = atomicAdd(ctr, (unsigned int)__popcll(m));
    return __builtin_amdgcn_readfirstlane(base) + rank;
}

DEV unsigned long long wave_fetch_add(unsigned long long* ctr)
{
    const uint64_t m = __builtin_amdgcn_ballot_w64(true);
    const unsigned int rank =
        __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    unsigned long long base = 0;
    if (rank == 0) base = atomicAdd(ctr, (unsigned long long)__popcll(m));
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)base);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(base >> 32));
    return ((unsigned long long)hi << 32 | lo) + rank;
}
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

// One particle in flight with its random stream.
struct Part {
    float x, y, z, u, v, w, e;
    int type;
    uint32_t h;              // history
    uint32_t slot;           // request slot (batched kernels)
    uint32_t l0, l1;         // lineage
    uint32_t d;              // next draw index
    uint32_t g;              // next block to generate; blocks g-2, g-1 are in the ring
    uint32_t nsp;            // secondaries spawned from this stream
    uint32_t r0, r1, r2, r3, r4, r5, r6, r7;  // ring: block k in words 4(k&1)..4(k&1)+3
    int ix, iy, iz;          // electron voxel (state, advanced across faces)
    uint32_t vrho, vmat;     // that voxel's density bits and material (enter_voxel)
    float nh, xi, kap;       // hard-event mfps to go, hinge fraction, hinge budget
    int before;              // 1 before the hinge of the current step
    int pend;                // 1: the segment ended at a hard event not yet sampled
};

// Particle record in a stack or queue: 48 bytes.
//   f0 = (x, y, z, E), f1 = (u, v, w, bits(type | slot << 4)), f2 = bits(l0, l1, h, d)
// A secondary not started yet holds its parent's lineage and
// d = kLineagePending | spawn index (start_particle resolves it).
DEV void store_rec(char* base, const Part& q)
{
    float4* r = (float4*)base;
    r[0] = make_float4(q.x, q.y, q.z, q.e);
    r[1] = make_float4(q.u, q.v, q.w, __uint_as_float((uint32_t)q.type | (q.slot << 4)));
    r[2] = make_float4(__uint_as_float(q.l0), __uint_as_float(q.l1), __uint_as_float(q.h),
                       __uint_as_float(q.d));
}

DEV void load_rec(const char* base, Part& q)
{
    const float4* r = (const float4*)base;
    const float4 a = r[0], b = r[1], c = r[2];
    q.x = a.x; q.y = a.y; q.z = a.z; q.e = a.w;
    q.u = b.x; q.v = b.y; q.w = b.z;
    const uint32_t ts = __float_as_uint(b.w);
    q.type = (int)(ts & 15u);
    q.slot = ts >> 4;
    q.l0 = __float_as_uint(c.x);
    q.l1 = __float_as_uint(c.y);
    q.h = __float_as_uint(c.z);
    q.d = __float_as_uint(c.w);
    q.g = q.d >> 2;
    q.nsp = 0;
    q.pend = 0;
}

// Read-only view of tables staged in LDS plus the phantom geometry.
struct Env {
    const float4* phot;      // LDS [n_mat * 512]
    const float4* elec;      // LDS [n_mat * 512]
    const float* maj;        // LDS [512]
    const float* r_abs;      // LDS [kMaxMat]
    const float* ray_b;      // LDS [kMaxMat]
    const float* r_abs_pos;  // LDS [kMaxMat]: R+(E_abs,e) (positron range)
    uint32_t seed, key;      // Philox key of the particle being transported
};

// REF: compiled with the physics refinements that tables may switch on
// (emission angles, Rayleigh scattering, the second-moment hinge, Bhabha
// events).  Tables that use none of them run the kernels built without that
// code, which keeps the transport loop smaller.
template <class D, bool DIAG, bool REF>
struct Transport {
    // Bound to the kernel argument itself, so that geometry and table scalars
    // stay wave-uniform scalar loads.
    const KGeom& gm;
    Env env;
    double e_src, e_csda, e_local, e_esc, e_miss, track;
    uint32_t c[kCounters];
    uint64_t p_hash;
    int failed;

    DEV explicit Transport(const KGeom& g) : gm(g) {}
    DEV D& self() { return *static_cast<D*>(this); }
    DEV const KGeom& G() const { return gm; }

    DEV void init_base()
    {
        e_src = e_csda = e_local = e_esc = e_miss = track = 0.0;
        failed = 0;
        p_hash = 0;
        if (DIAG)
            for (int i = 0; i < kCounters; ++i) c[i] = 0;
    }

    DEV void count(int i) { if (DIAG) ++c[i]; }
    DEV void ev(uint32_t code) { if (DIAG) p_hash = (p_hash ^ code) * 0x100000001b3ull; }

    // ------------------------------------------------------------- random
    DEV void refill(Part& q)
    {
        uint32_t c0 = q.h, c1 = q.l0, c2 = q.l1, c3 = q.g;
        philox10(env.seed, env.key, c0, c1, c2, c3);
        if (q.g & 1u) {
            q.r4 = c0; q.r5 = c1; q.r6 = c2; q.r7 = c3;
        } else {
            q.r0 = c0; q.r1 = c1; q.r2 = c2; q.r3 = c3;
        }
        ++q.g;
        count(MCD_C_PHILOX);
    }

    // Called once at the start of a step.  The ring can take the next block
    // once the lane draws from its newest block (at most four uniforms left).
    // The Philox rounds run when some active lane has fewer than two
    // uniforms left, the most a flight, a segment or a particle start draws
    // outside the rejection loops; every lane with a free slot then refills
    // at the same time, so the rounds run for many lanes at once instead of
    // for a few lanes at almost every step.  After it every lane holds at
    // least two words, which those draws take with uni_ready; later draws
    // check the ring (uni, or ensure once per rejection-loop try).  The
    // rejection samplers call it with n = 4 before their loops, so that their
    // first try (which most accept) draws without a refill of a few lanes.
    DEV void prefetch(Part& q, uint32_t n = 2u)
    {
        const bool slot = (q.d >> 2) + 1u >= q.g;
        const bool need = 4u * q.g - q.d < n;
        if (__builtin_amdgcn_ballot_w64(need) != 0 && slot) refill(q);
    }

    DEV float uni(Part& q)
    {
        if ((q.d >> 2) >= q.g) refill(q);
        return uni_ready(q);
    }

    // At least n <= 4 undrawn words in the ring.  With fewer left the lane
    // draws from its newest block, so the older slot is spent and one refill
    // suffices.  Rejection loops call it once per try and then draw with
    // uni_ready, one ring check where each draw would make its own.
    DEV void ensure(Part& q, uint32_t n)
    {
        if (4u * q.g - q.d < n) refill(q);
    }

    // Word d mod 8 of the ring, chosen by a select tree on the bits of d
    // (seven selects, no branch: the lanes of a wave draw different words).
    DEV float uni_ready(Part& q)
    {
        const uint32_t d = q.d;
        const bool b0 = (d & 1u) != 0, b1 = (d & 2u) != 0, b2 = (d & 4u) != 0;
        const uint32_t w01 = b0 ? q.r1 : q.r0, w23 = b0 ? q.r3 : q.r2;
        const uint32_t w45 = b0 ? q.r5 : q.r4, w67 = b0 ? q.r7 : q.r6;
        const uint32_t x = b2 ? (b1 ? w67 : w45) : (b1 ? w23 : w01);
        q.d = d + 1u;
        return ((float)(x >> 9) + 0.5f) * 0x1p-23f;
    }

    // A secondary's lineage is the Philox block (h, parent lineage, 2^31 |
    // spawn index) under the request key.  The parent only records its own
    // lineage and the index in the secondary (d = kLineagePending | index);
    // the block is computed when the secondary starts (start_particle), in a
    // fetch with the other starting lanes rather than in the parent's
    // interaction with the few lanes that spawn there.
    DEV void defer_lineage(Part& q, Part& s)
    {
        s.l0 = q.l0;
        s.l1 = q.l1;
        s.d = kLineagePending | q.nsp;
        ++q.nsp;
    }

    DEV void resolve_lineage(Part& q)
    {
        uint32_t c0 = q.h, c1 = q.l0, c2 = q.l1, c3 = 0x80000000u | (q.d & ~kLineagePending);
        philox10(env.seed, env.key, c0, c1, c2, c3);
        q.l0 = c0;
        q.l1 = c1;
        q.d = 0;
        q.g = 0;
        count(MCD_C_PHILOX);
    }

    // ------------------------------------------------------------ tables
    // Position of energy e on the grid in node units (e clamped to the grid).
    DEV float epos(float e) const
    {
        const DevTables& t = G().t;
        e = fminf(fmaxf(e, t.emin), t.emax);
        return (__log2f(e) - t.l2_emin) * t.inv_dl2;
    }

    DEV static void node(float x, int& i, float& fr)
    {
        i = min(max((int)x, 0), kNE - 2);
        fr = x - (float)i;
    }

    DEV void eidx(float e, int& i, float& fr) const { node(epos(e), i, fr); }

    // A positron under tables with the Bhabha flag takes its own range R+
    // and hard Bhabha cross section from the global (R+, Sigma_Bh) table, in
    // place of the electron R and Sigma_M in LDS; everything else is shared.
    DEV bool own_positron(const Part& q) const { return REF && G().t.bhabha && q.type == POSITRON; }

    // Range node j of material m (electron or positron range).
    DEV float range_node(int m, int j, bool pos) const
    {
        if (pos) return G().t.posi[m * kNE + j].x;
        return env.elec[m * kNE + j].x;
    }

    // Inverse of the interpolated (electron or positron) range of material m.
    DEV float range_inverse(int m, float r, int i0, bool pos) const
    {
        if (pos) return invert_range([&](int j) { return G().t.posi[m * kNE + j].x; }, r, i0);
        return invert_range([&](int j) { return env.elec[m * kNE + j].x; }, r, i0);
    }

    // The node interval holding r (the last node j <= i0 with R_j <= r; r does
    // not exceed the range at the start of the segment) is found by a fixed
    // four-step binary search over the 16 nodes from i0 down: a segment loses
    // at most the fraction f_E of its energy, under 12 nodes of the grid, so
    // every lane takes the same four steps instead of a walk of its own
    // length.  A range below that window (only the verification entry point
    // asks for one) is walked down to.  Then that linear piece is solved for
    // log E.
    template <class F> DEV float invert_range(F rnode, float r, int i0) const
    {
        int j = max(i0 - 15, 0);
        float rj = rnode(j);
        if (rj <= r) {
#pragma unroll
            for (int step = 8; step > 0; step >>= 1) {
                const int k = min(j + step, i0);
                const float rk = rnode(k);
                if (rk <= r) {
                    j = k;
                    rj = rk;
                }
            }
        }
        while (j > 0 && rj > r) rj = rnode(--j);
        if (rj > r) return G().t.emin;
        float rn = rnode(j + 1);
        while (j < kNE - 2 && rn <= r) {
            rj = rn;
            rn = rnode(++j + 1);
        }
        const float r0 = rj, r1 = rn;
        const float fr = fminf(fdiv(r - r0, r1 - r0), 1.0f);
        return fexp2(G().t.l2_emin + ((float)j + fr) * G().t.dl2);
    }

    // --------------------------------------------------------- geometry
    DEV bool inside(float x, float y, float z) const
    {
        const KGeom& g = G();
        return x >= g.x0 && x < g.x1 && y >= g.y0 && y < g.y1 && z >= g.z0 && z < g.z1;
    }

    DEV void floor_voxel(float x, float y, float z, int& ix, int& iy, int& iz) const
    {
        const KGeom& g = G();
        ix = min(max((int)floorf((x - g.x0) * g.idx), 0), g.nx - 1);
        iy = min(max((int)floorf((y - g.y0) * g.idy), 0), g.ny - 1);
        iz = min(max((int)floorf((z - g.z0) * g.idz), 0), g.nz - 1);
    }

    DEV int lin(int ix, int iy, int iz) const { return (iz * G().ny + iy) * G().nx + ix; }

    // Loads the density and material of a charged particle's voxel once per
    // voxel (its segments and hard events read them from the particle).
    DEV void enter_voxel(Part& q) const
    {
        const uint2 vd = G().vox[lin(q.ix, q.iy, q.iz)];
        q.vrho = vd.x;
        q.vmat = vd.y;
    }

    DEV void local(const Part& q, int v, float e)
    {
        count(MCD_C_LOCAL);
        e_local += (double)e;
        self().deposit(q, v, e);
    }

    // ------------------------------------------------------ secondaries
    // A secondary below its absorption energy is deposited on the spot (a
    // positron then annihilates with uniforms of the stream q); above it, it
    // gets q's next child lineage and is handed to the lane's spawn policy.
    DEV void emit_photon(Part& q, float e, float x, float y, float z, float u, float v, float w,
                         int vox)
    {
        if (e <= G().t.e_abs_g) {
            local(q, vox, e);
            return;
        }
        Part s;
        s.type = PHOTON;
        s.e = e;
        s.x = x; s.y = y; s.z = z;
        s.u = u; s.v = v; s.w = w;
        s.h = q.h;
        s.slot = q.slot;
        defer_lineage(q, s);
        count(MCD_C_SPAWNS);
        self().spawn(s);
    }

    DEV void annihilate(Part& q, float x, float y, float z, int vox)
    {
        const float cost = 2.f * uni(q) - 1.f;
        const float ph = uni(q);
        const float sint = fsqrt(fmaxf(0.f, 1.f - cost * cost));
        const float cp = __builtin_amdgcn_cosf(ph), sph = __builtin_amdgcn_sinf(ph);
        const float dx = sint * cp, dy = sint * sph;
        emit_photon(q, kMC2, x, y, z, dx, dy, cost, vox);
        emit_photon(q, kMC2, x, y, z, -dx, -dy, -cost, vox);
    }

    DEV void emit_charged(Part& q, int type, float e, float x, float y, float z, float u,
                          float v, float w, int vox)
    {
        if (e <= G().t.e_abs_e) {
            local(q, vox, e);
            if (type == POSITRON) annihilate(q, x, y, z, vox);
            return;
        }
        Part s;
        s.type = type;
        s.e = e;
        s.x = x; s.y = y; s.z = z;
        s.u = u; s.v = v; s.w = w;
        s.h = q.h;
        s.slot = q.slot;
        defer_lineage(q, s);
        count(MCD_C_SPAWNS);
        self().spawn(s);
    }

    // --------------------------------------------------- emission angles
    // beta of an electron of kinetic energy t, and 1/beta - 1 computed as
    // 1 / (beta gamma^2 (1 + beta)) (no cancellation near beta = 1)
    DEV static void beta_a(float t, float& b, float& a)
    {
        const float g = 1.f + fdiv(t, kMC2);
        b = fdiv(fsqrt(t * (t + 2.f * kMC2)), t + kMC2);
        a = __builtin_amdgcn_rcpf(b * g * g * (1.f + b));
    }

    // Forward-peaked polar angle about the emitter: p(cos) ~ (1 - beta cos)^-2
    // on [-1, 1]; inverse CDF cos = (2u - 1 + beta) / (1 - beta + 2 beta u).
    DEV float forward_cos(Part& q, float t)
    {
        float b, a;
        beta_a(t, b, a);
        const float omb = a * b;                 // 1 - beta
        const float u = uni(q);
        return fminf(fmaxf(fdiv(2.f * u - omb, omb + 2.f * b * u), -1.f), 1.f);
    }

    // Sauter K-shell photoelectron polar angle.  In nu = 1 - cos the law is
    // nu (2 - nu) / (A + nu)^4 (1 + c (A + nu)) with A = 1/beta - 1 and
    // c = gamma (gamma - 1) (gamma - 2) beta / 2; x = nu / (A + nu) is drawn
    // with density ~ x on [0, 2 / (A + 2)] and accepted with probability
    // (1 - x)(2 - nu)(1 + c (A + nu)) / (2 m), m the largest value of the last
    // factor on [0, 2].  Two uniforms per try.
    DEV float sauter_cos(Part& q, float t)
    {
        float b, a;
        beta_a(t, b, a);
        const float g = 1.f + fdiv(t, kMC2);
        const float c = 0.5f * g * (g - 1.f) * (g - 2.f) * b;
        const float xmax = fdiv(2.f, a + 2.f);
        const float m = c >= 0.f ? 1.f + c * (a + 2.f) : 1.f + c * a;
        for (;;) {
            const float x = xmax * fsqrt(uni(q));
            const float nu = fdiv(a * x, 1.f - x);
            const float acc = fdiv((1.f - x) * (2.f - nu) * (1.f + c * (a + nu)), 2.f * m);
            if (uni(q) <= acc) return fmaxf(1.f - nu, -1.f);
        }
    }

    // Rayleigh polar angle: p(c) ~ (1 + c^2) (1 + b (1 - c))^-4, the Thomson
    // law times the squared form factor of an exponentially screened atom.
    // s = 1 - c comes from (1 + b s)^-4 on [0, 2] by inverting its CDF,
    // (1 + b s)^-3 = 1 - u (1 - (1 + 2b)^-3), and is accepted with
    // probability (1 + c^2) / 2.  Two uniforms per try.  Photons above the
    // absorption energy have b > 1, where the base-2 forms below lose at most
    // a few ulp of 1 in c.
    DEV float rayleigh_cos(Part& q, float b)
    {
        const float w = 1.f - fexp2(-3.f * __log2f(1.f + 2.f * b));
        const float ib = __builtin_amdgcn_rcpf(b);
        for (;;) {
            const float u = uni(q);
            const float s = fminf((fexp2(__log2f(1.f - u * w) * (-1.f / 3.f)) - 1.f) * ib, 2.f);
            const float c = 1.f - s;
            if (uni(q) <= 0.5f * (1.f + c * c)) return c;
        }
    }

    // ---------------------------------------------------------- rotation
    // Rotates (u, v, w) by polar cosine cost and azimuth (cos, sin) = (cp, sph).
    DEV static void rotate(float& u, float& v, float& w, float cost, float cp, float sph)
    {
        const float sint = fsqrt(fmaxf(0.f, 1.f - cost * cost));
        const float s = fsqrt(u * u + v * v);
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

    // ------------------------------------------------------- particles
    // Start of transport of a particle taken from a stack or queue (or the
    // source): an electron is born with its hard-event mfps and hinge position.
    DEV void start_particle(Part& q)
    {
        q.pend = 0;
        if (q.d & kLineagePending) resolve_lineage(q);
        if (DIAG) p_hash = (0xcbf29ce484222325ull ^ ((uint64_t)q.l1 << 32 | q.l0)) * 0x100000001b3ull;
        if (q.type != PHOTON) {
            floor_voxel(q.x, q.y, q.z, q.ix, q.iy, q.iz);
            enter_voxel(q);
            prefetch(q);                       // leaves >= 2 words
            q.nh = neg_ln(uni_ready(q));
            q.xi = uni_ready(q);
            q.kap = q.xi * G().t.kappa_step;
            q.before = 1;
        }
    }

    DEV void end_particle(Part& q)
    {
        q.type = DEAD;
        self().particle_done(q, p_hash);
    }

    // Source particle of history q.h from block 0 of its primary stream
    // (u0, u1: field position; u2: histogram bin; u3: position in the bin).
    // Returns with q.type == DEAD when the primary misses the phantom or is
    // absorbed on the spot.
    DEV void start_history(Part& q, const DevSource& s, const float* edges, const float* cdf)
    {
        const KGeom& g = G();
        q.l0 = q.l1 = 0;
        q.d = 0;
        q.g = 0;
        q.nsp = 0;
        q.pend = 0;
        ensure(q, 4);                          // block 0
        const float u0 = uni_ready(q), u1 = uni_ready(q), u2 = uni_ready(q), u3 = uni_ready(q);
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
            const float dx = x - s.pos[0], dy = y - s.pos[1], dz = g.z0 - s.pos[2];
            const float n = __builtin_amdgcn_rsqf(dx * dx + dy * dy + dz * dz);
            u = dx * n;
            v = dy * n;
            w = dz * n;
        }
        count(MCD_C_HISTORIES);
        e_src += (double)e + s.extra;
        q.type = DEAD;
        if (!(x >= g.x0 && x < g.x1 && y >= g.y0 && y < g.y1 && w > 0.f)) {
            e_miss += (double)e + s.extra;
            count(MCD_C_MISSES);
            return;
        }
        q.x = x; q.y = y; q.z = g.z0;
        q.u = u; q.v = v; q.w = w;
        q.e = e;
        q.d = 4;                              // transport starts at block 1
        const float cut = s.particle == PHOTON ? g.t.e_abs_g : g.t.e_abs_e;
        if (e <= cut) {
            int ix, iy, iz;
            floor_voxel(q.x, q.y, q.z, ix, iy, iz);
            const int vx = lin(ix, iy, iz);
            local(q, vx, e);
            if (s.particle == POSITRON) annihilate(q, q.x, q.y, q.z, vx);
            self().flush_particle(q);
            return;
        }
        q.type = s.particle;
    }

    // Woodcock flights and, once a stop is real, its interaction.  Up to
    // FLIGHTS flights per step: a flight that ends in a virtual event is
    // followed by the next in the same step, so that the interaction runs
    // with more of the wave's lanes while the lanes whose stop was real wait
    // through the extra flight.  The wave-stack kernel takes two (a third
    // costs more than it brings); the kernels that hold a particle per lane
    // take one, which keeps their registers below the spill limit.  The
    // particle's draws and events do not depend on FLIGHTS.
    template <int FLIGHTS = 1>
    DEV void photon_step(Part& q)
    {
        int i, vx, m;
        float fr, mu_max, mu_c, s_pe, s_pp, s_r, xs;
        for (int t = 0;; ++t) {
            prefetch(q);
            eidx(q.e, i, fr);
            mu_max = lerp(env.maj[i], env.maj[i + 1], fr);
            const float s = fdiv(neg_ln(uni_ready(q)), mu_max);   // prefetch left >= 2 words
            count(MCD_C_FLIGHTS);
            q.x += s * q.u;
            q.y += s * q.v;
            q.z += s * q.w;
            if (!inside(q.x, q.y, q.z)) {
                ev(EV_G_ESCAPE);
                e_esc += (double)q.e;
                count(MCD_C_ESCAPES);
                self().escaped(q);
                end_particle(q);
                return;
            }
            int ix, iy, iz;
            floor_voxel(q.x, q.y, q.z, ix, iy, iz);
            vx = lin(ix, iy, iz);
            const uint2 vd = G().vox[vx];
            const float rho = __uint_as_float(vd.x);
            m = (int)vd.y;
            const float4 a = env.phot[m * kNE + i], b = env.phot[m * kNE + i + 1];
            mu_c = rho * lerp(a.x, b.x, fr);
            const float mu_pe = rho * lerp(a.y, b.y, fr);
            const float mu_pp = rho * lerp(a.z, b.z, fr);
            const float mu_r = REF ? rho * lerp(a.w, b.w, fr) : 0.f;
            {
                // running sums of the coefficients, each rounded on its own
                // (no multiply-add contraction), so that the interaction
                // tests below and the virtual test compare against the same
                // values in every kernel that inlines this step
#pragma clang fp contract(off)
                s_pe = mu_c + mu_pe;
                s_pp = s_pe + mu_pp;
                s_r = s_pp + mu_r;
            }
            xs = uni_ready(q) * mu_max;
            // virtual exactly when xs reaches the last sum (each earlier sum
            // is at most it)
            if (xs < (REF ? s_r : s_pp) || t == FLIGHTS - 1) break;
            ev(EV_VIRTUAL);
            count(MCD_C_VIRTUAL);
        }
        if (xs < mu_c) {
            ev(EV_COMPTON);
            count(MCD_C_COMPTON);
            compton(q, vx);
        } else if (xs < s_pe) {
            ev(EV_PHOTO);
            count(MCD_C_PHOTO);
            // the photoelectron leaves along the photon, or (angular tables,
            // if it is transported) at a Sauter angle to it
            float du = q.u, dv = q.v, dw = q.w;
            if (REF && G().t.angular && q.e > G().t.e_abs_e) {
                const float cost = sauter_cos(q, q.e);
                const float ph = uni(q);
                rotate(du, dv, dw, cost, __builtin_amdgcn_cosf(ph), __builtin_amdgcn_sinf(ph));
            }
            emit_charged(q, ELECTRON, q.e, q.x, q.y, q.z, du, dv, dw, vx);
            end_particle(q);
        } else if (xs < s_pp) {
            if (q.e > 2.f * kMC2) {
                ev(EV_PAIR);
                count(MCD_C_PAIR);
                const float ttot = q.e - 2.f * kMC2;
                const float tm = uni(q) * ttot;
                const float tp = ttot - tm;
                // both leptons along the photon, or (angular tables, each one
                // that is transported) at a forward angle to it
                float du = q.u, dv = q.v, dw = q.w;
                if (REF && G().t.angular && tm > G().t.e_abs_e) {
                    const float cost = forward_cos(q, tm);
                    const float ph = uni(q);
                    rotate(du, dv, dw, cost, __builtin_amdgcn_cosf(ph), __builtin_amdgcn_sinf(ph));
                }
                emit_charged(q, ELECTRON, tm, q.x, q.y, q.z, du, dv, dw, vx);
                du = q.u;
                dv = q.v;
                dw = q.w;
                if (REF && G().t.angular && tp > G().t.e_abs_e) {
                    const float cost = forward_cos(q, tp);
                    const float ph = uni(q);
                    rotate(du, dv, dw, cost, __builtin_amdgcn_cosf(ph), __builtin_amdgcn_sinf(ph));
                }
                emit_charged(q, POSITRON, tp, q.x, q.y, q.z, du, dv, dw, vx);
                end_particle(q);
            } else {
                ev(EV_PAIR_VOID);
                count(MCD_C_VOID);
            }
        } else if (REF && xs < s_r) {
            // coherent: same energy, new direction
            ev(EV_RAYLEIGH);
            count(MCD_C_RAYLEIGH);
            const float cost = rayleigh_cos(q, env.ray_b[m] * q.e * q.e);
            const float ph = uni(q);
            rotate(q.u, q.v, q.w, cost, __builtin_amdgcn_cosf(ph), __builtin_amdgcn_sinf(ph));
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
        prefetch(q, 4u);
        for (;;) {
            ensure(q, 4);                      // three for the try, one for the azimuth
            const float ua = uni_ready(q), ub = uni_ready(q), uc = uni_ready(q);
            count(MCD_C_COMPTON_TRIES);
            if (ua * (a1 + a2) < a1) tau = fexp2(ub * l2tmin);
            else tau = fsqrt(tmin * tmin + ub * (1.f - tmin * tmin));
            cost = 1.f - fdiv(1.f - tau, k * tau);
            const float sin2 = 1.f - cost * cost;
            if (uc <= 1.f - fdiv(tau * sin2, 1.f + tau * tau)) break;
        }
        const float ph = uni_ready(q);
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
        if (e1 <= G().t.e_abs_g) {
            ev(EV_G_ABSORB);
            local(q, vx, e1);
            end_particle(q);
        }
    }

    // Distance along the direction to the exit face of the electron's voxel.
    DEV float boundary(const Part& q, int& axis) const
    {
        const KGeom& g = G();
        // per axis with selects (lanes cross different faces); a direction
        // component of zero never reaches its faces
        const float fx = g.x0 + (float)(q.u > 0.f ? q.ix + 1 : q.ix) * g.dx;
        const float fy = g.y0 + (float)(q.v > 0.f ? q.iy + 1 : q.iy) * g.dy;
        const float fz = g.z0 + (float)(q.w > 0.f ? q.iz + 1 : q.iz) * g.dz;
        const float bx = q.u != 0.f ? fmaxf(0.f, fdiv(fx - q.x, q.u)) : kInf;
        const float by = q.v != 0.f ? fmaxf(0.f, fdiv(fy - q.y, q.v)) : kInf;
        const float bz = q.w != 0.f ? fmaxf(0.f, fdiv(fz - q.z, q.w)) : kInf;
        // ties go to the lower axis
        const bool y_lt = by < bx;
        const float bxy = y_lt ? by : bx;
        const bool z_lt = bz < bxy;
        axis = z_lt ? 2 : (y_lt ? 1 : 0);
        return z_lt ? bz : bxy;
    }

    // One condensed-history segment inside the current voxel.
    DEV void electron_step(Part& q)
    {
        prefetch(q);
        const KGeom& g = G();
        const int vx = lin(q.ix, q.iy, q.iz);
        const float rho = __uint_as_float(q.vrho);
        const float irho = __builtin_amdgcn_rcpf(rho);
        const int m = (int)q.vmat;
        const float T = q.e;
        const float xt = epos(T);
        int i;
        float fr;
        node(xt, i, fr);
        const float4 a = env.elec[m * kNE + i], b = env.elec[m * kNE + i + 1];
        float rt = lerp(a.x, b.x, fr);
        const float lam = lerp(a.y, b.y, fr);
        float s_inel = lerp(a.z, b.z, fr);
        const bool pos = own_positron(q);
        if (pos) {
            const float2 p0 = g.t.posi[m * kNE + i], p1 = g.t.posi[m * kNE + i + 1];
            rt = lerp(p0.x, p1.x, fr);
            s_inel = lerp(p0.y, p1.y, fr);
        }
        const float sh = s_inel + lerp(a.w, b.w, fr);
        // the five limits, ties resolved in the order E, h, kappa, b, f
        float l = fmaxf(0.f, (rt - (pos ? env.r_abs_pos[m] : env.r_abs[m])) * irho);
        int lim = LIM_E;
        const float l_h = sh > 0.f ? fmaxf(0.f, fdiv(q.nh, rho * sh)) : kInf;
        if (l_h < l) { l = l_h; lim = LIM_H; }
        const float l_k = fmaxf(0.f, fdiv(q.kap, rho * lam));
        if (l_k < l) { l = l_k; lim = LIM_K; }
        int axis;
        const float l_b = boundary(q, axis);
        if (l_b < l) { l = l_b; lim = LIM_B; }
        // R((1 - f_E) T): on the log-uniform grid that energy lies a fixed
        // number of nodes below T
        int jf;
        float ff;
        node(xt + g.t.f_shift, jf, ff);
        const float rf0 = range_node(m, jf, pos), rf1 = range_node(m, jf + 1, pos);
        const float l_f = (rt - (rf0 + (rf1 - rf0) * ff)) * irho;
        if (l_f < l) { l = l_f; lim = LIM_F; }
        // move and lose energy continuously
        q.x += l * q.u;
        q.y += l * q.v;
        q.z += l * q.w;
        float tn;
        if (lim == LIM_E) tn = T > g.t.e_abs_e ? g.t.e_abs_e : T;
        else tn = fminf(T, range_inverse(m, rt - rho * l, i, pos));
        const float dep = T - tn;
        e_csda += (double)dep;
        self().deposit(q, vx, dep);
        track += (double)l;
        self().add_track(q, l);
        q.nh -= l * rho * sh;
        q.kap -= l * rho * lam;
        q.e = tn;
        count(MCD_C_SEGMENTS);
        count(MCD_C_SEG_E + lim);
        ev(EV_SEG + (uint32_t)lim);

        if (lim == LIM_E) {
            local(q, vx, tn);
            if (q.type == POSITRON) annihilate(q, q.x, q.y, q.z, vx);
            end_particle(q);
        } else if (lim == LIM_H) {
            q.pend = 1;                   // sampled by hard_event when the wave runs them
        } else if (lim == LIM_K) {
            // one uniform for every lane: the hinge's polar draw, or after the
            // hinge the next step's hinge fraction; only the deflection is
            // left to the lanes at a hinge
            const float u = uni_ready(q);          // prefetch left >= 2 words
            const bool hinge = q.before != 0;
            if (hinge) {
                count(MCD_C_HINGES);
                float mu;
                if (REF && g.t.hinge2) {
                    // second-moment law at the energy the hinge is reached
                    // with: no deflection when u >= B, else a Wentzel angle
                    // of screening A compressed by S
                    int j;
                    float fj;
                    eidx(q.e, j, fj);
                    const float4 h0 = g.t.hinge[m * kNE + j], h1 = g.t.hinge[m * kNE + j + 1];
                    const float A = h0.x + (h1.x - h0.x) * fj;
                    const float B = h0.y + (h1.y - h0.y) * fj;
                    const float S = h0.z + (h1.z - h0.z) * fj;
                    const float v = fminf(fdiv(u, B), 1.f);
                    mu = u < B ? S * fdiv(A * v, 1.f + A - v) : 0.f;
                } else {
                    const float A = g.t.a_hinge;
                    mu = fdiv(A * u, 1.f + A - u);
                }
                const float ph = uni_ready(q);
                rotate(q.u, q.v, q.w, 1.f - 2.f * mu, __builtin_amdgcn_cosf(ph),
                       __builtin_amdgcn_sinf(ph));
            }
            q.kap = (hinge ? 1.f - q.xi : u) * g.t.kappa_step;
            q.xi = hinge ? q.xi : u;
            q.before = hinge ? 0 : 1;
        } else if (lim == LIM_B) {
            // one voxel along the crossed axis, with selects (lanes cross
            // different faces)
            const float da = axis == 0 ? q.u : (axis == 1 ? q.v : q.w);
            const int st = da > 0.f ? 1 : -1;
            q.ix += axis == 0 ? st : 0;
            q.iy += axis == 1 ? st : 0;
            q.iz += axis == 2 ? st : 0;
            const bool out = (unsigned)q.ix >= (unsigned)g.nx || (unsigned)q.iy >= (unsigned)g.ny ||
                             (unsigned)q.iz >= (unsigned)g.nz;
            if (!out) enter_voxel(q);
            if (out) {
                ev(EV_E_ESCAPE);
                e_esc += (double)q.e + (q.type == POSITRON ? 2.0 * (double)kMC2 : 0.0);
                count(MCD_C_ESCAPES);
                self().escaped(q);
                end_particle(q);
            }
        }
    }

    // The hard event that ended the last segment of q (Moller or
    // bremsstrahlung, chosen by their cross sections at T), then the number
    // of mean free paths to the next one.
    // Bhabha event of a positron of kinetic energy T (T updated): the atomic
    // electron takes W = e T, e on [w_cc / T, 1] with density
    // e^-2 [1 - b1 e + b2 e^2 - b3 e^3 + b4 e^4], drawn from e^-2 by inversion
    // and accepted with the bracket (two uniforms per try).  With tau = T/mc^2
    // and a = (tau / (tau + 1))^2: b1 = a (2 (tau + 2)^2 - 1) / (tau (tau + 2)),
    // b2 = a (3 (tau + 2)^2 + 1) / (tau + 2)^2, b3 = 2a (tau + 1) tau / (tau + 2)^2,
    // b4 = a tau^2 / (tau + 2)^2.  Both leave at the two-body angles.
    DEV void bhabha(Part& q, float& T, int vx)
    {
        const KGeom& g = G();
        if (T <= g.t.w_cc) {
            ev(EV_BHABHA_VOID);
            count(MCD_C_VOID);
            return;
        }
        ev(EV_BHABHA);
        count(MCD_C_BHABHA);
        const float e0 = fdiv(g.t.w_cc, T);
        const float tau = fdiv(T, kMC2);
        const float r = fdiv(tau, tau + 1.f);
        const float a = r * r;
        const float tp = tau + 2.f;
        const float itp2 = __builtin_amdgcn_rcpf(tp * tp);
        const float b1 = a * fdiv(2.f * tp * tp - 1.f, tau * tp);
        const float b2 = a * (3.f * tp * tp + 1.f) * itp2;
        const float b3 = 2.f * a * (tau + 1.f) * tau * itp2;
        const float b4 = a * tau * tau * itp2;
        float eps;
        for (;;) {
            eps = fdiv(e0, 1.f - uni(q) * (1.f - e0));
            const float ua = uni(q);
            count(MCD_C_MOLLER_TRIES);
            const float br = 1.f - eps * (b1 - eps * (b2 - eps * (b3 - eps * b4)));
            if (ua <= br) break;
        }
        eps = fminf(eps, 1.f);
        const float ph = uni(q);
        const float cp = __builtin_amdgcn_cosf(ph), sph = __builtin_amdgcn_sinf(ph);
        const float tn = T - eps * T;          // the positron keeps exactly T - W
        const float wd = T - tn;
        const float cs = fsqrt(fdiv(wd * (T + 2.f * kMC2), T * (wd + 2.f * kMC2)));
        const float cpr = fsqrt(fdiv(tn * (T + 2.f * kMC2), T * (tn + 2.f * kMC2)));
        float du = q.u, dv = q.v, dw = q.w;
        rotate(du, dv, dw, fminf(cs, 1.f), -cp, -sph);
        emit_charged(q, ELECTRON, wd, q.x, q.y, q.z, du, dv, dw, vx);
        rotate(q.u, q.v, q.w, fminf(cpr, 1.f), cp, sph);
        T = tn;
    }

    DEV void hard_event(Part& q)
    {
        const KGeom& g = G();
        q.pend = 0;
        prefetch(q, 4u);                       // the choice, a Moller try and its azimuth
        const int vx = lin(q.ix, q.iy, q.iz);
        const int m = (int)q.vmat;
        float T = q.e;
        int i;
        float fr;
        eidx(T, i, fr);
        const float4 a = env.elec[m * kNE + i], b = env.elec[m * kNE + i + 1];
        float sm = lerp(a.z, b.z, fr);
        const float sb = lerp(a.w, b.w, fr);
        const bool pos = own_positron(q);
        if (pos) {
            const float2 p0 = g.t.posi[m * kNE + i], p1 = g.t.posi[m * kNE + i + 1];
            sm = lerp(p0.y, p1.y, fr);
        }
        const bool inelastic = uni(q) * (sm + sb) < sm;
        if (pos && inelastic) {
            bhabha(q, T, vx);
        } else if (inelastic) {
            if (T <= 2.f * g.t.w_cc) {
                ev(EV_MOLLER_VOID);
                count(MCD_C_VOID);
            } else {
                ev(EV_MOLLER);
                count(MCD_C_MOLLER);
                const float e0 = fdiv(g.t.w_cc, T);
                const float tau = fdiv(T, kMC2);
                const float gg = fdiv(tau, tau + 1.f);
                const float c = fdiv(2.f * tau + 1.f, (tau + 1.f) * (tau + 1.f));
                float eps;
                for (;;) {
                    ensure(q, 3);              // two for the try, one for the azimuth
                    eps = fdiv(e0, 1.f - uni_ready(q) * (1.f - 2.f * e0));
                    const float ua = uni_ready(q);
                    count(MCD_C_MOLLER_TRIES);
                    const float r = fdiv(eps, 1.f - eps);
                    const float gv = 1.f + r * r + gg * gg * eps * eps - c * r;
                    if (ua * 2.25f <= gv) break;
                }
                const float ph = uni_ready(q);
                const float cp = __builtin_amdgcn_cosf(ph), sph = __builtin_amdgcn_sinf(ph);
                const float tn = T - eps * T;      // primary keeps exactly T - W
                const float wd = T - tn;
                const float cs = fsqrt(fdiv(wd * (T + 2.f * kMC2), T * (wd + 2.f * kMC2)));
                const float cpr = fsqrt(fdiv(tn * (T + 2.f * kMC2), T * (tn + 2.f * kMC2)));
                float du = q.u, dv = q.v, dw = q.w;
                rotate(du, dv, dw, fminf(cs, 1.f), -cp, -sph);
                emit_charged(q, ELECTRON, wd, q.x, q.y, q.z, du, dv, dw, vx);
                rotate(q.u, q.v, q.w, fminf(cpr, 1.f), cp, sph);
                T = tn;
            }
        } else {
            ev(EV_BREMS);
            count(MCD_C_BREMS);
            const float w = fminf(g.t.w_cr * fexp2(uni(q) * __log2f(fdiv(T, g.t.w_cr))), T);
            // the photon goes along the electron, or (angular tables) at a
            // forward angle to it; the azimuth is drawn either way
            const float ph = uni(q);
            float du = q.u, dv = q.v, dw = q.w;
            if (REF && g.t.angular) {
                const float cost = forward_cos(q, T);
                rotate(du, dv, dw, cost, __builtin_amdgcn_cosf(ph), __builtin_amdgcn_sinf(ph));
            }
            const float tn = T - w;
            emit_photon(q, T - tn, q.x, q.y, q.z, du, dv, dw, vx);
            T = tn;
        }
        q.e = T;
        if (T <= g.t.e_abs_e) {
            local(q, vx, T);
            if (q.type == POSITRON) annihilate(q, q.x, q.y, q.z, vx);
            end_particle(q);
            return;
        }
        q.nh = neg_ln(uni(q));
    }

    // ---------------------------------------------------- wave schedule
    // Each lane holds one particle in one of four states: it needs a new
    // particle (FETCH), it is a photon (PHOTON), an electron or positron
    // (ELECTRON), or its last segment ended at a hard event (HARD).  Every
    // iteration the wave picks one kind of work from the lanes' states and
    // only the lanes in that state run it, so the wave runs one code path with
    // as many lanes as it can: the rare, long paths (fetching a particle,
    // which includes starting and closing histories, and sampling a hard
    // event) wait until a share of the live lanes need them (1/fetch_div and
    // 1/hard_div), and photons run when they are at least 1/photon_div of the
    // electrons.  A lane's own particle and stream never change: only the
    // time at which its steps run.  Returns when the lane's fetch finds no
    // more work, or on failure.
    enum { ST_FETCH, ST_PHOTON, ST_ELECTRON, ST_HARD };

    DEV void run(Part& q, const Sched sc)
    {
        for (;;) {
            const int st = q.type == DEAD ? ST_FETCH
                         : (q.type == PHOTON ? ST_PHOTON : (q.pend ? ST_HARD : ST_ELECTRON));
            const uint64_t live = __builtin_amdgcn_ballot_w64(true);
            const int n = __popcll(live);
            const int nf = __popcll(__builtin_amdgcn_ballot_w64(st == ST_FETCH));
            const int np = __popcll(__builtin_amdgcn_ballot_w64(st == ST_PHOTON));
            const int nh = __popcll(__builtin_amdgcn_ballot_w64(st == ST_HARD));
            const int ne = n - nf - np - nh;
            int act;
            if (nf && (nf * sc.fetch_div >= n || nf == n)) act = ST_FETCH;
            else if (nh && (nh * sc.hard_div >= n || nh + nf == n)) act = ST_HARD;
            else if (np && np * sc.photon_div >= ne) act = ST_PHOTON;
            else if (ne) act = ST_ELECTRON;
            else act = nh ? ST_HARD : ST_FETCH;
            if (DIAG && __builtin_amdgcn_mbcnt_hi((uint32_t)(live >> 32),
                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)live, 0u)) == 0) {
                const int na = act == ST_FETCH ? nf : act == ST_PHOTON ? np : act == ST_ELECTRON ? ne : nh;
                ++c[MCD_C_ITERS];
                c[MCD_C_LIVE] += (uint32_t)n;
                ++c[MCD_C_IT_FETCH + act];
                c[MCD_C_LN_FETCH + act] += (uint32_t)na;
            }
            if (st == act) {
                if (act == ST_FETCH) {
                    if (!self().fetch(q)) break;
                } else if (act == ST_PHOTON) {
                    photon_step(q);
                } else if (act == ST_ELECTRON) {
                    electron_step(q);
                } else {
                    hard_event(q);
                }
            }
            if (failed) break;
        }
    }

    // Wave-level reduction of the energy balance and counters, one atomic per wave.
    DEV void reduce_out(double* bal, unsigned long long* cnt)
    {
        double b[kBal] = {e_src, e_csda, e_local, e_esc, e_miss, track};
#pragma unroll
        for (int k = 0; k < kBal; ++k)
            for (int o = 32; o > 0; o >>= 1) b[k] += __shfl_xor(b[k], o, 64);
        if ((threadIdx.x & 63) == 0)
            for (int k = 0; k < kBal; ++k) unsafeAtomicAdd(&bal[k], b[k]);
        if (DIAG) {
            for (int k = 0; k < kCounters; ++k) {
                if (k == MCD_C_MAX_STACK) {
                    uint32_t v = c[k];
                    for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, 64));
                    if ((threadIdx.x & 63) == 0) atomicMax(&cnt[k], (unsigned long long)v);
                } else {
                    unsigned long long v = c[k];
                    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
                    if ((threadIdx.x & 63) == 0 && v) atomicAdd(&cnt[k], v);
                }
            }
        }
    }
};

// Stages the material tables and the majorant into LDS (dynamic shared memory
// laid out as phot | elec | maj | r_abs | ray_b | r_abs_pos | extra floats).
// GTAB: the photon and electron tables stay in device memory (read through
// L1/L2); only the majorant and the per-material scalars go to LDS.
template <bool GTAB = false>
DEV void stage_tables(const KGeom& g, float4* lds, Env& env, float** extra)
{
    const int nt = GTAB ? 0 : g.t.n_mat * kNE;
    float4* s_phot = lds;
    float4* s_elec = lds + nt;
    float* s_maj = (float*)(lds + 2 * nt);
    float* s_rabs = s_maj + kNE;
    float* s_rayb = s_rabs + kMaxMat;
    float* s_rabp = s_rayb + kMaxMat;
    for (int i = threadIdx.x; i < nt; i += blockDim.x) {
        s_phot[i] = g.t.phot[i];
        s_elec[i] = g.t.elec[i];
    }
    for (int i = threadIdx.x; i < kNE; i += blockDim.x) s_maj[i] = g.maj[i];
    for (int i = threadIdx.x; i < kMaxMat; i += blockDim.x) {
        s_rabs[i] = g.t.r_abs[i];
        s_rayb[i] = g.t.ray_b[i];
        s_rabp[i] = g.t.r_abs_pos[i];
    }
    env.phot = GTAB ? g.t.phot : s_phot;
    env.elec = GTAB ? g.t.elec : s_elec;
    env.maj = s_maj;
    env.r_abs = s_rabs;
    env.ray_b = s_rayb;
    env.r_abs_pos = s_rabp;
    *extra = s_rabp + kMaxMat;
}

}  // namespace mcd
