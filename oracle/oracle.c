/*
 * FP64 reference for coupled electron-photon Monte Carlo dose (DPM scheme,
 * Jia et al. Sec. 2.1-2.4).  TEST INFRASTRUCTURE ONLY: loaded by the tests, the
 * smoke check and the benchmark's CPU-baseline leg, never by the product path.
 *
 * Every history follows the flow of Fig. 1 (Sec. 2.2): the source particle is
 * generated, transported, its secondaries are kept on a stack and popped until
 * the stack is empty, and the history's deposits are collected into the dose
 * counters.  The physics of each step follows Sec. 2.1:
 *   photons    Woodcock (delta) tracking against a majorant attenuation;
 *              Compton (Klein-Nishina), photoelectric and pair interactions;
 *   electrons  condensed history for elastic scattering (one random-hinge
 *              deflection per step of kappa_step transport mean free paths),
 *              continuous slowing down below the production thresholds, and
 *              detailed hard Moller and bremsstrahlung events above them.
 * The paper leaves the details of each model to DPM; the readings used here
 * are listed with the design notes of this repository and repeated at each
 * step below.
 *
 * Random numbers: Philox4x32-10 keyed by (seed, request key) with counter
 * (history, lineage lo, lineage hi, block); the i-th uniform of a particle is
 * word i mod 4 of block i / 4, converted as u = ((x >> 9) + 0.5) 2^-23.  A
 * secondary's lineage is words 0-1 of the block (history, parent lineage,
 * 0x80000000 | spawn index).  Block 0 of the primary
 * is reserved for source sampling.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define PI 3.14159265358979323846
#define MC2 0.51099895              /* MeV */
#define MEV_PER_G_TO_GY 1.602176634e-10
#define NE 512
#define NQ 13
#define A0 5.29177210903e-9         /* Bohr radius, cm */
#define HBARC 1.973269804e-11       /* MeV cm */

enum { Q_MUC, Q_MUPE, Q_MUPP, Q_R, Q_L1INV, Q_SM, Q_SB, Q_LR, Q_MUR, Q_L2INV, Q_RP, Q_SBH, Q_LRP };
enum { PHOTON = 0, ELECTRON = 1, POSITRON = 2 };
/* Blob flag: emission angles of photoelectrons (Sauter), bremsstrahlung
 * photons and pair leptons instead of their parent's direction. */
#define FLAG_ANGULAR 4u
/* Blob flag: the hinge angle matches the second Lewis moment as well. */
#define FLAG_HINGE2 32u
/* Blob flag: positrons take their own range (Q_RP) and hard Bhabha events
 * (Q_SBH) in place of the electron range and Moller events. */
#define FLAG_BHABHA 64u

/* ------------------------------------------------------------------ Philox */

void orc_philox(uint32_t k0, uint32_t k1, const uint32_t ctr[4], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {                       /* Weyl key schedule */
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* u = ((x >> 9) + 0.5) 2^-23 = (2k + 1) 2^-24: 23 random bits, strictly inside
 * (0, 1) and exactly representable in FP32 as well as FP64. */
double orc_uniform(uint32_t x)
{
    return ((double)(x >> 9) + 0.5) * (1.0 / 8388608.0);
}

/* ------------------------------------------------------------------ tables */

typedef struct {
    int n_mat;
    double emin, emax, e_abs_e, e_abs_g, w_cc, w_cr, kappa_step, f_e, a_hinge;
    uint32_t flags;
    double ln_emin, dlog;          /* ln E_0 and the grid step in ln E */
    double ray_b[256];             /* Rayleigh form factor: b = ray_b[m] E^2 */
    double* q;                     /* [n_mat][NQ][NE] */
} tables;

#define HDR_BYTES (8 + 4 * 4 + 9 * 8 + 2 * 4)
#define MAT_BYTES (16 + 6 * 8 + NQ * NE * 8)

static double rd_f64(const unsigned char* p) { double v; memcpy(&v, p, 8); return v; }
static uint32_t rd_u32(const unsigned char* p) { uint32_t v; memcpy(&v, p, 4); return v; }

/* Parses and validates the blob; returns 0 and fills t (caller frees t->q). */
static int load_tables(const void* blob, size_t nbytes, tables* t)
{
    const unsigned char* b = (const unsigned char*)blob;
    if (!blob || nbytes < HDR_BYTES || memcmp(b, "MCDTAB\0\1", 8) != 0) return -1;
    if (rd_u32(b + 8) != 4 || rd_u32(b + 16) != NE || rd_u32(b + 20) != NQ) return -1;
    int n_mat = (int)rd_u32(b + 12);
    if (n_mat < 1 || n_mat > 255 || nbytes != (size_t)HDR_BYTES + (size_t)n_mat * MAT_BYTES)
        return -1;
    const unsigned char* p = b + 24;
    t->n_mat = n_mat;
    t->emin = rd_f64(p); t->emax = rd_f64(p + 8); t->e_abs_e = rd_f64(p + 16);
    t->e_abs_g = rd_f64(p + 24); t->w_cc = rd_f64(p + 32); t->w_cr = rd_f64(p + 40);
    t->kappa_step = rd_f64(p + 48); t->f_e = rd_f64(p + 56); t->a_hinge = rd_f64(p + 64);
    t->flags = rd_u32(p + 72);
    if (t->flags & ~127u) return -1;   /* flags 1, 2, 4, 8, 16, 32, 64 only */
    if (!(t->emin > 0 && t->emax > t->emin && t->e_abs_e > t->emin && t->e_abs_e < t->emax &&
          t->e_abs_g > t->emin && t->e_abs_g < t->emax && t->w_cc > 0 && t->w_cr > 0 &&
          t->kappa_step > 0 && t->f_e > 0 && t->f_e < 1 && t->a_hinge > 0))
        return -1;
    t->ln_emin = log(t->emin);
    t->dlog = log(t->emax / t->emin) / (NE - 1);
    t->q = (double*)malloc(sizeof(double) * (size_t)n_mat * NQ * NE);
    if (!t->q) return -1;
    for (int m = 0; m < n_mat; ++m) {
        const unsigned char* mh = b + HDR_BYTES + (size_t)m * MAT_BYTES + 16;
        memcpy(t->q + (size_t)m * NQ * NE, mh + 6 * 8, sizeof(double) * NQ * NE);
        /* screening radius a = 0.885 a0 Z_s^(-1/3), Z_s = B / (Z/A) from the
         * material header (rho, Z/A, I, B, ...); b = 2 (k a)^2, k = E / (hbar c) */
        double zoa = rd_f64(mh + 8), bz = rd_f64(mh + 24);
        double a = 0.885 * A0 * pow(bz / zoa, -1.0 / 3.0);
        t->ray_b[m] = 2.0 * a * a / (HBARC * HBARC);
    }
    for (size_t i = 0; i < (size_t)n_mat * NQ * NE; ++i)
        if (!(t->q[i] >= 0.0) || !isfinite(t->q[i])) { free(t->q); return -1; }
    for (int m = 0; m < n_mat; ++m)
        for (int k = 0; k < 2; ++k) {
            const double* r = t->q + ((size_t)m * NQ + (k ? Q_RP : Q_R)) * NE;
            for (int i = 1; i < NE; ++i)
                if (!(r[i] > r[i - 1])) { free(t->q); return -1; }
        }
    return 0;
}

static const double* tab(const tables* t, int m, int q) { return t->q + ((size_t)m * NQ + q) * NE; }

/* f(E) = f_i + (f_{i+1} - f_i) (ln E - ln E_i) / dlog, E clamped to the grid. */
static double interp(const tables* t, const double* f, double e)
{
    if (e < t->emin) e = t->emin;
    if (e > t->emax) e = t->emax;
    double x = (log(e) - t->ln_emin) / t->dlog;
    int i = (int)floor(x);
    if (i < 0) i = 0;
    if (i > NE - 2) i = NE - 2;
    double fr = x - i;
    return f[i] + (f[i + 1] - f[i]) * fr;
}

/* Inverse of the interpolated range: locate the node interval holding r by
 * bisection, then solve that linear piece for ln T. */
static double range_inverse(const tables* t, const double* R, double r)
{
    if (r <= R[0]) return t->emin;
    if (r >= R[NE - 1]) return t->emax;
    int lo = 0, hi = NE - 1;
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (R[mid] <= r) lo = mid; else hi = mid;
    }
    double fr = (r - R[lo]) / (R[lo + 1] - R[lo]);
    return exp(t->ln_emin + (lo + fr) * t->dlog);
}

int orc_blob_check(const void* blob, size_t nbytes)
{
    tables t;
    if (load_tables(blob, nbytes, &t)) return -1;
    free(t.q);
    return t.n_mat;
}

int orc_interp(const void* blob, size_t nbytes, int m, int q, double e, double* out)
{
    tables t;
    if (load_tables(blob, nbytes, &t)) return -1;
    int rc = -1;
    if (m >= 0 && m < t.n_mat && q >= 0 && q < NQ) { *out = interp(&t, tab(&t, m, q), e); rc = 0; }
    free(t.q);
    return rc;
}

int orc_range_inverse(const void* blob, size_t nbytes, int m, double r, double* out)
{
    tables t;
    if (load_tables(blob, nbytes, &t)) return -1;
    int rc = -1;
    if (m >= 0 && m < t.n_mat) { *out = range_inverse(&t, tab(&t, m, Q_R), r); rc = 0; }
    free(t.q);
    return rc;
}

void orc_philox_n(uint32_t k0, uint32_t k1, const uint32_t* ctr, size_t n, uint32_t* out)
{
    for (size_t i = 0; i < n; ++i) orc_philox(k0, k1, ctr + 4 * i, out + 4 * i);
}

int orc_interp_n(const void* blob, size_t nbytes, int m, int q, const double* e, size_t n, double* out)
{
    tables t;
    if (load_tables(blob, nbytes, &t)) return -1;
    int rc = -1;
    if (m >= 0 && m < t.n_mat && q >= 0 && q < NQ) {
        for (size_t i = 0; i < n; ++i) out[i] = interp(&t, tab(&t, m, q), e[i]);
        rc = 0;
    }
    free(t.q);
    return rc;
}

int orc_range_inverse_n(const void* blob, size_t nbytes, int m, int q, const double* r, size_t n,
                        double* out)
{
    tables t;
    if (load_tables(blob, nbytes, &t)) return -1;
    int rc = -1;
    if (m >= 0 && m < t.n_mat && (q == Q_R || q == Q_RP)) {
        for (size_t i = 0; i < n; ++i) out[i] = range_inverse(&t, tab(&t, m, q), r[i]);
        rc = 0;
    }
    free(t.q);
    return rc;
}

/* ---------------------------------------------------------------- geometry */

typedef struct {
    orc_grid g;
    double xmax, ymax, zmax;
    const uint8_t* mat;
    const float* rho;
} geom;

static int check_phantom(const tables* t, const orc_grid* g, const uint8_t* mat, const float* rho)
{
    if (!g || !mat || !rho || g->nx < 1 || g->ny < 1 || g->nz < 1) return -1;
    if (!(g->dx > 0 && g->dy > 0 && g->dz > 0)) return -1;
    size_t nv = (size_t)g->nx * g->ny * g->nz;
    for (size_t v = 0; v < nv; ++v)
        if (mat[v] >= t->n_mat || !(rho[v] > 0.0f) || !isfinite(rho[v])) return -1;
    return 0;
}

static void make_geom(geom* G, const orc_grid* g, const uint8_t* mat, const float* rho)
{
    G->g = *g;
    G->xmax = g->x0 + g->nx * g->dx;
    G->ymax = g->y0 + g->ny * g->dy;
    G->zmax = g->z0 + g->nz * g->dz;
    G->mat = mat;
    G->rho = rho;
}

static int inside(const geom* G, double x, double y, double z)
{
    return x >= G->g.x0 && x < G->xmax && y >= G->g.y0 && y < G->ymax && z >= G->g.z0 &&
           z < G->zmax;
}

static int clampi(int a, int lo, int hi) { return a < lo ? lo : (a > hi ? hi : a); }

/* Voxel holding a point inside the box: floor of the scaled coordinates. */
static void floor_voxel(const geom* G, double x, double y, double z, int idx[3])
{
    idx[0] = clampi((int)floor((x - G->g.x0) / G->g.dx), 0, G->g.nx - 1);
    idx[1] = clampi((int)floor((y - G->g.y0) / G->g.dy), 0, G->g.ny - 1);
    idx[2] = clampi((int)floor((z - G->g.z0) / G->g.dz), 0, G->g.nz - 1);
}

static size_t lin_voxel(const geom* G, const int idx[3])
{
    return ((size_t)idx[2] * G->g.ny + idx[1]) * G->g.nx + idx[0];
}

/* Majorant mu_max(E_i) = max over materials present of rho_max,m * sum of the
 * photon attenuation coefficients per gram at node i (Woodcock, Sec. 2.1). */
static void build_majorant(const tables* t, const geom* G, double* mu)
{
    double rmax[256];
    for (int m = 0; m < 256; ++m) rmax[m] = 0.0;
    size_t nv = (size_t)G->g.nx * G->g.ny * G->g.nz;
    for (size_t v = 0; v < nv; ++v)
        if ((double)G->rho[v] > rmax[G->mat[v]]) rmax[G->mat[v]] = G->rho[v];
    for (int i = 0; i < NE; ++i) {
        double best = 0.0;
        for (int m = 0; m < t->n_mat; ++m) {
            if (rmax[m] <= 0.0) continue;
            double s = tab(t, m, Q_MUC)[i] + tab(t, m, Q_MUPE)[i] + tab(t, m, Q_MUPP)[i] +
                       tab(t, m, Q_MUR)[i];
            if (rmax[m] * s > best) best = rmax[m] * s;
        }
        mu[i] = best;
    }
}

int orc_majorant(const void* blob, size_t nbytes, const orc_grid* g, const uint8_t* mat,
                 const float* rho, double* out512)
{
    tables t;
    if (load_tables(blob, nbytes, &t)) return -1;
    int rc = -1;
    if (!check_phantom(&t, g, mat, rho)) {
        geom G;
        make_geom(&G, g, mat, rho);
        build_majorant(&t, &G, out512);
        rc = 0;
    }
    free(t.q);
    return rc;
}

/* ------------------------------------------------------------ rng streams */

typedef struct {
    uint32_t k0, k1, h;
    uint64_t lineage;
    uint32_t draw;        /* index of the next uniform */
    uint32_t nspawn;      /* secondaries spawned from this stream so far */
    uint32_t blk_id, blk[4];
    int have;
    uint64_t* cnt;
} stream;

static void stream_init(stream* s, uint32_t k0, uint32_t k1, uint32_t h, uint64_t lineage,
                        uint64_t* cnt)
{
    s->k0 = k0; s->k1 = k1; s->h = h; s->lineage = lineage;
    s->draw = 0; s->nspawn = 0; s->have = 0; s->blk_id = 0; s->cnt = cnt;
}

static double uni(stream* s)
{
    uint32_t b = s->draw >> 2;
    if (!s->have || s->blk_id != b) {
        uint32_t ctr[4] = {s->h, (uint32_t)s->lineage, (uint32_t)(s->lineage >> 32), b};
        orc_philox(s->k0, s->k1, ctr, s->blk);
        s->blk_id = b;
        s->have = 1;
        if (s->cnt) s->cnt[ORC_C_PHILOX]++;
    }
    return orc_uniform(s->blk[s->draw++ & 3]);
}

static uint64_t child_lineage(stream* s)
{
    uint32_t ctr[4] = {s->h, (uint32_t)s->lineage, (uint32_t)(s->lineage >> 32),
                       0x80000000u | s->nspawn};
    uint32_t o[4];
    orc_philox(s->k0, s->k1, ctr, o);
    s->nspawn++;
    if (s->cnt) s->cnt[ORC_C_PHILOX]++;
    return (uint64_t)o[0] | ((uint64_t)o[1] << 32);
}

/* ----------------------------------------------------------- directions */

/* Rotate unit vector d by polar cosine `cost` and azimuth `phi` about itself. */
static void rotate(double d[3], double cost, double phi)
{
    double sint = sqrt(fmax(0.0, 1.0 - cost * cost));
    double cp = cos(phi), sp = sin(phi);
    double s = sqrt(d[0] * d[0] + d[1] * d[1]);
    double u, v, w;
    if (s < 1e-7) {
        u = sint * cp;
        v = sint * sp;
        w = (d[2] > 0 ? 1.0 : -1.0) * cost;
    } else {
        u = d[0] * cost + sint * (d[0] * d[2] * cp - d[1] * sp) / s;
        v = d[1] * cost + sint * (d[1] * d[2] * cp + d[0] * sp) / s;
        w = d[2] * cost - s * sint * cp;
    }
    double n = 1.0 / sqrt(u * u + v * v + w * w);
    d[0] = u * n; d[1] = v * n; d[2] = w * n;
}

/* -------------------------------------------------------------- samplers */

/* Klein-Nishina by composition and rejection: tau = E'/E drawn from 1/tau with
 * weight ln(1 + 2k) or from tau with weight 2k(1+k)/(1+2k)^2, accepted with
 * probability 1 - tau sin^2(theta) / (1 + tau^2).  Three uniforms per try. */
static void sample_compton(stream* s, double e, double* cost_out, double* tau_out, uint64_t* cnt)
{
    double k = e / MC2;
    double tmin = 1.0 / (1.0 + 2.0 * k);
    double a1 = log(1.0 + 2.0 * k);
    double a2 = 2.0 * k * (1.0 + k) / ((1.0 + 2.0 * k) * (1.0 + 2.0 * k));
    for (;;) {
        double ua = uni(s), ub = uni(s), uc = uni(s);
        if (cnt) cnt[ORC_C_COMPTON_TRIES]++;
        double tau;
        if (ua * (a1 + a2) < a1) tau = exp(ub * log(tmin));
        else tau = sqrt(tmin * tmin + ub * (1.0 - tmin * tmin));
        double cost = 1.0 - (1.0 - tau) / (k * tau);
        double sin2 = 1.0 - cost * cost;
        if (uc <= 1.0 - tau * sin2 / (1.0 + tau * tau)) {
            *cost_out = cost;
            *tau_out = tau;
            return;
        }
    }
}

/* Hard Moller energy fraction eps on [W_cc/T, 1/2]: eps drawn from 1/eps^2 and
 * accepted with g(eps) / (9/4).  Two uniforms per try. */
static double sample_moller(stream* s, double t, double w_cc, uint64_t* cnt)
{
    double e0 = w_cc / t;
    double tau = t / MC2;
    double gg = tau / (tau + 1.0);
    double c = (2.0 * tau + 1.0) / ((tau + 1.0) * (tau + 1.0));
    for (;;) {
        double eps = e0 / (1.0 - uni(s) * (1.0 - 2.0 * e0));
        double ua = uni(s);
        if (cnt) cnt[ORC_C_MOLLER_TRIES]++;
        double r = eps / (1.0 - eps);
        double g = 1.0 + r * r + gg * gg * eps * eps - c * r;
        if (ua * 2.25 <= g) return eps;
    }
}

/* Bhabha: fraction e = W / t given to the atomic electron, on [w_cc / t, 1],
 * density ~ e^-2 [1 - b1 e + b2 e^2 - b3 e^3 + b4 e^4] with
 *   b1 = a (2 (g + 1)^2 - 1) / (g^2 - 1),  b2 = a (3 (g + 1)^2 + 1) / (g + 1)^2,
 *   b3 = a 2 g (g - 1) / (g + 1)^2,        b4 = a (g - 1)^2 / (g + 1)^2,
 * a = ((g - 1) / g)^2, g the positron's Lorentz factor.  e is drawn from e^-2
 * by inversion and accepted with the bracket (at most 1).  Two uniforms per
 * try. */
static double sample_bhabha(stream* s, double t, double w_cc, uint64_t* cnt)
{
    double e0 = w_cc / t;
    double g = 1.0 + t / MC2;
    double a = (g - 1.0) / g;
    a *= a;
    double gp = g + 1.0;
    double b1 = a * (2.0 * gp * gp - 1.0) / (g * g - 1.0);
    double b2 = a * (3.0 * gp * gp + 1.0) / (gp * gp);
    double b3 = a * 2.0 * g * (g - 1.0) / (gp * gp);
    double b4 = a * (g - 1.0) * (g - 1.0) / (gp * gp);
    for (;;) {
        double e = e0 / (1.0 - uni(s) * (1.0 - e0));
        double ua = uni(s);
        if (cnt) cnt[ORC_C_MOLLER_TRIES]++;
        double br = 1.0 - e * (b1 - e * (b2 - e * (b3 - e * b4)));
        if (ua <= br) return e;
    }
}

/* Kramers-type bremsstrahlung: W = W_cr (T / W_cr)^u, a 1/W law on [W_cr, T]. */
static double sample_brems(stream* s, double t, double w_cr)
{
    return w_cr * pow(t / w_cr, uni(s));
}

static double beta_of(double t) { return sqrt(t * (t + 2.0 * MC2)) / (t + MC2); }

/* Forward-peaked emission at leading relativistic order: the polar angle
 * about the emitter's direction has p(cos) proportional to (1 - beta cos)^-2
 * on [-1, 1], beta that of an electron of kinetic energy t.  Its CDF inverts
 * in closed form: cos = (2u - 1 + beta) / (1 - beta + 2 beta u). */
static double sample_forward_cos(stream* s, double t)
{
    double b = beta_of(t);
    double u = uni(s);
    return (2.0 * u - 1.0 + b) / (1.0 - b + 2.0 * b * u);
}

/* Sauter's K-shell photoelectron distribution for an electron of kinetic
 * energy t, in nu = 1 - cos:
 *   p(nu) ~ nu (2 - nu) / (A + nu)^4 * (1 + c (A + nu)),
 *   A = 1/beta - 1,  c = gamma (gamma - 1) (gamma - 2) beta / 2.
 * With x = nu / (A + nu) the factor nu / (A + nu)^4 dnu becomes x (1 - x) dx
 * / A^2, so x is drawn from p(x) ~ x on [0, 2 / (A + 2)] and accepted with
 * probability (1 - x)(2 - nu)(1 + c (A + nu)) / (2 m), m the largest value of
 * 1 + c (A + nu) on [0, 2] (the factor stays positive for every gamma > 1).
 * Two uniforms per try. */
static double sample_sauter_cos(stream* s, double t)
{
    double g = 1.0 + t / MC2, b = beta_of(t);
    double a = 1.0 / b - 1.0;
    double c = 0.5 * g * (g - 1.0) * (g - 2.0) * b;
    double xmax = 2.0 / (a + 2.0);
    double m = c >= 0.0 ? 1.0 + c * (a + 2.0) : 1.0 + c * a;
    for (;;) {
        double x = xmax * sqrt(uni(s));
        double nu = a * x / (1.0 - x);
        double acc = (1.0 - x) * (2.0 - nu) * (1.0 + c * (a + nu)) / (2.0 * m);
        if (uni(s) <= acc) return 1.0 - nu;
    }
}

/* Rayleigh polar angle: p(c) ~ (1 + c^2) (1 + b (1 - c))^-4 (screened
 * Thomson law), b = ray_b[m] E^2.  s = 1 - c is drawn from (1 + b s)^-4 on
 * [0, 2] by inverting its CDF,
 *   (1 + b s)^-3 = 1 - u (1 - (1 + 2b)^-3),
 * written with log1p / expm1, and accepted with probability (1 + c^2) / 2.
 * Two uniforms per try. */
static double sample_rayleigh_cos(stream* s, double b)
{
    double w = -expm1(-3.0 * log1p(2.0 * b));
    for (;;) {
        double u = uni(s);
        double sd = b > 0.0 ? expm1(-log1p(-u * w) / 3.0) / b : 2.0 * u;
        double c = 1.0 - sd;
        if (uni(s) <= 0.5 * (1.0 + c * c)) return c;
    }
}

/* Random hinge: Wentzel angular law with screening A, mu = (1 - cos)/2 =
 * A u / (1 + A - u). */
static double sample_hinge_cos(stream* s, double a)
{
    double u = uni(s);
    double mu = a * u / (1.0 + a - u);
    return 1.0 - 2.0 * mu;
}

/* Second-moment hinge.  After a step of kappa transport mean free paths the
 * Lewis moments of the deflection are <P1> = exp(-kappa) and
 * <P2> = exp(-kappa r), r = lambda1 / lambda2; in mu = (1 - cos)/2 (with
 * 1 - P2 = 6 mu (1 - mu)) that is
 *   m1 = <mu>   = (1 - exp(-kappa)) / 2,
 *   m2 = <mu^2> = m1 - (1 - exp(-kappa r)) / 6.
 * The first-moment Wentzel law (screening a1) fixes m1 only.  With
 * t = m2 / m1 and q(A) = <mu^2>_A / <mu>_A of the Wentzel law, increasing in A:
 *   t >= q(a1)  heavier tail: mixture (1 - B) delta(mu) + B Wentzel(A), with
 *               q(A) = t and B = m1 / <mu>_A;
 *   t <  q(a1)  lighter tail: Wentzel(A) compressed to [0, S], mu = S mu_A,
 *               with <mu>_A^2 / <mu^2>_A = m1^2 / m2 and S = t / q(A).
 * Either way mu = S * A u' / (1 + A - u') with u' = u / B when u < B, else
 * mu = 0: one uniform, as for the first-moment hinge.  If no root lies in
 * [a1, 1e3] the first-moment law is kept (A = a1, B = S = 1). */
static double wentzel_m1(double a) { return a * ((1.0 + a) * log1p(1.0 / a) - 1.0); }
static double wentzel_m2(double a)
{
    return a * ((1.0 + 2.0 * a) - 2.0 * a * (1.0 + a) * log1p(1.0 / a));
}
static double wentzel_q(double a) { return wentzel_m2(a) / wentzel_m1(a); }
static double wentzel_f(double a) { double m = wentzel_m1(a); return m * m / wentzel_m2(a); }

/* root of g(A) = target on [lo, hi] for increasing g, by bisection in ln A;
 * returns 0 if the target is not bracketed */
static int solve_increasing(double (*g)(double), double target, double lo, double hi, double* out)
{
    if (!(g(lo) <= target && g(hi) >= target)) return 0;
    for (int it = 0; it < 200 && hi / lo - 1.0 > 1e-15; ++it) {
        double mid = sqrt(lo * hi);
        if (g(mid) < target) lo = mid;
        else hi = mid;
    }
    *out = sqrt(lo * hi);
    return 1;
}

static void hinge2_params(double kappa, double a1, double r, double* A, double* B, double* S)
{
    double m1 = -0.5 * expm1(-kappa);
    double m2 = m1 + expm1(-kappa * r) / 6.0;
    *A = a1;
    *B = 1.0;
    *S = 1.0;
    if (!(m2 > m1 * m1) || !(m2 < m1)) return;
    double t = m2 / m1;
    double a;
    if (t >= wentzel_q(a1)) {
        if (solve_increasing(wentzel_q, t, a1, 1e3, &a)) {
            *A = a;
            *B = m1 / wentzel_m1(a);
        }
    } else if (solve_increasing(wentzel_f, m1 * m1 / m2, a1, 1e3, &a)) {
        *A = a;
        *S = t / wentzel_q(a);
    }
}

static double sample_hinge2_cos(stream* s, double kappa, double a1, double r)
{
    double A, B, S;
    hinge2_params(kappa, a1, r, &A, &B, &S);
    double u = uni(s);
    double mu = 0.0;
    if (u < B) {
        u /= B;
        mu = S * A * u / (1.0 + A - u);
    }
    return 1.0 - 2.0 * mu;
}

/* -------------------------------------------------------------- transport */

typedef struct {
    int type;
    double e;
    double r[3], d[3];
    uint64_t lineage;
} particle;

typedef struct {
    const tables* t;
    const geom* G;
    const double* mu_max;
    double r_abs[256];                 /* R(E_abs,e) per material */
    double r_abs_pos[256];             /* the same on the positron range */
    uint32_t k0, k1;
    uint32_t h;
    /* tally: per-history accumulation flushed at history end */
    double *S, *Q, *temp;
    double* Sb;                        /* optional: 16 group tallies, history mod 16 */
    size_t nv;
    unsigned char* touched;
    size_t *list, n_list, cap_list;
    double* bal;
    uint64_t* cnt;
    orc_history* hist;                 /* record of the current history or NULL */
    particle* stack;
    size_t sp, cap;
    int oom;
} ctx;

static uint64_t hash_init(uint64_t lineage) { return (0xcbf29ce484222325ull ^ lineage) * 0x100000001b3ull; }
static void hash_ev(uint64_t* hp, uint32_t code) { *hp = (*hp ^ code) * 0x100000001b3ull; }

enum { EV_VIRTUAL = 1, EV_COMPTON, EV_PHOTO, EV_PAIR, EV_PAIR_VOID, EV_G_ESCAPE, EV_G_ABSORB, EV_RAYLEIGH,
       EV_SEG = 10, EV_MOLLER = 20, EV_BREMS, EV_MOLLER_VOID, EV_E_ESCAPE, EV_BHABHA, EV_BHABHA_VOID };

static void deposit(ctx* c, size_t v, double e, int channel)
{
    if (e == 0.0) return;
    c->bal[channel] += e;
    if (c->hist) c->hist->edep += e;
    if (!c->touched[v]) {
        if (c->n_list == c->cap_list) {
            size_t nc = c->cap_list ? 2 * c->cap_list : 1024;
            size_t* nl = (size_t*)realloc(c->list, nc * sizeof(size_t));
            if (!nl) { c->oom = 1; return; }
            c->list = nl;
            c->cap_list = nc;
        }
        c->touched[v] = 1;
        c->list[c->n_list++] = v;
    }
    c->temp[v] += e;
}

/* Dose collection at the end of a history: S += e_{h,v}, Q += e_{h,v}^2. */
static void flush_history(ctx* c)
{
    for (size_t i = 0; i < c->n_list; ++i) {
        size_t v = c->list[i];
        c->S[v] += c->temp[v];
        c->Q[v] += c->temp[v] * c->temp[v];
        if (c->Sb) c->Sb[(size_t)(c->h & 15u) * c->nv + v] += c->temp[v];
        c->temp[v] = 0.0;
        c->touched[v] = 0;
    }
    c->cnt[ORC_C_FLUSHES] += c->n_list;
    c->n_list = 0;
}

static void push(ctx* c, const particle* p)
{
    if (c->sp == c->cap) {
        size_t nc = c->cap ? 2 * c->cap : 64;
        particle* ns = (particle*)realloc(c->stack, nc * sizeof(particle));
        if (!ns) { c->oom = 1; return; }
        c->stack = ns;
        c->cap = nc;
    }
    c->stack[c->sp++] = *p;
    if (c->sp > c->cnt[ORC_C_MAX_STACK]) c->cnt[ORC_C_MAX_STACK] = c->sp;
}

static void annihilate(ctx* c, stream* s, const double r[3], size_t v);

/* A secondary created at r (inside voxel v) with direction d: below its
 * absorption energy it is deposited on the spot (a positron also annihilates,
 * with uniforms from stream s); otherwise it is spawned with the next child
 * lineage of s. */
static void emit(ctx* c, stream* s, int type, double e, const double r[3], const double d[3],
                 size_t v)
{
    double cut = type == PHOTON ? c->t->e_abs_g : c->t->e_abs_e;
    if (e <= cut) {
        c->cnt[ORC_C_LOCAL]++;
        deposit(c, v, e, ORC_E_LOCAL);
        if (type == POSITRON) annihilate(c, s, r, v);
        return;
    }
    particle p;
    p.type = type;
    p.e = e;
    memcpy(p.r, r, sizeof p.r);
    memcpy(p.d, d, sizeof p.d);
    p.lineage = child_lineage(s);
    c->cnt[ORC_C_SPAWNS]++;
    push(c, &p);
}

/* Positron annihilation at rest: two m c^2 photons, isotropic and back to back. */
static void annihilate(ctx* c, stream* s, const double r[3], size_t v)
{
    double cost = 2.0 * uni(s) - 1.0;
    double phi = 2.0 * PI * uni(s);
    double sint = sqrt(fmax(0.0, 1.0 - cost * cost));
    double d1[3] = {sint * cos(phi), sint * sin(phi), cost};
    double d2[3] = {-d1[0], -d1[1], -d1[2]};
    emit(c, s, PHOTON, MC2, r, d1, v);
    emit(c, s, PHOTON, MC2, r, d2, v);
}

/* One Woodcock flight: fly an exponential distance with the majorant, then
 * accept the stop as Compton / photoelectric / pair in proportion to the local
 * coefficients, or as virtual.  Returns the event code (EV_G_ESCAPE if the
 * photon left the box) and the voxel of the stop. */
static int photon_flight(ctx* c, stream* s, double e, double r[3], const double d[3], int idx[3])
{
    const tables* t = c->t;
    double mu_max = interp(t, c->mu_max, e);
    double dist = -log(uni(s)) / mu_max;
    c->cnt[ORC_C_FLIGHTS]++;
    r[0] += dist * d[0];
    r[1] += dist * d[1];
    r[2] += dist * d[2];
    if (!inside(c->G, r[0], r[1], r[2])) return EV_G_ESCAPE;
    floor_voxel(c->G, r[0], r[1], r[2], idx);
    size_t v = lin_voxel(c->G, idx);
    int m = c->G->mat[v];
    double rho = c->G->rho[v];
    double mu_c = rho * interp(t, tab(t, m, Q_MUC), e);
    double mu_pe = rho * interp(t, tab(t, m, Q_MUPE), e);
    double mu_pp = rho * interp(t, tab(t, m, Q_MUPP), e);
    double mu_r = rho * interp(t, tab(t, m, Q_MUR), e);
    double x = uni(s) * mu_max;
    if (x < mu_c) return EV_COMPTON;
    if (x < mu_c + mu_pe) return EV_PHOTO;
    if (x < mu_c + mu_pe + mu_pp) return e > 2.0 * MC2 ? EV_PAIR : EV_PAIR_VOID;
    if (x < mu_c + mu_pe + mu_pp + mu_r) return EV_RAYLEIGH;
    return EV_VIRTUAL;
}

static void transport_photon(ctx* c, stream* s, double e, double r[3], double d[3], uint64_t* ph)
{
    const tables* t = c->t;
    int idx[3];
    for (;;) {
        int ev = photon_flight(c, s, e, r, d, idx);
        hash_ev(ph, (uint32_t)ev);
        if (ev == EV_G_ESCAPE) {
            c->bal[ORC_E_ESC] += e;
            c->cnt[ORC_C_ESCAPES]++;
            if (c->hist) c->hist->escaped = 1;
            return;
        }
        size_t v = lin_voxel(c->G, idx);
        if (ev == EV_VIRTUAL || ev == EV_PAIR_VOID) {
            c->cnt[ev == EV_VIRTUAL ? ORC_C_VIRTUAL : ORC_C_VOID]++;
            continue;
        }
        if (ev == EV_RAYLEIGH) {
            /* coherent: the photon keeps its energy and turns by a screened
             * Thomson angle */
            c->cnt[ORC_C_RAYLEIGH]++;
            double cost = sample_rayleigh_cos(s, t->ray_b[c->G->mat[v]] * e * e);
            rotate(d, cost, 2.0 * PI * uni(s));
            continue;
        }
        if (ev == EV_COMPTON) {
            c->cnt[ORC_C_COMPTON]++;
            double cost, tau;
            sample_compton(s, e, &cost, &tau, c->cnt);
            double phi = 2.0 * PI * uni(s);
            double e1 = tau * e;
            double te = e - e1;
            /* electron direction from momentum conservation, azimuth phi + pi */
            double pe = sqrt(e * e + e1 * e1 - 2.0 * e * e1 * cost);
            double cose = pe > 0.0 ? (e - e1 * cost) / pe : 1.0;
            if (cose > 1.0) cose = 1.0;
            if (cose < -1.0) cose = -1.0;
            double de[3] = {d[0], d[1], d[2]};
            rotate(de, cose, phi + PI);
            emit(c, s, ELECTRON, te, r, de, v);
            rotate(d, cost, phi);
            e = e1;
            if (e <= t->e_abs_g) {
                hash_ev(ph, EV_G_ABSORB);
                c->cnt[ORC_C_LOCAL]++;
                deposit(c, v, e, ORC_E_LOCAL);
                return;
            }
            continue;
        }
        const int angular = (t->flags & FLAG_ANGULAR) != 0;
        if (ev == EV_PHOTO) {
            /* photon absorbed; the photoelectron takes all of E, along d, or
             * (angular flag, if it is transported) at a Sauter angle to d */
            c->cnt[ORC_C_PHOTO]++;
            double de[3] = {d[0], d[1], d[2]};
            if (angular && e > t->e_abs_e) {
                double cost = sample_sauter_cos(s, e);
                rotate(de, cost, 2.0 * PI * uni(s));
            }
            emit(c, s, ELECTRON, e, r, de, v);
            return;
        }
        /* pair: kinetic energy E - 2mc^2 shared uniformly, both along d, or
         * (angular flag, each lepton that is transported) at a forward angle */
        c->cnt[ORC_C_PAIR]++;
        double ttot = e - 2.0 * MC2;
        double tm = uni(s) * ttot;
        double tp = ttot - tm;
        double dm[3] = {d[0], d[1], d[2]}, dp[3] = {d[0], d[1], d[2]};
        if (angular && tm > t->e_abs_e) {
            double cost = sample_forward_cos(s, tm);
            rotate(dm, cost, 2.0 * PI * uni(s));
        }
        emit(c, s, ELECTRON, tm, r, dm, v);
        if (angular && tp > t->e_abs_e) {
            double cost = sample_forward_cos(s, tp);
            rotate(dp, cost, 2.0 * PI * uni(s));
        }
        emit(c, s, POSITRON, tp, r, dp, v);
        return;
    }
}

/* Distance along d to the exit face of voxel idx; *axis gets the face's axis. */
static double boundary_distance(const geom* G, const double r[3], const double d[3],
                                const int idx[3], int* axis)
{
    const double o[3] = {G->g.x0, G->g.y0, G->g.z0};
    const double w[3] = {G->g.dx, G->g.dy, G->g.dz};
    double best = INFINITY;
    *axis = 0;
    for (int a = 0; a < 3; ++a) {
        double dist;
        if (d[a] > 0.0) dist = (o[a] + (idx[a] + 1) * w[a] - r[a]) / d[a];
        else if (d[a] < 0.0) dist = (o[a] + idx[a] * w[a] - r[a]) / d[a];
        else continue;
        if (dist < 0.0) dist = 0.0;
        if (dist < best) { best = dist; *axis = a; }
    }
    return best;
}

enum { LIM_E, LIM_H, LIM_K, LIM_B, LIM_F };

static void transport_electron(ctx* c, stream* s, int type, double T, double r[3], double d[3],
                               uint64_t* ph)
{
    const tables* t = c->t;
    const geom* G = c->G;
    int idx[3];
    floor_voxel(G, r[0], r[1], r[2], idx);
    /* birth: hard-event mean free paths to go, and the hinge position */
    double n_h = -log(uni(s));
    double xi = uni(s);
    double kap = xi * t->kappa_step;
    int before = 1;
    /* with the Bhabha flag a positron takes its own range and hard Bhabha
     * events; otherwise it shares the electron's quantities */
    const int bhabha = type == POSITRON && (t->flags & FLAG_BHABHA);
    const int q_r = bhabha ? Q_RP : Q_R, q_s = bhabha ? Q_SBH : Q_SM;
    const double* r_abs = bhabha ? c->r_abs_pos : c->r_abs;
    for (;;) {
        size_t v = lin_voxel(G, idx);
        int m = G->mat[v];
        double rho = G->rho[v];
        const double* R = tab(t, m, q_r);
        double rt = interp(t, R, T);
        double lam = interp(t, tab(t, m, Q_L1INV), T);
        double sh = interp(t, tab(t, m, q_s), T) + interp(t, tab(t, m, Q_SB), T);
        /* the five step limits, ties resolved in the order E, h, kappa, b, f */
        double l_e = fmax(0.0, (rt - r_abs[m]) / rho);
        double l_h = sh > 0.0 ? fmax(0.0, n_h / (rho * sh)) : INFINITY;
        double l_k = fmax(0.0, kap / (rho * lam));
        int axis;
        double l_b = boundary_distance(G, r, d, idx, &axis);
        double l_f = (rt - interp(t, R, (1.0 - t->f_e) * T)) / rho;
        double l = l_e;
        int lim = LIM_E;
        if (l_h < l) { l = l_h; lim = LIM_H; }
        if (l_k < l) { l = l_k; lim = LIM_K; }
        if (l_b < l) { l = l_b; lim = LIM_B; }
        if (l_f < l) { l = l_f; lim = LIM_F; }
        /* move and lose energy continuously (CSDA) */
        r[0] += l * d[0];
        r[1] += l * d[1];
        r[2] += l * d[2];
        double tn;
        if (lim == LIM_E) tn = T > t->e_abs_e ? t->e_abs_e : T;
        else tn = fmin(T, range_inverse(t, R, rt - rho * l));
        deposit(c, v, T - tn, ORC_E_CSDA);
        c->bal[ORC_TRACK_E] += l;
        if (c->hist) c->hist->track_e += l;
        n_h -= l * rho * sh;
        kap -= l * rho * lam;
        T = tn;
        c->cnt[ORC_C_SEGMENTS]++;
        c->cnt[ORC_C_SEG_E + lim]++;
        hash_ev(ph, EV_SEG + (uint32_t)lim);

        if (lim == LIM_E) {
            c->cnt[ORC_C_LOCAL]++;
            deposit(c, v, T, ORC_E_LOCAL);
            if (type == POSITRON) annihilate(c, s, r, v);
            return;
        }
        if (lim == LIM_H) {
            double sm = interp(t, tab(t, m, q_s), T);
            double sb = interp(t, tab(t, m, Q_SB), T);
            if (uni(s) * (sm + sb) < sm) {
                /* inelastic: Moller for electrons (the primary keeps the
                 * larger share, W <= T/2); with the Bhabha flag, Bhabha for
                 * positrons (the atomic electron may take any W <= T).  Both
                 * particles leave at the two-body angles. */
                double w_min = bhabha ? t->w_cc : 2.0 * t->w_cc;
                if (T <= w_min) {
                    /* interpolation tail below the threshold: no event */
                    c->cnt[ORC_C_VOID]++;
                    hash_ev(ph, bhabha ? EV_BHABHA_VOID : EV_MOLLER_VOID);
                } else {
                    c->cnt[bhabha ? ORC_C_BHABHA : ORC_C_MOLLER]++;
                    hash_ev(ph, bhabha ? EV_BHABHA : EV_MOLLER);
                    double eps = bhabha ? sample_bhabha(s, T, t->w_cc, c->cnt)
                                        : sample_moller(s, T, t->w_cc, c->cnt);
                    double phi = 2.0 * PI * uni(s);
                    double w = eps * T;
                    double cs = sqrt(w * (T + 2.0 * MC2) / (T * (w + 2.0 * MC2)));
                    double cp = sqrt((T - w) * (T + 2.0 * MC2) / (T * (T - w + 2.0 * MC2)));
                    double dd[3] = {d[0], d[1], d[2]};
                    rotate(dd, cs, phi + PI);
                    emit(c, s, ELECTRON, w, r, dd, v);
                    rotate(d, cp, phi);
                    T -= w;
                }
            } else {
                c->cnt[ORC_C_BREMS]++;
                hash_ev(ph, EV_BREMS);
                double w = sample_brems(s, T, t->w_cr);
                /* the photon goes along the electron, or (angular flag) at a
                 * forward angle to it; the azimuth is drawn either way */
                double phi = 2.0 * PI * uni(s);
                double dg[3] = {d[0], d[1], d[2]};
                if (t->flags & FLAG_ANGULAR) rotate(dg, sample_forward_cos(s, T), phi);
                emit(c, s, PHOTON, w, r, dg, v);
                T -= w;
            }
            if (T <= t->e_abs_e) {
                c->cnt[ORC_C_LOCAL]++;
                deposit(c, v, T, ORC_E_LOCAL);
                if (type == POSITRON) annihilate(c, s, r, v);
                return;
            }
            n_h = -log(uni(s));
            continue;
        }
        if (lim == LIM_K) {
            if (before) {
                c->cnt[ORC_C_HINGES]++;
                double cost;
                if (t->flags & FLAG_HINGE2) {
                    /* lambda1 / lambda2 at the energy the hinge is reached with */
                    double r = interp(t, tab(t, m, Q_L2INV), T) / interp(t, tab(t, m, Q_L1INV), T);
                    cost = sample_hinge2_cos(s, t->kappa_step, t->a_hinge, r);
                } else {
                    cost = sample_hinge_cos(s, t->a_hinge);
                }
                double phi = 2.0 * PI * uni(s);
                rotate(d, cost, phi);
                kap = (1.0 - xi) * t->kappa_step;
                before = 0;
            } else {
                xi = uni(s);
                kap = xi * t->kappa_step;
                before = 1;
            }
            continue;
        }
        if (lim == LIM_B) {
            idx[axis] += d[axis] > 0.0 ? 1 : -1;
            int n_ax = axis == 0 ? G->g.nx : (axis == 1 ? G->g.ny : G->g.nz);
            if (idx[axis] < 0 || idx[axis] >= n_ax) {
                c->bal[ORC_E_ESC] += T + (type == POSITRON ? 2.0 * MC2 : 0.0);
                c->cnt[ORC_C_ESCAPES]++;
                if (c->hist) c->hist->escaped = 1;
                hash_ev(ph, EV_E_ESCAPE);
                return;
            }
        }
        /* LIM_F: re-evaluate the tables at the new energy */
    }
}

static void transport(ctx* c, stream* s, int type, double e, double r[3], double d[3])
{
    uint64_t ph = hash_init(s->lineage);
    if (type == PHOTON) transport_photon(c, s, e, r, d, &ph);
    else transport_electron(c, s, type, e, r, d, &ph);
    if (c->hist) {
        c->hist->hash += ph;
        c->hist->n_particles++;
    }
}

/* ------------------------------------------------------------------ source */

static int check_source(const orc_source* src)
{
    if (!src || src->particle < 0 || src->particle > 2) return -1;
    if (src->energy_kind == 0) {
        if (!(src->e0 > 0.0) || src->e0 > 20.0) return -1;
    } else if (src->energy_kind == 1) {
        if (src->n_bins < 1 || src->n_bins > 64) return -1;
        double sw = 0.0;
        for (int b = 0; b < src->n_bins; ++b) {
            if (!(src->weights[b] >= 0.0) || !(src->edges[b + 1] > src->edges[b])) return -1;
            sw += src->weights[b];
        }
        if (!(sw > 0.0) || !(src->edges[0] > 0.0) || src->edges[src->n_bins] > 20.0) return -1;
    } else {
        return -1;
    }
    if (src->beam_kind != 0 && src->beam_kind != 1) return -1;
    if (src->beam_kind == 1 && !(src->field[2] >= 0.0 && src->field[3] >= 0.0)) return -1;
    return 0;
}

/* Samples the source particle from block 0 of the primary stream (u0..u3):
 * the field position from u0, u1 and a histogram energy from u2 (bin) and u3
 * (position in the bin).  Returns 1 if the particle enters the top face. */
static int sample_source(const orc_source* src, const geom* G, const double* cdf, stream* s,
                         double* e, double r[3], double d[3])
{
    double u0 = uni(s), u1 = uni(s), u2 = uni(s), u3 = uni(s);
    if (src->energy_kind == 0) {
        *e = src->e0;
    } else {
        int b = 0;
        while (b < src->n_bins - 1 && !(cdf[b] > u2)) ++b;
        *e = src->edges[b] + u3 * (src->edges[b + 1] - src->edges[b]);
    }
    if (src->beam_kind == 0) {
        r[0] = src->pos[0];
        r[1] = src->pos[1];
        d[0] = 0.0; d[1] = 0.0; d[2] = 1.0;
    } else {
        r[0] = src->field[0] - src->field[2] + 2.0 * src->field[2] * u0;
        r[1] = src->field[1] - src->field[3] + 2.0 * src->field[3] * u1;
        double dx = r[0] - src->pos[0], dy = r[1] - src->pos[1], dz = G->g.z0 - src->pos[2];
        double n = sqrt(dx * dx + dy * dy + dz * dz);
        d[0] = dx / n; d[1] = dy / n; d[2] = dz / n;
    }
    r[2] = G->g.z0;
    return r[0] >= G->g.x0 && r[0] < G->xmax && r[1] >= G->g.y0 && r[1] < G->ymax && d[2] > 0.0;
}

static void build_cdf(const orc_source* src, double* cdf)
{
    double tot = 0.0;
    for (int b = 0; b < src->n_bins; ++b) tot += src->weights[b];
    double acc = 0.0;
    for (int b = 0; b < src->n_bins; ++b) {
        acc += src->weights[b];
        cdf[b] = acc / tot;
    }
}

/* ---------------------------------------------------------------- simulate */

int orc_simulate(const void* blob, size_t nbytes, const orc_grid* g, const uint8_t* mat,
                 const float* rho, const orc_source* src, uint64_t first, uint64_t n,
                 uint32_t seed, uint32_t request_key, double* S, double* Q, double* bal,
                 uint64_t* cnt, orc_history* hist, double* Sb)
{
    tables t;
    if (load_tables(blob, nbytes, &t)) return -1;
    if (check_phantom(&t, g, mat, rho) || check_source(src) || !S || !Q || !bal || !cnt ||
        first + n > 0x100000000ull || first + n < first) {
        free(t.q);
        return -1;
    }
    geom G;
    make_geom(&G, g, mat, rho);
    size_t nv = (size_t)g->nx * g->ny * g->nz;
    double mu_max[NE];
    build_majorant(&t, &G, mu_max);
    double cdf[64];
    if (src->energy_kind == 1) build_cdf(src, cdf);

    ctx c;
    memset(&c, 0, sizeof c);
    c.t = &t;
    c.G = &G;
    c.mu_max = mu_max;
    for (int m = 0; m < t.n_mat; ++m) {
        c.r_abs[m] = interp(&t, tab(&t, m, Q_R), t.e_abs_e);
        c.r_abs_pos[m] = interp(&t, tab(&t, m, Q_RP), t.e_abs_e);
    }
    c.k0 = seed;
    c.k1 = request_key;
    c.S = S;
    c.Q = Q;
    c.Sb = Sb;
    c.nv = nv;
    c.bal = bal;
    c.cnt = cnt;
    c.temp = (double*)calloc(nv, sizeof(double));
    c.touched = (unsigned char*)calloc(nv, 1);
    if (!c.temp || !c.touched) {
        free(c.temp); free(c.touched); free(t.q);
        return -1;
    }
    double extra = src->particle == POSITRON ? 2.0 * MC2 : 0.0;

    for (uint64_t i = 0; i < n; ++i) {
        uint32_t h = (uint32_t)(first + i);
        c.h = h;
        c.hist = hist ? &hist[i] : NULL;
        if (c.hist) memset(c.hist, 0, sizeof *c.hist);
        cnt[ORC_C_HISTORIES]++;
        stream s;
        stream_init(&s, seed, request_key, h, 0, cnt);
        double e, r[3], d[3];
        int enters = sample_source(src, &G, cdf, &s, &e, r, d);
        bal[ORC_E_SRC] += e + extra;
        if (!enters) {
            bal[ORC_E_MISS] += e + extra;
            cnt[ORC_C_MISSES]++;
            continue;
        }
        s.draw = 4;                         /* transport starts at block 1 */
        double cut = src->particle == PHOTON ? t.e_abs_g : t.e_abs_e;
        if (e <= cut) {
            int idx[3];
            floor_voxel(&G, r[0], r[1], r[2], idx);
            size_t v = lin_voxel(&G, idx);
            cnt[ORC_C_LOCAL]++;
            deposit(&c, v, e, ORC_E_LOCAL);
            if (src->particle == POSITRON) annihilate(&c, &s, r, v);
        } else {
            transport(&c, &s, src->particle, e, r, d);
        }
        while (c.sp > 0) {
            particle p = c.stack[--c.sp];
            stream s2;
            stream_init(&s2, seed, request_key, h, p.lineage, cnt);
            transport(&c, &s2, p.type, p.e, p.r, p.d);
        }
        flush_history(&c);
        if (c.oom) break;
    }
    int rc = c.oom ? -2 : 0;
    free(c.temp);
    free(c.touched);
    free(c.list);
    free(c.stack);
    free(t.q);
    return rc;
}

int orc_first_interaction(const void* blob, size_t nbytes, const orc_grid* g,
                          const uint8_t* mat, const float* rho, const orc_source* src,
                          uint64_t n, uint32_t seed, uint32_t request_key, double* z_out,
                          int32_t* kind_out)
{
    tables t;
    if (load_tables(blob, nbytes, &t)) return -1;
    if (check_phantom(&t, g, mat, rho) || check_source(src) || src->particle != PHOTON ||
        n > 0x100000000ull || !z_out) {
        free(t.q);
        return -1;
    }
    geom G;
    make_geom(&G, g, mat, rho);
    double mu_max[NE];
    build_majorant(&t, &G, mu_max);
    double cdf[64];
    if (src->energy_kind == 1) build_cdf(src, cdf);
    uint64_t cnt[ORC_NCOUNT] = {0};
    ctx c;
    memset(&c, 0, sizeof c);
    c.t = &t;
    c.G = &G;
    c.mu_max = mu_max;
    c.cnt = cnt;
    for (uint64_t i = 0; i < n; ++i) {
        stream s;
        stream_init(&s, seed, request_key, (uint32_t)i, 0, NULL);
        double e, r[3], d[3];
        if (!sample_source(src, &G, cdf, &s, &e, r, d)) {
            z_out[i] = NAN;
            if (kind_out) kind_out[i] = 0;
            continue;
        }
        s.draw = 4;
        int idx[3], ev;
        do ev = photon_flight(&c, &s, e, r, d, idx);
        while (ev == EV_VIRTUAL || ev == EV_PAIR_VOID);
        z_out[i] = ev == EV_G_ESCAPE ? INFINITY : r[2];
        if (kind_out) kind_out[i] = ev;
    }
    free(t.q);
    return 0;
}

/* A fixed oblique unit direction for the kinematics checks. */
static void check_direction(double d[3])
{
    d[0] = 0.3; d[1] = -0.5; d[2] = 0.8;
    double n = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    d[0] /= n; d[1] /= n; d[2] /= n;
}

int orc_sample(const void* blob, size_t nbytes, int which, double e, uint64_t n, uint32_t seed,
               double* out)
{
    tables t;
    if (load_tables(blob, nbytes, &t)) return -1;
    int ok = (which >= 0 && which < 6 + t.n_mat) || (which >= 256 && which < 256 + t.n_mat) ||
             which == 512;
    if (!ok || !(e > 0.0) || !out) { free(t.q); return -1; }
    if (which == 1 && !(e > 2.0 * t.w_cc)) { free(t.q); return -1; }
    if (which == 2 && !(e > t.w_cr)) { free(t.q); return -1; }
    for (uint64_t i = 0; i < n; ++i) {
        double* o = out + 8 * i;
        for (int k = 0; k < 8; ++k) o[k] = 0.0;
        stream s;
        stream_init(&s, seed, 0, (uint32_t)i, 0, NULL);
        double d[3], dd[3];
        check_direction(d);
        check_direction(dd);
        if (which == 0) {
            /* same draws and kinematics as a Compton event in transport */
            double cost, tau;
            sample_compton(&s, e, &cost, &tau, NULL);
            double phi = 2.0 * PI * uni(&s);
            double e1 = tau * e, te = e - e1;
            double pe = sqrt(e * e + e1 * e1 - 2.0 * e * e1 * cost);
            double cose = pe > 0.0 ? (e - e1 * cost) / pe : 1.0;
            if (cose > 1.0) cose = 1.0;
            if (cose < -1.0) cose = -1.0;
            rotate(dd, cose, phi + PI);
            rotate(d, cost, phi);
            o[0] = cost; o[1] = tau;
            o[2] = d[0]; o[3] = d[1]; o[4] = d[2];
            o[5] = dd[0]; o[6] = dd[1]; o[7] = dd[2];
            (void)te;
        } else if (which == 1) {
            double eps = sample_moller(&s, e, t.w_cc, NULL);
            double phi = 2.0 * PI * uni(&s);
            double w = eps * e;
            double cs = sqrt(w * (e + 2.0 * MC2) / (e * (w + 2.0 * MC2)));
            double cp = sqrt((e - w) * (e + 2.0 * MC2) / (e * (e - w + 2.0 * MC2)));
            rotate(dd, cs, phi + PI);
            rotate(d, cp, phi);
            o[0] = eps; o[1] = cs;
            o[2] = d[0]; o[3] = d[1]; o[4] = d[2];
            o[5] = dd[0]; o[6] = dd[1]; o[7] = dd[2];
        } else if (which == 2) {
            o[0] = sample_brems(&s, e, t.w_cr);
        } else if (which == 4) {
            o[0] = sample_sauter_cos(&s, e);
        } else if (which == 5) {
            o[0] = sample_forward_cos(&s, e);
        } else if (which == 512) {
            o[0] = e > t.w_cc ? sample_bhabha(&s, e, t.w_cc, NULL) : 0.0;
        } else if (which >= 256) {
            int m = which - 256;
            double r = interp(&t, tab(&t, m, Q_L2INV), e) / interp(&t, tab(&t, m, Q_L1INV), e);
            o[0] = sample_hinge2_cos(&s, t.kappa_step, t.a_hinge, r);
            o[1] = r;
        } else if (which >= 6) {
            o[0] = sample_rayleigh_cos(&s, t.ray_b[which - 6] * e * e);
        } else {
            double cost = sample_hinge_cos(&s, t.a_hinge);
            double phi = 2.0 * PI * uni(&s);
            rotate(d, cost, phi);
            o[0] = cost;
            o[2] = d[0]; o[3] = d[1]; o[4] = d[2];
        }
    }
    free(t.q);
    return 0;
}

/* ---------------------------------------------------------------- finalize */

/* Dmax and sigma-bar are taken over tissue voxels only: density at least
 * 0.05 g/cm^3 (lung and denser).  The paper's phantoms hold no air; in a
 * CT-like phantom an air voxel's dose comes from a few deposits in a tiny
 * mass, so it would set Dmax and dominate sigma-bar with noise. */
#define ORC_TISSUE_RHO_MIN 0.05f

int orc_finalize(const orc_grid* g, const float* rho, const double* S, const double* Q,
                 uint64_t n, double* dose, double* sigma, double* dmax, double* sigma_bar)
{
    if (!g || !rho || !S || !Q || !dose || !sigma || n < 2) return -1;
    size_t nv = (size_t)g->nx * g->ny * g->nz;
    double vol = g->dx * g->dy * g->dz;
    double N = (double)n;
    double mx = 0.0;
    for (size_t v = 0; v < nv; ++v) {
        double scale = MEV_PER_G_TO_GY / ((double)rho[v] * vol);
        double mean = S[v] / N;
        double var = (Q[v] / N - mean * mean) / (N - 1.0);
        dose[v] = mean * scale;
        sigma[v] = sqrt(var > 0.0 ? var : 0.0) * scale;
        if (rho[v] >= ORC_TISSUE_RHO_MIN && dose[v] > mx) mx = dose[v];
    }
    double acc = 0.0;
    size_t cntv = 0;
    for (size_t v = 0; v < nv; ++v) {
        if (rho[v] >= ORC_TISSUE_RHO_MIN && dose[v] > 0.5 * mx) {
            acc += sigma[v] / dose[v];
            ++cntv;
        }
    }
    if (dmax) *dmax = mx;
    if (sigma_bar) *sigma_bar = cntv ? acc / (double)cntv : 0.0;
    return 0;
}

/* Group ("batch") statistics: the histories are split into 16 groups by
 * history mod 16 with nb[b] histories and group tallies Sb[b][v].  The dose
 * comes from S = sum_b Sb; the per-history variance is estimated from the
 * spread of the group means m_b = Sb/nb[b] around m = S/N,
 *     s^2 = sum_b nb[b] (m_b - m)^2 / (B' - 1),  sigma_mean^2 = s^2 / N,
 * with B' the number of non-empty groups.  s^2 is unbiased for any group
 * sizes, but its square root reads low: for normal group means
 * sum_b nb[b] (m_b - m)^2 / sigma^2 is chi-square with B' - 1 degrees of
 * freedom, so E[s] = c4(B') sigma with
 *     c4(k) = sqrt(2 / (k - 1)) Gamma(k / 2) / Gamma((k - 1) / 2)
 * (0.9835 for 16 groups).  The standard deviation sigma_D of Sec. 3 is
 * estimated as sigma_mean / c4(B'), so that the mean relative uncertainty
 * does not come out about 1.7% low. */
static double c4_factor(int k)
{
    if (k < 2) return 1.0;
    return sqrt(2.0 / (double)(k - 1)) * exp(lgamma(0.5 * k) - lgamma(0.5 * (k - 1)));
}

int orc_finalize_groups(const orc_grid* g, const float* rho, const double* Sb, const double* nb,
                        double* dose, double* sigma, double* dmax, double* sigma_bar)
{
    if (!g || !rho || !Sb || !nb || !dose || !sigma) return -1;
    size_t nv = (size_t)g->nx * g->ny * g->nz;
    double vol = g->dx * g->dy * g->dz;
    double N = 0.0;
    int groups = 0;
    for (int b = 0; b < 16; ++b) {
        N += nb[b];
        if (nb[b] > 0.0) ++groups;
    }
    if (!(N > 0.0)) return -1;
    double c4 = c4_factor(groups);
    double mx = 0.0;
    for (size_t v = 0; v < nv; ++v) {
        double S = 0.0;
        for (int b = 0; b < 16; ++b) S += Sb[(size_t)b * nv + v];
        double m = S / N;
        double ss = 0.0;
        for (int b = 0; b < 16; ++b) {
            if (nb[b] <= 0.0) continue;
            double dm = Sb[(size_t)b * nv + v] / nb[b] - m;
            ss += nb[b] * dm * dm;
        }
        double var = groups > 1 ? ss / (groups - 1) / N : 0.0;
        double scale = MEV_PER_G_TO_GY / ((double)rho[v] * vol);
        dose[v] = m * scale;
        sigma[v] = sqrt(var) / c4 * scale;
        if (rho[v] >= ORC_TISSUE_RHO_MIN && dose[v] > mx) mx = dose[v];
    }
    double acc = 0.0;
    size_t cntv = 0;
    for (size_t v = 0; v < nv; ++v)
        if (rho[v] >= ORC_TISSUE_RHO_MIN && dose[v] > 0.5 * mx) {
            acc += sigma[v] / dose[v];
            ++cntv;
        }
    if (dmax) *dmax = mx;
    if (sigma_bar) *sigma_bar = cntv ? acc / (double)cntv : 0.0;
    return 0;
}
