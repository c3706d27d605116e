// Host runtime of libmcdose: contexts, table and phantom residency, the
// blocking simulate call, and argument validation.  Implements include/mcdose.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "engine.h"
#include "mcdose.h"
#include "runtime.h"

using namespace mcd;

// ------------------------------------------------------------------ helpers

const char* mcd_status_string(int status)
{
    switch (status) {
    case MCD_OK: return "ok";
    case MCD_E_INVAL: return "invalid argument";
    case MCD_E_NOMEM: return "out of device memory or over the HBM budget";
    case MCD_E_NOTFOUND: return "unknown handle";
    case MCD_E_OVERFLOW: return "particle stack or local counter overflow";
    case MCD_E_DEVICE: return "HIP device error";
    case MCD_E_BUSY: return "request not finished";
    case MCD_E_CANCELED: return "request cancelled";
    default: return "unknown status";
    }
}

const char* mcd_last_error(mcd_ctx* ctx)
{
    if (!ctx) return "null context";
    return ctx->last_error.c_str();
}

int mcd_ctx::fail(int status, const std::string& msg)
{
    last_error = msg;
    return status;
}

int mcd_ctx::hip_fail(hipError_t e, const char* what)
{
    last_error = std::string(what) + ": " + hipGetErrorString(e);
    return MCD_E_DEVICE;
}

int mcd_ctx::alloc(void** p, size_t bytes, const char* what)
{
    *p = nullptr;
    if (bytes == 0) return MCD_OK;
    if (used + bytes > budget)
        return fail(MCD_E_NOMEM, std::string(what) + ": allocation of " + std::to_string(bytes) +
                                     " bytes exceeds the HBM budget");
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(MCD_E_NOMEM, std::string(what) + ": hipMalloc failed: " + hipGetErrorString(e));
    }
    used += bytes;
    return MCD_OK;
}

void mcd_ctx::release(void* p, size_t bytes)
{
    if (!p) return;
    (void)hipFree(p);
    used -= std::min(used, (uint64_t)bytes);
}

// ------------------------------------------------------------- create/destroy

int mcd_create(int device, uint64_t hbm_budget_bytes, mcd_ctx** out)
{
    if (!out) return MCD_E_INVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return MCD_E_INVAL;
    if (hipSetDevice(device) != hipSuccess) return MCD_E_DEVICE;
    mcd_ctx* c = new (std::nothrow) mcd_ctx();
    if (!c) return MCD_E_NOMEM;
    c->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete c;
        return MCD_E_DEVICE;
    }
    c->cu_count = prop.multiProcessorCount;
    c->max_lds = (int)prop.sharedMemPerBlock;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        delete c;
        return MCD_E_DEVICE;
    }
    c->budget = hbm_budget_bytes ? hbm_budget_bytes : (uint64_t)(0.9 * (double)free_b);
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return MCD_E_DEVICE;
    }
    if (c->alloc((void**)&c->small, kSmallBytes, "run scalars")) {
        (void)hipStreamDestroy(c->stream);
        delete c;
        return MCD_E_NOMEM;
    }
    for (auto& e : c->ev) (void)hipEventCreate(&e);
    *out = c;
    return MCD_OK;
}

int mcd_destroy(mcd_ctx* c)
{
    if (!c) return MCD_E_INVAL;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    c->shutdown_serving();
    for (auto& t : c->tables)
        if (t.live) {
            c->release(t.dev.phot, t.bytes / 2);
            c->release(t.dev.elec, t.bytes / 2);
        }
    for (auto& p : c->phantoms)
        if (p.live) {
            c->release(p.vox, p.nv * sizeof(uint2));
            c->release(p.maj, kNE * sizeof(float));
        }
    c->release(c->scratch, c->scratch_bytes);
    c->release(c->S, c->tally_cap * sizeof(double));
    c->release(c->Q, c->tally_cap * sizeof(double));
    c->release(c->dose, c->stage_cap * sizeof(double));
    c->release(c->sigma, c->stage_cap * sizeof(double));
    c->release(c->small, kSmallBytes);
    for (auto& e : c->ev) (void)hipEventDestroy(e);
    (void)hipStreamDestroy(c->stream);
    delete c;
    return MCD_OK;
}

// ------------------------------------------------------------------ tables

namespace {

constexpr size_t kHdr = 8 + 4 * 4 + 9 * 8 + 2 * 4;
constexpr size_t kMatHdr = 16 + 6 * 8;
constexpr int kNQ = 8;

template <class T> T rd(const unsigned char* p)
{
    T v;
    std::memcpy(&v, p, sizeof v);
    return v;
}

// Interpolant of a node array, linear in ln E (FP64, host side).
double host_interp(const double* f, double e, double emin, double emax)
{
    e = std::min(std::max(e, emin), emax);
    const double x = std::log(e / emin) / (std::log(emax / emin) / (kNE - 1));
    int i = std::min(std::max((int)std::floor(x), 0), kNE - 2);
    const double fr = x - i;
    return f[i] + (f[i + 1] - f[i]) * fr;
}

}  // namespace

int mcd_load_materials(mcd_ctx* c, const void* blob, size_t nbytes, int32_t* out_tables)
{
    if (!c || !blob || !out_tables) return MCD_E_INVAL;
    const unsigned char* b = (const unsigned char*)blob;
    if (nbytes < kHdr || std::memcmp(b, "MCDTAB\0\1", 8) != 0)
        return c->fail(MCD_E_INVAL, "table blob: bad magic or size");
    const uint32_t ver = rd<uint32_t>(b + 8), n_mat = rd<uint32_t>(b + 12);
    const uint32_t n_e = rd<uint32_t>(b + 16), n_q = rd<uint32_t>(b + 20);
    if (ver != 1 || n_e != (uint32_t)kNE || n_q != (uint32_t)kNQ)
        return c->fail(MCD_E_INVAL, "table blob: unsupported version or grid");
    if (n_mat < 1 || n_mat > (uint32_t)kMaxMat)
        return c->fail(MCD_E_INVAL, "table blob: 1 to 8 materials supported");
    const size_t mat_bytes = kMatHdr + (size_t)kNQ * kNE * 8;
    if (nbytes != kHdr + n_mat * mat_bytes) return c->fail(MCD_E_INVAL, "table blob: size mismatch");
    const unsigned char* s = b + 24;
    TableSet ts;
    ts.n_mat = (int)n_mat;
    ts.emin = rd<double>(s);
    ts.emax = rd<double>(s + 8);
    ts.e_abs_e = rd<double>(s + 16);
    ts.e_abs_g = rd<double>(s + 24);
    ts.w_cc = rd<double>(s + 32);
    ts.w_cr = rd<double>(s + 40);
    ts.kappa_step = rd<double>(s + 48);
    ts.f_e = rd<double>(s + 56);
    ts.a_hinge = rd<double>(s + 64);
    if (!(ts.emin > 0 && ts.emax > ts.emin && ts.e_abs_e > ts.emin && ts.e_abs_e < ts.emax &&
          ts.e_abs_g > ts.emin && ts.e_abs_g < ts.emax && ts.w_cc > 0 && ts.w_cr > 0 &&
          ts.kappa_step > 0 && ts.f_e > 0 && ts.f_e < 1 && ts.a_hinge > 0))
        return c->fail(MCD_E_INVAL, "table blob: scalar parameters out of range");
    ts.q.resize((size_t)n_mat * kNQ * kNE);
    for (uint32_t m = 0; m < n_mat; ++m)
        std::memcpy(&ts.q[(size_t)m * kNQ * kNE], b + kHdr + m * mat_bytes + kMatHdr,
                    (size_t)kNQ * kNE * 8);
    for (double v : ts.q)
        if (!(v >= 0.0) || !std::isfinite(v))
            return c->fail(MCD_E_INVAL, "table blob: negative or non-finite value");
    for (uint32_t m = 0; m < n_mat; ++m) {
        const double* r = ts.range(m);
        for (int i = 1; i < kNE; ++i)
            if (!(r[i] > r[i - 1])) return c->fail(MCD_E_INVAL, "table blob: range not increasing");
    }
    // FP32 device layout: float4 per node for the photon and electron groups
    std::vector<float4> ph((size_t)n_mat * kNE), el((size_t)n_mat * kNE);
    for (uint32_t m = 0; m < n_mat; ++m)
        for (int i = 0; i < kNE; ++i) {
            const double* q = &ts.q[(size_t)m * kNQ * kNE];
            ph[m * kNE + i] = make_float4((float)q[0 * kNE + i], (float)q[1 * kNE + i],
                                          (float)q[2 * kNE + i], 0.f);
            el[m * kNE + i] = make_float4((float)q[3 * kNE + i], (float)q[4 * kNE + i],
                                          (float)q[5 * kNE + i], (float)q[6 * kNE + i]);
        }
    (void)hipSetDevice(c->device);
    ts.bytes = 2 * ph.size() * sizeof(float4);
    int rc = c->alloc((void**)&ts.dev.phot, ts.bytes / 2, "tables");
    if (rc) return rc;
    rc = c->alloc((void**)&ts.dev.elec, ts.bytes / 2, "tables");
    if (rc) {
        c->release(ts.dev.phot, ts.bytes / 2);
        return rc;
    }
    hipError_t e = hipMemcpy(ts.dev.phot, ph.data(), ts.bytes / 2, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ts.dev.elec, el.data(), ts.bytes / 2, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        c->release(ts.dev.phot, ts.bytes / 2);
        c->release(ts.dev.elec, ts.bytes / 2);
        return c->hip_fail(e, "table upload");
    }
    DevTables& d = ts.dev;
    d.n_mat = (int)n_mat;
    for (int m = 0; m < kMaxMat; ++m)
        d.r_abs[m] = m < (int)n_mat ? (float)host_interp(ts.range(m), ts.e_abs_e, ts.emin, ts.emax) : 0.f;
    d.l2_emin = (float)std::log2(ts.emin);
    d.dl2 = (float)(std::log2(ts.emax / ts.emin) / (kNE - 1));
    d.inv_dl2 = (float)((kNE - 1) / std::log2(ts.emax / ts.emin));
    d.emin = (float)ts.emin;
    d.emax = (float)ts.emax;
    d.e_abs_e = (float)ts.e_abs_e;
    d.e_abs_g = (float)ts.e_abs_g;
    d.w_cc = (float)ts.w_cc;
    d.w_cr = (float)ts.w_cr;
    d.kappa_step = (float)ts.kappa_step;
    d.f_e = (float)ts.f_e;
    d.a_hinge = (float)ts.a_hinge;
    ts.live = true;
    std::lock_guard<std::mutex> g(c->mu);
    c->tables.push_back(std::move(ts));
    *out_tables = (int32_t)c->tables.size() - 1;
    return MCD_OK;
}

int mcd_unload_materials(mcd_ctx* c, int32_t t)
{
    if (!c) return MCD_E_INVAL;
    std::lock_guard<std::mutex> g(c->mu);
    if (t < 0 || t >= (int32_t)c->tables.size() || !c->tables[t].live) return MCD_E_NOTFOUND;
    for (auto& p : c->phantoms)
        if (p.live && p.tables == t) return c->fail(MCD_E_INVAL, "tables still used by a phantom");
    TableSet& ts = c->tables[t];
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    c->release(ts.dev.phot, ts.bytes / 2);
    c->release(ts.dev.elec, ts.bytes / 2);
    ts.live = false;
    ts.q.clear();
    return MCD_OK;
}

// ----------------------------------------------------------------- phantoms

int mcd_load_phantom(mcd_ctx* c, const mcd_grid* g, const uint8_t* mat, const float* rho,
                     int32_t tables, int32_t* out_phantom)
{
    if (!c || !g || !mat || !rho || !out_phantom) return MCD_E_INVAL;
    if (tables < 0 || tables >= (int32_t)c->tables.size() || !c->tables[tables].live)
        return c->fail(MCD_E_NOTFOUND, "unknown table handle");
    if (g->nx < 1 || g->ny < 1 || g->nz < 1 || !(g->dx > 0) || !(g->dy > 0) || !(g->dz > 0) ||
        !std::isfinite(g->x0) || !std::isfinite(g->y0) || !std::isfinite(g->z0))
        return c->fail(MCD_E_INVAL, "grid: sizes must be positive and the corner finite");
    const int64_t nv = (int64_t)g->nx * g->ny * g->nz;
    if (nv >= (int64_t)1 << 31) return c->fail(MCD_E_INVAL, "grid: at most 2^31 - 1 voxels");
    const TableSet& ts = c->tables[tables];
    std::vector<uint2> vox((size_t)nv);
    double rmax[kMaxMat] = {0};
    for (int64_t v = 0; v < nv; ++v) {
        if (mat[v] >= ts.n_mat || !(rho[v] > 0.f) || !std::isfinite(rho[v]))
            return c->fail(MCD_E_INVAL, "phantom: material index out of range or density <= 0 at voxel " +
                                            std::to_string(v));
        uint32_t bits;
        std::memcpy(&bits, &rho[v], 4);
        vox[v] = make_uint2(bits, mat[v]);
        rmax[mat[v]] = std::max(rmax[mat[v]], (double)rho[v]);
    }
    // Woodcock majorant at the nodes: max over present materials of
    // rho_max * (mu_C + mu_pe + mu_pp) per gram, rounded up to FP32.
    std::vector<float> maj(kNE);
    for (int i = 0; i < kNE; ++i) {
        double best = 0.0;
        for (int m = 0; m < ts.n_mat; ++m) {
            if (rmax[m] <= 0.0) continue;
            const double* q = &ts.q[(size_t)m * kNQ * kNE];
            best = std::max(best, rmax[m] * (q[i] + q[kNE + i] + q[2 * kNE + i]));
        }
        float f = (float)best;
        if ((double)f < best) f = std::nextafter(f, INFINITY);
        maj[i] = f;
    }
    PhantomRec p;
    p.g = *g;
    p.tables = tables;
    p.nv = nv;
    (void)hipSetDevice(c->device);
    int rc = c->alloc((void**)&p.vox, (size_t)nv * sizeof(uint2), "phantom");
    if (rc) return rc;
    rc = c->alloc((void**)&p.maj, kNE * sizeof(float), "majorant");
    if (rc) {
        c->release(p.vox, (size_t)nv * sizeof(uint2));
        return rc;
    }
    hipError_t e = hipMemcpy(p.vox, vox.data(), (size_t)nv * sizeof(uint2), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p.maj, maj.data(), kNE * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        c->release(p.vox, (size_t)nv * sizeof(uint2));
        c->release(p.maj, kNE * sizeof(float));
        return c->hip_fail(e, "phantom upload");
    }
    p.live = true;
    std::lock_guard<std::mutex> lk(c->mu);
    c->phantoms.push_back(p);
    *out_phantom = (int32_t)c->phantoms.size() - 1;
    return MCD_OK;
}

int mcd_unload_phantom(mcd_ctx* c, int32_t ph)
{
    if (!c) return MCD_E_INVAL;
    std::lock_guard<std::mutex> g(c->mu);
    if (ph < 0 || ph >= (int32_t)c->phantoms.size() || !c->phantoms[ph].live) return MCD_E_NOTFOUND;
    PhantomRec& p = c->phantoms[ph];
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    c->release(p.vox, (size_t)p.nv * sizeof(uint2));
    c->release(p.maj, kNE * sizeof(float));
    p.live = false;
    return MCD_OK;
}

// ---------------------------------------------------------------- simulate

int mcd_ctx::validate_source(const mcd_source* s, DevSource* d)
{
    if (!s) return fail(MCD_E_INVAL, "source: null");
    if (s->particle < MCD_PHOTON || s->particle > MCD_POSITRON)
        return fail(MCD_E_INVAL, "source: particle must be 0, 1 or 2");
    if (s->beam_kind != MCD_PENCIL && s->beam_kind != MCD_POINT_FIELD)
        return fail(MCD_E_INVAL, "source: unknown beam kind");
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(s->pos[i])) return fail(MCD_E_INVAL, "source: position not finite");
    if (s->beam_kind == MCD_POINT_FIELD &&
        !(s->field[2] >= 0 && s->field[3] >= 0 && std::isfinite(s->field[0]) && std::isfinite(s->field[1])))
        return fail(MCD_E_INVAL, "source: bad field rectangle");
    std::memset(d, 0, sizeof *d);
    d->particle = s->particle;
    d->energy_kind = s->energy_kind;
    d->beam_kind = s->beam_kind;
    for (int i = 0; i < 3; ++i) d->pos[i] = (float)s->pos[i];
    for (int i = 0; i < 4; ++i) d->field[i] = (float)s->field[i];
    d->extra = s->particle == MCD_POSITRON ? 2.0 * (double)0.51099895f : 0.0;
    if (s->energy_kind == MCD_MONO) {
        if (!(s->e0 > 0.0) || s->e0 > 20.0) return fail(MCD_E_INVAL, "source: energy must be in (0, 20] MeV");
        d->e0 = (float)s->e0;
        d->n_bins = 1;
    } else if (s->energy_kind == MCD_HISTOGRAM) {
        const int nb = s->n_bins;
        if (nb < 1 || nb > MCD_MAX_BINS) return fail(MCD_E_INVAL, "source: 1 to 64 bins");
        double tot = 0.0;
        for (int b = 0; b < nb; ++b) {
            if (!(s->weights[b] >= 0.0) || !(s->edges[b + 1] > s->edges[b]))
                return fail(MCD_E_INVAL, "source: bad histogram");
            tot += s->weights[b];
        }
        if (!(tot > 0.0) || !(s->edges[0] > 0.0) || s->edges[nb] > 20.0)
            return fail(MCD_E_INVAL, "source: histogram energies must be in (0, 20] MeV");
        double acc = 0.0;
        for (int b = 0; b < nb; ++b) {
            acc += s->weights[b];
            d->cdf[b] = (float)(acc / tot);
        }
        for (int b = 0; b <= nb; ++b) d->edges[b] = (float)s->edges[b];
        d->n_bins = nb;
    } else {
        return fail(MCD_E_INVAL, "source: unknown energy kind");
    }
    return MCD_OK;
}

int mcd_ctx::ensure_scratch(size_t lanes, int depth, int slots, hipStream_t s)
{
    const size_t lb = lane_scratch_bytes(depth, slots);
    if (scratch && lanes <= scratch_lanes && lb == lane_bytes && depth == stack_depth &&
        slots == slot_count && keys_clean)
        return MCD_OK;
    if (!scratch || lanes * lb > scratch_bytes) {
        if (scratch) {
            (void)hipStreamSynchronize(s);
            release(scratch, scratch_bytes);
            scratch = nullptr;
        }
        int rc = alloc((void**)&scratch, lanes * lb, "lane scratch");
        if (rc) {
            scratch_bytes = 0;
            return rc;
        }
        scratch_bytes = lanes * lb;
    }
    scratch_lanes = scratch_bytes / lb;
    lane_bytes = lb;
    stack_depth = depth;
    slot_count = slots;
    hipError_t e = launch_clear_lane_keys(scratch, scratch_lanes, lane_bytes, depth, slots, s);
    if (e != hipSuccess) return hip_fail(e, "clear lane scratch");
    keys_clean = true;
    return MCD_OK;
}

int mcd_ctx::ensure_tallies(int64_t nv, hipStream_t s)
{
    if (nv <= tally_cap) return MCD_OK;
    (void)hipStreamSynchronize(s);
    release(S, tally_cap * sizeof(double));
    release(Q, tally_cap * sizeof(double));
    S = Q = nullptr;
    tally_cap = 0;
    int rc = alloc((void**)&S, nv * sizeof(double), "tallies");
    if (rc) return rc;
    rc = alloc((void**)&Q, nv * sizeof(double), "tallies");
    if (rc) {
        release(S, nv * sizeof(double));
        S = nullptr;
        return rc;
    }
    tally_cap = nv;
    return MCD_OK;
}

int mcd_ctx::ensure_stage(int64_t nv, hipStream_t s)
{
    if (nv <= stage_cap) return MCD_OK;
    (void)hipStreamSynchronize(s);
    release(dose, stage_cap * sizeof(double));
    release(sigma, stage_cap * sizeof(double));
    dose = sigma = nullptr;
    stage_cap = 0;
    int rc = alloc((void**)&dose, nv * sizeof(double), "dose staging");
    if (rc) return rc;
    rc = alloc((void**)&sigma, nv * sizeof(double), "dose staging");
    if (rc) {
        release(dose, nv * sizeof(double));
        dose = nullptr;
        return rc;
    }
    stage_cap = nv;
    return MCD_OK;
}

void mcd_ctx::fill_params(KParams& p, const PhantomRec& ph, const DevSource& ds, uint64_t seed,
                          uint32_t key, uint64_t first, uint64_t n)
{
    std::memset(&p, 0, sizeof p);
    p.t = tables[ph.tables].dev;
    p.maj = ph.maj;
    p.vox = ph.vox;
    p.nx = ph.g.nx;
    p.ny = ph.g.ny;
    p.nz = ph.g.nz;
    p.dx = (float)ph.g.dx;
    p.dy = (float)ph.g.dy;
    p.dz = (float)ph.g.dz;
    p.x0 = (float)ph.g.x0;
    p.y0 = (float)ph.g.y0;
    p.z0 = (float)ph.g.z0;
    p.x1 = (float)(ph.g.x0 + ph.g.nx * ph.g.dx);
    p.y1 = (float)(ph.g.y0 + ph.g.ny * ph.g.dy);
    p.z1 = (float)(ph.g.z0 + ph.g.nz * ph.g.dz);
    p.idx = (float)(1.0 / ph.g.dx);
    p.idy = (float)(1.0 / ph.g.dy);
    p.idz = (float)(1.0 / ph.g.dz);
    p.src = ds;
    p.seed = (uint32_t)seed;
    p.key = key;
    p.first = (uint32_t)first;
    p.n = (uint32_t)n;
}

int mcd_ctx::launch_shape(const mcd_opts* o, int n_mat, int* blocks, int* threads)
{
    int t = o && o->block_size ? o->block_size : kDefaultBlock;
    if (t < 64 || t > 512 || (t & 63)) return fail(MCD_E_INVAL, "opts: block_size must be a multiple of 64 in [64, 512]");
    int b = o && o->grid_blocks ? o->grid_blocks : 0;
    if (b < 0) return fail(MCD_E_INVAL, "opts: grid_blocks must be >= 0");
    const int lds = transport_lds_bytes(n_mat);
    if (lds > max_lds)
        return fail(MCD_E_INVAL, "tables need " + std::to_string(lds) + " bytes of LDS per workgroup; the device allows " +
                                     std::to_string(max_lds));
    if (b == 0) {
        const int per_cu = std::max(1, std::min(kLdsPerCu / lds, 2048 / t));
        b = cu_count * per_cu;
    }
    *blocks = b;
    *threads = t;
    return MCD_OK;
}

int mcd_simulate(mcd_ctx* c, int32_t phantom, const mcd_source* src, uint64_t n_histories,
                 uint64_t seed, uint32_t request_key, const mcd_opts* opts, mcd_result* out,
                 void* hip_stream)
{
    if (!c || !out) return MCD_E_INVAL;
    std::lock_guard<std::mutex> run_lock(c->run_mu);
    if (phantom < 0 || phantom >= (int32_t)c->phantoms.size() || !c->phantoms[phantom].live)
        return c->fail(MCD_E_NOTFOUND, "unknown phantom handle");
    const PhantomRec& ph = c->phantoms[phantom];
    const uint64_t first = opts ? opts->first_history : 0;
    if (n_histories == 0 || n_histories >= ((uint64_t)1 << 32) || seed >= ((uint64_t)1 << 32) ||
        first >= ((uint64_t)1 << 32) || first + n_histories > ((uint64_t)1 << 32))
        return c->fail(MCD_E_INVAL, "need 1 <= n_histories < 2^32, seed < 2^32, first + n <= 2^32");
    if (n_histories < 2 && (out->dose || out->sigma))
        return c->fail(MCD_E_INVAL, "an uncertainty needs at least 2 histories");
    DevSource ds;
    int rc = c->validate_source(src, &ds);
    if (rc) return rc;
    const int depth = opts && opts->stack_depth ? opts->stack_depth : kDefaultDepth;
    const int slots = opts && opts->tally_slots ? opts->tally_slots : kDefaultSlots;
    if (depth < 4 || depth > 4096) return c->fail(MCD_E_INVAL, "opts: stack_depth in [4, 4096]");
    if (slots < 16 || slots > 32768 || (slots & (slots - 1)))
        return c->fail(MCD_E_INVAL, "opts: tally_slots must be a power of two in [16, 32768]");
    int blocks, threads;
    rc = c->launch_shape(opts, c->tables[ph.tables].n_mat, &blocks, &threads);
    if (rc) return rc;
    const bool diag = opts && opts->diagnostics;
    const bool accumulate = opts && opts->accumulate;
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : c->stream;
    (void)hipSetDevice(c->device);

    if ((rc = c->ensure_scratch((size_t)blocks * threads, depth, slots, s))) return rc;
    if ((rc = c->ensure_tallies(ph.nv, s))) return rc;
    const bool want_final = out->dose || out->sigma;
    if (want_final && (!out->on_device || !out->dose || !out->sigma))
        if ((rc = c->ensure_stage(ph.nv, s))) return rc;
    if (accumulate && c->tally_owner != phantom)
        return c->fail(MCD_E_INVAL, "opts.accumulate: the previous run used another phantom");

    KParams p;
    c->fill_params(p, ph, ds, seed, request_key, first, n_histories);
    p.S = c->S;
    p.Q = c->Q;
    p.bal = (double*)(c->small + kOffBal);
    p.cnt = (unsigned long long*)(c->small + kOffCnt);
    p.err = (int*)(c->small + kOffErr);
    p.next = (unsigned long long*)(c->small + kOffNext);
    p.scratch = c->scratch;
    p.stack_depth = depth;
    p.slots = slots;
    p.lane_bytes = c->lane_bytes;
    p.hist = diag && opts ? opts->history_records : nullptr;
    p.lockstep = opts && opts->lockstep ? 1 : 0;
    if (p.lockstep && (threads & 63)) return c->fail(MCD_E_INVAL, "lockstep needs whole waves");
    if (p.hist && !diag) return c->fail(MCD_E_INVAL, "history records need diagnostics");
    double* red = (double*)(c->small + kOffRed);

    hipError_t e = hipEventRecord(c->ev[0], s);
    if (e == hipSuccess && !accumulate) {
        e = launch_fill_u32(c->S, (size_t)ph.nv * 2, 0u, s);
        if (e == hipSuccess) e = launch_fill_u32(c->Q, (size_t)ph.nv * 2, 0u, s);
    }
    if (e == hipSuccess) e = launch_fill_u32(c->small, kSmallBytes / 4, 0u, s);
    if (e == hipSuccess) e = hipEventRecord(c->ev[1], s);
    if (e == hipSuccess) e = launch_transport(p, blocks, threads, diag, s);
    if (e == hipSuccess) e = hipEventRecord(c->ev[2], s);
    double* d_dose = nullptr;
    double* d_sigma = nullptr;
    if (e == hipSuccess && want_final) {
        d_dose = out->on_device && out->dose && out->sigma ? out->dose : c->dose;
        d_sigma = out->on_device && out->dose && out->sigma ? out->sigma : c->sigma;
        e = launch_finalize(c->S, c->Q, ph.vox, ph.nv, ph.g.dx * ph.g.dy * ph.g.dz,
                            n_histories + (accumulate ? c->tally_hist : 0), d_dose, d_sigma, red, s);
    }
    if (e == hipSuccess) e = hipEventRecord(c->ev[3], s);
    unsigned char host_small[kSmallBytes];
    if (e == hipSuccess) e = hipMemcpyAsync(host_small, c->small, kSmallBytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return c->hip_fail(e, "transport launch");
    int err;
    std::memcpy(&err, host_small + kOffErr, 4);
    if (err) {
        c->keys_clean = false;          // lanes stopped mid-history
        c->tally_owner = -1;
        return c->fail(err, err == MCD_E_OVERFLOW
                                ? "particle stack or local counter overflow: raise stack_depth or tally_slots"
                                : "device error");
    }
    c->tally_owner = phantom;
    c->tally_hist = n_histories + (accumulate ? c->tally_hist : 0);

    // outputs
    const size_t vb = (size_t)ph.nv * sizeof(double);
    const hipMemcpyKind k_out = out->on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (out->dose && d_dose != out->dose) e = hipMemcpyAsync(out->dose, d_dose, vb, k_out, s);
    if (e == hipSuccess && out->sigma && d_sigma != out->sigma)
        e = hipMemcpyAsync(out->sigma, d_sigma, vb, k_out, s);
    if (e == hipSuccess && out->S) e = hipMemcpyAsync(out->S, c->S, vb, k_out, s);
    if (e == hipSuccess && out->Q) e = hipMemcpyAsync(out->Q, c->Q, vb, k_out, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return c->hip_fail(e, "result copy");

    double bal[kBal];
    std::memcpy(bal, host_small + kOffBal, sizeof bal);
    out->eb.e_src = bal[0];
    out->eb.e_csda = bal[1];
    out->eb.e_local = bal[2];
    out->eb.e_esc = bal[3];
    out->eb.e_miss = bal[4];
    out->eb.track_e = bal[5];
    std::memcpy(out->counters, host_small + kOffCnt, sizeof out->counters);
    double r3[3];
    std::memcpy(r3, host_small + kOffRed, sizeof r3);
    out->dmax = want_final ? r3[0] : 0.0;
    out->sigma_bar = want_final && r3[2] > 0 ? r3[1] / r3[2] : 0.0;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, c->ev[1], c->ev[2]);
    out->kernel_ms = ms;
    (void)hipEventElapsedTime(&ms, c->ev[0], c->ev[3]);
    out->total_ms = ms;
    return MCD_OK;
}
