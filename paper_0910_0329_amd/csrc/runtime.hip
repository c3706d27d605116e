// Host runtime of libmcdose: contexts, table and phantom residency, the
// blocking simulate call, and argument validation.  Implements include/mcdose.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
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

// Error messages are kept per calling thread and context, so that the serving
// worker and the callers of a context do not overwrite each other's.
static std::string& error_slot(const mcd_ctx* c)
{
    thread_local std::map<const mcd_ctx*, std::string> slots;
    return slots[c];
}

const char* mcd_last_error(mcd_ctx* ctx)
{
    if (!ctx) return "null context";
    return error_slot(ctx).c_str();
}

const std::string& mcd_ctx::last_error() const { return error_slot(this); }

int mcd_ctx::fail(int status, const std::string& msg)
{
    error_slot(this) = msg;
    return status;
}

int mcd_ctx::hip_fail(hipError_t e, const char* what)
{
    error_slot(this) = std::string(what) + ": " + hipGetErrorString(e);
    return MCD_E_DEVICE;
}

int mcd_ctx::alloc(void** p, size_t bytes, const char* what)
{
    *p = nullptr;
    if (bytes == 0) return MCD_OK;
    std::lock_guard<std::mutex> g(mu_alloc);
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
    std::lock_guard<std::mutex> g(mu_alloc);
    (void)hipFree(p);
    used -= std::min(used, (uint64_t)bytes);
}

// Grows a device buffer to at least `need` bytes (contents are not kept).
int mcd_ctx::grow(void** p, size_t* have, size_t need, const char* what)
{
    if (*p && *have >= need) return MCD_OK;
    if (*p) {
        (void)hipDeviceSynchronize();
        release(*p, *have);
        *p = nullptr;
        *have = 0;
    }
    int rc = alloc(p, need, what);
    if (rc == MCD_OK) *have = need;
    return rc;
}

// ------------------------------------------------------------- create/destroy

int mcd_create(int device, uint64_t hbm_budget_bytes, mcd_ctx** out)
{
    if (!out) return MCD_E_INVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return MCD_E_INVAL;
    mcd::DeviceGuard dg(device);
    if (!dg.ok()) return MCD_E_DEVICE;
    mcd_ctx* c = new (std::nothrow) mcd_ctx();
    if (!c) return MCD_E_NOMEM;
    c->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete c;
        return MCD_E_DEVICE;
    }
    c->cu_count = prop.multiProcessorCount;
    c->clock_khz = prop.clockRate;
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
    if (init_kernels(c->max_lds) != hipSuccess) {
        mcd_destroy(c);
        return MCD_E_DEVICE;
    }
    // the no-allocation entry point's scratch on this device (its status is
    // kept and reported by that entry point; the rest of the library does not
    // depend on it)
    (void)mcd::noalloc_setup(device);
    *out = c;
    return MCD_OK;
}

int mcd_destroy(mcd_ctx* c)
{
    if (!c) return MCD_E_INVAL;
    mcd::DeviceGuard dg(c->device);
    (void)hipStreamSynchronize(c->stream);
    c->shutdown_serving();
    for (auto& t : c->tables)
        if (t.live) {
            c->release(t.dev.phot, t.bytes);
            c->release(t.dev.elec, t.bytes);
            c->release((void*)t.dev.hinge, t.bytes);
            c->release((void*)t.dev.posi, t.bytes / 2);
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
    c->release_graph();
    RegroupBufs& rb = c->rb;
    c->release(rb.queues, (size_t)4 * rb.cap * kRec);
    c->release(rb.ctl, 4 * sizeof(QCtl));
    c->release(rb.claim, (size_t)rb.claim_cap * 4);
    c->release(rb.req, (size_t)rb.req_cap * sizeof(ReqDev));
    c->release(rb.fin, (size_t)rb.req_cap * sizeof(FinalReq));
    c->release(rb.red, (size_t)rb.req_cap * 3 * sizeof(double));
    c->release(rb.tally, rb.tally_bytes);
    c->release(rb.dose, rb.stage_bytes);
    c->release(rb.sigma, rb.stage_bytes);
    c->release(rb.scratch, rb.scratch_bytes);
    for (auto& e : c->ev) (void)hipEventDestroy(e);
    (void)hipStreamDestroy(c->stream);
    delete c;
    return MCD_OK;
}

// ------------------------------------------------------------------ tables

namespace {

constexpr size_t kHdr = 8 + 4 * 4 + 9 * 8 + 2 * 4;
constexpr size_t kMatHdr = 16 + 6 * 8;
constexpr double kBohr = 5.29177210903e-9;    // cm
constexpr double kHbarC = 1.973269804e-11;    // MeV cm

template <class T> T rd(const unsigned char* p)
{
    T v;
    std::memcpy(&v, p, sizeof v);
    return v;
}

// Second-moment hinge law.  A step of kappa transport mean free paths has
// Lewis moments <mu> = (1 - e^-kappa)/2 and
// <mu^2> = <mu> - (1 - e^(-kappa r))/6 in mu = (1 - cos)/2, r = lambda1/lambda2.
// The law is  mu = S A v / (1 + A - v),  v = u / B, when the uniform u < B,
// and mu = 0 otherwise: a Wentzel law of screening A, either mixed with no
// deflection (B < 1, S = 1: a heavier tail than the first-moment Wentzel law
// a1) or compressed to [0, S] (S < 1, B = 1: a lighter tail).  A comes from
// a bisection in ln A on [a1, 1e3]; without a root the first-moment law
// (a1, 1, 1) is kept.
struct WentzelMoments {
    double m1, m2;
    explicit WentzelMoments(double a)
    {
        const double l = std::log1p(1.0 / a);
        m1 = a * ((1.0 + a) * l - 1.0);
        m2 = a * ((1.0 + 2.0 * a) - 2.0 * a * (1.0 + a) * l);
    }
};

template <class F> bool bisect_log(F f, double target, double lo, double hi, double& x)
{
    if (f(lo) > target || f(hi) < target) return false;
    while (hi / lo - 1.0 > 1e-15) {
        const double mid = std::sqrt(lo * hi);
        if (mid <= lo || mid >= hi) break;
        (f(mid) < target ? lo : hi) = mid;
    }
    x = std::sqrt(lo * hi);
    return true;
}

float4 hinge_law(double kappa, double a1, double r)
{
    const double m1 = -0.5 * std::expm1(-kappa);
    const double m2 = m1 + std::expm1(-kappa * r) / 6.0;
    float4 out = make_float4((float)a1, 1.f, 1.f, 0.f);
    if (!(m2 > m1 * m1 && m2 < m1)) return out;
    const double t = m2 / m1;
    auto ratio = [](double a) { WentzelMoments w(a); return w.m2 / w.m1; };
    auto spread = [](double a) { WentzelMoments w(a); return w.m1 * w.m1 / w.m2; };
    double a;
    if (t >= ratio(a1)) {
        if (bisect_log(ratio, t, a1, 1e3, a)) {
            out.x = (float)a;
            out.y = (float)(m1 / WentzelMoments(a).m1);
        }
    } else if (bisect_log(spread, m1 * m1 / m2, a1, 1e3, a)) {
        out.x = (float)a;
        out.z = (float)(t / ratio(a));
    }
    return out;
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
    if (ver != 4 || n_e != (uint32_t)kNE || n_q != (uint32_t)kNQ)
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
    const uint32_t flags = rd<uint32_t>(s + 72);
    if (flags & ~127u) return c->fail(MCD_E_INVAL, "table blob: unknown flags");
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
    for (uint32_t m = 0; m < n_mat; ++m)
        for (const double* r : {ts.range(m), ts.range_pos(m)})
            for (int i = 1; i < kNE; ++i)
                if (!(r[i] > r[i - 1])) return c->fail(MCD_E_INVAL, "table blob: range not increasing");
    // FP32 device layout: float4 per node for the photon and electron groups
    // and for the second-moment hinge law (left zero unless the blob asks)
    const bool hinge2 = (flags & 32u) != 0;
    std::vector<float4> ph((size_t)n_mat * kNE), el((size_t)n_mat * kNE), hl((size_t)n_mat * kNE);
    std::vector<float2> po((size_t)n_mat * kNE);
    for (uint32_t m = 0; m < n_mat; ++m)
        for (int i = 0; i < kNE; ++i) {
            const double* q = &ts.q[(size_t)m * kNQ * kNE];
            ph[m * kNE + i] = make_float4((float)q[0 * kNE + i], (float)q[1 * kNE + i],
                                          (float)q[2 * kNE + i], (float)q[8 * kNE + i]);
            el[m * kNE + i] = make_float4((float)q[3 * kNE + i], (float)q[4 * kNE + i],
                                          (float)q[5 * kNE + i], (float)q[6 * kNE + i]);
            po[m * kNE + i] = make_float2((float)q[10 * kNE + i], (float)q[11 * kNE + i]);
            hl[m * kNE + i] = hinge2 && q[4 * kNE + i] > 0.0
                                  ? hinge_law(ts.kappa_step, ts.a_hinge, q[9 * kNE + i] / q[4 * kNE + i])
                                  : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    mcd::DeviceGuard dg(c->device);
    ts.bytes = ph.size() * sizeof(float4);
    void* dev[4] = {nullptr, nullptr, nullptr, nullptr};            // phot, elec, hinge, posi
    const void* host[4] = {ph.data(), el.data(), hl.data(), po.data()};
    const size_t size[4] = {ts.bytes, ts.bytes, ts.bytes, po.size() * sizeof(float2)};
    auto release_all = [&] {
        for (int k = 0; k < 4; ++k) c->release(dev[k], size[k]);
    };
    for (int k = 0; k < 4; ++k) {
        const int rc = c->alloc(&dev[k], size[k], "tables");
        if (rc) {
            release_all();
            return rc;
        }
    }
    for (int k = 0; k < 4; ++k) {
        const hipError_t e = hipMemcpy(dev[k], host[k], size[k], hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            release_all();
            return c->hip_fail(e, "table upload");
        }
    }
    ts.dev.phot = (float4*)dev[0];
    ts.dev.elec = (float4*)dev[1];
    ts.dev.hinge = (const float4*)dev[2];
    ts.dev.posi = (const float2*)dev[3];
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
    d.angular = (flags & 4u) ? 1 : 0;
    d.hinge2 = hinge2 ? 1 : 0;
    d.bhabha = (flags & 64u) ? 1 : 0;
    bool any_mu_r = false;
    for (const float4& v : ph) any_mu_r = any_mu_r || v.w > 0.f;
    d.refined = (d.angular || d.hinge2 || d.bhabha || any_mu_r) ? 1 : 0;
    for (int m = 0; m < kMaxMat; ++m)
        d.r_abs_pos[m] =
            m < (int)n_mat ? (float)host_interp(ts.range_pos(m), ts.e_abs_e, ts.emin, ts.emax) : 0.f;
    // Rayleigh angular law of an exponentially screened atom: screening
    // radius a = 0.885 a0 Z_s^(-1/3), Z_s = B / (Z/A) from the material
    // header (rho, Z/A, I, B, ...); b = 2 (a E / hbar c)^2
    for (int m = 0; m < kMaxMat; ++m) {
        d.ray_b[m] = 0.f;
        if (m >= (int)n_mat) continue;
        const unsigned char* mh = b + kHdr + m * mat_bytes + 16;
        const double zoa = rd<double>(mh + 8), bz = rd<double>(mh + 24);
        if (zoa > 0.0 && bz > 0.0) {
            const double a = 0.885 * kBohr * std::cbrt(zoa / bz);
            d.ray_b[m] = (float)(2.0 * a * a / (kHbarC * kHbarC));
        }
    }
    d.f_shift = (float)(std::log2(1.0 - ts.f_e) * (kNE - 1) / std::log2(ts.emax / ts.emin));
    d.a_hinge = (float)ts.a_hinge;
    ts.live = true;
    std::lock_guard<mcd::FairMutex> run(c->run_mu);
    std::lock_guard<std::mutex> g(c->mu);
    c->tables.push_back(std::move(ts));
    *out_tables = (int32_t)c->tables.size() - 1;
    return MCD_OK;
}

int mcd_unload_materials(mcd_ctx* c, int32_t t)
{
    if (!c) return MCD_E_INVAL;
    std::lock_guard<mcd::FairMutex> run(c->run_mu);
    std::lock_guard<std::mutex> g(c->mu);
    if (t < 0 || t >= (int32_t)c->tables.size() || !c->tables[t].live) return MCD_E_NOTFOUND;
    for (auto& p : c->phantoms)
        if (p.live && p.tables == t) return c->fail(MCD_E_INVAL, "tables still used by a phantom");
    TableSet& ts = c->tables[t];
    mcd::DeviceGuard dg(c->device);
    (void)hipDeviceSynchronize();
    c->release(ts.dev.phot, ts.bytes);
    c->release(ts.dev.elec, ts.bytes);
    c->release((void*)ts.dev.hinge, ts.bytes);
    c->release((void*)ts.dev.posi, ts.bytes / 2);
    ts.live = false;
    ts.q.clear();
    return MCD_OK;
}

// ----------------------------------------------------------------- phantoms

int mcd_load_phantom(mcd_ctx* c, const mcd_grid* g, const uint8_t* mat, const float* rho,
                     int32_t tables, int32_t* out_phantom)
{
    if (!c || !g || !mat || !rho || !out_phantom) return MCD_E_INVAL;
    std::lock_guard<mcd::FairMutex> run(c->run_mu);
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
    // rho_max * (mu_C + mu_pe + mu_pp + mu_R) per gram, rounded up to FP32.
    std::vector<float> maj(kNE);
    for (int i = 0; i < kNE; ++i) {
        double best = 0.0;
        for (int m = 0; m < ts.n_mat; ++m) {
            if (rmax[m] <= 0.0) continue;
            const double* q = &ts.q[(size_t)m * kNQ * kNE];
            best = std::max(best, rmax[m] * (q[i] + q[kNE + i] + q[2 * kNE + i] + q[8 * kNE + i]));
        }
        float f = (float)best;
        if ((double)f < best) f = std::nextafter(f, INFINITY);
        maj[i] = f;
    }
    PhantomRec p;
    p.g = *g;
    p.tables = tables;
    p.nv = nv;
    mcd::DeviceGuard dg(c->device);
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
    std::lock_guard<mcd::FairMutex> run(c->run_mu);
    std::lock_guard<std::mutex> g(c->mu);
    if (ph < 0 || ph >= (int32_t)c->phantoms.size() || !c->phantoms[ph].live) return MCD_E_NOTFOUND;
    if (c->serving_uses(ph)) return c->fail(MCD_E_BUSY, "phantom has requests that are not collected yet");
    PhantomRec& p = c->phantoms[ph];
    mcd::DeviceGuard dg(c->device);
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
    const size_t lb = plain_lane_bytes(depth, slots);
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

