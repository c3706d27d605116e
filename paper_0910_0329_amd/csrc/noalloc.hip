// mcd_simulate_noalloc: the regrouped transport of mcd_simulate for callers
// that cannot allocate device memory (code under HIP graph capture, tight
// serving loops, harnesses that forbid hipMalloc).  Every buffer the run needs
// beyond the caller's inputs and outputs (run scalars, queue control and claim
// counters, request and finaliser tables, the 16 sub-tallies and the lane
// stacks) is carved out of one file-scope device array of kNoAllocBytes.  Each
// device holds its own copy of the array from the first use of this library
// on it until the process ends; its address is looked up once per device, at
// context creation, with hipGetSymbolAddress.  Calls on one device share the
// array and keep the last call's contents, so a per-device mutex orders them
// and every counter and tally is cleared by a fill kernel before a run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>

#include "engine.h"
#include "mcdose.h"
#include "runtime.h"

namespace mcd {
constexpr size_t kNoAllocBytes = (size_t)512 << 20;   // 512 MiB per device
// Default lane-stack depth of this entry point: 26 records fill the 1280-byte
// lane slot that 24 would take anyway, and the deepest stack seen over 1e6
// histories of 20 MeV electrons is 15 (8 for 6 MV photons).
constexpr int kNoAllocDepth = 26;
constexpr int kNoAllocDevices = 64;
}  // namespace mcd

static __device__ __align__(256) unsigned char scratch[mcd::kNoAllocBytes];

namespace {

struct DeviceScratch {
    std::mutex run;            // one no-allocation run at a time on the device
    void* ptr = nullptr;       // this device's copy of `scratch`
    hipError_t status = hipErrorNotInitialized;
};

std::mutex g_setup;
DeviceScratch g_dev[mcd::kNoAllocDevices];

size_t carve(size_t& off, size_t bytes)
{
    const size_t at = off;
    off = (off + bytes + 255) & ~(size_t)255;
    return at;
}

}  // namespace

// Looks up this device's address of `scratch` (the calling thread has made
// `device` current).  Done once per device; later calls return the outcome
// of the first.
hipError_t mcd::noalloc_setup(int device)
{
    if (device < 0 || device >= kNoAllocDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_setup);
    DeviceScratch& d = g_dev[device];
    if (d.status == hipErrorNotInitialized) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        d.status = e;
        d.ptr = e == hipSuccess ? p : nullptr;
    }
    return d.status;
}

using namespace mcd;

int mcd_simulate_noalloc(mcd_ctx* c, int32_t phantom, const mcd_source* src, uint64_t n_histories,
                         uint64_t seed, uint32_t request_key, const mcd_opts* opts, mcd_result* out,
                         void* hip_stream)
{
    if (!c || !out) return MCD_E_INVAL;
    std::lock_guard<mcd::FairMutex> run_lock(c->run_mu);
    if (phantom < 0 || phantom >= (int32_t)c->phantoms.size() || !c->phantoms[phantom].live)
        return c->fail(MCD_E_NOTFOUND, "unknown phantom handle");
    const uint64_t first = opts ? opts->first_history : 0;
    if (n_histories < 2 || n_histories >= ((uint64_t)1 << 32) || seed >= ((uint64_t)1 << 32) ||
        first >= ((uint64_t)1 << 32) || first + n_histories > ((uint64_t)1 << 32))
        return c->fail(MCD_E_INVAL, "need 2 <= n_histories < 2^32, seed < 2^32, first + n <= 2^32");
    if (!out->on_device || !out->dose || !out->sigma || out->Q)
        return c->fail(MCD_E_INVAL, "noalloc: dose and sigma must be device buffers (S optional, no Q)");
    if (opts && (opts->kernel != MCD_KERNEL_REGROUPED || opts->regroup == 1 || opts->use_graph ||
                 opts->accumulate))
        return c->fail(MCD_E_INVAL, "noalloc: regrouped kernel with lane stacks only; no use_graph, no accumulate");
    mcd_opts o;
    std::memset(&o, 0, sizeof o);
    if (opts) o = *opts;
    if (!o.stack_depth) o.stack_depth = kNoAllocDepth;
    o.regroup = 2;

    RegroupPlan plan;
    int rc = c->prepare_regroup(phantom, &src, &n_histories, &request_key, 1, seed, &o, plan);
    if (rc) return rc;
    const PhantomRec& ph = c->phantoms[phantom];

    // layout of the scratch: scalars | queue control | claim counters |
    // request table | finaliser table | reductions | sub-tallies | lane stacks
    RegroupBufs B;
    size_t off = 0;
    const size_t o_small = carve(off, kSmallBytes);
    const size_t o_ctl = carve(off, 4 * sizeof(QCtl));
    B.claim_cap = plan.cycles + kExtraCycles;
    const size_t o_claim = carve(off, (size_t)B.claim_cap * sizeof(unsigned int));
    const size_t o_req = carve(off, sizeof(ReqDev));
    const size_t o_fin = carve(off, sizeof(FinalReq));
    const size_t o_red = carve(off, 3 * sizeof(double));
    B.tally_bytes = (size_t)kBatches * (size_t)ph.nv * (plan.fp32 ? sizeof(float) : sizeof(double));
    const size_t o_tally = carve(off, B.tally_bytes);
    B.scratch_bytes = (size_t)plan.blocks * plan.threads * phase_lane_bytes(plan.depth);
    const size_t o_stack = carve(off, B.scratch_bytes);
    if (off > kNoAllocBytes)
        return c->fail(MCD_E_INVAL, "noalloc: the run needs " + std::to_string(off) +
                                        " bytes of scratch and the entry point holds " +
                                        std::to_string(kNoAllocBytes) +
                                        " (lower grid_blocks or stack_depth, or set tally_fp32)");

    mcd::DeviceGuard dg(c->device);
    if (!dg.ok()) return c->fail(MCD_E_DEVICE, "noalloc: cannot make the context's device current");
    DeviceScratch& d = g_dev[c->device];
    if (d.status != hipSuccess || !d.ptr) return c->hip_fail(d.status, "noalloc: scratch address");
    std::lock_guard<std::mutex> dev_lock(d.run);
    unsigned char* base = (unsigned char*)d.ptr;
    B.ctl = (QCtl*)(base + o_ctl);
    B.claim = (unsigned int*)(base + o_claim);
    B.req = (ReqDev*)(base + o_req);
    B.req_cap = 1;
    B.fin = (FinalReq*)(base + o_fin);
    B.red = (double*)(base + o_red);
    B.tally = base + o_tally;
    B.scratch = (char*)(base + o_stack);
    plan.bufs = &B;
    plan.small = base + o_small;
    plan.req[0].tally = B.tally;
    FinalReq& f = plan.fin[0];
    std::memset(&f, 0, sizeof f);
    f.tally = B.tally;
    f.S = out->S;
    f.dose = out->dose;
    f.sigma = out->sigma;
    f.red = B.red;
    for (int b = 0; b < kBatches; ++b) f.nb[b] = plan.nb[b];

    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : c->stream;
    hipError_t e = hipMemcpyAsync(B.req, plan.req.data(), sizeof(ReqDev), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(B.fin, plan.fin.data(), sizeof(FinalReq), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return c->hip_fail(e, "noalloc: request table upload");
    if ((rc = c->enqueue_regroup(plan, true, false, s))) return rc;
    int cycles_run = 0;
    if ((rc = c->finish_regroup(plan, s, &cycles_run))) return rc;
    plan.launches = cycles_run;
    mcd_result* outs[1] = {out};
    return c->collect_regroup(plan, outs, out, s);
}
