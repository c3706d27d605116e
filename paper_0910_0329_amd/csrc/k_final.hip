// Dose finalisation (Sec. 3: dose per voxel, its standard deviation, Dmax and
// the mean relative uncertainty over voxels above half of Dmax) and small
// utility kernels.  FP64 throughout.
#include "engine.h"

namespace mcd {

constexpr double kMevPerGToGy = 1.602176634e-10;
// Dmax and sigma-bar cover tissue voxels only (density >= 0.05 g/cm^3: lung and
// denser): an air voxel's dose rests on a few deposits in a tiny mass and
// would set Dmax and dominate sigma-bar with noise.  Dose and sigma are still
// written for every voxel.
constexpr float kTissueRhoMin = 0.05f;

#define DEV_INLINE __device__ __forceinline__

DEV_INLINE void block_max_to(double mx, double* red)
{
    __shared__ double smax[16];
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if ((threadIdx.x & 63) == 0) smax[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < (int)(blockDim.x >> 6); ++i) mx = fmax(mx, smax[i]);
        atomicMax((unsigned long long*)&red[0], (unsigned long long)__double_as_longlong(mx));
    }
}

DEV_INLINE void wave_add_to(double acc, double cnt, double* red)
{
    for (int o = 32; o > 0; o >>= 1) {
        acc += __shfl_xor(acc, o, 64);
        cnt += __shfl_xor(cnt, o, 64);
    }
    if ((threadIdx.x & 63) == 0 && cnt > 0.0) {
        unsafeAtomicAdd(&red[1], acc);
        unsafeAtomicAdd(&red[2], cnt);
    }
}

// History-by-history statistics: dose = S / (N rho V), sigma^2 = (Q/N - (S/N)^2) / (N - 1).
__global__ void k_dose(const double* S, const double* Q, const uint2* vox, int64_t nv,
                       double vol, double N, double* dose, double* sigma, double* red)
{
    double mx = 0.0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv;
         v += (int64_t)gridDim.x * blockDim.x) {
        const float rho = __uint_as_float(vox[v].x);
        const double scale = kMevPerGToGy / ((double)rho * vol);
        const double mean = S[v] / N;
        const double var = (Q[v] / N - mean * mean) / (N - 1.0);
        const double d = mean * scale;
        dose[v] = d;
        sigma[v] = sqrt(var > 0.0 ? var : 0.0) * scale;
        if (rho >= kTissueRhoMin) mx = fmax(mx, d);
    }
    block_max_to(mx, red);
}

// sigma-bar: mean of sigma/D over voxels with D > Dmax / 2 (red[1] sum, red[2] count).
__global__ void k_sigma_bar(const double* dose, const double* sigma, const uint2* vox, int64_t nv,
                            double* red)
{
    const double half = 0.5 * red[0];
    double acc = 0.0, cnt = 0.0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv;
         v += (int64_t)gridDim.x * blockDim.x) {
        const double d = dose[v];
        if (d > half && __uint_as_float(vox[v].x) >= kTissueRhoMin) {
            acc += sigma[v] / d;
            cnt += 1.0;
        }
    }
    wave_add_to(acc, cnt, red);
}

static int final_blocks(int64_t nv)
{
    int64_t b = (nv + 255) / 256;
    return (int)(b > 4096 ? 4096 : (b < 1 ? 1 : b));
}

hipError_t launch_finalize(const double* S, const double* Q, const uint2* vox, int64_t nv,
                           double vol, uint64_t n, double* dose, double* sigma, double* red,
                           hipStream_t s)
{
    const int blocks = final_blocks(nv);
    hipLaunchKernelGGL(k_dose, dim3(blocks), dim3(256), 0, s, S, Q, vox, nv, vol, (double)n, dose,
                       sigma, red);
    hipLaunchKernelGGL(k_sigma_bar, dim3(blocks), dim3(256), 0, s, dose, sigma, vox, nv, red);
    return hipGetLastError();
}

// Batch statistics: the request's histories are split into kBatches groups
// (history mod kBatches) with nb[b] histories and sub-tallies T_b.  Dose from
// S = sum_b T_b; the per-history variance is estimated from the spread of the
// group means m_b = T_b / nb[b] around m = S / N,
//     s^2 = sum_b nb[b] (m_b - m)^2 / (B' - 1),   sigma_mean^2 = s^2 / N,
// with B' the number of non-empty groups.  The square root of that unbiased
// variance reads low by c4(B') (normal group means: the weighted sum of
// squares is chi-square with B' - 1 degrees of freedom), so the reported
// sigma is sigma_mean / c4(B'), c4(k) = sqrt(2/(k-1)) Gamma(k/2) / Gamma((k-1)/2).
DEV_INLINE double c4_of(int k)
{
    if (k < 2) return 1.0;
    return sqrt(2.0 / (double)(k - 1)) * exp(lgamma(0.5 * (double)k) - lgamma(0.5 * (double)(k - 1)));
}

template <class T>
__global__ void k_dose_batches(const FinalReq* reqs, const uint2* vox, int64_t nv, double vol)
{
    const FinalReq& r = reqs[blockIdx.y];
    const T* tal = (const T*)r.tally;
    double N = 0.0;
    int nz = 0;
    for (int b = 0; b < kBatches; ++b) {
        N += r.nb[b];
        nz += r.nb[b] > 0.0;
    }
    const double inv_c4 = 1.0 / c4_of(nz);
    double mx = 0.0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv;
         v += (int64_t)gridDim.x * blockDim.x) {
        double tb[kBatches];
        double S = 0.0;
#pragma unroll
        for (int b = 0; b < kBatches; ++b) {
            tb[b] = (double)tal[(int64_t)b * nv + v];
            S += tb[b];
        }
        const double m = S / N;
        double ss = 0.0;
#pragma unroll
        for (int b = 0; b < kBatches; ++b)
            if (r.nb[b] > 0.0) {
                const double dm = tb[b] / r.nb[b] - m;
                ss += r.nb[b] * dm * dm;
            }
        const double var = nz > 1 ? ss / (double)(nz - 1) / N : 0.0;
        const float rho = __uint_as_float(vox[v].x);
        const double scale = kMevPerGToGy / ((double)rho * vol);
        const double d = m * scale;
        if (r.S) r.S[v] = S;
        if (r.dose) r.dose[v] = d;
        if (r.sigma) r.sigma[v] = sqrt(var) * inv_c4 * scale;
        if (rho >= kTissueRhoMin) mx = fmax(mx, d);
    }
    block_max_to(mx, r.red);
}

__global__ void k_sigma_bar_batches(const FinalReq* reqs, const uint2* vox, int64_t nv)
{
    const FinalReq& r = reqs[blockIdx.y];
    const double half = 0.5 * r.red[0];
    double acc = 0.0, cnt = 0.0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv;
         v += (int64_t)gridDim.x * blockDim.x) {
        const double d = r.dose[v];
        if (d > half && __uint_as_float(vox[v].x) >= kTissueRhoMin) {
            acc += r.sigma[v] / d;
            cnt += 1.0;
        }
    }
    wave_add_to(acc, cnt, r.red);
}

hipError_t launch_finalize_batches(const FinalReq* reqs, int n_req, const uint2* vox,
                                   int64_t nv, double vol, int fp32, hipStream_t s)
{
    if (n_req <= 0) return hipSuccess;      // nothing to finalise (e.g. a serving epoch)
    int bx = final_blocks(nv);
    if ((int64_t)bx * n_req > 65536) bx = (int)(65536 / n_req) + 1;
    const dim3 grid(bx, n_req);
    if (fp32) hipLaunchKernelGGL(k_dose_batches<float>, grid, dim3(256), 0, s, reqs, vox, nv, vol);
    else hipLaunchKernelGGL(k_dose_batches<double>, grid, dim3(256), 0, s, reqs, vox, nv, vol);
    hipLaunchKernelGGL(k_sigma_bar_batches, grid, dim3(256), 0, s, reqs, vox, nv);
    return hipGetLastError();
}

// Zeroes the local-counter keys of every lane of the plain kernel (once after
// allocation and after a run that stopped on an error with keys still set).
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

hipError_t launch_clear_lane_keys(char* scratch, size_t lanes, size_t lane_bytes, int stack_depth,
                                  int slots, hipStream_t s)
{
    hipLaunchKernelGGL(k_clear_keys, dim3(4096), dim3(256), 0, s, scratch, lanes, lane_bytes,
                       (size_t)stack_depth * kRec, slots);
    return hipGetLastError();
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

}  // namespace mcd
