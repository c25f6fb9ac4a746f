// The robust objective of Problem 1 at caller arrays with no handle and no
// workspace, for callers that cannot allocate device memory.  Its only
// device memory beyond the caller's inputs and output is `scratch`, a
// file-scope array of per-block partial sums: every GPU the library runs on
// holds its own copy until the process ends, and every call on that GPU
// shares it, so calls that overlap on one GPU race.
#include "daba.h"
#include "daba_eval.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

namespace {

constexpr int kThreads = 256;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[DABA_NOALLOC_BLOCKS];

std::mutex g_mutex;
void* g_scratch[kMaxDevices] = {};  // the address of `scratch` on each device, once taken

// The partial sums of F = sum 1/2 rho(|e|^2) (eq. error, caller units: pixels
// and the caller's intrinsics) over the observations o = b * 256 + thread,
// stepping by nb * 256, in that order; a block sum in a fixed order.  An
// observation with an index out of range or |l - t|^2 <= 1e-24 (Assumption 2)
// makes its block's sum NaN.
template <int LOSS>
__global__ __launch_bounds__(kThreads) void k_partial(int64_t M, int64_t N, int64_t K,
                                                      const int32_t* __restrict__ oc, const int32_t* __restrict__ ol,
                                                      const double* __restrict__ uv, const double* __restrict__ cams,
                                                      const double* __restrict__ lms, double delta,
                                                      double* __restrict__ part, int nb) {
    __shared__ double red[kThreads / 64];
    double acc = 0.0;
    bool bad = false;
    for (int64_t o = (int64_t)blockIdx.x * kThreads + threadIdx.x; o < K; o += (int64_t)nb * kThreads) {
        const int32_t i = oc[o], j = ol[o];
        if (i < 0 || i >= M || j < 0 || j >= N) {
            bad = true;
            continue;
        }
        const daba::CamT<double> c = daba::load_cam<double>(cams + 15 * (size_t)i);
        const double* l = lms + 3 * (size_t)j;
        const double ux = uv[2 * o], uy = uv[2 * o + 1];
        const double r2u = ux * ux + uy * uy;
        daba::ObsEvalCF<LOSS, double> e;
        daba::eval_obs_cf<LOSS, double>(c, l[0], l[1], l[2], ux, uy, r2u, r2u * r2u, delta, e);
        bad |= !(e.r2 > 1e-24);
        acc += 0.5 * e.rho;
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    bad = __any(bad);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x / 64] = bad ? NAN : acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) s += red[w];
        part[blockIdx.x] = s;
    }
}

// F = the nb partial sums added in a fixed order (strided per thread, then
// per wave and per block).
__global__ __launch_bounds__(kThreads) void k_total(const double* __restrict__ part, int nb, double* __restrict__ F) {
    __shared__ double red[kThreads / 64];
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += kThreads) acc += part[b];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x / 64] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) s += red[w];
        *F = s;
    }
}

}  // namespace

extern "C" int daba_objective_noalloc(int64_t n_cameras, int64_t n_landmarks, int64_t n_obs,
                                      const int32_t* obs_camera, const int32_t* obs_landmark, const double* obs_uv,
                                      const double* cameras, const double* landmarks, int loss, double loss_delta,
                                      double* F_out, void* hip_stream) {
    if (n_cameras < 1 || n_landmarks < 1 || n_obs < 0 || n_cameras > INT32_MAX || n_landmarks > INT32_MAX ||
        n_obs > DABA_NOALLOC_MAX_OBS)
        return DABA_E_INVAL;
    if (!cameras || !landmarks || !F_out || (n_obs > 0 && (!obs_camera || !obs_landmark || !obs_uv)))
        return DABA_E_INVAL;
    if (loss < DABA_LOSS_TRIVIAL || loss > DABA_LOSS_WELSCH) return DABA_E_INVAL;
    if (loss != DABA_LOSS_TRIVIAL && !(loss_delta > 0.0 && std::isfinite(loss_delta))) return DABA_E_INVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return DABA_E_HIP;
    double* part = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mutex);
        if (!g_scratch[dev]) {
            void* ptr = nullptr;
            if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return DABA_E_HIP;
            g_scratch[dev] = ptr;
        }
        part = static_cast<double*>(g_scratch[dev]);
    }
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int64_t want = (n_obs + kThreads - 1) / kThreads;
    const int nb = (int)(want < DABA_NOALLOC_BLOCKS ? want : DABA_NOALLOC_BLOCKS);
    const double delta = loss == DABA_LOSS_TRIVIAL ? 1.0 : loss_delta;
    if (nb > 0) {
        const dim3 grid(nb), block(kThreads);
        if (loss == DABA_LOSS_HUBER)
            hipLaunchKernelGGL((k_partial<1>), grid, block, 0, s, n_cameras, n_landmarks, n_obs, obs_camera,
                               obs_landmark, obs_uv, cameras, landmarks, delta, part, nb);
        else if (loss == DABA_LOSS_WELSCH)
            hipLaunchKernelGGL((k_partial<2>), grid, block, 0, s, n_cameras, n_landmarks, n_obs, obs_camera,
                               obs_landmark, obs_uv, cameras, landmarks, delta, part, nb);
        else
            hipLaunchKernelGGL((k_partial<0>), grid, block, 0, s, n_cameras, n_landmarks, n_obs, obs_camera,
                               obs_landmark, obs_uv, cameras, landmarks, delta, part, nb);
    }
    hipLaunchKernelGGL(k_total, dim3(1), dim3(kThreads), 0, s, part, nb, F_out);
    return hipGetLastError() == hipSuccess ? DABA_OK : DABA_E_HIP;
}
