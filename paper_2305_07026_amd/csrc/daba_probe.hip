// Measurement only: a plain streaming copy, the bandwidth ceiling that the
// iteration's kernels are compared with next to the vendor peak.  It
// computes nothing of the method.

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "daba.h"

namespace {

// dst[i] = src[i] over n 16-byte elements, grid-stride.
__global__ __launch_bounds__(256) void k_stream_copy(const float4* __restrict__ src, float4* __restrict__ dst,
                                                     size_t n) {
    const size_t step = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) dst[i] = src[i];
}

}  // namespace

extern "C" int daba_stream_copy(void* dst, const void* src, size_t bytes, int blocks, void* hip_stream) {
    if (!dst || !src || bytes % 16 != 0 || blocks < 1 || blocks > (1 << 20)) return DABA_E_INVAL;
    if ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) % 16 != 0) return DABA_E_INVAL;
    if (bytes == 0) return DABA_OK;
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)hip_stream,
                       static_cast<const float4*>(src), static_cast<float4*>(dst), bytes / 16);
    return hipGetLastError() == hipSuccess ? DABA_OK : DABA_E_HIP;
}
