// Roofline calibration kernels: the two denominators the rooflines are
// quoted against, measured on the device instead of taken from the sheet.
//
//   k_calib_copy  streaming copy, four independent 16-byte loads
//                 per lane in flight, a grid of 8 workgroups of 256 per CU
//                 striding over the buffers: HBM bytes moved = 2 x nbytes
//                 (read + write).
//   k_calib_fma   kCalibChains independent FP32 FMA chains per lane, iters
//                 rounds: lane-FMA operations = threads x kCalibChains x
//                 iters (one non-packed v_fma_f32 each; packed FP32 is off
//                 in this build).  The chains' sum is written so that the
//                 compiler keeps them.
#pragma once
#include "vsr_internal.h"

namespace vsr {

constexpr int kCalibChains = 8;

constexpr int kCalibUnroll = 4;  // independent 16-byte loads in flight per lane

__global__ __launch_bounds__(256) void k_calib_copy(const float4* __restrict__ src, float4* __restrict__ dst,
                                                    int64_t n) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    for (; i + (kCalibUnroll - 1) * stride < n; i += kCalibUnroll * stride) {
        float4 v[kCalibUnroll];
#pragma unroll
        for (int u = 0; u < kCalibUnroll; ++u) v[u] = src[i + u * stride];
#pragma unroll
        for (int u = 0; u < kCalibUnroll; ++u) dst[i + u * stride] = v[u];
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

__global__ __launch_bounds__(256) void k_calib_fma(float* __restrict__ out, int32_t iters, float m, float c) {
    float x[kCalibChains];
#pragma unroll
    for (int k = 0; k < kCalibChains; ++k) x[k] = float(threadIdx.x + k) * 1e-3f;
    for (int32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kCalibChains; ++k) x[k] = fmaf(x[k], m, c);
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < kCalibChains; ++k) s += x[k];
    out[int64_t(blockIdx.x) * blockDim.x + threadIdx.x] = s;
}

inline hipError_t launch_calib_copy(const void* src, void* dst, int64_t nbytes, hipStream_t st) {
    const int64_t n = nbytes / 16;
    hipLaunchKernelGGL(k_calib_copy, dim3(256 * 8), dim3(256), 0, st, reinterpret_cast<const float4*>(src),
                       reinterpret_cast<float4*>(dst), n);
    return hipGetLastError();
}

inline hipError_t launch_calib_fma(float* out, int64_t nthreads, int32_t iters, hipStream_t st) {
    // m, c keep the values bounded: x -> 0.5 x + 0.25 converges to 0.5
    hipLaunchKernelGGL(k_calib_fma, dim3(unsigned(nthreads / 256)), dim3(256), 0, st, out, iters, 0.5f, 0.25f);
    return hipGetLastError();
}

}  // namespace vsr
