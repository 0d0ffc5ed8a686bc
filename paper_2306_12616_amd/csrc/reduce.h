// Deterministic wavefront / workgroup reductions (fixed combination order).
#pragma once

#include <hip/hip_runtime.h>

namespace chebdm {

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline double wave_min(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ inline double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Sum over a workgroup of NT threads; every thread receives the result.
// smem must hold NT/64 doubles and is reused after a barrier.
template <int NT>
__device__ inline double block_sum(double v, double* smem) {
    static_assert(NT % 64 == 0 && NT <= 1024, "workgroup must be whole wavefronts");
    constexpr int NW = NT / 64;
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) smem[wid] = v;
    __syncthreads();
    double r = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) r += smem[w];
    return r;
}

template <int NT>
__device__ inline double block_min(double v, double* smem) {
    constexpr int NW = NT / 64;
    v = wave_min(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) smem[wid] = v;
    __syncthreads();
    double r = smem[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) r = fmin(r, smem[w]);
    return r;
}

template <int NT>
__device__ inline double block_max(double v, double* smem) {
    constexpr int NW = NT / 64;
    v = wave_max(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) smem[wid] = v;
    __syncthreads();
    double r = smem[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) r = fmax(r, smem[w]);
    return r;
}

}  // namespace chebdm
