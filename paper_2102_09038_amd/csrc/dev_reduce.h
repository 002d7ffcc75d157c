// Fixed-order reductions over a work-group of 256 threads (four waves of 64), shared by the
// all-direction CG and the multigrid kernels: every work-group of a direction that sums the same
// partials gets the same bits.
#pragma once

#include <hip/hip_runtime.h>

namespace rte {
namespace dev {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// sum over the work-group in a fixed order; the result is returned to every thread
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    const double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return r;
}

// maximum over the work-group (order-free); the result is returned to every thread
__device__ __forceinline__ double block_max(double v, double* sh) {
    v = wave_max(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    const double r = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    __syncthreads();
    return r;
}

// sum of n partials in a fixed order (lane l takes l, l + 64, ...; then a fixed butterfly),
// computed by every thread of the work-group, identical bits in every work-group
__device__ __forceinline__ double partial_sum(const double* __restrict__ part, int n, double* sh) {
    double v = 0.0;
    if (threadIdx.x < 64)
        for (int i = threadIdx.x; i < n; i += 64) v += part[i];
    if (threadIdx.x < 64) v = wave_sum(v);
    __syncthreads();
    if (threadIdx.x == 0) sh[4] = v;
    __syncthreads();
    const double r = sh[4];
    __syncthreads();
    return r;
}

// work-group b of a (row tile, direction) grid: XCD b mod 8, every tile of direction k on one
// XCD (k = xcd + 8 (local / ntiles)); false past the last direction
__device__ __forceinline__ bool dir_tile(int ntiles, int nS, int& k, int& t) {
    const int b = blockIdx.x;
    const int xcd = b & 7, local = b >> 3;
    k = xcd + 8 * (local / ntiles);
    t = local % ntiles;
    return k < nS;
}

}  // namespace dev
}  // namespace rte
