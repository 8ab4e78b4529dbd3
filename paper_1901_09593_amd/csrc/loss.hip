// The masked mean-L1 loss around the fused backward of the differentiable
// finest level: the loss pixels are counted before it (the gradient of a mean
// divides by the count), and the loss value is formed after it from the sum
// of |d_soft - gt| the fused backward accumulated.
#include <hip/hip_runtime.h>

#include "backward_impl.hpp"

namespace msibm {

// Sum of the mask over [first, first + count) of a row-major pitch-W map (16
// pixels per thread), added into *out once per wave.
__device__ __forceinline__ void count_span(const uint8_t* __restrict__ mask, size_t first, size_t total,
                                           int* out)
{
    int c = 0;
#pragma unroll
    for (int m = 0; m < ZERO_TILE / 256; ++m) {
        const size_t i = first + (size_t)m * 256 + threadIdx.x;
        if (i < total) c += mask[i] != 0;
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(out, c);
}

__global__ __launch_bounds__(256) void mask_count_kernel(const uint8_t* mask, size_t total, int* count)
{
    count_span(mask, (size_t)blockIdx.x * ZERO_TILE, total, count);
}

// Counts of every pair of a launch: one segment per pair, ZERO_TILE pixels per block.
__global__ __launch_bounds__(256) void mask_count_multi_kernel(MultiArgs a)
{
    const Segment s = a.segs[segment_of(a.segs, a.nseg, blockIdx.x)];
    const BackArgs& b = a.back[s.pair];
    count_span(b.mask, (size_t)(blockIdx.x - s.task0) * ZERO_TILE, (size_t)b.H * b.W, b.count);
}

__global__ void l1_finalize_kernel(const float* sum, const int* count, float* loss)
{
    if (threadIdx.x == 0) *loss = *sum / (float)max(*count, 1);
}

// One thread per pair of the launch's backward table.
__global__ __launch_bounds__(256) void l1_finalize_multi_kernel(MultiArgs a, int np)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p < np) {
        const BackArgs& b = a.back[p];
        *b.loss_out = *b.loss_sum / (float)max(*b.count, 1);
    }
}

hipError_t launch_mask_count(const uint8_t* mask, size_t total, int* count, hipStream_t s)
{
    const size_t blocks = (total + ZERO_TILE - 1) / ZERO_TILE;
    hipLaunchKernelGGL(mask_count_kernel, dim3((unsigned)(blocks ? blocks : 1)), dim3(256), 0, s, mask, total,
                       count);
    return hipGetLastError();
}

hipError_t launch_mask_count_multi(const MultiArgs& a, int blocks, hipStream_t s)
{
    if (blocks < 1 || a.nseg < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(mask_count_multi_kernel, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_l1_finalize(const float* sum, const int* count, float* loss, hipStream_t s)
{
    hipLaunchKernelGGL(l1_finalize_kernel, dim3(1), dim3(64), 0, s, sum, count, loss);
    return hipGetLastError();
}

hipError_t launch_l1_finalize_multi(const MultiArgs& a, int np, hipStream_t s)
{
    if (np < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(l1_finalize_multi_kernel, dim3((np + 255) / 256), dim3(256), 0, s, a, np);
    return hipGetLastError();
}

}  // namespace msibm
