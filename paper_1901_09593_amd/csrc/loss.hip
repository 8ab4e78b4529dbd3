// The masked mean-L1 loss around the fused backward of the differentiable
// finest level: the loss pixels are counted before it (the gradient of a mean
// divides by the count), and the loss value is formed after it from the sum
// of |d_soft - gt| the fused backward accumulated.
#include <hip/hip_runtime.h>

#include "backward_impl.hpp"

namespace msibm {

// Nonzero bytes of a 32-bit word.
__device__ __forceinline__ int nonzero_bytes(unsigned w)
{
    return ((w & 0xffu) != 0) + ((w & 0xff00u) != 0) + ((w & 0xff0000u) != 0) + ((w & 0xff000000u) != 0);
}

// Nonzero entries of the mask in [first, first + COUNT_TILE) of a row-major
// pitch-W map, clipped to `total`, added into *out once per workgroup (all
// pixels of a pair share one counter, so fewer, larger adds).  Each thread
// takes 16 consecutive bytes per step: one 16-byte load where the whole span
// is inside and aligned, bytewise otherwise.
__device__ __forceinline__ void count_span(const uint8_t* __restrict__ mask, size_t first, size_t total,
                                           int* out)
{
    __shared__ int part[256 / 64];
    int c = 0;
    for (int m = 0; m < COUNT_TILE / (256 * 16); ++m) {
        const size_t i0 = first + (size_t)m * 256 * 16 + 16 * (size_t)threadIdx.x;
        if (i0 + 16 <= total && ((reinterpret_cast<uintptr_t>(mask + i0) & 15) == 0)) {
            const uint4 v = *reinterpret_cast<const uint4*>(mask + i0);
            c += nonzero_bytes(v.x) + nonzero_bytes(v.y) + nonzero_bytes(v.z) + nonzero_bytes(v.w);
        } else {
            for (int k = 0; k < 16; ++k)
                if (i0 + k < total) c += mask[i0 + k] != 0;
        }
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int t = part[0] + part[1] + part[2] + part[3];
        if (t) atomicAdd(out, t);
    }
}

__global__ __launch_bounds__(256) void mask_count_kernel(const uint8_t* mask, size_t total, int* count)
{
    count_span(mask, (size_t)blockIdx.x * COUNT_TILE, total, count);
}

// Counts of every pair of a launch: one segment per pair, COUNT_TILE pixels per block.
__global__ __launch_bounds__(256) void mask_count_multi_kernel(MultiArgs a)
{
    const Segment s = a.segs[segment_of(a.segs, a.nseg, blockIdx.x)];
    const BackArgs& b = a.back[s.pair];
    count_span(b.mask, (size_t)(blockIdx.x - s.task0) * COUNT_TILE, (size_t)b.H * b.W, b.count);
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
    const size_t blocks = (total + COUNT_TILE - 1) / COUNT_TILE;
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
