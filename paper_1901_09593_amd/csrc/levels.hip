// Pyramid construction and per-level window statistics.
//
// reduce: one Gaussian-pyramid step (Section III) for both views in one launch.
//   The blur is the separable 5-tap binomial [1 4 6 4 1]/16 with clamp-to-edge
//   reads, evaluated only at even rows and columns.  Integer weights with a final
//   exact scale by 2^-8 keep every partial sum exact for uint8 input up to level
//   2 (values need at most 8 + 8k significant bits).  HBM-bound: 1 or 4 bytes
//   read per source pixel (mostly from L2), 4 bytes written per output pixel.
// stats: per pixel and view, the window mean (as a float plus its rounding
//   remainder, so the matching kernel can centre windows without losing the
//   mean's low bits) and 1/sqrt(A) with A the sum of squared deviations over the
//   clamped (2n+1)^2 window (the denominators of Eq. 2), or 0 when the window
//   variance A/N is at most var_eps (flat window).  Separable box sums over an
//   LDS tile, accumulated in double precision so the flat test and A match the
//   double-precision definition.
#include "common.hpp"

namespace msibm {

template <typename T>
__global__ __launch_bounds__(256) void reduce_kernel(ReduceArgs a)
{
    const int view = blockIdx.z;
    const T* __restrict__ src = static_cast<const T*>(a.src[view]);
    float* __restrict__ dst = a.dst[view];
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= a.Wo || y >= a.Ho) return;
    const float w[5] = {1.f, 4.f, 6.f, 4.f, 1.f};
    int cx[5];
#pragma unroll
    for (int b = 0; b < 5; ++b) cx[b] = clampi(2 * x + b - 2, 0, a.W - 1);
    float acc = 0.f;
#pragma unroll
    for (int t = 0; t < 5; ++t) {
        const T* row = src + (size_t)clampi(2 * y + t - 2, 0, a.H - 1) * a.spitch;
        float h = 0.f;
#pragma unroll
        for (int b = 0; b < 5; ++b) h = fmaf(w[b], to_f(row[cx[b]]), h);
        acc = fmaf(w[t], h, acc);
    }
    dst[(size_t)y * a.dpitch + x] = acc * (1.f / 256.f);
}

template <typename T>
__global__ __launch_bounds__(256) void convert_kernel(ConvertArgs a)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= a.W || y >= a.H) return;
    a.dst[(size_t)y * a.dpitch + x] = to_f(static_cast<const T*>(a.src)[(size_t)y * a.spitch + x]);
}

constexpr int ST_W = 64, ST_H = 16, ST_MAXN = 6;
constexpr int ST_RW = ST_W + 2 * ST_MAXN;  // 76
constexpr int ST_RH = ST_H + 2 * ST_MAXN;  // 28

template <typename T>
__global__ __launch_bounds__(256) void stats_kernel(StatsArgs a)
{
    __shared__ float tile[ST_RH][ST_RW + 1];
    __shared__ double h1[ST_RH][ST_W];
    __shared__ double h2[ST_RH][ST_W];
    const int view = blockIdx.z;
    const T* __restrict__ src = static_cast<const T*>(a.src[view]);
    float4* __restrict__ dst = a.dst[view];
    const int n = a.n, wn = 2 * n + 1;
    const int x0 = blockIdx.x * ST_W, y0 = blockIdx.y * ST_H;
    const int rows = ST_H + 2 * n, cols = ST_W + 2 * n;
    // centre on one pixel of the tile: the sums below then stay small
    const float c = to_f(src[(size_t)min(y0, a.H - 1) * a.spitch + min(x0, a.W - 1)]);
    for (int idx = threadIdx.x; idx < rows * cols; idx += 256) {
        const int rr = idx / cols, cc = idx - rr * cols;
        const int gy = clampi(y0 - n + rr, 0, a.H - 1), gx = clampi(x0 - n + cc, 0, a.W - 1);
        tile[rr][cc] = to_f(src[(size_t)gy * a.spitch + gx]) - c;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < rows * ST_W; idx += 256) {
        const int rr = idx / ST_W, cc = idx - rr * ST_W;
        double s1 = 0.0, s2 = 0.0;
        for (int b = 0; b < wn; ++b) {
            const double v = tile[rr][cc + b];
            s1 += v;
            s2 += v * v;
        }
        h1[rr][cc] = s1;
        h2[rr][cc] = s2;
    }
    __syncthreads();
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const double N = (double)(wn * wn);
    for (int oy = ty; oy < ST_H; oy += 4) {
        const int gy = y0 + oy, gx = x0 + tx;
        if (gy >= a.H || gx >= a.W) continue;
        double s1 = 0.0, s2 = 0.0;
        for (int t = 0; t < wn; ++t) {
            s1 += h1[oy + t][tx];
            s2 += h2[oy + t][tx];
        }
        const double A = s2 - s1 * s1 / N;
        const float inv = (A <= N * a.var_eps) ? 0.f : (float)(1.0 / sqrt(A));
        const double mu = (double)c + s1 / N;
        const float hi = (float)mu;
        dst[(size_t)gy * a.dpitch + gx] = make_float4(hi, (float)(mu - (double)hi), inv, 0.f);
    }
}

hipError_t launch_reduce(int dtype, const ReduceArgs& a, hipStream_t s)
{
    dim3 grid((a.Wo + 63) / 64, (a.Ho + 3) / 4, a.views);
    if (dtype == 0)
        hipLaunchKernelGGL(reduce_kernel<uint8_t>, grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(reduce_kernel<float>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_convert(int dtype, const ConvertArgs& a, hipStream_t s)
{
    dim3 grid((a.W + 63) / 64, (a.H + 3) / 4, 1);
    if (dtype == 0)
        hipLaunchKernelGGL(convert_kernel<uint8_t>, grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(convert_kernel<float>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_stats(int dtype, const StatsArgs& a, hipStream_t s)
{
    if (a.n < 1 || a.n > ST_MAXN) return hipErrorInvalidValue;
    dim3 grid((a.W + ST_W - 1) / ST_W, (a.H + ST_H - 1) / ST_H, a.views);
    if (dtype == 0)
        hipLaunchKernelGGL(stats_kernel<uint8_t>, grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(stats_kernel<float>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace msibm
