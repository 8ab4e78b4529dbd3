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
//   variance A/N is at most var_eps (flat window).  Separable running box sums
//   accumulated in double precision, so the flat test and A match the
//   double-precision definition; every level and view of a pair in one launch.
//   HBM-bound: 1 or 4 bytes read and 16 bytes written per pixel.
#include "common.hpp"

namespace msibm {

constexpr int RD_W = 64, RD_H = 16;                 // output tile
constexpr int RD_IW = 2 * RD_W + 3, RD_IH = 2 * RD_H + 3;  // input region (5-tap halo)

// One 16 x 64 output tile of one view: the input region is staged in LDS once,
// the horizontal 5-tap sums are taken at even columns, then the vertical ones at
// even rows.  Same arithmetic order as a direct evaluation: h = sum_b w_b x,
// out = 2^-8 sum_t w_t h_t with integer weights, all partial sums exact for
// uint8 input up to level 2.
template <typename T>
__global__ __launch_bounds__(256) void reduce_kernel(ReduceArgs a)
{
    __shared__ float in[RD_IH][RD_IW + 1];
    __shared__ float hs[RD_IH][RD_W + 1];
    const int view = blockIdx.z;
    const T* __restrict__ src = static_cast<const T*>(a.src[view]);
    float* __restrict__ dst = a.dst[view];
    const int ox0 = blockIdx.x * RD_W, oy0 = blockIdx.y * RD_H;
    const int ix0 = 2 * ox0 - 2, iy0 = 2 * oy0 - 2;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // stage: every load of the thread issued before the LDS stores
    constexpr int RI = (RD_IH + 3) / 4, CI = (RD_IW + 63) / 64;
    T v[RI][CI];
#pragma unroll
    for (int ri = 0; ri < RI; ++ri) {
        const int rr = wave + 4 * ri;
        const T* srow = src + (size_t)clampi(iy0 + rr, 0, a.H - 1) * a.spitch;
#pragma unroll
        for (int ci = 0; ci < CI; ++ci) {
            const int cc = lane + 64 * ci;
            if (rr < RD_IH && cc < RD_IW) v[ri][ci] = srow[clampi(ix0 + cc, 0, a.W - 1)];
        }
    }
#pragma unroll
    for (int ri = 0; ri < RI; ++ri) {
        const int rr = wave + 4 * ri;
#pragma unroll
        for (int ci = 0; ci < CI; ++ci) {
            const int cc = lane + 64 * ci;
            if (rr < RD_IH && cc < RD_IW) in[rr][cc] = to_f(v[ri][ci]);
        }
    }
    __syncthreads();
    const float w[5] = {1.f, 4.f, 6.f, 4.f, 1.f};
    for (int rr = wave; rr < RD_IH; rr += 4) {
        float h = 0.f;
#pragma unroll
        for (int b = 0; b < 5; ++b) h = fmaf(w[b], in[rr][2 * lane + b], h);
        hs[rr][lane] = h;
    }
    __syncthreads();
    const int x = ox0 + lane;
#pragma unroll
    for (int k = 0; k < RD_H / 4; ++k) {
        const int oy = wave + 4 * k, y = oy0 + oy;
        float acc = 0.f;
#pragma unroll
        for (int t = 0; t < 5; ++t) acc = fmaf(w[t], hs[2 * oy + t][lane], acc);
        if (x < a.Wo && y < a.Ho) dst[(size_t)y * a.dpitch + x] = acc * (1.f / 256.f);
    }
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
constexpr int ST_SEG = 8;                               // outputs per thread, horizontal pass
constexpr int ST_RH = ST_H + 2 * ST_MAXN;               // 28 rows with halo

// One 16 x 64 tile of one view of one level.  Horizontal window sums of x and x^2
// in double precision (running sums over 8 outputs per thread, read straight from
// global memory), then vertical running sums over 4 outputs per thread.  Values
// are centred on the tile's first pixel before squaring, so the sums stay small.
template <typename T, int NW>
__device__ __forceinline__ void stats_tile(const T* __restrict__ src, int H, int W, int spitch,
                                           float4* __restrict__ dst, int dpitch, double var_eps,
                                           int x0, int y0, double (*h1)[ST_W], double (*h2)[ST_W])
{
    constexpr int n = NW, wn = 2 * NW + 1, rows = ST_H + 2 * NW;
    const double c = (double)to_f(src[(size_t)min(y0, H - 1) * spitch + min(x0, W - 1)]);
    // horizontal pass: thread = (row, 8-column segment)
    {
        const int seg = threadIdx.x & 7, rr = threadIdx.x >> 3;  // 32 rows x 8 segments
        if (rr < rows) {
            const T* srow = src + (size_t)clampi(y0 - n + rr, 0, H - 1) * spitch;
            const int cx = x0 + ST_SEG * seg - n;
            float f[ST_SEG + 2 * NW];
#pragma unroll
            for (int t = 0; t < ST_SEG + 2 * NW; ++t) f[t] = to_f(srow[clampi(cx + t, 0, W - 1)]);
            double v[ST_SEG + 2 * NW];
#pragma unroll
            for (int t = 0; t < ST_SEG + 2 * NW; ++t) v[t] = (double)f[t] - c;
            double s1 = 0.0, s2 = 0.0;
#pragma unroll
            for (int t = 0; t < wn; ++t) {
                s1 += v[t];
                s2 = fma(v[t], v[t], s2);
            }
            h1[rr][ST_SEG * seg] = s1;
            h2[rr][ST_SEG * seg] = s2;
#pragma unroll
            for (int k = 1; k < ST_SEG; ++k) {
                const double add = v[k - 1 + wn], drop = v[k - 1];
                s1 += add - drop;
                s2 += fma(add, add, -drop * drop);
                h1[rr][ST_SEG * seg + k] = s1;
                h2[rr][ST_SEG * seg + k] = s2;
            }
        }
    }
    __syncthreads();
    // vertical pass: thread = (column, 4-row segment)
    const int col = threadIdx.x & 63, rs = (threadIdx.x >> 6) * 4;
    const double N = (double)(wn * wn), invN = 1.0 / N;
    double s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int t = 0; t < wn; ++t) {
        s1 += h1[rs + t][col];
        s2 += h2[rs + t][col];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (k > 0) {
            s1 += h1[rs + k - 1 + wn][col] - h1[rs + k - 1][col];
            s2 += h2[rs + k - 1 + wn][col] - h2[rs + k - 1][col];
        }
        const int gy = y0 + rs + k, gx = x0 + col;
        if (gy < H && gx < W) {
            const double A = s2 - s1 * s1 * invN;
            const float inv = (A <= N * var_eps) ? 0.f : rsqrtf((float)A);
            const double mu = c + s1 * invN;
            const float hi = (float)mu;
            dst[(size_t)gy * dpitch + gx] = make_float4(hi, (float)(mu - (double)hi), inv, 0.f);
        }
    }
}

// Statistics of every (level, view) segment listed in the arguments, one launch.
template <int NW>
__global__ __launch_bounds__(256) void stats_kernel(StatsArgs a)
{
    __shared__ double h1[ST_RH][ST_W];
    __shared__ double h2[ST_RH][ST_W];
    int b = blockIdx.x, sgi = 0;
    while (sgi + 1 < a.nseg && b >= a.seg[sgi + 1].tile0) ++sgi;
    const StatsSeg& g = a.seg[sgi];
    const int t = b - g.tile0;
    const int tw = (g.W + ST_W - 1) / ST_W;
    const int x0 = (t % tw) * ST_W, y0 = (t / tw) * ST_H;
    if (g.dtype == 0)
        stats_tile<uint8_t, NW>((const uint8_t*)g.src, g.H, g.W, g.spitch, g.dst, g.dpitch, a.var_eps, x0,
                                y0, h1, h2);
    else
        stats_tile<float, NW>((const float*)g.src, g.H, g.W, g.spitch, g.dst, g.dpitch, a.var_eps, x0, y0,
                              h1, h2);
}

__global__ __launch_bounds__(256) void zero_kernel(float* a, float* b, size_t count)
{
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (size_t)gridDim.x * 256) {
        a[i] = 0.f;
        if (b) b[i] = 0.f;
    }
}

hipError_t launch_zero(float* a, float* b, size_t count, hipStream_t s)
{
    const size_t blocks = (count + 255) / 256;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256), 0, s, a, b,
                       count);
    return hipGetLastError();
}

int stats_tiles(int H, int W) { return ((W + ST_W - 1) / ST_W) * ((H + ST_H - 1) / ST_H); }

hipError_t launch_reduce(int dtype, const ReduceArgs& a, hipStream_t s)
{
    dim3 grid((a.Wo + RD_W - 1) / RD_W, (a.Ho + RD_H - 1) / RD_H, a.views);
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

hipError_t launch_stats(StatsArgs a, hipStream_t s)
{
    if (a.n < 1 || a.n > ST_MAXN || a.nseg < 1 || a.nseg > STATS_MAX_SEG) return hipErrorInvalidValue;
    int tiles = 0;
    for (int i = 0; i < a.nseg; ++i) {
        a.seg[i].tile0 = tiles;
        tiles += stats_tiles(a.seg[i].H, a.seg[i].W);
    }
    switch (a.n) {
        case 1: hipLaunchKernelGGL(stats_kernel<1>, dim3(tiles), dim3(256), 0, s, a); break;
        case 2: hipLaunchKernelGGL(stats_kernel<2>, dim3(tiles), dim3(256), 0, s, a); break;
        case 3: hipLaunchKernelGGL(stats_kernel<3>, dim3(tiles), dim3(256), 0, s, a); break;
        case 4: hipLaunchKernelGGL(stats_kernel<4>, dim3(tiles), dim3(256), 0, s, a); break;
        case 5: hipLaunchKernelGGL(stats_kernel<5>, dim3(tiles), dim3(256), 0, s, a); break;
        case 6: hipLaunchKernelGGL(stats_kernel<6>, dim3(tiles), dim3(256), 0, s, a); break;
    }
    return hipGetLastError();
}

}  // namespace msibm
