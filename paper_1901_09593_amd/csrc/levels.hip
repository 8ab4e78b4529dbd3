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
#include "levels_impl.hpp"

namespace msibm {

template <typename T>
__global__ __launch_bounds__(256) void convert_kernel(ConvertArgs a)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= a.W || y >= a.H) return;
    a.dst[(size_t)y * a.dpitch + x] = to_f(static_cast<const T*>(a.src)[(size_t)y * a.spitch + x]);
}

// Statistics of every (level, view) segment listed in the arguments, one launch.
template <int NW>
__global__ __launch_bounds__(256) void stats_kernel(StatsArgs a)
{
    __shared__ StatsSmem sm;
    int b = blockIdx.x, sgi = 0;
    while (sgi + 1 < a.nseg && b >= a.seg[sgi + 1].tile0) ++sgi;
    const StatsSeg& g = a.seg[sgi];
    const int t = b - g.tile0;
    const int tw = (g.W + ST_W - 1) / ST_W;
    const int x0 = (t % tw) * ST_W, y0 = (t / tw) * ST_H;
    if (g.dtype == 0)
        stats_tile<uint8_t, NW>((const uint8_t*)g.src, g.H, g.W, g.spitch, g.dst, g.dpitch, a.var_eps, x0,
                                y0, sm);
    else
        stats_tile<float, NW>((const float*)g.src, g.H, g.W, g.spitch, g.dst, g.dpitch, a.var_eps, x0, y0,
                              sm);
}

// Pyramid reduce of several (pair, level) segments in one launch; a tile reads
// level k-1 of its pair (the caller's input at k = 1) and writes level k.
__global__ __launch_bounds__(256) void reduce_multi_kernel(MultiArgs a)
{
    __shared__ ReduceSmem sm;
    const Segment s = a.segs[segment_of(a.segs, a.nseg, blockIdx.x)];
    const LevelDesc* lv = a.levels + a.level_base[s.pair];
    const LevelDesc& P = lv[s.level - 1];
    const LevelDesc& L = lv[s.level];
    const int per = s.tiles_x * s.tiles_y, t = blockIdx.x - s.task0;
    const int v = t / per, tx = (t % per) % s.tiles_x, ty = (t % per) / s.tiles_x;
    ReduceArgs ra{};  // the tile's view only, so no dynamic indexing
    ra.src[0] = v ? P.img[1] : P.img[0];
    ra.dst[0] = (float*)(v ? L.img[1] : L.img[0]);
    ra.views = 1;
    ra.H = P.H;
    ra.W = P.W;
    ra.spitch = P.pitch;
    ra.Ho = L.H;
    ra.Wo = L.W;
    ra.dpitch = L.pitch;
    if (P.dtype == 0) reduce_tile<uint8_t>(ra, 0, tx, ty, sm);
    else reduce_tile<float>(ra, 0, tx, ty, sm);
}

// Window statistics of several (pair, level) segments in one launch.
template <int NW>
__global__ __launch_bounds__(256) void stats_multi_kernel(MultiArgs a)
{
    __shared__ StatsSmem sm;
    const Segment s = a.segs[segment_of(a.segs, a.nseg, blockIdx.x)];
    const LevelDesc& L = a.levels[a.level_base[s.pair] + s.level];
    const int per = s.tiles_x * s.tiles_y, t = blockIdx.x - s.task0;
    const int v = t / per, x0 = ((t % per) % s.tiles_x) * ST_W, y0 = ((t % per) / s.tiles_x) * ST_H;
    if (L.dtype == 0)
        stats_tile<uint8_t, NW>((const uint8_t*)L.img[v], L.H, L.W, L.pitch, L.stat[v], L.W, a.var_eps, x0, y0,
                                sm);
    else
        stats_tile<float, NW>((const float*)L.img[v], L.H, L.W, L.pitch, L.stat[v], L.W, a.var_eps, x0, y0,
                              sm);
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

hipError_t launch_reduce_multi(const MultiArgs& a, int blocks, hipStream_t s)
{
    if (blocks < 1 || a.nseg < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(reduce_multi_kernel, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_stats_multi(int n, const MultiArgs& a, int blocks, hipStream_t s)
{
    if (blocks < 1 || a.nseg < 1) return hipErrorInvalidValue;
    switch (n) {
        case 1: hipLaunchKernelGGL(stats_multi_kernel<1>, dim3(blocks), dim3(256), 0, s, a); break;
        case 2: hipLaunchKernelGGL(stats_multi_kernel<2>, dim3(blocks), dim3(256), 0, s, a); break;
        case 3: hipLaunchKernelGGL(stats_multi_kernel<3>, dim3(blocks), dim3(256), 0, s, a); break;
        case 4: hipLaunchKernelGGL(stats_multi_kernel<4>, dim3(blocks), dim3(256), 0, s, a); break;
        case 5: hipLaunchKernelGGL(stats_multi_kernel<5>, dim3(blocks), dim3(256), 0, s, a); break;
        case 6: hipLaunchKernelGGL(stats_multi_kernel<6>, dim3(blocks), dim3(256), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace msibm
