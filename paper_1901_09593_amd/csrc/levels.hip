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
//   HBM-bound: 1 or 4 bytes read and 12 bytes written per pixel.
#include <type_traits>

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

// Statistics tile b of a list of segment pairs (the two views of one level);
// a tile covers both views.
template <int NW>
__device__ __forceinline__ void stats_block(const StatsArgs& a, int b, StatsSmem<NW>& sm)
{
    int sgi = 0;
    while (sgi + 2 < a.nseg && b >= a.seg[sgi + 2].tile0) sgi += 2;
    const StatsSeg& g = a.seg[sgi];
    const StatsSeg& h = a.seg[sgi + 1];
    const int t = b - g.tile0;
    const int tw = (g.W + ST_W - 1) / ST_W;
    const int x0 = (t % tw) * ST_W, y0 = (t / tw) * stats_tile_h(g.dtype);
    if (g.dtype == 0)
        stats_tile_u8<NW>((const uint8_t*)g.src, g.dst, (const uint8_t*)h.src, h.dst, g.H, g.W, g.spitch, g.dpitch,
                          a.var_eps, x0, y0, sm.i);
    else
        stats_tile<float, NW>((const float*)g.src, g.dst, (const float*)h.src, h.dst, g.H, g.W, g.spitch,
                              g.dpitch, a.var_eps, x0, y0, sm);
}

// Statistics of every level listed in the arguments, one launch.
template <int NW>
__global__ __launch_bounds__(256) void stats_kernel(StatsArgs a)
{
    __shared__ StatsSmem<NW> sm;
    stats_block<NW>(a, blockIdx.x, sm);
}

// Two or three pyramid steps of both views in one launch (grid: last-level
// tiles x 2 views); the small levels' reduces alone would each be a launch
// whose few workgroups leave most of the chip idle.
template <typename T, int S>
__global__ __launch_bounds__(TW_THREADS) void tower_kernel(TowerArgs a)
{
    __shared__ TowerSmem<T, S> sm;
    tower_tile<T, S>(a, blockIdx.z, blockIdx.x, blockIdx.y, sm);
}

// Tile t of a reduce segment: reads level k-1 of its pair (the caller's input
// at k = 1, also where level 0 is matched on its blurred copy) and writes
// level k of one view.
template <typename S>
__device__ __forceinline__ void reduce_seg_tile(const MultiArgs& a, const Segment& s, int t, ReduceSmemT<S>& sm)
{
    const LevelDesc* lv = a.levels + a.level_base[s.pair];
    const LevelDesc& P = lv[s.level - 1];
    const LevelDesc& L = lv[s.level];
    const int per = s.tiles_x * s.tiles_y;
    const int v = t / per, tx = (t % per) % s.tiles_x, ty = (t % per) / s.tiles_x;
    ReduceArgs ra{};  // the tile's view only, so no dynamic indexing
    const bool own = P.src[0] != nullptr;
    ra.src[0] = own ? (v ? P.src[1] : P.src[0]) : (v ? P.img[1] : P.img[0]);
    ra.dst[0] = (float*)(v ? L.img[1] : L.img[0]);
    ra.views = 1;
    ra.H = P.H;
    ra.W = P.W;
    ra.spitch = own ? P.spitch : P.pitch;
    ra.Ho = L.H;
    ra.Wo = L.W;
    ra.dpitch = L.pitch;
    if constexpr (std::is_same<S, uint8_t>::value) {
        reduce_tile<uint8_t, uint8_t>(ra, 0, tx, ty, sm);  // the launch holds uint8 sources only
    } else {
        if ((own ? P.sdtype : P.dtype) == 0) reduce_tile<uint8_t, float>(ra, 0, tx, ty, sm);
        else reduce_tile<float, float>(ra, 0, tx, ty, sm);
    }
}

// Tile t of a statistics segment: both views of one level of its pair.
template <int NW>
__device__ __forceinline__ void stats_seg_tile(const MultiArgs& a, const Segment& s, int t, StatsSmem<NW>& sm)
{
    const LevelDesc& L = a.levels[a.level_base[s.pair] + s.level];
    const int x0 = (t % s.tiles_x) * ST_W, y0 = (t / s.tiles_x) * stats_tile_h(L.dtype);
    if (L.dtype == 0)
        stats_tile_u8<NW>((const uint8_t*)L.img[0], L.stat[0], (const uint8_t*)L.img[1], L.stat[1], L.H, L.W,
                          L.pitch, L.W, a.var_eps, x0, y0, sm.i);
    else
        stats_tile<float, NW>((const float*)L.img[0], L.stat[0], (const float*)L.img[1], L.stat[1], L.H, L.W,
                              L.pitch, L.W, a.var_eps, x0, y0, sm);
}

// Window statistics of several (pair, level) segments in one launch.
template <int NW>
__global__ __launch_bounds__(256) void stats_multi_kernel(MultiArgs a)
{
    __shared__ StatsSmem<NW> sm;
    const int b = xcd_task(blockIdx.x);
    const Segment s = a.segs[segment_of(a.segs, a.nseg, b)];
    stats_seg_tile<NW>(a, s, b - s.task0, sm);
}

// Statistics and reduce segments side by side in one launch (one pyramid step
// of every pair of a batch).
template <int NW>
__global__ __launch_bounds__(256) void levels_multi_kernel(MultiArgs a)
{
    __shared__ union {
        StatsSmem<NW> st;
        ReduceSmem rd;
    } sm;
    const int b = xcd_task(blockIdx.x);
    const Segment s = a.segs[segment_of(a.segs, a.nseg, b)];
    if (s.type == SEG_STATS) stats_seg_tile<NW>(a, s, b - s.task0, sm.st);
    else reduce_seg_tile(a, s, b - s.task0, sm.rd);
}

// The same for a pyramid step whose statistics and reduce tiles all read
// uint8 levels (level 0 of uint8 pairs): integer statistics only and the
// reduce's input staged as bytes, so the LDS (and the registers of the float
// paths) no longer limit how many workgroups share a CU.
constexpr int LEVELS_U8_MIN_BLOCKS = 7;
template <int NW>
__global__ __launch_bounds__(256, LEVELS_U8_MIN_BLOCKS) void levels_u8_multi_kernel(MultiArgs a)
{
    __shared__ union {
        StatsSmemI<NW> st;
        ReduceSmemU8 rd;
    } sm;
    const int b = xcd_task(blockIdx.x);
    const Segment s = a.segs[segment_of(a.segs, a.nseg, b)];
    const int t = b - s.task0;
    if (s.type == SEG_STATS) {
        const LevelDesc& L = a.levels[a.level_base[s.pair] + s.level];
        const int x0 = (t % s.tiles_x) * ST_W, y0 = (t / s.tiles_x) * SU_H;
        stats_tile_u8<NW>((const uint8_t*)L.img[0], L.stat[0], (const uint8_t*)L.img[1], L.stat[1], L.H, L.W,
                          L.pitch, L.W, a.var_eps, x0, y0, sm.st);
    } else {
        reduce_seg_tile(a, s, t, sm.rd);
    }
}

__global__ __launch_bounds__(256) void zero_kernel(float* a, float* b, size_t count)
{
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (size_t)gridDim.x * 256) {
        a[i] = 0.f;
        if (b) b[i] = 0.f;
    }
}

__global__ __launch_bounds__(256) void fill_kernel(float* a, float v, size_t count)
{
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (size_t)gridDim.x * 256) a[i] = v;
}

hipError_t launch_fill(float* a, float v, size_t count, hipStream_t s)
{
    const size_t blocks = (count + 255) / 256;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256), 0, s, a, v, count);
    return hipGetLastError();
}

hipError_t launch_zero(float* a, float* b, size_t count, hipStream_t s)
{
    const size_t blocks = (count + 255) / 256;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256), 0, s, a, b,
                       count);
    return hipGetLastError();
}

int stats_tiles(int H, int W, int dtype)
{
    const int th = stats_tile_h(dtype);
    return ((W + ST_W - 1) / ST_W) * ((H + th - 1) / th);
}

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

// Checks the segment pairs and numbers their tiles; returns the tile count, or
// -1 when the list is invalid.
static int number_stats_tiles(StatsArgs& a)
{
    if (a.n < 1 || a.n > ST_MAXN || a.nseg < 2 || a.nseg > STATS_MAX_SEG || (a.nseg & 1)) return -1;
    int tiles = 0;
    for (int i = 0; i < a.nseg; i += 2) {
        const StatsSeg& g = a.seg[i];
        const StatsSeg& h = a.seg[i + 1];
        if (g.H != h.H || g.W != h.W || g.dtype != h.dtype || g.spitch != h.spitch || g.dpitch != h.dpitch)
            return -1;  // a tile covers both views of one level
        a.seg[i].tile0 = a.seg[i + 1].tile0 = tiles;
        tiles += stats_tiles(g.H, g.W, g.dtype);
    }
    return tiles;
}

template <typename T>
__global__ __launch_bounds__(256) void blur_kernel(BlurArgs a)
{
    __shared__ BlurSmem sm;
    const int v = blockIdx.z;
    blur_tile<T>(static_cast<const T*>(v ? a.src[1] : a.src[0]), v ? a.dst[1] : a.dst[0], a.H, a.W, a.spitch,
                 a.dpitch, blockIdx.x, blockIdx.y, sm);
}

hipError_t launch_blur(int dtype, const BlurArgs& a, hipStream_t s)
{
    dim3 grid((a.W + BL_W - 1) / BL_W, (a.H + BL_H - 1) / BL_H, 2);
    if (dtype == 0) hipLaunchKernelGGL(blur_kernel<uint8_t>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(blur_kernel<float>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// Selective median filter (Eq. 10), one pixel per thread.  A filtered pixel
// gathers the disparities of the good pixels of its 5x5 patch (32767 for the
// others), sorts the 32 values with a bitonic network in registers and takes
// the lower median of the good ones.
__device__ __forceinline__ void cswap(int& a, int& b)
{
    const int lo = min(a, b), hi = max(a, b);
    a = lo;
    b = hi;
}

// Selective median (Eq. 10), one 64 x 4 tile per workgroup (one pixel per
// thread: the small levels need the workgroups).  The tile and its
// 2-pixel ring are staged in LDS once as sort keys: a neighbour's disparity
// where it lies in the image and its cost exceeds alpha (a good pixel), else
// INT_MAX.  A filtered pixel sorts its 25 keys (with 7 more INT_MAX, a 32-key
// bitonic network; comparators against the constant INT_MAX padding fold away
// at compile time) and takes the lower median of the good ones, the keys below
// INT_MAX; disparities are int16, so no disparity equals INT_MAX.
__device__ __forceinline__ void median_tile(const MedianArgs& a, int bx, int by)
{
    __shared__ int key[MD_H + 4][MD_W + 4];
    __shared__ int any_filtered;
    const int x0 = bx * MD_W, y0 = by * MD_H;
    const int c = threadIdx.x & 63, r0 = threadIdx.x >> 6;  // the thread's pixel
    if (threadIdx.x == 0) any_filtered = 0;
    for (int idx = threadIdx.x; idx < (MD_H + 4) * (MD_W + 4); idx += 256) {
        const int rr = idx / (MD_W + 4), cc = idx - rr * (MD_W + 4);
        const int y = y0 - 2 + rr, x = x0 - 2 + cc;
        int k = INT_MAX;
        if (y >= 0 && y < a.H && x >= 0 && x < a.W && (double)a.cost[(size_t)y * a.cpitch + x] > a.alpha)
            k = a.d_in[(size_t)y * a.ipitch + x];
        key[rr][cc] = k;
    }
    __syncthreads();
    constexpr int Q = MD_H / 4;  // pixels per thread
    int dv[Q];
    bool filt[Q];
    bool some = false;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int i = y0 + r0 + q, j = x0 + c;
        filt[q] = false;
        dv[q] = 0;
        if (i < a.H && j < a.W) {
            dv[q] = a.d_in[(size_t)i * a.ipitch + j];
            filt[q] = !((double)a.cost[(size_t)i * a.cpitch + j] > a.alpha);
        }
        some = some || filt[q];
    }
    if (some) any_filtered = 1;
    __syncthreads();
    if (!any_filtered) {
        // no pixel of the tile is filtered: copy
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int i = y0 + r0 + q, j = x0 + c;
            if (i < a.H && j < a.W) a.d_out[(size_t)i * a.opitch + j] = (int16_t)dv[q];
        }
        return;
    }
#pragma unroll 1
    for (int q = 0; q < Q; ++q) {
        const int i = y0 + r0 + q, j = x0 + c;
        if (i >= a.H || j >= a.W) continue;
        int out = dv[q];
        if (filt[q]) {
            int v[32];
#pragma unroll
            for (int t = 0; t < 25; ++t) v[t] = key[r0 + q + t / 5][c + t % 5];
#pragma unroll
            for (int t = 25; t < 32; ++t) v[t] = INT_MAX;
#pragma unroll
            for (int k = 2; k <= 32; k <<= 1)
#pragma unroll
                for (int jj = k >> 1; jj > 0; jj >>= 1)
#pragma unroll
                    for (int t = 0; t < 32; ++t) {
                        const int l = t ^ jj;
                        if (l > t) {
                            if ((t & k) == 0) cswap(v[t], v[l]);
                            else cswap(v[l], v[t]);
                        }
                    }
            int m = 0;
#pragma unroll
            for (int t = 0; t < 25; ++t) m += v[t] != INT_MAX;
            const int want = (m - 1) / 2;
            int med = out;
#pragma unroll
            for (int t = 0; t < 13; ++t) med = (t == want) ? v[t] : med;
            if (m > 0) out = med;
        }
        a.d_out[(size_t)i * a.opitch + j] = (int16_t)out;
    }
}

__global__ __launch_bounds__(256) void median_kernel(MedianArgs a) { median_tile(a, blockIdx.x, blockIdx.y); }

// The median of several (pair, level) maps in one launch.
__global__ __launch_bounds__(256) void median_multi_kernel(MultiArgs a)
{
    const Segment s = a.segs[segment_of(a.segs, a.nseg, blockIdx.x)];
    const LevelDesc& L = a.levels[a.level_base[s.pair] + s.level];
    const MedianArgs m{L.raw, L.mcost, L.map, L.H, L.W, L.W, L.W, L.W, a.median_alpha};
    const int t = blockIdx.x - s.task0;
    median_tile(m, t % s.tiles_x, t / s.tiles_x);
}

// Weight with which coarse row (or column) y of a reduce step reads fine row p:
// the binomial taps a with clamp(2y + a) = p, summed (several taps clamp to the
// same edge row).
__device__ __forceinline__ float adj_weight(int p, int y, int H)
{
    const float w[5] = {1.f / 16, 4.f / 16, 6.f / 16, 4.f / 16, 1.f / 16};
    float s = 0.f;
#pragma unroll
    for (int a = -2; a <= 2; ++a) s += (clampi(2 * y + a, 0, H - 1) == p) ? w[a + 2] : 0.f;
    return s;
}

// out(p, q) += sum over the coarse pixels that read fine pixel (p, q) of their
// weight times g: at most 3 coarse rows (y in [ceil((p-2)/2), floor((p+2)/2)])
// and 3 coarse columns.  One thread per fine pixel, no atomics.
__global__ __launch_bounds__(256) void adjoint_kernel(AdjArgs a)
{
    const int q = blockIdx.x * 64 + (threadIdx.x & 63), p = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int v = blockIdx.z;
    if (p >= a.H || q >= a.W) return;
    const int y0 = max(0, (p - 1) / 2), y1 = min(a.Hc - 1, (p + 2) / 2);
    const int x0 = max(0, (q - 1) / 2), x1 = min(a.Wc - 1, (q + 2) / 2);
    const float* g = a.g[v];
    float s = 0.f;
    for (int y = y0; y <= y1; ++y) {
        const float wy = adj_weight(p, y, a.H);
        float r = 0.f;
        for (int x = x0; x <= x1; ++x) r += adj_weight(q, x, a.W) * g[(size_t)y * a.gpitch + x];
        s += wy * r;
    }
    float* o = a.out[v] + (size_t)p * a.opitch + q;
    *o += s;
}

hipError_t launch_adjoint(const AdjArgs& a, hipStream_t s)
{
    if (a.views < 1 || a.views > 2 || a.Hc != (a.H + 1) / 2 || a.Wc != (a.W + 1) / 2) return hipErrorInvalidValue;
    dim3 grid((a.W + 63) / 64, (a.H + 3) / 4, a.views);
    hipLaunchKernelGGL(adjoint_kernel, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_median_multi(const MultiArgs& a, int blocks, hipStream_t s)
{
    if (blocks < 1 || a.nseg < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(median_multi_kernel, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_median(const MedianArgs& a, hipStream_t s)
{
    dim3 grid((a.W + MD_W - 1) / MD_W, (a.H + MD_H - 1) / MD_H, 1);
    hipLaunchKernelGGL(median_kernel, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_tower(int dtype, const TowerArgs& a, hipStream_t s)
{
    if (a.steps < 2 || a.steps > TW_MAXS) return hipErrorInvalidValue;
    const int Hl = a.H[a.steps - 1], Wl = a.W[a.steps - 1];
    dim3 grid((Wl + TW_FW - 1) / TW_FW, (Hl + TW_FH - 1) / TW_FH, 2);
    if (dtype == 0) {
        if (a.steps == 2) hipLaunchKernelGGL((tower_kernel<uint8_t, 2>), grid, dim3(TW_THREADS), 0, s, a);
        else hipLaunchKernelGGL((tower_kernel<uint8_t, 3>), grid, dim3(TW_THREADS), 0, s, a);
    } else {
        if (a.steps == 2) hipLaunchKernelGGL((tower_kernel<float, 2>), grid, dim3(TW_THREADS), 0, s, a);
        else hipLaunchKernelGGL((tower_kernel<float, 3>), grid, dim3(TW_THREADS), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_stats(StatsArgs a, hipStream_t s)
{
    const int tiles = number_stats_tiles(a);
    if (tiles < 0) return hipErrorInvalidValue;
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

hipError_t launch_levels_multi(int n, int dtype, const MultiArgs& a, int blocks, hipStream_t s)
{
    if (blocks < 1 || a.nseg < 1) return hipErrorInvalidValue;
    if (dtype == MSIBM_U8) {
        switch (n) {
            case 1: hipLaunchKernelGGL(levels_u8_multi_kernel<1>, dim3(blocks), dim3(256), 0, s, a); break;
            case 2: hipLaunchKernelGGL(levels_u8_multi_kernel<2>, dim3(blocks), dim3(256), 0, s, a); break;
            case 3: hipLaunchKernelGGL(levels_u8_multi_kernel<3>, dim3(blocks), dim3(256), 0, s, a); break;
            case 4: hipLaunchKernelGGL(levels_u8_multi_kernel<4>, dim3(blocks), dim3(256), 0, s, a); break;
            case 5: hipLaunchKernelGGL(levels_u8_multi_kernel<5>, dim3(blocks), dim3(256), 0, s, a); break;
            case 6: hipLaunchKernelGGL(levels_u8_multi_kernel<6>, dim3(blocks), dim3(256), 0, s, a); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (n) {
        case 1: hipLaunchKernelGGL(levels_multi_kernel<1>, dim3(blocks), dim3(256), 0, s, a); break;
        case 2: hipLaunchKernelGGL(levels_multi_kernel<2>, dim3(blocks), dim3(256), 0, s, a); break;
        case 3: hipLaunchKernelGGL(levels_multi_kernel<3>, dim3(blocks), dim3(256), 0, s, a); break;
        case 4: hipLaunchKernelGGL(levels_multi_kernel<4>, dim3(blocks), dim3(256), 0, s, a); break;
        case 5: hipLaunchKernelGGL(levels_multi_kernel<5>, dim3(blocks), dim3(256), 0, s, a); break;
        case 6: hipLaunchKernelGGL(levels_multi_kernel<6>, dim3(blocks), dim3(256), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
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
