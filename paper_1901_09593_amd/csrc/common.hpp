// Shared definitions of the gfx950 kernels and the host library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "msibm.h"

namespace msibm {

// ---------------------------------------------------------------- tiling
// The matching kernels give each thread a 2x2 block of pixels.  Pixels of one
// block share the propagated prior (nearest-neighbour upsampling maps the 2x2
// block onto one coarser pixel), so they share one window of candidate slots,
// and their four windows share most of their row products.
constexpr int MATCH_TX = 64;               // threads across a workgroup (one wave)
constexpr int MATCH_TY = 4;                // waves per workgroup
constexpr int MATCH_THREADS = MATCH_TX * MATCH_TY;
constexpr int TILE_W = 2 * MATCH_TX;       // 128 pixel columns per workgroup
constexpr int TILE_H1 = 2 * MATCH_TY;      // 8 pixel rows per block row of the workgroup
constexpr int FULL_NC = 8;                 // slots per step of a full search

enum MatchMode { MODE_FULL = 0, MODE_REFINE = 1, MODE_SOFT = 2 };

// Per-pixel window statistics of one view at one level (12 bytes): x + y = the
// window mean as an unevaluated sum of two floats (x = the mean rounded to
// float, y = the rounding remainder), z = 1/sqrt(sum of squared deviations) or 0
// for a flat window.
struct WinStat {
    float x, y, z;
};

// Window statistics of a uint8 level, written in place of WinStat (the same
// buffers, 8 bytes per pixel at the same row pitch in records): the window sum
// S1 (an integer below 2^24, exact in float) and 1/sqrt(A), 0 for a flat
// window.  With uint8 values every window sum of products is an exact
// integer too, so the cross term is formed exactly as C N = N S - S1_l S1_r.
struct WinStatU8 {
    float s1, z;
};

struct MatchArgs {
    const void* L;
    const void* R;
    int H, W, pitch;          // level image size and row pitch (elements)
    const WinStat* statL;      // H x W, row pitch spitch
    const WinStat* statR;
    int spitch;
    int Dk;                   // candidates at this level
    const int16_t* prior;     // level k+1 map (refine / soft), else unused
    int Hc, Wc, ppitch;
    int r;                    // refine or soft radius
    int16_t* d_out;           // H x W, row pitch opitch
    float* c_out;             // nullable
    float* soft_out;          // soft mode only
    int opitch;
    float inv_tau;
    int variant;              // VARIANT_* bits (kernel shape chosen by the tuner)
    float* costvol;           // nullable: H x W x Dk scores of every scored candidate
};

// Kernel shape variants of the matching kernel (bits of MatchArgs::variant).
constexpr int VARIANT_STATS_LDS = 1;  // right statistics staged in LDS (full search only)
constexpr int VARIANT_XCD = 2;        // XCD-aware tile order
constexpr int VARIANT_SPLIT = 4;      // full / restricted search: 2-row tiles, the 4 waves split the candidates
constexpr int VARIANT_FIXW = 8;       // restricted search: stage the whole candidate range up front
constexpr int VARIANT_SHORT = 16;     // short right chunk: 48 (full) or 128 (restricted) candidates
constexpr int VARIANT_TALL = 32;      // 16-row tiles of 8 waves (not with the candidate split)
constexpr int VARIANT_MASK = 63;

// Tile of block b in a grid of gx x gy tiles.  The hardware deals consecutive
// workgroups round-robin to the 8 XCDs, each with its own L2; the XCD-aware
// order gives every XCD one contiguous, row-major run of tiles, so neighbouring
// tiles (which share window halos) meet in the same L2.
__device__ __forceinline__ void tile_of(int variant, int* bx, int* by)
{
    if (!(variant & VARIANT_XCD)) return;
    const int gx = gridDim.x, total = gx * gridDim.y;
    const int b = *by * gx + *bx, xcd = b & 7, k = b >> 3;
    const int per = total >> 3, rem = total & 7;
    const int t = xcd * per + min(xcd, rem) + k;
    *bx = t % gx;
    *by = t / gx;
}

struct ReduceArgs {
    const void* src[2];
    float* dst[2];
    int views;                // 1 or 2 (grid z)
    int H, W, spitch;         // source level
    int Ho, Wo, dpitch;       // destination level
};

// One (level, view) image whose window statistics a stats launch computes.
struct StatsSeg {
    const void* src;
    WinStat* dst;
    int dtype;                // MSIBM_U8 / MSIBM_F32 element type of src
    int H, W, spitch, dpitch;
    int tile0;                // first tile index (filled by the launcher)
};
constexpr int STATS_MAX_SEG = 16;

struct StatsArgs {
    StatsSeg seg[STATS_MAX_SEG];
    int nseg;
    int n;
    double var_eps;
};

// Two or three pyramid steps in one launch: source level (the caller's input or
// a float level) to levels +1 .. +steps, both views.
// Selective median filtering of one map (Eq. 10).
struct MedianArgs {
    const int16_t* d_in;
    const float* cost;
    int16_t* d_out;
    int H, W, ipitch, cpitch, opitch;
    double alpha;
};

// Confidence gating of one level (Eqs. 5-9), in place on its map d and cost c.
// Full-search mode: pixels whose bicubic-upsampled coarser cost is at most
// `thresh` (beta) take the full search.  Re-pick mode: pixels whose cost is at
// most `thresh` (alpha) take the argmax of the 5x5-averaged scores.  Fused
// mode: both, the full search where the doubled cost is at most `thresh2`
// (beta), then the re-pick where the resulting cost is at most `thresh`.
enum GateMode { GATE_MODE_FULL = 0, GATE_MODE_REPICK = 1, GATE_MODE_FUSED = 2 };
struct GateArgs {
    const void* L;
    const void* R;
    int pitch;                  // image row pitch (elements)
    int H, W, Dk;
    const WinStat* statL;
    const WinStat* statR;
    int spitch;
    int16_t* d;
    float* c;
    int opitch;
    const float* ccost;         // coarser level's cost (full-search mode)
    int Hc, Wc, cpitch;
    double thresh;
    double thresh2;
};

// Adjoint of one pyramid step for up to two views: out (fine, H x W) +=
// reduce^T(g) (coarse, ceil(H/2) x ceil(W/2)).
struct AdjArgs {
    const float* g[2];
    float* out[2];
    int views;
    int Hc, Wc, gpitch;
    int H, W, opitch;
};

// Full-resolution binomial blur of both views (the pre-blur variant's level 0).
struct BlurArgs {
    const void* src[2];
    float* dst[2];
    int H, W, spitch, dpitch;
};

constexpr int TW_MAXS = 3;
struct TowerArgs {
    const void* src[2];
    float* dst[TW_MAXS][2];   // level +1+j of each view (float, pitch W[j])
    int Hs, Ws, spitch;       // source level
    int H[TW_MAXS], W[TW_MAXS];  // levels +1 .. +steps
    int steps;                // 2 or 3
};

struct ConvertArgs {
    const void* src;
    float* dst;
    int H, W, spitch, dpitch;
};

// ---------------------------------------------------------------- batches
// The batched forward describes its work as segments, one per (pair, stage,
// level); a launch covers the tiles of several segments of one stage.

enum SegType {
    SEG_REDUCE = 0, SEG_STATS = 1, SEG_FULL = 2, SEG_REFINE = 3, SEG_SOFT = 4, SEG_ZERO = 5, SEG_BACKWARD = 6,
    SEG_MEDIAN = 7, SEG_GATE = 8, SEG_COUNT = 9
};

struct BackArgs;

// One level of one pair.
struct LevelDesc {
    const void* img[2];   // level image of both views (level 0: the caller's input)
    int pitch, H, W;
    WinStat* stat[2];      // window statistics, row pitch W
    int16_t* map;         // winner-take-all map, row pitch W (level 0: the caller's output)
    int16_t* raw;         // with the median: the unfiltered map the search writes (else NULL)
    float* mcost;         // with the median: the cost the search writes and the filter reads
    float* cost;          // level 0 only, nullable
    float* soft;          // level 0 only, soft mode
    int Dk;
    int dtype;            // element type of img (MSIBM_U8 / MSIBM_F32)
    // level 0 matched on another image than the pyramid is built from (the
    // pre-blur): the pyramid's source (the caller's input), else src[0] = NULL
    const void* src[2];
    int spitch, sdtype;
};

// Tiles [task0, task0 + tiles_x * tiles_y * views) of a launch belong to this
// segment; tile t is view t / (tiles_x * tiles_y) (reduce and statistics do one
// view per tile, matching reads both).
struct Segment {
    int type, pair, level;
    int tiles_x, tiles_y, views;
    int task0;
};

// Arguments of a launch over several segments: block b runs tile b - task0 of
// the last segment whose task0 <= b.
struct MultiArgs {
    const Segment* segs;      // this launch's segments, task0 ascending from 0
    int nseg;
    const LevelDesc* levels;  // a pair's levels start at levels[level_base[pair]]
    const int* level_base;
    const BackArgs* back;     // backward launches: one entry per pair
    int variant;              // matching kernel shape bits that apply per segment
    int r, rs;                // refine and soft radius
    double var_eps;
    float inv_tau;
    double median_alpha;      // median launches
    double gate_alpha, gate_beta;  // gating launches
    int fused;                // backward launches: the fused masked-L1 form
};

// Tile of the gating kernel: 8 rows by as many columns as keep the tile, its
// re-pick halo and its windows' halo within 128 columns (one column-sum lane
// per column).
constexpr int GATE_TH = 8;
constexpr int GATE_EW = 128;
__host__ __device__ constexpr int gate_tile_w(int dtype, int n, int mode)
{
    return (void)dtype, GATE_EW - 2 * n - (mode == GATE_MODE_FULL ? 0 : 4);
}

// Tile of the selective median filter.
constexpr int MD_W = 64, MD_H = 4;

// Floats a zero-fill tile clears in each gradient (256 threads x 16).
constexpr int ZERO_TILE = 4096;
// Mask bytes a loss-count workgroup sums (256 threads x 16 bytes x 16 steps).
constexpr int COUNT_TILE = 65536;

// Segment of launch block b: binary search over the launch's segment table
// (block-uniform, so it runs on the scalar unit).
__device__ __forceinline__ int segment_of(const Segment* segs, int nseg, int b)
{
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].task0 <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

// Task index of workgroup b of a multi-segment launch.  The hardware deals
// workgroups round-robin to the 8 XCDs, each with its own L2; here the k-th
// workgroup of XCD x takes task (k / XCD_RUN * 8 + x) * XCD_RUN + k % XCD_RUN,
// so every XCD works through runs of XCD_RUN consecutive tiles (neighbours,
// which share window halos, meet in one L2) while the runs of every segment
// are spread over all XCDs.  Workgroups past the last whole group of 8 runs
// keep their index.  A bijection on [0, gridDim.x).
constexpr int XCD_RUN = 64;
__device__ __forceinline__ int xcd_task(int b)
{
    const int full = (int)(gridDim.x / (8 * XCD_RUN)) * (8 * XCD_RUN);
    if (b >= full) return b;
    const int x = b & 7, k = b >> 3;
    return ((k / XCD_RUN) * 8 + x) * XCD_RUN + (k % XCD_RUN);
}

template <typename T>
__device__ __forceinline__ float to_f(T v) { return static_cast<float>(v); }

// Host-side launchers (one translation unit per half-window size for the
// matching kernels, so the template instances compile in parallel).
hipError_t launch_reduce(int dtype, const ReduceArgs& a, hipStream_t s);
hipError_t launch_convert(int dtype, const ConvertArgs& a, hipStream_t s);
hipError_t launch_stats(StatsArgs a, hipStream_t s);
hipError_t launch_tower(int dtype, const TowerArgs& a, hipStream_t s);
hipError_t launch_blur(int dtype, const BlurArgs& a, hipStream_t s);
hipError_t launch_median(const MedianArgs& a, hipStream_t s);
hipError_t launch_median_multi(const MultiArgs& a, int blocks, hipStream_t s);
hipError_t launch_adjoint(const AdjArgs& a, hipStream_t s);
hipError_t launch_gate(int n, int dtype, int mode, const GateArgs& a, hipStream_t s);
hipError_t launch_gate_multi(int n, int dtype, int mode, const MultiArgs& a, int blocks, hipStream_t s);
hipError_t launch_upsample_cost(const float* cc, int Hc, int Wc, int cpitch, int H, int W, double* out,
                                int opitch, hipStream_t s);
hipError_t launch_match(int n, int dtype, int mode, int nc, const MatchArgs& a, hipStream_t s);

// Multi-segment launches (batched path); `blocks` = total tiles of the segments.
hipError_t launch_match_multi(int n, int dtype, int mode, int nc, const MultiArgs& a, int blocks, hipStream_t s);
// dtype MSIBM_U8: every statistics and reduce tile of the launch reads a
// uint8 level (a leaner kernel); anything else: the general kernel.
hipError_t launch_levels_multi(int n, int dtype, const MultiArgs& a, int blocks, hipStream_t s);
hipError_t launch_stats_multi(int n, const MultiArgs& a, int blocks, hipStream_t s);
hipError_t launch_match_multi_n1(int dtype, int mode, int nc, const MultiArgs& a, int blocks, hipStream_t s);
hipError_t launch_match_multi_n2(int dtype, int mode, int nc, const MultiArgs& a, int blocks, hipStream_t s);
hipError_t launch_match_multi_n3(int dtype, int mode, int nc, const MultiArgs& a, int blocks, hipStream_t s);
hipError_t launch_match_multi_n4(int dtype, int mode, int nc, const MultiArgs& a, int blocks, hipStream_t s);
hipError_t launch_match_multi_n5(int dtype, int mode, int nc, const MultiArgs& a, int blocks, hipStream_t s);
hipError_t launch_match_multi_n6(int dtype, int mode, int nc, const MultiArgs& a, int blocks, hipStream_t s);

hipError_t launch_match_n1(int dtype, int mode, int nc, const MatchArgs& a, hipStream_t s);
hipError_t launch_match_n2(int dtype, int mode, int nc, const MatchArgs& a, hipStream_t s);
hipError_t launch_match_n3(int dtype, int mode, int nc, const MatchArgs& a, hipStream_t s);
hipError_t launch_match_n4(int dtype, int mode, int nc, const MatchArgs& a, hipStream_t s);
hipError_t launch_match_n5(int dtype, int mode, int nc, const MatchArgs& a, hipStream_t s);
hipError_t launch_match_n6(int dtype, int mode, int nc, const MatchArgs& a, hipStream_t s);

hipError_t launch_backward(int n, int nc, const BackArgs& a, hipStream_t s);
hipError_t launch_backward_multi(int n, int nc, const MultiArgs& a, int blocks, hipStream_t s);
hipError_t launch_backward_multi_n1(int nc, const MultiArgs& a, int blocks, hipStream_t s);
hipError_t launch_backward_multi_n2(int nc, const MultiArgs& a, int blocks, hipStream_t s);
hipError_t launch_backward_multi_n3(int nc, const MultiArgs& a, int blocks, hipStream_t s);
hipError_t launch_backward_multi_n4(int nc, const MultiArgs& a, int blocks, hipStream_t s);
hipError_t launch_backward_multi_n5(int nc, const MultiArgs& a, int blocks, hipStream_t s);
hipError_t launch_backward_multi_n6(int nc, const MultiArgs& a, int blocks, hipStream_t s);
hipError_t launch_zero_multi(const MultiArgs& a, int blocks, hipStream_t s);
hipError_t launch_backward_n1(int nc, const BackArgs& a, hipStream_t s);
hipError_t launch_backward_n2(int nc, const BackArgs& a, hipStream_t s);
hipError_t launch_backward_n3(int nc, const BackArgs& a, hipStream_t s);
hipError_t launch_backward_n4(int nc, const BackArgs& a, hipStream_t s);
hipError_t launch_backward_n5(int nc, const BackArgs& a, hipStream_t s);
hipError_t launch_backward_n6(int nc, const BackArgs& a, hipStream_t s);
// Zero `count` floats at each of up to two pointers (graph-capturable fill).
hipError_t launch_zero(float* a, float* b, size_t count, hipStream_t s);
hipError_t launch_mask_count(const uint8_t* mask, size_t total, int* count, hipStream_t s);
hipError_t launch_mask_count_multi(const MultiArgs& a, int blocks, hipStream_t s);
hipError_t launch_l1_finalize(const float* sum, const int* count, float* loss, hipStream_t s);
hipError_t launch_l1_finalize_multi(const MultiArgs& a, int np, hipStream_t s);
hipError_t launch_fill(float* a, float v, size_t count, hipStream_t s);

// Slots evaluated per block: 2r+1, but at least 2 so that a block whose prior
// is clipped by the left image border (pixel columns j0 and j0+1 then centre
// on j0 and j0+1) still fits one window.
__host__ __device__ inline int slots_for_radius(int r) { return 2 * r + 1 < 2 ? 2 : 2 * r + 1; }

}  // namespace msibm
