// Pyramid reduce and window-statistics tile functions (see levels.hip).
#pragma once

#include "common.hpp"

namespace msibm {

constexpr int RD_W = 64, RD_H = 16;                 // output tile
constexpr int RD_IW = 2 * RD_W + 3, RD_IH = 2 * RD_H + 3;  // input region (5-tap halo)

// The staged input region (floats, or the bytes themselves for a uint8
// source, a quarter of the LDS) and the horizontal sums.
template <typename S>
struct ReduceSmemT {
    S in[RD_IH][RD_IW + 1];
    float hs[RD_IH][RD_W + 1];
};
using ReduceSmem = ReduceSmemT<float>;
using ReduceSmemU8 = ReduceSmemT<uint8_t>;

// One 16 x 64 output tile of one view: the input region is staged in LDS once,
// the horizontal 5-tap sums are taken at even columns, then the vertical ones at
// even rows.  Same arithmetic order as a direct evaluation: h = sum_b w_b x,
// out = 2^-8 sum_t w_t h_t with integer weights, all partial sums exact for
// uint8 input up to level 2.  Every thread of the workgroup must call it.
template <typename T, typename S>
__device__ __forceinline__ void reduce_tile(const ReduceArgs& a, int view, int bx, int by, ReduceSmemT<S>& sm)
{
    S (*in)[RD_IW + 1] = sm.in;
    float (*hs)[RD_W + 1] = sm.hs;
    const T* __restrict__ src = static_cast<const T*>(a.src[view]);
    float* __restrict__ dst = a.dst[view];
    const int ox0 = bx * RD_W, oy0 = by * RD_H;
    const int ix0 = 2 * ox0 - 2, iy0 = 2 * oy0 - 2;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // stage: every load of the thread issued, unconditionally, before the LDS
    // stores (positions past the region re-read its last row or column), so
    // that the loads share one latency
    constexpr int RI = (RD_IH + 3) / 4, CI = (RD_IW + 63) / 64;
    T v[RI][CI];
#pragma unroll
    for (int ri = 0; ri < RI; ++ri) {
        const int rr = min(wave + 4 * ri, RD_IH - 1);
        const T* srow = src + (size_t)clampi(iy0 + rr, 0, a.H - 1) * a.spitch;
#pragma unroll
        for (int ci = 0; ci < CI; ++ci) {
            const int cc = min(lane + 64 * ci, RD_IW - 1);
            v[ri][ci] = srow[clampi(ix0 + cc, 0, a.W - 1)];
        }
    }
#pragma unroll
    for (int ri = 0; ri < RI; ++ri) {
        const int rr = wave + 4 * ri;
#pragma unroll
        for (int ci = 0; ci < CI; ++ci) {
            const int cc = lane + 64 * ci;
            if (rr < RD_IH && cc < RD_IW) in[rr][cc] = (S)v[ri][ci];
        }
    }
    __syncthreads();
    const float w[5] = {1.f, 4.f, 6.f, 4.f, 1.f};
    for (int rr = wave; rr < RD_IH; rr += 4) {
        float h = 0.f;
#pragma unroll
        for (int b = 0; b < 5; ++b) h = fmaf(w[b], to_f(in[rr][2 * lane + b]), h);
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
    __syncthreads();  // LDS may be reused by the caller's next tile
}

template <typename T>
__global__ __launch_bounds__(256) void reduce_kernel(ReduceArgs a)
{
    __shared__ ReduceSmem sm;
    reduce_tile<T, float>(a, blockIdx.z, blockIdx.x, blockIdx.y, sm);
}

// One 16 x 64 tile of the same binomial blur at every pixel (stride 1) of one
// view, with the arithmetic of reduce_tile: h = sum_b w_b x, out = 2^-8 sum_t
// w_t h_t with integer weights (exact for uint8 input).  256 threads.
constexpr int BL_W = 64, BL_H = 16, BL_IW = BL_W + 4, BL_IH = BL_H + 4;
struct BlurSmem {
    float in[BL_IH][BL_IW + 1];
    float hs[BL_IH][BL_W + 1];
};

template <typename T>
__device__ __forceinline__ void blur_tile(const T* __restrict__ src, float* __restrict__ dst, int H, int W,
                                          int spitch, int dpitch, int bx, int by, BlurSmem& sm)
{
    const int x0 = bx * BL_W, y0 = by * BL_H;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // stage: every load issued before the LDS stores
    constexpr int RI = (BL_IH + 3) / 4, CI = (BL_IW + 63) / 64;
    T v[RI][CI];
#pragma unroll
    for (int ri = 0; ri < RI; ++ri) {
        const T* srow = src + (size_t)clampi(y0 - 2 + min(wave + 4 * ri, BL_IH - 1), 0, H - 1) * spitch;
#pragma unroll
        for (int ci = 0; ci < CI; ++ci) v[ri][ci] = srow[clampi(x0 - 2 + min(lane + 64 * ci, BL_IW - 1), 0, W - 1)];
    }
#pragma unroll
    for (int ri = 0; ri < RI; ++ri) {
        const int rr = wave + 4 * ri;
#pragma unroll
        for (int ci = 0; ci < CI; ++ci) {
            const int cc = lane + 64 * ci;
            if (rr < BL_IH && cc < BL_IW) sm.in[rr][cc] = to_f(v[ri][ci]);
        }
    }
    __syncthreads();
    const float w[5] = {1.f, 4.f, 6.f, 4.f, 1.f};
    for (int rr = wave; rr < BL_IH; rr += 4) {
        float h = 0.f;
#pragma unroll
        for (int b = 0; b < 5; ++b) h = fmaf(w[b], sm.in[rr][lane + b], h);
        sm.hs[rr][lane] = h;
    }
    __syncthreads();
    const int x = x0 + lane;
#pragma unroll
    for (int k = 0; k < BL_H / 4; ++k) {
        const int oy = wave + 4 * k, y = y0 + oy;
        float acc = 0.f;
#pragma unroll
        for (int t = 0; t < 5; ++t) acc = fmaf(w[t], sm.hs[oy + t][lane], acc);
        if (x < W && y < H) dst[(size_t)y * dpitch + x] = acc * (1.f / 256.f);
    }
}

// Several pyramid steps in one workgroup ("tower"): the tile of the last level
// (TW_FH x TW_FW pixels) together with every level's region that it depends on.
// Step j maps the region of level j-1 to that of level j: region rows
// R_{j-1} = 2 R_j + 3 (the 5-tap halo at stride 2), origin o_{j-1} = 2 o_j - 2.
// Region row r of level j holds level row clamp(o_j + r), so the clamp-to-edge
// reads of a plain reduce become reads at clamped region indices, and every
// value is computed with the same operations in the same order as reduce_tile:
// the results are identical.  The tile writes the part of each level it owns
// (the last-level tile scaled by 2^(S-j)).
constexpr int TW_FH = 8, TW_FW = 16, TW_THREADS = 512;
constexpr int tw_rows(int S, int j) { return j >= S ? TW_FH : 2 * tw_rows(S, j + 1) + 3; }
constexpr int tw_cols(int S, int j) { return j >= S ? TW_FW : 2 * tw_cols(S, j + 1) + 3; }
constexpr int tw_level_floats(int S)  // regions of levels 1 .. S-1
{
    int f = 0;
    for (int j = 1; j < S; ++j) f += tw_rows(S, j) * tw_cols(S, j);
    return f;
}
constexpr int tw_max(int a, int b) { return a > b ? a : b; }

template <typename T, int S>
struct TowerSmem {
    static constexpr int IR = tw_rows(S, 0), IC = tw_cols(S, 0);
    static constexpr int A_BYTES = tw_max(IR * IC * (int)sizeof(T), tw_level_floats(S) * 4);
    // area a: the staged source region, then the regions of levels 1 .. S-1
    alignas(16) unsigned char a[(A_BYTES + 15) / 16 * 16];
    // area b: horizontal sums of the current step
    float b[IR * tw_cols(S, 1)];
};

// Step j of a tower: horizontal 5-tap sums at even region columns of the level
// j-1 region `in` (IR x 2 OC + 3), then vertical sums at even rows into the
// level j region (OR x OC), stored to `out` (LDS) or, for the last step, only to
// global memory; a pixel the tile owns also goes to `dst`.
template <typename Tin, int IR, int OR, int OC>
__device__ __forceinline__ void tower_step(const Tin* in, float* hs, float* out, int o_r, int o_c, int Ho, int Wo,
                                           int own_r, int own_c, int own_n_r, int own_n_c, float* __restrict__ dst,
                                           int dpitch)
{
    constexpr int IC = 2 * OC + 3;
    const float w[5] = {1.f, 4.f, 6.f, 4.f, 1.f};
#pragma unroll 4
    for (int idx = threadIdx.x; idx < IR * OC; idx += TW_THREADS) {
        const int r = idx / OC, c = idx - r * OC;
        const int cc = 2 * (clampi(o_c + c, 0, Wo - 1) - o_c);
        const Tin* row = in + r * IC + cc;
        float h = 0.f;
#pragma unroll
        for (int b = 0; b < 5; ++b) h = fmaf(w[b], to_f(row[b]), h);
        hs[idx] = h;
    }
    __syncthreads();
#pragma unroll 4
    for (int idx = threadIdx.x; idx < OR * OC; idx += TW_THREADS) {
        const int r = idx / OC, c = idx - r * OC;
        const int rr = 2 * (clampi(o_r + r, 0, Ho - 1) - o_r);
        float acc = 0.f;
#pragma unroll
        for (int t = 0; t < 5; ++t) acc = fmaf(w[t], hs[(rr + t) * OC + c], acc);
        acc *= (1.f / 256.f);
        if (out) out[idx] = acc;
        const int gy = o_r + r, gx = o_c + c;
        if (r >= own_r && r < own_r + own_n_r && c >= own_c && c < own_c + own_n_c && gy < Ho && gx < Wo)
            dst[(size_t)gy * dpitch + gx] = acc;
    }
    __syncthreads();  // the next step overwrites hs, and reads out
}

// One tower tile of one view: S pyramid steps from the source level.
template <typename T, int S>
__device__ __forceinline__ void tower_tile(const TowerArgs& a, int view, int tx, int ty, TowerSmem<T, S>& sm)
{
    static_assert(S >= 2 && S <= TW_MAXS, "tower of 2 or 3 steps");
    constexpr int IR = tw_rows(S, 0), IC = tw_cols(S, 0);
    // region origins, last level first
    int o_r[S + 1], o_c[S + 1];
    o_r[S] = ty * TW_FH;
    o_c[S] = tx * TW_FW;
#pragma unroll
    for (int j = S; j > 0; --j) {
        o_r[j - 1] = 2 * o_r[j] - 2;
        o_c[j - 1] = 2 * o_c[j] - 2;
    }
    // stage the source region: lanes along columns (64-column groups), waves
    // down the rows; every load issued before the LDS stores, so that they share
    // one latency (positions past the region re-read its last row or column)
    const T* __restrict__ src = static_cast<const T*>(a.src[view]);
    T* in = reinterpret_cast<T*>(sm.a);
    constexpr int NWV = TW_THREADS / 64, RI = (IR + NWV - 1) / NWV, CI = (IC + 63) / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    {
        int col[CI];
#pragma unroll
        for (int ci = 0; ci < CI; ++ci) col[ci] = clampi(o_c[0] + min(lane + 64 * ci, IC - 1), 0, a.Ws - 1);
        T v[RI][CI];
#pragma unroll
        for (int ri = 0; ri < RI; ++ri) {
            const T* srow = src + (size_t)clampi(o_r[0] + min(wave + NWV * ri, IR - 1), 0, a.Hs - 1) * a.spitch;
#pragma unroll
            for (int ci = 0; ci < CI; ++ci) v[ri][ci] = srow[col[ci]];
        }
#pragma unroll
        for (int ri = 0; ri < RI; ++ri) {
            const int r = wave + NWV * ri;
#pragma unroll
            for (int ci = 0; ci < CI; ++ci) {
                const int c = lane + 64 * ci;
                if (r < IR && c < IC) in[r * IC + c] = v[ri][ci];
            }
        }
    }
    __syncthreads();
    float* lev = reinterpret_cast<float*>(sm.a);
    constexpr int L1 = tw_rows(S, 1) * tw_cols(S, 1);
    // step 1 reads the source (area a) and writes level 1 into area a: the
    // horizontal pass has consumed the source before the vertical pass writes
    tower_step<T, IR, tw_rows(S, 1), tw_cols(S, 1)>(in, sm.b, lev, o_r[1], o_c[1], a.H[0], a.W[0],
                                                    2 * (1 << (S - 1)) - 2, 2 * (1 << (S - 1)) - 2,
                                                    TW_FH << (S - 1), TW_FW << (S - 1), a.dst[0][view], a.W[0]);
    if (S == 3) {
        tower_step<float, tw_rows(S, 1), tw_rows(S, 2), tw_cols(S, 2)>(lev, sm.b, lev + L1, o_r[2], o_c[2], a.H[1],
                                                                       a.W[1], 2, 2, TW_FH << 1, TW_FW << 1,
                                                                       a.dst[1][view], a.W[1]);
        tower_step<float, tw_rows(S, 2), TW_FH, TW_FW>(lev + L1, sm.b, nullptr, o_r[3], o_c[3], a.H[2], a.W[2], 0, 0,
                                                       TW_FH, TW_FW, a.dst[2][view], a.W[2]);
    } else {
        tower_step<float, tw_rows(S, 1), TW_FH, TW_FW>(lev, sm.b, nullptr, o_r[2], o_c[2], a.H[1], a.W[1], 0, 0,
                                                       TW_FH, TW_FW, a.dst[1][view], a.W[1]);
    }
}

constexpr int ST_W = 64, ST_H = 16, ST_MAXN = 6;
constexpr int ST_SEG = 8;                               // outputs per thread, horizontal pass

// One 16 x 64 tile of one view of one level.  Horizontal window sums of x and x^2
// in double precision (running sums over 8 outputs per thread, read straight from
// global memory), then vertical running sums over 4 outputs per thread.  Values
// are centred on the tile's first pixel before squaring, so the sums stay small.
// The horizontal sums sit in LDS with each 8-column segment padded to 9 entries
// and rows to 73, so that the horizontal pass (a wave spans 8 rows x 8
// segments) spreads its stores over the banks instead of hitting two.
constexpr int ST_HS = 73;  // row stride (doubles)
__device__ __forceinline__ int st_idx(int row, int col) { return row * ST_HS + (col >> 3) * 9 + (col & 7); }

// uint8 levels use 32-row tiles with integer sums: centred pixel values, their
// squares and every window sum are exact integers (below 2^24 for n <= 6), and
// the tile's sums fit the LDS space of a 16-row double tile.  The int sums sit
// in rows of 65, so that a wave's horizontal stores (8 rows x 8 segments at one
// offset) fall in distinct banks.
constexpr int SU_H = 32, SU_HS = 65;
__host__ __device__ inline int stats_tile_h(int dtype) { return dtype == 0 ? SU_H : ST_H; }

template <int NW>
struct StatsSmemD {  // horizontal sums of the tile's rows with their window halo
    double h1[(ST_H + 2 * NW) * ST_HS];
    double h2[(ST_H + 2 * NW) * ST_HS];
};
template <int NW>
struct StatsSmemI {
    int h1[(SU_H + 2 * NW) * SU_HS];
    int h2[(SU_H + 2 * NW) * SU_HS];
};
template <int NW>
union StatsSmem {
    StatsSmemD<NW> d;
    StatsSmemI<NW> i;
};
static_assert(sizeof(StatsSmemI<1>) <= sizeof(StatsSmemD<1>) && sizeof(StatsSmemI<6>) <= sizeof(StatsSmemD<6>),
              "uint8 tiles fit the double tiles' space");

// Statistics of one 16 x 64 tile of both views (A and B) of one level.  Every
// input load of both views is issued first, so view B's loads are in flight
// while view A is computed.
template <typename T, int NW>
__device__ __forceinline__ void stats_tile(const T* __restrict__ srcA, WinStat* __restrict__ dstA,
                                           const T* __restrict__ srcB, WinStat* __restrict__ dstB, int H, int W,
                                           int spitch, int dpitch, double var_eps, int x0, int y0, StatsSmem<NW>& sm)
{
    double* h1 = sm.d.h1;
    double* h2 = sm.d.h2;
    constexpr int n = NW, wn = 2 * NW + 1, rows = ST_H + 2 * NW, NF = ST_SEG + 2 * NW;
    const size_t corner = (size_t)min(y0, H - 1) * spitch + min(x0, W - 1);
    const double cv[2] = {(double)to_f(srcA[corner]), (double)to_f(srcB[corner])};
    // horizontal pass inputs: thread = (row, 8-column segment)
    const int seg = threadIdx.x & 7, rr = threadIdx.x >> 3;  // 32 rows x 8 segments
    const size_t ro = (size_t)clampi(y0 - n + min(rr, rows - 1), 0, H - 1) * spitch;
    const int cx = x0 + ST_SEG * seg - n;
    float f[2][NF];
#pragma unroll
    for (int t = 0; t < NF; ++t) {
        f[0][t] = to_f(srcA[ro + clampi(cx + t, 0, W - 1)]);
        f[1][t] = to_f(srcB[ro + clampi(cx + t, 0, W - 1)]);
    }
    const int col = threadIdx.x & 63, rs = (threadIdx.x >> 6) * 4;
    const double N = (double)(wn * wn), invN = 1.0 / N;
#pragma unroll
    for (int vw = 0; vw < 2; ++vw) {
        const double c = cv[vw];
        WinStat* __restrict__ dst = vw ? dstB : dstA;
        if (rr < rows) {
            double v[NF];
#pragma unroll
            for (int t = 0; t < NF; ++t) v[t] = (double)f[vw][t] - c;
            double s1 = 0.0, s2 = 0.0;
#pragma unroll
            for (int t = 0; t < wn; ++t) {
                s1 += v[t];
                s2 = fma(v[t], v[t], s2);
            }
            h1[st_idx(rr, ST_SEG * seg)] = s1;
            h2[st_idx(rr, ST_SEG * seg)] = s2;
#pragma unroll
            for (int k = 1; k < ST_SEG; ++k) {
                const double add = v[k - 1 + wn], drop = v[k - 1];
                s1 += add - drop;
                s2 += fma(add, add, -drop * drop);
                h1[st_idx(rr, ST_SEG * seg + k)] = s1;
                h2[st_idx(rr, ST_SEG * seg + k)] = s2;
            }
        }
        __syncthreads();
        // vertical pass: thread = (column, 4-row segment)
        double s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int t = 0; t < wn; ++t) {
            s1 += h1[st_idx(rs + t, col)];
            s2 += h2[st_idx(rs + t, col)];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (k > 0) {
                s1 += h1[st_idx(rs + k - 1 + wn, col)] - h1[st_idx(rs + k - 1, col)];
                s2 += h2[st_idx(rs + k - 1 + wn, col)] - h2[st_idx(rs + k - 1, col)];
            }
            const int gy = y0 + rs + k, gx = x0 + col;
            if (gy < H && gx < W) {
                const double A = s2 - s1 * s1 * invN;
                const float inv = (A <= N * var_eps) ? 0.f : rsqrtf((float)A);
                const double mu = c + s1 * invN;
                const float hi = (float)mu;
                dst[(size_t)gy * dpitch + gx] = WinStat{hi, (float)(mu - (double)hi), inv};
            }
        }
        __syncthreads();  // LDS is reused by the next view and the caller's next tile
    }
}

// Statistics of one 32 x 64 tile of both views of a uint8 level, from exact
// integer window sums: the window sum S1 and 1/sqrt(A) as WinStatU8 records
// (8 bytes per pixel, written into the statistics buffer at the same pitch).
template <int NW>
__device__ __forceinline__ void stats_tile_u8(const uint8_t* __restrict__ srcA, WinStat* __restrict__ dstA,
                                              const uint8_t* __restrict__ srcB, WinStat* __restrict__ dstB, int H,
                                              int W, int spitch, int dpitch, double var_eps, int x0, int y0,
                                              StatsSmemI<NW>& sm)
{
    int* h1 = sm.h1;
    int* h2 = sm.h2;
    constexpr int n = NW, wn = 2 * NW + 1, rows = SU_H + 2 * NW, NF = ST_SEG + 2 * NW;
    constexpr int TASKS = rows * 8, NT = (TASKS + 255) / 256;  // (row, 8-column segment) tasks
    const size_t corner = (size_t)min(y0, H - 1) * spitch + min(x0, W - 1);
    const int cv[2] = {srcA[corner], srcB[corner]};
    // interior tiles load whole aligned words: a thread's NF bytes start at
    // byte offset sh (of its row's address) within the first of NG + 1 words,
    // and v_alignbyte lines them up four at a time (any row pitch); edge tiles
    // load byte by byte (clamped) and pack the bytes into words (offset 0).
    // The words are kept packed until each view is summed.
    constexpr int NG = (NF + 3) / 4;
    const bool words = x0 - n >= 0 && x0 + ST_W + n + 8 <= W;
    uint32_t wd[NT][2][NG + 1], sh[NT][2];
#pragma unroll
    for (int q = 0; q < NT; ++q) {
        const int task = min((int)threadIdx.x + 256 * q, TASKS - 1);
        const int tr = task >> 3, seg = task & 7;
        const size_t ro = (size_t)clampi(y0 - n + tr, 0, H - 1) * spitch;
        const int cx = x0 + ST_SEG * seg - n;
        if (words) {
#pragma unroll
            for (int vw = 0; vw < 2; ++vw) {
                const uintptr_t ad = reinterpret_cast<uintptr_t>((vw ? srcB : srcA) + ro + cx);
                const uint32_t* pw = reinterpret_cast<const uint32_t*>(ad & ~(uintptr_t)3);
                sh[q][vw] = (uint32_t)(ad & 3);
#pragma unroll
                for (int d = 0; d <= NG; ++d) wd[q][vw][d] = pw[d];
            }
        } else {
#pragma unroll
            for (int vw = 0; vw < 2; ++vw) {
                const uint8_t* src = vw ? srcB : srcA;
                sh[q][vw] = 0;
#pragma unroll
                for (int g = 0; g <= NG; ++g) {
                    uint32_t w = 0;
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        if (4 * g + b < NF) w |= (uint32_t)src[ro + clampi(cx + 4 * g + b, 0, W - 1)] << (8 * b);
                    wd[q][vw][g] = w;
                }
            }
        }
    }
    const int col = threadIdx.x & 63, rs = (threadIdx.x >> 6) * 8;
    const double N = (double)(wn * wn), invN = 1.0 / N;
#pragma unroll
    for (int vw = 0; vw < 2; ++vw) {
        const int c = cv[vw];
        WinStat* __restrict__ dst = vw ? dstB : dstA;
#pragma unroll
        for (int q = 0; q < NT; ++q) {
            const int task = threadIdx.x + 256 * q;
            if (task < TASKS) {
                int v[NF], sq[NF];
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    const uint32_t w = __builtin_amdgcn_alignbyte(wd[q][vw][g + 1], wd[q][vw][g], sh[q][vw]);
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        if (4 * g + b < NF) v[4 * g + b] = (int)((w >> (8 * b)) & 0xffu) - c;
                }
#pragma unroll
                for (int t = 0; t < NF; ++t) sq[t] = v[t] * v[t];
                int s1 = 0, s2 = 0;
#pragma unroll
                for (int t = 0; t < wn; ++t) {
                    s1 += v[t];
                    s2 += sq[t];
                }
                const int base = (task >> 3) * SU_HS + ST_SEG * (task & 7);
                h1[base] = s1;
                h2[base] = s2;
#pragma unroll
                for (int k = 1; k < ST_SEG; ++k) {
                    s1 += v[k - 1 + wn] - v[k - 1];
                    s2 += sq[k - 1 + wn] - sq[k - 1];
                    h1[base + k] = s1;
                    h2[base + k] = s2;
                }
            }
        }
        __syncthreads();
        // vertical pass: thread = (column, 8-row segment)
        int s1 = 0, s2 = 0;
#pragma unroll
        for (int t = 0; t < wn; ++t) {
            s1 += h1[(rs + t) * SU_HS + col];
            s2 += h2[(rs + t) * SU_HS + col];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (k > 0) {
                s1 += h1[(rs + k - 1 + wn) * SU_HS + col] - h1[(rs + k - 1) * SU_HS + col];
                s2 += h2[(rs + k - 1 + wn) * SU_HS + col] - h2[(rs + k - 1) * SU_HS + col];
            }
            const int gy = y0 + rs + k, gx = x0 + col;
            if (gy < H && gx < W) {
                const double d1 = (double)s1, d2 = (double)s2;
                const double A = d2 - d1 * d1 * invN;
                const float inv = (A <= N * var_eps) ? 0.f : rsqrtf((float)A);
                // the window sum of the uncentred values, an exact integer
                reinterpret_cast<WinStatU8*>(dst)[(size_t)gy * dpitch + gx] =
                    WinStatU8{(float)(s1 + wn * wn * c), inv};
            }
        }
        __syncthreads();  // LDS is reused by the next view and the caller's next tile
    }
}

}  // namespace msibm
