// Pyramid reduce and window-statistics tile functions (see levels.hip).
#pragma once

#include "common.hpp"

namespace msibm {

constexpr int RD_W = 64, RD_H = 16;                 // output tile
constexpr int RD_IW = 2 * RD_W + 3, RD_IH = 2 * RD_H + 3;  // input region (5-tap halo)

struct ReduceSmem {
    float in[RD_IH][RD_IW + 1];
    float hs[RD_IH][RD_W + 1];
};

// One 16 x 64 output tile of one view: the input region is staged in LDS once,
// the horizontal 5-tap sums are taken at even columns, then the vertical ones at
// even rows.  Same arithmetic order as a direct evaluation: h = sum_b w_b x,
// out = 2^-8 sum_t w_t h_t with integer weights, all partial sums exact for
// uint8 input up to level 2.  Every thread of the workgroup must call it.
template <typename T>
__device__ __forceinline__ void reduce_tile(const ReduceArgs& a, int view, int bx, int by, ReduceSmem& sm)
{
    float (*in)[RD_IW + 1] = sm.in;
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
    __syncthreads();  // LDS may be reused by the caller's next tile
}

template <typename T>
__global__ __launch_bounds__(256) void reduce_kernel(ReduceArgs a)
{
    __shared__ ReduceSmem sm;
    reduce_tile<T>(a, blockIdx.z, blockIdx.x, blockIdx.y, sm);
}

constexpr int ST_W = 64, ST_H = 16, ST_MAXN = 6;
constexpr int ST_SEG = 8;                               // outputs per thread, horizontal pass
constexpr int ST_RH = ST_H + 2 * ST_MAXN;               // 28 rows with halo

// One 16 x 64 tile of one view of one level.  Horizontal window sums of x and x^2
// in double precision (running sums over 8 outputs per thread, read straight from
// global memory), then vertical running sums over 4 outputs per thread.  Values
// are centred on the tile's first pixel before squaring, so the sums stay small.
// The horizontal sums sit in LDS with each 8-column segment padded to 9 entries
// and rows to 73, so that the horizontal pass (a wave spans 8 rows x 8
// segments) spreads its stores over the banks instead of hitting two.
constexpr int ST_HS = 73;  // row stride (doubles)
__device__ __forceinline__ int st_idx(int row, int col) { return row * ST_HS + (col >> 3) * 9 + (col & 7); }

struct StatsSmem {
    double h1[ST_RH * ST_HS];
    double h2[ST_RH * ST_HS];
};

template <typename T, int NW>
__device__ __forceinline__ void stats_tile(const T* __restrict__ src, int H, int W, int spitch,
                                           float4* __restrict__ dst, int dpitch, double var_eps,
                                           int x0, int y0, StatsSmem& sm)
{
    double* h1 = sm.h1;
    double* h2 = sm.h2;
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
    }
    __syncthreads();
    // vertical pass: thread = (column, 4-row segment)
    const int col = threadIdx.x & 63, rs = (threadIdx.x >> 6) * 4;
    const double N = (double)(wn * wn), invN = 1.0 / N;
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
            dst[(size_t)gy * dpitch + gx] = make_float4(hi, (float)(mu - (double)hi), inv, 0.f);
        }
    }
    __syncthreads();  // LDS may be reused by the caller's next tile
}

}  // namespace msibm
