// ZNCC winner-take-all matching of one pyramid level (Eqs. 1-4 and 8-9), with
// the soft-argmax of the differentiable finest level.
//
// Work split.  A workgroup of 4 waves covers a TILE_H x 128 pixel tile, TILE_H =
// 8 BY; each thread owns BY 2x2 pixel blocks stacked 8 rows apart.  The left
// tile with its window halo sits in LDS once; the right image and its window
// statistics are staged in LDS one chunk of candidate disparities at a time.
// For a block and a window of NC consecutive candidate slots, the thread walks
// the 2n+2 window rows: it loads the 2n+2 left values and 2n+1+NC right values
// of the row from LDS and accumulates, per slot, the products shared by both
// pixel columns once plus one edge product per column.  That costs (2n+2)^2
// fused multiply-adds per slot for the block's 4 window sums instead of
// 4 (2n+1)^2 for four independent windows.  The cross sum is then normalised
// with per-pixel statistics (window mean, 1/sqrt(A)) and a running
// winner-take-all keeps the lowest z among equal scores.
//
// Modes
//   MODE_FULL   every valid candidate 0..min(D_k-1, j) in steps of NC slots
//               (coarsest level, and standard block matching at level 0);
//   MODE_REFINE one window of NC = max(2r+1, 2) slots around the doubled,
//               nearest-neighbour-upsampled prior (Eqs. 8-9, first branch);
//   MODE_SOFT   as refine, plus p = softmax(rho / tau) and d_soft = sum p z.
//
// LDS layout.  Each tile row stores its even columns first, then its odd
// columns.  A wave's 64 lanes read columns 2*lane + t, which this layout turns
// into 64 consecutive words (no bank conflicts), and t's parity is a
// compile-time constant, so every load is one ds_read with an immediate offset.
// Staging writes one even and one odd column per lane and iteration, straight
// to their two halves.
//
// Precision.  The score is invariant to a constant offset of either window, so
// each thread centres its left windows on a = the window mean of its block's
// first pixel (subtracted as the left values are loaded), and the right tile is
// centred on one right pixel of the tile (cR, subtracted when staging).  The
// products then stay near the window's own spread and the cross term
//   C = sum (l - a)(r - cR) - N (mu_l - a)(mu_r - cR)
// cancels little; the window means carry their float rounding remainder so
// (mu - a) and (mu - cR) keep their low bits.  rho = C * invsd_l * invsd_r,
// clamped to [-1, 1].  uint8 levels need none of this: staged as they are,
// every product is an integer up to 255^2 and every window sum of products an
// integer below 2^24, exact in float, so with the exact window sums S1 of the
// statistics the cross term is formed exactly, N C = N S - S1_l S1_r (in 32-bit
// integers: 24-bit multiplies, the difference within +-2^31), and only the
// final products round.
#pragma once

#include <type_traits>

#include "common.hpp"

namespace msibm {

// Candidates per right-image chunk.  A full search streams through every
// candidate 96 at a time.  A restricted search stages, in one go, the union of
// the candidate windows of all blocks of the tile (up to 320 candidates): the
// blocks' windows are data dependent (occluded regions give scattered priors),
// and with short chunks a wave whose blocks fall into several chunks would run
// the window code once per chunk with most lanes idle.
//
// A short chunk (the VARIANT_SHORT shape: 48 candidates for a full search, 128
// for a restricted one) halves the right tile's LDS, so more workgroups fit a
// CU, at the cost of more chunks per tile where the candidates spread.
template <int MODE, bool SHORT = false>
struct ChunkOf {
    static constexpr int value = (MODE == MODE_FULL) ? (SHORT ? 48 : 96) : (SHORT ? 128 : 320);
};
// The backward's LDS also holds gradient tiles beside the images; 112 candidates
// keep a right row (128 + 2n + 111 columns) within two 128-column groups for
// every n <= 6, so the chunk costs no more LDS than a short one.
constexpr int BACK_CHUNK = 112;

// LDS geometry.  Each staged row keeps its even logical columns in the first
// half and its odd ones in the second; a half holds whole groups of 64 column
// pairs (one per lane of a staging wave), so staging stores need no per-element
// bounds test, and one padding word separates the rows.
template <int NW, int CH, int TH_>
struct Geo {
    static constexpr int TH = TH_;                // tile height in pixels
    static constexpr int WN = 2 * NW + 2;         // rows/cols spanned by a block's windows
    static constexpr int LROWS = TH + 2 * NW;     // LDS rows (both views)
    static constexpr int LCOLS = TILE_W + 2 * NW; // left tile logical width
    static constexpr int LHALF = MATCH_TX * ((LCOLS + 2 * MATCH_TX - 1) / (2 * MATCH_TX));
    static constexpr int LSTRIDE = 2 * LHALF + 1;
    static constexpr int RCOLS = TILE_W + 2 * NW + CH - 1;
    static constexpr int RHALF = MATCH_TX * ((RCOLS + 2 * MATCH_TX - 1) / (2 * MATCH_TX));
    static constexpr int RSTRIDE = 2 * RHALF + 1;
    static constexpr int SCOLS = TILE_W + CH - 1;  // right statistics columns
    static constexpr int SHALF = MATCH_TX * ((SCOLS + 2 * MATCH_TX - 1) / (2 * MATCH_TX));
    static constexpr int SSTRIDE = 2 * SHALF + 1;
};

// LDS of one matching tile: the left tile, one chunk of the right tile, and the
// right window statistics of the chunk's columns (window mean minus the right
// centring constant, and 1/sd).
template <int NW, int CH, int TH, int SL>
struct MatchSmem {
    using G = Geo<NW, CH, TH>;
    static constexpr int SN = SL ? G::TH * G::SSTRIDE : 1;  // statistics planes only when staged
    float Ls[G::LROWS * G::LSTRIDE];
    float Rs[G::LROWS * G::RSTRIDE];
    float Sm[SN];
    float Si[SN];
    // candidate-split tiles (fewer rows than a block row per wave): per wave,
    // pixel and lane, the best score and its z
    static constexpr int CN = (TH < TILE_H1) ? 2 * 4 * MATCH_THREADS : 1;
    float cmb[CN];
    int lo, hi;
    unsigned mask;
};

// Position of logical column c in a split-layout row whose odd columns start at `half`.
__device__ __forceinline__ int split_pos(int c, int half) { return (c & 1) ? half + (c >> 1) : (c >> 1); }

// Stage rows [gy0, gy0+ROWS) x cols [gx0, gx0+cols) (cols <= MAXCOLS) of `src`,
// clamped to the image, into LDS in split layout (even columns at [0, half),
// odd ones at [half, ...)), centred by c.  Each wave takes whole rows; lane l of
// group k stages columns 2(l + 64k) and 2(l + 64k) + 1.  Every load of the
// thread is issued, unconditionally, before its first LDS store so that their
// latencies overlap (a load under a branch would be waited for inside it):
// columns past `cols` re-read the last staged column, and only the groups that
// hold staged columns are stored (a wave-uniform test).  A half holds whole
// groups, and columns past `cols` are never read.
// uint8 rows read as 32-bit words: lane l of group q takes the 4 columns
// 4 (l + 64 q) .. + 3 of each row as one byte-aligned window of two aligned
// words (the row's byte offset within a word is the same for every lane), and
// writes them, as floats, to the even and odd halves.  The caller guarantees
// that every row's columns [gx0 - 4, gx0 + cols + 8) are inside the image, so
// no read is clamped; lanes past `cols` re-read the last word group and store
// nothing (columns past `cols` are never read, and a stored pair index stays
// below `half`).  Loads are all issued before the first store.
template <int ROWS, int MAXCOLS, int NWAVES>
struct RowWordsU8 {
    static constexpr int RI = (ROWS + NWAVES - 1) / NWAVES;
    static constexpr int QI = (MAXCOLS + 4 * MATCH_TX - 1) / (4 * MATCH_TX);
    uint32_t w0[RI][QI], w1[RI][QI];
    uint32_t sh[RI];

    __device__ __forceinline__ void load(const uint8_t* __restrict__ src, int pitch, int H, int gy0, int gx0,
                                         int cols)
    {
        const int lane = threadIdx.x & (MATCH_TX - 1), wave = threadIdx.x / MATCH_TX;
        const int last = (cols - 1) & ~3;
#pragma unroll
        for (int ri = 0; ri < RI; ++ri) {
            const int rr = wave + NWAVES * ri;
            const uintptr_t a = reinterpret_cast<uintptr_t>(src + (size_t)clampi(gy0 + rr, 0, H - 1) * pitch + gx0);
            sh[ri] = (uint32_t)(a & 3);
            const uint32_t* wp = reinterpret_cast<const uint32_t*>(a & ~(uintptr_t)3);
#pragma unroll
            for (int qi = 0; qi < QI; ++qi) {
                const int col = min(4 * (lane + MATCH_TX * qi), last);
                w0[ri][qi] = wp[col >> 2];
                w1[ri][qi] = wp[(col >> 2) + 1];
            }
        }
    }

    __device__ __forceinline__ void store(float* dst, int stride, int half, int cols) const
    {
        const int lane = threadIdx.x & (MATCH_TX - 1), wave = threadIdx.x / MATCH_TX;
#pragma unroll
        for (int ri = 0; ri < RI; ++ri) {
            const int rr = wave + NWAVES * ri;
            if (rr >= ROWS) continue;
            float* drow = dst + rr * stride;
#pragma unroll
            for (int qi = 0; qi < QI; ++qi) {
                const int m = lane + MATCH_TX * qi;
                if (4 * m < cols) {
                    const uint32_t w = __builtin_amdgcn_alignbyte(w1[ri][qi], w0[ri][qi], sh[ri]);
                    drow[2 * m] = (float)(w & 0xffu);
                    drow[2 * m + 1] = (float)((w >> 16) & 0xffu);
                    drow[half + 2 * m] = (float)((w >> 8) & 0xffu);
                    drow[half + 2 * m + 1] = (float)(w >> 24);
                }
            }
        }
    }
};

// Whether rows of a uint8 image may be staged with RowWordsU8 (no clamped column).
__device__ __forceinline__ bool words_inside(int gx0, int cols, int W) { return gx0 >= 4 && gx0 + cols + 8 <= W; }

template <typename T, int ROWS, int MAXCOLS, int NWAVES = MATCH_TY>
__device__ __forceinline__ void stage_tile(float* dst, int stride, int half, const T* __restrict__ src,
                                           int pitch, int H, int W, int gy0, int gx0, int cols, float c)
{
    if constexpr (std::is_same<T, uint8_t>::value) {
        // uint8 levels are staged uncentred (c = 0)
        if (words_inside(gx0, cols, W)) {
            RowWordsU8<ROWS, MAXCOLS, NWAVES> rw;
            rw.load(src, pitch, H, gy0, gx0, cols);
            rw.store(dst, stride, half, cols);
            return;
        }
    }
    constexpr int RI = (ROWS + NWAVES - 1) / NWAVES;
    constexpr int CI = (MAXCOLS + 2 * MATCH_TX - 1) / (2 * MATCH_TX);
    const int lane = threadIdx.x & (MATCH_TX - 1), wave = threadIdx.x / MATCH_TX;
    const int groups = (cols + 2 * MATCH_TX - 1) / (2 * MATCH_TX);
    T v0[RI][CI], v1[RI][CI];
    // rows whose columns all lie inside the image need no column clamp
    const bool inside = gx0 >= 0 && gx0 + cols <= W;
#pragma unroll
    for (int ri = 0; ri < RI; ++ri) {
        const int rr = wave + NWAVES * ri;
        const T* srow = src + (size_t)clampi(gy0 + rr, 0, H - 1) * pitch;
        if (inside) {
            const T* sp = srow + gx0;
#pragma unroll
            for (int ci = 0; ci < CI; ++ci) {
                const int cc = 2 * (lane + MATCH_TX * ci);
                v0[ri][ci] = sp[min(cc, cols - 1)];
                v1[ri][ci] = sp[min(cc + 1, cols - 1)];
            }
        } else {
#pragma unroll
            for (int ci = 0; ci < CI; ++ci) {
                const int cc = 2 * (lane + MATCH_TX * ci);
                v0[ri][ci] = srow[clampi(gx0 + min(cc, cols - 1), 0, W - 1)];
                v1[ri][ci] = srow[clampi(gx0 + min(cc + 1, cols - 1), 0, W - 1)];
            }
        }
    }
#pragma unroll
    for (int ri = 0; ri < RI; ++ri) {
        const int rr = wave + NWAVES * ri;
        if (rr >= ROWS) continue;
        float* drow = dst + rr * stride;
#pragma unroll
        for (int ci = 0; ci < CI; ++ci) {
            if (ci < groups) {
                const int ch = lane + MATCH_TX * ci;  // column pair index
                drow[ch] = to_f(v0[ri][ci]) - c;
                drow[half + ch] = to_f(v1[ri][ci]) - c;
            }
        }
    }
}

// Both tiles of a fixed-window restricted search in one go: every load of the
// left and the right tile is issued before the first LDS store, so the two
// stagings share one memory latency.
template <typename T, int ROWS, int LMAX, int RMAX, int NWAVES = MATCH_TY>
__device__ __forceinline__ void stage_pair(float* ldst, int lstride, int lhalf, float* rdst, int rstride,
                                           int rhalf, const T* __restrict__ lsrc, const T* __restrict__ rsrc,
                                           int pitch, int H, int W, int gy0, int lx0, int lcols, int rx0,
                                           int rcols, float c)
{
    if constexpr (std::is_same<T, uint8_t>::value) {
        // uint8 levels are staged uncentred (c = 0)
        if (words_inside(lx0, lcols, W) && words_inside(rx0, rcols, W)) {
            RowWordsU8<ROWS, LMAX, NWAVES> lw;
            RowWordsU8<ROWS, RMAX, NWAVES> rw;
            lw.load(lsrc, pitch, H, gy0, lx0, lcols);
            rw.load(rsrc, pitch, H, gy0, rx0, rcols);
            lw.store(ldst, lstride, lhalf, lcols);
            rw.store(rdst, rstride, rhalf, rcols);
            return;
        }
    }
    constexpr int RI = (ROWS + NWAVES - 1) / NWAVES;
    constexpr int LI = (LMAX + 2 * MATCH_TX - 1) / (2 * MATCH_TX);
    constexpr int CI = (RMAX + 2 * MATCH_TX - 1) / (2 * MATCH_TX);
    const int lane = threadIdx.x & (MATCH_TX - 1), wave = threadIdx.x / MATCH_TX;
    const int lgroups = (lcols + 2 * MATCH_TX - 1) / (2 * MATCH_TX);
    const int rgroups = (rcols + 2 * MATCH_TX - 1) / (2 * MATCH_TX);
    T l0[RI][LI], l1[RI][LI], r0[RI][CI], r1[RI][CI];
    // rows whose columns all lie inside the image need no column clamp
    const bool inside = lx0 >= 0 && lx0 + lcols <= W && rx0 >= 0 && rx0 + rcols <= W;
#pragma unroll
    for (int ri = 0; ri < RI; ++ri) {
        const int rr = wave + NWAVES * ri;
        const size_t ro = (size_t)clampi(gy0 + rr, 0, H - 1) * pitch;
        if (inside) {
            const T* lp = lsrc + ro + lx0;
            const T* rp = rsrc + ro + rx0;
#pragma unroll
            for (int ci = 0; ci < LI; ++ci) {
                const int cc = 2 * (lane + MATCH_TX * ci);
                l0[ri][ci] = lp[min(cc, lcols - 1)];
                l1[ri][ci] = lp[min(cc + 1, lcols - 1)];
            }
#pragma unroll
            for (int ci = 0; ci < CI; ++ci) {
                const int cc = 2 * (lane + MATCH_TX * ci);
                r0[ri][ci] = rp[min(cc, rcols - 1)];
                r1[ri][ci] = rp[min(cc + 1, rcols - 1)];
            }
        } else {
#pragma unroll
            for (int ci = 0; ci < LI; ++ci) {
                const int cc = 2 * (lane + MATCH_TX * ci);
                l0[ri][ci] = lsrc[ro + clampi(lx0 + min(cc, lcols - 1), 0, W - 1)];
                l1[ri][ci] = lsrc[ro + clampi(lx0 + min(cc + 1, lcols - 1), 0, W - 1)];
            }
#pragma unroll
            for (int ci = 0; ci < CI; ++ci) {
                const int cc = 2 * (lane + MATCH_TX * ci);
                r0[ri][ci] = rsrc[ro + clampi(rx0 + min(cc, rcols - 1), 0, W - 1)];
                r1[ri][ci] = rsrc[ro + clampi(rx0 + min(cc + 1, rcols - 1), 0, W - 1)];
            }
        }
    }
#pragma unroll
    for (int ri = 0; ri < RI; ++ri) {
        const int rr = wave + NWAVES * ri;
        if (rr >= ROWS) continue;
#pragma unroll
        for (int ci = 0; ci < LI; ++ci)
            if (ci < lgroups) {
                const int ch = lane + MATCH_TX * ci;
                ldst[rr * lstride + ch] = to_f(l0[ri][ci]);
                ldst[rr * lstride + lhalf + ch] = to_f(l1[ri][ci]);
            }
#pragma unroll
        for (int ci = 0; ci < CI; ++ci)
            if (ci < rgroups) {
                const int ch = lane + MATCH_TX * ci;
                rdst[rr * rstride + ch] = to_f(r0[ri][ci]) - c;
                rdst[rr * rstride + rhalf + ch] = to_f(r1[ri][ci]) - c;
            }
    }
}

// Stage the right statistics of rows [gy0, gy0+ROWS) x cols [gx0, gx0+cols)
// into two split-layout LDS planes: the window mean minus c (its float value and
// rounding remainder summed after the subtraction) and 1/sd.  Same staging
// scheme as stage_tile.
template <int ROWS, int MAXCOLS, int NWAVES = MATCH_TY, bool U8 = false>
__device__ __forceinline__ void stage_stats(float* mc, float* is, int stride, int half,
                                            const WinStat* __restrict__ src, int spitch, int H, int W,
                                            int gy0, int gx0, int cols, float c)
{
    if constexpr (U8) {
        // uint8 level: the exact window sum S1 and 1/sd
        constexpr int RI = (ROWS + NWAVES - 1) / NWAVES;
        constexpr int CI = (MAXCOLS + 2 * MATCH_TX - 1) / (2 * MATCH_TX);
        const int lane = threadIdx.x & (MATCH_TX - 1), wave = threadIdx.x / MATCH_TX;
        const int groups = (cols + 2 * MATCH_TX - 1) / (2 * MATCH_TX);
        const WinStatU8* s8 = reinterpret_cast<const WinStatU8*>(src);
        WinStatU8 v0[RI][CI], v1[RI][CI];
#pragma unroll
        for (int ri = 0; ri < RI; ++ri) {
            const int rr = wave + NWAVES * ri;
            const WinStatU8* srow = s8 + (size_t)clampi(gy0 + rr, 0, H - 1) * spitch;
#pragma unroll
            for (int ci = 0; ci < CI; ++ci) {
                const int cc = 2 * (lane + MATCH_TX * ci);
                v0[ri][ci] = srow[clampi(gx0 + min(cc, cols - 1), 0, W - 1)];
                v1[ri][ci] = srow[clampi(gx0 + min(cc + 1, cols - 1), 0, W - 1)];
            }
        }
#pragma unroll
        for (int ri = 0; ri < RI; ++ri) {
            const int rr = wave + NWAVES * ri;
            if (rr >= ROWS) continue;
#pragma unroll
            for (int ci = 0; ci < CI; ++ci) {
                if (ci < groups) {
                    const int ch = lane + MATCH_TX * ci;
                    mc[rr * stride + ch] = v0[ri][ci].s1;
                    is[rr * stride + ch] = v0[ri][ci].z;
                    mc[rr * stride + half + ch] = v1[ri][ci].s1;
                    is[rr * stride + half + ch] = v1[ri][ci].z;
                }
            }
        }
        return;
    }
    constexpr int RI = (ROWS + NWAVES - 1) / NWAVES;
    constexpr int CI = (MAXCOLS + 2 * MATCH_TX - 1) / (2 * MATCH_TX);
    const int lane = threadIdx.x & (MATCH_TX - 1), wave = threadIdx.x / MATCH_TX;
    const int groups = (cols + 2 * MATCH_TX - 1) / (2 * MATCH_TX);
    WinStat v0[RI][CI], v1[RI][CI];
#pragma unroll
    for (int ri = 0; ri < RI; ++ri) {
        const int rr = wave + NWAVES * ri;
        const WinStat* srow = src + (size_t)clampi(gy0 + rr, 0, H - 1) * spitch;
#pragma unroll
        for (int ci = 0; ci < CI; ++ci) {
            const int cc = 2 * (lane + MATCH_TX * ci);
            v0[ri][ci] = srow[clampi(gx0 + min(cc, cols - 1), 0, W - 1)];
            v1[ri][ci] = srow[clampi(gx0 + min(cc + 1, cols - 1), 0, W - 1)];
        }
    }
#pragma unroll
    for (int ri = 0; ri < RI; ++ri) {
        const int rr = wave + NWAVES * ri;
        if (rr >= ROWS) continue;
#pragma unroll
        for (int ci = 0; ci < CI; ++ci) {
            if (ci < groups) {
                const int ch = lane + MATCH_TX * ci;
                mc[rr * stride + ch] = (v0[ri][ci].x - c) + v0[ri][ci].y;
                is[rr * stride + ch] = v0[ri][ci].z;
                mc[rr * stride + half + ch] = (v1[ri][ci].x - c) + v1[ri][ci].y;
                is[rr * stride + half + ch] = v1[ri][ci].z;
            }
        }
    }
}

// One window row: load the block's 2n+2 left values (centred by ca) and
// 2n+1+NC right values.
template <int NW, int NC, int LSTRIDE, int LHALF, int RSTRIDE, bool CENTRE = true>
__device__ __forceinline__ void load_row(const float* __restrict__ Ls, const float* __restrict__ Rs,
                                         int row, int ltx, int pa, int pb, float ca,
                                         float (&l)[2 * NW + 2], float (&r)[2 * NW + 1 + NC])
{
    const float* lr_ = Ls + row * LSTRIDE + ltx;
    const float* rr_ = Rs + row * RSTRIDE;
#pragma unroll
    for (int t = 0; t < 2 * NW + 2; ++t) {
        l[t] = lr_[(t & 1) ? LHALF + (t >> 1) : (t >> 1)];
        if constexpr (CENTRE) l[t] -= ca;
    }
#pragma unroll
    for (int u = 0; u < 2 * NW + 1 + NC; ++u) r[u] = (u & 1) ? rr_[pb + (u >> 1)] : rr_[pa + (u >> 1)];
}

// Window sums for one block and NC candidate slots.
//   lrow0   LDS row of the block's first window row
//   ltx     thread column index (the block's first window column is 2*ltx)
//   rcol0   logical LDS column of the right value that pairs with the first
//           window column at the LAST slot (largest z)
//   ca      the thread's left centring constant
// S[p][s]: p = 0 (row 0, col 0), 1 (row 0, col 1), 2 (row 1, col 0), 3 (row 1, col 1).
// Rows 1..2n feed both pixel rows (accumulated once: MC for the columns both
// pixel columns share, M0/M1 for each column's extra edge column); row 0 feeds
// only the upper pixels and row 2n+1 only the lower ones.
// CENTRE = false (uint8 levels): the values are used as staged, uncentred;
// every product and sum is then an exact integer below 2^24.
template <int NW, int NC, class G, bool CENTRE = true>
__device__ __forceinline__ void window_sums(const float* __restrict__ Ls, const float* __restrict__ Rs,
                                            int lrow0, int ltx, int rcol0, float ca, float (&S)[4][NC])
{
    constexpr int WN = G::WN;
    // right row: even logical offsets u come from base pa, odd ones from pb
    int pa, pb;
    if ((rcol0 & 1) == 0) {
        pa = rcol0 >> 1;
        pb = G::RHALF + (rcol0 >> 1);
    } else {
        pa = G::RHALF + (rcol0 >> 1);
        pb = (rcol0 + 1) >> 1;
    }
    float l[WN], r[WN + NC - 1];
    float MC[NC], M0[NC], M1[NC];
    // first row: upper pixels only
    load_row<NW, NC, G::LSTRIDE, G::LHALF, G::RSTRIDE, CENTRE>(Ls, Rs, lrow0, ltx, pa, pb, ca, l, r);
#pragma unroll
    for (int s = 0; s < NC; ++s) {
        const int o = NC - 1 - s;  // slot s pairs column t with right value t + o
        float c = 0.f;
#pragma unroll
        for (int t = 1; t < WN - 1; ++t) c = fmaf(l[t], r[t + o], c);
        S[0][s] = fmaf(l[0], r[o], c);
        S[1][s] = fmaf(l[WN - 1], r[WN - 1 + o], c);
        MC[s] = M0[s] = M1[s] = 0.f;
    }
    // shared rows
#pragma unroll 2
    for (int y = 1; y < WN - 1; ++y) {
        load_row<NW, NC, G::LSTRIDE, G::LHALF, G::RSTRIDE, CENTRE>(Ls, Rs, lrow0 + y, ltx, pa, pb, ca, l, r);
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            const int o = NC - 1 - s;
            float c = MC[s];
#pragma unroll
            for (int t = 1; t < WN - 1; ++t) c = fmaf(l[t], r[t + o], c);
            MC[s] = c;
            M0[s] = fmaf(l[0], r[o], M0[s]);
            M1[s] = fmaf(l[WN - 1], r[WN - 1 + o], M1[s]);
        }
    }
    // last row: lower pixels only
    load_row<NW, NC, G::LSTRIDE, G::LHALF, G::RSTRIDE, CENTRE>(Ls, Rs, lrow0 + WN - 1, ltx, pa, pb, ca, l, r);
#pragma unroll
    for (int s = 0; s < NC; ++s) {
        const int o = NC - 1 - s;
        float c = 0.f;
#pragma unroll
        for (int t = 1; t < WN - 1; ++t) c = fmaf(l[t], r[t + o], c);
        const float m0 = MC[s] + M0[s], m1 = MC[s] + M1[s];
        S[0][s] += m0;
        S[1][s] += m1;
        S[2][s] = m0 + fmaf(l[0], r[o], c);
        S[3][s] = m1 + fmaf(l[WN - 1], r[WN - 1 + o], c);
    }
}

// Per-block state: the block's pixel coordinates (clamped into the image), which
// of its pixels exist, each pixel's candidate interval, the block's first slot.
struct BlockState {
    int ia, ib, ja, jb;
    bool act[4];
    int lo[4], hi[4];
    int zs;
};

// One TILE_H x TILE_W tile (tile column bx, tile row by) of one level.  Called
// by the per-level kernel below and by the stage-batched kernel; every
// thread of the workgroup must call it (it synchronises the workgroup).
// SL selects where the right statistics come from: staged in LDS with the right
// tile (1), or read by each thread from global memory (0).
// Pixel rows of a tile: 2 for the candidate split, else one block row (two
// pixel rows) per wave: 8 for the usual 4 waves, 16 for the tall shape (8 waves).
template <int SPLIT, int TY = MATCH_TY>
struct TileRows {
    static constexpr int value = SPLIT ? 2 : 2 * TY;
};

template <typename T, int NW, int NC, int MODE, int SPLIT, int SL, bool CV = false, int TY = MATCH_TY,
          bool SHORT = false>
__device__ __forceinline__ void match_tile(
    const MatchArgs& a, int bx, int by,
    MatchSmem<NW, ChunkOf<MODE, SHORT>::value, TileRows<SPLIT, TY>::value, SL>& sm)
{
    constexpr int CH = ChunkOf<MODE, SHORT>::value;
    constexpr int BY = 1;
    using G = Geo<NW, CH, TileRows<SPLIT, TY>::value>;
    static_assert(!SPLIT || MODE != MODE_SOFT, "the soft level needs every slot of a block in one thread");
    static_assert(!SPLIT || TY == MATCH_TY, "the candidate split combines the winners of four waves");
    constexpr int NN = (2 * NW + 1) * (2 * NW + 1);
    constexpr float Nf = (float)NN;
    // A block of a restricted search scores the candidate slots [zs, zs + NCF).
    // Unsplit, that is one window of NC = NCF slots; split (RSPLIT), the span is
    // covered by windows of NC slots, one per wave (NCX: the span rounded up to
    // whole windows), so every wave's chain is a fraction of the block's.
    // Each slot's score is computed by the same operations either way.
    constexpr bool RSPLIT = SPLIT && MODE == MODE_REFINE;
    const int NCF = RSPLIT ? slots_for_radius(a.r) : NC;
    const int NCX = RSPLIT ? (NCF + NC - 1) / NC * NC : NC;
    const int STEP = (MODE == MODE_FULL) ? CH : (CH - NCX + 1);
    static_assert(MODE != MODE_FULL || CH % NC == 0, "full search steps must tile a chunk");
    static_assert(CH >= NC, "a chunk must hold one slot window");
    static_assert(MODE == MODE_FULL || (MSIBM_MAX_DISP - 1) / (CH - 4 * NC + 1) < 32,
                  "chunk mask must hold every chunk");

    const T* __restrict__ Lg = static_cast<const T*>(a.L);
    const T* __restrict__ Rg = static_cast<const T*>(a.R);
    const int tx = threadIdx.x & (MATCH_TX - 1), ty = threadIdx.x / MATCH_TX;
    // block row of the thread: one per wave, or (SPLIT) the tile's single block
    // row shared by all waves, which then take every 4th candidate window
    const int tyb = SPLIT ? 0 : ty;
    const int x0 = bx * TILE_W, y0 = by * G::TH;
    const int j0 = x0 + 2 * tx;

    // per block: coordinates, candidate intervals and first slot
    BlockState bs[BY];
#pragma unroll
    for (int b = 0; b < BY; ++b) {
        BlockState& q = bs[b];
        const int i0 = y0 + 2 * tyb + TILE_H1 * b;
        q.act[0] = i0 < a.H && j0 < a.W;
        q.act[1] = i0 < a.H && j0 + 1 < a.W;
        q.act[2] = i0 + 1 < a.H && j0 < a.W;
        q.act[3] = i0 + 1 < a.H && j0 + 1 < a.W;
        // clamped coordinates keep every load inside the image even for pixels
        // of a block that hang over the image edge
        q.ia = min(i0, a.H - 1);
        q.ib = min(i0 + 1, a.H - 1);
        q.ja = min(j0, a.W - 1);
        q.jb = min(j0 + 1, a.W - 1);
        const int jp[4] = {q.ja, q.jb, q.ja, q.jb};
        if (MODE == MODE_FULL) {
            q.zs = 0;
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                q.lo[p] = 0;
                q.hi[p] = min(a.Dk - 1, jp[p]);
            }
        } else {
            // out-of-range prior values (never produced by the coarser level)
            // are clamped so that every index below stays inside its buffer
            const int dh = clampi(2 * (int)a.prior[(size_t)(q.ia >> 1) * a.ppitch + (q.ja >> 1)], 0, a.Dk - 1);
            q.zs = (dh <= j0) ? dh - a.r : j0 + 2 - NCF;
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const int c = min(dh, jp[p]);
                q.lo[p] = max(0, c - a.r);
                q.hi[p] = min(min(a.Dk - 1, jp[p]), c + a.r);
            }
        }
    }
    // right centring value: one pixel per 16-row band of tiles, whatever the
    // tile height (2, 8 or 16 rows), so that every kernel shape rounds the
    // scores identically
    const int cy = min((y0 & ~15) + 8, a.H - 1), cx = min(x0 + TILE_W / 2, a.W - 1);
    // (uint8 levels are not centred: their sums are exact integers)
    constexpr bool U8 = std::is_same<T, uint8_t>::value;
    const float cR = U8 ? 0.f : to_f(Rg[(size_t)cy * a.pitch + cx]);

    // Fixed window (restricted searches whose whole candidate range fits one
    // chunk): every block's slots lie in [zlo_f, zhi_f], so both tiles are
    // staged at once, before any block's prior is known, and no workgroup-wide
    // range is needed.
    const int zlo_f = min(-a.r, 2 - NCF), zhi_f = a.Dk - 1 - a.r;
    const bool fixw = MODE != MODE_FULL && (a.variant & VARIANT_FIXW) && zhi_f - zlo_f + 1 <= STEP;
    if (fixw) {
        const int ztop = zhi_f + NCX - 1;
        stage_pair<T, G::LROWS, G::LCOLS, G::RCOLS, TY>(sm.Ls, G::LSTRIDE, G::LHALF, sm.Rs, G::RSTRIDE, G::RHALF,
                                                        Lg, Rg, a.pitch, a.H, a.W, y0 - NW, x0 - NW, G::LCOLS,
                                                        x0 - NW - ztop, TILE_W + 2 * NW + (ztop - zlo_f), cR);
    } else {
        // left tile (uncentred: each thread centres its own windows)
        stage_tile<T, G::LROWS, G::LCOLS, TY>(sm.Ls, G::LSTRIDE, G::LHALF, Lg, a.pitch, a.H, a.W, y0 - NW,
                                              x0 - NW, G::LCOLS, 0.f);
    }

    // workgroup-wide candidate range; for a restricted search also the set of
    // right-image chunks some block of the tile needs
    if (!fixw) {
    if (threadIdx.x == 0) {
        sm.lo = 0x7fffffff;
        sm.hi = -0x7fffffff;
        sm.mask = 0u;
    }
    __syncthreads();
    if (MODE == MODE_FULL) {
        if (threadIdx.x == 0) {
            sm.lo = 0;
            sm.hi = min(a.Dk - 1, min(x0 + TILE_W, a.W) - 1);
        }
    } else {
#pragma unroll
        for (int b = 0; b < BY; ++b)
            if (bs[b].act[0]) {
                atomicMin(&sm.lo, bs[b].zs);
                atomicMax(&sm.hi, bs[b].zs);
            }
    }
    __syncthreads();
    if (MODE != MODE_FULL) {
#pragma unroll
        for (int b = 0; b < BY; ++b)
            if (bs[b].act[0]) atomicOr(&sm.mask, 1u << ((bs[b].zs - sm.lo) / STEP));
    }
    __syncthreads();
    }
    const int zlo = fixw ? zlo_f : sm.lo, zhi = fixw ? zhi_f : sm.hi;
    const unsigned mask = (MODE == MODE_FULL || fixw) ? 0xffffffffu : sm.mask;

    constexpr int SB = (MODE == MODE_SOFT) ? BY : 1, SN = (MODE == MODE_SOFT) ? NC : 1;
    float best[BY][4], rho_keep[SB][4][SN];
    int bz[BY][4];
#pragma unroll
    for (int b = 0; b < BY; ++b)
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            best[b][p] = -3.f;
            bz[b][p] = 0;
        }

    for (int zc = zlo, ci = 0; zc <= zhi; zc += STEP, ++ci) {
        if (MODE != MODE_FULL && !((mask >> ci) & 1u)) continue;
        // largest candidate slot of this chunk: the right tile's column 0 pairs
        // with the first window column of that slot, and statistics column 0 is
        // the window centre of the tile's first pixel column at that slot
        const int ztop = min(zc + CH - 1, zhi + NCX - 1);
        if (zc != zlo) __syncthreads();  // previous chunk fully consumed
        if (!fixw)
            stage_tile<T, G::LROWS, G::RCOLS, TY>(sm.Rs, G::RSTRIDE, G::RHALF, Rg, a.pitch, a.H, a.W, y0 - NW,
                                                  x0 - NW - ztop, TILE_W + 2 * NW + (ztop - zc), cR);
        if (SL)
            stage_stats<G::TH, G::SCOLS, TY, U8>(sm.Sm, sm.Si, G::SSTRIDE, G::SHALF, a.statR, a.spitch, a.H,
                                                 a.W, y0, x0 - ztop, TILE_W + (ztop - zc), cR);
        __syncthreads();

#pragma unroll
        for (int b = 0; b < BY; ++b) {
            const BlockState& q = bs[b];
            if (!q.act[0]) continue;
            // slot windows of this block in this chunk
            int w_first, w_last;
            if (MODE == MODE_FULL) {
                w_first = zc;
                w_last = min(zc + CH - 1, max(q.hi[0], q.hi[1]));
            } else {
                w_first = q.zs;
                w_last = (q.zs >= zc && q.zs < zc + STEP) ? q.zs + NCX - NC : q.zs - 1;
            }
            if (w_first > w_last) continue;
            // left statistics.  Float levels: the block's left windows are
            // centred on its first pixel's window mean, ndl = -N (mu_l - ca).
            // uint8 levels: ndl = -S1_l (the exact window sum), invl = 1/(sd N)
            const size_t lo0 = (size_t)q.ia * a.spitch, lo1 = (size_t)q.ib * a.spitch;
            const size_t so[4] = {lo0 + q.ja, lo0 + q.jb, lo1 + q.ja, lo1 + q.jb};
            float ca = 0.f;
            float ndl[4], invl[4];
            if constexpr (U8) {
                const WinStatU8* s8 = reinterpret_cast<const WinStatU8*>(a.statL);
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    const WinStatU8 st = s8[so[p]];
                    ndl[p] = -st.s1;
                    invl[p] = st.z * (1.f / Nf);
                }
            } else {
                WinStat stl[4];
#pragma unroll
                for (int p = 0; p < 4; ++p) stl[p] = a.statL[so[p]];
                ca = stl[0].x;
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    ndl[p] = -Nf * ((stl[p].x - ca) + stl[p].y);
                    invl[p] = stl[p].z;
                }
            }
            const int lrow0 = 2 * tyb + TILE_H1 * b;
            for (int wz = w_first + (SPLIT ? ty * NC : 0); wz <= w_last; wz += NC * (SPLIT ? MATCH_TY : 1)) {
                float S[4][NC];
                const int rcol0 = 2 * tx + (ztop - wz) - (NC - 1);
                window_sums<NW, NC, G, !U8>(sm.Ls, sm.Rs, lrow0, tx, rcol0, ca, S);
                // right statistics of columns c0 - q, q = 0..NC (c0 = the centre
                // of pixel column j0 + 1 at slot 0): pixel column cp at slot s is
                // q = s + 1 - cp
                const int c0 = 2 * tx + (ztop - wz) + 1;
                const int be = (c0 & 1) ? G::SHALF + (c0 >> 1) : (c0 >> 1);      // q even
                const int bo = (c0 & 1) ? (c0 >> 1) : G::SHALF + (c0 >> 1) - 1;  // q odd
                // right statistics from global memory: every load of the window
                // issued before the first use, so they share one latency
                using SR = typename std::conditional<U8, WinStatU8, WinStat>::type;
                SR stg[2][SL ? 1 : NC + 1];
                if (!SL) {
#pragma unroll
                    for (int rowp = 0; rowp < 2; ++rowp) {
                        // columns j0 + 1 - wz - q of pixel row ia or ib
                        const SR* srow = reinterpret_cast<const SR*>(a.statR) + (size_t)(rowp ? q.ib : q.ia) * a.spitch;
#pragma unroll
                        for (int qq = 0; qq <= NC; ++qq) stg[rowp][SL ? 0 : qq] = srow[clampi(j0 + 1 - wz - qq, 0, a.W - 1)];
                    }
                    asm volatile("" ::: "memory");  // keep the loads ahead of their uses
                }
#pragma unroll
                for (int rowp = 0; rowp < 2; ++rowp) {
                    float smc[NC + 1], sis[NC + 1];
                    int smi[NC + 1];  // uint8: the exact right window sums as integers
                    if (SL) {
                        const int so = (lrow0 + rowp) * G::SSTRIDE;
#pragma unroll
                        for (int qq = 0; qq <= NC; ++qq) {
                            const int o = so + ((qq & 1) ? bo - (qq >> 1) : be - (qq >> 1));
                            smc[qq] = sm.Sm[o];
                            sis[qq] = sm.Si[o];
                            if constexpr (U8) smi[qq] = (int)smc[qq];
                        }
                    } else {
#pragma unroll
                        for (int qq = 0; qq <= NC; ++qq) {
                            const SR st = stg[rowp][SL ? 0 : qq];
                            if constexpr (U8) {
                                smc[qq] = st.s1;
                                smi[qq] = (int)st.s1;
                            } else {
                                smc[qq] = (st.x - cR) + st.y;
                            }
                            sis[qq] = st.z;
                        }
                    }
#pragma unroll
                    for (int cp = 0; cp < 2; ++cp) {
                        const int p = 2 * rowp + cp;
#pragma unroll
                        for (int s = 0; s < NC; ++s) {
                            const int z = wz + s;
                            const int qq = s + 1 - cp;
                            float C;
                            if constexpr (U8) {
                                // C N = N S - S1_l S1_r in 32-bit integers: every factor
                                // is an integer below 2^24 and the difference lies within
                                // +-2^31 up to 13x13 windows, so C N is exact and rounds
                                // to float once
                                const int ncn = __mul24((int)ndl[p], smi[qq]) +
                                                (int)__umul24((unsigned)NN, (unsigned)(int)S[p][s]);
                                C = (float)ncn;
                            } else {
                                C = fmaf(ndl[p], smc[qq], S[p][s]);
                            }
                            float rho = C * invl[p] * sis[qq];
                            rho = fminf(fmaxf(rho, -1.f), 1.f);
                            const bool ok = (z >= q.lo[p]) && (z <= q.hi[p]);
                            if (CV && ok && q.act[p])
                                a.costvol[((size_t)(rowp ? q.ib : q.ia) * a.W + (cp ? q.jb : q.ja)) * a.Dk + z] = rho;
                            if (MODE == MODE_SOFT) rho_keep[MODE == MODE_SOFT ? b : 0][p][MODE == MODE_SOFT ? s : 0] = ok ? rho : -1e30f;
                            if (ok && rho > best[b][p]) {
                                best[b][p] = rho;
                                bz[b][p] = z;
                            }
                        }
                    }
                }
            }
        }
    }
    if (SPLIT) {
        // every wave scored a disjoint set of candidate windows for the same
        // pixels: combine in LDS, highest score, then lowest z
        float* cb = sm.cmb;                                 // [wave][pixel][lane]
        int* cz = reinterpret_cast<int*>(sm.cmb) + MATCH_THREADS * 4;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            cb[(ty * 4 + p) * MATCH_TX + tx] = best[0][p];
            cz[(ty * 4 + p) * MATCH_TX + tx] = bz[0][p];
        }
        __syncthreads();
        if (ty == 0) {
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int w = 1; w < MATCH_TY; ++w) {
                    const float v = cb[(w * 4 + p) * MATCH_TX + tx];
                    const int z = cz[(w * 4 + p) * MATCH_TX + tx];
                    if (v > best[0][p] || (v == best[0][p] && z < bz[0][p])) {
                        best[0][p] = v;
                        bz[0][p] = z;
                    }
                }
        }
    }
#pragma unroll
    for (int b = 0; b < BY; ++b) {
        if (SPLIT && ty != 0) break;
        const BlockState& q = bs[b];
        const int ip[4] = {q.ia, q.ia, q.ib, q.ib};
        const int jp[4] = {q.ja, q.jb, q.ja, q.jb};
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            if (!q.act[p]) continue;
            const size_t o = (size_t)ip[p] * a.opitch + jp[p];
            a.d_out[o] = (int16_t)bz[b][p];
            if (a.c_out) a.c_out[o] = best[b][p];
            if (MODE == MODE_SOFT) {
                float se = 0.f, sz = 0.f;
#pragma unroll
                for (int s = 0; s < SN; ++s) {
                    const float e = __expf((rho_keep[MODE == MODE_SOFT ? b : 0][p][s] - best[b][p]) * a.inv_tau);
                    se += e;
                    sz = fmaf(e, (float)(q.zs + s), sz);
                }
                a.soft_out[o] = sz / se;
            }
        }
    }
    __syncthreads();  // LDS may be reused by the caller's next tile
}

template <typename T, int NW, int NC, int MODE, int SPLIT, int SL, int TY = MATCH_TY, bool SHORT = false>
__global__ __launch_bounds__(MATCH_TX * TY, (MODE == MODE_REFINE && NC <= 7) ? 3 : 1) void match_kernel(MatchArgs a)
{
    __shared__ MatchSmem<NW, ChunkOf<MODE, SHORT>::value, TileRows<SPLIT, TY>::value, SL> sm;
    int bx = blockIdx.x, by = blockIdx.y;
    tile_of(a.variant, &bx, &by);
    match_tile<T, NW, NC, MODE, SPLIT, SL, false, TY, SHORT>(a, bx, by, sm);
}

// The same search writing every scored candidate's score to a.costvol (a
// testing aid: its own instantiation, so the production kernels carry no trace
// of it).
template <typename T, int NW, int NC, int MODE>
__global__ __launch_bounds__(MATCH_THREADS) void match_costvol_kernel(MatchArgs a)
{
    __shared__ MatchSmem<NW, ChunkOf<MODE>::value, TILE_H1, 0> sm;
    match_tile<T, NW, NC, MODE, 0, 0, true>(a, blockIdx.x, blockIdx.y, sm);
}

template <typename T, int NW, int NC, int MODE, int SPLIT, int TY, bool SHORT>
static hipError_t launch_shape_ts(const MatchArgs& a, hipStream_t s)
{
    constexpr int TH = TileRows<SPLIT, TY>::value;
    dim3 grid((a.W + TILE_W - 1) / TILE_W, (a.H + TH - 1) / TH, 1);
    // statistics staged in LDS is a full-search shape only: a restricted search
    // reads a few statistics per pixel, and its wide right tile leaves no LDS for
    // them
    if (MODE == MODE_FULL && (a.variant & VARIANT_STATS_LDS))
        hipLaunchKernelGGL((match_kernel<T, NW, NC, MODE, SPLIT, MODE == MODE_FULL ? 1 : 0, TY, SHORT>), grid,
                           dim3(MATCH_TX * TY), 0, s, a);
    else
        hipLaunchKernelGGL((match_kernel<T, NW, NC, MODE, SPLIT, 0, TY, SHORT>), grid, dim3(MATCH_TX * TY), 0, s,
                           a);
    return hipGetLastError();
}

// Tile height (the tall shape: 16 rows, 8 waves; not with the candidate split)
// and chunk length from the variant bits.
template <typename T, int NW, int NC, int MODE, int SPLIT>
static hipError_t launch_shape(const MatchArgs& a, hipStream_t s)
{
    const bool shrt = (a.variant & VARIANT_SHORT) != 0;
    if constexpr (!SPLIT) {
        if (a.variant & VARIANT_TALL)
            return shrt ? launch_shape_ts<T, NW, NC, MODE, SPLIT, 2 * MATCH_TY, true>(a, s)
                        : launch_shape_ts<T, NW, NC, MODE, SPLIT, 2 * MATCH_TY, false>(a, s);
    }
    return shrt ? launch_shape_ts<T, NW, NC, MODE, SPLIT, MATCH_TY, true>(a, s)
                : launch_shape_ts<T, NW, NC, MODE, SPLIT, MATCH_TY, false>(a, s);
}

// Slots per wave of a split restricted search: a quarter of the block's span,
// rounded up, so the four waves cover it with one window each.
constexpr int split_slots(int nc) { return (nc + MATCH_TY - 1) / MATCH_TY; }

template <typename T, int NW, int NC, int MODE>
static hipError_t launch_one(const MatchArgs& a, hipStream_t s)
{
    if (a.costvol) {
        if (MODE == MODE_SOFT) return hipErrorInvalidValue;
        dim3 grid((a.W + TILE_W - 1) / TILE_W, (a.H + TILE_H1 - 1) / TILE_H1, 1);
        hipLaunchKernelGGL((match_costvol_kernel<T, NW, NC, MODE == MODE_SOFT ? MODE_REFINE : MODE>), grid,
                           dim3(MATCH_THREADS), 0, s, a);
        return hipGetLastError();
    }
    if (MODE == MODE_FULL && (a.variant & VARIANT_SPLIT))
        return launch_shape<T, NW, NC, MODE, MODE == MODE_FULL ? 1 : 0>(a, s);
    if (MODE == MODE_REFINE && (a.variant & VARIANT_SPLIT)) {
        if (slots_for_radius(a.r) != NC) return hipErrorInvalidValue;  // the span the kernel splits
        return launch_shape<T, NW, split_slots(NC), MODE, MODE == MODE_REFINE ? 1 : 0>(a, s);
    }
    return launch_shape<T, NW, NC, MODE, 0>(a, s);
}

template <typename T, int NW>
static hipError_t dispatch_nc(int mode, int nc, const MatchArgs& a, hipStream_t s)
{
    if (mode == MODE_FULL) return launch_one<T, NW, FULL_NC, MODE_FULL>(a, s);
    if (mode == MODE_REFINE) {
        switch (nc) {
            case 2: return launch_one<T, NW, 2, MODE_REFINE>(a, s);
            case 3: return launch_one<T, NW, 3, MODE_REFINE>(a, s);
            case 5: return launch_one<T, NW, 5, MODE_REFINE>(a, s);
            case 7: return launch_one<T, NW, 7, MODE_REFINE>(a, s);
            case 9: return launch_one<T, NW, 9, MODE_REFINE>(a, s);
        }
        return hipErrorInvalidValue;
    }
    switch (nc) {
        case 3: return launch_one<T, NW, 3, MODE_SOFT>(a, s);
        case 5: return launch_one<T, NW, 5, MODE_SOFT>(a, s);
        case 7: return launch_one<T, NW, 7, MODE_SOFT>(a, s);
        case 9: return launch_one<T, NW, 9, MODE_SOFT>(a, s);
    }
    return hipErrorInvalidValue;
}

template <int NW>
static hipError_t dispatch_match(int dtype, int mode, int nc, const MatchArgs& a, hipStream_t s)
{
    if (dtype == 0 && mode == MODE_SOFT) return hipErrorInvalidValue;  // soft mode takes float images
    if (dtype == 0) return dispatch_nc<uint8_t, NW>(mode, nc, a, s);
    return dispatch_nc<float, NW>(mode, nc, a, s);
}

// Matching of several (pair, level) segments of one mode and element type in
// one launch: the level's arguments come from its pair's level descriptors.
template <typename T, int NW, int NC, int MODE, int SL>
__global__ __launch_bounds__(MATCH_THREADS, (MODE == MODE_REFINE && NC <= 7) ? 3 : 1) void match_multi_kernel(MultiArgs a)
{
    __shared__ MatchSmem<NW, ChunkOf<MODE>::value, TILE_H1, SL> sm;
    const Segment s = a.segs[segment_of(a.segs, a.nseg, blockIdx.x)];
    const LevelDesc* lv = a.levels + a.level_base[s.pair];
    const LevelDesc& L = lv[s.level];
    MatchArgs m{};
    m.L = L.img[0];
    m.R = L.img[1];
    m.H = L.H;
    m.W = L.W;
    m.pitch = L.pitch;
    m.statL = L.stat[0];
    m.statR = L.stat[1];
    m.spitch = L.W;
    m.Dk = L.Dk;
    if (MODE != MODE_FULL) {
        const LevelDesc& C = lv[s.level + 1];
        m.prior = C.map;
        m.Hc = C.H;
        m.Wc = C.W;
        m.ppitch = C.W;
    }
    m.r = (MODE == MODE_SOFT) ? a.rs : a.r;
    m.d_out = L.raw ? L.raw : L.map;  // with the median the filter fills L.map
    m.c_out = L.raw ? L.mcost : L.cost;
    m.soft_out = L.soft;
    m.opitch = L.W;
    m.inv_tau = a.inv_tau;
    m.variant = a.variant;
    const int t = blockIdx.x - s.task0;
    match_tile<T, NW, NC, MODE, 0, SL>(m, t % s.tiles_x, t / s.tiles_x, sm);
}

// Statistics placement per mode: staged in LDS for the full search (every
// staged column serves all candidates), read from memory for restricted ones.
template <typename T, int NW, int NC, int MODE>
static hipError_t launch_multi_one(const MultiArgs& a, int blocks, hipStream_t s)
{
    constexpr int SL = (MODE == MODE_FULL) ? 1 : 0;
    hipLaunchKernelGGL((match_multi_kernel<T, NW, NC, MODE, SL>), dim3(blocks), dim3(MATCH_THREADS), 0, s, a);
    return hipGetLastError();
}

template <typename T, int NW>
static hipError_t dispatch_multi_nc(int mode, int nc, const MultiArgs& a, int blocks, hipStream_t s)
{
    if (mode == MODE_FULL) return launch_multi_one<T, NW, FULL_NC, MODE_FULL>(a, blocks, s);
    if (mode == MODE_REFINE) {
        switch (nc) {
            case 2: return launch_multi_one<T, NW, 2, MODE_REFINE>(a, blocks, s);
            case 3: return launch_multi_one<T, NW, 3, MODE_REFINE>(a, blocks, s);
            case 5: return launch_multi_one<T, NW, 5, MODE_REFINE>(a, blocks, s);
            case 7: return launch_multi_one<T, NW, 7, MODE_REFINE>(a, blocks, s);
            case 9: return launch_multi_one<T, NW, 9, MODE_REFINE>(a, blocks, s);
        }
        return hipErrorInvalidValue;
    }
    if constexpr (std::is_same<T, float>::value) {
        switch (nc) {
            case 3: return launch_multi_one<T, NW, 3, MODE_SOFT>(a, blocks, s);
            case 5: return launch_multi_one<T, NW, 5, MODE_SOFT>(a, blocks, s);
            case 7: return launch_multi_one<T, NW, 7, MODE_SOFT>(a, blocks, s);
            case 9: return launch_multi_one<T, NW, 9, MODE_SOFT>(a, blocks, s);
        }
    }
    return hipErrorInvalidValue;
}

template <int NW>
static hipError_t dispatch_match_multi(int dtype, int mode, int nc, const MultiArgs& a, int blocks, hipStream_t s)
{
    if (blocks < 1 || a.nseg < 1) return hipErrorInvalidValue;
    if (dtype == 0) return dispatch_multi_nc<uint8_t, NW>(mode, nc, a, blocks, s);
    return dispatch_multi_nc<float, NW>(mode, nc, a, blocks, s);
}

}  // namespace msibm
