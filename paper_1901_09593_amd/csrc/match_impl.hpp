// ZNCC winner-take-all matching of one pyramid level (Eqs. 1-4 and 8-9), with
// the soft-argmax of the differentiable finest level.
//
// Work split.  A workgroup of 4 waves covers a TILE_H x TILE_W (8 x 128) pixel
// tile; each thread owns one 2x2 pixel block.  The left tile with its window
// halo sits in LDS once; the right image is staged in LDS one CHUNK of candidate
// disparities at a time.  For a block and a window of NC consecutive candidate
// slots, the thread walks the 2n+2 window rows: it loads the 2n+2 left values
// and 2n+1+NC right values of the row from LDS and accumulates, per slot, the
// products shared by both pixel columns once plus one edge product per column.
// That costs (2n+2)^2 fused multiply-adds per slot for the block's 4 window
// sums instead of 4 (2n+1)^2 for four independent windows.  The cross sum is
// then normalised with per-pixel statistics (window mean, 1/sqrt(A)) and the
// running winner-take-all keeps the lowest z among equal scores.
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
//
// Precision.  The score is invariant to a constant offset of either window, so
// each thread centres its left windows on a = the window mean of its block's
// first pixel (subtracted as the left values are loaded), and the right tile is
// centred on one right pixel of the tile (cR, subtracted when staging).  The
// products then stay near the window's own spread and the cross term
//   C = sum (l - a)(r - cR) - N (mu_l - a)(mu_r - cR)
// cancels little; the window means carry their float rounding remainder so
// (mu - a) and (mu - cR) keep their low bits.  rho = C * invsd_l * invsd_r,
// clamped to [-1, 1].
#pragma once

#include "common.hpp"

namespace msibm {

template <int NW>
struct Geo {
    static constexpr int WN = 2 * NW + 2;          // rows/cols spanned by a block's windows
    static constexpr int LROWS = TILE_H + 2 * NW;  // LDS rows (both views)
    static constexpr int LCOLS = TILE_W + 2 * NW;  // left tile logical width
    static constexpr int LHALF = (LCOLS + 1) / 2;
    static constexpr int LSTRIDE = 2 * LHALF + 1;
    static constexpr int RCOLS = TILE_W + 2 * NW + CHUNK - 1;
    static constexpr int RHALF = (RCOLS + 1) / 2;
    static constexpr int RSTRIDE = 2 * RHALF + 1;
};

__device__ __forceinline__ int split_pos(int c, int half) { return (c & 1) ? half + (c >> 1) : (c >> 1); }

// Stage rows [gy0, gy0+rows) x cols [gx0, gx0+cols) of `src` (clamped to the
// image) into LDS in split layout, centred by c.  Each wave takes whole rows and
// its lanes consecutive columns, so global reads coalesce.
template <typename T>
__device__ __forceinline__ void stage_tile(float* dst, int stride, int half, const T* __restrict__ src,
                                           int pitch, int H, int W, int gy0, int gx0, int rows, int cols,
                                           float c)
{
    const int lane = threadIdx.x & (MATCH_TX - 1), wave = threadIdx.x / MATCH_TX;
    for (int rr = wave; rr < rows; rr += MATCH_TY) {
        const T* srow = src + (size_t)clampi(gy0 + rr, 0, H - 1) * pitch;
        float* drow = dst + rr * stride;
        for (int cc = lane; cc < cols; cc += MATCH_TX)
            drow[split_pos(cc, half)] = to_f(srow[clampi(gx0 + cc, 0, W - 1)]) - c;
    }
}

// Window sums for one block and NC candidate slots.
//   lrow0   LDS row of the block's first window row (2*ty)
//   ltx     thread column index (the block's first window column is 2*ltx)
//   rcol0   logical LDS column of the right value that pairs with the first
//           window column at the LAST slot (largest z)
//   ca      the thread's left centring constant
// S[p][s]: p = 0 (row 0, col 0), 1 (row 0, col 1), 2 (row 1, col 0), 3 (row 1, col 1).
// One window row: load the block's 2n+2 left values and 2n+1+NC right values.
template <int NW, int NC>
__device__ __forceinline__ void load_row(const float* __restrict__ Ls, const float* __restrict__ Rs,
                                         int row, int ltx, int pa, int pb, float ca,
                                         float (&l)[2 * NW + 2], float (&r)[2 * NW + 1 + NC])
{
    using G = Geo<NW>;
    const float* lr_ = Ls + row * G::LSTRIDE + ltx;
    const float* rr_ = Rs + row * G::RSTRIDE;
#pragma unroll
    for (int t = 0; t < 2 * NW + 2; ++t) l[t] = lr_[(t & 1) ? G::LHALF + (t >> 1) : (t >> 1)] - ca;
#pragma unroll
    for (int u = 0; u < 2 * NW + 1 + NC; ++u) r[u] = (u & 1) ? rr_[pb + (u >> 1)] : rr_[pa + (u >> 1)];
}

// Window sums for one block and NC candidate slots.
//   lrow0   LDS row of the block's first window row (2*ty)
//   ltx     thread column index (the block's first window column is 2*ltx)
//   rcol0   logical LDS column of the right value that pairs with the first
//           window column at the LAST slot (largest z)
//   ca      the thread's left centring constant
// S[p][s]: p = 0 (row 0, col 0), 1 (row 0, col 1), 2 (row 1, col 0), 3 (row 1, col 1).
// Rows 1..2n feed both pixel rows (accumulated once: MC for the columns both
// pixel columns share, M0/M1 for each column's extra edge column); row 0 feeds
// only the upper pixels (T0/T1) and row 2n+1 only the lower ones (B0/B1).
template <int NW, int NC>
__device__ __forceinline__ void window_sums(const float* __restrict__ Ls, const float* __restrict__ Rs,
                                            int lrow0, int ltx, int rcol0, float ca, float (&S)[4][NC])
{
    using G = Geo<NW>;
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
    load_row<NW, NC>(Ls, Rs, lrow0, ltx, pa, pb, ca, l, r);
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
        load_row<NW, NC>(Ls, Rs, lrow0 + y, ltx, pa, pb, ca, l, r);
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
    load_row<NW, NC>(Ls, Rs, lrow0 + WN - 1, ltx, pa, pb, ca, l, r);
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

template <typename T, int NW, int NC, int MODE>
__global__ __launch_bounds__(MATCH_THREADS) void match_kernel(MatchArgs a)
{
    using G = Geo<NW>;
    constexpr float Nf = (float)((2 * NW + 1) * (2 * NW + 1));
    constexpr int STEP = (MODE == MODE_FULL) ? CHUNK : (CHUNK - NC + 1);
    static_assert(MODE != MODE_FULL || CHUNK % NC == 0, "full search steps must tile a chunk");

    __shared__ float Ls[G::LROWS * G::LSTRIDE];
    __shared__ float Rs[G::LROWS * G::RSTRIDE];
    __shared__ int s_lo, s_hi;
    __shared__ unsigned s_mask;

    const T* __restrict__ Lg = static_cast<const T*>(a.L);
    const T* __restrict__ Rg = static_cast<const T*>(a.R);
    const int tx = threadIdx.x & (MATCH_TX - 1), ty = threadIdx.x / MATCH_TX;
    const int x0 = blockIdx.x * TILE_W, y0 = blockIdx.y * TILE_H;
    const int i0 = y0 + 2 * ty, j0 = x0 + 2 * tx;
    const bool act[4] = {i0 < a.H && j0 < a.W, i0 < a.H && j0 + 1 < a.W,
                         i0 + 1 < a.H && j0 < a.W, i0 + 1 < a.H && j0 + 1 < a.W};
    const bool any = act[0];
    // clamped coordinates: every load below stays inside the image even for
    // pixels of a block that hang over the image edge
    const int ia = min(i0, a.H - 1), ib = min(i0 + 1, a.H - 1);
    const int ja = min(j0, a.W - 1), jb = min(j0 + 1, a.W - 1);
    const int ip[4] = {ia, ia, ib, ib};
    const int jp[4] = {ja, jb, ja, jb};

    // candidate interval of each pixel and the block's first slot
    int lo[4], hi[4], zs = 0;
    if (MODE == MODE_FULL) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            lo[p] = 0;
            hi[p] = min(a.Dk - 1, jp[p]);
        }
    } else {
        int dh = 0;
        // out-of-range prior values (never produced by the coarser level) are
        // clamped so that every index below stays inside its buffer
        if (any) dh = clampi(2 * (int)a.prior[(size_t)(ia >> 1) * a.ppitch + (ja >> 1)], 0, a.Dk - 1);
        zs = (dh <= j0) ? dh - a.r : j0 + 2 - NC;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int c = min(dh, jp[p]);
            lo[p] = max(0, c - a.r);
            hi[p] = min(min(a.Dk - 1, jp[p]), c + a.r);
        }
    }

    // workgroup-wide candidate range; for a restricted search also the set of
    // right-image chunks some block of the tile needs
    if (threadIdx.x == 0) {
        s_lo = 0x7fffffff;
        s_hi = -0x7fffffff;
        s_mask = 0u;
    }
    __syncthreads();
    if (MODE == MODE_FULL) {
        if (threadIdx.x == 0) {
            s_lo = 0;
            s_hi = min(a.Dk - 1, min(x0 + TILE_W, a.W) - 1);
        }
    } else if (any) {
        atomicMin(&s_lo, zs);
        atomicMax(&s_hi, zs);
    }
    __syncthreads();
    const int zlo = s_lo, zhi = s_hi;
    if (MODE != MODE_FULL && any) atomicOr(&s_mask, 1u << ((zs - zlo) / STEP));
    __syncthreads();
    const unsigned mask = (MODE == MODE_FULL) ? 0xffffffffu : s_mask;

    // right-tile centring constant (offsets do not change the score)
    const int cy = min(y0 + TILE_H / 2, a.H - 1), cx = min(x0 + TILE_W / 2, a.W - 1);
    const float cR = to_f(Rg[(size_t)cy * a.pitch + cx]);
    stage_tile<T>(Ls, G::LSTRIDE, G::LHALF, Lg, a.pitch, a.H, a.W, y0 - NW, x0 - NW, G::LROWS,
                  G::LCOLS, 0.f);

    // per-pixel left statistics; the block's left windows are centred on its
    // first pixel's window mean
    float ndl[4], invl[4], ca;
    {
        float4 st[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) st[p] = a.statL[(size_t)ip[p] * a.spitch + jp[p]];
        ca = st[0].x;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            ndl[p] = -Nf * ((st[p].x - ca) + st[p].y);
            invl[p] = st[p].z;
        }
    }

    float best[4] = {-3.f, -3.f, -3.f, -3.f};
    int bz[4] = {0, 0, 0, 0};
    float rho_keep[(MODE == MODE_SOFT) ? 4 : 1][(MODE == MODE_SOFT) ? NC : 1];

    for (int zc = zlo, ci = 0; zc <= zhi; zc += STEP, ++ci) {
        if (MODE != MODE_FULL && !((mask >> ci) & 1u)) continue;
        // largest candidate slot of this chunk: the right tile's column 0 pairs
        // with the first window column of that slot
        const int ztop = min(zc + CHUNK - 1, zhi + NC - 1);
        __syncthreads();  // previous chunk fully consumed (and left tile staged)
        stage_tile<T>(Rs, G::RSTRIDE, G::RHALF, Rg, a.pitch, a.H, a.W, y0 - NW, x0 - NW - ztop,
                      G::LROWS, TILE_W + 2 * NW + (ztop - zc), cR);
        __syncthreads();
        if (!any) continue;

        // slot windows this thread evaluates in this chunk
        int w_first, w_last;
        if (MODE == MODE_FULL) {
            w_first = zc;
            w_last = min(zc + CHUNK - 1, max(hi[0], hi[1]));
        } else {
            w_first = zs;
            w_last = (zs >= zc && zs < zc + STEP) ? zs : zs - 1;
        }
        for (int wz = w_first; wz <= w_last; wz += NC) {
            float S[4][NC];
            const int rcol0 = 2 * tx + (ztop - wz) - (NC - 1);
            window_sums<NW, NC>(Ls, Rs, 2 * ty, tx, rcol0, ca, S);
            // right statistics for columns j0 + 1 - wz - q, q = 0..NC
#pragma unroll
            for (int rowp = 0; rowp < 2; ++rowp) {
                const float4* srow = a.statR + (size_t)ip[2 * rowp] * a.spitch;
                float4 sr[NC + 1];
#pragma unroll
                for (int q = 0; q <= NC; ++q) sr[q] = srow[clampi(j0 + 1 - wz - q, 0, a.W - 1)];
#pragma unroll
                for (int cp = 0; cp < 2; ++cp) {
                    const int p = 2 * rowp + cp;
#pragma unroll
                    for (int s = 0; s < NC; ++s) {
                        const int z = wz + s;
                        const float4 st = sr[s + 1 - cp];
                        const float C = fmaf(ndl[p], (st.x - cR) + st.y, S[p][s]);
                        float rho = C * invl[p] * st.z;
                        rho = fminf(fmaxf(rho, -1.f), 1.f);
                        const bool ok = (z >= lo[p]) && (z <= hi[p]);
                        if (MODE == MODE_SOFT) rho_keep[p][s] = ok ? rho : -1e30f;
                        if (ok && rho > best[p]) {
                            best[p] = rho;
                            bz[p] = z;
                        }
                    }
                }
            }
        }
    }
    if (!any) return;

#pragma unroll
    for (int p = 0; p < 4; ++p) {
        if (!act[p]) continue;
        const size_t o = (size_t)ip[p] * a.opitch + jp[p];
        a.d_out[o] = (int16_t)bz[p];
        if (a.c_out) a.c_out[o] = best[p];
        if (MODE == MODE_SOFT) {
            float se = 0.f, sz = 0.f;
#pragma unroll
            for (int s = 0; s < NC; ++s) {
                const float e = __expf((rho_keep[p][s] - best[p]) * a.inv_tau);
                se += e;
                sz = fmaf(e, (float)(zs + s), sz);
            }
            a.soft_out[o] = sz / se;
        }
    }
}

template <typename T, int NW, int NC, int MODE>
static hipError_t launch_one(const MatchArgs& a, hipStream_t s)
{
    dim3 grid((a.W + TILE_W - 1) / TILE_W, (a.H + TILE_H - 1) / TILE_H, 1);
    hipLaunchKernelGGL((match_kernel<T, NW, NC, MODE>), grid, dim3(MATCH_THREADS), 0, s, a);
    return hipGetLastError();
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
    if (dtype == 0) {
        if (mode == MODE_SOFT) return hipErrorInvalidValue;  // soft mode takes float images
        return dispatch_nc<uint8_t, NW>(mode, nc, a, s);
    }
    return dispatch_nc<float, NW>(mode, nc, a, s);
}

}  // namespace msibm
