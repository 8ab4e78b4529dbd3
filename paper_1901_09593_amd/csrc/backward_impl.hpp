// Backward pass of the differentiable finest level: gradient of
// sum_ij g(i,j) d_soft(i,j) with respect to the level-0 left and right images,
// the level-1 prior held fixed.
//
// Chain rule per pixel (i, j) and candidate z of its soft-argmax interval:
//   d_soft = sum_z p_z z, p = softmax(rho / tau)      ->  dd/drho_z = p_z (z - d_soft) / tau
//   rho = C / sqrt(A B)                                ->
//     drho/dl_ab = (r_ab - mu_r) / sqrt(AB) - rho (l_ab - mu_l) / A
//     drho/dr_ab = (l_ab - mu_l) / sqrt(AB) - rho (r_ab - mu_r) / B
// so with gz = g p_z (z - d_soft) / tau, k1 = gz / sqrt(AB), kL = gz rho / A and
// kR = gz rho / B, a window position (a, b) receives
//   dL/dl_ab += k1 (r_ab - mu_r) - kL (l_ab - mu_l)
//   dL/dr_ab += k1 (l_ab - mu_l) - kR (r_ab - mu_r).
// Flat candidates (1/sd = 0) get k1 = kL = kR = 0; clamped window reads send
// their gradient to the edge pixel they read.
//
// Work split.  Same tiles, blocks and LDS staging as the forward matching
// kernel; each thread recomputes its block's scores with the shared window sums,
// then walks each of its pixels' window rows, forms that row's gradient values
// in registers and adds them into LDS gradient tiles (the left tile and the
// current right chunk) with LDS atomics.  Finished tiles are added to the
// global gradients with hardware float atomics (tiles overlap by their window
// halos), so the global gradients must be zeroed first.  No cost volume is
// stored: scores are recomputed from the images and window statistics.
#pragma once

#include "match_impl.hpp"

namespace msibm {

struct BackArgs {
    const float* L;
    const float* R;
    int H, W, pitch;
    const float4* statL;
    const float4* statR;
    int spitch;
    int D;                    // candidates at level 0
    const int16_t* prior;     // level-1 map
    int Hc, Wc, ppitch;
    int rs;                   // soft-argmax radius
    float inv_tau;
    const float* g;           // dLoss/dd_soft, H x W, pitch gpitch
    int gpitch;
    float* gL;                // H x W, pitch gpitch; accumulated (zero first)
    float* gR;
};

template <int NW, int CH>
struct BackSmem {
    using G = Geo<NW, CH, 1>;
    float Ls[G::LROWS * G::LSTRIDE];
    float Rs[G::LROWS * G::RSTRIDE];
    float GLs[G::LROWS * G::LSTRIDE];   // left gradient tile (same layout as Ls)
    float GRs[G::LROWS * G::RSTRIDE];   // right gradient tile of the current chunk
    int lo, hi;
    unsigned mask;
};

__device__ __forceinline__ void lds_add(float* p, float v) { atomicAdd(p, v); }

// Add an LDS tile in split layout to a global image with float atomics;
// logical column c of LDS row rr maps to global (clamp(gy0 + rr), clamp(gx0 + c)).
__device__ __forceinline__ void flush_tile(const float* tile, int stride, int half, int rows, int cols,
                                           float* dst, int dpitch, int H, int W, int gy0, int gx0)
{
    const int lane = threadIdx.x & (MATCH_TX - 1), wave = threadIdx.x / MATCH_TX;
    for (int rr = wave; rr < rows; rr += MATCH_TY) {
        float* drow = dst + (size_t)clampi(gy0 + rr, 0, H - 1) * dpitch;
        for (int c = lane; c < cols; c += MATCH_TX) {
            const float v = tile[rr * stride + split_pos(c, half)];
            if (v != 0.f) unsafeAtomicAdd(drow + clampi(gx0 + c, 0, W - 1), v);
        }
    }
}

__device__ __forceinline__ void zero_lds(float* p, int count)
{
    for (int i = threadIdx.x; i < count; i += MATCH_THREADS) p[i] = 0.f;
}

template <int NW, int NC>
__device__ __forceinline__ void backward_tile(const BackArgs& a, int bx, int by, BackSmem<NW, BACK_CHUNK>& sm)
{
    constexpr int CH = BACK_CHUNK;
    using G = Geo<NW, CH, 1>;
    constexpr int WS = 2 * NW + 1;          // window side
    constexpr float Nf = (float)(WS * WS);
    constexpr int STEP = CH - NC + 1;
    constexpr int RU = WS + NC - 1;         // right values a pixel's window row touches
    static_assert((MSIBM_MAX_DISP - 1) / STEP < 32, "chunk mask must hold every chunk");

    const int tx = threadIdx.x & (MATCH_TX - 1), ty = threadIdx.x / MATCH_TX;
    const int x0 = bx * TILE_W, y0 = by * G::TH;
    const int i0 = y0 + 2 * ty, j0 = x0 + 2 * tx;
    const bool act[4] = {i0 < a.H && j0 < a.W, i0 < a.H && j0 + 1 < a.W, i0 + 1 < a.H && j0 < a.W,
                         i0 + 1 < a.H && j0 + 1 < a.W};
    const int ia = min(i0, a.H - 1), ib = min(i0 + 1, a.H - 1);
    const int ja = min(j0, a.W - 1), jb = min(j0 + 1, a.W - 1);
    const int ip[4] = {ia, ia, ib, ib};
    const int jp[4] = {ja, jb, ja, jb};

    // candidate intervals (as in the forward soft level)
    const int dh = clampi(2 * (int)a.prior[(size_t)(ia >> 1) * a.ppitch + (ja >> 1)], 0, a.D - 1);
    const int zs = (dh <= j0) ? dh - a.rs : j0 + 2 - NC;
    int lo[4], hi[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int c = min(dh, jp[p]);
        lo[p] = max(0, c - a.rs);
        hi[p] = min(min(a.D - 1, jp[p]), c + a.rs);
    }
    const int cy = min(y0 + G::TH / 2, a.H - 1), cx = min(x0 + TILE_W / 2, a.W - 1);
    const float cR = a.R[(size_t)cy * a.pitch + cx];

    stage_tile<float, G::LROWS, G::LCOLS>(sm.Ls, G::LSTRIDE, G::LHALF, a.L, a.pitch, a.H, a.W, y0 - NW,
                                          x0 - NW, G::LCOLS, 0.f);
    zero_lds(sm.GLs, G::LROWS * G::LSTRIDE);
    if (threadIdx.x == 0) {
        sm.lo = 0x7fffffff;
        sm.hi = -0x7fffffff;
        sm.mask = 0u;
    }
    __syncthreads();
    if (act[0]) {
        atomicMin(&sm.lo, zs);
        atomicMax(&sm.hi, zs);
    }
    __syncthreads();
    const int zlo = sm.lo, zhi = sm.hi;
    if (act[0]) atomicOr(&sm.mask, 1u << ((zs - zlo) / STEP));
    __syncthreads();
    const unsigned mask = sm.mask;

    for (int zc = zlo, ci = 0; zc <= zhi; zc += STEP, ++ci) {
        if (!((mask >> ci) & 1u)) continue;
        const int ztop = min(zc + CH - 1, zhi + NC - 1);
        const int rcols = TILE_W + 2 * NW + (ztop - zc);
        if (zc != zlo) __syncthreads();
        stage_tile<float, G::LROWS, G::RCOLS>(sm.Rs, G::RSTRIDE, G::RHALF, a.R, a.pitch, a.H, a.W, y0 - NW,
                                              x0 - NW - ztop, rcols, cR);
        zero_lds(sm.GRs, G::LROWS * G::RSTRIDE);
        __syncthreads();

        if (act[0] && zs >= zc && zs < zc + STEP) {
            // --- recompute the block's scores
            float4 stl[4];
#pragma unroll
            for (int p = 0; p < 4; ++p) stl[p] = a.statL[(size_t)ip[p] * a.spitch + jp[p]];
            const float ca = stl[0].x;
            float S[4][NC];
            const int rcol0 = 2 * tx + (ztop - zs) - (NC - 1);
            window_sums<NW, NC, G>(sm.Ls, sm.Rs, 2 * ty, tx, rcol0, ca, S);
            // right-value base offsets (split layout) for logical column rcol0 + u
            int pa, pb;
            if ((rcol0 & 1) == 0) {
                pa = rcol0 >> 1;
                pb = G::RHALF + (rcol0 >> 1);
            } else {
                pa = G::RHALF + (rcol0 >> 1);
                pb = (rcol0 + 1) >> 1;
            }
            // one pixel row at a time; its two pixels' contributions are summed in
            // registers over the union of their windows (WS + 1 left and RU + 1
            // right columns per row) before they are added into LDS
#pragma unroll
            for (int pr = 0; pr < 2; ++pr) {
                float k1[2][NC], kl[2], cl[2], qb[RU + 1], qc[RU + 1];
#pragma unroll
                for (int u = 0; u <= RU; ++u) {
                    qb[u] = 0.f;
                    qc[u] = 0.f;
                }
#pragma unroll
                for (int pc = 0; pc < 2; ++pc) {
                    const int p = 2 * pr + pc;
                    kl[pc] = 0.f;
                    cl[pc] = 0.f;
#pragma unroll
                    for (int s = 0; s < NC; ++s) k1[pc][s] = 0.f;
                    if (!act[p]) continue;  // contributes nothing
                    const float dl = (stl[p].x - ca) + stl[p].y;  // mu_l - ca
                    const float invl = stl[p].z;
                    // right statistics of this pixel's candidates: column jp - z
                    const float4* srow = a.statR + (size_t)ip[p] * a.spitch;
                    float mr[NC], invr[NC], rho[NC];
                    bool ok[NC];
                    float best = -3.f;
#pragma unroll
                    for (int s = 0; s < NC; ++s) {
                        const int z = zs + s;
                        const float4 st = srow[clampi(jp[p] - z, 0, a.W - 1)];
                        mr[s] = (st.x - cR) + st.y;  // mu_r - cR
                        invr[s] = st.z;
                        const float C = fmaf(-Nf * dl, mr[s], S[p][s]);
                        float rr = C * invl * invr[s];
                        rr = fminf(fmaxf(rr, -1.f), 1.f);
                        ok[s] = (z >= lo[p]) && (z <= hi[p]);
                        rho[s] = rr;
                        if (ok[s] && rr > best) best = rr;
                    }
                    // soft-argmax and its derivative
                    float e[NC], se = 0.f, sz = 0.f;
#pragma unroll
                    for (int s = 0; s < NC; ++s) {
                        e[s] = ok[s] ? __expf((rho[s] - best) * a.inv_tau) : 0.f;
                        se += e[s];
                        sz = fmaf(e[s], (float)(zs + s), sz);
                    }
                    const float ds = sz / se;
                    const float gpx = a.g[(size_t)ip[p] * a.gpitch + jp[p]];
                    const float gs = gpx * a.inv_tau / se;
                    float k2r[NC], klp = 0.f, clp = 0.f;
#pragma unroll
                    for (int s = 0; s < NC; ++s) {
                        const float gz = gs * e[s] * ((float)(zs + s) - ds);
                        k1[pc][s] = gz * invl * invr[s];
                        const float kls = gz * rho[s] * invl * invl;
                        k2r[s] = gz * rho[s] * invr[s] * invr[s];
                        klp += kls;
                        clp = fmaf(-k1[pc][s], mr[s], clp);
                    }
                    kl[pc] = klp;
                    cl[pc] = fmaf(klp, dl, clp);
                    // right offsets u of this pixel are union columns u + pc:
                    // slots touching them and their summed coefficients
#pragma unroll
                    for (int u = 0; u < RU; ++u) {
#pragma unroll
                        for (int s = 0; s < NC; ++s) {
                            const int b = u - (NC - 1 - s);
                            if (b >= 0 && b < WS) {
                                qb[u + pc] += k2r[s];
                                qc[u + pc] += fmaf(k2r[s], mr[s], -k1[pc][s] * dl);
                            }
                        }
                    }
                }
                float k1s[NC];
#pragma unroll
                for (int s = 0; s < NC; ++s) k1s[s] = k1[0][s] + k1[1][s];
                const float kls = kl[0] + kl[1], cls = cl[0] + cl[1];
                // window rows of this pixel row
#pragma unroll 1
                for (int y = 0; y < WS; ++y) {
                    const int row = 2 * ty + pr + y;
                    const float* lr_ = sm.Ls + row * G::LSTRIDE + tx;
                    const float* rr_ = sm.Rs + row * G::RSTRIDE;
                    float* glr = sm.GLs + row * G::LSTRIDE + tx;
                    float* grr = sm.GRs + row * G::RSTRIDE;
                    float l[WS + 1], r[RU + 1];
#pragma unroll
                    for (int t = 0; t <= WS; ++t) l[t] = lr_[(t & 1) ? G::LHALF + (t >> 1) : (t >> 1)] - ca;
#pragma unroll
                    for (int v = 0; v <= RU; ++v) r[v] = (v & 1) ? rr_[pb + (v >> 1)] : rr_[pa + (v >> 1)];
                    // left gradient at union column t: pixel 0 covers t <= WS - 1,
                    // pixel 1 covers t >= 1 (both fold into compile-time choices)
#pragma unroll
                    for (int t = 0; t <= WS; ++t) {
                        const bool v0 = t <= WS - 1, v1 = t >= 1;
                        const float klt = (v0 && v1) ? kls : (v0 ? kl[0] : kl[1]);
                        const float clt = (v0 && v1) ? cls : (v0 ? cl[0] : cl[1]);
                        float acc = fmaf(-klt, l[t], clt);
#pragma unroll
                        for (int s = 0; s < NC; ++s) {
                            const float c = (v0 && v1) ? k1s[s] : (v0 ? k1[0][s] : k1[1][s]);
                            acc = fmaf(c, r[t + NC - 1 - s], acc);
                        }
                        lds_add(glr + ((t & 1) ? G::LHALF + (t >> 1) : (t >> 1)), acc);
                    }
                    // right gradient at union column v: slot s pairs it with left
                    // union column v - (NC - 1 - s), which pixel pc covers when that
                    // column lies in [pc, WS - 1 + pc]
#pragma unroll
                    for (int v = 0; v <= RU; ++v) {
                        float acc = fmaf(-qb[v], r[v], qc[v]);
#pragma unroll
                        for (int s = 0; s < NC; ++s) {
                            const int t = v - (NC - 1 - s);
                            const bool v0 = t >= 0 && t <= WS - 1, v1 = t >= 1 && t <= WS;
                            if (v0 || v1) {
                                const float c = (v0 && v1) ? k1s[s] : (v0 ? k1[0][s] : k1[1][s]);
                                acc = fmaf(c, l[t], acc);
                            }
                        }
                        lds_add(grr + ((v & 1) ? pb + (v >> 1) : pa + (v >> 1)), acc);
                    }
                }
            }
        }
        __syncthreads();
        flush_tile(sm.GRs, G::RSTRIDE, G::RHALF, G::LROWS, rcols, a.gR, a.gpitch, a.H, a.W, y0 - NW,
                   x0 - NW - ztop);
    }
    __syncthreads();
    flush_tile(sm.GLs, G::LSTRIDE, G::LHALF, G::LROWS, G::LCOLS, a.gL, a.gpitch, a.H, a.W, y0 - NW,
               x0 - NW);
    __syncthreads();
}

template <int NW, int NC>
__global__ __launch_bounds__(MATCH_THREADS) void backward_kernel(BackArgs a)
{
    __shared__ BackSmem<NW, BACK_CHUNK> sm;
    backward_tile<NW, NC>(a, blockIdx.x, blockIdx.y, sm);
}

template <int NW>
static hipError_t dispatch_backward(int nc, const BackArgs& a, hipStream_t s)
{
    dim3 grid((a.W + TILE_W - 1) / TILE_W, (a.H + TILE_H1 - 1) / TILE_H1, 1);
    switch (nc) {
        case 3: hipLaunchKernelGGL((backward_kernel<NW, 3>), grid, dim3(MATCH_THREADS), 0, s, a); break;
        case 5: hipLaunchKernelGGL((backward_kernel<NW, 5>), grid, dim3(MATCH_THREADS), 0, s, a); break;
        case 7: hipLaunchKernelGGL((backward_kernel<NW, 7>), grid, dim3(MATCH_THREADS), 0, s, a); break;
        case 9: hipLaunchKernelGGL((backward_kernel<NW, 9>), grid, dim3(MATCH_THREADS), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Backward tiles of several pairs in one launch (level 0 of each pair).
template <int NW, int NC>
__global__ __launch_bounds__(MATCH_THREADS) void backward_multi_kernel(MultiArgs a)
{
    __shared__ BackSmem<NW, BACK_CHUNK> sm;
    const Segment s = a.segs[segment_of(a.segs, a.nseg, blockIdx.x)];
    const int t = blockIdx.x - s.task0;
    backward_tile<NW, NC>(a.back[s.pair], t % s.tiles_x, t / s.tiles_x, sm);
}

template <int NW>
static hipError_t dispatch_backward_multi(int nc, const MultiArgs& a, int blocks, hipStream_t s)
{
    if (blocks < 1 || a.nseg < 1) return hipErrorInvalidValue;
    switch (nc) {
        case 3: hipLaunchKernelGGL((backward_multi_kernel<NW, 3>), dim3(blocks), dim3(MATCH_THREADS), 0, s, a); break;
        case 5: hipLaunchKernelGGL((backward_multi_kernel<NW, 5>), dim3(blocks), dim3(MATCH_THREADS), 0, s, a); break;
        case 7: hipLaunchKernelGGL((backward_multi_kernel<NW, 7>), dim3(blocks), dim3(MATCH_THREADS), 0, s, a); break;
        case 9: hipLaunchKernelGGL((backward_multi_kernel<NW, 9>), dim3(blocks), dim3(MATCH_THREADS), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace msibm
