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
// Work split.  Same tiles (128 x 8 pixels) and LDS staging as the forward
// matching kernel, 4 waves per workgroup: a thread owns a 2x2 pixel block.  It
// recomputes the block's scores with the forward's window sums (products
// shared by the four windows, so the soft disparities are the forward's bit for
// bit), then walks the 2n+2 rows of the union of the block's windows: per row
// it sums, in registers, every pixel's gradient value at each union column
// (over the candidates and over the pixels whose window covers that cell) and
// adds one value per cell into LDS gradient tiles (the left tile and the
// current right chunk).  The first and last union rows are covered by one pixel
// row, the others by both, so their coefficients are the sums of the two
// rows' (formed once).  Finished tiles are added to the global gradients with
// hardware float atomics (tiles overlap by their window halos), so the global
// gradients must be zeroed first.  No cost volume is stored: scores are
// recomputed from the images and window statistics.
//
// LDS accumulation is in 32-bit fixed point: integer LDS atomics are tens of
// times faster than float ones on this chip, and 32-bit cells keep the four
// tiles within 80 KB (two workgroups per CU for windows up to 11 x 11).  Per
// chunk the workgroup bounds every value it will add (from the ranges of the
// staged images and the largest gradient coefficients) and picks a
// power-of-two scale that maps that bound below 2^23: each added value (at
// most half the bound) becomes an integer (rounded) with a resolution of 2^-23
// of the bound, and a cell, which receives at most one value per thread and
// chunk (256), stays below 2^30.
#pragma once

#include "match_impl.hpp"

namespace msibm {

struct BackArgs {
    const float* L;
    const float* R;
    int H, W, pitch;
    const WinStat* statL;
    const WinStat* statR;
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
    // Fused masked-L1 form (the FUSED kernels): the upstream gradient is formed
    // in the kernel from the soft disparity it computes, g = sign(d_soft - gt) /
    // |M| on the loss pixels M and 0 elsewhere, instead of being read from g;
    // the kernel also writes the soft level's outputs and adds the pair's
    // sum over M of |d_soft - gt| into loss_sum.
    const float* gt;          // ground-truth disparity, pitch gpitch
    const uint8_t* mask;      // nonzero on M, pitch gpitch
    int* count;               // |M| (the mask count kernel's result)
    float* loss_sum;          // one float per pair, zeroed before the launch
    float* loss_out;          // the pair's loss, sum / |M| (the finalize kernel)
    float* soft_out;          // d_soft, pitch gpitch
    int16_t* d_out;           // hard winner over the soft interval, pitch gpitch
    float* c_out;             // its score (NULL: not written), pitch gpitch
};

template <int NW, int CH>
struct BackSmem {
    using G = Geo<NW, CH, TILE_H1>;
    float Ls[G::LROWS * G::LSTRIDE];
    float Rs[G::LROWS * G::RSTRIDE];
    int GLs[G::LROWS * G::LSTRIDE];        // left gradient tile (same layout as Ls), fixed point
    int GRs[G::LROWS * G::RSTRIDE];        // right gradient tile of the current chunk, fixed point
    int lo, hi;
    unsigned mask;
    int lmin, lmax, rmin, rmax;            // value ranges of the staged tiles (ordered float keys)
    unsigned kmax[5];                      // largest coefficient magnitudes (float bits)
    float red[16];                         // per-wave partial loss sums (fused form)
};

// Order-preserving int key of a float (signed comparison), and its inverse.
__device__ __forceinline__ int fkey(float f)
{
    const int b = __float_as_int(f);
    return b >= 0 ? b : b ^ 0x7fffffff;
}
__device__ __forceinline__ float fval(int k) { return __int_as_float(k >= 0 ? k : k ^ 0x7fffffff); }

constexpr int BACK_WAVES = MATCH_TY;
constexpr int BACK_THREADS = BACK_WAVES * MATCH_TX;
// Fixed-point headroom: the chunk's bound is below 2^BACK_VBITS in cell units
// and every value is at most half the bound; a cell receives at most one value
// per thread and chunk.
constexpr int BACK_VBITS = 23;
static_assert((BACK_VBITS - 1) + 9 <= 31 && BACK_THREADS <= 512, "a cell's sum must fit an int32");

// Add v (|v * scale| <= 2^22) to a fixed-point LDS cell, rounded to the
// nearest integer: an error of at most 2^-24 of the chunk's bound per value,
// unbiased, far inside the gradient tolerance.  Zeros are added too: a test
// per value costs more than the add.
__device__ __forceinline__ void lds_add(int* p, float v, float scale)
{
    atomicAdd(p, __float2int_rn(v * scale));
}

// Add a fixed-point LDS tile in split layout to a global image with float
// atomics (value = cell / scale); logical column c of LDS row rr maps to global
// (clamp(gy0 + rr), clamp(gx0 + c)).  The tile is zeroed behind the reads.
__device__ __forceinline__ void flush_tile(int* tile, int stride, int half, int rows, int cols, float inv_scale,
                                           float* dst, int dpitch, int H, int W, int gy0, int gx0)
{
    const int lane = threadIdx.x & (MATCH_TX - 1), wave = threadIdx.x / MATCH_TX;
    for (int rr = wave; rr < rows; rr += BACK_WAVES) {
        float* drow = dst + (size_t)clampi(gy0 + rr, 0, H - 1) * dpitch;
        for (int c = lane; c < cols; c += MATCH_TX) {
            int* cell = tile + rr * stride + split_pos(c, half);
            const int v = *cell;
            if (v != 0) {
                unsafeAtomicAdd(drow + clampi(gx0 + c, 0, W - 1), (float)v * inv_scale);
                *cell = 0;
            }
        }
    }
}

__device__ __forceinline__ void zero_lds(int* p, int count)
{
    for (int i = threadIdx.x; i < count; i += BACK_THREADS) p[i] = 0;
}

// Min and max over the logical region rows x cols of a split-layout LDS tile,
// folded into the workgroup's keys.
__device__ __forceinline__ void tile_range(const float* t, int stride, int half, int rows, int cols, int* kmin,
                                           int* kmax)
{
    float mn = 3.4e38f, mx = -3.4e38f;
    for (int i = threadIdx.x; i < rows * cols; i += BACK_THREADS) {
        const int r = i / cols, c = i - r * cols;
        const float v = t[r * stride + split_pos(c, half)];
        mn = fminf(mn, v);
        mx = fmaxf(mx, v);
    }
    atomicMin(kmin, fkey(mn));
    atomicMax(kmax, fkey(mx));
}

// Gradient values of one union row of a 2x2 block's windows, added into the
// LDS tiles.  The row is covered by the pixel rows whose coefficients were
// summed into kl (per pixel column), cl, k1 (per pixel column and slot), qb
// and qc (per union column of the right tile).  Left union column t is
// covered by pixel column 0 for t <= WS - 1 and by column 1 for t >= 1; right
// union column v pairs slot s with left union column v - (NC - 1 - s).
template <int NW, int NC, class G>
__device__ __forceinline__ void grad_row(const float* __restrict__ Ls, const float* __restrict__ Rs, int* GLs,
                                         int* GRs, int row, int tx, int pa, int pb, float ca, const float (&kl)[2],
                                         const float (&cl)[2], const float (&k1)[2][NC],
                                         const float (&qb)[2 * NW + NC + 1], const float (&qc)[2 * NW + NC + 1],
                                         float scale)
{
    constexpr int WS = 2 * NW + 1;
    constexpr int RU = WS + NC - 1;  // right values one pixel column's window row touches
    const float* lr_ = Ls + row * G::LSTRIDE + tx;
    const float* rr_ = Rs + row * G::RSTRIDE;
    int* glr = GLs + row * G::LSTRIDE + tx;
    int* grr = GRs + row * G::RSTRIDE;
    float l[WS + 1], r[RU + 1];
#pragma unroll
    for (int t = 0; t <= WS; ++t) l[t] = lr_[(t & 1) ? G::LHALF + (t >> 1) : (t >> 1)] - ca;
#pragma unroll
    for (int v = 0; v <= RU; ++v) r[v] = (v & 1) ? rr_[pb + (v >> 1)] : rr_[pa + (v >> 1)];
#pragma unroll
    for (int t = 0; t <= WS; ++t) {
        const bool v0 = t <= WS - 1, v1 = t >= 1;
        const float klt = (v0 && v1) ? kl[0] + kl[1] : (v0 ? kl[0] : kl[1]);
        const float clt = (v0 && v1) ? cl[0] + cl[1] : (v0 ? cl[0] : cl[1]);
        float acc = fmaf(-klt, l[t], clt);
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            const float c = (v0 && v1) ? k1[0][s] + k1[1][s] : (v0 ? k1[0][s] : k1[1][s]);
            acc = fmaf(c, r[t + NC - 1 - s], acc);
        }
        lds_add(glr + ((t & 1) ? G::LHALF + (t >> 1) : (t >> 1)), acc, scale);
    }
#pragma unroll
    for (int v = 0; v <= RU; ++v) {
        float acc = fmaf(-qb[v], r[v], qc[v]);
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            const int t = v - (NC - 1 - s);
            const bool v0 = t >= 0 && t <= WS - 1, v1 = t >= 1 && t <= WS;
            if (v0 || v1) {
                const float c = (v0 && v1) ? k1[0][s] + k1[1][s] : (v0 ? k1[0][s] : k1[1][s]);
                acc = fmaf(c, l[t], acc);
            }
        }
        lds_add(grr + ((v & 1) ? pb + (v >> 1) : pa + (v >> 1)), acc, scale);
    }
}

template <int NW, int NC, bool FUSED = false>
__device__ __forceinline__ void backward_tile(const BackArgs& a, int bx, int by, BackSmem<NW, BACK_CHUNK>& sm)
{
    constexpr int CH = BACK_CHUNK;
    using G = Geo<NW, CH, TILE_H1>;
    constexpr int WS = 2 * NW + 1;          // window side
    constexpr float Nf = (float)(WS * WS);
    constexpr int STEP = CH - NC + 1;
    constexpr int RU = WS + NC - 1;         // right values a pixel's window row touches
    static_assert((MSIBM_MAX_DISP - 1) / STEP < 32, "chunk mask must hold every chunk");

    const int tx = threadIdx.x & (MATCH_TX - 1), ty = threadIdx.x / MATCH_TX;  // block column and row
    const int x0 = bx * TILE_W, y0 = by * G::TH;
    const int i0 = y0 + 2 * ty, j0 = x0 + 2 * tx;
    const bool blk = i0 < a.H && j0 < a.W;  // the block has pixels
    // pixel p = 2 * pr + pc: row i0 + pr, column j0 + pc (clamped for loads)
    const int ip[2] = {min(i0, a.H - 1), min(i0 + 1, a.H - 1)};
    const int jp[2] = {min(j0, a.W - 1), min(j0 + 1, a.W - 1)};
    bool act[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) act[p] = i0 + (p >> 1) < a.H && j0 + (p & 1) < a.W;

    // candidate intervals (as in the forward soft level); the block shares the prior
    const int dh = clampi(2 * (int)a.prior[(size_t)(ip[0] >> 1) * a.ppitch + (jp[0] >> 1)], 0, a.D - 1);
    const int zs = (dh <= j0) ? dh - a.rs : j0 + 2 - NC;
    int lo[2], hi[2];
#pragma unroll
    for (int pc = 0; pc < 2; ++pc) {
        const int c = min(dh, jp[pc]);
        lo[pc] = max(0, c - a.rs);
        hi[pc] = min(min(a.D - 1, jp[pc]), c + a.rs);
    }
    // the forward's right centring (one pixel per 16-row band), so that the
    // recomputed scores are the forward's
    const int cy = min((y0 & ~15) + 8, a.H - 1), cx = min(x0 + TILE_W / 2, a.W - 1);
    const float cR = a.R[(size_t)cy * a.pitch + cx];

    stage_tile<float, G::LROWS, G::LCOLS, BACK_WAVES>(sm.Ls, G::LSTRIDE, G::LHALF, a.L, a.pitch, a.H, a.W,
                                                      y0 - NW, x0 - NW, G::LCOLS, 0.f);
    zero_lds(sm.GLs, G::LROWS * G::LSTRIDE);
    zero_lds(sm.GRs, G::LROWS * G::RSTRIDE);
    if (threadIdx.x == 0) {
        sm.lo = 0x7fffffff;
        sm.hi = -0x7fffffff;
        sm.mask = 0u;
        sm.lmin = 0x7fffffff;
        sm.lmax = -0x7fffffff - 1;
    }
    __syncthreads();
    if (blk) {
        atomicMin(&sm.lo, zs);
        atomicMax(&sm.hi, zs);
    }
    tile_range(sm.Ls, G::LSTRIDE, G::LHALF, G::LROWS, G::LCOLS, &sm.lmin, &sm.lmax);
    __syncthreads();
    const int zlo = sm.lo, zhi = sm.hi;
    // |l - ca| <= the left tile's range (ca is a window mean inside it)
    const float lrange = fval(sm.lmax) - fval(sm.lmin);
    if (blk) atomicOr(&sm.mask, 1u << ((zs - zlo) / STEP));
    __syncthreads();
    const unsigned mask = sm.mask;
    // fused form: 1/|M| (as a float reciprocal of the float count) and this
    // thread's share of the loss sum
    const float inv_count = FUSED ? 1.f / (float)max(*a.count, 1) : 0.f;
    float lsum = 0.f;

    for (int zc = zlo, ci = 0; zc <= zhi; zc += STEP, ++ci) {
        if (!((mask >> ci) & 1u)) continue;
        const int ztop = min(zc + CH - 1, zhi + NC - 1);
        const int rcols = TILE_W + 2 * NW + (ztop - zc);
        if (zc != zlo) __syncthreads();  // previous chunk flushed
        stage_tile<float, G::LROWS, G::RCOLS, BACK_WAVES>(sm.Rs, G::RSTRIDE, G::RHALF, a.R, a.pitch, a.H, a.W,
                                                          y0 - NW, x0 - NW - ztop, rcols, cR);
        if (threadIdx.x == 0) {
            sm.rmin = 0x7fffffff;
            sm.rmax = -0x7fffffff - 1;
#pragma unroll
            for (int q = 0; q < 5; ++q) sm.kmax[q] = 0u;
        }
        __syncthreads();

        const bool part = blk && zs >= zc && zs < zc + STEP;
        const int rcol0 = 2 * tx + (ztop - zs) - (NC - 1);
        // right-value base offsets (split layout) for logical column rcol0 + u
        int pa, pb;
        if ((rcol0 & 1) == 0) {
            pa = rcol0 >> 1;
            pb = G::RHALF + (rcol0 >> 1);
        } else {
            pa = G::RHALF + (rcol0 >> 1);
            pb = (rcol0 + 1) >> 1;
        }
        // per pixel row pr: the gradient coefficients of its two pixels (left:
        // kl, cl per pixel column, k1 per pixel column and slot) and the sums
        // of its right coefficients over the union columns of its windows
        // (right offset u of pixel column pc is union column u + pc)
        float kl[2][2], cl[2][2], k1[2][2][NC], qb[2][RU + 1], qc[2][RU + 1];
#pragma unroll
        for (int pr = 0; pr < 2; ++pr) {
#pragma unroll
            for (int u = 0; u <= RU; ++u) {
                qb[pr][u] = 0.f;
                qc[pr][u] = 0.f;
            }
#pragma unroll
            for (int pc = 0; pc < 2; ++pc) {
                kl[pr][pc] = 0.f;
                cl[pr][pc] = 0.f;
#pragma unroll
                for (int s = 0; s < NC; ++s) k1[pr][pc][s] = 0.f;
            }
        }
        float ca = 0.f;
        if (part) {
            // left statistics and upstream gradients of the four pixels, loaded
            // before the window sums so that their latency overlaps them (the
            // right statistics are read per pixel below: holding all four
            // pixels' would cost 12 NC registers)
            WinStat stl4[4];
            float gpx4[4];
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const size_t o = (size_t)ip[p >> 1] * a.spitch + jp[p & 1];
                stl4[p] = a.statL[o];
                gpx4[p] = FUSED ? a.gt[(size_t)ip[p >> 1] * a.gpitch + jp[p & 1]]
                                : a.g[(size_t)ip[p >> 1] * a.gpitch + jp[p & 1]];
            }
            asm volatile("" ::: "memory");  // keep the loads ahead of the window sums
            ca = stl4[0].x;                 // the block's windows are centred on its first pixel's mean
            float S[4][NC];
            window_sums<NW, NC, G>(sm.Ls, sm.Rs, 2 * ty, tx, rcol0, ca, S);
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                if (!act[p]) continue;  // contributes nothing
                const int pr = p >> 1, pc = p & 1;
                const WinStat stl = stl4[p];
                const float dl = (stl.x - ca) + stl.y;  // mu_l - ca
                const float invl = stl.z;
                // right statistics of this pixel's candidates: column jp - z
                float mr[NC], invr[NC], rho[NC];
                bool ok[NC];
                float best = -3.f;
                int bz = 0;
                const WinStat* srow = a.statR + (size_t)ip[pr] * a.spitch;
#pragma unroll
                for (int s = 0; s < NC; ++s) {
                    const WinStat st = srow[clampi(jp[pc] - (zs + s), 0, a.W - 1)];
                    mr[s] = (st.x - cR) + st.y;  // mu_r - cR
                    invr[s] = st.z;
                }
#pragma unroll
                for (int s = 0; s < NC; ++s) {
                    const int z = zs + s;
                    const float C = fmaf(-Nf * dl, mr[s], S[p][s]);
                    float rr = C * invl * invr[s];
                    rr = fminf(fmaxf(rr, -1.f), 1.f);
                    ok[s] = (z >= lo[pc]) && (z <= hi[pc]);
                    rho[s] = rr;
                    if (ok[s] && rr > best) {
                        best = rr;
                        bz = z;
                    }
                }
                float e[NC], se = 0.f, sz = 0.f;
#pragma unroll
                for (int s = 0; s < NC; ++s) {
                    e[s] = ok[s] ? __expf((rho[s] - best) * a.inv_tau) : 0.f;
                    se += e[s];
                    sz = fmaf(e[s], (float)(zs + s), sz);
                }
                const float ds = sz / se;
                float gpx = gpx4[p];
                if (FUSED) {
                    // the soft level's outputs, and the masked-L1 gradient of
                    // this pixel: sign(d_soft - gt) / |M| on M
                    const size_t o = (size_t)ip[pr] * a.gpitch + jp[pc];
                    a.soft_out[o] = ds;
                    a.d_out[o] = (int16_t)bz;
                    if (a.c_out) a.c_out[o] = best;
                    const float diff = ds - gpx;
                    const bool m = a.mask[o] != 0;
                    gpx = m ? (float)((diff > 0.f) - (diff < 0.f)) * inv_count : 0.f;
                    if (m) lsum += fabsf(diff);
                }
                const float gs = gpx * a.inv_tau / se;
                float klp = 0.f, clp = 0.f;
#pragma unroll
                for (int s = 0; s < NC; ++s) {
                    const float gz = gs * e[s] * ((float)(zs + s) - ds);
                    const float k1s = gz * invl * invr[s];
                    k1[pr][pc][s] = k1s;
                    klp += gz * rho[s] * invl * invl;
                    clp = fmaf(-k1s, mr[s], clp);
                    // slot s pairs right offset u with window column u - (NC - 1 - s):
                    // its right coefficients reach offsets NC - 1 - s .. NC - 2 - s + WS
                    const float k2r = gz * rho[s] * invr[s] * invr[s];
                    const float cq = fmaf(k2r, mr[s], -k1s * dl);
#pragma unroll
                    for (int u = NC - 1 - s; u < NC - 1 - s + WS; ++u) {
                        qb[pr][u + pc] += k2r;
                        qc[pr][u + pc] += cq;
                    }
                }
                kl[pr][pc] = klp;
                cl[pr][pc] = fmaf(klp, dl, clp);
            }
        }
        // bounds of every value a cell receives: the coefficient magnitudes of
        // all four pixels together cover any one union row's combination
        float ka = 0.f, kla = 0.f, cla = 0.f, qba = 0.f, qca = 0.f;
#pragma unroll
        for (int pr = 0; pr < 2; ++pr)
#pragma unroll
            for (int pc = 0; pc < 2; ++pc) {
                kla += fabsf(kl[pr][pc]);
                cla += fabsf(cl[pr][pc]);
#pragma unroll
                for (int s = 0; s < NC; ++s) ka += fabsf(k1[pr][pc][s]);
            }
#pragma unroll
        for (int u = 0; u <= RU; ++u) {
            qba = fmaxf(qba, fabsf(qb[0][u]) + fabsf(qb[1][u]));
            qca = fmaxf(qca, fabsf(qc[0][u]) + fabsf(qc[1][u]));
        }
        // workgroup maxima of the coefficient magnitudes and the right range
        tile_range(sm.Rs, G::RSTRIDE, G::RHALF, G::LROWS, rcols, &sm.rmin, &sm.rmax);
        if (part) {
            atomicMax(&sm.kmax[0], __float_as_uint(kla));
            atomicMax(&sm.kmax[1], __float_as_uint(cla));
            atomicMax(&sm.kmax[2], __float_as_uint(ka));
            atomicMax(&sm.kmax[3], __float_as_uint(qba));
            atomicMax(&sm.kmax[4], __float_as_uint(qca));
        }
        __syncthreads();
        // every added value: left |kl l + cl + sum k1 r| <= KL Lr + CL + K1 Rr,
        // right |qb r + qc + sum k1 l| <= QB Rr + QC + K1 Lr (r centred on cR, a
        // value of the right tile, so |r| <= its range)
        const float rrange = fmaxf(fval(sm.rmax) - fval(sm.rmin), fmaxf(fabsf(fval(sm.rmax)), fabsf(fval(sm.rmin))));
        const float KL = __uint_as_float(sm.kmax[0]), CL = __uint_as_float(sm.kmax[1]),
                    K1 = __uint_as_float(sm.kmax[2]), QB = __uint_as_float(sm.kmax[3]),
                    QC = __uint_as_float(sm.kmax[4]);
        const float bound = 2.f * fmaxf(KL * lrange + CL + K1 * rrange, QB * rrange + QC + K1 * lrange);
        int be = 0;
        frexpf(bound, &be);  // bound < 2^be
        // (at most 2^100, a finite float, for vanishing bounds)
        const int sh = (bound > 0.f && isfinite(bound)) ? min(BACK_VBITS - be, 100) : 0;
        const float scale = ldexpf(1.f, sh);
        const float inv_scale = ldexpf(1.f, -sh);

        if (part && bound > 0.f && isfinite(bound)) {
            // union row 0: the upper pixel row only; the last one: the lower
            // pixel row only; the rows between: both (coefficients summed once)
            const int row0 = 2 * ty;
            grad_row<NW, NC, G>(sm.Ls, sm.Rs, sm.GLs, sm.GRs, row0, tx, pa, pb, ca, kl[0], cl[0], k1[0], qb[0], qc[0],
                                scale);
            grad_row<NW, NC, G>(sm.Ls, sm.Rs, sm.GLs, sm.GRs, row0 + WS, tx, pa, pb, ca, kl[1], cl[1], k1[1], qb[1],
                                qc[1], scale);
#pragma unroll
            for (int pc = 0; pc < 2; ++pc) {
                kl[0][pc] += kl[1][pc];
                cl[0][pc] += cl[1][pc];
#pragma unroll
                for (int s = 0; s < NC; ++s) k1[0][pc][s] += k1[1][pc][s];
            }
#pragma unroll
            for (int u = 0; u <= RU; ++u) {
                qb[0][u] += qb[1][u];
                qc[0][u] += qc[1][u];
            }
#pragma unroll 1
            for (int y = 1; y < WS; ++y)
                grad_row<NW, NC, G>(sm.Ls, sm.Rs, sm.GLs, sm.GRs, row0 + y, tx, pa, pb, ca, kl[0], cl[0], k1[0],
                                    qb[0], qc[0], scale);
        }
        __syncthreads();
        // both tiles carry this chunk's scale: flush (and clear) them now
        flush_tile(sm.GRs, G::RSTRIDE, G::RHALF, G::LROWS, rcols, inv_scale, a.gR, a.gpitch, a.H, a.W, y0 - NW,
                   x0 - NW - ztop);
        flush_tile(sm.GLs, G::LSTRIDE, G::LHALF, G::LROWS, G::LCOLS, inv_scale, a.gL, a.gpitch, a.H, a.W, y0 - NW,
                   x0 - NW);
    }
    if (FUSED) {
        // the tile's loss sum: waves reduce across lanes, then one add per tile
        for (int off = MATCH_TX / 2; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off);
        if ((threadIdx.x & (MATCH_TX - 1)) == 0) sm.red[threadIdx.x / MATCH_TX] = lsum;
        __syncthreads();
        if (threadIdx.x == 0) {
            float t = 0.f;
            for (int q = 0; q < BACK_WAVES; ++q) t += sm.red[q];
            if (t != 0.f) atomicAdd(a.loss_sum, t);
        }
    }
    __syncthreads();  // LDS may be reused by the caller's next tile
}

template <int NW, int NC, bool FUSED>
__global__ __launch_bounds__(BACK_THREADS, 2) void backward_kernel(BackArgs a)
{
    __shared__ BackSmem<NW, BACK_CHUNK> sm;
    backward_tile<NW, NC, FUSED>(a, blockIdx.x, blockIdx.y, sm);
}

template <int NW, int NC>
static void launch_backward_nc(const BackArgs& a, dim3 grid, hipStream_t s)
{
    // the fused masked-L1 form is the instance whose upstream gradient comes
    // from a ground-truth map
    if (a.gt) hipLaunchKernelGGL((backward_kernel<NW, NC, true>), grid, dim3(BACK_THREADS), 0, s, a);
    else hipLaunchKernelGGL((backward_kernel<NW, NC, false>), grid, dim3(BACK_THREADS), 0, s, a);
}

template <int NW>
static hipError_t dispatch_backward(int nc, const BackArgs& a, hipStream_t s)
{
    dim3 grid((a.W + TILE_W - 1) / TILE_W, (a.H + TILE_H1 - 1) / TILE_H1, 1);
    switch (nc) {
        case 3: launch_backward_nc<NW, 3>(a, grid, s); break;
        case 5: launch_backward_nc<NW, 5>(a, grid, s); break;
        case 7: launch_backward_nc<NW, 7>(a, grid, s); break;
        case 9: launch_backward_nc<NW, 9>(a, grid, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Backward tiles of several pairs in one launch (level 0 of each pair).
template <int NW, int NC, bool FUSED>
__global__ __launch_bounds__(BACK_THREADS, 2) void backward_multi_kernel(MultiArgs a)
{
    __shared__ BackSmem<NW, BACK_CHUNK> sm;
    const Segment s = a.segs[segment_of(a.segs, a.nseg, blockIdx.x)];
    const int t = blockIdx.x - s.task0;
    backward_tile<NW, NC, FUSED>(a.back[s.pair], t % s.tiles_x, t / s.tiles_x, sm);
}

// Backward tiles of several soft levels of one pair in one launch.  Their
// backwards are independent (each adds into its own level's gradients), so the
// small levels' few tiles run beside level 0's instead of after them.  The
// arguments travel by value: entry i owns blocks [task0[i], task0[i + 1]).
struct BackLevels {
    BackArgs lev[MSIBM_MAX_LEVELS];
    int task0[MSIBM_MAX_LEVELS];
    int tiles_x[MSIBM_MAX_LEVELS];
    int n;
};

template <int NW, int NC>
__global__ __launch_bounds__(BACK_THREADS, 2) void backward_levels_kernel(BackLevels a)
{
    __shared__ BackSmem<NW, BACK_CHUNK> sm;
    int i = 0;
    while (i + 1 < a.n && a.task0[i + 1] <= (int)blockIdx.x) ++i;
    const int t = (int)blockIdx.x - a.task0[i];
    backward_tile<NW, NC, false>(a.lev[i], t % a.tiles_x[i], t / a.tiles_x[i], sm);
}

template <int NW>
static hipError_t dispatch_backward_levels(int nc, const BackLevels& a, int blocks, hipStream_t s)
{
    if (blocks < 1 || a.n < 1 || a.n > MSIBM_MAX_LEVELS) return hipErrorInvalidValue;
    switch (nc) {
        case 3: hipLaunchKernelGGL((backward_levels_kernel<NW, 3>), dim3(blocks), dim3(BACK_THREADS), 0, s, a); break;
        case 5: hipLaunchKernelGGL((backward_levels_kernel<NW, 5>), dim3(blocks), dim3(BACK_THREADS), 0, s, a); break;
        case 7: hipLaunchKernelGGL((backward_levels_kernel<NW, 7>), dim3(blocks), dim3(BACK_THREADS), 0, s, a); break;
        case 9: hipLaunchKernelGGL((backward_levels_kernel<NW, 9>), dim3(blocks), dim3(BACK_THREADS), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_backward_levels_n1(int nc, const BackLevels& a, int blocks, hipStream_t s);
hipError_t launch_backward_levels_n2(int nc, const BackLevels& a, int blocks, hipStream_t s);
hipError_t launch_backward_levels_n3(int nc, const BackLevels& a, int blocks, hipStream_t s);
hipError_t launch_backward_levels_n4(int nc, const BackLevels& a, int blocks, hipStream_t s);
hipError_t launch_backward_levels_n5(int nc, const BackLevels& a, int blocks, hipStream_t s);
hipError_t launch_backward_levels_n6(int nc, const BackLevels& a, int blocks, hipStream_t s);

template <int NW, int NC>
static void launch_backward_multi_nc(const MultiArgs& a, int blocks, hipStream_t s)
{
    if (a.fused) hipLaunchKernelGGL((backward_multi_kernel<NW, NC, true>), dim3(blocks), dim3(BACK_THREADS), 0, s, a);
    else hipLaunchKernelGGL((backward_multi_kernel<NW, NC, false>), dim3(blocks), dim3(BACK_THREADS), 0, s, a);
}

template <int NW>
static hipError_t dispatch_backward_multi(int nc, const MultiArgs& a, int blocks, hipStream_t s)
{
    if (blocks < 1 || a.nseg < 1) return hipErrorInvalidValue;
    switch (nc) {
        case 3: launch_backward_multi_nc<NW, 3>(a, blocks, s); break;
        case 5: launch_backward_multi_nc<NW, 5>(a, blocks, s); break;
        case 7: launch_backward_multi_nc<NW, 7>(a, blocks, s); break;
        case 9: launch_backward_multi_nc<NW, 9>(a, blocks, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace msibm
