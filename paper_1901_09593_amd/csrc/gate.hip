// Confidence gating of one level (Section III.B Eqs. 5-7, Section III.C Eqs.
// 8-9) and the bicubic doubling of a coarser cost map that drives it.
//
// Both gating steps need, for a tile of pixels, the score of every candidate
// z of the full interval: the fallback full search (pixels whose upsampled
// coarser cost is at most beta) takes each pixel's best z, and the re-pick
// (pixels whose cost is at most alpha) takes the best z of the scores averaged
// over each pixel's 5x5 neighbourhood.  One workgroup handles an 8-row tile
// and walks z upwards; at each z it scores a region (the tile, plus the 5x5
// halo for the re-pick) with box sums instead of per-window loops:
//   V(y, e) = sum over the 2n+1 window rows of L(v, e) R(v, e - z)   (columns)
//   S(y, u) = sum over the 2n+1 window columns of V                  (rows)
// so a score costs O(1) instead of O((2n+1)^2) multiply-adds.  With the window
// statistics the cross term is
//   C = S - N mu_l mu_r   (= sum (l - mu_l)(r - mu_r))
// exact in 32-bit integers on a uint8 level and formed in double on a float
// level (its cancellation is what needs the precision), and
// rho = C * invsd_l * invsd_r clamped to [-1, 1], 0 for a flat window
// (invsd = 0).  Tiles without a gated pixel leave at once; the z range stops
// at the rightmost gated pixel's last candidate.
#include <type_traits>

#include "common.hpp"

namespace msibm {

namespace {

constexpr int GT_H = GATE_TH;  // tile rows
constexpr int GT_THREADS = 256;

// Keys' cubic weights (a = -1/2) of the four coarse taps around fine index i
// at scale 2 with aligned pixel centres: the fine pixel sits 3/4 (even i) or
// 1/4 (odd i) past its second tap.  All are multiples of 1/128.
__device__ __forceinline__ double cubic_w(int odd, int m)
{
    const int t = odd ? 3 - m : m;
    return t == 0 ? -3.0 / 128 : t == 1 ? 29.0 / 128 : t == 2 ? 111.0 / 128 : -9.0 / 128;
}

// Bicubic value of the coarser cost at fine pixel (i, j): the 16-tap sum in a
// fixed order with separately rounded products and sums (no contraction), so
// the result does not depend on how the compiler schedules it.
__device__ double upsampled_cost(const float* cc, int Hc, int Wc, int cpitch, int i, int j)
{
    const int i0 = (i >> 1) - 1 + (i & 1), j0 = (j >> 1) - 1 + (j & 1);
    double s = 0.0;
    for (int m = 0; m < 4; ++m) {
        const float* row = cc + (size_t)clampi(i0 - 1 + m, 0, Hc - 1) * cpitch;
        const double wm = cubic_w(i & 1, m);
        for (int q = 0; q < 4; ++q) {
            const double w = __dmul_rn(wm, cubic_w(j & 1, q));
            s = __dadd_rn(s, __dmul_rn(w, (double)row[clampi(j0 - 1 + q, 0, Wc - 1)]));
        }
    }
    return s;
}

__global__ __launch_bounds__(256) void upsample_kernel(const float* cc, int Hc, int Wc, int cpitch, int H,
                                                       int W, double* out, int opitch)
{
    const int j = blockIdx.x * 64 + (threadIdx.x & 63), i = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= H || j >= W) return;
    out[(size_t)i * opitch + j] = upsampled_cost(cc, Hc, Wc, cpitch, i, j);
}

// MODE: GATE_FULL (the fallback full search), GATE_REPICK (the averaged-score
// re-pick), GATE_FUSED (both in one walk: the fallback search's scores of the
// tile pixels are region scores of the re-pick, and the re-pick decision needs
// the fallback's result only at the end).
constexpr int GATE_FULL = GATE_MODE_FULL, GATE_REPICK = GATE_MODE_REPICK, GATE_FUSED = GATE_MODE_FUSED;

// ---- the three-pass tile ---------------------------------------------------
//
// The tile the gating runs on: 8 output rows and as many columns as keep the
// extended region (tile, re-pick halo, windows' halo) within 128 columns.  Per
// candidate three passes share the work:
//  * column pass (lanes 128..255, one column of the extended region each):
//    prefix sums of the products down the column give every (2n+1)-row sum
//    as the difference of two prefixes.  On a uint8 level the left column is
//    held packed four rows to a word and the right column is staged in LDS
//    the same way, so one v_dot4_u32_u8 adds four row products (exact 32-bit
//    integers); on a float level each product is formed exactly in double
//    (the left column held in double, the staged right pixel converted).
//  * row pass (16 lanes per region row, 8 region columns each): a sliding
//    (2n+1)-column sum of the column sums gives S.  uint8: N C = N S - S1_l
//    S1_r is exact (every factor below 2^24, the difference within +-2^31 up
//    to 13x13 windows) and the score is N C * (invsd_l / N) * invsd_r; float:
//    C = S - N mu_l mu_r in double, the score C * invsd_l * invsd_r; both
//    clamped to [-1, 1].  The re-pick's 5-column sums of the scores take the
//    next lane's first four scores across the 16-lane row with a DPP shift.
//  * box pass (re-pick; one output column and four output rows per lane):
//    five-row sums of the 5-column sums.
// Two barriers per candidate: [row pass z] then [column pass z + 1, box pass
// z].  Candidates up to x0 - 2 (x0 for the plain fallback search) lie left of
// every region pixel and leave every output's neighbour count at its full
// value, so they run without the per-pixel candidate checks.
constexpr int GU_EW = GATE_EW;     // extended-region columns
constexpr int GU_RUN = 8;          // region columns a row-pass lane scores
constexpr int GU_VP = 144;         // LDS row pitch of the column and 5-column sums (16 mod 32 banks)

// LDS index of region column u in a row of sums: one pad word per 8 columns,
// so the 16 runs of a row start on 16 distinct banks and the next row's on
// the other 16.
__host__ __device__ constexpr int gu_idx(int u) { return u + (u >> 3); }

// S1_r (an integer) and invsd_r of a uint8 window as one 64-bit register pair.
__device__ __forceinline__ uint64_t pack_stat(const WinStatU8& st)
{
    return ((uint64_t)__float_as_uint(st.z) << 32) | (uint32_t)(int)st.s1;
}

// Lane i of each 16-lane row takes lane i + 1's value (0 past the row's end).
__device__ __forceinline__ float next_lane_in_row(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x101, 0xf, 0xf, true));
}

template <typename T, int NW, int MODE, bool PF = false>
__device__ __forceinline__ void gate_tile_box(const GateArgs& a, int bx, int by)
{
    constexpr bool U8 = std::is_same<T, uint8_t>::value;
    using VT = typename std::conditional<U8, int, double>::type;  // column and window sums
    constexpr bool REPICK = MODE != GATE_FULL;
    constexpr bool FUSED = MODE == GATE_FUSED;
    constexpr int HB = REPICK ? 2 : 0;            // halo of the averaged scores
    constexpr int TH = GATE_TH;
    constexpr int RR = TH + 2 * HB;               // region rows
    constexpr int ER = RR + 2 * NW;               // extended rows
    constexpr int RW = GU_EW - 2 * NW;            // region columns
    constexpr int TW = RW - 2 * HB;               // tile columns
    constexpr int NWORD = (ER + 3) / 4;           // packed 4-row words per column
    constexpr int CP = NWORD | 1;                 // staged column pitch in words (odd: distinct banks)
    // (each staged word is held as its first 1, 2, 3 and 4 rows, 16 bytes)
    constexpr int ZC = U8 ? 32 : 16;              // candidates per staged right chunk
    constexpr int RSC = GU_EW + ZC - 1;           // staged right columns per chunk
    // float levels: a staged column's rows in 16-byte groups, the column pitch
    // 4 mod 8 words so eight lanes' 16-byte reads fall on distinct banks
    constexpr int RP = ((ER + 3) & ~3) % 8 == 0 ? ((ER + 3) & ~3) + 4 : ((ER + 3) & ~3);
    constexpr int VREAD = GU_RUN + 2 * NW;        // column sums a run reads
    constexpr int NN = (2 * NW + 1) * (2 * NW + 1);
    // all 16 runs of a row are scored (uniform lanes); runs past the region
    // read past its column sums and their scores are discarded
    constexpr int VTAIL = gu_idx(GU_RUN * 15 + VREAD - 1) + 1 - GU_VP;
    static_assert(RW <= 16 * GU_RUN && RR * 16 <= 256 && TW <= 128 && gu_idx(GU_EW - 1) < GU_VP && VTAIL > 0,
                  "tile shape");
    static_assert(TW == gate_tile_w(MSIBM_U8, NW, MODE) && TW == gate_tile_w(MSIBM_F32, NW, MODE),
                  "host tile width");

    // the staged right pixels; before the walk and after it the same memory
    // holds the fused mode's fallback flags and results
    constexpr int STAGE_B = U8 ? RSC * CP * 16 : RSC * RP * 4;
    static_assert(!FUSED || 7 * TH * TW <= STAGE_B, "fused arrays fit the staging memory");
    __shared__ uint4 stage_mem[STAGE_B / 16];
    uint4* const RsT = stage_mem;
    float* const RsF = reinterpret_cast<float*>(stage_mem);
    float* const fbe = reinterpret_cast<float*>(stage_mem);
    short* const fbz = reinterpret_cast<short*>(fbe + TH * TW);
    uint8_t* const fgs = reinterpret_cast<uint8_t*>(fbz + TH * TW);
    __shared__ __attribute__((aligned(16))) float LsF[U8 ? 1 : GU_EW * RP];  // float: the left columns
    // uint8 tiles up to 9 x 9 windows walk the candidates in a pipeline (the
    // row pass of z beside the column pass of z + 1 and the box pass of z - 1,
    // one barrier per candidate), with the column and 5-column sums in two
    // buffers by candidate parity, within the 40 KB that keep four workgroups
    // on a CU; float tiles (double column sums) and larger windows would lose a
    // workgroup per CU, and take two barriers per candidate and one buffer,
    // except in the float launches too small to fill two workgroups per CU
    // (PF), where the residency does not matter
    constexpr bool PIPE = U8 ? NW <= 4 : PF;
    constexpr int NB = PIPE ? 2 : 1;
    constexpr int VSZ = RR * GU_VP + VTAIL, HSZ = REPICK ? RR * GU_VP : 1;
    __shared__ VT Vs[NB * VSZ];
    __shared__ float Hs[NB * HSZ];
    __shared__ float rcpT[36];
    __shared__ int s_xmax;

    const int tid = threadIdx.x;
    const int x0 = bx * TW, y0 = by * TH;
    const int ry0 = y0 - HB, rx0 = x0 - HB;       // region origin
    const int ey0 = ry0 - NW, ex0 = rx0 - NW;     // extended origin
    const int H = a.H, W = a.W;
    const T* Limg = (const T*)a.L;
    const T* Rimg = (const T*)a.R;

    // row-pass lanes: 16 per region row; with the re-pick halo the first wave
    // takes the four halo rows, so the fallback tracking skips it as a whole
    const int g = tid >> 4, kr = tid & 15;
    int sy = g;
    if constexpr (REPICK) sy = g < 2 ? g : (g < 4 ? g + RR - 4 : g - 2);
    const bool scorer = g < RR;
    const int su = kr * GU_RUN;
    // column-pass lanes
    const bool colw = tid >= 256 - GU_EW;
    const int ce = tid - (256 - GU_EW);
    // box-pass lanes (re-pick): output column bc (none past the tile), rows
    // 4 bh .. 4 bh + 3
    const int bc = tid & 127, bh = tid >> 7;
    const bool boxer = REPICK && bc < TW;  // owns outputs

    if (tid == 0) s_xmax = -1;
    if (tid < 36) {
        const int r = tid / 6, c = tid - 6 * r;
        rcpT[tid] = (r > 0 && c > 0) ? 1.f / (float)(r * c) : 0.f;
    }
    __syncthreads();

    // owned output pixels: the box lanes' four (re-pick), else the row lanes' run
    constexpr int OWN = REPICK ? 4 : GU_RUN;
    bool act[OWN], fg[OWN];
#pragma unroll
    for (int p = 0; p < OWN; ++p) {
        const int t = REPICK ? 4 * bh + p : sy;
        const int tx = REPICK ? bc : su + p;
        const bool own = REPICK ? boxer : (scorer && su + p < TW);
        const int i = y0 + t, j = x0 + tx;
        act[p] = false;
        fg[p] = false;
        if (own && i < H && j < W) {
            if constexpr (MODE == GATE_REPICK) {
                act[p] = !((double)a.c[(size_t)i * a.opitch + j] > a.thresh);
            } else if constexpr (MODE == GATE_FULL) {
                act[p] = !(upsampled_cost(a.ccost, a.Hc, a.Wc, a.cpitch, i, j) > a.thresh);
            } else {
                fg[p] = !(upsampled_cost(a.ccost, a.Hc, a.Wc, a.cpitch, i, j) > a.thresh2);
                act[p] = fg[p] || !((double)a.c[(size_t)i * a.opitch + j] > a.thresh);
            }
            if (act[p]) atomicMax(&s_xmax, j);
        }
        if constexpr (FUSED)
            if (own) fgs[t * TW + tx] = fg[p];
    }
    __syncthreads();
    const int xmax = s_xmax;
    if (xmax < 0) return;  // uniform: no gated pixel in the tile
    const int zmax = min(a.Dk - 1, xmax);
    const int zbulk = x0 - HB;  // last candidate valid for the whole region (none if negative)

    // ---- row-pass state: left statistics, right statistics of the run at the
    // current candidate, and the tracked best of the fallback (or plain) search
    // uint8: -S1_l and invsd_l / N; float: N mu_l and invsd_l (invsd 0
    // outside the image: the score is 0)
    int ns1l[U8 ? GU_RUN : 1];
    double nmul[U8 ? 1 : GU_RUN];
    float isn[GU_RUN];
    // the right statistics at the current candidate.  uint8: S1_r (low half)
    // and invsd_r (high half) in one 64-bit register pair per column, so the
    // shift per candidate moves pairs; float: mu_r and invsd_r
    uint64_t rst[U8 ? GU_RUN : 1];
    double rmu[U8 ? 1 : GU_RUN];
    float ris[U8 ? 1 : GU_RUN];
    float tb[GU_RUN];   // tracked best (4: never replaced)
    int tz[GU_RUN];
    const int yy = ry0 + sy;
    using SR = typename std::conditional<U8, WinStatU8, WinStat>::type;
    const SR* srow = reinterpret_cast<const SR*>(a.statR) + (size_t)clampi(yy, 0, H - 1) * a.spitch;
    auto shift_in = [&](int q, const SR& st) {
        if constexpr (U8) {
            rst[q] = pack_stat(st);
        } else {
            rmu[q] = (double)st.x + (double)st.y;
            ris[q] = st.z;
        }
    };
#pragma unroll
    for (int q = 0; q < GU_RUN; ++q) {
        const int xx = rx0 + su + q;
        const bool in = scorer && su + q < RW && yy >= 0 && yy < H && xx >= 0 && xx < W;
        if constexpr (U8) ns1l[q] = 0;
        else nmul[q] = 0.0;
        isn[q] = 0.f;
        if (in) {
            const SR st = reinterpret_cast<const SR*>(a.statL)[(size_t)yy * a.spitch + xx];
            if constexpr (U8) {
                ns1l[q] = -(int)st.s1;
                isn[q] = st.z * (float)(1.0 / NN);
            } else {
                nmul[q] = (double)NN * ((double)st.x + (double)st.y);
                isn[q] = st.z;
            }
        }
        const int ty = sy - HB, tx = su + q - HB;
        bool trk = false;
        if constexpr (FUSED) trk = scorer && ty >= 0 && ty < TH && tx >= 0 && tx < TW && fgs[ty * TW + tx];
        else if constexpr (!REPICK) trk = act[q];
        tb[q] = trk ? -3.0f : 4.0f;
        tz[q] = 0;
        // the run's right statistics at candidate -1 (each row pass first
        // shifts them to its own candidate)
        shift_in(q, scorer ? srow[clampi(xx + 1, 0, W - 1)] : SR{});
    }
    SR nxt{};
    if (scorer) nxt = srow[clampi(rx0 + su, 0, W - 1)];
    // the fallback tracking skips the halo-only first wave (re-pick modes)
    const bool track_wave = !REPICK || (FUSED && __builtin_amdgcn_readfirstlane(tid) >= 64);

    // ---- column-pass state: the left column, packed four rows to a word
    // (uint8), or staged in LDS and widened at each use (float)
    uint32_t Lw[U8 ? NWORD : 1];
    {
        const int xx = clampi(ex0 + ce, 0, W - 1);
        if constexpr (U8) {
#pragma unroll
            for (int k = 0; k < NWORD; ++k) {
                uint32_t w = 0;
                if (colw) {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (4 * k + i < ER)
                            w |= (uint32_t)Limg[(size_t)clampi(ey0 + 4 * k + i, 0, H - 1) * a.pitch + xx]
                                 << (8 * i);
                }
                Lw[k] = w;
            }
        } else {
            if (colw)
                for (int t = 0; t < ER; ++t)
                    LsF[ce * RP + t] = (float)Limg[(size_t)clampi(ey0 + t, 0, H - 1) * a.pitch + xx];
        }
    }

    // ---- box-pass state
    // (neighbour counts: rows inside the image times columns inside at or
    // right of the pixel, plus the columns left of it the candidate allows;
    // reciprocals from the table, the full-row one held)
    float bb[4];
    int bzv[4];
    float r5[4];
    const int bj = x0 + bc;
    const int cols_r = max(1, min(bj + 2, W - 1) - bj + 1);
    auto rows_in = [&](int p) {
        const int i = y0 + 4 * bh + p;
        return max(1, min(i + 2, H - 1) - max(i - 2, 0) + 1);
    };
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        bb[p] = (REPICK && act[p & (OWN - 1)]) ? -3.0f : 4.0f;
        bzv[p] = 0;
        r5[p] = 1.f / (float)(rows_in(p) * (cols_r + 2));
    }

    // right columns ex0 - zhi .. ex0 - zhi + RSC - 1 of the extended rows for
    // the chunk of candidates ending at zhi, packed four rows to a word
    auto stage = [&](int zc) {
        const int zhi = zc + ZC - 1;
        if constexpr (!U8) {
            // float: one pixel per lane and step, columns fastest
            for (int idx = tid; idx < RSC * ER; idx += 256) {
                const int v = idx / RSC, col = idx - v * RSC;
                RsF[col * RP + v] =
                    Rimg[(size_t)clampi(ey0 + v, 0, H - 1) * a.pitch + clampi(ex0 - zhi + col, 0, W - 1)];
            }
            return;
        }
        for (int idx = tid; idx < RSC * NWORD; idx += 256) {
            const int w = idx / RSC, col = idx - w * RSC;
            const int xx = clampi(ex0 - zhi + col, 0, W - 1);
            uint32_t word = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (4 * w + i < ER)
                    word |= (uint32_t)Rimg[(size_t)clampi(ey0 + 4 * w + i, 0, H - 1) * a.pitch + xx] << (8 * i);
            RsT[col * CP + w] = make_uint4(word & 0xffu, word & 0xffffu, word & 0xffffffu, word);
        }
    };

    // column sums of the products at candidate z: V(y) = P(y + 2n + 1) - P(y)
    // with P the prefix sums down the column (a partial word's products take
    // the right word cut to its first rows)
    auto colpass = [&](int z) {
        const int zhi = (z & ~(ZC - 1)) + ZC - 1;
        if constexpr (!U8) {
            // each column sum is written as soon as its upper prefix exists,
            // so at most 2n + 2 prefixes are live
            const float4* rc = reinterpret_cast<const float4*>(RsF + (ce + zhi - z) * RP);
            const float4* lc = reinterpret_cast<const float4*>(LsF + ce * RP);
            VT* vc = Vs + (z & (NB - 1)) * VSZ + gu_idx(ce);
            double P[ER + 1];
            P[0] = 0.0;
#pragma unroll
            for (int k = 0; k < (ER + 3) / 4; ++k) {
                const float4 r4 = rc[k], l4 = lc[k];
                const float rv[4] = {r4.x, r4.y, r4.z, r4.w}, lv[4] = {l4.x, l4.y, l4.z, l4.w};
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int t = 4 * k + i + 1;
                    if (t <= ER) {
                        P[t] = fma((double)lv[i], (double)rv[i], P[t - 1]);
                        if (t >= 2 * NW + 1) vc[(t - 2 * NW - 1) * GU_VP] = P[t] - P[t - 2 * NW - 1];
                    }
                }
            }
            return;
        }
        const uint4* rc = RsT + (ce + zhi - z) * CP;
        uint32_t P[4 * NWORD + 1];
        P[0] = 0;
#pragma unroll
        for (int k = 0; k < NWORD; ++k) {
            const uint4 rw = rc[k];
            const uint32_t cut[4] = {rw.x, rw.y, rw.z, rw.w};
#pragma unroll
            for (int m = 1; m <= 4; ++m)
                if (4 * k + m <= ER) P[4 * k + m] = __builtin_amdgcn_udot4(Lw[k], cut[m - 1], P[4 * k], false);
        }
        VT* vc = Vs + (z & (NB - 1)) * VSZ + gu_idx(ce);
#pragma unroll
        for (int y = 0; y < RR; ++y) vc[y * GU_VP] = (int)(P[y + 2 * NW + 1] - P[y]);
    };

    // scores of the run at candidate z, the tracked best, and (re-pick) the
    // run's 5-column sums of the scores
    auto rowpass = [&](int z, auto bulk_tag) {
        constexpr bool BULK = decltype(bulk_tag)::value;
        // column q at z is column q - 1 at z - 1: one new right statistic
#pragma unroll
        for (int q = GU_RUN - 1; q > 0; --q) {
            if constexpr (U8) {
                rst[q] = rst[q - 1];
            } else {
                rmu[q] = rmu[q - 1];
                ris[q] = ris[q - 1];
            }
        }
        shift_in(0, nxt);
        nxt = srow[clampi(rx0 + su - (z + 1), 0, W - 1)];
        const VT* vr = Vs + (z & (NB - 1)) * VSZ + sy * GU_VP + gu_idx(su);
        VT v[VREAD];
#pragma unroll
        for (int b = 0; b < VREAD; ++b) v[b] = vr[gu_idx(b)];
        VT S = 0;
#pragma unroll
        for (int b = 0; b <= 2 * NW; ++b) S += v[b];
        float E[GU_RUN];
#pragma unroll
        for (int q = 0; q < GU_RUN; ++q) {
            if (q > 0) S += v[q + 2 * NW] - v[q - 1];
            float e;
            if constexpr (U8) {
                const int rs1 = (int)(uint32_t)rst[q];
                const float rz = __uint_as_float((uint32_t)(rst[q] >> 32));
                const int nc = (int)__umul24((unsigned)NN, (unsigned)S) + __mul24(ns1l[q], rs1);  // N C
                e = fminf(1.f, fmaxf(-1.f, (float)nc * isn[q] * rz));
            } else {
                const float c = (float)fma(-nmul[q], rmu[q], S);  // C
                e = fminf(1.f, fmaxf(-1.f, c * isn[q] * ris[q]));
            }
            bool valid = true;
            if constexpr (!BULK) {
                valid = z <= rx0 + su + q;
                e = valid ? e : 0.f;
            }
            E[q] = e;
        }
        if constexpr (!REPICK || FUSED) {
            if (track_wave) {
#pragma unroll
                for (int q = 0; q < GU_RUN; ++q) {
                    const bool better = (BULK || z <= rx0 + su + q) && E[q] > tb[q];
                    tb[q] = better ? E[q] : tb[q];
                    tz[q] = better ? z : tz[q];
                }
            }
        }
        if constexpr (REPICK) {
            // H(q) = E(q) + .. + E(q + 4), sliding; E(8..11) are the next
            // run's first four scores
            float Ex[GU_RUN + 4];
#pragma unroll
            for (int q = 0; q < GU_RUN; ++q) Ex[q] = E[q];
#pragma unroll
            for (int m = 0; m < 4; ++m) Ex[GU_RUN + m] = next_lane_in_row(E[m]);
            float* hr = Hs + (z & (NB - 1)) * HSZ + sy * GU_VP + gu_idx(su);
            float h = ((Ex[0] + Ex[1]) + (Ex[2] + Ex[3])) + Ex[4];
            hr[0] = h;
#pragma unroll
            for (int q = 1; q < GU_RUN; ++q) {
                h += Ex[q + 4] - Ex[q - 1];
                hr[q] = h;
            }
        }
    };

    // 5x5 sums of the scores at candidate z for the lane's four outputs
    auto boxpass = [&](int z, auto bulk_tag) {
        constexpr bool BULK = decltype(bulk_tag)::value;
        const float* hc = Hs + (z & (NB - 1)) * HSZ + 4 * bh * GU_VP + gu_idx(bc);
        float h[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) h[m] = hc[m * GU_VP];
        const float s01 = h[0] + h[1], s23 = h[2] + h[3], s45 = h[4] + h[5], s67 = h[6] + h[7];
        const float s2345 = s23 + s45;
        const float A[4] = {(s01 + s23) + h[4], h[1] + s2345, s2345 + h[6], h[3] + (s45 + s67)};
        const int left = (z <= bj - 2) ? 2 : (z == bj - 1 ? 1 : 0);
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const float rc = BULK ? r5[p] : rcpT[rows_in(p) * 6 + cols_r + left];
            const float ebar = A[p] * rc;
            const bool better = (BULK || z <= bj) && ebar > bb[p];
            bb[p] = better ? ebar : bb[p];
            bzv[p] = better ? z : bzv[p];
        }
    };

    // one candidate: [row pass z] [column pass z + 1, box pass z]
    auto step = [&](int z, auto bulk_tag) {
        if (scorer) rowpass(z, bulk_tag);
        const int zn = z + 1;
        if (zn <= zmax && (zn & (ZC - 1)) == 0) stage(zn);  // the row pass reads no staged pixel
        __syncthreads();
        if (colw && zn <= zmax) colpass(zn);
        if constexpr (REPICK) boxpass(z, bulk_tag);  // every lane (those past the tile own nothing)
        __syncthreads();
    };
    if constexpr (FUSED) __syncthreads();  // the fallback flags are read: the staging memory is free
    stage(0);
    __syncthreads();
    if (colw) colpass(0);
    __syncthreads();
    // the candidates valid for the whole region, then the rest (separate
    // loops: no merge of the two forms inside the loop)
    const int zb = min(zbulk, zmax);
    if constexpr (PIPE) {
        using Tt = std::true_type;
        using Ft = std::false_type;
        // phase t: [staging of the chunk starting at t + 1 and a barrier]
        // [row pass t, column pass t + 1, box pass t - 1]
        auto phase = [&](int t, auto row_tag, auto box_tag, bool row, bool box) {
            const int zn = t + 1;
            if (zn <= zmax && (zn & (ZC - 1)) == 0) {  // the column pass of t read the last chunk
                stage(zn);
                __syncthreads();
            }
            if (row && scorer) rowpass(t, row_tag);
            if (colw && zn <= zmax) colpass(zn);
            if constexpr (REPICK)
                if (box) boxpass(t - 1, box_tag);
            __syncthreads();
        };
        if (zb >= 0) phase(0, Tt{}, Tt{}, true, false);
        else phase(0, Ft{}, Ft{}, true, false);
        // the loops take phases two at a time from an odd candidate (written
        // 2k + 1 and 2k + 2, so each phase's buffer parity is a constant)
        int t = 1;
        for (int k = 0; 2 * k + 2 <= zb; ++k) {
            phase(2 * k + 1, Tt{}, Tt{}, true, true);
            phase(2 * k + 2, Tt{}, Tt{}, true, true);
            t = 2 * k + 3;
        }
        if (t <= zb) phase(t++, Tt{}, Tt{}, true, true);
        if (zb >= 0 && t == zb + 1 && t <= zmax) {
            phase(t, Ft{}, Tt{}, true, true);
            ++t;
        }
        if (t <= zmax && !(t & 1)) phase(t++, Ft{}, Ft{}, true, true);
        for (int k = t >> 1; 2 * k + 2 <= zmax; ++k) {
            phase(2 * k + 1, Ft{}, Ft{}, true, true);
            phase(2 * k + 2, Ft{}, Ft{}, true, true);
            t = 2 * k + 3;
        }
        if (t <= zmax) phase(t++, Ft{}, Ft{}, true, true);
        if constexpr (REPICK) {
            if (zb == zmax) phase(zmax + 1, Ft{}, Tt{}, false, true);
            else phase(zmax + 1, Ft{}, Ft{}, false, true);
        }
    } else {
        int z = 0;
        for (; z <= zb; ++z) step(z, std::true_type{});
        for (; z <= zmax; ++z) step(z, std::false_type{});
    }

    if constexpr (FUSED) {
        // the fallback results to their owners
        if (scorer) {
#pragma unroll
            for (int q = 0; q < GU_RUN; ++q) {
                const int ty = sy - HB, tx = su + q - HB;
                if (ty >= 0 && ty < TH && tx >= 0 && tx < TW) {
                    fbe[ty * TW + tx] = tb[q];
                    fbz[ty * TW + tx] = (short)tz[q];
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int p = 0; p < OWN; ++p) {
        if (!act[p]) continue;
        const int t = REPICK ? 4 * bh + p : sy;
        const int tx = REPICK ? bc : su + p;
        const size_t o = (size_t)(y0 + t) * a.opitch + (x0 + tx);
        if constexpr (FUSED) {
            // Eqs. 8-9 (the fallback or the restricted search's result), then
            // Eqs. 5-7 on that cost
            const int d1 = fg[p] ? (int)fbz[t * TW + tx] : (int)a.d[o];
            const float c1 = fg[p] ? fbe[t * TW + tx] : a.c[o];
            const bool pick = !((double)c1 > a.thresh);
            a.d[o] = (int16_t)(pick ? bzv[p] : d1);
            a.c[o] = pick ? bb[p] : c1;
        } else if constexpr (REPICK) {
            a.d[o] = (int16_t)bzv[p];
            a.c[o] = bb[p];
        } else {
            a.d[o] = (int16_t)tz[p];
            a.c[o] = tb[p];
        }
    }
}

// uint8 tiles at most 128 VGPRs (four waves per SIMD), float ones 168
// (three), the float pipelined ones 256 (two: their LDS holds two per CU)
template <typename T, bool PF>
constexpr int GATE_MIN_WAVES = std::is_same<T, uint8_t>::value ? 4 : (PF ? 2 : 3);
// float launches of at most this many workgroups take the pipelined walk
constexpr int GATE_PF_MAX_BLOCKS = 512;

template <typename T, int NW, int MODE, bool PF>
__device__ __forceinline__ void gate_tile_any(const GateArgs& a, int bx, int by)
{
    gate_tile_box<T, NW, MODE, PF>(a, bx, by);
}

template <typename T, int NW, int MODE, bool PF>
__global__ __launch_bounds__(GT_THREADS, (GATE_MIN_WAVES<T, PF>)) void gate_kernel(GateArgs a)
{
    gate_tile_any<T, NW, MODE, PF>(a, blockIdx.x, blockIdx.y);
}

// Gating of several (pair, level) segments of one mode and element type in one
// launch; a level's map and cost are those its search wrote (the scratch map
// with the median), the coarser level's cost that of its own gating.
template <typename T, int NW, int MODE, bool PF>
__global__ __launch_bounds__(GT_THREADS, (GATE_MIN_WAVES<T, PF>)) void gate_multi_kernel(MultiArgs m)
{
    const Segment s = m.segs[segment_of(m.segs, m.nseg, blockIdx.x)];
    const LevelDesc* lv = m.levels + m.level_base[s.pair];
    const LevelDesc& L = lv[s.level];
    GateArgs g{};
    g.L = L.img[0];
    g.R = L.img[1];
    g.pitch = L.pitch;
    g.H = L.H;
    g.W = L.W;
    g.Dk = L.Dk;
    g.statL = L.stat[0];
    g.statR = L.stat[1];
    g.spitch = L.W;
    g.d = L.raw ? L.raw : L.map;
    g.c = L.raw ? L.mcost : L.cost;
    g.opitch = L.W;
    g.thresh = m.gate_alpha;
    g.thresh2 = m.gate_beta;
    if (MODE != GATE_REPICK) {
        const LevelDesc& C = lv[s.level + 1];
        g.ccost = C.raw ? C.mcost : C.cost;
        g.Hc = C.H;
        g.Wc = C.W;
        g.cpitch = C.W;
    }
    const int t = blockIdx.x - s.task0;
    gate_tile_any<T, NW, MODE, PF>(g, t % s.tiles_x, t / s.tiles_x);
}

template <typename T, int MODE, bool PF>
hipError_t launch_gate_multi_p(int n, const MultiArgs& a, int blocks, hipStream_t s)
{
    switch (n) {
        case 1: hipLaunchKernelGGL((gate_multi_kernel<T, 1, MODE, PF>), dim3(blocks), dim3(GT_THREADS), 0, s, a); break;
        case 2: hipLaunchKernelGGL((gate_multi_kernel<T, 2, MODE, PF>), dim3(blocks), dim3(GT_THREADS), 0, s, a); break;
        case 3: hipLaunchKernelGGL((gate_multi_kernel<T, 3, MODE, PF>), dim3(blocks), dim3(GT_THREADS), 0, s, a); break;
        case 4: hipLaunchKernelGGL((gate_multi_kernel<T, 4, MODE, PF>), dim3(blocks), dim3(GT_THREADS), 0, s, a); break;
        case 5: hipLaunchKernelGGL((gate_multi_kernel<T, 5, MODE, PF>), dim3(blocks), dim3(GT_THREADS), 0, s, a); break;
        case 6: hipLaunchKernelGGL((gate_multi_kernel<T, 6, MODE, PF>), dim3(blocks), dim3(GT_THREADS), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int MODE>
hipError_t launch_gate_multi_t(int n, const MultiArgs& a, int blocks, hipStream_t s)
{
    if constexpr (!std::is_same<T, uint8_t>::value)
        if (blocks <= GATE_PF_MAX_BLOCKS) return launch_gate_multi_p<T, MODE, true>(n, a, blocks, s);
    return launch_gate_multi_p<T, MODE, false>(n, a, blocks, s);
}

template <typename T, int MODE, bool PF>
hipError_t launch_gate_p(int n, const GateArgs& a, dim3 grid, hipStream_t s)
{
    switch (n) {
        case 1: hipLaunchKernelGGL((gate_kernel<T, 1, MODE, PF>), grid, dim3(GT_THREADS), 0, s, a); break;
        case 2: hipLaunchKernelGGL((gate_kernel<T, 2, MODE, PF>), grid, dim3(GT_THREADS), 0, s, a); break;
        case 3: hipLaunchKernelGGL((gate_kernel<T, 3, MODE, PF>), grid, dim3(GT_THREADS), 0, s, a); break;
        case 4: hipLaunchKernelGGL((gate_kernel<T, 4, MODE, PF>), grid, dim3(GT_THREADS), 0, s, a); break;
        case 5: hipLaunchKernelGGL((gate_kernel<T, 5, MODE, PF>), grid, dim3(GT_THREADS), 0, s, a); break;
        case 6: hipLaunchKernelGGL((gate_kernel<T, 6, MODE, PF>), grid, dim3(GT_THREADS), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int MODE>
hipError_t launch_gate_t(int n, const GateArgs& a, hipStream_t s)
{
    const int tw = gate_tile_w(std::is_same<T, uint8_t>::value ? MSIBM_U8 : MSIBM_F32, n, MODE);
    dim3 grid((a.W + tw - 1) / tw, (a.H + GT_H - 1) / GT_H, 1);
    // (the separate gated search, mode GATE_FULL, keeps one form)
    if constexpr (!std::is_same<T, uint8_t>::value && MODE != GATE_FULL)
        if ((long)grid.x * grid.y <= GATE_PF_MAX_BLOCKS) return launch_gate_p<T, MODE, true>(n, a, grid, s);
    return launch_gate_p<T, MODE, false>(n, a, grid, s);
}

}  // namespace

hipError_t launch_gate(int n, int dtype, int mode, const GateArgs& a, hipStream_t s)
{
    if (a.H < 1 || a.W < 1 || a.Dk < 1) return hipErrorInvalidValue;
    if (mode != GATE_REPICK && (a.Hc != (a.H + 1) / 2 || a.Wc != (a.W + 1) / 2)) return hipErrorInvalidValue;
    if (dtype == MSIBM_U8) {
        if (mode == GATE_FULL) return launch_gate_t<uint8_t, GATE_FULL>(n, a, s);
        if (mode == GATE_REPICK) return launch_gate_t<uint8_t, GATE_REPICK>(n, a, s);
        return launch_gate_t<uint8_t, GATE_FUSED>(n, a, s);
    }
    if (mode == GATE_FULL) return launch_gate_t<float, GATE_FULL>(n, a, s);
    if (mode == GATE_REPICK) return launch_gate_t<float, GATE_REPICK>(n, a, s);
    return launch_gate_t<float, GATE_FUSED>(n, a, s);
}

hipError_t launch_gate_multi(int n, int dtype, int mode, const MultiArgs& a, int blocks, hipStream_t s)
{
    if (blocks < 1 || a.nseg < 1 || (mode != GATE_REPICK && mode != GATE_FUSED)) return hipErrorInvalidValue;
    if (dtype == MSIBM_U8)
        return mode == GATE_REPICK ? launch_gate_multi_t<uint8_t, GATE_REPICK>(n, a, blocks, s)
                                   : launch_gate_multi_t<uint8_t, GATE_FUSED>(n, a, blocks, s);
    return mode == GATE_REPICK ? launch_gate_multi_t<float, GATE_REPICK>(n, a, blocks, s)
                               : launch_gate_multi_t<float, GATE_FUSED>(n, a, blocks, s);
}

hipError_t launch_upsample_cost(const float* cc, int Hc, int Wc, int cpitch, int H, int W, double* out,
                                int opitch, hipStream_t s)
{
    dim3 grid((W + 63) / 64, (H + 3) / 4, 1);
    hipLaunchKernelGGL(upsample_kernel, grid, dim3(256), 0, s, cc, Hc, Wc, cpitch, H, W, out, opitch);
    return hipGetLastError();
}

}  // namespace msibm
