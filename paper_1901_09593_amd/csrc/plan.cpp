// Launch sequences of the plain (one pair at a time) forward pass.
#include <hip/hip_runtime.h>

#include "backward_impl.hpp"
#include "common.hpp"
#include "plan.hpp"
#include "timing.hpp"
#include "tune.hpp"

#include <cstdio>
#include <cstdlib>

namespace msibm {

hipError_t launch_match(int n, int dtype, int mode, int nc, const MatchArgs& a, hipStream_t s)
{
    switch (n) {
        case 1: return launch_match_n1(dtype, mode, nc, a, s);
        case 2: return launch_match_n2(dtype, mode, nc, a, s);
        case 3: return launch_match_n3(dtype, mode, nc, a, s);
        case 4: return launch_match_n4(dtype, mode, nc, a, s);
        case 5: return launch_match_n5(dtype, mode, nc, a, s);
        case 6: return launch_match_n6(dtype, mode, nc, a, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_match_multi(int n, int dtype, int mode, int nc, const MultiArgs& a, int blocks, hipStream_t s)
{
    switch (n) {
        case 1: return launch_match_multi_n1(dtype, mode, nc, a, blocks, s);
        case 2: return launch_match_multi_n2(dtype, mode, nc, a, blocks, s);
        case 3: return launch_match_multi_n3(dtype, mode, nc, a, blocks, s);
        case 4: return launch_match_multi_n4(dtype, mode, nc, a, blocks, s);
        case 5: return launch_match_multi_n5(dtype, mode, nc, a, blocks, s);
        case 6: return launch_match_multi_n6(dtype, mode, nc, a, blocks, s);
    }
    return hipErrorInvalidValue;
}

static int hip_err(hipError_t e, const char* what, std::string* err)
{
    *err = std::string(what) + ": " + hipGetErrorString(e);
    return MSIBM_ERR_HIP;
}

hipError_t launch_backward_levels(int n, int nc, const BackLevels& a, int blocks, hipStream_t s);

// Level images of a pair: level 0 is the caller's input, levels k >= 1 are
// built into the workspace, up to three reduce steps per launch.
static int build_pyramid(const msibm_pair& P, const PairLayout& lay, char* ws, const void* img[][2], int* pitch,
                         hipStream_t s, std::string* err)
{
    const int K = lay.K;
    hipError_t e = hipSuccess;
    img[0][0] = P.left;
    img[0][1] = P.right;
    pitch[0] = P.pitch;
    // the pyramid: up to three steps per launch
    for (int k = 1; k < K;) {
        const int steps = K - k < TW_MAXS ? K - k : TW_MAXS;
        const int dt = k == 1 ? P.dtype : MSIBM_F32;
        for (int j = 0; j < steps; ++j) {
            img[k + j][0] = ws + lay.img[k + j][0];
            img[k + j][1] = ws + lay.img[k + j][1];
            pitch[k + j] = lay.w[k + j];
        }
        char lab[32];
        snprintf(lab, sizeof(lab), steps == 1 ? "reduce_l%d" : "pyramid_l%d", k);
        TimedLaunch t(lab, s);
        if (steps == 1) {
            ReduceArgs r{};
            r.src[0] = img[k - 1][0];
            r.src[1] = img[k - 1][1];
            r.dst[0] = (float*)img[k][0];
            r.dst[1] = (float*)img[k][1];
            r.views = 2;
            r.H = lay.h[k - 1];
            r.W = lay.w[k - 1];
            r.spitch = pitch[k - 1];
            r.Ho = lay.h[k];
            r.Wo = lay.w[k];
            r.dpitch = lay.w[k];
            e = launch_reduce(dt, r, s);
        } else {
            TowerArgs ta{};
            ta.src[0] = img[k - 1][0];
            ta.src[1] = img[k - 1][1];
            ta.Hs = lay.h[k - 1];
            ta.Ws = lay.w[k - 1];
            ta.spitch = pitch[k - 1];
            for (int j = 0; j < steps; ++j) {
                ta.dst[j][0] = (float*)img[k + j][0];
                ta.dst[j][1] = (float*)img[k + j][1];
                ta.H[j] = lay.h[k + j];
                ta.W[j] = lay.w[k + j];
            }
            ta.steps = steps;
            e = launch_tower(dt, ta, s);
        }
        if (e != hipSuccess) return hip_err(e, "pyramid launch", err);
        k += steps;
    }
    return MSIBM_OK;
}

// Window statistics of every level: one launch per distinct window size.
static int build_stats(const PairLayout& lay, const msibm_config* cfg, char* ws, const void* const img[][2],
                       const int* pitch, const int* dtype, hipStream_t s, std::string* err)
{
    const int K = lay.K;
    for (int k0 = 0; k0 < K; ++k0) {
        bool first = true;
        for (int k = 0; k < k0; ++k) first = first && level_n(cfg, k) != level_n(cfg, k0);
        if (!first) continue;
        StatsArgs sa{};
        for (int k = k0; k < K; ++k) {
            if (level_n(cfg, k) != level_n(cfg, k0)) continue;
            for (int v = 0; v < 2; ++v)
                sa.seg[sa.nseg++] = StatsSeg{img[k][v], (WinStat*)(ws + lay.stat[k][v]), dtype[k], lay.h[k],
                                             lay.w[k], pitch[k], lay.w[k], 0};
        }
        sa.n = level_n(cfg, k0);
        sa.var_eps = cfg->var_eps;
        TimedLaunch t("stats", s);
        const hipError_t e = launch_stats(sa, s);
        if (e != hipSuccess) return hip_err(e, "stats launch", err);
    }
    return MSIBM_OK;
}

int run_pair_plain(const msibm_pair& P, const PairLayout& lay, const msibm_config* cfg, char* ws,
                   int16_t* disp, float* cost, float* soft, int16_t* prior1, hipStream_t s,
                   std::string* err, int lowest_level)
{
    const int K = lay.K;
    hipError_t e;
    // image pointers per level and view (level 0 is the caller's input)
    const void* img[MSIBM_MAX_LEVELS][2];
    int pitch[MSIBM_MAX_LEVELS];
    {
        const int st = build_pyramid(P, lay, ws, img, pitch, s, err);
        if (st != MSIBM_OK) return st;
    }
    // pre-blur variant: level 0 is matched on the blurred input (the pyramid
    // above was built from the input itself)
    const bool preblur = (cfg->flags & MSIBM_FLAG_PREBLUR) != 0;
    if (preblur) {
        BlurArgs b{};
        for (int v = 0; v < 2; ++v) {
            b.src[v] = img[0][v];
            b.dst[v] = (float*)(ws + lay.blur[v]);
        }
        b.H = P.height;
        b.W = P.width;
        b.spitch = P.pitch;
        b.dpitch = P.width;
        TimedLaunch t("preblur_l0", s);
        e = launch_blur(P.dtype, b, s);
        if (e != hipSuccess) return hip_err(e, "blur launch", err);
        img[0][0] = b.dst[0];
        img[0][1] = b.dst[1];
        pitch[0] = P.width;
    }
    // element type of level k's images
    auto dtype_of = [&](int k) { return (k == 0 && !preblur) ? P.dtype : MSIBM_F32; };
    // statistics: one launch per distinct window size (one for a common n)
    {
        int dts[MSIBM_MAX_LEVELS];
        for (int k = 0; k < K; ++k) dts[k] = dtype_of(k);
        const int st = build_stats(lay, cfg, ws, img, pitch, dts, s, err);
        if (st != MSIBM_OK) return st;
    }
    for (int k = K - 1; k >= lowest_level; --k) {
        MatchArgs a{};
        a.L = img[k][0];
        a.R = img[k][1];
        a.H = lay.h[k];
        a.W = lay.w[k];
        a.pitch = pitch[k];
        a.statL = (const WinStat*)(ws + lay.stat[k][0]);
        a.statR = (const WinStat*)(ws + lay.stat[k][1]);
        a.spitch = lay.w[k];
        a.Dk = level_range(P.max_disp, k);
        const bool coarsest = (k == K - 1);
        if (!coarsest) {
            a.prior = (k + 1 == 1 && prior1) ? prior1 : (const int16_t*)(ws + lay.map[k + 1]);
            a.Hc = lay.h[k + 1];
            a.Wc = lay.w[k + 1];
            a.ppitch = lay.w[k + 1];
        }
        const bool soft_level = (k == 0 && cfg->soft_radius > 0);
        a.r = soft_level ? cfg->soft_radius : cfg->refine_radius;
        if (k == 0) {
            a.d_out = disp;
            a.c_out = cost;
            a.soft_out = soft;
        } else {
            a.d_out = (k == 1 && prior1) ? prior1 : (int16_t*)(ws + lay.map[k]);
            a.c_out = nullptr;
            a.soft_out = nullptr;
        }
        a.opitch = lay.w[k];
        a.inv_tau = soft_level ? 1.f / cfg->tau : 0.f;
        const int mode = coarsest ? MODE_FULL : (soft_level ? MODE_SOFT : MODE_REFINE);
        const int nc = coarsest ? FULL_NC : slots_for_radius(a.r);
        char lab[32];
        snprintf(lab, sizeof(lab), "match_%s_l%d",
                 mode == MODE_FULL ? "full" : (mode == MODE_SOFT ? "soft" : "refine"), k);
        // with the selective median, a hard level's map is matched into a
        // scratch map and filtered into its place; the gating keeps every
        // level's cost (the next finer level reads it) and revises the map and
        // cost in place before the filter
        int16_t* const dest = a.d_out;
        const bool filt = (cfg->flags & MSIBM_FLAG_MEDIAN) && mode != MODE_SOFT;
        const bool gated = (cfg->flags & MSIBM_FLAG_GATED) && mode != MODE_SOFT;
        if (gated && k > 0) a.c_out = (float*)(ws + lay.cmap[k]);
        if (filt) a.d_out = (int16_t*)(ws + lay.dtmp);
        if ((filt || gated) && !a.c_out) a.c_out = (float*)(ws + lay.ctmp);
        const int n = level_n(cfg, k);
        {
            TimedLaunch t(lab, s);
            a.variant = select_variant(a, n, dtype_of(k), mode, nc, s);
            e = launch_match(n, dtype_of(k), mode, nc, a, s);
        }
        if (e != hipSuccess) return hip_err(e, "match launch", err);
        if (gated) {
            GateArgs g{};
            g.L = a.L;
            g.R = a.R;
            g.pitch = a.pitch;
            g.H = a.H;
            g.W = a.W;
            g.Dk = a.Dk;
            g.statL = a.statL;
            g.statR = a.statR;
            g.spitch = a.spitch;
            g.d = a.d_out;
            g.c = a.c_out;
            g.opitch = a.opitch;
            // below the coarsest level one walk does both: the full search
            // where the doubled coarser cost is low (Eqs. 8-9), then the
            // re-pick of low-cost pixels (Eqs. 5-7); the coarsest re-picks only
            g.thresh = cfg->gate_alpha;
            g.thresh2 = cfg->gate_beta;
            if (!coarsest) {
                g.ccost = (const float*)(ws + lay.cmap[k + 1]);
                g.Hc = lay.h[k + 1];
                g.Wc = lay.w[k + 1];
                g.cpitch = lay.w[k + 1];
            }
            char glab[32];
            snprintf(glab, sizeof(glab), coarsest ? "gate_repick_l%d" : "gate_fused_l%d", k);
            TimedLaunch t(glab, s);
            e = launch_gate(n, dtype_of(k), coarsest ? GATE_MODE_REPICK : GATE_MODE_FUSED, g, s);
            if (e != hipSuccess) return hip_err(e, "gating launch", err);
        }
        if (filt) {
            MedianArgs m{a.d_out, a.c_out, dest, lay.h[k], lay.w[k], lay.w[k], lay.w[k], lay.w[k],
                         (double)cfg->median_alpha};
            char mlab[32];
            snprintf(mlab, sizeof(mlab), "median_l%d", k);
            TimedLaunch t(mlab, s);
            e = launch_median(m, s);
            if (e != hipSuccess) return hip_err(e, "median launch", err);
        }
    }
    return MSIBM_OK;
}

int run_pair_levels(const msibm_pair& P, const PairLayout& lay, const msibm_config* cfg, char* ws,
                    float* const* soft, int16_t* const* maps, hipStream_t s, std::string* err)
{
    const int K = lay.K;
    const void* img[MSIBM_MAX_LEVELS][2];
    int pitch[MSIBM_MAX_LEVELS];
    int st = build_pyramid(P, lay, ws, img, pitch, s, err);
    if (st != MSIBM_OK) return st;
    int dts[MSIBM_MAX_LEVELS];
    for (int k = 0; k < K; ++k) dts[k] = MSIBM_F32;
    st = build_stats(lay, cfg, ws, img, pitch, dts, s, err);
    if (st != MSIBM_OK) return st;
    for (int k = K - 1; k >= 0; --k) {
        const bool coarsest = (k == K - 1);
        MatchArgs a{};
        a.L = img[k][0];
        a.R = img[k][1];
        a.H = lay.h[k];
        a.W = lay.w[k];
        a.pitch = pitch[k];
        a.statL = (const WinStat*)(ws + lay.stat[k][0]);
        a.statR = (const WinStat*)(ws + lay.stat[k][1]);
        a.spitch = lay.w[k];
        a.Dk = level_range(P.max_disp, k);
        if (!coarsest) {
            a.prior = maps[k + 1];
            a.Hc = lay.h[k + 1];
            a.Wc = lay.w[k + 1];
            a.ppitch = lay.w[k + 1];
        }
        a.r = coarsest ? 0 : cfg->soft_radius;
        a.d_out = maps[k];
        a.c_out = nullptr;
        a.soft_out = coarsest ? nullptr : soft[k];
        a.opitch = lay.w[k];
        a.inv_tau = coarsest ? 0.f : 1.f / cfg->tau;
        const int mode = coarsest ? MODE_FULL : MODE_SOFT;
        const int nc = coarsest ? FULL_NC : slots_for_radius(a.r);
        const int n = level_n(cfg, k);
        char lab[32];
        snprintf(lab, sizeof(lab), "match_%s_l%d", coarsest ? "full" : "soft", k);
        TimedLaunch t(lab, s);
        a.variant = select_variant(a, n, MSIBM_F32, mode, nc, s);
        const hipError_t e = launch_match(n, MSIBM_F32, mode, nc, a, s);
        if (e != hipSuccess) return hip_err(e, "match launch", err);
    }
    return MSIBM_OK;
}

int run_pair_backward_levels(const msibm_pair& P, const PairLayout& lay, const msibm_config* cfg, char* ws,
                             const int16_t* const* maps, const float* const* grad_soft, float* grad_left,
                             float* grad_right, hipStream_t s, std::string* err)
{
    const int K = lay.K;
    const void* img[MSIBM_MAX_LEVELS][2];
    int pitch[MSIBM_MAX_LEVELS];
    int st = build_pyramid(P, lay, ws, img, pitch, s, err);
    if (st != MSIBM_OK) return st;
    int dts[MSIBM_MAX_LEVELS];
    for (int k = 0; k < K; ++k) dts[k] = MSIBM_F32;
    st = build_stats(lay, cfg, ws, img, pitch, dts, s, err);
    if (st != MSIBM_OK) return st;
    // image gradients per level: the caller's at level 0, the workspace's above
    float* gl[MSIBM_MAX_LEVELS];
    float* gr[MSIBM_MAX_LEVELS];
    gl[0] = grad_left;
    gr[0] = grad_right;
    for (int k = 1; k <= K - 2; ++k) {
        gl[k] = (float*)(ws + lay.grad[k][0]);
        gr[k] = (float*)(ws + lay.grad[k][1]);
    }
    hipError_t e;
    for (int k = 0; k <= K - 2; ++k) {
        TimedLaunch t("bwd_zero", s);
        e = launch_zero(gl[k], gr[k], (size_t)lay.h[k] * lay.w[k], s);
        if (e != hipSuccess) return hip_err(e, "zero launch", err);
    }
    // every soft level's own gradient, all levels' tiles in one launch per
    // window size (the levels' backwards are independent: each adds into its
    // own level's gradients) ...
    for (int k0 = 0; k0 <= K - 2; ++k0) {
        if (!grad_soft[k0]) continue;
        bool first = true;
        for (int k = 0; k < k0; ++k) first = first && !(grad_soft[k] && level_n(cfg, k) == level_n(cfg, k0));
        if (!first) continue;
        BackLevels bl{};
        int blocks = 0;
        for (int k = k0; k <= K - 2; ++k) {
            if (!grad_soft[k] || level_n(cfg, k) != level_n(cfg, k0)) continue;
            BackArgs& b = bl.lev[bl.n];
            b.L = (const float*)img[k][0];
            b.R = (const float*)img[k][1];
            b.H = lay.h[k];
            b.W = lay.w[k];
            b.pitch = pitch[k];
            b.statL = (const WinStat*)(ws + lay.stat[k][0]);
            b.statR = (const WinStat*)(ws + lay.stat[k][1]);
            b.spitch = lay.w[k];
            b.D = level_range(P.max_disp, k);
            b.prior = maps[k + 1];
            b.Hc = lay.h[k + 1];
            b.Wc = lay.w[k + 1];
            b.ppitch = lay.w[k + 1];
            b.rs = cfg->soft_radius;
            b.inv_tau = 1.f / cfg->tau;
            b.g = grad_soft[k];
            b.gpitch = lay.w[k];
            b.gL = gl[k];
            b.gR = gr[k];
            bl.task0[bl.n] = blocks;
            bl.tiles_x[bl.n] = (lay.w[k] + TILE_W - 1) / TILE_W;
            blocks += bl.tiles_x[bl.n] * ((lay.h[k] + TILE_H1 - 1) / TILE_H1);
            ++bl.n;
        }
        TimedLaunch t("backward_levels", s);
        e = launch_backward_levels(level_n(cfg, k0), slots_for_radius(cfg->soft_radius), bl, blocks, s);
        if (e != hipSuccess) return hip_err(e, "backward launch", err);
    }
    // ... then, from the coarsest soft level down, each level's total carried
    // one level down through the reduce's adjoint
    for (int k = K - 2; k >= 1; --k) {
        AdjArgs ad{};
        ad.g[0] = gl[k];
        ad.g[1] = gr[k];
        ad.out[0] = gl[k - 1];
        ad.out[1] = gr[k - 1];
        ad.views = 2;
        ad.Hc = lay.h[k];
        ad.Wc = lay.w[k];
        ad.gpitch = lay.w[k];
        ad.H = lay.h[k - 1];
        ad.W = lay.w[k - 1];
        ad.opitch = lay.w[k - 1];
        char lab[32];
        snprintf(lab, sizeof(lab), "adjoint_l%d", k);
        TimedLaunch t(lab, s);
        e = launch_adjoint(ad, s);
        if (e != hipSuccess) return hip_err(e, "adjoint launch", err);
    }
    return MSIBM_OK;
}

hipError_t launch_backward(int n, int nc, const BackArgs& a, hipStream_t s)
{
    switch (n) {
        case 1: return launch_backward_n1(nc, a, s);
        case 2: return launch_backward_n2(nc, a, s);
        case 3: return launch_backward_n3(nc, a, s);
        case 4: return launch_backward_n4(nc, a, s);
        case 5: return launch_backward_n5(nc, a, s);
        case 6: return launch_backward_n6(nc, a, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_backward_levels(int n, int nc, const BackLevels& a, int blocks, hipStream_t s)
{
    switch (n) {
        case 1: return launch_backward_levels_n1(nc, a, blocks, s);
        case 2: return launch_backward_levels_n2(nc, a, blocks, s);
        case 3: return launch_backward_levels_n3(nc, a, blocks, s);
        case 4: return launch_backward_levels_n4(nc, a, blocks, s);
        case 5: return launch_backward_levels_n5(nc, a, blocks, s);
        case 6: return launch_backward_levels_n6(nc, a, blocks, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_backward_multi(int n, int nc, const MultiArgs& a, int blocks, hipStream_t s)
{
    switch (n) {
        case 1: return launch_backward_multi_n1(nc, a, blocks, s);
        case 2: return launch_backward_multi_n2(nc, a, blocks, s);
        case 3: return launch_backward_multi_n3(nc, a, blocks, s);
        case 4: return launch_backward_multi_n4(nc, a, blocks, s);
        case 5: return launch_backward_multi_n5(nc, a, blocks, s);
        case 6: return launch_backward_multi_n6(nc, a, blocks, s);
    }
    return hipErrorInvalidValue;
}

// Backward of one pair: level-0 window statistics, zeroed gradients, then the
// backward tiles (which add into the gradients).
int run_pair_backward(const msibm_pair& P, const PairLayout& lay, const msibm_config* cfg, char* ws,
                      const int16_t* prior1, const float* grad_soft, float* grad_left, float* grad_right,
                      hipStream_t s, std::string* err)
{
    hipError_t e;
    const int H = P.height, W = P.width;
    StatsArgs sa{};
    sa.seg[0] = StatsSeg{P.left, (WinStat*)(ws + lay.stat[0][0]), MSIBM_F32, H, W, P.pitch, W, 0};
    sa.seg[1] = StatsSeg{P.right, (WinStat*)(ws + lay.stat[0][1]), MSIBM_F32, H, W, P.pitch, W, 0};
    sa.nseg = 2;
    sa.n = level_n(cfg, 0);
    sa.var_eps = cfg->var_eps;
    {
        TimedLaunch t("bwd_stats", s);
        e = launch_stats(sa, s);
    }
    if (e != hipSuccess) return hip_err(e, "stats launch", err);
    {
        TimedLaunch t("bwd_zero", s);
        e = launch_zero(grad_left, grad_right, (size_t)H * W, s);
    }
    if (e != hipSuccess) return hip_err(e, "zero launch", err);
    BackArgs b{};
    b.L = (const float*)P.left;
    b.R = (const float*)P.right;
    b.H = H;
    b.W = W;
    b.pitch = P.pitch;
    b.statL = (const WinStat*)(ws + lay.stat[0][0]);
    b.statR = (const WinStat*)(ws + lay.stat[0][1]);
    b.spitch = W;
    b.D = P.max_disp;
    b.prior = prior1;
    b.Hc = lay.h[1];
    b.Wc = lay.w[1];
    b.ppitch = lay.w[1];
    b.rs = cfg->soft_radius;
    b.inv_tau = 1.f / cfg->tau;
    b.g = grad_soft;
    b.gpitch = W;
    b.gL = grad_left;
    b.gR = grad_right;
    {
        TimedLaunch t("backward_l0", s);
        e = launch_backward(level_n(cfg, 0), slots_for_radius(cfg->soft_radius), b, s);
    }
    if (e != hipSuccess) return hip_err(e, "backward launch", err);
    return MSIBM_OK;
}

// The fused training step of one pair: the forward down to level 1, then one
// launch for level 0 that computes the soft level, forms the masked-L1
// gradient sign(d_soft - gt) / |M| per pixel and runs the backward with it,
// reusing the level-0 statistics the forward stored.
int run_pair_fused_l1(const msibm_pair& P, const PairLayout& lay, const msibm_config* cfg, char* ws,
                      const FusedL1Pair& io, hipStream_t s, std::string* err)
{
    hipError_t e;
    const int H = P.height, W = P.width;
    int* count = (int*)(ws + lay.l1acc);
    float* lsum = (float*)(ws + lay.l1acc) + 1;
    {
        TimedLaunch t("fused_zero", s);
        e = launch_zero(io.grad_left, io.grad_right, (size_t)H * W, s);
        if (e == hipSuccess) e = launch_fill((float*)count, 0.f, 2, s);  // count and sum: all-zero bits
    }
    if (e != hipSuccess) return hip_err(e, "zero launch", err);
    {
        TimedLaunch t("fused_count", s);
        e = launch_mask_count(io.mask, (size_t)H * W, count, s);
    }
    if (e != hipSuccess) return hip_err(e, "mask count launch", err);
    const int st = run_pair_plain(P, lay, cfg, ws, io.disp, io.cost, io.soft, io.prior1, s, err, 1);
    if (st != MSIBM_OK) return st;
    BackArgs b{};
    b.L = (const float*)P.left;
    b.R = (const float*)P.right;
    b.H = H;
    b.W = W;
    b.pitch = P.pitch;
    b.statL = (const WinStat*)(ws + lay.stat[0][0]);
    b.statR = (const WinStat*)(ws + lay.stat[0][1]);
    b.spitch = W;
    b.D = P.max_disp;
    b.prior = io.prior1 ? io.prior1 : (const int16_t*)(ws + lay.map[1]);
    b.Hc = lay.h[1];
    b.Wc = lay.w[1];
    b.ppitch = lay.w[1];
    b.rs = cfg->soft_radius;
    b.inv_tau = 1.f / cfg->tau;
    b.gpitch = W;
    b.gL = io.grad_left;
    b.gR = io.grad_right;
    b.gt = io.gt;
    b.mask = io.mask;
    b.count = count;
    b.loss_sum = lsum;
    b.loss_out = io.loss;
    b.soft_out = io.soft;
    b.d_out = io.disp;
    b.c_out = io.cost;
    {
        TimedLaunch t("fused_backward_l0", s);
        e = launch_backward(level_n(cfg, 0), slots_for_radius(cfg->soft_radius), b, s);
    }
    if (e != hipSuccess) return hip_err(e, "fused backward launch", err);
    e = launch_l1_finalize(lsum, count, io.loss, s);
    if (e != hipSuccess) return hip_err(e, "loss launch", err);
    return MSIBM_OK;
}

}  // namespace msibm
