// C ABI of libmsibm: argument validation, workspace layout and launch sequencing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "msibm.h"
#include "plan.hpp"
#include "tune.hpp"

using namespace msibm;

namespace {

thread_local std::string g_err;

msibm_status fail(msibm_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

msibm_status ok()
{
    g_err.clear();
    return MSIBM_OK;
}

msibm_status hip_fail(hipError_t e, const char* what)
{
    return fail(MSIBM_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace

// ------------------------------------------------------------------ helpers

namespace msibm {

int level_dim(int v, int k)
{
    for (int i = 0; i < k; ++i) v = (v + 1) / 2;
    return v;
}

int level_range(int D, int k) { return (int)(((long long)D + (1LL << k) - 1) >> k); }

int auto_levels(int D)
{
    int k = 1;
    while (level_range(D, k - 1) > 32 && k < MSIBM_MAX_LEVELS) ++k;
    return k;
}

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

msibm_status validate_config(const msibm_config* cfg)
{
    if (!cfg) return fail(MSIBM_ERR_INVALID_ARG, "cfg is NULL");
    if (cfg->half_window < 1 || cfg->half_window > MSIBM_MAX_HALF_WINDOW)
        return fail(MSIBM_ERR_UNSUPPORTED, "half_window %d outside 1..%d", cfg->half_window,
                    MSIBM_MAX_HALF_WINDOW);
    for (int k = 0; k < MSIBM_MAX_LEVELS; ++k) {
        const int v = cfg->half_window_levels[k];
        if (v < 0 || v > MSIBM_MAX_HALF_WINDOW)
            return fail(MSIBM_ERR_UNSUPPORTED, "half_window_levels[%d] = %d outside 0..%d", k, v,
                        MSIBM_MAX_HALF_WINDOW);
    }
    if (cfg->refine_radius < 0 || cfg->refine_radius > MSIBM_MAX_RADIUS)
        return fail(MSIBM_ERR_UNSUPPORTED, "refine_radius %d outside 0..%d", cfg->refine_radius,
                    MSIBM_MAX_RADIUS);
    if (!(cfg->var_eps >= 0.f) || !std::isfinite(cfg->var_eps))
        return fail(MSIBM_ERR_INVALID_ARG, "var_eps must be finite and >= 0");
    if (cfg->soft_radius < 0 || cfg->soft_radius > MSIBM_MAX_RADIUS)
        return fail(MSIBM_ERR_UNSUPPORTED, "soft_radius %d outside 0..%d", cfg->soft_radius,
                    MSIBM_MAX_RADIUS);
    if (cfg->soft_radius > 0 && (!(cfg->tau > 0.f) || !std::isfinite(cfg->tau)))
        return fail(MSIBM_ERR_INVALID_ARG, "tau must be finite and > 0");
    if (cfg->flags & MSIBM_FLAG_PERSISTENT)
        return fail(MSIBM_ERR_UNSUPPORTED, "the persistent single-launch scheduler is switched off");
    if (cfg->flags &
        ~(MSIBM_FLAG_BATCHED | MSIBM_FLAG_GRAPH | MSIBM_FLAG_PREBLUR | MSIBM_FLAG_MEDIAN | MSIBM_FLAG_GATED))
        return fail(MSIBM_ERR_INVALID_ARG, "unknown flags 0x%x", cfg->flags);
    if ((cfg->flags & MSIBM_FLAG_MEDIAN) && !std::isfinite(cfg->median_alpha))
        return fail(MSIBM_ERR_INVALID_ARG, "median_alpha must be finite");
    if ((cfg->flags & MSIBM_FLAG_GATED) && (!std::isfinite(cfg->gate_alpha) || !std::isfinite(cfg->gate_beta)))
        return fail(MSIBM_ERR_INVALID_ARG, "gate_alpha and gate_beta must be finite");
    if ((cfg->flags & MSIBM_FLAG_GRAPH) && !(cfg->flags & MSIBM_FLAG_BATCHED))
        return fail(MSIBM_ERR_INVALID_ARG, "MSIBM_FLAG_GRAPH needs MSIBM_FLAG_BATCHED");
    return MSIBM_OK;
}

msibm_status validate_pair(const msibm_pair& p, int idx, const msibm_config* cfg, int* K_out)
{
    if (!p.left || !p.right) return fail(MSIBM_ERR_INVALID_ARG, "pair %d: NULL image", idx);
    if (p.dtype != MSIBM_U8 && p.dtype != MSIBM_F32)
        return fail(MSIBM_ERR_INVALID_ARG, "pair %d: dtype %d", idx, p.dtype);
    if (p.height < 1 || p.width < 1) return fail(MSIBM_ERR_SHAPE, "pair %d: size %dx%d", idx, p.height, p.width);
    if (p.pitch < p.width) return fail(MSIBM_ERR_SHAPE, "pair %d: pitch %d < width %d", idx, p.pitch, p.width);
    if (p.max_disp < 1 || p.max_disp > MSIBM_MAX_DISP)
        return fail(MSIBM_ERR_UNSUPPORTED, "pair %d: max_disp %d outside 1..%d", idx, p.max_disp, MSIBM_MAX_DISP);
    if (p.num_levels < 0 || p.num_levels > MSIBM_MAX_LEVELS)
        return fail(MSIBM_ERR_UNSUPPORTED, "pair %d: num_levels %d outside 0..%d", idx, p.num_levels,
                    MSIBM_MAX_LEVELS);
    const int K = p.num_levels ? p.num_levels : auto_levels(p.max_disp);
    if (cfg->soft_radius > 0) {
        if (p.dtype != MSIBM_F32)
            return fail(MSIBM_ERR_UNSUPPORTED, "pair %d: the soft-argmax level takes float images", idx);
        if (K < 2) return fail(MSIBM_ERR_UNSUPPORTED, "pair %d: the soft-argmax level needs K >= 2", idx);
    }
    *K_out = K;
    return MSIBM_OK;
}

// Workspace layout of one pair (offsets from the pair's base).
PairLayout pair_layout(const msibm_pair& p, int K, bool preblur, bool median, bool gated, bool level_grads)
{
    PairLayout L{};
    L.K = K;
    size_t off = 0;
    for (int k = 0; k < K; ++k) {
        L.h[k] = level_dim(p.height, k);
        L.w[k] = level_dim(p.width, k);
        const size_t px = (size_t)L.h[k] * L.w[k];
        for (int v = 0; v < 2; ++v) {
            if (k > 0) {
                L.img[k][v] = off;
                off = align_up(off + px * sizeof(float));
            }
            L.stat[k][v] = off;
            off = align_up(off + px * sizeof(WinStat));
        }
        if (k > 0) {
            L.map[k] = off;
            off = align_up(off + px * sizeof(int16_t));
        }
        if (k > 0 && gated) {
            L.cmap[k] = off;
            off = align_up(off + px * sizeof(float));
        }
    }
    if (preblur)
        for (int v = 0; v < 2; ++v) {
            L.blur[v] = off;
            off = align_up(off + (size_t)p.height * p.width * sizeof(float));
        }
    if (median) {
        L.dtmp = off;
        off = align_up(off + (size_t)p.height * p.width * sizeof(int16_t));
    }
    if (median || gated) {
        L.ctmp = off;
        off = align_up(off + (size_t)p.height * p.width * sizeof(float));
    }
    L.l1acc = off;
    off = align_up(off + 2 * sizeof(float));
    if (level_grads)
        for (int k = 1; k <= K - 2; ++k)
            for (int v = 0; v < 2; ++v) {
                L.grad[k][v] = off;
                off = align_up(off + (size_t)L.h[k] * L.w[k] * sizeof(float));
            }
    L.bytes = off;
    return L;
}

}  // namespace msibm

// ------------------------------------------- scratch of the allocation-free entry point
// One copy of this array exists on every device the library runs on, for the
// life of the process.  Host code never passes the array's name to a kernel
// or a copy (on the host it only stands for the symbol): it looks up the
// device address once per device and uses that.
static __device__ __align__(256) unsigned char scratch[MSIBM_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices];  // device address of `scratch`, per device

// Address of the current device's scratch array, looked up on the first call
// on that device (with that device current).
msibm_status scratch_address(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxScratchDevices)
        return fail(MSIBM_ERR_UNSUPPORTED, "device %d: the allocation-free entry point serves devices 0..%d", dev,
                    kMaxScratchDevices - 1);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(MSIBM_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return MSIBM_OK;
}

}  // namespace

// ------------------------------------------------------------------ C ABI

extern "C" {

const char* msibm_last_error(void) { return g_err.c_str(); }

const char* msibm_version(void) { return "msibm 0.1 gfx950"; }

msibm_status msibm_force_variant(int32_t variant)
{
    if (variant < -1 || variant > VARIANT_MASK)
        return fail(MSIBM_ERR_INVALID_ARG, "variant %d outside -1..%d", variant, VARIANT_MASK);
    force_variant(variant);
    return ok();
}

msibm_status msibm_autotune(int32_t enable, const char* cache_path)
{
    std::string err;
    if (!set_autotune(enable != 0, cache_path ? cache_path : "", &err)) return fail(MSIBM_ERR_INVALID_ARG, "%s", err.c_str());
    return ok();
}

int64_t msibm_autotune_table(char* buf, size_t len)
{
    const std::string t = autotune_table();
    if (buf && len > 0) {
        const size_t n = t.size() < len - 1 ? t.size() : len - 1;
        memcpy(buf, t.data(), n);
        buf[n] = '\0';
    }
    return (int64_t)t.size();
}

msibm_status msibm_pyramid(const void* img, int32_t dtype, int32_t H, int32_t W, int32_t pitch,
                           int32_t K, float* const* levels, const int32_t* level_pitch, void* stream)
{
    if (!img || !levels || !level_pitch) return fail(MSIBM_ERR_INVALID_ARG, "NULL pointer argument");
    if (dtype != MSIBM_U8 && dtype != MSIBM_F32) return fail(MSIBM_ERR_INVALID_ARG, "dtype %d", dtype);
    if (H < 1 || W < 1 || pitch < W) return fail(MSIBM_ERR_SHAPE, "size %dx%d pitch %d", H, W, pitch);
    if (K < 1 || K > MSIBM_MAX_LEVELS) return fail(MSIBM_ERR_UNSUPPORTED, "K %d outside 1..%d", K, MSIBM_MAX_LEVELS);
    for (int k = 0; k < K; ++k) {
        if (!levels[k]) return fail(MSIBM_ERR_INVALID_ARG, "levels[%d] is NULL", k);
        if (level_pitch[k] < level_dim(W, k))
            return fail(MSIBM_ERR_SHAPE, "level_pitch[%d] = %d < %d", k, level_pitch[k], level_dim(W, k));
    }
    hipStream_t s = (hipStream_t)stream;
    ConvertArgs c{img, levels[0], H, W, pitch, level_pitch[0]};
    hipError_t e = launch_convert(dtype, c, s);
    if (e != hipSuccess) return hip_fail(e, "pyramid convert launch");
    for (int k = 1; k < K; ++k) {
        ReduceArgs r{};
        r.src[0] = levels[k - 1];
        r.dst[0] = levels[k];
        r.views = 1;
        r.H = level_dim(H, k - 1);
        r.W = level_dim(W, k - 1);
        r.spitch = level_pitch[k - 1];
        r.Ho = level_dim(H, k);
        r.Wo = level_dim(W, k);
        r.dpitch = level_pitch[k];
        e = launch_reduce(MSIBM_F32, r, s);
        if (e != hipSuccess) return hip_fail(e, "pyramid reduce launch");
    }
    return ok();
}

msibm_status msibm_median_filter(const int16_t* d_in, int32_t in_pitch, const float* cost, int32_t cost_pitch,
                                 int32_t H, int32_t W, double alpha, int16_t* d_out, int32_t out_pitch,
                                 void* stream)
{
    if (!d_in || !cost || !d_out) return fail(MSIBM_ERR_INVALID_ARG, "NULL map or cost");
    if (H < 1 || W < 1 || in_pitch < W || cost_pitch < W || out_pitch < W)
        return fail(MSIBM_ERR_SHAPE, "size %dx%d pitches %d %d %d", H, W, in_pitch, cost_pitch, out_pitch);
    if (!std::isfinite(alpha)) return fail(MSIBM_ERR_INVALID_ARG, "alpha must be finite");
    const char* a0 = (const char*)d_in;
    const char* a1 = a0 + ((size_t)(H - 1) * in_pitch + W) * sizeof(int16_t);
    const char* b0 = (const char*)d_out;
    const char* b1 = b0 + ((size_t)(H - 1) * out_pitch + W) * sizeof(int16_t);
    if (a0 < b1 && b0 < a1) return fail(MSIBM_ERR_INVALID_ARG, "d_out overlaps d_in");
    MedianArgs m{d_in, cost, d_out, H, W, in_pitch, cost_pitch, out_pitch, alpha};
    const hipError_t e = launch_median(m, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "median launch");
    return ok();
}

size_t msibm_level_workspace_size(int32_t H, int32_t W)
{
    if (H < 1 || W < 1) return 0;
    return 2 * align_up((size_t)H * W * sizeof(WinStat));
}

msibm_status msibm_match_level(const void* L, const void* R, int32_t dtype, int32_t H, int32_t W,
                               int32_t pitch, int32_t n, int32_t Dk, const int16_t* prior, int32_t Hc,
                               int32_t Wc, int32_t prior_pitch, int32_t r, float var_eps, int16_t* d_out,
                               float* cost_out, int32_t out_pitch, float* costvol, void* workspace,
                               size_t ws_bytes, void* stream)
{
    if (!L || !R || !d_out) return fail(MSIBM_ERR_INVALID_ARG, "NULL image or output");
    if (dtype != MSIBM_U8 && dtype != MSIBM_F32) return fail(MSIBM_ERR_INVALID_ARG, "dtype %d", dtype);
    if (H < 1 || W < 1 || pitch < W || out_pitch < W)
        return fail(MSIBM_ERR_SHAPE, "size %dx%d pitch %d out_pitch %d", H, W, pitch, out_pitch);
    if (n < 1 || n > MSIBM_MAX_HALF_WINDOW) return fail(MSIBM_ERR_UNSUPPORTED, "n %d outside 1..%d", n, MSIBM_MAX_HALF_WINDOW);
    if (Dk < 1 || Dk > MSIBM_MAX_DISP) return fail(MSIBM_ERR_UNSUPPORTED, "D_k %d outside 1..%d", Dk, MSIBM_MAX_DISP);
    if (!(var_eps >= 0.f) || !std::isfinite(var_eps)) return fail(MSIBM_ERR_INVALID_ARG, "var_eps");
    if (prior) {
        if (r < 0 || r > MSIBM_MAX_RADIUS) return fail(MSIBM_ERR_UNSUPPORTED, "r %d outside 0..%d", r, MSIBM_MAX_RADIUS);
        if (Hc != (H + 1) / 2 || Wc != (W + 1) / 2 || prior_pitch < Wc)
            return fail(MSIBM_ERR_SHAPE, "prior %dx%d (pitch %d) does not match level %dx%d", Hc, Wc,
                        prior_pitch, H, W);
    }
    const size_t need = msibm_level_workspace_size(H, W);
    if (!workspace || ws_bytes < need)
        return fail(MSIBM_ERR_WORKSPACE, "workspace %zu bytes < %zu needed", workspace ? ws_bytes : (size_t)0, need);
    hipStream_t s = (hipStream_t)stream;
    WinStat* st = (WinStat*)workspace;
    WinStat* st_r = (WinStat*)((char*)workspace + align_up((size_t)H * W * sizeof(WinStat)));
    StatsArgs sa{};
    sa.seg[0] = StatsSeg{L, st, dtype, H, W, pitch, W, 0};
    sa.seg[1] = StatsSeg{R, st_r, dtype, H, W, pitch, W, 0};
    sa.nseg = 2;
    sa.n = n;
    sa.var_eps = var_eps;
    hipError_t e = launch_stats(sa, s);
    if (e != hipSuccess) return hip_fail(e, "stats launch");
    MatchArgs a{};
    a.L = L;
    a.R = R;
    a.H = H;
    a.W = W;
    a.pitch = pitch;
    a.statL = st;
    a.statR = st_r;
    a.spitch = W;
    a.Dk = Dk;
    a.prior = prior;
    a.Hc = Hc;
    a.Wc = Wc;
    a.ppitch = prior_pitch;
    a.r = r;
    a.d_out = d_out;
    a.c_out = cost_out;
    a.soft_out = nullptr;
    a.opitch = out_pitch;
    a.inv_tau = 0.f;
    const int mode = prior ? MODE_REFINE : MODE_FULL;
    const int nc = prior ? slots_for_radius(r) : FULL_NC;
    a.variant = select_variant(a, n, dtype, mode, nc, s);
    if (costvol) {
        e = launch_fill(costvol, -2.f, (size_t)H * W * Dk, s);
        if (e != hipSuccess) return hip_fail(e, "cost volume fill launch");
        a.costvol = costvol;
    }
    e = launch_match(n, dtype, mode, nc, a, s);
    if (e != hipSuccess) return hip_fail(e, "match launch");
    return ok();
}

msibm_status msibm_upsample_cost(const float* coarse, int32_t Hc, int32_t Wc, int32_t coarse_pitch, int32_t H,
                                 int32_t W, double* out, int32_t out_pitch, void* stream)
{
    if (!coarse || !out) return fail(MSIBM_ERR_INVALID_ARG, "NULL map");
    if (H < 1 || W < 1 || Hc != (H + 1) / 2 || Wc != (W + 1) / 2 || coarse_pitch < Wc || out_pitch < W)
        return fail(MSIBM_ERR_SHAPE, "coarse %dx%d (pitch %d) for %dx%d (pitch %d)", Hc, Wc, coarse_pitch, H, W,
                    out_pitch);
    const hipError_t e = launch_upsample_cost(coarse, Hc, Wc, coarse_pitch, H, W, out, out_pitch,
                                              (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "upsample launch");
    return ok();
}

static GateArgs gate_args(const void* L, const void* R, int H, int W, int pitch, int Dk, void* workspace,
                          int16_t* d, float* c, int opitch, double thresh)
{
    GateArgs g{};
    g.L = L;
    g.R = R;
    g.pitch = pitch;
    g.H = H;
    g.W = W;
    g.Dk = Dk;
    g.statL = (const WinStat*)workspace;
    g.statR = (const WinStat*)((char*)workspace + align_up((size_t)H * W * sizeof(WinStat)));
    g.spitch = W;
    g.d = d;
    g.c = c;
    g.opitch = opitch;
    g.thresh = thresh;
    return g;
}

msibm_status msibm_match_level_gated(const void* L, const void* R, int32_t dtype, int32_t H, int32_t W,
                                     int32_t pitch, int32_t n, int32_t Dk, const int16_t* prior,
                                     const float* prior_cost, int32_t Hc, int32_t Wc, int32_t prior_pitch,
                                     int32_t r, double beta, float var_eps, int16_t* d_out, float* cost_out,
                                     int32_t out_pitch, void* workspace, size_t ws_bytes, void* stream)
{
    if (!prior || !prior_cost || !cost_out) return fail(MSIBM_ERR_INVALID_ARG, "NULL prior, prior cost or cost");
    if (!std::isfinite(beta)) return fail(MSIBM_ERR_INVALID_ARG, "beta must be finite");
    // statistics and the restricted search of every pixel
    const msibm_status st = msibm_match_level(L, R, dtype, H, W, pitch, n, Dk, prior, Hc, Wc, prior_pitch, r,
                                              var_eps, d_out, cost_out, out_pitch, nullptr, workspace, ws_bytes,
                                              stream);
    if (st != MSIBM_OK) return st;
    GateArgs g = gate_args(L, R, H, W, pitch, Dk, workspace, d_out, cost_out, out_pitch, beta);
    g.ccost = prior_cost;
    g.Hc = Hc;
    g.Wc = Wc;
    g.cpitch = prior_pitch;
    const hipError_t e = launch_gate(n, dtype, GATE_MODE_FULL, g, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "gated full search launch");
    return ok();
}

msibm_status msibm_aggregate_refine(const void* L, const void* R, int32_t dtype, int32_t H, int32_t W,
                                    int32_t pitch, int32_t n, int32_t Dk, int16_t* d, float* cost,
                                    int32_t dc_pitch, double alpha, float var_eps, void* workspace,
                                    size_t ws_bytes, void* stream)
{
    if (!L || !R || !d || !cost) return fail(MSIBM_ERR_INVALID_ARG, "NULL image, map or cost");
    if (dtype != MSIBM_U8 && dtype != MSIBM_F32) return fail(MSIBM_ERR_INVALID_ARG, "dtype %d", dtype);
    if (!std::isfinite(alpha)) return fail(MSIBM_ERR_INVALID_ARG, "alpha must be finite");
    if (!(var_eps >= 0.f) || !std::isfinite(var_eps)) return fail(MSIBM_ERR_INVALID_ARG, "var_eps");
    if (H < 1 || W < 1 || pitch < W || dc_pitch < W)
        return fail(MSIBM_ERR_SHAPE, "size %dx%d pitch %d map pitch %d", H, W, pitch, dc_pitch);
    if (n < 1 || n > MSIBM_MAX_HALF_WINDOW) return fail(MSIBM_ERR_UNSUPPORTED, "n %d outside 1..%d", n, MSIBM_MAX_HALF_WINDOW);
    if (Dk < 1 || Dk > MSIBM_MAX_DISP) return fail(MSIBM_ERR_UNSUPPORTED, "D_k %d outside 1..%d", Dk, MSIBM_MAX_DISP);
    const size_t need = msibm_level_workspace_size(H, W);
    if (!workspace || ws_bytes < need)
        return fail(MSIBM_ERR_WORKSPACE, "workspace %zu bytes < %zu needed", workspace ? ws_bytes : (size_t)0, need);
    hipStream_t s = (hipStream_t)stream;
    GateArgs g = gate_args(L, R, H, W, pitch, Dk, workspace, d, cost, dc_pitch, alpha);
    StatsArgs sa{};
    sa.seg[0] = StatsSeg{L, (WinStat*)g.statL, dtype, H, W, pitch, W, 0};
    sa.seg[1] = StatsSeg{R, (WinStat*)g.statR, dtype, H, W, pitch, W, 0};
    sa.nseg = 2;
    sa.n = n;
    sa.var_eps = var_eps;
    hipError_t e = launch_stats(sa, s);
    if (e != hipSuccess) return hip_fail(e, "stats launch");
    e = launch_gate(n, dtype, GATE_MODE_REPICK, g, s);
    if (e != hipSuccess) return hip_fail(e, "re-pick launch");
    return ok();
}

size_t msibm_workspace_size(const msibm_pair* pairs, int32_t n_pairs, const msibm_config* cfg)
{
    if (!pairs || n_pairs < 1 || n_pairs > MSIBM_MAX_PAIRS || !cfg) return 0;
    if (validate_config(cfg) != MSIBM_OK) return 0;
    size_t tot = 0;
    for (int p = 0; p < n_pairs; ++p) {
        int K;
        if (validate_pair(pairs[p], p, cfg, &K) != MSIBM_OK) return 0;
        tot += pair_layout(pairs[p], K, (cfg->flags & MSIBM_FLAG_PREBLUR) != 0,
                           (cfg->flags & MSIBM_FLAG_MEDIAN) != 0, (cfg->flags & MSIBM_FLAG_GATED) != 0).bytes;
    }
    tot += batch_extra_bytes(pairs, n_pairs, cfg);
    return tot;
}

msibm_status msibm_disparity(const msibm_pair* pairs, int32_t n_pairs, const msibm_config* cfg,
                             int16_t* const* disp, float* const* cost, float* const* soft_disp,
                             int16_t* const* prior1, void* workspace, size_t ws_bytes, void* stream)
{
    if (!pairs || !disp) return fail(MSIBM_ERR_INVALID_ARG, "pairs or disp is NULL");
    if (n_pairs < 1 || n_pairs > MSIBM_MAX_PAIRS)
        return fail(MSIBM_ERR_INVALID_ARG, "n_pairs %d outside 1..%d", n_pairs, MSIBM_MAX_PAIRS);
    msibm_status st = validate_config(cfg);
    if (st != MSIBM_OK) return st;
    std::vector<int> Ks(n_pairs);
    for (int p = 0; p < n_pairs; ++p) {
        st = validate_pair(pairs[p], p, cfg, &Ks[p]);
        if (st != MSIBM_OK) return st;
        if (!disp[p]) return fail(MSIBM_ERR_INVALID_ARG, "disp[%d] is NULL", p);
        if (cfg->soft_radius > 0 && (!soft_disp || !soft_disp[p]))
            return fail(MSIBM_ERR_INVALID_ARG, "soft_disp[%d] is NULL but soft_radius > 0", p);
    }
    const size_t need = msibm_workspace_size(pairs, n_pairs, cfg);
    if (!workspace || ws_bytes < need)
        return fail(MSIBM_ERR_WORKSPACE, "workspace %zu bytes < %zu needed", workspace ? ws_bytes : (size_t)0, need);

    hipStream_t s = (hipStream_t)stream;
    if (cfg->flags & MSIBM_FLAG_BATCHED) {
        BatchOutputs out{disp, cost, soft_disp, prior1};
        std::string err;
        const int rc = run_batched(pairs, n_pairs, cfg, out, workspace, ws_bytes, s, &err);
        if (rc != MSIBM_OK) return fail(rc, "%s", err.c_str());
        return ok();
    }
    size_t base = 0;
    for (int p = 0; p < n_pairs; ++p) {
        const msibm_pair& P = pairs[p];
        const PairLayout lay = pair_layout(P, Ks[p], (cfg->flags & MSIBM_FLAG_PREBLUR) != 0,
                                           (cfg->flags & MSIBM_FLAG_MEDIAN) != 0,
                                           (cfg->flags & MSIBM_FLAG_GATED) != 0);
        char* ws = (char*)workspace + base;
        base += lay.bytes;
        std::string err;
        const int rc = run_pair_plain(P, lay, cfg, ws, disp[p], cost ? cost[p] : nullptr,
                                      soft_disp ? soft_disp[p] : nullptr, prior1 ? prior1[p] : nullptr, s,
                                      &err);
        if (rc != MSIBM_OK) return fail(rc, "pair %d: %s", p, err.c_str());
    }
    return ok();
}

msibm_status msibm_disparity_noalloc(const msibm_pair* pair, const msibm_config* cfg, int16_t* disp, float* cost,
                                     float* soft_disp, int16_t* prior1, void* stream)
{
    if (!pair || !disp) return fail(MSIBM_ERR_INVALID_ARG, "pair or disp is NULL");
    msibm_status st = validate_config(cfg);
    if (st != MSIBM_OK) return st;
    if (cfg->flags & (MSIBM_FLAG_BATCHED | MSIBM_FLAG_GRAPH))
        return fail(MSIBM_ERR_UNSUPPORTED, "the allocation-free entry point runs the plain path (no BATCHED, GRAPH)");
    int K;
    st = validate_pair(*pair, 0, cfg, &K);
    if (st != MSIBM_OK) return st;
    if (cfg->soft_radius > 0 && !soft_disp)
        return fail(MSIBM_ERR_INVALID_ARG, "soft_disp is NULL but soft_radius > 0");
    const PairLayout lay = pair_layout(*pair, K, (cfg->flags & MSIBM_FLAG_PREBLUR) != 0,
                                       (cfg->flags & MSIBM_FLAG_MEDIAN) != 0, (cfg->flags & MSIBM_FLAG_GATED) != 0);
    if (lay.bytes > (size_t)MSIBM_NOALLOC_SCRATCH_BYTES)
        return fail(MSIBM_ERR_WORKSPACE,
                    "the pair needs %zu bytes of scratch, more than the %zu bytes the allocation-free entry "
                    "point holds (use msibm_disparity with a workspace)",
                    lay.bytes, (size_t)MSIBM_NOALLOC_SCRATCH_BYTES);
    void* ws = nullptr;
    st = scratch_address(&ws);
    if (st != MSIBM_OK) return st;
    // nothing in the plain forward reads scratch it has not written in the
    // same call, so nothing needs clearing first
    NoAllocScope no_alloc;
    std::string err;
    const int rc = run_pair_plain(*pair, lay, cfg, (char*)ws, disp, cost, soft_disp, prior1, (hipStream_t)stream,
                                  &err);
    if (rc != MSIBM_OK) return fail(rc, "%s", err.c_str());
    return ok();
}

msibm_status msibm_backward(const msibm_pair* pairs, int32_t n_pairs, const msibm_config* cfg,
                            const int16_t* const* prior1, const float* const* grad_soft,
                            float* const* grad_left, float* const* grad_right, void* workspace,
                            size_t ws_bytes, void* stream)
{
    if (!pairs || !prior1 || !grad_soft || !grad_left || !grad_right)
        return fail(MSIBM_ERR_INVALID_ARG, "NULL argument");
    if (n_pairs < 1 || n_pairs > MSIBM_MAX_PAIRS)
        return fail(MSIBM_ERR_INVALID_ARG, "n_pairs %d outside 1..%d", n_pairs, MSIBM_MAX_PAIRS);
    msibm_status st = validate_config(cfg);
    if (st != MSIBM_OK) return st;
    if (cfg->soft_radius < 1) return fail(MSIBM_ERR_INVALID_ARG, "backward needs soft_radius >= 1");
    if (cfg->flags & (MSIBM_FLAG_PREBLUR | MSIBM_FLAG_MEDIAN | MSIBM_FLAG_GATED))
        return fail(MSIBM_ERR_UNSUPPORTED, "PREBLUR, MEDIAN and GATED are forward-only variants");
    std::vector<int> Ks(n_pairs);
    for (int p = 0; p < n_pairs; ++p) {
        st = validate_pair(pairs[p], p, cfg, &Ks[p]);
        if (st != MSIBM_OK) return st;
        if (!prior1[p] || !grad_soft[p] || !grad_left[p] || !grad_right[p])
            return fail(MSIBM_ERR_INVALID_ARG, "pair %d: NULL prior or gradient buffer", p);
    }
    const size_t need = msibm_workspace_size(pairs, n_pairs, cfg);
    if (!workspace || ws_bytes < need)
        return fail(MSIBM_ERR_WORKSPACE, "workspace %zu bytes < %zu needed", workspace ? ws_bytes : (size_t)0, need);
    hipStream_t s = (hipStream_t)stream;
    if (cfg->flags & MSIBM_FLAG_BATCHED) {
        BatchGrads g{prior1, grad_soft, grad_left, grad_right};
        std::string err;
        const int rc = run_batched_backward(pairs, n_pairs, cfg, g, workspace, ws_bytes, s, &err);
        if (rc != MSIBM_OK) return fail(rc, "%s", err.c_str());
        return ok();
    }
    size_t base = 0;
    for (int p = 0; p < n_pairs; ++p) {
        const PairLayout lay = pair_layout(pairs[p], Ks[p]);
        char* ws = (char*)workspace + base;
        base += lay.bytes;
        std::string err;
        const int rc = run_pair_backward(pairs[p], lay, cfg, ws, prior1[p], grad_soft[p], grad_left[p],
                                         grad_right[p], s, &err);
        if (rc != MSIBM_OK) return fail(rc, "pair %d: %s", p, err.c_str());
    }
    return ok();
}

msibm_status msibm_fwd_bwd_l1(const msibm_pair* pairs, int32_t n_pairs, const msibm_config* cfg,
                              const float* const* d_gt, const uint8_t* const* mask, int16_t* const* disp,
                              float* const* cost, float* const* soft_disp, int16_t* const* prior1,
                              float* const* grad_left, float* const* grad_right, float* const* loss,
                              void* workspace, size_t ws_bytes, void* stream)
{
    if (!pairs || !d_gt || !mask || !disp || !soft_disp || !grad_left || !grad_right || !loss)
        return fail(MSIBM_ERR_INVALID_ARG, "NULL argument");
    if (n_pairs < 1 || n_pairs > MSIBM_MAX_PAIRS)
        return fail(MSIBM_ERR_INVALID_ARG, "n_pairs %d outside 1..%d", n_pairs, MSIBM_MAX_PAIRS);
    msibm_status st = validate_config(cfg);
    if (st != MSIBM_OK) return st;
    if (cfg->soft_radius < 1) return fail(MSIBM_ERR_INVALID_ARG, "the fused step needs soft_radius >= 1");
    if (cfg->flags & (MSIBM_FLAG_PREBLUR | MSIBM_FLAG_MEDIAN | MSIBM_FLAG_GATED))
        return fail(MSIBM_ERR_UNSUPPORTED, "PREBLUR, MEDIAN and GATED are forward-only variants");
    std::vector<FusedL1Pair> io(n_pairs);
    for (int p = 0; p < n_pairs; ++p) {
        int K;
        st = validate_pair(pairs[p], p, cfg, &K);  // float images and K >= 2 (soft level)
        if (st != MSIBM_OK) return st;
        if (!d_gt[p] || !mask[p] || !disp[p] || !soft_disp[p] || !grad_left[p] || !grad_right[p] || !loss[p])
            return fail(MSIBM_ERR_INVALID_ARG, "pair %d: NULL input or output buffer", p);
        io[p] = FusedL1Pair{d_gt[p], mask[p], disp[p], cost ? cost[p] : nullptr, soft_disp[p],
                            prior1 ? prior1[p] : nullptr, grad_left[p], grad_right[p], loss[p]};
    }
    const size_t need = msibm_workspace_size(pairs, n_pairs, cfg);
    if (!workspace || ws_bytes < need)
        return fail(MSIBM_ERR_WORKSPACE, "workspace %zu bytes < %zu needed", workspace ? ws_bytes : (size_t)0, need);
    hipStream_t s = (hipStream_t)stream;
    std::string err;
    if (cfg->flags & MSIBM_FLAG_BATCHED) {
        const int rc = run_batched_fused_l1(pairs, n_pairs, cfg, io.data(), workspace, ws_bytes, s, &err);
        if (rc != MSIBM_OK) return fail(rc, "%s", err.c_str());
        return ok();
    }
    size_t base = 0;
    for (int p = 0; p < n_pairs; ++p) {
        int K;
        validate_pair(pairs[p], p, cfg, &K);
        const PairLayout lay = pair_layout(pairs[p], K);
        const int rc = run_pair_fused_l1(pairs[p], lay, cfg, (char*)workspace + base, io[p], s, &err);
        base += lay.bytes;
        if (rc != MSIBM_OK) return fail(rc, "pair %d: %s", p, err.c_str());
    }
    return ok();
}

msibm_status msibm_pyramid_adjoint(const float* g_coarse, int32_t Hc, int32_t Wc, int32_t coarse_pitch,
                                   float* g_fine, int32_t H, int32_t W, int32_t fine_pitch, void* stream)
{
    if (!g_coarse || !g_fine) return fail(MSIBM_ERR_INVALID_ARG, "NULL gradient");
    if (H < 1 || W < 1 || Hc != (H + 1) / 2 || Wc != (W + 1) / 2 || coarse_pitch < Wc || fine_pitch < W)
        return fail(MSIBM_ERR_SHAPE, "coarse %dx%d (pitch %d) for fine %dx%d (pitch %d)", Hc, Wc, coarse_pitch, H,
                    W, fine_pitch);
    AdjArgs a{};
    a.g[0] = g_coarse;
    a.out[0] = g_fine;
    a.views = 1;
    a.Hc = Hc;
    a.Wc = Wc;
    a.gpitch = coarse_pitch;
    a.H = H;
    a.W = W;
    a.opitch = fine_pitch;
    const hipError_t e = launch_adjoint(a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "adjoint launch");
    return ok();
}

// Shared checks of the every-level soft path: one float pair, K >= 2, a soft
// radius, no variant flags.
static msibm_status validate_levels(const msibm_pair* pair, const msibm_config* cfg, int* K)
{
    if (!pair || !cfg) return fail(MSIBM_ERR_INVALID_ARG, "NULL pair or config");
    msibm_status st = validate_config(cfg);
    if (st != MSIBM_OK) return st;
    if (cfg->flags) return fail(MSIBM_ERR_UNSUPPORTED, "the every-level soft path takes no flags");
    if (cfg->soft_radius < 1) return fail(MSIBM_ERR_INVALID_ARG, "soft_radius must be >= 1");
    st = validate_pair(*pair, 0, cfg, K);
    if (st != MSIBM_OK) return st;
    if (*K < 2) return fail(MSIBM_ERR_UNSUPPORTED, "the every-level soft path needs K >= 2");
    return MSIBM_OK;
}

size_t msibm_levels_workspace_size(const msibm_pair* pair, const msibm_config* cfg)
{
    int K;
    if (validate_levels(pair, cfg, &K) != MSIBM_OK) return 0;
    return pair_layout(*pair, K, false, false, false, true).bytes;
}

msibm_status msibm_disparity_levels(const msibm_pair* pair, const msibm_config* cfg, float* const* soft,
                                    int16_t* const* maps, void* workspace, size_t ws_bytes, void* stream)
{
    int K;
    msibm_status st = validate_levels(pair, cfg, &K);
    if (st != MSIBM_OK) return st;
    if (!soft || !maps) return fail(MSIBM_ERR_INVALID_ARG, "NULL output arrays");
    for (int k = 0; k < K; ++k) {
        if (!maps[k]) return fail(MSIBM_ERR_INVALID_ARG, "maps[%d] is NULL", k);
        if (k < K - 1 && !soft[k]) return fail(MSIBM_ERR_INVALID_ARG, "soft[%d] is NULL", k);
    }
    const PairLayout lay = pair_layout(*pair, K, false, false, false, true);
    if (!workspace || ws_bytes < lay.bytes)
        return fail(MSIBM_ERR_WORKSPACE, "workspace %zu bytes < %zu needed", workspace ? ws_bytes : (size_t)0,
                    lay.bytes);
    std::string err;
    const int rc = run_pair_levels(*pair, lay, cfg, (char*)workspace, soft, maps, (hipStream_t)stream, &err);
    if (rc != MSIBM_OK) return fail(rc, "%s", err.c_str());
    return ok();
}

msibm_status msibm_backward_levels(const msibm_pair* pair, const msibm_config* cfg, const int16_t* const* maps,
                                   const float* const* grad_soft, float* grad_left, float* grad_right,
                                   void* workspace, size_t ws_bytes, void* stream)
{
    int K;
    msibm_status st = validate_levels(pair, cfg, &K);
    if (st != MSIBM_OK) return st;
    if (pair->dtype != MSIBM_F32) return fail(MSIBM_ERR_UNSUPPORTED, "the backward takes float images");
    if (!maps || !grad_soft || !grad_left || !grad_right) return fail(MSIBM_ERR_INVALID_ARG, "NULL argument");
    for (int k = 1; k < K; ++k)
        if (!maps[k]) return fail(MSIBM_ERR_INVALID_ARG, "maps[%d] is NULL", k);
    const PairLayout lay = pair_layout(*pair, K, false, false, false, true);
    if (!workspace || ws_bytes < lay.bytes)
        return fail(MSIBM_ERR_WORKSPACE, "workspace %zu bytes < %zu needed", workspace ? ws_bytes : (size_t)0,
                    lay.bytes);
    std::string err;
    const int rc = run_pair_backward_levels(*pair, lay, cfg, (char*)workspace, maps, grad_soft, grad_left,
                                            grad_right, (hipStream_t)stream, &err);
    if (rc != MSIBM_OK) return fail(rc, "%s", err.c_str());
    return ok();
}

}  // extern "C"
