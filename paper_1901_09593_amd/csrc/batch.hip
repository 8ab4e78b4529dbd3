// Batched forward: all pairs of a call advance stage by stage, one launch per
// stage whose grid holds the tiles of every pair at that stage.
//
// Stages, in stream order: the pyramid reduce of level k for k = 1..K_max-1,
// the window statistics of every level, the full search of every pair's
// coarsest level (one launch for all levels), then the restricted search of
// level k from k = K_max-2 down to 0, each refining the map the previous step
// wrote.  Within a launch no tile waits on another; the stream order between
// launches carries every dependency.  A matching step holds one launch per
// (mode, element type, window size) present, since those are separate kernel
// instances.
//
// Launches find their tiles through a table of segments (one per pair and
// level) and per-level descriptors.  Without MSIBM_FLAG_GRAPH the table is
// uploaded into the workspace for every call from pinned host staging; with it
// the whole sequence is captured once into a hipGraph that owns a device copy of
// its table, and later calls with the same key replay the graph.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "backward_impl.hpp"
#include "levels_impl.hpp"
#include "plan.hpp"
#include "timing.hpp"

namespace msibm {

static int cdiv(int a, int b) { return (a + b - 1) / b; }
static int levels_of(const msibm_pair& p) { return p.num_levels ? p.num_levels : auto_levels(p.max_disp); }

enum StageKind {
    STAGE_LEVELS = 0, STAGE_STATS = 1, STAGE_MATCH = 2, STAGE_ZERO = 3, STAGE_BACKWARD = 4, STAGE_MEDIAN = 5,
    STAGE_GATE = 6, STAGE_BLUR = 7, STAGE_COUNT = 8, STAGE_FUSED = 9, STAGE_L1_FINAL = 10
};

struct StageLaunch {
    int kind, level;
    int mode, dtype, nc;  // matching only
    int first, nseg, blocks;
};

struct BatchPlan {
    std::vector<Segment> segs;
    std::vector<LevelDesc> levels;
    std::vector<int> level_base;
    std::vector<BackArgs> back;
    std::vector<StageLaunch> launches;
    size_t off_levels = 0, off_base = 0, off_back = 0, bytes = 0;  // table layout
};

// Zero both gradients of every pair of a backward launch (a fill kernel rather
// than a memset, so the sequence can be captured into a graph).
__global__ __launch_bounds__(256) void zero_multi_kernel(MultiArgs a)
{
    const Segment s = a.segs[segment_of(a.segs, a.nseg, blockIdx.x)];
    const BackArgs& b = a.back[s.pair];
    const size_t count = (size_t)b.H * b.W;
    const size_t base = (size_t)(blockIdx.x - s.task0) * ZERO_TILE + threadIdx.x;
    // the fused masked-L1 step also clears the pair's count and loss sum
    if (b.count && (int)blockIdx.x == s.task0 && threadIdx.x == 0) {
        *b.count = 0;
        *b.loss_sum = 0.f;
    }
#pragma unroll 4
    for (int m = 0; m < ZERO_TILE / 256; ++m) {
        const size_t i = base + (size_t)m * 256;
        if (i < count) {
            b.gL[i] = 0.f;
            b.gR[i] = 0.f;
        }
    }
}

// Tiles of one level: reduce tiles cover one view each, statistics and
// matching tiles both.
static Segment make_seg(int type, int p, int k, int h, int w, int dtype, int task0, int n = 0, int gmode = 0)
{
    Segment s{};
    s.type = type;
    s.pair = p;
    s.level = k;
    if (type == SEG_REDUCE) {
        s.tiles_x = cdiv(w, RD_W);
        s.tiles_y = cdiv(h, RD_H);
        s.views = 2;
    } else if (type == SEG_STATS) {  // a statistics tile covers both views
        s.tiles_x = cdiv(w, ST_W);
        s.tiles_y = cdiv(h, stats_tile_h(dtype));
        s.views = 1;
    } else if (type == SEG_GATE) {
        s.tiles_x = cdiv(w, gate_tile_w(dtype, n, gmode));
        s.tiles_y = cdiv(h, GATE_TH);
        s.views = 1;
    } else if (type == SEG_MEDIAN) {
        s.tiles_x = cdiv(w, MD_W);
        s.tiles_y = cdiv(h, MD_H);
        s.views = 1;
    } else if (type == SEG_ZERO) {
        s.tiles_x = (int)(((size_t)h * w + ZERO_TILE - 1) / ZERO_TILE);
        s.tiles_y = 1;
        s.views = 1;
    } else if (type == SEG_COUNT) {
        s.tiles_x = (int)(((size_t)h * w + COUNT_TILE - 1) / COUNT_TILE);
        s.tiles_y = 1;
        s.views = 1;
    } else {
        s.tiles_x = cdiv(w, TILE_W);
        s.tiles_y = cdiv(h, TILE_H1);
        s.views = 1;
    }
    s.task0 = task0;
    return s;
}

static int seg_tiles(const Segment& s) { return s.tiles_x * s.tiles_y * s.views; }

// Table: segments, level descriptors, level bases, backward arguments.
static void table_layout(BatchPlan& pl, int nlevels, int np, int nback)
{
    size_t off = align_up(sizeof(Segment) * pl.segs.size());
    pl.off_levels = off;
    off = align_up(off + sizeof(LevelDesc) * (size_t)nlevels);
    pl.off_base = off;
    off = align_up(off + sizeof(int) * (size_t)np);
    pl.off_back = off;
    pl.bytes = align_up(off + sizeof(BackArgs) * (size_t)nback);
}

// Segments and launches (no device pointers yet).  Levels below `lowest` are
// not matched (their pyramid images and statistics are still made).
static void plan_stages(const msibm_pair* pairs, int np, const msibm_config* cfg, BatchPlan& pl, int lowest = 0)
{
    std::vector<int> K(np);
    int Kmax = 0;
    for (int p = 0; p < np; ++p) {
        K[p] = levels_of(pairs[p]);
        Kmax = K[p] > Kmax ? K[p] : Kmax;
    }
    auto h_of = [&](int p, int k) { return level_dim(pairs[p].height, k); };
    auto w_of = [&](int p, int k) { return level_dim(pairs[p].width, k); };
    // element type of the image level k is matched on (the pre-blur matches
    // level 0 on a float copy)
    const bool preblur = (cfg->flags & MSIBM_FLAG_PREBLUR) != 0;
    auto dtype_at = [&](int p, int k) { return (k == 0 && !preblur) ? pairs[p].dtype : MSIBM_F32; };
    auto begin = [&](int kind, int level, int mode, int dtype, int nc) {
        StageLaunch l{};
        l.kind = kind;
        l.level = level;
        l.mode = mode;
        l.dtype = dtype;
        l.nc = nc;
        l.first = (int)pl.segs.size();
        pl.launches.push_back(l);
    };
    auto add = [&](int type, int p, int k) {
        StageLaunch& l = pl.launches.back();
        const Segment s =
            make_seg(type, p, k, h_of(p, k), w_of(p, k), dtype_at(p, k), l.blocks, level_n(cfg, k), l.mode);
        l.blocks += seg_tiles(s);
        l.nseg++;
        pl.segs.push_back(s);
    };
    // the pre-blur: one blur launch per pair (no segments) before everything
    if (preblur) begin(STAGE_BLUR, 0, 0, 0, 0);
    // pyramid step k: level k's statistics (heavier tiles first) side by side
    // with the reduce that makes level k + 1
    for (int k = 0; k < Kmax; ++k) {
        // a step whose statistics all read uint8 levels (their reduces then read
        // the same uint8 images) takes the leaner uint8 kernel
        bool all_u8 = true;
        for (int p = 0; p < np; ++p)
            if (k < K[p]) all_u8 = all_u8 && dtype_at(p, k) == MSIBM_U8;
        begin(STAGE_LEVELS, k, 0, all_u8 ? MSIBM_U8 : MSIBM_F32, 0);
        for (int p = 0; p < np; ++p)
            if (k < K[p]) add(SEG_STATS, p, k);
        for (int p = 0; p < np; ++p)
            if (k + 1 < K[p]) add(SEG_REDUCE, p, k + 1);
    }
    const int modes[3] = {MODE_FULL, MODE_REFINE, MODE_SOFT};
    const int segtype[3] = {SEG_FULL, SEG_REFINE, SEG_SOFT};
    auto mode_of = [&](int p, int k) {
        return (k == K[p] - 1) ? MODE_FULL : ((k == 0 && cfg->soft_radius > 0) ? MODE_SOFT : MODE_REFINE);
    };
    // A pair's coarsest level is searched in full from that level's statistics
    // alone, so the full searches of all levels share one launch per window
    // size and element type ahead of the refinement chain.
    {
        std::vector<int> ns;
        for (int k = Kmax - 1; k >= lowest; --k) {
            const int n = level_n(cfg, k);
            bool seen = false;
            for (int v : ns) seen = seen || v == n;
            if (!seen) ns.push_back(n);
        }
        for (int n : ns)
            for (int dt = 0; dt < 2; ++dt) {
                bool opened = false;
                for (int k = Kmax - 1; k >= lowest; --k) {
                    if (level_n(cfg, k) != n) continue;
                    for (int p = 0; p < np; ++p) {
                        if (k != K[p] - 1 || dtype_at(p, k) != dt) continue;
                        if (!opened) {
                            begin(STAGE_MATCH, k, MODE_FULL, dt, FULL_NC);
                            opened = true;
                        }
                        add(SEG_FULL, p, k);
                    }
                }
            }
    }
    for (int k = Kmax - 1; k >= lowest; --k) {
        for (int m = 1; m < 3; ++m)
            for (int dt = 0; dt < 2; ++dt) {
                bool opened = false;
                for (int p = 0; p < np; ++p) {
                    if (k >= K[p]) continue;
                    const int mode = mode_of(p, k);
                    const int dtype = dtype_at(p, k);
                    if (mode != modes[m] || dtype != dt) continue;
                    if (!opened) {
                        const int nc = mode == MODE_FULL
                                           ? FULL_NC
                                           : slots_for_radius(mode == MODE_SOFT ? cfg->soft_radius
                                                                                : cfg->refine_radius);
                        begin(STAGE_MATCH, k, mode, dt, nc);
                        opened = true;
                    }
                    add(segtype[m], p, k);
                }
            }
        // with the gating: the coarsest level of a pair re-picks, a finer one
        // runs the fused fallback search and re-pick (one launch per mode and
        // element type)
        if (cfg->flags & MSIBM_FLAG_GATED) {
            for (int gm = 0; gm < 2; ++gm)
                for (int dt = 0; dt < 2; ++dt) {
                    const int want = gm == 0 ? GATE_MODE_REPICK : GATE_MODE_FUSED;
                    bool opened = false;
                    for (int p = 0; p < np; ++p) {
                        if (k >= K[p] || mode_of(p, k) == MODE_SOFT) continue;
                        const int gmode = (k == K[p] - 1) ? GATE_MODE_REPICK : GATE_MODE_FUSED;
                        const int dtype = dtype_at(p, k);
                        if (gmode != want || dtype != dt) continue;
                        if (!opened) {
                            begin(STAGE_GATE, k, want, dt, 0);
                            opened = true;
                        }
                        add(SEG_GATE, p, k);
                    }
                }
        }
        // with the selective median: every pair's hard map of this level is
        // filtered before the next finer level reads it as its prior
        if (cfg->flags & MSIBM_FLAG_MEDIAN) {
            bool opened = false;
            for (int p = 0; p < np; ++p) {
                if (k >= K[p] || mode_of(p, k) == MODE_SOFT) continue;
                if (!opened) {
                    begin(STAGE_MEDIAN, k, 0, 0, 0);
                    opened = true;
                }
                add(SEG_MEDIAN, p, k);
            }
        }
    }
    int nl = 0;
    for (int p = 0; p < np; ++p) nl += K[p];
    table_layout(pl, nl, np, 0);
}

// Backward: level-0 statistics of every pair, zeroed gradients, backward tiles.
static void plan_backward_stages(const msibm_pair* pairs, int np, BatchPlan& pl)
{
    const int kinds[3] = {STAGE_STATS, STAGE_ZERO, STAGE_BACKWARD};
    const int types[3] = {SEG_STATS, SEG_ZERO, SEG_BACKWARD};
    for (int q = 0; q < 3; ++q) {
        StageLaunch l{};
        l.kind = kinds[q];
        l.first = (int)pl.segs.size();
        for (int p = 0; p < np; ++p) {
            const Segment sg = make_seg(types[q], p, 0, pairs[p].height, pairs[p].width, pairs[p].dtype, l.blocks);
            l.blocks += seg_tiles(sg);
            l.nseg++;
            pl.segs.push_back(sg);
        }
        pl.launches.push_back(l);
    }
    table_layout(pl, np, np, np);
}

// Launch over one segment per pair (tiles of `type`, level 0) appended to the plan.
static void add_pair_stage(const msibm_pair* pairs, int np, int kind, int type, BatchPlan& pl)
{
    StageLaunch l{};
    l.kind = kind;
    l.first = (int)pl.segs.size();
    for (int p = 0; p < np; ++p) {
        const Segment sg = make_seg(type, p, 0, pairs[p].height, pairs[p].width, pairs[p].dtype, l.blocks);
        l.blocks += seg_tiles(sg);
        l.nseg++;
        pl.segs.push_back(sg);
    }
    pl.launches.push_back(l);
}

// The fused masked-L1 step: gradients and loss accumulators cleared and the
// loss pixels counted, the forward down to level 1, one fused soft-level and
// backward launch for level 0 of every pair, the loss values.
static void plan_fused_stages(const msibm_pair* pairs, int np, const msibm_config* cfg, BatchPlan& pl)
{
    add_pair_stage(pairs, np, STAGE_ZERO, SEG_ZERO, pl);
    add_pair_stage(pairs, np, STAGE_COUNT, SEG_COUNT, pl);
    plan_stages(pairs, np, cfg, pl, 1);
    add_pair_stage(pairs, np, STAGE_FUSED, SEG_BACKWARD, pl);
    StageLaunch fin{};
    fin.kind = STAGE_L1_FINAL;
    fin.first = (int)pl.segs.size();
    fin.blocks = (np + 255) / 256;
    pl.launches.push_back(fin);
    int nl = 0;
    for (int p = 0; p < np; ++p) nl += levels_of(pairs[p]);
    table_layout(pl, nl, np, np);
}

// Workspace layout of one pair on the batched path (the same as the size query's).
static PairLayout batch_layout(const msibm_pair& P, const msibm_config* cfg)
{
    return pair_layout(P, levels_of(P), (cfg->flags & MSIBM_FLAG_PREBLUR) != 0,
                       (cfg->flags & MSIBM_FLAG_MEDIAN) != 0, (cfg->flags & MSIBM_FLAG_GATED) != 0);
}

// Level descriptors of every pair, with its workspace region and outputs.
static void plan_levels(const msibm_pair* pairs, int np, const msibm_config* cfg, const BatchOutputs& out,
                        char* workspace, BatchPlan& pl)
{
    size_t base = 0;
    const bool median = (cfg->flags & MSIBM_FLAG_MEDIAN) != 0;
    const bool gated = (cfg->flags & MSIBM_FLAG_GATED) != 0;
    const bool preblur = (cfg->flags & MSIBM_FLAG_PREBLUR) != 0;
    for (int p = 0; p < np; ++p) {
        const msibm_pair& P = pairs[p];
        const int K = levels_of(P);
        const PairLayout lay = batch_layout(P, cfg);
        char* ws = workspace + base;
        base += lay.bytes;
        pl.level_base.push_back((int)pl.levels.size());
        for (int k = 0; k < K; ++k) {
            LevelDesc d{};
            if (k == 0) {
                d.img[0] = P.left;
                d.img[1] = P.right;
                d.pitch = P.pitch;
                d.dtype = P.dtype;
                d.map = out.disp[p];
                d.cost = out.cost ? out.cost[p] : nullptr;
                d.soft = out.soft ? out.soft[p] : nullptr;
                if (preblur) {
                    // matched on the blurred copy; the pyramid reads the input
                    d.src[0] = P.left;
                    d.src[1] = P.right;
                    d.spitch = P.pitch;
                    d.sdtype = P.dtype;
                    d.img[0] = ws + lay.blur[0];
                    d.img[1] = ws + lay.blur[1];
                    d.pitch = lay.w[0];
                    d.dtype = MSIBM_F32;
                }
            } else {
                d.img[0] = ws + lay.img[k][0];
                d.img[1] = ws + lay.img[k][1];
                d.pitch = lay.w[k];
                d.dtype = MSIBM_F32;
                d.map = (k == 1 && out.prior1 && out.prior1[p]) ? out.prior1[p] : (int16_t*)(ws + lay.map[k]);
            }
            d.H = lay.h[k];
            d.W = lay.w[k];
            d.stat[0] = (WinStat*)(ws + lay.stat[k][0]);
            d.stat[1] = (WinStat*)(ws + lay.stat[k][1]);
            d.Dk = level_range(P.max_disp, k);
            // the gating keeps every hard level's cost (the next finer level's
            // gate reads it); the median filters every hard level: the search
            // writes the pair's scratch map (reused level after level) and the
            // cost, which the filter reads
            const bool soft_level = (k == 0 && K >= 2 && cfg->soft_radius > 0);
            if (gated && !soft_level && !d.cost)
                d.cost = k == 0 ? (float*)(ws + lay.ctmp) : (float*)(ws + lay.cmap[k]);
            if (median && !soft_level) {
                d.raw = (int16_t*)(ws + lay.dtmp);
                d.mcost = d.cost ? d.cost : (float*)(ws + lay.ctmp);
            }
            pl.levels.push_back(d);
        }
    }
}

static size_t pairs_bytes(const msibm_pair* pairs, int np, const msibm_config* cfg)
{
    size_t b = 0;
    for (int p = 0; p < np; ++p) b += batch_layout(pairs[p], cfg).bytes;
    return b;
}

size_t batch_extra_bytes(const msibm_pair* pairs, int n_pairs, const msibm_config* cfg)
{
    if (!(cfg->flags & MSIBM_FLAG_BATCHED)) return 0;
    BatchPlan fw, bw, fu;
    plan_stages(pairs, n_pairs, cfg, fw);
    plan_backward_stages(pairs, n_pairs, bw);
    size_t b = fw.bytes > bw.bytes ? fw.bytes : bw.bytes;
    if (cfg->soft_radius > 0) {
        plan_fused_stages(pairs, n_pairs, cfg, fu);
        b = fu.bytes > b ? fu.bytes : b;
    }
    return b;
}

// Host image of the table: segments, level descriptors, level bases.
static void pack_table(const BatchPlan& pl, std::vector<char>& host)
{
    host.assign(pl.bytes, 0);
    std::memcpy(host.data(), pl.segs.data(), sizeof(Segment) * pl.segs.size());
    std::memcpy(host.data() + pl.off_levels, pl.levels.data(), sizeof(LevelDesc) * pl.levels.size());
    std::memcpy(host.data() + pl.off_base, pl.level_base.data(), sizeof(int) * pl.level_base.size());
    if (!pl.back.empty()) std::memcpy(host.data() + pl.off_back, pl.back.data(), sizeof(BackArgs) * pl.back.size());
}

// Enqueue every stage launch; `table` is the device copy of the plan's table.
static hipError_t enqueue_stages(const BatchPlan& pl, const char* table, const msibm_config* cfg, bool timed,
                                 hipStream_t s)
{
    MultiArgs a{};
    a.levels = (const LevelDesc*)(table + pl.off_levels);
    a.level_base = (const int*)(table + pl.off_base);
    a.back = (const BackArgs*)(table + pl.off_back);
    a.r = cfg->refine_radius;
    a.rs = cfg->soft_radius;
    a.var_eps = cfg->var_eps;
    a.inv_tau = cfg->soft_radius > 0 ? 1.f / cfg->tau : 0.f;
    a.median_alpha = cfg->median_alpha;
    a.gate_alpha = cfg->gate_alpha;
    a.gate_beta = cfg->gate_beta;
    // restricted searches stage their whole candidate range at once wherever it
    // fits one chunk (decided per segment by the kernel)
    a.variant = VARIANT_FIXW;
    static const char* mode_name[3] = {"full", "refine", "soft"};
    for (const StageLaunch& l : pl.launches) {
        a.segs = (const Segment*)table + l.first;
        a.nseg = l.nseg;
        char lab[40];
        const bool bwd = !pl.back.empty();
        if (l.kind == STAGE_LEVELS) snprintf(lab, sizeof(lab), "batch_levels_l%d", l.level);
        else if (l.kind == STAGE_STATS) snprintf(lab, sizeof(lab), bwd ? "batch_bwd_stats" : "batch_stats");
        else if (l.kind == STAGE_ZERO) snprintf(lab, sizeof(lab), "batch_bwd_zero");
        else if (l.kind == STAGE_BACKWARD) snprintf(lab, sizeof(lab), "batch_backward_l0");
        else if (l.kind == STAGE_MEDIAN) snprintf(lab, sizeof(lab), "batch_median_l%d", l.level);
        else if (l.kind == STAGE_GATE)
            snprintf(lab, sizeof(lab), l.mode == GATE_MODE_FUSED ? "batch_gate_fused_l%d" : "batch_gate_repick_l%d",
                     l.level);
        else if (l.kind == STAGE_BLUR) snprintf(lab, sizeof(lab), "batch_preblur_l0");
        else if (l.kind == STAGE_COUNT) snprintf(lab, sizeof(lab), "batch_fused_count");
        else if (l.kind == STAGE_FUSED) snprintf(lab, sizeof(lab), "batch_fused_backward_l0");
        else if (l.kind == STAGE_L1_FINAL) snprintf(lab, sizeof(lab), "batch_fused_loss");
        else if (l.mode == MODE_FULL) snprintf(lab, sizeof(lab), "batch_match_full");
        else snprintf(lab, sizeof(lab), "batch_match_%s_l%d", mode_name[l.mode], l.level);
        const int slot = timed ? timing_begin(lab, s) : -1;
        hipError_t e = hipSuccess;
        if (l.kind == STAGE_BLUR) {
            // level 0 of every pair: its input blurred into the float copy it is matched on
            for (size_t p = 0; p < pl.level_base.size() && e == hipSuccess; ++p) {
                const LevelDesc& d = pl.levels[pl.level_base[p]];
                BlurArgs b{};
                for (int v = 0; v < 2; ++v) {
                    b.src[v] = d.src[v];
                    b.dst[v] = (float*)d.img[v];
                }
                b.H = d.H;
                b.W = d.W;
                b.spitch = d.spitch;
                b.dpitch = d.pitch;
                e = launch_blur(d.sdtype, b, s);
            }
        } else if (l.kind == STAGE_LEVELS) e = launch_levels_multi(level_n(cfg, l.level), l.dtype, a, l.blocks, s);
        else if (l.kind == STAGE_STATS) e = launch_stats_multi(level_n(cfg, 0), a, l.blocks, s);
        else if (l.kind == STAGE_ZERO) {
            hipLaunchKernelGGL(zero_multi_kernel, dim3(l.blocks), dim3(256), 0, s, a);
            e = hipGetLastError();
        } else if (l.kind == STAGE_BACKWARD || l.kind == STAGE_FUSED) {
            a.fused = l.kind == STAGE_FUSED;
            e = launch_backward_multi(level_n(cfg, 0), slots_for_radius(cfg->soft_radius), a, l.blocks, s);
            a.fused = 0;
        } else if (l.kind == STAGE_COUNT)
            e = launch_mask_count_multi(a, l.blocks, s);
        else if (l.kind == STAGE_L1_FINAL)
            e = launch_l1_finalize_multi(a, (int)pl.back.size(), s);
        else if (l.kind == STAGE_MEDIAN)
            e = launch_median_multi(a, l.blocks, s);
        else if (l.kind == STAGE_GATE)
            e = launch_gate_multi(level_n(cfg, l.level), l.dtype, l.mode, a, l.blocks, s);
        else e = launch_match_multi(level_n(cfg, l.level), l.dtype, l.mode, l.nc, a, l.blocks, s);
        if (timed) timing_end(slot, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ------------------------------------------------------------ per-device state
// Pinned host staging for table uploads: a ring of slots, each reused only after
// the copy that last read it has completed (its event).  A private stream per
// device for graph capture (the caller's stream may be the null stream, which
// cannot be captured).
struct StagingSlot {
    char* host = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
    bool used = false;
};
struct DeviceState {
    StagingSlot slot[8];
    int next = 0;
    hipStream_t capture = nullptr;
};
static std::mutex g_dev_mu;
static std::map<int, DeviceState> g_dev;

static hipError_t upload_table(int dev, char* dst, const std::vector<char>& src, hipStream_t s)
{
    std::lock_guard<std::mutex> g(g_dev_mu);
    DeviceState& st = g_dev[dev];
    StagingSlot& sl = st.slot[st.next];
    st.next = (st.next + 1) % 8;
    hipError_t e = hipSuccess;
    if (!sl.done) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
    if (e == hipSuccess && sl.used) e = hipEventSynchronize(sl.done);
    if (e == hipSuccess && sl.cap < src.size()) {
        if (sl.host) hipHostFree(sl.host);
        sl.host = nullptr;
        sl.cap = 0;
        e = hipHostMalloc((void**)&sl.host, src.size(), hipHostMallocDefault);
        if (e == hipSuccess) sl.cap = src.size();
    }
    if (e != hipSuccess) return e;
    std::memcpy(sl.host, src.data(), src.size());
    e = hipMemcpyAsync(dst, sl.host, src.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(sl.done, s);
    sl.used = (e == hipSuccess);
    return e;
}

static hipError_t capture_stream(int dev, hipStream_t* out)
{
    std::lock_guard<std::mutex> g(g_dev_mu);
    DeviceState& st = g_dev[dev];
    if (!st.capture) {
        hipError_t e = hipStreamCreateWithFlags(&st.capture, hipStreamNonBlocking);
        if (e != hipSuccess) return e;
    }
    *out = st.capture;
    return hipSuccess;
}

// ------------------------------------------------------------------ graph cache
// Key: device, pairs (pointers, shapes, D, K), cfg, output pointers, workspace.
struct GraphKey {
    std::vector<char> bytes;
    bool operator<(const GraphKey& o) const { return bytes < o.bytes; }
};
struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    char* table = nullptr;      // device copy of the plan's table, owned by the entry
    hipEvent_t done = nullptr;  // recorded after each replay: the last replay's end
    uint64_t last_use = 0;
};
static std::mutex g_graph_mu;
static std::map<GraphKey, GraphEntry> g_graphs;
static uint64_t g_graph_clock = 0;
static const size_t GRAPH_CACHE_MAX = 64;

// Key bytes: direction tag, device, pairs, cfg, then the call's buffer pointers.
static GraphKey make_key(char tag, int dev, const msibm_pair* pairs, int np, const msibm_config* cfg,
                         const std::vector<const void*>& bufs, void* ws, size_t ws_bytes)
{
    GraphKey k;
    auto put = [&](const void* p, size_t n) {
        const char* c = (const char*)p;
        k.bytes.insert(k.bytes.end(), c, c + n);
    };
    put(&tag, 1);
    put(&dev, sizeof(dev));
    put(pairs, sizeof(msibm_pair) * np);
    put(cfg, sizeof(msibm_config));
    put(bufs.data(), sizeof(void*) * bufs.size());
    put(&ws, sizeof(ws));
    put(&ws_bytes, sizeof(ws_bytes));
    return k;
}

static void destroy_entry(GraphEntry& e)
{
    if (e.exec) hipGraphExecDestroy(e.exec);
    if (e.table) hipFree(e.table);
    if (e.done) hipEventDestroy(e.done);
    e = GraphEntry{};
}

static int hip_fail(hipError_t e, const char* what, std::string* err)
{
    *err = std::string(what) + ": " + hipGetErrorString(e);
    return MSIBM_ERR_HIP;
}

// Capture the stage sequence on the private stream, with a device table of its own.
static int capture_graph(int dev, const BatchPlan& pl, const msibm_config* cfg, GraphEntry* ent,
                         std::string* err)
{
    std::vector<char> host;
    pack_table(pl, host);
    hipError_t e = hipMalloc((void**)&ent->table, host.size());
    if (e != hipSuccess) return hip_fail(e, "graph table", err);
    e = hipMemcpy(ent->table, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        destroy_entry(*ent);
        return hip_fail(e, "graph table upload", err);
    }
    hipStream_t cs;
    e = capture_stream(dev, &cs);
    if (e != hipSuccess) {
        destroy_entry(*ent);
        return hip_fail(e, "capture stream", err);
    }
    hipGraph_t graph = nullptr;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const hipError_t e2 = enqueue_stages(pl, ent->table, cfg, false, cs);
        e = hipStreamEndCapture(cs, &graph);
        if (e2 != hipSuccess) e = e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&ent->exec, graph, nullptr, nullptr, 0);
    if (graph) hipGraphDestroy(graph);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ent->done, hipEventDisableTiming);
    if (e != hipSuccess) {
        destroy_entry(*ent);
        return hip_fail(e, "graph capture", err);
    }
    return MSIBM_OK;
}

// Runs a plan made by `build`: replayed from the graph cache under `key` when
// graphs are on, else uploaded into the workspace table region and launched.
template <class Build>
static int run_plan(int dev, const msibm_config* cfg, const GraphKey* key, Build build, char* table,
                    hipStream_t s, std::string* err)
{
    hipError_t e;
    if (key) {
        // a full cache gives up its least recently replayed entry; the entry
        // leaves the map under the lock and is freed after the lock, once its
        // last replay has ended (a wait on that replay only)
        GraphEntry victim;
        {
            std::lock_guard<std::mutex> g(g_graph_mu);
            auto it = g_graphs.find(*key);
            if (it == g_graphs.end()) {
                BatchPlan pl;
                build(pl);
                GraphEntry ent;
                const int rc = capture_graph(dev, pl, cfg, &ent, err);
                if (rc != MSIBM_OK) return rc;
                if (g_graphs.size() >= GRAPH_CACHE_MAX) {
                    auto lru = g_graphs.begin();
                    for (auto jt = g_graphs.begin(); jt != g_graphs.end(); ++jt)
                        if (jt->second.last_use < lru->second.last_use) lru = jt;
                    victim = lru->second;
                    g_graphs.erase(lru);
                }
                it = g_graphs.emplace(*key, ent).first;
            }
            it->second.last_use = ++g_graph_clock;
            const int slot = timing_begin("batch_graph", s);
            e = hipGraphLaunch(it->second.exec, s);
            timing_end(slot, s);
            if (e == hipSuccess) e = hipEventRecord(it->second.done, s);
        }
        if (victim.exec) {
            hipEventSynchronize(victim.done);
            destroy_entry(victim);
        }
        if (e != hipSuccess) return hip_fail(e, "graph launch", err);
        return MSIBM_OK;
    }
    BatchPlan pl;
    build(pl);
    std::vector<char> host;
    pack_table(pl, host);
    e = upload_table(dev, table, host, s);
    if (e != hipSuccess) return hip_fail(e, "table upload", err);
    e = enqueue_stages(pl, table, cfg, true, s);
    if (e != hipSuccess) return hip_fail(e, "batched launch", err);
    return MSIBM_OK;
}

int run_batched(const msibm_pair* pairs, int np, const msibm_config* cfg, const BatchOutputs& out,
                void* workspace, size_t ws_bytes, hipStream_t s, std::string* err)
{
    int dev = 0;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "device", err);
    GraphKey key;
    const bool graph = (cfg->flags & MSIBM_FLAG_GRAPH) != 0;
    if (graph) {
        std::vector<const void*> bufs;
        for (int p = 0; p < np; ++p) {
            bufs.push_back(out.disp[p]);
            bufs.push_back(out.cost ? out.cost[p] : nullptr);
            bufs.push_back(out.soft ? out.soft[p] : nullptr);
            bufs.push_back(out.prior1 ? out.prior1[p] : nullptr);
        }
        key = make_key('F', dev, pairs, np, cfg, bufs, workspace, ws_bytes);
    }
    auto build = [&](BatchPlan& pl) {
        plan_stages(pairs, np, cfg, pl);
        plan_levels(pairs, np, cfg, out, (char*)workspace, pl);
    };
    return run_plan(dev, cfg, graph ? &key : nullptr, build, (char*)workspace + pairs_bytes(pairs, np, cfg), s,
                    err);
}

int run_batched_backward(const msibm_pair* pairs, int np, const msibm_config* cfg, const BatchGrads& g,
                         void* workspace, size_t ws_bytes, hipStream_t s, std::string* err)
{
    int dev = 0;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "device", err);
    GraphKey key;
    const bool graph = (cfg->flags & MSIBM_FLAG_GRAPH) != 0;
    if (graph) {
        std::vector<const void*> bufs;
        for (int p = 0; p < np; ++p) {
            bufs.push_back(g.prior1[p]);
            bufs.push_back(g.grad_soft[p]);
            bufs.push_back(g.grad_left[p]);
            bufs.push_back(g.grad_right[p]);
        }
        key = make_key('B', dev, pairs, np, cfg, bufs, workspace, ws_bytes);
    }
    auto build = [&](BatchPlan& pl) {
        plan_backward_stages(pairs, np, pl);
        size_t base = 0;
        for (int p = 0; p < np; ++p) {
            const msibm_pair& P = pairs[p];
            const PairLayout lay = batch_layout(P, cfg);
            char* ws = (char*)workspace + base;
            base += lay.bytes;
            LevelDesc d{};
            d.img[0] = P.left;
            d.img[1] = P.right;
            d.pitch = P.pitch;
            d.dtype = P.dtype;
            d.H = P.height;
            d.W = P.width;
            d.stat[0] = (WinStat*)(ws + lay.stat[0][0]);
            d.stat[1] = (WinStat*)(ws + lay.stat[0][1]);
            d.Dk = P.max_disp;
            pl.levels.push_back(d);
            pl.level_base.push_back(p);
            BackArgs b{};
            b.L = (const float*)P.left;
            b.R = (const float*)P.right;
            b.H = P.height;
            b.W = P.width;
            b.pitch = P.pitch;
            b.statL = d.stat[0];
            b.statR = d.stat[1];
            b.spitch = P.width;
            b.D = P.max_disp;
            b.prior = g.prior1[p];
            b.Hc = lay.h[1];
            b.Wc = lay.w[1];
            b.ppitch = lay.w[1];
            b.rs = cfg->soft_radius;
            b.inv_tau = 1.f / cfg->tau;
            b.g = g.grad_soft[p];
            b.gpitch = P.width;
            b.gL = g.grad_left[p];
            b.gR = g.grad_right[p];
            pl.back.push_back(b);
        }
    };
    return run_plan(dev, cfg, graph ? &key : nullptr, build, (char*)workspace + pairs_bytes(pairs, np, cfg), s,
                    err);
}

int run_batched_fused_l1(const msibm_pair* pairs, int np, const msibm_config* cfg, const FusedL1Pair* io,
                         void* workspace, size_t ws_bytes, hipStream_t s, std::string* err)
{
    int dev = 0;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "device", err);
    GraphKey key;
    const bool graph = (cfg->flags & MSIBM_FLAG_GRAPH) != 0;
    if (graph) {
        std::vector<const void*> bufs;
        for (int p = 0; p < np; ++p) {
            const FusedL1Pair& q = io[p];
            const void* b[9] = {q.gt, q.mask, q.disp, q.cost, q.soft, q.prior1, q.grad_left, q.grad_right, q.loss};
            bufs.insert(bufs.end(), b, b + 9);
        }
        key = make_key('L', dev, pairs, np, cfg, bufs, workspace, ws_bytes);
    }
    std::vector<int16_t*> disp(np), prior(np);
    std::vector<float*> cost(np), soft(np);
    for (int p = 0; p < np; ++p) {
        disp[p] = io[p].disp;
        prior[p] = io[p].prior1;
        cost[p] = io[p].cost;
        soft[p] = io[p].soft;
    }
    const BatchOutputs out{disp.data(), cost.data(), soft.data(), prior.data()};
    auto build = [&](BatchPlan& pl) {
        plan_fused_stages(pairs, np, cfg, pl);
        plan_levels(pairs, np, cfg, out, (char*)workspace, pl);
        size_t base = 0;
        for (int p = 0; p < np; ++p) {
            const msibm_pair& P = pairs[p];
            const PairLayout lay = batch_layout(P, cfg);
            char* ws = (char*)workspace + base;
            base += lay.bytes;
            BackArgs b{};
            b.L = (const float*)P.left;
            b.R = (const float*)P.right;
            b.H = P.height;
            b.W = P.width;
            b.pitch = P.pitch;
            b.statL = (const WinStat*)(ws + lay.stat[0][0]);
            b.statR = (const WinStat*)(ws + lay.stat[0][1]);
            b.spitch = P.width;
            b.D = P.max_disp;
            b.prior = io[p].prior1 ? io[p].prior1 : (const int16_t*)(ws + lay.map[1]);
            b.Hc = lay.h[1];
            b.Wc = lay.w[1];
            b.ppitch = lay.w[1];
            b.rs = cfg->soft_radius;
            b.inv_tau = 1.f / cfg->tau;
            b.gpitch = P.width;
            b.gL = io[p].grad_left;
            b.gR = io[p].grad_right;
            b.gt = io[p].gt;
            b.mask = io[p].mask;
            b.count = (int*)(ws + lay.l1acc);
            b.loss_sum = (float*)(ws + lay.l1acc) + 1;
            b.loss_out = io[p].loss;
            b.soft_out = io[p].soft;
            b.d_out = io[p].disp;
            b.c_out = io[p].cost;
            pl.back.push_back(b);
        }
    };
    return run_plan(dev, cfg, graph ? &key : nullptr, build, (char*)workspace + pairs_bytes(pairs, np, cfg), s,
                    err);
}

}  // namespace msibm
