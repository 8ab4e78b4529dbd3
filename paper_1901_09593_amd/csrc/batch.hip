// Batched forward: task layout on the host, persistent-kernel launch, and the
// cached hipGraph of [counter reset + persistent kernel].
#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "batch_impl.hpp"
#include "plan.hpp"
#include "timing.hpp"

namespace msibm {

// Window sizes, refine radii and soft radii the persistent kernel is built for.
static bool batch_supported(const msibm_config* cfg)
{
    const int n = cfg->half_window, r = cfg->refine_radius, rs = cfg->soft_radius;
    return n >= 3 && n <= 5 && (r == 2 || r == 3) && (rs == 0 || rs == 3);
}

struct BatchPlan {
    std::vector<Segment> segs;
    std::vector<LevelDesc> levels;
    std::vector<int> level_base;
    int ntasks = 0, nbands = 0;
    // byte offsets inside the batch region of the workspace
    size_t off_counters, off_head, off_segs, off_levels, off_base, bytes;
};

static int cdiv(int a, int b) { return (a + b - 1) / b; }

// Segments in topological order: all pyramid reduces (by level), all window
// statistics, then the matching levels from each pair's coarsest level down.
static void build_segments(const msibm_pair* pairs, int np, const msibm_config* cfg, const int* K,
                           BatchPlan& pl)
{
    int Kmax = 0;
    for (int p = 0; p < np; ++p) Kmax = K[p] > Kmax ? K[p] : Kmax;
    std::vector<std::vector<int>> red(np, std::vector<int>(MSIBM_MAX_LEVELS, -1)),
        sta(np, std::vector<int>(MSIBM_MAX_LEVELS, -1)), mat(np, std::vector<int>(MSIBM_MAX_LEVELS, -1));
    auto add = [&](int type, int p, int k, int tx, int ty, int d0, int d1) {
        Segment s{};
        s.type = type;
        s.pair = p;
        s.level = k;
        s.tiles_x = tx;
        s.tiles_y = ty;
        s.task0 = pl.ntasks;
        s.band0 = pl.nbands;
        s.dep_seg[0] = d0;
        s.dep_seg[1] = d1;
        pl.ntasks += tx * ty;
        pl.nbands += ty;
        pl.segs.push_back(s);
        return (int)pl.segs.size() - 1;
    };
    for (int k = 1; k < Kmax; ++k)
        for (int p = 0; p < np; ++p)
            if (k < K[p]) {
                const int h = level_dim(pairs[p].height, k), w = level_dim(pairs[p].width, k);
                red[p][k] = add(SEG_REDUCE, p, k, cdiv(w, RD_W), cdiv(h, RD_H), k >= 2 ? red[p][k - 1] : -1, -1);
            }
    for (int k = 0; k < Kmax; ++k)
        for (int p = 0; p < np; ++p)
            if (k < K[p]) {
                const int h = level_dim(pairs[p].height, k), w = level_dim(pairs[p].width, k);
                sta[p][k] = add(SEG_STATS, p, k, cdiv(w, ST_W), cdiv(h, ST_H), k >= 1 ? red[p][k] : -1, -1);
            }
    for (int d = 0; d < Kmax; ++d)
        for (int p = 0; p < np; ++p) {
            const int k = K[p] - 1 - d;
            if (k < 0) continue;
            const int h = level_dim(pairs[p].height, k), w = level_dim(pairs[p].width, k);
            const bool coarsest = (k == K[p] - 1);
            const int type = coarsest ? SEG_FULL : ((k == 0 && cfg->soft_radius > 0) ? SEG_SOFT : SEG_REFINE);
            mat[p][k] = add(type, p, k, cdiv(w, TILE_W), cdiv(h, TILE_H1), sta[p][k], coarsest ? -1 : mat[p][k + 1]);
        }
}

static void plan_layout(BatchPlan& pl, int np, int nlevels)
{
    size_t off = 0;
    pl.off_counters = off;
    off = align_up(off + sizeof(int) * (size_t)pl.nbands);
    pl.off_head = off;  // head, error
    off = align_up(off + 2 * sizeof(int));
    pl.off_segs = off;
    off = align_up(off + sizeof(Segment) * pl.segs.size());
    pl.off_levels = off;
    off = align_up(off + sizeof(LevelDesc) * (size_t)nlevels);
    pl.off_base = off;
    off = align_up(off + sizeof(int) * (size_t)np);
    pl.bytes = off;
}

static int levels_of(const msibm_pair& p) { return p.num_levels ? p.num_levels : auto_levels(p.max_disp); }

size_t batch_extra_bytes(const msibm_pair* pairs, int n_pairs, const msibm_config* cfg)
{
    if (!(cfg->flags & MSIBM_FLAG_BATCHED)) return 0;
    std::vector<int> K(n_pairs);
    int nl = 0;
    for (int p = 0; p < n_pairs; ++p) {
        K[p] = levels_of(pairs[p]);
        nl += K[p];
    }
    BatchPlan pl;
    build_segments(pairs, n_pairs, cfg, K.data(), pl);
    plan_layout(pl, n_pairs, nl);
    return pl.bytes;
}

template <int NW, int NCR, int NCS>
static hipError_t launch_persistent_t(const BatchArgs& a, hipStream_t s)
{
    static int grid = 0;
    if (!grid) {
        int dev = 0, cus = 0, per_cu = 0;
        hipGetDevice(&dev);
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persistent_kernel<NW, NCR, NCS>, MATCH_THREADS, 0);
        grid = cus * (per_cu > 0 ? per_cu : 1);
    }
    hipLaunchKernelGGL((persistent_kernel<NW, NCR, NCS>), dim3(grid), dim3(MATCH_THREADS), 0, s, a);
    return hipGetLastError();
}

template <int NW>
static hipError_t launch_persistent_n(int ncr, int ncs, const BatchArgs& a, hipStream_t s)
{
    if (ncr == 5 && ncs == 0) return launch_persistent_t<NW, 5, 0>(a, s);
    if (ncr == 7 && ncs == 0) return launch_persistent_t<NW, 7, 0>(a, s);
    if (ncr == 5 && ncs == 7) return launch_persistent_t<NW, 5, 7>(a, s);
    if (ncr == 7 && ncs == 7) return launch_persistent_t<NW, 7, 7>(a, s);
    return hipErrorInvalidValue;
}

static hipError_t launch_persistent(int n, int ncr, int ncs, const BatchArgs& a, hipStream_t s)
{
    switch (n) {
        case 3: return launch_persistent_n<3>(ncr, ncs, a, s);
        case 4: return launch_persistent_n<4>(ncr, ncs, a, s);
        case 5: return launch_persistent_n<5>(ncr, ncs, a, s);
    }
    return hipErrorInvalidValue;
}

// Two seconds of wall_clock64() ticks: far longer than any task, short enough
// that a broken table ends the kernel promptly.
static long long wait_ticks()
{
    static long long ticks = 0;
    if (!ticks) {
        int dev = 0, khz = 0;
        hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
            khz = 100000;  // 100 MHz
        ticks = 2000LL * khz;
    }
    return ticks;
}

__global__ void zero_ints(int* p, int count)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) p[i] = 0;
}

// Enqueue [counter reset, persistent kernel] for a plan whose tables are in place.
static hipError_t enqueue_batch(const BatchPlan& pl, char* bw, const msibm_config* cfg, hipStream_t s)
{
    BatchArgs a{};
    a.segs = (const Segment*)(bw + pl.off_segs);
    a.nseg = (int)pl.segs.size();
    a.ntasks = pl.ntasks;
    a.levels = (const LevelDesc*)(bw + pl.off_levels);
    a.level_base = (const int*)(bw + pl.off_base);
    a.counters = (int*)(bw + pl.off_counters);
    a.head = (int*)(bw + pl.off_head);
    a.error = a.head + 1;
    a.n = cfg->half_window;
    a.r = cfg->refine_radius;
    a.rs = cfg->soft_radius;
    a.var_eps = cfg->var_eps;
    a.inv_tau = cfg->soft_radius > 0 ? 1.f / cfg->tau : 0.f;
    a.wait_ticks = wait_ticks();
    // counters, head and error are contiguous from off_counters up to the tables
    const int nints = (int)((pl.off_segs - pl.off_counters) / sizeof(int));
    hipLaunchKernelGGL(zero_ints, dim3((nints + 255) / 256 < 1024 ? (nints + 255) / 256 : 1024), dim3(256), 0, s,
                       a.counters, nints);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    TimedLaunch t("persistent", s);
    return launch_persistent(cfg->half_window, slots_for_radius(cfg->refine_radius),
                             cfg->soft_radius ? slots_for_radius(cfg->soft_radius) : 0, a, s);
}

// Graph cache: one instantiated graph per (pairs, outputs, workspace, config).
struct GraphKey {
    std::vector<char> bytes;
    bool operator<(const GraphKey& o) const { return bytes < o.bytes; }
};
struct GraphEntry {
    hipGraphExec_t exec = nullptr;
};
static std::mutex g_graph_mu;
static std::map<GraphKey, GraphEntry> g_graphs;

static GraphKey make_key(const msibm_pair* pairs, int np, const msibm_config* cfg, const BatchOutputs& out,
                         void* ws, size_t ws_bytes, hipStream_t s)
{
    GraphKey k;
    auto put = [&](const void* p, size_t n) {
        const char* c = (const char*)p;
        k.bytes.insert(k.bytes.end(), c, c + n);
    };
    put(pairs, sizeof(msibm_pair) * np);
    put(cfg, sizeof(msibm_config));
    for (int p = 0; p < np; ++p) {
        const void* q[4] = {out.disp[p], out.cost ? out.cost[p] : nullptr, out.soft ? out.soft[p] : nullptr,
                            out.prior1 ? out.prior1[p] : nullptr};
        put(q, sizeof(q));
    }
    put(&ws, sizeof(ws));
    put(&ws_bytes, sizeof(ws_bytes));
    put(&s, sizeof(s));
    return k;
}

// Offset of the batched scheduler's error flag inside the workspace.
size_t batch_error_offset(const msibm_pair* pairs, int np, const msibm_config* cfg)
{
    std::vector<int> K(np);
    int nl = 0;
    size_t base = 0;
    for (int p = 0; p < np; ++p) {
        K[p] = levels_of(pairs[p]);
        nl += K[p];
        base += pair_layout(pairs[p], K[p]).bytes;
    }
    BatchPlan pl;
    build_segments(pairs, np, cfg, K.data(), pl);
    plan_layout(pl, np, nl);
    return base + pl.off_head + sizeof(int);
}

int run_batched(const msibm_pair* pairs, int np, const msibm_config* cfg, const BatchOutputs& out,
                void* workspace, size_t ws_bytes, hipStream_t s, std::string* err)
{
    if (!batch_supported(cfg)) {
        *err = "the batched launch supports half_window 3..5, refine_radius 2 or 3 and soft_radius 0 or 3";
        return MSIBM_ERR_UNSUPPORTED;
    }
    for (int p = 1; p < np; ++p)
        if (pairs[p].dtype != pairs[0].dtype) {
            *err = "every pair of a batched call must have the same dtype";
            return MSIBM_ERR_UNSUPPORTED;
        }
    const bool use_graph = (cfg->flags & MSIBM_FLAG_GRAPH) != 0;
    GraphKey key;
    if (use_graph) {
        key = make_key(pairs, np, cfg, out, workspace, ws_bytes, s);
        std::lock_guard<std::mutex> g(g_graph_mu);
        auto it = g_graphs.find(key);
        if (it != g_graphs.end()) {
            TimedLaunch t("graph", s);
            hipError_t e = hipGraphLaunch(it->second.exec, s);
            if (e != hipSuccess) {
                *err = std::string("graph launch: ") + hipGetErrorString(e);
                return MSIBM_ERR_HIP;
            }
            return MSIBM_OK;
        }
    }
    // per-pair layouts and level descriptors
    std::vector<int> K(np);
    int nl = 0;
    for (int p = 0; p < np; ++p) {
        K[p] = levels_of(pairs[p]);
        nl += K[p];
    }
    BatchPlan pl;
    build_segments(pairs, np, cfg, K.data(), pl);
    plan_layout(pl, np, nl);
    size_t base = 0;
    for (int p = 0; p < np; ++p) {
        const msibm_pair& P = pairs[p];
        const PairLayout lay = pair_layout(P, K[p]);
        char* ws = (char*)workspace + base;
        base += lay.bytes;
        pl.level_base.push_back((int)pl.levels.size());
        for (int k = 0; k < K[p]; ++k) {
            LevelDesc d{};
            if (k == 0) {
                d.img[0] = P.left;
                d.img[1] = P.right;
                d.pitch = P.pitch;
                d.dtype = P.dtype;
                d.map = out.disp[p];
                d.cost = out.cost ? out.cost[p] : nullptr;
                d.soft = out.soft ? out.soft[p] : nullptr;
            } else {
                d.img[0] = ws + lay.img[k][0];
                d.img[1] = ws + lay.img[k][1];
                d.pitch = lay.w[k];
                d.dtype = MSIBM_F32;
                d.map = (k == 1 && out.prior1 && out.prior1[p]) ? out.prior1[p] : (int16_t*)(ws + lay.map[k]);
            }
            d.H = lay.h[k];
            d.W = lay.w[k];
            d.stat[0] = (float4*)(ws + lay.stat[k][0]);
            d.stat[1] = (float4*)(ws + lay.stat[k][1]);
            d.Dk = level_range(P.max_disp, k);
            pl.levels.push_back(d);
        }
    }
    char* bw = (char*)workspace + base;
    // tables: one host staging buffer, copied in one transfer
    std::vector<char> host(pl.bytes - pl.off_segs);
    std::memcpy(host.data(), pl.segs.data(), sizeof(Segment) * pl.segs.size());
    std::memcpy(host.data() + (pl.off_levels - pl.off_segs), pl.levels.data(), sizeof(LevelDesc) * pl.levels.size());
    std::memcpy(host.data() + (pl.off_base - pl.off_segs), pl.level_base.data(), sizeof(int) * pl.level_base.size());
    hipError_t e = hipMemcpyAsync(bw + pl.off_segs, host.data(), host.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // host buffer is released on return
    if (e != hipSuccess) {
        *err = std::string("table upload: ") + hipGetErrorString(e);
        return MSIBM_ERR_HIP;
    }
    if (!use_graph) {
        e = enqueue_batch(pl, bw, cfg, s);
        if (e != hipSuccess) {
            *err = std::string("persistent launch: ") + hipGetErrorString(e);
            return MSIBM_ERR_HIP;
        }
        return MSIBM_OK;
    }
    // capture [reset + persistent kernel] once, then replay
    hipGraph_t graph = nullptr;
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t e2 = enqueue_batch(pl, bw, cfg, s);
        e = hipStreamEndCapture(s, &graph);
        if (e2 != hipSuccess) e = e2;
    }
    GraphEntry ent;
    if (e == hipSuccess) e = hipGraphInstantiate(&ent.exec, graph, nullptr, nullptr, 0);
    if (graph) hipGraphDestroy(graph);
    if (e == hipSuccess) e = hipGraphLaunch(ent.exec, s);
    if (e != hipSuccess) {
        *err = std::string("graph capture: ") + hipGetErrorString(e);
        return MSIBM_ERR_HIP;
    }
    std::lock_guard<std::mutex> g(g_graph_mu);
    g_graphs[key] = ent;
    return MSIBM_OK;
}

}  // namespace msibm
