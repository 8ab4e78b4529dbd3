// Persistent batched forward: every pair and every level of a batch in one
// kernel launch.
//
// The host lays the work out as "segments": one per (pair, stage, level), a
// stage being a pyramid reduce, the window statistics, or the matching of a
// level.  A segment is a grid of tiles (the same tiles the per-level kernels
// use), and its tile rows are "bands".  Segments are listed in a topological
// order (every dependency of a segment comes earlier), so numbering all tiles
// of all segments in list order gives a global task order in which every task
// depends only on earlier tasks.
//
// Each resident workgroup repeatedly takes the next task number with one
// atomic add, waits until the bands it reads are complete (band counters reach
// the segment's tile-column count), runs the tile function, then releases its
// results (device-scope fence) and bumps its own band counter.  A task waits only
// on tasks dequeued before it, by workgroups that are already running, so the
// scheme cannot deadlock for any grid size.
//
// Waiting polls the counters with relaxed device-scope atomic loads (coherent
// across the XCDs' L2 caches) and performs one acquire fence after the last
// counter is seen complete: an acquire on every poll would invalidate the L2
// on every iteration of every waiting workgroup.  The producer side is one
// release fence (L2 write-back) per task before its relaxed counter increment.
// Every wait is bounded by wall-clock time; on expiry the workgroup raises the
// error flag and all workgroups stop taking tasks, so the kernel always ends.
#pragma once

#include "levels_impl.hpp"
#include "match_impl.hpp"

namespace msibm {

struct BatchArgs {
    const Segment* segs;
    int nseg;
    int ntasks;
    const LevelDesc* levels;  // K entries per pair, from level_base[pair]
    const int* level_base;
    int* counters;            // band counters (zeroed before the launch)
    int* head;                // task counter (zeroed)
    int* error;               // set when a wait times out (zeroed)
    int n, r, rs;
    double var_eps;
    float inv_tau;
    long long wait_ticks;     // bound of one wait, in wall_clock64() ticks
};

// Band range [lo, hi] of segment `d` that a task of segment `s` at tile row ty
// reads.
__device__ __forceinline__ void dep_bands(const Segment& s, const Segment& d, const LevelDesc* lv, int ty,
                                          int n, int* lo, int* hi)
{
    int r0, r1, dh;  // rows of the dependency's level and its tile height
    if (s.type == SEG_REDUCE) {  // input rows of the 5-tap reduce, level k-1
        r0 = 2 * RD_H * ty - 2;
        r1 = 2 * RD_H * ty + 2 * RD_H;
        dh = RD_H;
    } else if (s.type == SEG_STATS) {  // window rows, level k (reduced images)
        r0 = ST_H * ty - n;
        r1 = ST_H * ty + ST_H - 1 + n;
        dh = RD_H;
    } else if (d.type == SEG_STATS) {  // matching reads statistics of its own rows
        r0 = TILE_H1 * ty;
        r1 = TILE_H1 * ty + TILE_H1 - 1;
        dh = ST_H;
    } else {  // refine reads the coarser map at half the rows
        r0 = (TILE_H1 * ty) >> 1;
        r1 = (TILE_H1 * ty + TILE_H1 - 1) >> 1;
        dh = TILE_H1;
    }
    const int Hd = lv[d.level].H;
    *lo = max(0, r0) / dh;
    *hi = min(Hd - 1, r1) / dh;
}

// NW: half window, NCR: slots of a restricted search, NCS: slots of the soft
// level (0 = no soft level).  Both input element types are handled per level.
template <int NW, int NCR, int NCS>
__global__ __launch_bounds__(MATCH_THREADS) void persistent_kernel(BatchArgs a)
{
    __shared__ union Smem {
        MatchSmem<NW, ChunkOf<MODE_FULL>::value, 1> full;
        MatchSmem<NW, ChunkOf<MODE_REFINE>::value, 1> refine;
        ReduceSmem red;
        StatsSmem st;
    } sm;
    __shared__ int s_task, s_seg, s_abort;

    for (;;) {
        if (threadIdx.x == 0) {
            const int t = atomicAdd(a.head, 1);
            int seg = -1, abort = 0;
            if (t < a.ntasks) {
                // segment of task t: last segment whose task0 <= t
                int lo = 0, hi = a.nseg - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (a.segs[mid].task0 <= t) lo = mid;
                    else hi = mid - 1;
                }
                seg = lo;
                const Segment s = a.segs[seg];
                const LevelDesc* lv = a.levels + a.level_base[s.pair];
                const int ty = (t - s.task0) / s.tiles_x;
                const long long t0 = wall_clock64();
                for (int k = 0; k < 2 && !abort; ++k) {
                    if (s.dep_seg[k] < 0) continue;
                    const Segment d = a.segs[s.dep_seg[k]];
                    int blo, bhi;
                    dep_bands(s, d, lv, ty, a.n, &blo, &bhi);
                    for (int b = blo; b <= bhi && !abort; ++b) {
                        while (__hip_atomic_load(a.counters + d.band0 + b, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT) < d.tiles_x) {
                            if (wall_clock64() - t0 > a.wait_ticks ||
                                __hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                                __hip_atomic_store(a.error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                                abort = 1;
                                break;
                            }
                            __builtin_amdgcn_s_sleep(8);
                        }
                    }
                }
                // make the producers' released data visible to this workgroup
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            s_task = t;
            s_seg = seg;
            s_abort = abort;
        }
        __syncthreads();
        const int t = s_task;
        if (t >= a.ntasks || s_abort) break;
        const Segment s = a.segs[s_seg];
        const LevelDesc* lv = a.levels + a.level_base[s.pair];
        const int idx = t - s.task0, tx = idx % s.tiles_x, ty = idx / s.tiles_x;
        const LevelDesc& L = lv[s.level];
        if (s.type == SEG_REDUCE) {
            const LevelDesc& P = lv[s.level - 1];
            ReduceArgs ra{};
            ra.src[0] = P.img[0];
            ra.src[1] = P.img[1];
            ra.dst[0] = (float*)L.img[0];
            ra.dst[1] = (float*)L.img[1];
            ra.views = 2;
            ra.H = P.H;
            ra.W = P.W;
            ra.spitch = P.pitch;
            ra.Ho = L.H;
            ra.Wo = L.W;
            ra.dpitch = L.pitch;
            for (int v = 0; v < 2; ++v) {
                if (P.dtype == 0) reduce_tile<uint8_t>(ra, v, tx, ty, sm.red);
                else reduce_tile<float>(ra, v, tx, ty, sm.red);
            }
        } else if (s.type == SEG_STATS) {
            for (int v = 0; v < 2; ++v) {
                if (L.dtype == 0)
                    stats_tile<uint8_t, NW>((const uint8_t*)L.img[v], L.H, L.W, L.pitch, L.stat[v], L.W, a.var_eps,
                                            tx * ST_W, ty * ST_H, sm.st);
                else
                    stats_tile<float, NW>((const float*)L.img[v], L.H, L.W, L.pitch, L.stat[v], L.W, a.var_eps,
                                          tx * ST_W, ty * ST_H, sm.st);
            }
        } else {
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
            if (s.type != SEG_FULL) {
                const LevelDesc& C = lv[s.level + 1];
                m.prior = C.map;
                m.Hc = C.H;
                m.Wc = C.W;
                m.ppitch = C.W;
            }
            m.r = (s.type == SEG_SOFT) ? a.rs : a.r;
            m.d_out = L.map;
            m.c_out = L.cost;
            m.soft_out = L.soft;
            m.opitch = L.W;
            m.inv_tau = a.inv_tau;
            if (s.type == SEG_FULL) {
                if (L.dtype == 0) match_tile<uint8_t, NW, FULL_NC, MODE_FULL, 1, 1>(m, tx, ty, sm.full);
                else match_tile<float, NW, FULL_NC, MODE_FULL, 1, 1>(m, tx, ty, sm.full);
            } else if (s.type == SEG_REFINE) {
                if (L.dtype == 0) match_tile<uint8_t, NW, NCR, MODE_REFINE, 1, 0>(m, tx, ty, sm.refine);
                else match_tile<float, NW, NCR, MODE_REFINE, 1, 0>(m, tx, ty, sm.refine);
            } else {
                if constexpr (NCS > 0) match_tile<float, NW, NCS, MODE_SOFT, 1, 0>(m, tx, ty, sm.refine);
            }
        }
        // tile functions end with a workgroup barrier: every store of the tile
        // has been issued; release them device-wide, then publish the band
        if (threadIdx.x == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_fetch_add(a.counters + s.band0 + ty, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

}  // namespace msibm
