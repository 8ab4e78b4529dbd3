#!/usr/bin/env python3
"""Throughput of the hierarchical ZNCC block-matching forward pass on one MI355X.

A step is one hierarchical forward of a batch of 32 uint8 stereo pairs of
uneven sizes (W ~ U{640..2880}, H ~ U{480..1988}, D ~ U{64..400}; 9x9 ZNCC
windows, refine radius 2, per pair the smallest level count whose coarsest
level has at most 32 candidates): pyramid of both views, window statistics,
full search at each pair's coarsest level, restricted search at every finer
level, for all 32 pairs, replayed from one captured hipGraph of the
stage-batched launches.  Inputs, workspace and outputs are resident in device
memory before the timed region starts.

Prints ONE JSON line.  `value` = pixel-disparity ZNCC evaluations per second
(valid candidates actually scored, summed over levels and pairs).  Extra fields:
  batch             the same batch as 32 plain per-pair calls, as stage-batched
                    launches without the graph, and per-stage HIP-event times;
  roofline          the dominant kernel (the batched level-0 restricted search)
                    against the FP32 vector peak, with HBM traffic from
                    hardware counters;
  single_pair       the 1436x992 pair alone (plain per-pair path, K = 4 and
                    K = 5) and by flat full-range block matching;
  batch_variants    the batch with the selective median, the confidence
                    gating and the paper's whole method, plain vs graph;
  fwd_bwd           forward + masked-L1 loss gradient + backward of 8 x 960x540
                    and 4 x 2880x1988 float pairs: plain per-pair forward plus
                    separate backward, the same as batched graphs, and the fused
                    step (one call, one graph for forward, loss and backward);
  cpu_baseline      the FP64 oracle timed on the host cores over pairs of the
                    same batch (a reported baseline, not a target).
`python bench.py --copy-probe BYTES` only runs a plain device copy of known
size (used to check how the hardware traffic counters count bytes) and prints
nothing.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X figures used for the roofline
CU, SIMD_PER_CU, LANES, CLOCK_HZ = 256, 4, 16, 2.4e9
PEAK_FP32_UNPACKED = CU * SIMD_PER_CU * LANES * 2 * CLOCK_HZ / 1e12   # 78.6 TFLOP/s (FMA = 2)
PEAK_FP32_PUBLISHED = 157.3                                           # packed dual-issue figure
PEAK_HBM = 8000.0                                                     # GB/s
MEDIAN_ALPHA = 0.9  # the threshold of the selective median filter that Section IV reports
GATE_ALPHA = GATE_BETA = 0.9  # the gating thresholds Section IV reports

METRIC = "pixel-disparity ZNCC evals/s + ms/pair, batched vs plain; fwd+bwd ms"
DOMINANT = "batch_match_refine_l0"   # timing label of the batched level-0 restricted search
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "match_multi_refine_l0_batch32_traffic.md")
# sources of the dominant kernel: a recorded traffic figure holds only while
# these files are unchanged
KERNEL_SOURCES = ["paper_1901_09593_amd/csrc/match_impl.hpp", "paper_1901_09593_amd/csrc/common.hpp",
                  "paper_1901_09593_amd/csrc/match_n4.hip"]


def direct_flops_per_eval(n: int) -> float:
    """Algorithmic FP32 operations per evaluation of a restricted search with
    precomputed window statistics: N = (2n+1)^2 multiply-adds for the cross sum
    (2 flops each) plus 8 to normalise and compare."""
    return 2.0 * (2 * n + 1) ** 2 + 8.0


def kernel_flops_per_eval(n: int) -> float:
    """FP32 operations the matching kernel issues per evaluation: a thread scores
    a 2x2 pixel block, sharing (2n+2)^2 multiply-adds per candidate slot over the
    block's four windows, plus 6 adds to split them and 5 flops per evaluation to
    normalise and compare."""
    return (2.0 * (2 * n + 2) ** 2 + 6.0) / 4.0 + 5.0


def algorithmic_bytes_per_px_u8() -> float:
    """HBM bytes a restricted search of a uint8 level must move per pixel: both
    views read once (2), the coarser int16 prior (2 bytes per 4 pixels), the
    int16 disparity and the float score written (6).  Window statistics are
    this build's intermediate, not part of the algorithm's bytes."""
    return 2.0 + 0.5 + 6.0


def kernel_sha() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic():
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, or None when it is missing or the kernel changed since."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    m = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    h = re.search(r"kernel_sources_sha256:\s*([0-9a-f]{64})", text)
    if not m or not h or h.group(1) != kernel_sha():
        return None
    return float(m.group(1))


# --------------------------------------------------------------------------- counting

def level_counts(torch, maps, D, K, r):
    """Valid candidates scored per level, from every level's winner-take-all map
    (the restricted interval of each pixel follows from the coarser map)."""
    counts = []
    for k in range(K):
        h, w = maps[k].shape
        dev = maps[k].device
        Dk = -(-D // (1 << k))
        j = torch.arange(w, device=dev, dtype=torch.int64)
        top = torch.clamp(j, max=Dk - 1)
        if k == K - 1:
            counts.append(int((top + 1).sum()) * h)
            continue
        i = torch.arange(h, device=dev, dtype=torch.int64)
        dh = 2 * maps[k + 1].long()[i // 2][:, j // 2]
        c = torch.minimum(dh, j[None, :])
        lo = torch.clamp(c - r, min=0)
        hi = torch.minimum(top[None, :], c + r)
        counts.append(int((hi - lo + 1).sum()))
    return counts


def hier_counts(torch, M, L, R, D, K, n, r, eps):
    PL, PR = M.pyramid(L, K), M.pyramid(R, K)
    maps = [None] * K
    for k in range(K - 1, -1, -1):
        maps[k], _ = M.match_level(L if k == 0 else PL[k], R if k == 0 else PR[k], n, -(-D // (1 << k)),
                                   None if k == K - 1 else maps[k + 1], r, eps, with_cost=True)
    return level_counts(torch, maps, D, K, r)


def tune_summary(table):
    """Kernel shapes the autotuner measured and how often each shape won."""
    mode = ["full", "refine", "soft"]
    wins = {}
    for t in table:
        wins[str(t[7])] = wins.get(str(t[7]), 0) + 1
    return {"variant_bits": "1 = statistics in LDS (full search), 2 = XCD-aware tile order, 4 = candidates split over "
                            "waves, 8 = fixed candidate window (restricted search)",
            "wins_over_all_shapes": wins, "shapes_measured": len(table),
            "level0_shapes": [{"mode": mode[t[0]], "dtype": ["u8", "f32"][t[3]], "H": t[4], "W": t[5], "Dk": t[6],
                               "variant": t[7], "us": round(t[8], 2)} for t in table if t[1] == 4 and t[0] == 1][:8]}


def time_ms(torch, fn, steps, warmup):
    """Mean milliseconds per call between HIP events on the current stream."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


# --------------------------------------------------------------------------- sections

def batch_setup(torch, M, synth):
    """The 32-pair uneven batch on the device, with the valid candidates scored
    per pair and level (from every level's winner map)."""
    dev = torch.device("cuda:0")
    work = synth.batch_workload(32, 1000, workers=8)
    L = [torch.from_numpy(p.left).to(dev) for p, _ in work]
    R = [torch.from_numpy(p.right).to(dev) for p, _ in work]
    D = [c.max_disp for _, c in work]
    K = [c.levels for _, c in work]
    n, r, eps = work[0][1].half_window, work[0][1].refine_radius, work[0][1].var_eps
    counts = [hier_counts(torch, M, L[i], R[i], D[i], K[i], n, r, eps) for i in range(len(L))]
    return {"work": work, "L": L, "R": R, "D": D, "K": K, "n": n, "r": r, "eps": eps, "counts": counts,
            "evals": sum(sum(c) for c in counts), "evals_l0": sum(c[0] for c in counts),
            "level0_px": sum(p.left.size for p, _ in work)}


BATCH_WORKLOAD = ("32 uint8 pairs, W ~ U{640..2880}, H ~ U{480..1988}, D ~ U{64..400} (shape seed 1000, "
                  "pair i seed i), 8 slanted planes d in [0.05 D, 0.9 D], noise 2; 9x9 ZNCC, refine +-2, K per "
                  "pair (smallest with D_(K-1) <= 32); batched stages replayed from one hipGraph")


def section_batch_variants(torch, M, B, steps):
    """The batch with the selective median (Eq. 10), with the confidence gating
    (Eqs. 5-9), and with the paper's whole method (pre-blur, gating, median,
    windows halved from 11 x 11 level by level, refine +-1): plain per-pair
    calls against the batched graph."""
    dev = torch.device("cuda:0")
    L, R, D, K, n, r, eps = B["L"], B["R"], B["D"], B["K"], B["n"], B["r"], B["eps"]
    pairs_arr = M._pairs(L, R, D, K)[0]
    gate = {"gate": (GATE_ALPHA, GATE_BETA)}
    res = {}
    for key, opts, vflags, vn, vr in (
            ("with_median", {"median_alpha": MEDIAN_ALPHA}, 0, n, r),
            ("with_gating", gate, 0, n, r),
            ("with_paper_method", dict(gate, median_alpha=MEDIAN_ALPHA), M.FLAG_PREBLUR, [5, 2, 1, 1, 1], 1)):
        var = {}
        for name, flags in (("plain", vflags), ("graph", vflags | M.FLAG_BATCHED | M.FLAG_GRAPH)):
            cfg = M.make_config(vn, vr, eps, flags=flags, **opts)
            ws = torch.empty(M.workspace_bytes(pairs_arr, len(L), cfg), dtype=torch.uint8, device=dev)
            outs = M.disparity_many(L, R, D, K, vn, vr, eps, flags=flags, workspace=ws, **opts)

            def step():
                M.disparity_many(L, R, D, K, vn, vr, eps, flags=flags, workspace=ws, outputs=outs, **opts)
            var[name] = {"ms_per_batch": time_ms(torch, step, steps, 3)}
            if name == "plain":
                vref = outs
            else:
                var[name]["identical_to_plain"] = all(torch.equal(a[k], b[k]) for a, b in zip(vref, outs)
                                                      for k in a)
            del ws
        var["graph_speedup_vs_plain"] = var["plain"]["ms_per_batch"] / var["graph"]["ms_per_batch"]
        res[key] = var
    return res


def section_single(torch, M, synth, steps):
    """The 1436x992 pair alone on the plain per-pair path (K = 4, and K = 5:
    16 candidates at the coarsest level), per-launch HIP-event times, and flat
    full-range block matching of the same pair."""
    dev = torch.device("cuda:0")
    p, cfg = synth.workload("mid1436")
    H, W, D, n, r, eps = cfg.height, cfg.width, cfg.max_disp, cfg.half_window, cfg.refine_radius, cfg.var_eps
    Lg = torch.from_numpy(p.left).to(dev)
    Rg = torch.from_numpy(p.right).to(dev)
    res = {"workload": "1436x992 uint8 stereo pair, 8 slanted planes d 10..250, gain 0.9, offset +8, noise 4; "
                       "9x9 ZNCC, D=256, refine +-2, plain per-pair forward"}
    for K in (cfg.levels, cfg.levels + 1):
        counts = hier_counts(torch, M, Lg, Rg, D, K, n, r, eps)
        ws = torch.empty(M.workspace_bytes(M._pairs([Lg], [Rg], [D], [K])[0], 1, M.make_config(n, r, eps)),
                         dtype=torch.uint8, device=dev)
        outs = M.disparity_many([Lg], [Rg], [D], [K], n, r, eps, with_cost=True, workspace=ws)

        def step():
            M.disparity_many([Lg], [Rg], [D], [K], n, r, eps, with_cost=True, workspace=ws, outputs=outs)
        ms = time_ms(torch, step, steps, 5)
        M.timing_enable(True)
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        tim = M.timing_read()
        M.timing_enable(False)
        res[f"K{K}"] = {"ms_per_pair": ms, "evals_per_pair": sum(counts), "evals_per_level": counts,
                        "evals_per_s": sum(counts) / (ms * 1e-3),
                        "kernels_us": {k: round(1e3 * v[0] / v[1], 2) for k, v in sorted(tim.items())}}
        del ws
    # flat full search at full resolution (standard block matching) for comparison
    flat_evals = int(sum(min(D, j + 1) for j in range(W)) * H)
    dflat = torch.empty((H, W), dtype=torch.int16, device=dev)
    wsl = torch.empty(M.lib().msibm_level_workspace_size(H, W), dtype=torch.uint8, device=dev)

    def flat():
        M._check(M.lib().msibm_match_level(
            M._ptr(Lg), M._ptr(Rg), 0, H, W, W, n, D, None, 0, 0, 0, 0, float(eps),
            M._ptr(dflat), None, W, None, M._ptr(wsl), wsl.numel(), M._stream(dev)))
    flat_ms = time_ms(torch, flat, max(3, steps // 4), 3)
    res["flat_full_search"] = {"ms_per_pair": flat_ms, "evals_per_pair": flat_evals,
                               "evals_per_s": flat_evals / (flat_ms * 1e-3),
                               "hierarchical_speedup": flat_ms / res[f"K{cfg.levels}"]["ms_per_pair"]}
    return res

def section_accuracy(torch, M, synth, steps):
    """Disparity error against the generator's ground truth (the synthetic
    stand-in for the paper's accuracy table): the configured hierarchy, with
    and without the selective median filter, the paper's own parameters (refine
    +-1, block size halving per level from 11x11, level 0 pre-blurred, the
    median filter at alpha 0.9) and flat block matching, on non-occluded pixels
    away from the borders.  Also the median kernel's own time at level 0 and its
    bandwidth (8 algorithmic bytes per pixel: the map and cost read, the map
    written)."""
    dev = torch.device("cuda:0")
    res = {}
    for name in ("small320", "mid1436"):
        p, cfg = synth.workload(name)
        H, W, D, K, n, r, eps = cfg.height, cfg.width, cfg.max_disp, cfg.levels, cfg.half_window, \
            cfg.refine_radius, cfg.var_eps
        Lg, Rg = torch.from_numpy(p.left).to(dev), torch.from_numpy(p.right).to(dev)
        halving = [max(1, 5 >> k) for k in range(K)]  # 11x11, 5x5, 3x3, 3x3 ...
        b = max(halving[0], n) + 1
        vis = p.nonocc.copy()
        vis[:b, :] = vis[H - b:, :] = False
        vis[:, :b] = vis[:, W - b:] = False
        gate = (GATE_ALPHA, GATE_BETA)
        runs = {
            "hierarchy": dict(n=n, r=r, preblur=False, K=K, alpha=None, gate=None),
            "hierarchy_median": dict(n=n, r=r, preblur=False, K=K, alpha=MEDIAN_ALPHA, gate=None),
            "hierarchy_gated": dict(n=n, r=r, preblur=False, K=K, alpha=None, gate=gate),
            "hierarchy_gated_median": dict(n=n, r=r, preblur=False, K=K, alpha=MEDIAN_ALPHA, gate=gate),
            "paper_parameters": dict(n=halving, r=1, preblur=True, K=K, alpha=MEDIAN_ALPHA, gate=gate),
            "flat_block_matching": dict(n=n, r=0, preblur=False, K=1, alpha=None, gate=None),
        }
        out = {"workload": f"{W}x{H} uint8 pair ({name}), D={D}", "pixels_scored": int(vis.sum()),
               "paper_parameters": f"refine +-1, windows {[2 * v + 1 for v in halving]} by level, level 0 "
                                   f"pre-blurred, gating alpha {GATE_ALPHA} beta {GATE_BETA}, selective "
                                   f"median at alpha {MEDIAN_ALPHA}"}
        for label, c in runs.items():
            def fwd():
                return M.disparity(Lg, Rg, D, c["K"], c["n"], c["r"], eps, preblur=c["preblur"],
                                   median_alpha=c["alpha"], gate=c["gate"])
            d = fwd()["disp"].cpu().numpy().astype(np.float64)
            err = np.abs(d - p.disp)[vis]
            ms = time_ms(torch, fwd, steps, 2)
            out[label] = {"mean_abs_err_px": float(err.mean()), "bad_1px": float((err > 1).mean()),
                          "bad_2px": float((err > 2).mean()), "ms_per_pair": ms}
            if label in ("hierarchy_median", "hierarchy_gated"):
                M.timing_enable(True)
                for _ in range(steps):
                    fwd()
                torch.cuda.synchronize()
                tim = M.timing_read()
                M.timing_enable(False)
                out[label]["kernels_us"] = {k: 1e3 * v[0] / v[1] for k, v in sorted(tim.items())}
            if label == "hierarchy_median":
                us = out[label]["kernels_us"]["median_l0"]
                out["median_l0_kernel"] = {"avg_us": us, "GB_per_s": 8.0 * H * W / (us * 1e-6) / 1e9,
                                           "frac_of_hbm_peak": 8.0 * H * W / (us * 1e-6) / 1e9 / PEAK_HBM}
        res[name] = out
    return res


def section_gated(torch, M, synth, steps):
    """The paper's confidence gating (Eqs. 5-9) on the 1436x992 pair: time per
    pair, per-kernel times, and the work of the level-0 gate launch (the
    fallback full search and the re-pick fused in one walk).  It scores, for
    every tile (8 rows x (128 - 2n - 4) columns) holding a pixel that takes
    the fallback search or whose restricted-search cost is at most alpha, every
    region pixel (the tile plus a 2-pixel ring) at every candidate up to the
    tile's last such column's range; the scores per launch are counted here
    from the same inputs the launch sees."""
    dev = torch.device("cuda:0")
    p, cfg = synth.workload("mid1436")
    H, W, D, K, n, r, eps = cfg.height, cfg.width, cfg.max_disp, cfg.levels, cfg.half_window, \
        cfg.refine_radius, cfg.var_eps
    gate = (GATE_ALPHA, GATE_BETA)
    Lg, Rg = torch.from_numpy(p.left).to(dev), torch.from_numpy(p.right).to(dev)

    def fwd():
        return M.disparity(Lg, Rg, D, K, n, r, eps, gate=gate)
    out = fwd()
    ms = time_ms(torch, fwd, steps, 2)
    M.timing_enable(True)
    for _ in range(steps):
        fwd()
    torch.cuda.synchronize()
    tim = M.timing_read()
    M.timing_enable(False)
    kern = {k: 1e3 * v[0] / v[1] for k, v in sorted(tim.items())}
    # the level-0 launches' inputs: level 1's map and Eq. 7 cost, then the gated search
    PL, PR = M.pyramid(Lg, 2), M.pyramid(Rg, 2)
    lvl1 = M.disparity(PL[1], PR[1], -(-D // 2), K - 1, n, r, eps, gate=gate)
    assert torch.equal(lvl1["disp"], M.disparity(Lg, Rg, D, K, n, r, eps, gate=gate, with_prior1=True)["prior1"])
    up = M.upsample_cost(lvl1["cost"], H, W)
    d1, C1 = M.match_level_gated(Lg, Rg, n, D, lvl1["disp"], lvl1["cost"], r, gate[1], eps)
    _, Cr = M.match_level(Lg, Rg, n, D, lvl1["disp"], r, eps)
    full_mask = (~(up > gate[1])).cpu().numpy()
    pick_mask = (~(C1.double() > gate[0])).cpu().numpy()
    walk_mask = full_mask | (~(Cr.double() > gate[0])).cpu().numpy()

    def scores(mask, halo):
        th, tw = 8, 128 - 2 * n - 2 * halo
        total = 0
        for y0 in range(0, H, th):
            for x0 in range(0, W, tw):
                m = mask[y0:y0 + th, x0:x0 + tw]
                if not m.any():
                    continue
                xmax = x0 + int(np.nonzero(m.any(axis=0))[0].max())
                total += (th + 2 * halo) * (tw + 2 * halo) * (min(D - 1, xmax) + 1)
        return total
    res = {"workload": f"{W}x{H} uint8 pair (mid1436), K={K}, {2 * n + 1}x{2 * n + 1} ZNCC, D={D}, "
                       f"refine +-{r}, gating alpha {gate[0]} beta {gate[1]}",
           "ms_per_pair": ms, "kernels_us": kern,
           "level0_full_search_fraction": float(full_mask.mean()), "level0_repick_fraction": float(pick_mask.mean())}
    sc = scores(walk_mask, 2)
    us = kern["gate_fused_l0"]
    res["gate_fused_l0"] = {"avg_us": us, "region_scores_per_launch": sc, "scores_per_s": sc / (us * 1e-6)}
    return res


def section_levels(torch, M, synth, steps):
    """Soft output at every level (an extension): forward and backward through
    every level and the pyramid for the 960x540 float pairs, per pair."""
    dev = torch.device("cuda:0")
    p, cfg = synth.workload("diff960", 0)
    H, W, D, K, n, eps, rs, tau = cfg.height, cfg.width, cfg.max_disp, cfg.levels, cfg.half_window, \
        cfg.var_eps, cfg.soft_radius, cfg.tau
    Lg, Rg = torch.from_numpy(p.left).to(dev), torch.from_numpy(p.right).to(dev)
    soft, maps = M.disparity_levels(Lg, Rg, D, K, n, eps, rs, tau)
    grads = [torch.ones_like(s) / s.numel() for s in soft]
    fwd_ms = time_ms(torch, lambda: M.disparity_levels(Lg, Rg, D, K, n, eps, rs, tau), steps, 2)
    bwd_ms = time_ms(torch, lambda: M.backward_levels(Lg, Rg, maps, grads, D, K, n, eps, rs, tau), steps, 2)
    M.timing_enable(True)
    for _ in range(steps):
        M.backward_levels(Lg, Rg, maps, grads, D, K, n, eps, rs, tau)
    torch.cuda.synchronize()
    tim = M.timing_read()
    M.timing_enable(False)
    return {"workload": f"{W}x{H} float pair (diff960), K={K}, {2 * n + 1}x{2 * n + 1} ZNCC, D={D}, soft-argmax "
                        f"+-{rs} (tau {tau}) at levels 0..{K - 2}, loss = mean of every level's soft output",
            "fwd_ms": fwd_ms, "bwd_ms": bwd_ms,
            "bwd_kernels_us": {k: 1e3 * v[0] / v[1] for k, v in sorted(tim.items())}}


def section_fwd_bwd(torch, M, synth, name, count, steps):
    """Forward + masked mean-L1 loss gradient + backward for `count` float pairs."""
    dev = torch.device("cuda:0")
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats(dev)
    base = torch.cuda.memory_allocated(dev)
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(min(count, 8)) as ex:
        work = list(ex.map(lambda i: synth.workload(name, i), range(count)))
    cfg = work[0][1]
    H, W, D, K, n, r, eps, rs, tau = cfg.height, cfg.width, cfg.max_disp, cfg.levels, cfg.half_window, \
        cfg.refine_radius, cfg.var_eps, cfg.soft_radius, cfg.tau
    L = [torch.from_numpy(p.left).to(dev) for p, _ in work]
    R = [torch.from_numpy(p.right).to(dev) for p, _ in work]
    gt = [torch.from_numpy(p.disp.astype(np.float32)).to(dev) for p, _ in work]
    # loss pixels: the one mask definition the tests and the oracle use too
    mask = [torch.from_numpy(synth.loss_mask(p.nonocc, n, D)).to(dev) for p, _ in work]
    cnt = [mm.sum().clamp(min=1).float() for mm in mask]
    Ds, Ks = [D] * count, [K] * count
    pairs_arr = M._pairs(L, R, Ds, Ks)[0]
    res = {"workload": f"{count} x {W}x{H} float pairs ({name}), K={K}, {2 * n + 1}x{2 * n + 1} ZNCC, "
                       f"D={D}, refine +-{r}, soft-argmax +-{rs} at level 0 (tau {tau}), masked mean L1 "
                       "to the generator's disparity",
           "pairs": count}
    evals = None
    for label, flags in (("plain", 0), ("batched_graph", M.FLAG_BATCHED | M.FLAG_GRAPH)):
        ws = torch.empty(M.workspace_bytes(pairs_arr, count, M.make_config(n, r, eps, rs, tau, flags)),
                         dtype=torch.uint8, device=dev)
        outs = M.disparity_many(L, R, Ds, Ks, n, r, eps, soft_radius=rs, tau=tau, flags=flags, workspace=ws)
        g = [torch.zeros((H, W), dtype=torch.float32, device=dev) for _ in range(count)]
        grads = M.backward_many(L, R, [o["prior1"] for o in outs], g, Ds, Ks, n, r, eps, rs, tau, flags=flags,
                                workspace=ws)

        def fwd():
            M.disparity_many(L, R, Ds, Ks, n, r, eps, soft_radius=rs, tau=tau, flags=flags, workspace=ws,
                             outputs=outs)

        def loss_grad():
            for i in range(count):
                torch.mul(torch.sign(outs[i]["soft"] - gt[i]) * mask[i], 1.0 / cnt[i], out=g[i])

        def bwd():
            M.backward_many(L, R, [o["prior1"] for o in outs], g, Ds, Ks, n, r, eps, rs, tau, flags=flags,
                            workspace=ws, outputs=grads)

        def step():
            fwd()
            loss_grad()
            bwd()
        if evals is None:
            fwd()
            evals = 0
            for i in range(count):
                c = hier_counts(torch, M, L[i], R[i], D, K, n, r, eps)
                # the soft level scores its own +-rs interval
                c[0] = level_counts(torch, [outs[i]["disp"], outs[i]["prior1"]], D, 2, rs)[0]
                evals += sum(c)
        ms_fwd = time_ms(torch, fwd, steps, 2)
        step()
        torch.cuda.synchronize()
        ms_bwd = time_ms(torch, bwd, steps, 2)
        ms_step = time_ms(torch, step, steps, 2)
        res[label] = {"fwd_ms": ms_fwd, "bwd_ms": ms_bwd, "fwd_bwd_ms": ms_step,
                      "fwd_bwd_ms_per_pair": ms_step / count, "workspace_bytes": ws.numel()}
        del ws
    # the fused step: forward, loss and backward in one call (msibm_fwd_bwd_l1);
    # with the graph flag one captured graph for all of it
    mask8 = [m.to(torch.uint8) for m in mask]
    for label, flags in (("fused_plain", 0), ("fused_batched_graph", M.FLAG_BATCHED | M.FLAG_GRAPH)):
        ws = torch.empty(M.workspace_bytes(pairs_arr, count, M.make_config(n, r, eps, rs, tau, flags)),
                         dtype=torch.uint8, device=dev)
        fo = M.fwd_bwd_l1(L, R, gt, mask8, Ds, Ks, n, r, eps, rs, tau, flags=flags, workspace=ws)

        def fused():
            M.fwd_bwd_l1(L, R, gt, mask8, Ds, Ks, n, r, eps, rs, tau, flags=flags, workspace=ws, outputs=fo)
        ms = time_ms(torch, fused, steps, 2)
        res[label] = {"fwd_bwd_ms": ms, "fwd_bwd_ms_per_pair": ms / count, "workspace_bytes": ws.numel(),
                      "loss_pair0": float(fo[0]["loss"])}
        if label == "fused_batched_graph":
            M.timing_enable(True)
            for _ in range(steps):
                M.fwd_bwd_l1(L, R, gt, mask8, Ds, Ks, n, r, eps, rs, tau, flags=M.FLAG_BATCHED, workspace=ws,
                             outputs=fo)
            torch.cuda.synchronize()
            tim = M.timing_read()
            M.timing_enable(False)
            res[label]["stages_us"] = {k: round(1e3 * v[0] / v[1], 2) for k, v in sorted(tim.items())}
        del ws
    res["evals_per_batch_forward"] = evals
    res["fwd_bwd_speedup_batched_vs_plain"] = res["plain"]["fwd_bwd_ms"] / res["batched_graph"]["fwd_bwd_ms"]
    res["fwd_bwd_speedup_fused_graph_vs_plain"] = res["plain"]["fwd_bwd_ms"] / res["fused_batched_graph"]["fwd_bwd_ms"]
    res["peak_hbm_bytes"] = torch.cuda.max_memory_allocated(dev) - base
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="wall time budget of the oracle baseline sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tune-cache", default=None,
                    help="kernel-shape table to read and extend (profiling runs reuse a plain run's choices)")
    ap.add_argument("--sections", default="single,variants,fwd_bwd,accuracy,gated,levels",
                    help="extra sections beside the headline step: single, variants, fwd_bwd, accuracy, gated, "
                         "levels, or none")
    ap.add_argument("--no-tune", action="store_true",
                    help="use the default kernel shapes instead of measuring them first")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes five times")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the method's hot path has no cross-GPU exchange, and the library "
              "runs on a single MI355X (use --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1901_09593_amd import msibm, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.copy_probe:
        # an elementwise kernel (b = a * 1) rather than copy_, which may take the
        # DMA path: it reads and writes exactly BYTES bytes per launch
        a = torch.ones(args.copy_probe // 4, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(5):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        return
    sections = [s for s in args.sections.split(",") if s and s != "none"]

    if not args.no_tune:
        # first use of each level shape measures its kernel shapes (or takes
        # them from the cache file, which profiling runs share with a plain one)
        msibm.autotune(True, args.tune_cache)
    B = batch_setup(torch, msibm, synth)
    L, R, D, K, n, r, eps = B["L"], B["R"], B["D"], B["K"], B["n"], B["r"], B["eps"]
    npairs, evals = len(L), B["evals"]
    pairs_arr = msibm._pairs(L, R, D, K)[0]

    # resident buffers for the three forms of the same batch
    runs = {}
    for name, flags in (("graph", msibm.FLAG_BATCHED | msibm.FLAG_GRAPH), ("batched", msibm.FLAG_BATCHED),
                        ("plain", 0)):
        ws = torch.empty(msibm.workspace_bytes(pairs_arr, npairs, msibm.make_config(n, r, eps, flags=flags)),
                         dtype=torch.uint8, device=dev)
        outs = msibm.disparity_many(L, R, D, K, n, r, eps, flags=flags, workspace=ws)
        runs[name] = (flags, ws, outs)

    def step_of(name):
        flags, ws, outs = runs[name]
        return lambda: msibm.disparity_many(L, R, D, K, n, r, eps, flags=flags, workspace=ws, outputs=outs)

    # the timed region: K steps of the graph-replayed batch
    step = step_of("graph")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = e0.elapsed_time(e1) / args.steps
    value = evals / (ms_step * 1e-3)

    nsteps = max(3, min(args.steps, 20))
    plain_ms = time_ms(torch, step_of("plain"), nsteps, 3)
    batched_ms = time_ms(torch, step_of("batched"), nsteps, 3)
    ref = runs["plain"][2]
    identical = {nm: all(torch.equal(a[k], b[k]) for a, b in zip(ref, runs[nm][2]) for k in a)
                 for nm in ("graph", "batched")}

    # per-stage HIP-event timings: the stage-batched launches (the kernels the
    # graph replays), each bracketed by events on the stream it is launched on
    msibm.timing_enable(True)
    bstep = step_of("batched")
    for _ in range(args.steps):
        bstep()
    torch.cuda.synchronize()
    tim = msibm.timing_read()
    msibm.timing_enable(False)
    stages = {k: {"avg_us": round(1e3 * v[0] / v[1], 2), "launches": v[1]} for k, v in sorted(tim.items())}

    dom_us = stages[DOMINANT]["avg_us"]
    ev0 = B["evals_l0"]
    ach = direct_flops_per_eval(n) * ev0 / (dom_us * 1e-6) / 1e12
    issued = kernel_flops_per_eval(n) * ev0 / (dom_us * 1e-6) / 1e12
    traffic = recorded_traffic()
    alg_bytes = algorithmic_bytes_per_px_u8() * B["level0_px"]
    roof = {
        "kernel": DOMINANT + " (match_multi_kernel<u8, n=4, 5 slots, refine>)",
        "bound": "alu",
        "achieved": round(ach, 2),
        "peak": PEAK_FP32_PUBLISHED,
        "unit": "TFLOP/s",
        "frac": round(ach / PEAK_FP32_PUBLISHED, 4),
        "traffic": traffic,
        "flops_per_eval": direct_flops_per_eval(n),
        "evals_per_launch": ev0,
        "avg_launch_us": dom_us,
        "frac_of_unpacked_78_6": round(ach / PEAK_FP32_UNPACKED, 4),
        "issued_flops_per_eval": kernel_flops_per_eval(n),
        "issued_tflops": round(issued, 2),
        "issued_frac": round(issued / PEAK_FP32_PUBLISHED, 4),
        "issued_frac_of_unpacked": round(issued / PEAK_FP32_UNPACKED, 4),
        "algorithmic_bytes_per_launch": alg_bytes,
        "traffic_over_algorithmic": None if traffic is None else round(traffic / alg_bytes, 3),
        "hbm_gbps_from_traffic": None if traffic is None else round(traffic / (dom_us * 1e-6) / 1e9, 1),
    }
    batch = {
        "pairs": npairs, "level0_pixels": B["level0_px"], "evals_per_batch": evals, "evals_level0": ev0,
        "levels": sorted(set(K)),
        "graph": {"ms_per_batch": ms_step, "ms_per_pair": ms_step / npairs, "evals_per_s": value,
                  "identical_to_plain": identical["graph"]},
        "batched": {"ms_per_batch": batched_ms, "ms_per_pair": batched_ms / npairs,
                    "evals_per_s": evals / (batched_ms * 1e-3), "identical_to_plain": identical["batched"]},
        "plain": {"ms_per_batch": plain_ms, "ms_per_pair": plain_ms / npairs,
                  "evals_per_s": evals / (plain_ms * 1e-3)},
        "graph_speedup_vs_plain": plain_ms / ms_step,
        "stages_us": stages,
    }
    for nm in ("batched", "plain"):
        del runs[nm]
    torch.cuda.empty_cache()

    extra = {}
    if "single" in sections:
        extra["single_pair"] = section_single(torch, msibm, synth, nsteps)
    if "variants" in sections:
        extra["batch_variants"] = section_batch_variants(torch, msibm, B, nsteps)
    torch.cuda.empty_cache()
    if "fwd_bwd" in sections:
        extra["fwd_bwd"] = {
            "diff960x8": section_fwd_bwd(torch, msibm, synth, "diff960", 8, nsteps),
            "hires2880x4": section_fwd_bwd(torch, msibm, synth, "hires2880", 4, max(3, nsteps // 2)),
        }
    if "accuracy" in sections:
        extra["accuracy"] = section_accuracy(torch, msibm, synth, nsteps)
    if "gated" in sections:
        extra["gated"] = section_gated(torch, msibm, synth, nsteps)
    if "levels" in sections:
        extra["levels"] = section_levels(torch, msibm, synth, nsteps)

    # the FP64 oracle on the host cores: the batch's pairs in order until the
    # time budget is used (the whole batch if it fits)
    cpu = None
    if not args.no_cpu:
        import oracle
        done, done_evals, t0 = 0, 0, time.perf_counter()
        for (p, c), cnt in zip(B["work"], B["counts"]):
            oracle.disparity(p.left, p.right, c.max_disp, c.levels, c.half_window, c.refine_radius, c.var_eps)
            done += 1
            done_evals += sum(cnt)
            el = time.perf_counter() - t0
            if el >= args.cpu_seconds:
                break
        # one core, on the 320x240 pair (the paper's CPU setting is one process)
        ps, cs = synth.workload("small320")
        oracle.set_threads(1)
        reps1, t1 = 0, time.perf_counter()
        while True:
            oracle.disparity(ps.left, ps.right, cs.max_disp, cs.levels, cs.half_window, cs.refine_radius,
                             cs.var_eps)
            reps1 += 1
            el1 = time.perf_counter() - t1
            if el1 >= min(5.0, args.cpu_seconds):
                break
        oracle.set_threads(oracle.num_threads())
        model = ""
        try:
            with open("/proc/cpuinfo") as f:
                model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
        except OSError:
            pass
        cpu = {"value": done_evals / el, "unit": "evals/s", "cores": oracle.num_threads(), "kind": "oracle",
               "ms_per_pair": 1e3 * el / done,
               "sample": f"pairs 0..{done - 1} of the 32-pair batch, one full hierarchical forward each "
                         f"({done_evals} evaluations, {el:.1f} s)",
               "cpu_model": model,
               "one_core_small320_ms_per_pair": 1e3 * el1 / reps1,
               "one_core_sample": f"{reps1} forwards of the 320x240 pair on one thread ({el1:.1f} s)"}

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": BATCH_WORKLOAD, "pairs": npairs, "evals_per_batch": evals},
        "ms_per_pair": ms_step / npairs,
        "host_wall_ms_per_step": 1e3 * wall / args.steps,
        "batch": batch,
        "autotune": tune_summary(msibm.autotune_table()),
        "roofline": roof,
        **extra,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
