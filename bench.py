#!/usr/bin/env python3
"""Throughput of the hierarchical ZNCC block-matching forward pass on one MI355X.

A step is one hierarchical forward of the 1436x992 uint8 pair (4 levels, 9x9
ZNCC windows, 256 candidates at full resolution, refine radius 2): pyramid of
both views, window statistics, full search at the coarsest level, restricted
search at the three finer levels.  Inputs, workspace and outputs are resident in
device memory before the timed region starts.

Prints ONE JSON line.  `value` = pixel-disparity ZNCC evaluations per second
(valid candidates actually scored, summed over levels) of the plain per-pair
path.  Extra fields: the flat full-search comparison, per-kernel HIP-event
timings, the dominant kernel's roofline, and the FP64 oracle timed on the host
cores (a reported baseline, not a target).
"""
import argparse
import json
import os
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


def flops_per_eval(n: int) -> float:
    """FP32 operations per candidate evaluation of the matching kernel.

    A thread scores one window of candidate slots for a 2x2 pixel block: per slot
    (2n+2)^2 fused multiply-adds (2 flops each) build the block's four window
    cross sums, plus 6 adds to combine the shared and edge parts; per evaluation
    one subtract, one FMA and two multiplies normalise the score."""
    return (2.0 * (2 * n + 2) ** 2 + 6.0) / 4.0 + 5.0


def direct_flops_per_eval(n: int) -> float:
    """Direct-definition count with precomputed window statistics: N FMAs for
    the cross sum plus normalisation (context only)."""
    return 2.0 * (2 * n + 1) ** 2 + 8.0


def level_eval_counts(maps, H, W, D, K, r):
    """Valid candidates per level given every level's winner-take-all map."""
    counts = []
    for k in range(K):
        h, w = maps[k].shape
        Dk = -(-D // (1 << k))
        jj = np.arange(w)[None, :]
        top = np.minimum(Dk - 1, jj)
        if k == K - 1:
            counts.append(int(((top + 1) * np.ones((h, 1), dtype=np.int64)).sum()))
            continue
        ii = np.arange(h)[:, None]
        dh = 2 * maps[k + 1].astype(np.int64)[ii // 2, jj // 2]
        c = np.minimum(dh, jj)
        lo = np.maximum(0, c - r)
        hi = np.minimum(top, c + r)
        counts.append(int((hi - lo + 1).sum()))
    return counts


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="wall time budget of the oracle baseline sample")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the method has no cross-GPU exchange on its hot "
              "path and this build runs on a single MI355X (use --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1901_09593_amd import msibm, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    p, cfg = synth.workload("mid1436")
    H, W, D, K, n, r, eps = cfg.height, cfg.width, cfg.max_disp, cfg.levels, cfg.half_window, \
        cfg.refine_radius, cfg.var_eps
    Lg = torch.from_numpy(p.left).to(dev)
    Rg = torch.from_numpy(p.right).to(dev)

    # evaluation counts from the per-level maps (same kernels as the timed call)
    PL, PR = msibm.pyramid(Lg, K), msibm.pyramid(Rg, K)
    maps = [None] * K
    for k in range(K - 1, -1, -1):
        maps[k], _ = msibm.match_level(Lg if k == 0 else PL[k], Rg if k == 0 else PR[k], n,
                                       -(-D // (1 << k)), None if k == K - 1 else maps[k + 1], r,
                                       eps, with_cost=False)
    torch.cuda.synchronize()
    maps_h = [m.cpu().numpy() for m in maps]
    counts = level_eval_counts(maps_h, H, W, D, K, r)
    evals = sum(counts)

    # resident buffers, then the timed loop
    ws = None
    outs = msibm.disparity_many([Lg], [Rg], [D], [K], n, r, eps, with_cost=True)
    pairs_ws = msibm.workspace_bytes(msibm._pairs([Lg], [Rg], [D], [K])[0], 1,
                                     msibm.make_config(n, r, eps))
    ws = torch.empty(pairs_ws, dtype=torch.uint8, device=dev)

    def step():
        msibm.disparity_many([Lg], [Rg], [D], [K], n, r, eps, with_cost=True, workspace=ws,
                             outputs=outs)

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

    # per-kernel HIP-event timings: the same steps again with every launch
    # bracketed by events on the launch stream
    msibm.timing_enable(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    tim = msibm.timing_read()
    msibm.timing_enable(False)
    kernels = {k: {"avg_us": 1e3 * v[0] / v[1], "launches": v[1]} for k, v in sorted(tim.items())}

    dom = "match_refine_l0"
    dom_us = kernels[dom]["avg_us"]
    ach = flops_per_eval(n) * counts[0] / (dom_us * 1e-6) / 1e12
    roof = {
        "kernel": dom,
        "bound": "alu",
        "achieved": round(ach, 2),
        "peak": round(PEAK_FP32_UNPACKED, 1),
        "unit": "TFLOP/s",
        "frac": round(ach / PEAK_FP32_UNPACKED, 4),
        "traffic": None,
        "flops_per_eval": flops_per_eval(n),
        "evals_per_launch": counts[0],
        "avg_launch_us": round(dom_us, 2),
        "frac_of_published_fp32_157_3": round(ach / PEAK_FP32_PUBLISHED, 4),
        "direct_definition_equiv_tflops": round(direct_flops_per_eval(n) * counts[0] /
                                                (dom_us * 1e-6) / 1e12, 2),
    }

    # flat full search at full resolution (standard block matching) for comparison
    flat_evals = int(sum(min(D, j + 1) for j in range(W)) * H)
    dflat = torch.empty((H, W), dtype=torch.int16, device=dev)
    wsl = torch.empty(msibm.lib().msibm_level_workspace_size(H, W), dtype=torch.uint8, device=dev)

    def flat():
        msibm._check(msibm.lib().msibm_match_level(
            msibm._ptr(Lg), msibm._ptr(Rg), 0, H, W, W, n, D, None, 0, 0, 0, 0, float(eps),
            msibm._ptr(dflat), None, W, msibm._ptr(wsl), wsl.numel(), msibm._stream(dev)))

    for _ in range(3):
        flat()
    torch.cuda.synchronize()
    nflat = max(3, args.steps // 20)
    e0.record()
    for _ in range(nflat):
        flat()
    e1.record()
    torch.cuda.synchronize()
    flat_ms = e0.elapsed_time(e1) / nflat

    # the FP64 oracle on the host cores: whole pairs until the time budget is used
    cpu = None
    if not args.no_cpu:
        import oracle
        reps, t0 = 0, time.perf_counter()
        while True:
            oracle.disparity(p.left, p.right, D, K, n, r, eps)
            reps += 1
            el = time.perf_counter() - t0
            if el >= args.cpu_seconds:
                break
        cpu = {"value": evals * reps / el, "unit": "evals/s", "cores": oracle.num_threads(),
               "kind": "oracle", "ms_per_pair": 1e3 * el / reps,
               "sample": f"{reps} full hierarchical forwards of the 1436x992 pair ({el:.1f} s)"}

    line = {
        "metric": "pixel-disparity ZNCC evals/s + ms/pair, batched vs plain; fwd+bwd ms",
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
        "config": {"workload": "1436x992 uint8 stereo pair, 8 slanted planes d 10..250, gain 0.9, "
                               "offset +8, noise 4; K=4 levels, 9x9 ZNCC, D=256, refine +-2, "
                               "plain per-pair forward",
                   "evals_per_pair": evals, "evals_per_level": counts},
        "ms_per_pair": ms_step,
        "host_wall_ms_per_step": 1e3 * wall / args.steps,
        "flat_full_search": {"ms_per_pair": flat_ms, "evals_per_pair": flat_evals,
                             "evals_per_s": flat_evals / (flat_ms * 1e-3),
                             "hierarchical_speedup": flat_ms / ms_step},
        "kernels": kernels,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
