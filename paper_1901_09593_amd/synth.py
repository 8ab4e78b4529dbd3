"""Seeded synthetic stereo pairs.

The paper evaluates on the Middlebury V3 stereo set (Section IV), which is not
available here; these generated pairs stand in for it.  Each pair has a textured
left view, a piecewise-planar ground-truth disparity, and a right view obtained by
warping the left view with that disparity (left-reference convention: the left
pixel (y, x) appears in the right view at column x - d).  Occluded right pixels are
filled with an independent texture of the same process, and the right view then
gets a gain, an offset and additive Gaussian noise.

This module draws inputs only.  It holds none of the matching arithmetic (no
pyramid, no correlation, no winner-take-all), so both the FP64 oracle tests and the
GPU path can use it without sharing any of the method's computation.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

__all__ = [
    "StereoPair",
    "MatchConfig",
    "make_pair",
    "texture",
    "disparity_layout",
    "warp_left_to_right",
    "workload",
    "batch_workload",
    "auto_levels",
    "grad_seed",
    "loss_mask",
]


@dataclasses.dataclass
class StereoPair:
    left: np.ndarray        # (H, W) uint8 or float32
    right: np.ndarray       # (H, W) same dtype as left
    disp: np.ndarray        # (H, W) float64 ground-truth disparity of each left pixel
    nonocc: np.ndarray      # (H, W) bool, left pixels visible in the right view
    seed: int


@dataclasses.dataclass
class MatchConfig:
    """Parameters of one matching run (the knobs of Section III)."""
    height: int
    width: int
    max_disp: int           # D: candidates 0..D-1 at full resolution
    levels: int             # K: number of pyramid images, level 0 = input
    half_window: int        # n: window is (2n+1) x (2n+1)
    refine_radius: int      # r: candidates [c-r, c+r] around the propagated prior
    dtype: str = "u8"       # "u8" (0..255) or "f32" (0..1)
    soft_radius: int = 0    # r_s: soft-argmax radius at level 0 (0 = hard only)
    tau: float = 0.05

    @property
    def var_eps(self) -> float:
        """Flat-window variance floor: (1e-3 of the intensity range)^2."""
        rng = 255.0 if self.dtype == "u8" else 1.0
        return (1e-3 * rng) ** 2


def auto_levels(max_disp: int, coarse_limit: int = 32) -> int:
    """Smallest K whose coarsest level searches at most `coarse_limit` candidates."""
    k = 1
    while -(-max_disp // (1 << (k - 1))) > coarse_limit:
        k += 1
    return k


def _gauss_taps(sigma: float, taps: int = 11) -> np.ndarray:
    h = taps // 2
    x = np.arange(-h, h + 1, dtype=np.float64)
    w = np.exp(-0.5 * (x / sigma) ** 2)
    return w / w.sum()


def _blur(img: np.ndarray, sigma: float) -> np.ndarray:
    """Separable Gaussian blur, reflect padding (texture synthesis only)."""
    w = _gauss_taps(sigma)
    h = len(w) // 2
    p = np.pad(img, ((0, 0), (h, h)), mode="reflect")
    out = np.zeros_like(img)
    for t, wt in enumerate(w):
        out += wt * p[:, t:t + img.shape[1]]
    p = np.pad(out, ((h, h), (0, 0)), mode="reflect")
    out2 = np.zeros_like(img)
    for t, wt in enumerate(w):
        out2 += wt * p[t:t + img.shape[0], :]
    return out2


def texture(rng: np.random.Generator, H: int, W: int, sigma: float = 1.5) -> np.ndarray:
    """Uniform noise, Gaussian-blurred, min-max scaled to [0, 1] (float64)."""
    t = _blur(rng.random((H, W)), sigma)
    lo, hi = t.min(), t.max()
    return (t - lo) / (hi - lo)


def disparity_layout(rng: np.random.Generator, H: int, W: int, n_seg: int,
                     d_lo: float, d_hi: float, slanted: bool,
                     gmax: float = 0.1) -> np.ndarray:
    """Voronoi partition into `n_seg` planar segments.

    Fronto-parallel segments get a constant disparity drawn from U[d_lo, d_hi];
    slanted ones d0 + gx (x - xc) + gy (y - yc) with |g| <= gmax, clipped to
    [d_lo, d_hi].
    """
    sy = rng.random(n_seg) * H
    sx = rng.random(n_seg) * W
    d0 = d_lo + rng.random(n_seg) * (d_hi - d_lo)
    gx = (rng.random(n_seg) * 2 - 1) * gmax
    gy = (rng.random(n_seg) * 2 - 1) * gmax
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    best = np.full((H, W), np.inf)
    label = np.zeros((H, W), dtype=np.int32)
    for s in range(n_seg):
        dist = (yy - sy[s]) ** 2 + (xx - sx[s]) ** 2
        m = dist < best
        best[m] = dist[m]
        label[m] = s
    if slanted:
        d = d0[label] + gx[label] * (xx - sx[label]) + gy[label] * (yy - sy[label])
        d = np.clip(d, d_lo, d_hi)
    else:
        d = d0[label].copy()
    return d


def warp_left_to_right(left: np.ndarray, disp: np.ndarray, fill: np.ndarray):
    """Forward-splat the left view to the right view at column round(x - d).

    A z-buffer keeps the largest disparity (the nearest surface) when several left
    pixels land on one right pixel.  Right pixels that receive nothing keep the
    `fill` texture.  Returns (right, nonocc) where nonocc marks the left pixels
    whose splat survived inside the image.
    """
    H, W = left.shape
    yy, xx = np.mgrid[0:H, 0:W]
    xr = np.rint(xx - disp).astype(np.int64)
    inb = (xr >= 0) & (xr < W)
    zbuf = np.full((H, W), -np.inf)
    np.maximum.at(zbuf, (yy[inb], xr[inb]), disp[inb])
    win = np.zeros((H, W), dtype=bool)
    win[inb] = disp[inb] == zbuf[yy[inb], xr[inb]]
    right = fill.copy()
    right[yy[win], xr[win]] = left[yy[win], xx[win]]
    return right, win


def make_pair(seed: int, H: int, W: int, n_seg: int, d_lo: float, d_hi: float,
              slanted: bool, gain: float = 1.0, offset: float = 0.0,
              sigma: float = 0.0, dtype: str = "u8") -> StereoPair:
    """One seeded pair.  `offset` and `sigma` are in the output intensity scale
    (0..255 for "u8", 0..1 for "f32")."""
    rng = np.random.Generator(np.random.PCG64(seed))
    scale = 255.0 if dtype == "u8" else 1.0
    left = texture(rng, H, W) * scale
    fill = texture(rng, H, W) * scale
    if dtype == "u8":
        left = np.rint(left)
        fill = np.rint(fill)
    disp = disparity_layout(rng, H, W, n_seg, d_lo, d_hi, slanted)
    right, nonocc = warp_left_to_right(left, disp, fill)
    right = gain * right + offset
    if sigma > 0:
        right = right + rng.normal(0.0, sigma, size=(H, W))
    right = np.clip(right, 0.0, scale)
    if dtype == "u8":
        left_o = left.astype(np.uint8)
        right_o = np.rint(right).astype(np.uint8)
    else:
        left_o = left.astype(np.float32)
        right_o = right.astype(np.float32)
    return StereoPair(left_o, right_o, disp, nonocc, seed)


# ---------------------------------------------------------------------------
# The five workloads.  Numbers marked "reading" are not fixed by the workload
# statements and were chosen once, for every consumer alike.
# ---------------------------------------------------------------------------

def workload(name: str, index: int = 0):
    """Return (pair, MatchConfig) for a named single-pair workload.

    small320  : 320x240 u8, 4 fronto segments d in [4,60], noise 2;
                K=3, 7x7, D=64, r=2.
    mid1436   : 1436x992 u8, 8 slanted segments d in [10,250], gain 0.9,
                offset +8, noise 4; K=4, 9x9, D=256, r=2.
    diff960   : pair `index` (seed index) of 960x540 f32, 6 slanted segments
                d in [4,115] (reading), noise 2/255; K=4, 7x7, D=128, r=2,
                soft r_s=3, tau=0.05.
    hires2880 : pair `index` of 2880x1988 f32, 8 slanted d in [20,360] (reading),
                gain 0.8, offset 10/255, noise 8/255; K=5, 11x11, D=400, r=3,
                soft r_s=3, tau=0.05.
    """
    if name == "small320":
        p = make_pair(0, 240, 320, 4, 4, 60, False, 1.0, 0.0, 2.0, "u8")
        return p, MatchConfig(240, 320, 64, 3, 3, 2, "u8")
    if name == "mid1436":
        p = make_pair(0, 992, 1436, 8, 10, 250, True, 0.9, 8.0, 4.0, "u8")
        return p, MatchConfig(992, 1436, 256, 4, 4, 2, "u8")
    if name == "diff960":
        p = make_pair(index, 540, 960, 6, 4, 115, True, 1.0, 0.0, 2.0 / 255, "f32")
        return p, MatchConfig(540, 960, 128, 4, 3, 2, "f32", soft_radius=3, tau=0.05)
    if name == "hires2880":
        p = make_pair(index, 1988, 2880, 8, 20, 360, True, 0.8, 10.0 / 255, 8.0 / 255, "f32")
        return p, MatchConfig(1988, 2880, 400, 5, 5, 3, "f32", soft_radius=3, tau=0.05)
    raise KeyError(name)


def batch_shapes(n_pairs: int = 32, shape_seed: int = 1000):
    """Shapes and ranges of the uneven batch: W ~ U{640..2880},
    H ~ U{480..1988}, D ~ U{64..400}, drawn from one seed."""
    rng = np.random.Generator(np.random.PCG64(shape_seed))
    W = rng.integers(640, 2881, size=n_pairs)
    H = rng.integers(480, 1989, size=n_pairs)
    D = rng.integers(64, 401, size=n_pairs)
    return [(int(h), int(w), int(d)) for h, w, d in zip(H, W, D)]


def batch_workload(n_pairs: int = 32, shape_seed: int = 1000,
                   only: Optional[List[int]] = None, workers: int = 1):
    """The uneven batch: pair i uses seed i, u8, 8 slanted segments with
    d in [0.05 D, 0.9 D], noise 2; 9x9, r=2, K = auto_levels(D).  Every pair has
    its own generator, so `workers` threads give the same pairs."""
    todo = [(i, H, W, D) for i, (H, W, D) in enumerate(batch_shapes(n_pairs, shape_seed))
            if only is None or i in only]

    def one(t):
        i, H, W, D = t
        p = make_pair(i, H, W, 8, 0.05 * D, 0.9 * D, True, 1.0, 0.0, 2.0, "u8")
        return p, MatchConfig(H, W, D, auto_levels(D), 4, 2, "u8")

    if workers <= 1:
        return [one(t) for t in todo]
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(workers) as ex:
        return list(ex.map(one, todo))


def grad_seed(seed: int, H: int, W: int) -> np.ndarray:
    """Seeded upstream gradient dL/d(d_soft) for backward tests (float64)."""
    rng = np.random.Generator(np.random.PCG64(10_000 + seed))
    return rng.standard_normal((H, W))


def loss_mask(nonocc: np.ndarray, n: int, max_disp: int) -> np.ndarray:
    """Pixels that enter the masked mean-L1 training loss (the paper has no loss;
    this is the reading of the differentiable workloads): visible in the right
    view, the (2n+1)^2 window inside the image (n <= i <= H-1-n, n <= j <= W-1-n),
    and j >= n + D - 1, so that the right window of every candidate z <= D-1
    lies inside the image too (a fixed sufficient condition: no loss pixel
    reaches a clamped read, whatever its candidate interval)."""
    H, W = nonocc.shape
    m = np.asarray(nonocc, dtype=bool).copy()
    m[:n, :] = False
    m[max(H - n, 0):, :] = False
    m[:, :min(W, n + max_disp - 1)] = False
    m[:, max(W - n, 0):] = False
    return m


def level_sizes(H: int, W: int, K: int):
    """(H_k, W_k) for k = 0..K-1 with ceil halving."""
    out = [(H, W)]
    for _ in range(K - 1):
        h, w = out[-1]
        out.append(((h + 1) // 2, (w + 1) // 2))
    return out


def level_range(D: int, k: int) -> int:
    """D_k = ceil(D / 2^k): candidate count at level k."""
    return -(-D // (1 << k))


def expected_evals(cfg: MatchConfig) -> int:
    """Upper bound on ZNCC evaluations of one hierarchical pass (no clipping):
    sum over levels of H_k W_k x candidates per pixel."""
    sizes = level_sizes(cfg.height, cfg.width, cfg.levels)
    tot = 0
    for k, (h, w) in enumerate(sizes):
        if k == cfg.levels - 1:
            tot += h * w * level_range(cfg.max_disp, k)
        elif k == 0 and cfg.soft_radius > 0:
            tot += h * w * (2 * cfg.soft_radius + 1)
        else:
            tot += h * w * (2 * cfg.refine_radius + 1)
    return tot

