"""FP64 CPU oracle for the hierarchical ZNCC block-matching hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  The product library shares no code
with it and never calls it.

The arithmetic lives in `msibm_oracle.c` (plain C, double precision, direct loops);
this module compiles it with gcc, loads it with ctypes, and composes the per-step
functions into the method's steps in the paper's order (Section III):

  1. a K-level Gaussian pyramid of both views;
  2. a full winner-take-all ZNCC search at the coarsest level (Eqs. 3-4);
  3. for each finer level, a search restricted to +-r around the doubled,
     nearest-neighbour-upsampled coarser map (Eqs. 8-9, first branch).

Optional steps of the paper: the confidence gating (the full search where the
bicubic-upsampled coarser cost is low, Eqs. 8-9 second branch; the re-pick of
low-cost pixels by the neighbourhood-averaged DSI, Eqs. 5-7), the selective
median filter (Eq. 10) and matching on a blurred level 0.

Plus the differentiable finest level (soft-argmax) and its gradient, which the
paper does not have.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "msibm_oracle.c")
_LIB = os.path.join(_HERE, "libmsibm_oracle.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I16 = ctypes.POINTER(ctypes.c_int16)
_U8 = ctypes.POINTER(ctypes.c_uint8)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP).  Returns the library path."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        c_int, c_double = ctypes.c_int, ctypes.c_double
        lib.orc_reduce.argtypes = [_D, c_int, c_int, _D]
        lib.orc_reduce.restype = None
        lib.orc_reduce_adjoint.argtypes = [_D, c_int, c_int, _D]
        lib.orc_reduce_adjoint.restype = None
        lib.orc_blur.argtypes = [_D, c_int, c_int, _D]
        lib.orc_blur.restype = None
        lib.orc_median.argtypes = [_I16, _D, c_int, c_int, c_double, _I16]
        lib.orc_median.restype = None
        lib.orc_bicubic_up.argtypes = [_D, c_int, c_int, c_int, c_int, c_double, _D]
        lib.orc_bicubic_up.restype = None
        lib.orc_match_gated.argtypes = [_D, _D, c_int, c_int, c_int, c_int, _I16, _D, c_int, c_int,
                                        c_int, c_double, c_double, _I16, _D, _D, _U8]
        lib.orc_match_gated.restype = None
        lib.orc_aggregate.argtypes = [_D, _D, c_int, c_int, c_int, c_int, _I16, _D, c_double,
                                      c_double, _I16, _D, _D]
        lib.orc_aggregate.restype = None
        _I32 = ctypes.POINTER(ctypes.c_int32)
        lib.orc_aggregate_pixels.argtypes = [_D, _D, c_int, c_int, c_int, c_int, _I16, _D, c_double,
                                             c_double, _I32, _I32, c_int, _I16, _D, _D]
        lib.orc_aggregate_pixels.restype = None
        lib.orc_avg_score_many.argtypes = [_D, _D, c_int, c_int, c_int, c_double, _I32, _I32, _I32, c_int, _D]
        lib.orc_avg_score_many.restype = None
        lib.orc_zncc.argtypes = [_D, _D, c_int, c_int, c_int, c_int, c_int, c_int, c_double]
        lib.orc_zncc.restype = c_double
        lib.orc_match_level.argtypes = [_D, _D, c_int, c_int, c_int, c_int, _I16, c_int, c_int,
                                        c_int, c_double, _I16, _D, _D]
        lib.orc_match_level.restype = None
        lib.orc_soft_level0.argtypes = [_D, _D, c_int, c_int, c_int, c_int, _I16, c_int, c_int,
                                        c_int, c_double, c_double, _D, _I16, _D, _D]
        lib.orc_soft_level0.restype = None
        lib.orc_backward.argtypes = [_D, _D, c_int, c_int, c_int, c_int, _I16, c_int, c_int,
                                     c_int, c_double, c_double, _D, c_int, c_int, _D, _D]
        lib.orc_backward.restype = None
        _I32P = ctypes.POINTER(ctypes.c_int32)
        lib.orc_zncc_many.argtypes = [_D, _D, c_int, c_int, c_int, c_double, _I32P, _I32P, _I32P,
                                      c_int, _D]
        lib.orc_zncc_many.restype = None
        lib.orc_match_pixels.argtypes = [_D, _D, c_int, c_int, c_int, c_int, _I16, c_int, c_int,
                                         c_int, c_double, _I32P, _I32P, c_int, _I16, _D, _D]
        lib.orc_match_pixels.restype = None
        _lib = lib
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a, t):
    return a.ctypes.data_as(t)


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops from now on (for timing)."""
    lib = _load()
    lib.orc_set_threads.argtypes = [ctypes.c_int]
    lib.orc_set_threads.restype = None
    lib.orc_set_threads(int(n))


def num_threads() -> int:
    """OpenMP threads the oracle will use (OMP_NUM_THREADS, else the CPU count)."""
    v = os.environ.get("OMP_NUM_THREADS")
    return int(v) if v else (os.cpu_count() or 1)


# --------------------------------------------------------------------------- steps

def reduce(img: np.ndarray) -> np.ndarray:
    """One pyramid step: 5x5 binomial blur, clamp-to-edge, keep even samples."""
    x = _f64(img)
    H, W = x.shape
    out = np.empty(((H + 1) // 2, (W + 1) // 2), dtype=np.float64)
    _load().orc_reduce(_p(x, _D), H, W, _p(out, _D))
    return out


def blur(img: np.ndarray) -> np.ndarray:
    """The pyramid's 5x5 binomial blur at every pixel, clamp-to-edge (the blur of
    the original image that Section IV credits for robustness to noise)."""
    x = _f64(img)
    H, W = x.shape
    out = np.empty((H, W), dtype=np.float64)
    _load().orc_blur(_p(x, _D), H, W, _p(out, _D))
    return out


def reduce_adjoint(G: np.ndarray, H: int, W: int) -> np.ndarray:
    """The transpose of reduce(): an H x W gradient from the ceil(H/2) x ceil(W/2)
    gradient of the reduced image."""
    GG = _f64(G)
    assert GG.shape == ((H + 1) // 2, (W + 1) // 2)
    out = np.empty((H, W), dtype=np.float64)
    _load().orc_reduce_adjoint(_p(GG, _D), H, W, _p(out, _D))
    return out


def pyramid(img: np.ndarray, K: int) -> List[np.ndarray]:
    """Levels 0..K-1; level 0 is the input converted to float64."""
    levels = [_f64(img)]
    for _ in range(K - 1):
        levels.append(reduce(levels[-1]))
    return levels


def level_range(D: int, k: int) -> int:
    """D_k = ceil(D / 2^k) candidates at level k (reading of d_max^k = D_max/2^k)."""
    return -(-D // (1 << k))


def zncc(L: np.ndarray, R: np.ndarray, n: int, i: int, j: int, z: int, eps: float) -> float:
    """Score of left pixel (i, j) against right pixel (i, j - z) (Eqs. 1-2)."""
    L = _f64(L)
    R = _f64(R)
    H, W = L.shape
    return _load().orc_zncc(_p(L, _D), _p(R, _D), H, W, n, i, j, z, eps)


def zncc_many(L: np.ndarray, R: np.ndarray, n: int, ii, jj, zz, eps: float) -> np.ndarray:
    """Scores at arrays of (i, j, z) triples."""
    L = _f64(L)
    R = _f64(R)
    H, W = L.shape
    ii = np.ascontiguousarray(ii, dtype=np.int32)
    jj = np.ascontiguousarray(jj, dtype=np.int32)
    zz = np.ascontiguousarray(zz, dtype=np.int32)
    assert ii.shape == jj.shape == zz.shape
    out = np.empty(ii.shape, dtype=np.float64)
    I32P = ctypes.POINTER(ctypes.c_int32)
    _load().orc_zncc_many(_p(L, _D), _p(R, _D), H, W, n, eps, _p(ii, I32P), _p(jj, I32P),
                          _p(zz, I32P), ii.size, _p(out, _D))
    return out


def match_pixels(L: np.ndarray, R: np.ndarray, n: int, Dk: int, coarse: Optional[np.ndarray],
                 r: int, eps: float, ii, jj):
    """match_level evaluated only at the pixels (ii[q], jj[q]); returns (d, C, C2)."""
    L = _f64(L)
    R = _f64(R)
    H, W = L.shape
    ii = np.ascontiguousarray(ii, dtype=np.int32)
    jj = np.ascontiguousarray(jj, dtype=np.int32)
    cnt = ii.size
    d = np.empty(cnt, dtype=np.int16)
    C = np.empty(cnt, dtype=np.float64)
    C2 = np.empty(cnt, dtype=np.float64)
    if coarse is not None:
        cz = np.ascontiguousarray(coarse, dtype=np.int16)
        Hc, Wc = cz.shape
        assert Hc == (H + 1) // 2 and Wc == (W + 1) // 2, "prior shape"
        cptr = _p(cz, _I16)
    else:
        cz, Hc, Wc, cptr = None, 0, 0, None
    I32P = ctypes.POINTER(ctypes.c_int32)
    _load().orc_match_pixels(_p(L, _D), _p(R, _D), H, W, n, Dk, cptr, Hc, Wc, r, eps,
                             _p(ii, I32P), _p(jj, I32P), cnt, _p(d, _I16), _p(C, _D), _p(C2, _D))
    return d, C, C2


def match_level(L: np.ndarray, R: np.ndarray, n: int, Dk: int,
                coarse: Optional[np.ndarray], r: int, eps: float):
    """Winner-take-all of one level.  `coarse` = level k+1 map (int16) for the
    restricted search, or None for a full search.  Returns (d, C, C2)."""
    L = _f64(L)
    R = _f64(R)
    H, W = L.shape
    d = np.empty((H, W), dtype=np.int16)
    C = np.empty((H, W), dtype=np.float64)
    C2 = np.empty((H, W), dtype=np.float64)
    if coarse is not None:
        cz = np.ascontiguousarray(coarse, dtype=np.int16)
        Hc, Wc = cz.shape
        assert Hc == (H + 1) // 2 and Wc == (W + 1) // 2, "prior shape"
        cptr = _p(cz, _I16)
    else:
        cz, Hc, Wc, cptr = None, 0, 0, None
    _load().orc_match_level(_p(L, _D), _p(R, _D), H, W, n, Dk, cptr, Hc, Wc, r, eps,
                            _p(d, _I16), _p(C, _D), _p(C2, _D))
    return d, C, C2


def median_filter(d: np.ndarray, C: np.ndarray, alpha: float) -> np.ndarray:
    """Selective median filtering (Eq. 10): pixels with C <= alpha take the lower
    median disparity of the good (C > alpha) pixels of their 5x5 patch."""
    dd = np.ascontiguousarray(d, dtype=np.int16)
    CC = _f64(C)
    H, W = dd.shape
    assert CC.shape == dd.shape
    out = np.empty_like(dd)
    _load().orc_median(_p(dd, _I16), _p(CC, _D), H, W, float(alpha), _p(out, _I16))
    return out


def bicubic_up(Cc: np.ndarray, H: int, W: int, a: float = -0.5) -> np.ndarray:
    """A coarse cost map doubled to H x W by bicubic interpolation (Section III.C)."""
    CC = _f64(Cc)
    Hc, Wc = CC.shape
    assert Hc <= H <= 2 * Hc and Wc <= W <= 2 * Wc
    out = np.empty((H, W), dtype=np.float64)
    _load().orc_bicubic_up(_p(CC, _D), Hc, Wc, H, W, float(a), _p(out, _D))
    return out


def match_gated(L: np.ndarray, R: np.ndarray, n: int, Dk: int, coarse: np.ndarray,
                coarse_cost: np.ndarray, r: int, beta: float, eps: float):
    """Eqs. 8-9: restricted search where the upsampled coarse cost exceeds beta,
    full search elsewhere.  Returns (d', C', C2', full mask)."""
    L = _f64(L)
    R = _f64(R)
    H, W = L.shape
    cz = np.ascontiguousarray(coarse, dtype=np.int16)
    cc = _f64(coarse_cost)
    Hc, Wc = cz.shape
    assert Hc == (H + 1) // 2 and Wc == (W + 1) // 2 and cc.shape == cz.shape, "prior shape"
    d = np.empty((H, W), dtype=np.int16)
    C = np.empty((H, W), dtype=np.float64)
    C2 = np.empty((H, W), dtype=np.float64)
    full = np.empty((H, W), dtype=np.uint8)
    _load().orc_match_gated(_p(L, _D), _p(R, _D), H, W, n, Dk, _p(cz, _I16), _p(cc, _D), Hc, Wc, r,
                            float(beta), eps, _p(d, _I16), _p(C, _D), _p(C2, _D), _p(full, _U8))
    return d, C, C2, full.astype(bool)


def aggregate(L: np.ndarray, R: np.ndarray, n: int, Dk: int, d1: np.ndarray, C1: np.ndarray,
              alpha: float, eps: float):
    """Eqs. 5-7: pixels with C' <= alpha re-picked by the 5x5-averaged DSI.
    Returns (d, C, C2), C2 the runner-up averaged score of a re-picked pixel."""
    L = _f64(L)
    R = _f64(R)
    H, W = L.shape
    dd = np.ascontiguousarray(d1, dtype=np.int16)
    CC = _f64(C1)
    assert dd.shape == (H, W) and CC.shape == (H, W)
    d = np.empty((H, W), dtype=np.int16)
    C = np.empty((H, W), dtype=np.float64)
    C2 = np.empty((H, W), dtype=np.float64)
    _load().orc_aggregate(_p(L, _D), _p(R, _D), H, W, n, Dk, _p(dd, _I16), _p(CC, _D), float(alpha),
                          eps, _p(d, _I16), _p(C, _D), _p(C2, _D))
    return d, C, C2


def aggregate_pixels(L: np.ndarray, R: np.ndarray, n: int, Dk: int, d1: np.ndarray, C1: np.ndarray,
                     alpha: float, eps: float, ii, jj):
    """aggregate() at the listed pixels only: (d, C, C2) per pixel."""
    L = _f64(L)
    R = _f64(R)
    H, W = L.shape
    dd = np.ascontiguousarray(d1, dtype=np.int16)
    CC = _f64(C1)
    i32 = np.ascontiguousarray(ii, dtype=np.int32)
    j32 = np.ascontiguousarray(jj, dtype=np.int32)
    m = len(i32)
    d = np.empty(m, dtype=np.int16)
    C = np.empty(m, dtype=np.float64)
    C2 = np.empty(m, dtype=np.float64)
    P32 = ctypes.POINTER(ctypes.c_int32)
    _load().orc_aggregate_pixels(_p(L, _D), _p(R, _D), H, W, n, Dk, _p(dd, _I16), _p(CC, _D), float(alpha),
                                 eps, _p(i32, P32), _p(j32, P32), m, _p(d, _I16), _p(C, _D), _p(C2, _D))
    return d, C, C2


def avg_score_many(L: np.ndarray, R: np.ndarray, n: int, ii, jj, zz, eps: float) -> np.ndarray:
    """The 5x5-averaged score (Eq. 5) at (i, j, z) triples."""
    L = _f64(L)
    R = _f64(R)
    H, W = L.shape
    i32 = np.ascontiguousarray(ii, dtype=np.int32)
    j32 = np.ascontiguousarray(jj, dtype=np.int32)
    z32 = np.ascontiguousarray(zz, dtype=np.int32)
    out = np.empty(len(i32), dtype=np.float64)
    P32 = ctypes.POINTER(ctypes.c_int32)
    _load().orc_avg_score_many(_p(L, _D), _p(R, _D), H, W, n, eps, _p(i32, P32), _p(j32, P32), _p(z32, P32),
                               len(i32), _p(out, _D))
    return out


def disparity(left: np.ndarray, right: np.ndarray, D: int, K: int, n, r: int,
              eps: float, priors: Optional[List[Optional[np.ndarray]]] = None, preblur: bool = False,
              median_alpha: Optional[float] = None, gate: Optional[tuple] = None):
    """The hierarchical forward pass (Section III, hot path).

    n is the window half-width of every level, or a sequence of per-level
    half-widths (level 0 first, its last entry for the levels past its end): the
    block size that Section III shrinks level by level.  Returns a list, index
    k = level, of (d_k, C_k, C2_k).  `priors[k]`, if given, replaces the map that
    feeds level k (teacher forcing: the level-(k+1) map used as the prior of
    level k).  With `preblur`, level 0 is matched on the blurred input (the
    pyramid is still built from the input itself).  With `median_alpha`, every
    level's map goes through the selective median filter (Eq. 10) before it is
    returned and propagated; C is the matched cost before the filter.  With
    `gate` = (alpha, beta), the paper's confidence gating: every level below the
    coarsest takes the full search where the bicubic-upsampled coarser cost is at
    most beta (Eqs. 8-9), and every level re-picks its pixels with cost at most
    alpha by the neighbourhood-averaged DSI (Eqs. 5-7); the cost propagated and
    returned is that of Eq. 7."""
    def nk(k):
        return n if isinstance(n, (int, np.integer)) else n[min(k, len(n) - 1)]
    PL = pyramid(left, K)
    PR = pyramid(right, K)
    if preblur:
        PL[0] = blur(left)
        PR[0] = blur(right)
    def filtered(res):
        if median_alpha is None:
            return res
        return (median_filter(res[0], res[1], median_alpha),) + tuple(res[1:])
    def refined(k, res):
        if gate is None:
            return res
        return aggregate(PL[k], PR[k], nk(k), level_range(D, k), res[0], res[1], gate[0], eps)
    out: List = [None] * K
    kc = K - 1
    out[kc] = filtered(refined(kc, match_level(PL[kc], PR[kc], nk(kc), level_range(D, kc), None, r, eps)))
    for k in range(K - 2, -1, -1):
        prior = out[k + 1][0]
        if priors is not None and priors[k] is not None:
            prior = priors[k]
        if gate is None:
            res = match_level(PL[k], PR[k], nk(k), level_range(D, k), prior, r, eps)
        else:
            res = match_gated(PL[k], PR[k], nk(k), level_range(D, k), prior, out[k + 1][1], r, gate[1],
                              eps)[:3]
        out[k] = filtered(refined(k, res))
    return out


def flat_bm(left: np.ndarray, right: np.ndarray, D: int, n: int, eps: float):
    """Standard block matching: a full search at full resolution."""
    return match_level(_f64(left), _f64(right), n, D, None, 0, eps)


def soft_level0(L0: np.ndarray, R0: np.ndarray, n: int, D: int, coarse1: np.ndarray,
                rs: int, tau: float, eps: float):
    """Soft-argmax at level 0 over the radius-rs interval around the doubled
    level-1 map.  Returns (d_soft, d_hard, C, C2)."""
    assert 0 <= rs < 500
    L0 = _f64(L0)
    R0 = _f64(R0)
    H, W = L0.shape
    cz = np.ascontiguousarray(coarse1, dtype=np.int16)
    Hc, Wc = cz.shape
    assert Hc == (H + 1) // 2 and Wc == (W + 1) // 2, "prior shape"
    ds = np.empty((H, W), dtype=np.float64)
    dh = np.empty((H, W), dtype=np.int16)
    C = np.empty((H, W), dtype=np.float64)
    C2 = np.empty((H, W), dtype=np.float64)
    _load().orc_soft_level0(_p(L0, _D), _p(R0, _D), H, W, n, D, _p(cz, _I16), Hc, Wc, rs, tau,
                            eps, _p(ds, _D), _p(dh, _I16), _p(C, _D), _p(C2, _D))
    return ds, dh, C, C2


def backward(L0: np.ndarray, R0: np.ndarray, n: int, D: int, coarse1: np.ndarray, rs: int,
             tau: float, eps: float, gd: np.ndarray, rows: Optional[tuple] = None):
    """(dL/dL0, dL/dR0) for L = sum gd * d_soft with the level-1 prior frozen.
    `rows` = (i0, i1) restricts the contributing source pixels to those rows."""
    assert 0 <= rs < 500
    L0 = _f64(L0)
    R0 = _f64(R0)
    g = _f64(gd)
    H, W = L0.shape
    cz = np.ascontiguousarray(coarse1, dtype=np.int16)
    Hc, Wc = cz.shape
    assert Hc == (H + 1) // 2 and Wc == (W + 1) // 2, "prior shape"
    i0, i1 = rows if rows is not None else (0, H)
    gL = np.empty((H, W), dtype=np.float64)
    gR = np.empty((H, W), dtype=np.float64)
    _load().orc_backward(_p(L0, _D), _p(R0, _D), H, W, n, D, _p(cz, _I16), Hc, Wc, rs, tau, eps,
                         _p(g, _D), int(i0), int(i1), _p(gL, _D), _p(gR, _D))
    return gL, gR


def l1_loss(dsoft: np.ndarray, dgt: np.ndarray, mask: np.ndarray):
    """Masked mean absolute error and its gradient with respect to d_soft
    (sign(0) = 0)."""
    cnt = int(mask.sum())
    diff = dsoft - dgt
    loss = float(np.abs(diff[mask]).sum() / max(cnt, 1))
    g = np.where(mask, np.sign(diff), 0.0) / max(cnt, 1)
    return loss, g


def soft_levels(left: np.ndarray, right: np.ndarray, D: int, K: int, n: int, rs: int, tau: float,
                eps: float):
    """Soft output at every level below the coarsest (an extension of the
    paper): the coarsest level is the hard full search; every finer level k takes
    the soft-argmax over the radius-rs interval around the doubled hard map of
    level k+1, and its hard winner over the same interval is the next level's
    prior.  Returns a list, index k = level: (d_soft, d_hard, C, C2) for k < K-1,
    (None, d, C, C2) at the coarsest level."""
    PL = pyramid(left, K)
    PR = pyramid(right, K)
    out: List = [None] * K
    d, C, C2 = match_level(PL[K - 1], PR[K - 1], n, level_range(D, K - 1), None, 0, eps)
    out[K - 1] = (None, d, C, C2)
    for k in range(K - 2, -1, -1):
        out[k] = soft_level0(PL[k], PR[k], n, level_range(D, k), out[k + 1][1], rs, tau, eps)
    return out


def backward_levels(left: np.ndarray, right: np.ndarray, D: int, K: int, n: int, rs: int, tau: float,
                    eps: float, maps: List[np.ndarray], grads: List[Optional[np.ndarray]]):
    """Gradient of sum_k sum g_k d_soft^k with respect to both level-0 images,
    every level's prior (maps[k + 1]) held fixed: each level's gradient with
    respect to its own pyramid images (the soft level's backward), carried down
    by the adjoint of the reduce (the chain rule through the pyramid)."""
    PL = pyramid(left, K)
    PR = pyramid(right, K)
    gL = np.zeros_like(PL[K - 2]) if K >= 2 else None
    gR = np.zeros_like(PR[K - 2]) if K >= 2 else None
    for k in range(K - 2, -1, -1):
        if gL.shape != PL[k].shape:
            gL = reduce_adjoint(gL, *PL[k].shape)
            gR = reduce_adjoint(gR, *PR[k].shape)
        if grads[k] is not None:
            a, b = backward(PL[k], PR[k], n, level_range(D, k), maps[k + 1], rs, tau, eps, grads[k])
            gL = gL + a
            gR = gR + b
    return gL, gR
