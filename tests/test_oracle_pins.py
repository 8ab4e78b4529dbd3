"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these re-types the oracle's formulas: each check uses a library routine
(numpy's Pearson correlation, scipy's correlation filter), a closed form, an
invariant or brute force on tiny inputs, so a dropped term, a wrong sign or index,
or a transposed operand in the oracle fails at least one of them.
"""
import numpy as np
import pytest
from scipy import ndimage

import oracle
from paper_1901_09593_amd import synth


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _window(img, i, j, n):
    """Clamp-to-edge (2n+1)^2 window via numpy's edge padding."""
    p = np.pad(img, n, mode="edge")
    return p[i:i + 2 * n + 1, j:j + 2 * n + 1]


def _pearson(a, b):
    return float(np.corrcoef(a.ravel(), b.ravel())[0, 1])


# ---------------------------------------------------------------- ZNCC (Eq. 2)

@pytest.mark.parametrize("n", [1, 2, 3])
def test_zncc_equals_pearson_interior_and_border(n):
    rng = _rng(1)
    L = rng.random((15, 19))
    R = rng.random((15, 19))
    for (i, j, z) in [(7, 9, 0), (7, 9, 3), (0, 0, 0), (14, 18, 5), (3, 4, 4), (10, 2, 2),
                      (1, 18, 18)]:
        ref = _pearson(_window(L, i, j, n), _window(R, i, j - z, n))
        got = oracle.zncc(L, R, n, i, j, z, 1e-12)
        assert abs(got - ref) < 1e-12, (i, j, z, got, ref)


@pytest.mark.parametrize("a,b", [(2.5, 0.3), (-0.7, 4.0), (1e-3, -9.0)])
def test_zncc_linear_relation_closed_form(a, b):
    # R(y, x) = a L(y, x + z0) + b: the right window at (i, j - z0) is an affine
    # image of the left window at (i, j), so the score is exactly sign(a).
    rng = _rng(2)
    z0, n = 4, 2
    T = rng.random((12, 30))
    L = T[:, :26]
    R = a * T[:, z0:z0 + 26] + b
    for (i, j) in [(5, 10), (6, 20), (2, 13)]:
        got = oracle.zncc(L, R, n, i, j, z0, 0.0)
        assert abs(got - np.sign(a)) < 1e-12
        other = oracle.zncc(L, R, n, i, j, z0 + 1, 0.0)
        assert abs(other) < 0.999  # the wrong shift does not reach the bound


def test_zncc_gain_offset_invariance_and_bounds():
    rng = _rng(3)
    L = rng.random((13, 17))
    R = rng.random((13, 17))
    for (i, j, z) in [(6, 8, 2), (0, 16, 7), (12, 5, 0)]:
        base = oracle.zncc(L, R, 2, i, j, z, 1e-12)
        assert -1.0 <= base <= 1.0
        assert abs(oracle.zncc(L, 3.0 * R + 7.0, 2, i, j, z, 1e-12) - base) < 1e-12
        assert abs(oracle.zncc(0.25 * L - 1.0, R, 2, i, j, z, 1e-12) - base) < 1e-12
        assert abs(oracle.zncc(L, -2.0 * R, 2, i, j, z, 1e-12) + base) < 1e-12


def test_zncc_identical_windows_and_flat_windows():
    rng = _rng(4)
    L = rng.random((9, 9))
    assert abs(oracle.zncc(L, L, 2, 4, 4, 0, 1e-12) - 1.0) < 1e-12
    flat = np.full((9, 9), 0.5)
    assert oracle.zncc(L, flat, 2, 4, 4, 0, 1e-12) == 0.0
    assert oracle.zncc(flat, L, 2, 4, 4, 0, 1e-12) == 0.0
    # variance floor: a window with variance below eps scores 0, above it does not
    tiny = 0.5 + 1e-4 * rng.standard_normal((9, 9))
    var = np.var(_window(tiny, 4, 4, 2))
    assert oracle.zncc(L, tiny, 2, 4, 4, 0, var * 1.01) == 0.0
    assert oracle.zncc(L, tiny, 2, 4, 4, 0, var * 0.99) != 0.0


# ----------------------------------------------------------- pyramid (Sec. III)

@pytest.mark.parametrize("shape", [(16, 16), (17, 23), (5, 3), (1, 7)])
def test_reduce_equals_scipy_binomial_filter(shape):
    rng = _rng(5)
    img = rng.random(shape) * 255
    w = np.array([1, 4, 6, 4, 1], dtype=np.float64) / 16
    ref = ndimage.correlate(img, np.outer(w, w), mode="nearest")[::2, ::2]
    got = oracle.reduce(img)
    assert got.shape == ((shape[0] + 1) // 2, (shape[1] + 1) // 2)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)


def test_reduce_constant_and_linear():
    assert np.all(oracle.reduce(np.full((11, 14), 37.0)) == 37.0)
    # the binomial kernel is symmetric with unit sum, so a linear image keeps its
    # value at the sampled positions away from the border
    yy, xx = np.mgrid[0:20, 0:24].astype(np.float64)
    img = 3.0 * xx - 2.0 * yy + 5.0
    out = oracle.reduce(img)
    inner = out[1:-1, 1:-1]
    ys, xs = np.mgrid[1:out.shape[0] - 1, 1:out.shape[1] - 1]
    np.testing.assert_allclose(inner, 3.0 * 2 * xs - 2.0 * 2 * ys + 5.0, atol=1e-12)


def test_pyramid_levels_and_sizes():
    img = _rng(6).integers(0, 256, size=(37, 50)).astype(np.uint8)
    lv = oracle.pyramid(img, 4)
    assert [l.shape for l in lv] == [(37, 50), (19, 25), (10, 13), (5, 7)]
    # uint8 input: level k values are multiples of 2^-8k (dyadic weights)
    for k in (1, 2):
        scaled = lv[k] * (1 << (8 * k))
        assert np.all(scaled == np.rint(scaled))


# ------------------------------------------------ winner-take-all (Eqs. 3-4, 8-9)

def _brute_level(L, R, n, Dk, coarse, r, eps):
    """Exhaustive search with Pearson scores from numpy; lowest z on ties."""
    H, W = L.shape
    d = np.zeros((H, W), dtype=np.int16)
    C = np.zeros((H, W))
    for i in range(H):
        for j in range(W):
            top = min(Dk - 1, j)
            if coarse is None:
                lo, hi = 0, top
            else:
                c = min(2 * int(coarse[i // 2, j // 2]), j)
                lo, hi = max(0, c - r), min(top, c + r)
            best, bz = -np.inf, lo
            for z in range(lo, hi + 1):
                lw = _window(L, i, j, n)
                rw = _window(R, i, j - z, n)
                if lw.var() <= eps or rw.var() <= eps:
                    s = 0.0
                else:
                    s = _pearson(lw, rw)
                if s > best:
                    best, bz = s, z
            d[i, j] = bz
            C[i, j] = best
    return d, C


@pytest.mark.parametrize("shape,n,D", [((12, 10), 1, 6), ((9, 17), 2, 5), ((7, 8), 1, 3)])
def test_full_search_brute_force(shape, n, D):
    rng = _rng(7)
    L = rng.integers(0, 256, size=shape).astype(np.float64)
    R = rng.integers(0, 256, size=shape).astype(np.float64)
    L[:3, :3] = 9.0  # a flat patch exercises the floor
    d, C, C2 = oracle.match_level(L, R, n, D, None, 0, 0.065)
    bd, bC = _brute_level(L, R, n, D, None, 0, 0.065)
    assert np.array_equal(d, bd)
    np.testing.assert_allclose(C, bC, atol=1e-12)
    assert np.all(C >= C2)


@pytest.mark.parametrize("r", [0, 1, 2])
def test_restricted_search_brute_force(r):
    rng = _rng(8)
    H, W, D, n = 11, 14, 8, 1
    L = rng.random((H, W))
    R = rng.random((H, W))
    coarse = rng.integers(0, (D + 1) // 2, size=((H + 1) // 2, (W + 1) // 2)).astype(np.int16)
    d, C, _ = oracle.match_level(L, R, n, D, coarse, r, 1e-9)
    bd, bC = _brute_level(L, R, n, D, coarse, r, 1e-9)
    assert np.array_equal(d, bd)
    np.testing.assert_allclose(C, bC, atol=1e-12)


def test_ties_break_to_lowest_disparity():
    # a texture periodic in x with period p: the right view equals the left one,
    # so z = 0 and z = p tie at score 1 in the interior; the lowest must win
    p, n = 5, 2
    base = _rng(9).random((16, p))
    L = np.tile(base, (1, 8))
    d, C, C2 = oracle.match_level(L, L, n, 12, None, 0, 1e-12)
    inner = (slice(n, -n), slice(p + n, -n))
    assert np.all(d[inner] == 0)
    assert np.allclose(C[inner], 1.0) and np.allclose(C2[inner], 1.0)


def _shifted_pair(H, W, s, seed=10):
    T = synth.texture(_rng(seed), H, W + s) * 255
    return T[:, :W].copy(), T[:, s:s + W].copy()


@pytest.mark.parametrize("K,s", [(3, 8), (2, 6), (4, 16)])
def test_constant_shift_recovered_at_every_level(K, s):
    # R(y, x - s) = L(y, x); decimation commutes with shifts that are multiples of
    # 2^(K-1), so every level recovers s / 2^k away from the borders
    H, W, n, D = 64, 96, 2, 40
    L, R = _shifted_pair(H, W, s)
    out = oracle.disparity(L, R, D, K, n, 1, 0.065)
    for k in range(K):
        dk = out[k][0]
        m = 3 * (1 << (K - 1 - k)) + n + 3
        inner = dk[m:-m, s // (1 << k) + m:-m]
        assert np.all(inner == s >> k), (k, np.unique(inner))


def test_constant_shift_recovered_with_halving_windows():
    # Section III's block size halving per level (n = 4, 2, 1): the shift is still
    # recovered at every level, and the coarsest level's search is the flat
    # search of that level with its own window
    H, W, D, K, s = 64, 96, 40, 3, 8
    ns = [4, 2, 1]
    L, R = _shifted_pair(H, W, s, seed=5)
    out = oracle.disparity(L, R, D, K, ns, 1, 0.065)
    for k in range(K):
        dk = out[k][0]
        m = 3 * (1 << (K - 1 - k)) + ns[k] + 3
        inner = dk[m:-m, s // (1 << k) + m:-m]
        assert np.all(inner == s >> k), (k, np.unique(inner))
    top = oracle.flat_bm(oracle.pyramid(L, K)[K - 1], oracle.pyramid(R, K)[K - 1], oracle.level_range(D, K - 1),
                         ns[K - 1], 0.065)
    assert np.array_equal(top[0], out[K - 1][0])


def test_blur_pins():
    # kernel sums to 1 (a constant stays constant), an impulse spreads into the
    # outer product of the binomial weights, linear functions pass unchanged and
    # x^2 + y^2 gains the kernel's second moment (1 per axis) away from the borders
    w = np.array([1, 4, 6, 4, 1], dtype=np.float64) / 16
    assert np.array_equal(oracle.blur(np.full((9, 11), 37.0)), np.full((9, 11), 37.0))
    imp = np.zeros((11, 13))
    imp[5, 6] = 1.0
    b = oracle.blur(imp)
    assert np.allclose(b[3:8, 4:9], np.outer(w, w), atol=0, rtol=1e-15) and b.sum() == 1.0
    yy, xx = np.mgrid[0:20, 0:24].astype(np.float64)
    lin = oracle.blur(3 * xx - 2 * yy + 5)
    assert np.allclose(lin[2:-2, 2:-2], (3 * xx - 2 * yy + 5)[2:-2, 2:-2], atol=1e-12)
    quad = oracle.blur(xx ** 2 + yy ** 2)
    assert np.allclose(quad[2:-2, 2:-2], (xx ** 2 + yy ** 2 + 2)[2:-2, 2:-2], atol=1e-9)
    # one pyramid step is the blur kept at even rows and columns
    img = _rng(21).integers(0, 256, size=(17, 22)).astype(np.float64)
    assert np.array_equal(oracle.reduce(img), oracle.blur(img)[::2, ::2])


def test_preblur_matches_blurred_level_zero():
    # the pre-blur variant matches level 0 on the blurred images and leaves the
    # coarser levels alone
    p = synth.make_pair(6, 40, 72, 4, 2, 20, True, 1.0, 0.0, 2.0, "u8")
    a = oracle.disparity(p.left, p.right, 24, 2, 2, 2, 0.065)
    b = oracle.disparity(p.left, p.right, 24, 2, 2, 2, 0.065, preblur=True)
    assert np.array_equal(a[1][0], b[1][0])
    ref = oracle.match_level(oracle.blur(p.left), oracle.blur(p.right), 2, 24, a[1][0], 2, 0.065)
    assert np.array_equal(ref[0], b[0][0])


def test_selective_median_pins():
    rng = _rng(31)
    d = rng.integers(0, 40, size=(9, 12)).astype(np.int16)
    C = rng.uniform(-1, 1, size=(9, 12))
    # every pixel good (C > -2) or every pixel bad (no good neighbour): unchanged
    assert np.array_equal(oracle.median_filter(d, C, -2.0), d)
    assert np.array_equal(oracle.median_filter(d, C, 2.0), d)
    # a bad pixel among good ones takes the lower median of its good 5x5 patch,
    # read from the unfiltered map; good pixels keep their value
    C = np.full((9, 12), 0.95)
    C[4, 5] = C[4, 6] = 0.2       # two bad neighbours
    C[2, 3] = 0.5                  # a bad pixel inside the patch of (4, 5)
    out = oracle.median_filter(d, C, 0.9)
    good = C > 0.9
    for (i, j) in ((4, 5), (4, 6), (2, 3)):
        ys, xs = np.mgrid[max(0, i - 2):min(9, i + 3), max(0, j - 2):min(12, j + 3)]
        vals = np.sort(d[ys, xs][good[ys, xs]])
        assert out[i, j] == vals[(len(vals) - 1) // 2], (i, j)
    keep = np.ones_like(good)
    keep[4, 5] = keep[4, 6] = keep[2, 3] = False
    assert np.array_equal(out[keep], d[keep])
    # patches are clipped at the image: a corner pixel sees only its 3x3 in-image part
    C2 = np.full((9, 12), 0.95)
    C2[0, 0] = 0.0
    out2 = oracle.median_filter(d, C2, 0.9)
    vals = np.sort(np.delete(d[0:3, 0:3].ravel(), 0))
    assert out2[0, 0] == vals[(len(vals) - 1) // 2]


def test_median_in_the_hierarchy():
    # with the filter, each level's map is the filtered matching result and C is
    # the cost before filtering; a threshold below every score changes nothing
    p = synth.make_pair(7, 48, 80, 4, 2, 20, True, 1.0, 0.0, 6.0, "u8")
    a = oracle.disparity(p.left, p.right, 24, 2, 2, 2, 0.065)
    b = oracle.disparity(p.left, p.right, 24, 2, 2, 2, 0.065, median_alpha=-2.0)
    for k in range(2):
        assert np.array_equal(a[k][0], b[k][0])
    c = oracle.disparity(p.left, p.right, 24, 2, 2, 2, 0.065, median_alpha=0.9)
    top = oracle.median_filter(a[1][0], a[1][1], 0.9)
    assert np.array_equal(c[1][0], top) and np.array_equal(c[1][1], a[1][1])
    PL, PR = oracle.pyramid(p.left, 2), oracle.pyramid(p.right, 2)
    l0 = oracle.match_level(PL[0], PR[0], 2, 24, top, 2, 0.065)
    assert np.array_equal(c[0][0], oracle.median_filter(l0[0], l0[1], 0.9))


def test_odd_shift_recovered_at_level_zero():
    H, W, n, D = 48, 80, 2, 30
    L, R = _shifted_pair(H, W, 7, seed=11)
    out = oracle.disparity(L, R, D, 2, n, 2, 0.065)
    inner = out[0][0][8:-8, 7 + 8:-8]
    assert np.all(inner == 7)


def test_single_level_equals_flat_and_wide_refine_equals_flat():
    p = synth.make_pair(3, 40, 64, 3, 2, 14, True, 1.0, 0.0, 1.0, "u8")
    eps, n, D = 0.065, 2, 16
    flat = oracle.flat_bm(p.left, p.right, D, n, eps)
    one = oracle.disparity(p.left, p.right, D, 1, n, 2, eps)[0]
    assert np.array_equal(flat[0], one[0])
    # a refine radius covering every candidate makes level 0 a full search,
    # whatever the prior says
    rnd = _rng(12).integers(0, 8, size=(20, 32)).astype(np.int16)
    wide = oracle.disparity(p.left, p.right, D, 2, n, 2 * D, eps, priors=[rnd, None])[0]
    assert np.array_equal(flat[0], wide[0])
    np.testing.assert_allclose(flat[1], wide[1], atol=1e-12)


def test_disparity_invariant_to_right_gain_and_offset():
    p = synth.make_pair(4, 48, 72, 4, 2, 20, True, 1.0, 0.0, 2.0, "u8")
    L = p.left.astype(np.float64)
    R = p.right.astype(np.float64)
    a = oracle.disparity(L, R, 24, 3, 2, 2, 0.065)
    b = oracle.disparity(L, 0.8 * R + 11.0, 24, 3, 2, 2, 0.065 * 0.64)
    for k in range(3):
        gap = a[k][1] - a[k][2]
        same = (a[k][0] == b[k][0]) | (gap < 1e-9)
        assert same.all()


def test_prior_range_never_exceeds_level_range():
    # 2 d^{k+1} <= D_k - 1 whenever d^{k+1} <= D_{k+1} - 1
    for D in range(1, 1200):
        for k in range(0, 7):
            Dk, Dk1 = oracle.level_range(D, k), oracle.level_range(D, k + 1)
            assert 2 * (Dk1 - 1) <= Dk - 1


# --------------------------------------------------- soft-argmax and gradient

def _soft_case(seed=13, H=12, W=16, D=8):
    rng = _rng(seed)
    L = rng.random((H, W))
    R = rng.random((H, W))
    coarse = rng.integers(0, (D + 1) // 2, size=((H + 1) // 2, (W + 1) // 2)).astype(np.int16)
    return L, R, coarse


def test_soft_argmax_limits():
    L, R, coarse = _soft_case()
    n, D, rs = 1, 8, 2
    ds, dh, C, C2 = oracle.soft_level0(L, R, n, D, coarse, rs, 1e-4, 1e-9)
    sharp = (C - C2) > 0.01
    np.testing.assert_allclose(ds[sharp], dh[sharp], atol=1e-12)
    ds_hot, *_ = oracle.soft_level0(L, R, n, D, coarse, rs, 1e9, 1e-9)
    H, W = L.shape
    for i in range(H):
        for j in range(W):
            c = min(2 * int(coarse[i // 2, j // 2]), j)
            lo, hi = max(0, c - rs), min(D - 1, j, c + rs)
            assert abs(ds_hot[i, j] - 0.5 * (lo + hi)) < 1e-6
    one, *_ = oracle.soft_level0(L, R, n, 1, np.zeros_like(coarse), rs, 0.05, 1e-9)
    assert np.all(one == 0.0)


@pytest.mark.parametrize("n,rs", [(1, 2), (2, 1)])
def test_backward_matches_central_differences(n, rs):
    L, R, coarse = _soft_case(seed=14, H=10, W=13)
    D, tau, eps = 8, 0.3, 1e-12
    g = _rng(15).standard_normal(L.shape)
    gL, gR = oracle.backward(L, R, n, D, coarse, rs, tau, eps, g)

    def f(Lx, Rx):
        ds, *_ = oracle.soft_level0(Lx, Rx, n, D, coarse, rs, tau, eps)
        return float((g * ds).sum())

    h = 1e-6
    fdL = np.zeros_like(L)
    fdR = np.zeros_like(R)
    for idx in np.ndindex(L.shape):
        e = np.zeros_like(L)
        e[idx] = h
        fdL[idx] = (f(L + e, R) - f(L - e, R)) / (2 * h)
        fdR[idx] = (f(L, R + e) - f(L, R - e)) / (2 * h)
    for got, ref in ((gL, fdL), (gR, fdR)):
        rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert rel < 1e-6, rel


def test_backward_sum_rules():
    # adding a constant to, or scaling, either view leaves every score unchanged,
    # so sum dL/dI = 0 and sum I dL/dI = 0 for both views
    L, R, coarse = _soft_case(seed=16, H=14, W=18, D=10)
    g = _rng(17).standard_normal(L.shape)
    gL, gR = oracle.backward(L, R, 2, 10, coarse, 2, 0.05, 1e-12, g)
    scale = np.abs(gL).sum() + np.abs(gR).sum()
    assert scale > 0
    for grad, img in ((gL, L), (gR, R)):
        assert abs(grad.sum()) < 1e-12 * scale * 10
        assert abs((grad * img).sum()) < 1e-12 * scale * 10


def test_backward_row_restriction_is_a_partition():
    L, R, coarse = _soft_case(seed=18, H=12, W=12)
    g = _rng(19).standard_normal(L.shape)
    full = oracle.backward(L, R, 1, 8, coarse, 2, 0.1, 1e-12, g)
    a = oracle.backward(L, R, 1, 8, coarse, 2, 0.1, 1e-12, g, rows=(0, 5))
    b = oracle.backward(L, R, 1, 8, coarse, 2, 0.1, 1e-12, g, rows=(5, 12))
    np.testing.assert_allclose(full[0], a[0] + b[0], atol=1e-12)
    np.testing.assert_allclose(full[1], a[1] + b[1], atol=1e-12)


def test_l1_loss_gradient():
    rng = _rng(20)
    ds = rng.random((6, 7)) * 10
    gt = rng.random((6, 7)) * 10
    m = rng.random((6, 7)) > 0.3
    loss, g = oracle.l1_loss(ds, gt, m)
    assert abs(loss - np.abs(ds - gt)[m].mean()) < 1e-12
    h = 1e-7
    for idx in [(0, 0), (2, 3), (5, 6)]:
        e = np.zeros_like(ds)
        e[idx] = h
        fd = (oracle.l1_loss(ds + e, gt, m)[0] - oracle.l1_loss(ds - e, gt, m)[0]) / (2 * h)
        assert abs(fd - g[idx]) < 1e-6


# ------------------------------------------- confidence gating (Eqs. 5-9)

@pytest.mark.parametrize("Hc,Wc,H,W", [(5, 7, 10, 14), (6, 9, 11, 17), (1, 3, 2, 5), (4, 4, 7, 8)])
def test_bicubic_up_equals_torch_bicubic_with_its_parameter(Hc, Wc, H, W):
    # torch's bicubic (Keys' kernel with a = -0.75, clamped taps, half-pixel
    # centres) at scale factor 2: the oracle with the same parameter agrees
    torch = pytest.importorskip("torch")
    Cc = _rng(31).random((Hc, Wc)) * 2 - 1
    ref = torch.nn.functional.interpolate(torch.from_numpy(Cc)[None, None], scale_factor=2, mode="bicubic",
                                          align_corners=False)[0, 0].numpy()[:H, :W]
    np.testing.assert_allclose(oracle.bicubic_up(Cc, H, W, a=-0.75), ref, atol=1e-12)


def test_bicubic_up_reproduces_quadratics_and_constants():
    # Keys' kernel with a = -1/2 reproduces polynomials up to degree two wherever
    # no tap is clamped; weights sum to one, so constants survive everywhere
    Hc, Wc = 9, 12
    yy, xx = np.mgrid[0:Hc, 0:Wc].astype(np.float64)

    def q(y, x):
        return 0.3 + 0.7 * y - 0.2 * x + 0.05 * y * y - 0.03 * x * y + 0.02 * x * x
    up = oracle.bicubic_up(q(yy, xx), 2 * Hc, 2 * Wc)
    fy, fx = np.mgrid[0:2 * Hc, 0:2 * Wc].astype(np.float64)
    exact = q((fy + 0.5) / 2 - 0.5, (fx + 0.5) / 2 - 0.5)
    inner = (slice(4, 2 * Hc - 4), slice(4, 2 * Wc - 4))
    np.testing.assert_allclose(up[inner], exact[inner], atol=1e-12)
    assert np.abs(up - exact).max() > 1e-3  # the clamped border is not exact
    np.testing.assert_allclose(oracle.bicubic_up(np.full((3, 5), 0.625), 5, 10), 0.625, atol=1e-15)
    # a single coarse impulse spreads over eight fine rows with Keys' weights at
    # distances 7/4, 5/4, 3/4, 1/4, ... : (-3, -9, 29, 111, 111, 29, -9, -3)/128
    imp = np.zeros((7, 7))
    imp[3, 3] = 1.0
    up = oracle.bicubic_up(imp, 14, 14)
    w = np.array([-3, -9, 29, 111, 111, 29, -9, -3]) / 128.0
    np.testing.assert_allclose(up[3:11, 7], w * (111 / 128.0), atol=1e-15)
    np.testing.assert_allclose(up[7, 3:11], w * (111 / 128.0), atol=1e-15)
    assert np.all(up[:3, :] == 0) and np.all(up[11:, :] == 0)


def _brute_gated(L, R, n, Dk, coarse, ccost, r, beta, eps):
    up = oracle.bicubic_up(ccost, *L.shape)
    dr, Cr = _brute_level(L, R, n, Dk, coarse, r, eps)
    df, Cf = _brute_level(L, R, n, Dk, None, 0, eps)
    full = ~(up > beta)
    return np.where(full, df, dr), np.where(full, Cf, Cr), full


@pytest.mark.parametrize("beta", [-2.0, 0.1, 2.0])
def test_gated_search_branches(beta):
    rng = _rng(32)
    H, W, D, n, r = 11, 14, 8, 1, 1
    L = rng.random((H, W))
    R = rng.random((H, W))
    coarse = rng.integers(0, (D + 1) // 2, size=((H + 1) // 2, (W + 1) // 2)).astype(np.int16)
    ccost = rng.random(coarse.shape) * 0.6 - 0.2
    d, C, C2, full = oracle.match_gated(L, R, n, D, coarse, ccost, r, beta, 1e-9)
    bd, bC, bfull = _brute_gated(L, R, n, D, coarse, ccost, r, beta, 1e-9)
    assert np.array_equal(full, bfull) and np.array_equal(d, bd)
    np.testing.assert_allclose(C, bC, atol=1e-12)
    if beta < -1:
        assert not full.any()
    if beta > 1:
        assert full.all()
    if beta == 0.1:
        assert 0 < full.mean() < 1


def _brute_aggregate(L, R, n, Dk, d1, C1, alpha, eps):
    """Eqs. 5-7 with numpy Pearson scores: mean over the in-image 5x5 neighbours
    for which z is a candidate, lowest z on ties."""
    H, W = L.shape

    def E(i, j, z):
        lw, rw = _window(L, i, j, n), _window(R, i, j - z, n)
        return 0.0 if (lw.var() <= eps or rw.var() <= eps) else _pearson(lw, rw)
    d, C = d1.copy(), C1.copy()
    for i in range(H):
        for j in range(W):
            if C1[i, j] > alpha:
                continue
            best, bz = -np.inf, 0
            for z in range(min(Dk - 1, j) + 1):
                vals = [E(m, q, z) for m in range(i - 2, i + 3) for q in range(j - 2, j + 3)
                        if 0 <= m < H and 0 <= q < W and z <= q]
                e = float(np.mean(vals))
                if e > best:
                    best, bz = e, z
            d[i, j], C[i, j] = bz, best
    return d, C


@pytest.mark.parametrize("alpha", [-2.0, 0.3, 2.0])
def test_aggregate_brute_force(alpha):
    rng = _rng(33)
    H, W, D, n = 9, 13, 6, 1
    L = rng.integers(0, 256, (H, W)).astype(np.float64)
    R = rng.integers(0, 256, (H, W)).astype(np.float64)
    L[:3, :4] = 7.0  # flat windows score 0
    d1, C1, _ = oracle.match_level(L, R, n, D, None, 0, 0.065)
    d, C, C2 = oracle.aggregate(L, R, n, D, d1, C1, alpha, 0.065)
    bd, bC = _brute_aggregate(L, R, n, D, d1, C1, alpha, 0.065)
    assert np.array_equal(d, bd)
    np.testing.assert_allclose(C, bC, atol=1e-12)
    picked = ~(C1 > alpha)
    assert np.all(np.isneginf(C2[~picked])) and np.all(C[picked] >= C2[picked])
    if alpha < -1:
        assert np.array_equal(d, d1) and np.array_equal(C, C1)
    if alpha > 1:
        assert picked.all()


def test_aggregate_recovers_a_constant_shift_with_perfect_score():
    # a pure shift: away from the borders every neighbour scores 1 at the true
    # disparity, so the averaged DSI picks it with C = 1 even when every pixel is
    # re-picked
    H, W, n, s = 24, 48, 2, 5
    L, R = _shifted_pair(H, W, s, seed=34)
    d1 = np.zeros((H, W), np.int16)
    C1 = np.full((H, W), -1.0)
    d, C, _ = oracle.aggregate(L, R, n, 12, d1, C1, 0.9, 0.065)
    inner = (slice(n + 2, -n - 2), slice(s + n + 4, -n - 2))
    assert np.all(d[inner] == s)
    np.testing.assert_allclose(C[inner], 1.0, atol=1e-12)


def test_gated_hierarchy_limits():
    p = synth.make_pair(35, 40, 72, 3, 2, 12, True, 0.9, 5.0, 3.0, "u8")
    D, K, n, r, eps = 24, 3, 2, 1, 0.065
    plain = oracle.disparity(p.left, p.right, D, K, n, r, eps)
    # nothing gated: the plain hierarchy
    off = oracle.disparity(p.left, p.right, D, K, n, r, eps, gate=(-2.0, -2.0))
    for k in range(K):
        assert np.array_equal(off[k][0], plain[k][0]) and np.array_equal(off[k][1], plain[k][1])
    # beta above every cost: every finer level is a full search, so level 0 is
    # flat block matching whatever the coarser levels found
    full = oracle.disparity(p.left, p.right, D, K, n, r, eps, gate=(-2.0, 2.0))
    flat = oracle.flat_bm(p.left, p.right, D, n, eps)
    assert np.array_equal(full[0][0], flat[0]) and np.array_equal(full[0][1], flat[1])
    # the paper's thresholds: each level is the chain of its steps
    g = oracle.disparity(p.left, p.right, D, K, n, r, eps, gate=(0.9, 0.9))
    PL, PR = oracle.pyramid(p.left, K), oracle.pyramid(p.right, K)
    d1, C1, _, _ = oracle.match_gated(PL[0], PR[0], n, D, g[1][0], g[1][1], r, 0.9, eps)
    d, C, _ = oracle.aggregate(PL[0], PR[0], n, D, d1, C1, 0.9, eps)
    assert np.array_equal(d, g[0][0]) and np.array_equal(C, g[0][1])
    assert (d != d1).any()


def test_aggregate_pixel_list_and_scores_agree_with_the_map():
    rng = _rng(36)
    H, W, D, n = 10, 15, 7, 1
    L = rng.random((H, W))
    R = rng.random((H, W))
    d1, C1, _ = oracle.match_level(L, R, n, D, None, 0, 1e-9)
    d, C, C2 = oracle.aggregate(L, R, n, D, d1, C1, 0.5, 1e-9)
    ii, jj = np.nonzero(np.ones((H, W), bool))
    pd, pC, pC2 = oracle.aggregate_pixels(L, R, n, D, d1, C1, 0.5, 1e-9, ii, jj)
    assert np.array_equal(pd, d.ravel()) and np.array_equal(pC, C.ravel()) and np.array_equal(pC2, C2.ravel())
    picked = ~(C1 > 0.5)
    s = oracle.avg_score_many(L, R, n, ii[picked.ravel()], jj[picked.ravel()], d[picked], 1e-9)
    np.testing.assert_array_equal(s, C[picked])


# ----------------------------- soft output at every level (an extension)

@pytest.mark.parametrize("H,W", [(9, 14), (10, 7), (1, 5), (16, 16)])
def test_reduce_adjoint_is_the_transpose(H, W):
    rng = _rng(40 + H)
    x = rng.random((H, W))
    y = rng.random(((H + 1) // 2, (W + 1) // 2))
    lhs = float((oracle.reduce(x) * y).sum())
    rhs = float((x * oracle.reduce_adjoint(y, H, W)).sum())
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))
    # the reduce's weights sum to one per output, so the adjoint keeps the total
    assert abs(oracle.reduce_adjoint(y, H, W).sum() - y.sum()) <= 1e-12 * y.size


def test_soft_levels_hard_maps_are_the_hierarchy_with_the_soft_radius():
    p = synth.make_pair(41, 40, 64, 3, 2, 12, True, 0.9, 0.02, 2 / 255, "f32")
    D, K, n, rs = 24, 3, 2, 2
    out = oracle.soft_levels(p.left, p.right, D, K, n, rs, 0.05, 1e-6)
    ref = oracle.disparity(p.left, p.right, D, K, n, rs, 1e-6)
    for k in range(K):
        assert np.array_equal(out[k][1], ref[k][0]) and np.allclose(out[k][2], ref[k][1])
    # a tiny temperature makes each soft output the hard one
    cold = oracle.soft_levels(p.left, p.right, D, K, n, rs, 1e-5, 1e-6)
    for k in range(K - 1):
        near = (cold[k][2] - cold[k][3]) < 1e-3
        assert np.allclose(cold[k][0][~near], cold[k][1][~near], atol=1e-6)


def test_backward_levels_matches_central_differences():
    rng = _rng(42)
    H, W, D, K, n, rs, tau, eps = 18, 26, 10, 3, 1, 1, 0.2, 1e-6
    L = synth.texture(rng, H, W + 4)[:, 4:].copy()
    R = synth.texture(rng, H, W + 4)[:, :W].copy()
    fwd = oracle.soft_levels(L, R, D, K, n, rs, tau, eps)
    maps = [o[1] for o in fwd]
    grads = [rng.standard_normal(fwd[k][0].shape) for k in range(K - 1)] + [None]
    gL, gR = oracle.backward_levels(L, R, D, K, n, rs, tau, eps, maps, grads)

    def loss(Lx, Rx):
        PL, PR = oracle.pyramid(Lx, K), oracle.pyramid(Rx, K)
        tot = 0.0
        for k in range(K - 1):
            ds = oracle.soft_level0(PL[k], PR[k], n, oracle.level_range(D, k), maps[k + 1], rs, tau, eps)[0]
            tot += float((grads[k] * ds).sum())
        return tot
    h = 1e-6
    for (i, j) in [(5, 7), (9, 12), (0, 0), (17, 25), (8, 3)]:
        for which, G in (("L", gL), ("R", gR)):
            Lp, Rp, Lm, Rm = L.copy(), R.copy(), L.copy(), R.copy()
            if which == "L":
                Lp[i, j] += h
                Lm[i, j] -= h
            else:
                Rp[i, j] += h
                Rm[i, j] -= h
            fd = (loss(Lp, Rp) - loss(Lm, Rm)) / (2 * h)
            assert abs(fd - G[i, j]) <= 1e-5 * max(1.0, abs(fd)), (which, i, j, fd, G[i, j])


# ----------------------------- sampled-evaluation helpers the full-size tests use

def test_zncc_many_equals_zncc_triple_by_triple():
    """The list form scores each (i, j, z) exactly as the single-triple form,
    on a non-square image, at border rows and columns, and for z > j (the right
    window clamps at the left edge), in a shuffled order."""
    rng = _rng(50)
    H, W, n = 9, 17, 2
    L = rng.random((H, W))
    R = rng.random((H, W))
    ii, jj, zz = [], [], []
    for i in (0, 1, 4, H - 2, H - 1):
        for j in (0, 1, 2, 8, W - 2, W - 1):
            for z in (0, 1, 3, j, j + 2):
                ii.append(i)
                jj.append(j)
                zz.append(z)
    perm = rng.permutation(len(ii))
    ii, jj, zz = (np.array(x)[perm] for x in (ii, jj, zz))
    got = oracle.zncc_many(L, R, n, ii, jj, zz, 1e-9)
    want = np.array([oracle.zncc(L, R, n, int(i), int(j), int(z), 1e-9) for i, j, z in zip(ii, jj, zz)])
    np.testing.assert_array_equal(got, want)
    # and the single form against an independent Pearson correlation at one
    # interior triple, so a transposed pair of indices shows up
    i, j, z = 4, 8, 3
    wl = _window(L, i, j, n)
    wr = _window(R, i, j - z, n)
    assert abs(want[(ii == i) & (jj == j) & (zz == z)][0] - _pearson(wl, wr)) < 1e-12


@pytest.mark.parametrize("restricted", [False, True])
def test_match_pixels_equals_match_level_at_the_listed_pixels(restricted):
    """The pixel-list form returns, pixel by pixel, the map's winner, its score
    and the runner-up score, for a full and a restricted search, with the list
    holding border columns (clipped candidate intervals) in a shuffled order."""
    rng = _rng(51 + restricted)
    H, W, n, Dk, r = 11, 19, 1, 9, 2
    L = rng.random((H, W))
    R = rng.random((H, W))
    coarse = None
    if restricted:
        coarse = rng.integers(0, (Dk - 1) // 2 + 1, size=((H + 1) // 2, (W + 1) // 2)).astype(np.int16)
    d, C, C2 = oracle.match_level(L, R, n, Dk, coarse, r, 1e-9)
    ii, jj = np.nonzero(np.ones((H, W), dtype=bool))
    perm = rng.permutation(ii.size)
    ii, jj = ii[perm], jj[perm]
    pd, pC, pC2 = oracle.match_pixels(L, R, n, Dk, coarse, r, 1e-9, ii, jj)
    np.testing.assert_array_equal(pd, d[ii, jj])
    np.testing.assert_array_equal(pC, C[ii, jj])
    np.testing.assert_array_equal(pC2, C2[ii, jj])
    # a short list (the sampled tests' use) gives the same values
    sel = perm[:7]
    qi, qj = np.nonzero(np.ones((H, W), dtype=bool))
    qd, qC, _ = oracle.match_pixels(L, R, n, Dk, coarse, r, 1e-9, qi[sel], qj[sel])
    np.testing.assert_array_equal(qd, d[qi[sel], qj[sel]])
    np.testing.assert_array_equal(qC, C[qi[sel], qj[sel]])
