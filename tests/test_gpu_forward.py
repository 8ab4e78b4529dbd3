"""GPU forward parity: pyramid, full search, restricted search, the whole
hierarchy and the soft-argmax level, against the FP64 oracle (through the C ABI)."""
import numpy as np
import pytest

import oracle
from paper_1901_09593_amd import synth
from parity import TOL_ZNCC, cand_bounds, check_level, check_pixels

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1901_09593_amd import msibm
    msibm.lib()
    return msibm


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _tex_pair(seed, H, W, s, dtype="u8", noise=2.0):
    """A textured pair with a smooth disparity field (slanted planes)."""
    p = synth.make_pair(seed, H, W, 3, max(1, s // 2), s, True, 0.9, 5.0 if dtype == "u8" else 0.02,
                        noise if dtype == "u8" else noise / 255, dtype)
    return p


# ------------------------------------------------------------------ pyramid

@pytest.mark.parametrize("dtype,shape", [("u8", (240, 320)), ("u8", (37, 53)), ("f32", (61, 90))])
def test_pyramid_matches_oracle(M, dtype, shape):
    p = _tex_pair(1, shape[0], shape[1], 8, dtype)
    K = 5
    lv = M.pyramid(dev(p.left), K)
    ref = oracle.pyramid(p.left, K)
    for k in range(K):
        got = host(lv[k]).astype(np.float64)
        assert got.shape == ref[k].shape
        if dtype == "u8" and k <= 2:
            assert np.array_equal(got, ref[k]), f"level {k} not bit-exact"
        else:
            # float rounding from level 3 on (uint8) or level 1 on (float input):
            # a few units in the last place of the intensity range
            scale = 255.0 if dtype == "u8" else 1.0
            assert np.abs(got - ref[k]).max() <= 4e-7 * scale


# ------------------------------------------------------------------ full search

FULL_CASES = [
    # (H, W, n, D, dtype, seed)
    (60, 80, 3, 16, "u8", 0),
    (37, 150, 2, 40, "u8", 1),     # several candidate steps, ragged tile
    (23, 301, 4, 200, "f32", 2),   # several right-image chunks
    (9, 17, 1, 30, "u8", 3),       # D > W: clipped by the column index
    (12, 12, 6, 5, "f32", 4),      # window larger than the image
    (1, 40, 2, 8, "u8", 5),        # one row
    (33, 1, 1, 4, "f32", 6),       # one column
    (16, 130, 5, 1, "u8", 7),      # a single candidate
    (6, 2100, 2, 2048, "u8", 8),   # the largest D: 22 candidate chunks
]


@pytest.mark.parametrize("H,W,n,D,dtype,seed", FULL_CASES)
def test_full_search_parity(M, H, W, n, D, dtype, seed):
    p = _tex_pair(seed, H, W, max(2, D // 2), dtype)
    eps = 0.065 if dtype == "u8" else 1e-6
    d, C = M.match_level(dev(p.left), dev(p.right), n, D, None, 0, eps)
    st = check_level(host(d), host(C), p.left, p.right, n, D, None, 0, eps)
    assert st["mismatch"] <= 0.01


def test_flat_block_matching_small320(M):
    p, cfg = synth.workload("small320")
    d, C = M.match_level(dev(p.left), dev(p.right), cfg.half_window, cfg.max_disp, None, 0,
                         cfg.var_eps)
    st = check_level(host(d), host(C), p.left, p.right, cfg.half_window, cfg.max_disp, None, 0,
                     cfg.var_eps)
    print("flat BM small320", st)


# ------------------------------------------------------------------ restricted search

REFINE_CASES = [
    # (H, W, n, Dk, r, dtype, seed)
    (48, 70, 2, 24, 0, "u8", 10),
    (48, 70, 2, 24, 1, "u8", 11),
    (64, 200, 3, 60, 2, "u8", 12),
    (31, 133, 4, 64, 3, "f32", 13),
    (40, 100, 1, 40, 4, "f32", 14),
    (17, 45, 6, 30, 2, "u8", 15),
    (25, 257, 5, 128, 2, "f32", 16),
    (20, 2100, 3, 2048, 4, "u8", 17),  # the largest D and radius: priors over 7 chunks
]


@pytest.mark.parametrize("H,W,n,Dk,r,dtype,seed", REFINE_CASES)
def test_restricted_search_parity(M, H, W, n, Dk, r, dtype, seed):
    p = _tex_pair(seed, H, W, Dk * 3 // 4, dtype)
    eps = 0.065 if dtype == "u8" else 1e-6
    rng = np.random.Generator(np.random.PCG64(seed))
    Hc, Wc = (H + 1) // 2, (W + 1) // 2
    Dc = -(-Dk // 2)
    # half the priors from the ground truth (a plausible coarse map), half random
    # (outliers spread over the whole range, several right-image chunks per tile)
    gt = np.clip(np.rint(p.disp[::2, ::2] / 2), 0, Dc - 1).astype(np.int16)
    rnd = rng.integers(0, Dc, size=(Hc, Wc)).astype(np.int16)
    prior = np.where(rng.random((Hc, Wc)) < 0.5, gt, rnd).astype(np.int16)
    d, C = M.match_level(dev(p.left), dev(p.right), n, Dk, dev(prior), r, eps)
    st = check_level(host(d), host(C), p.left, p.right, n, Dk, prior, r, eps)
    assert st["mismatch"] <= 0.01


@pytest.mark.parametrize("H,W,n,Dk,r,dtype,restricted", [(37, 150, 2, 40, 0, "u8", False),
                                                       (23, 301, 4, 200, 0, "f32", False),
                                                       (64, 200, 3, 60, 2, "u8", True),
                                                       (31, 133, 5, 64, 4, "f32", True)])
def test_every_scored_candidate_matches_oracle(M, H, W, n, Dk, r, dtype, restricted):
    """The score of every candidate a search scores (not only the winner's),
    against the oracle's score of the same (pixel, candidate); exactly the
    candidate set of each pixel is scored."""
    p = _tex_pair(60 + Dk, H, W, max(2, Dk // 2), dtype)
    eps = 0.065 if dtype == "u8" else 1e-6
    prior = None
    if restricted:
        rng = np.random.Generator(np.random.PCG64(Dk))
        prior = rng.integers(0, -(-Dk // 2), size=((H + 1) // 2, (W + 1) // 2)).astype(np.int16)
    d, C, V = M.match_level(dev(p.left), dev(p.right), n, Dk, None if prior is None else dev(prior), r, eps,
                            with_costvol=True)
    V = host(V)
    lo, hi = cand_bounds(H, W, Dk, prior, r)
    zz = np.arange(Dk)[None, None, :]
    scored = (zz >= lo[:, :, None]) & (zz <= hi[:, :, None])
    assert np.all(V[~scored] == -2.0)
    ii, jj, kk = np.nonzero(scored)
    rho = oracle.zncc_many(p.left, p.right, n, ii, jj, kk, eps)
    err = np.abs(V[ii, jj, kk].astype(np.float64) - rho)
    print("all scored candidates", ii.size, "max |dZNCC|", err.max())
    assert err.max() <= TOL_ZNCC
    # the winner is the lowest z of the best score among them
    best = np.where(scored, V, -3.0).max(axis=2)
    first = np.argmax(np.where(scored, V, -3.0) == best[:, :, None], axis=2)
    assert np.array_equal(host(d), first) and np.array_equal(host(C), best)


# ------------------------------------------------------------------ hierarchy

def test_hierarchy_small320_per_level_and_end_to_end(M):
    p, cfg = synth.workload("small320")
    K, n, r, D, eps = cfg.levels, cfg.half_window, cfg.refine_radius, cfg.max_disp, cfg.var_eps
    Lg, Rg = dev(p.left), dev(p.right)
    out = M.disparity(Lg, Rg, D, K, n, r, eps, with_prior1=True)
    # the same kernels level by level: GPU pyramid, then teacher-forced levels
    PL = M.pyramid(Lg, K)
    PR = M.pyramid(Rg, K)
    maps = [None] * K
    costs = [None] * K
    for k in range(K - 1, -1, -1):
        Lk = Lg if k == 0 else PL[k]
        Rk = Rg if k == 0 else PR[k]
        prior = None if k == K - 1 else maps[k + 1]
        maps[k], costs[k] = M.match_level(Lk, Rk, n, -(-D // (1 << k)), prior, r, eps)
    assert torch.equal(maps[0], out["disp"]) and torch.equal(costs[0], out["cost"])
    assert torch.equal(maps[1], out["prior1"])
    # each level against the oracle with the GPU's own prior (teacher forcing)
    for k in range(K):
        Lk = host(PL[k]).astype(np.float64)
        Rk = host(PR[k]).astype(np.float64)
        prior = None if k == K - 1 else host(maps[k + 1])
        st = check_level(host(maps[k]), host(costs[k]), Lk, Rk, n, -(-D // (1 << k)), prior, r, eps)
        print(f"level {k}", st)
    # end to end without teacher forcing: report the cascaded mismatch rate
    ref = oracle.disparity(p.left, p.right, D, K, n, r, eps)
    mism = float((host(out["disp"]) != ref[0][0]).mean())
    print("end-to-end level-0 mismatch rate", mism)
    assert mism < 0.01


@pytest.mark.parametrize("dtype,K", [("u8", 2), ("u8", 3), ("u8", 5), ("u8", 7), ("f32", 3), ("f32", 4),
                                     ("f32", 6)])
def test_pyramid_launches_match_level_by_level(M, dtype, K):
    """The forward builds its pyramid with up to three reduce steps per launch;
    its maps and scores equal those of single-step pyramids matched level by
    level (every step count of a launch, both element types)."""
    p = _tex_pair(40 + K, 150, 262, 8, dtype)
    D, n, r = 200, 2, 1
    eps = 0.065 if dtype == "u8" else 1e-6
    Lg, Rg = dev(p.left), dev(p.right)
    out = M.disparity(Lg, Rg, D, K, n, r, eps, with_prior1=True)
    PL, PR = M.pyramid(Lg, K), M.pyramid(Rg, K)
    maps, costs = [None] * K, [None] * K
    for k in range(K - 1, -1, -1):
        Lk = Lg if k == 0 else PL[k]
        Rk = Rg if k == 0 else PR[k]
        prior = None if k == K - 1 else maps[k + 1]
        maps[k], costs[k] = M.match_level(Lk, Rk, n, -(-D // (1 << k)), prior, r, eps)
    assert torch.equal(maps[0], out["disp"]) and torch.equal(costs[0], out["cost"])
    assert torch.equal(maps[1], out["prior1"])


@pytest.mark.parametrize("dtype,ns", [("u8", [4, 2, 1]), ("f32", [3, 3, 2, 1])])
def test_per_level_windows(M, dtype, ns):
    """Per-level window sizes (the block size that shrinks with the level): the
    forward equals level-by-level matching with each level's window, each level
    agrees with the oracle fed the GPU's coarser map, and the batched path
    (with its graph) gives the same maps."""
    K = len(ns)
    p = _tex_pair(70 + K, 120, 200, 16, dtype)
    D, r = 64, 2
    eps = 0.065 if dtype == "u8" else 1e-6
    Lg, Rg = dev(p.left), dev(p.right)
    out = M.disparity(Lg, Rg, D, K, ns, r, eps, with_prior1=True)
    PL, PR = M.pyramid(Lg, K), M.pyramid(Rg, K)
    maps, costs = [None] * K, [None] * K
    for k in range(K - 1, -1, -1):
        Lk = Lg if k == 0 else PL[k]
        Rk = Rg if k == 0 else PR[k]
        prior = None if k == K - 1 else maps[k + 1]
        maps[k], costs[k] = M.match_level(Lk, Rk, ns[k], -(-D // (1 << k)), prior, r, eps)
    assert torch.equal(maps[0], out["disp"]) and torch.equal(costs[0], out["cost"])
    assert torch.equal(maps[1], out["prior1"])
    for k in range(K):
        Lk, Rk = host(PL[k]).astype(np.float64), host(PR[k]).astype(np.float64)
        prior = None if k == K - 1 else host(maps[k + 1])
        st = check_level(host(maps[k]), host(costs[k]), Lk, Rk, ns[k], -(-D // (1 << k)), prior, r, eps)
        print(f"level {k} n={ns[k]}", st)
    for flags in (M.FLAG_BATCHED, M.FLAG_BATCHED | M.FLAG_GRAPH):
        got = M.disparity_many([Lg], [Rg], [D], [K], ns, r, eps, with_prior1=True, flags=flags)[0]
        assert torch.equal(got["disp"], out["disp"]) and torch.equal(got["prior1"], out["prior1"])
        assert torch.equal(got["cost"], out["cost"])


@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_preblur_level_zero(M, dtype):
    """The pre-blur variant: level 0 is matched on the blurred input (checked
    against the oracle on its own blurred images, fed the GPU's level-1 map);
    the coarser levels are those of the plain forward."""
    p = _tex_pair(81, 96, 170, 12, dtype)
    D, K, n, r = 48, 3, 3, 2
    eps = 0.065 if dtype == "u8" else 1e-6
    Lg, Rg = dev(p.left), dev(p.right)
    plain = M.disparity(Lg, Rg, D, K, n, r, eps, with_prior1=True)
    out = M.disparity(Lg, Rg, D, K, n, r, eps, with_prior1=True, preblur=True)
    assert torch.equal(plain["prior1"], out["prior1"])
    Lb, Rb = oracle.blur(p.left), oracle.blur(p.right)
    st = check_level(host(out["disp"]), host(out["cost"]), Lb, Rb, n, D, host(out["prior1"]), r, eps)
    print("preblur level 0", st)
    assert st["mismatch"] <= 0.01
    # the batched path and its graph give the plain path's outputs
    for flags in (M.FLAG_BATCHED, M.FLAG_BATCHED | M.FLAG_GRAPH):
        got = M.disparity_many([Lg], [Rg], [D], [K], n, r, eps, with_prior1=True,
                               flags=flags | M.FLAG_PREBLUR)[0]
        for key in ("disp", "cost", "prior1"):
            assert torch.equal(got[key], out[key]), key


def test_batched_preblur_uneven_pairs_equals_plain(M):
    """The pre-blur on the batched path with uneven pairs and depths (one of
    them a single level), uint8 and float, alone and with the paper's other
    options (gating, median, per-level windows, refine +-1): every output
    equals the plain path's."""
    shapes = [(96, 150, 48, 0), (61, 200, 100, 0), (40, 70, 16, 1), (130, 90, 20, 2)]
    Ds = [s[2] for s in shapes]
    Ks = [s[3] for s in shapes]
    for dt, eps, n, r, opts in (("u8", 0.065, 3, 2, {}), ("f32", 1e-6, 3, 2, {}),
                                ("u8", 0.065, [5, 2, 1, 1], 1, dict(gate=(0.9, 0.9), median_alpha=0.9)),
                                ("f32", 1e-6, [5, 2, 1, 1], 1, dict(gate=(0.9, 0.9), median_alpha=0.9))):
        pairs = [_tex_pair(760 + i, h, w, max(3, D // 2), dt) for i, (h, w, D, K) in enumerate(shapes)]
        L = [dev(p.left) for p in pairs]
        R = [dev(p.right) for p in pairs]
        plain = M.disparity_many(L, R, Ds, Ks, n, r, eps, with_prior1=True, flags=M.FLAG_PREBLUR, **opts)
        for flags in (M.FLAG_BATCHED, M.FLAG_BATCHED | M.FLAG_GRAPH):
            got = M.disparity_many(L, R, Ds, Ks, n, r, eps, with_prior1=True, flags=flags | M.FLAG_PREBLUR,
                                   **opts)
            for a, b in zip(got, plain):
                assert set(a) == set(b)
                for key in a:
                    assert torch.equal(a[key], b[key]), (key, flags, opts)


@pytest.mark.parametrize("H,W,alpha", [(61, 90, 0.9), (37, 150, 0.97), (1, 1, 0.9), (5, 300, 0.5),
                                         (70, 65, -5.0), (70, 65, 5.0)])
def test_median_filter_matches_oracle_bit_exact(M, H, W, alpha):
    """The selective median filter (Eq. 10) on the GPU's own level map and
    costs equals the oracle's filter on the same values, pixel for pixel
    (alpha below every cost filters nothing; above every cost there are no
    good pixels, so every pixel keeps its disparity)."""
    p = _tex_pair(90 + H, max(H, 8), max(W, 8), 12)
    Lg, Rg = dev(p.left[:H, :W]), dev(p.right[:H, :W])
    d, C = M.match_level(Lg, Rg, 2, 40, None, 0, 0.065)
    got = host(M.median_filter(d, C, alpha))
    ref = oracle.median_filter(host(d), host(C).astype(np.float64), alpha)
    assert np.array_equal(got, ref)
    changed = float((got != host(d)).mean())
    print(f"{H}x{W} alpha={alpha}: {changed:.3f} of the pixels changed")
    if alpha < -1 or alpha > 1:
        assert changed == 0


def test_median_filter_any_int16_and_pitched_rows(M):
    """Arbitrary int16 values (negative, the int16 extremes, ties) and costs
    around the threshold, read from row-pitched views."""
    rng = np.random.Generator(np.random.PCG64(5))
    H, W = 83, 131
    d = rng.integers(-32768, 32768, (H, W + 7)).astype(np.int16)
    d[::3, ::2] = 32767
    d[1::4, 1::3] = -32768
    d[10:20, 10:30] = 4
    C = rng.choice(np.array([-1.0, 0.3, 0.5, np.float32(0.5) + 1e-7, 0.9, 1.0], np.float32),
                   (H, W + 5)).astype(np.float32)
    dg = dev(d)[:, :W]
    Cg = dev(C)[:, :W]
    got = host(M.median_filter(dg, Cg, 0.5))
    ref = oracle.median_filter(d[:, :W], C[:, :W].astype(np.float64), 0.5)
    assert np.array_equal(got, ref)
    assert (got != d[:, :W]).mean() > 0.2


def test_median_filter_rejects_bad_calls(M):
    d = torch.zeros((8, 8), dtype=torch.int16, device="cuda")
    C = torch.zeros((8, 8), dtype=torch.float32, device="cuda")
    e = M.lib()
    assert e.msibm_median_filter(d.data_ptr(), 8, C.data_ptr(), 8, 8, 8, 0.5, d.data_ptr(), 8, None) == -1
    assert b"overlaps" in e.msibm_last_error()
    out = torch.empty_like(d)
    assert e.msibm_median_filter(d.data_ptr(), 8, C.data_ptr(), 8, 8, 8, float("nan"), out.data_ptr(), 8,
                                 None) == -1
    assert e.msibm_median_filter(d.data_ptr(), 7, C.data_ptr(), 8, 8, 8, 0.5, out.data_ptr(), 8, None) == -2
    assert e.msibm_median_filter(None, 8, C.data_ptr(), 8, 8, 8, 0.5, out.data_ptr(), 8, None) == -1


@pytest.mark.parametrize("dtype,K,alpha", [("u8", 3, 0.9), ("u8", 4, 0.95), ("f32", 3, 0.9)])
def test_median_in_the_hierarchy(M, dtype, K, alpha):
    """With the selective median after every level, the forward equals the
    level-by-level chain of match_level and median_filter (the filtered map is
    the prior of the next level, the cost stays the matched one), and follows
    the oracle's filtered hierarchy up to near-ties."""
    p = _tex_pair(110 + K, 130, 230, 14, dtype, noise=6.0)
    D, n, r = 80, 3, 2
    eps = 0.065 if dtype == "u8" else 1e-6
    Lg, Rg = dev(p.left), dev(p.right)
    out = M.disparity(Lg, Rg, D, K, n, r, eps, with_prior1=True, median_alpha=alpha)
    PL, PR = M.pyramid(Lg, K), M.pyramid(Rg, K)
    maps, costs, raw = [None] * K, [None] * K, [None] * K
    for k in range(K - 1, -1, -1):
        Lk = Lg if k == 0 else PL[k]
        Rk = Rg if k == 0 else PR[k]
        prior = None if k == K - 1 else maps[k + 1]
        raw[k], costs[k] = M.match_level(Lk, Rk, n, -(-D // (1 << k)), prior, r, eps)
        maps[k] = M.median_filter(raw[k], costs[k], alpha)
    assert torch.equal(maps[0], out["disp"]) and torch.equal(costs[0], out["cost"])
    assert torch.equal(maps[1], out["prior1"])
    changed = [float((maps[k] != raw[k]).float().mean()) for k in range(K)]
    print("fraction changed by the filter per level", changed)
    assert max(changed) > 0
    # no cost output: the filter reads the scratch cost map
    nocost = M.disparity(Lg, Rg, D, K, n, r, eps, with_cost=False, median_alpha=alpha)
    assert torch.equal(nocost["disp"], out["disp"])
    ref = oracle.disparity(p.left, p.right, D, K, n, r, eps, median_alpha=alpha)
    mism = float((host(out["disp"]) != ref[0][0]).mean())
    print("end-to-end level-0 mismatch rate with the median", mism)
    assert mism < 0.01
    # the batched path (and its graph) filters the same way
    for flags in (M.FLAG_BATCHED, M.FLAG_BATCHED | M.FLAG_GRAPH):
        got = M.disparity_many([Lg], [Rg], [D], [K], n, r, eps, flags=flags, with_prior1=True,
                               median_alpha=alpha)[0]
        assert torch.equal(got["disp"], out["disp"]) and torch.equal(got["cost"], out["cost"])
        assert torch.equal(got["prior1"], out["prior1"])


@pytest.mark.parametrize("K", [4, 5])
def test_mid1436_full_size_sampled(M, K):
    """The 1436x992 workload at full size, in the launch configuration the
    benchmark times, with 4 levels (32 candidates at the coarsest level) and 5
    (16 at the coarsest); level 0 checked on sampled pixels against the oracle
    fed the GPU's level-1 map."""
    p, cfg = synth.workload("mid1436")
    n, r, D, eps = cfg.half_window, cfg.refine_radius, cfg.max_disp, cfg.var_eps
    out = M.disparity(dev(p.left), dev(p.right), D, K, n, r, eps, with_prior1=True)
    d, C, p1 = host(out["disp"]), host(out["cost"]), host(out["prior1"])
    rng = np.random.Generator(np.random.PCG64(99))
    H, W = d.shape
    ii = rng.integers(0, H, 6000)
    jj = rng.integers(0, W, 6000)
    # include the borders and the left strip where priors get clipped
    ii = np.concatenate([ii, np.zeros(50, int), np.full(50, H - 1), rng.integers(0, H, 100)])
    jj = np.concatenate([jj, rng.integers(0, W, 100), np.arange(100) % 7])
    st = check_pixels(d, C, p.left, p.right, n, D, p1, r, eps, ii, jj)
    print("mid1436 sampled", st)
    # accuracy sanity against the generator's ground truth
    vis = p.nonocc
    err = np.abs(d.astype(np.float64) - p.disp)
    print("mid1436 mean |d - gt| on visible pixels", err[vis].mean(), "bad>2px", (err[vis] > 2).mean())
    assert (err[vis] <= 2).mean() > 0.8


def test_mid1436_flat_block_matching_full_size_sampled(M):
    """Flat block matching (the full 256-candidate search at level 0) of the
    1436x992 uint8 pair at full size, the comparison the benchmark times: the
    default kernel shape on sampled pixels (borders and the left strip where
    the candidate range is clipped included) against the oracle, and every
    full-search shape (statistics in LDS, XCD order, candidate split, short
    chunk, tall tiles) identical to it."""
    p, cfg = synth.workload("mid1436")
    n, D, eps = cfg.half_window, cfg.max_disp, cfg.var_eps
    Lg, Rg = dev(p.left), dev(p.right)
    M.force_variant(-1)
    d, C = M.match_level(Lg, Rg, n, D, None, 0, eps)
    d, C = host(d), host(C)
    H, W = d.shape
    rng = np.random.Generator(np.random.PCG64(98))
    ii = np.concatenate([rng.integers(0, H, 4000), np.zeros(40, int), np.full(40, H - 1), rng.integers(0, H, 300)])
    jj = np.concatenate([rng.integers(0, W, 4000), rng.integers(0, W, 80), np.arange(300) % 260])
    st = check_pixels(d, C, p.left, p.right, n, D, None, 0, eps, ii, jj)
    print("mid1436 flat block matching sampled", st)
    try:
        for v in list(range(8)) + [16, 17, 19, 32, 33, 35, 48, 49, 51]:
            M.force_variant(v)
            dv, Cv = M.match_level(Lg, Rg, n, D, None, 0, eps)
            assert np.array_equal(host(dv), d) and np.array_equal(host(Cv), C), v
    finally:
        M.force_variant(-1)


def test_repeatable(M):
    p, cfg = synth.workload("small320")
    a = M.disparity(dev(p.left), dev(p.right), cfg.max_disp, cfg.levels, cfg.half_window,
                    cfg.refine_radius, cfg.var_eps)
    b = M.disparity(dev(p.left), dev(p.right), cfg.max_disp, cfg.levels, cfg.half_window,
                    cfg.refine_radius, cfg.var_eps)
    assert torch.equal(a["disp"], b["disp"]) and torch.equal(a["cost"], b["cost"])


@pytest.mark.parametrize("H,W,K", [(1, 1, 1), (1, 1, 3), (3, 2, 2), (5, 9, 8), (2, 300, 4)])
def test_degenerate_shapes(M, H, W, K):
    rng = np.random.Generator(np.random.PCG64(H * 100 + W))
    L = rng.integers(0, 256, size=(H, W)).astype(np.uint8)
    R = rng.integers(0, 256, size=(H, W)).astype(np.uint8)
    D, n, r, eps = 12, 2, 1, 0.065
    out = M.disparity(dev(L), dev(R), D, K, n, r, eps, with_prior1=K >= 2)
    ref = oracle.disparity(L, R, D, K, n, r, eps)
    d = host(out["disp"])
    # teacher-forced level 0 check with the GPU's level-1 map
    prior = host(out["prior1"]) if K >= 2 else None
    check_level(d, host(out["cost"]), L, R, n, D, prior, r, eps)
    if K == 1:
        gap = ref[0][1] - ref[0][2]
        assert np.all((d == ref[0][0]) | (gap <= TOL_ZNCC))


@pytest.mark.parametrize("pitch,offset", [(384, 0), (331, 0), (384, 1), (331, 3)])
def test_pitched_input(M, pitch, offset):
    """Views with a wider row pitch, odd pitches and unaligned first pixels
    (uint8 rows then start off word boundaries) give the same maps and scores
    as a contiguous copy."""
    p, cfg = synth.workload("small320")
    big_l = torch.zeros((240, pitch), dtype=torch.uint8, device="cuda")
    big_r = torch.zeros((240, pitch), dtype=torch.uint8, device="cuda")
    big_l[:, offset:offset + 320] = dev(p.left)
    big_r[:, offset:offset + 320] = dev(p.right)
    a = M.disparity(big_l[:, offset:offset + 320], big_r[:, offset:offset + 320], cfg.max_disp, cfg.levels,
                    cfg.half_window, cfg.refine_radius, cfg.var_eps)
    b = M.disparity(dev(p.left), dev(p.right), cfg.max_disp, cfg.levels, cfg.half_window,
                    cfg.refine_radius, cfg.var_eps)
    assert torch.equal(a["disp"], b["disp"]) and torch.equal(a["cost"], b["cost"])


# ------------------------------------------------------------------ soft level

def test_soft_level_parity_diff960_crop(M):
    p, cfg = synth.workload("diff960", 0)
    L = np.ascontiguousarray(p.left[:180, :320])
    R = np.ascontiguousarray(p.right[:180, :320])
    K, n, r, D, eps, rs, tau = cfg.levels, cfg.half_window, cfg.refine_radius, cfg.max_disp, \
        cfg.var_eps, cfg.soft_radius, cfg.tau
    out = M.disparity(dev(L), dev(R), D, K, n, r, eps, soft_radius=rs, tau=tau)
    p1 = host(out["prior1"])
    ds_o, dh_o, C_o, C2_o = oracle.soft_level0(L, R, n, D, p1, rs, tau, eps)
    ds = host(out["soft"]).astype(np.float64)
    assert np.abs(ds - ds_o).max() <= 1e-2
    print("soft max |dd|", np.abs(ds - ds_o).max())
    check_level(host(out["disp"]), host(out["cost"]), L, R, n, D, p1, rs, eps,
                ref=(dh_o, C_o, C2_o))


@pytest.mark.parametrize("variant", list(range(64)))
def test_every_kernel_variant_gives_identical_results(M, variant):
    p, cfg = synth.workload("small320")
    K, n, r, D, eps = cfg.levels, cfg.half_window, cfg.refine_radius, cfg.max_disp, cfg.var_eps
    Lg, Rg = dev(p.left), dev(p.right)
    M.force_variant(-1)
    ref = M.disparity(Lg, Rg, D, K, n, r, eps, with_prior1=True)
    flat_ref = M.match_level(Lg, Rg, n, 40, None, 0, eps)
    try:
        M.force_variant(variant)
        got = M.disparity(Lg, Rg, D, K, n, r, eps, with_prior1=True)
        flat = M.match_level(Lg, Rg, n, 40, None, 0, eps)
    finally:
        M.force_variant(-1)
    assert torch.equal(ref["disp"], got["disp"]) and torch.equal(ref["cost"], got["cost"])
    assert torch.equal(ref["prior1"], got["prior1"])
    assert torch.equal(flat_ref[0], flat[0]) and torch.equal(flat_ref[1], flat[1])


def test_restricted_shapes_identical_at_largest_range(M):
    """Every restricted-search shape (candidate split or not, fixed window or
    chunked, tile order, short chunk, tall tiles) gives the same maps and scores where the candidate
    range spans several chunks (D_k = 2048, r = 4, priors over the whole
    range)."""
    H, W, n, Dk, r = 20, 2100, 3, 2048, 4
    p = _tex_pair(18, H, W, 1500, "u8")
    rng = np.random.Generator(np.random.PCG64(18))
    prior = dev(rng.integers(0, Dk // 2, size=((H + 1) // 2, (W + 1) // 2)).astype(np.int16))
    Lg, Rg = dev(p.left), dev(p.right)
    outs = []
    try:
        for v in (0, 2, 4, 6, 8, 12, 14, 16, 20, 24, 32, 40, 48, 56):
            M.force_variant(v)
            outs.append(M.match_level(Lg, Rg, n, Dk, prior, r, 0.065))
    finally:
        M.force_variant(-1)
    for d, C in outs[1:]:
        assert torch.equal(outs[0][0], d) and torch.equal(outs[0][1], C)


def test_autotune_picks_per_shape_and_keeps_results(M, tmp_path):
    """The autotuner measures each level shape once, records it in its cache
    file, reloads it, and its choices leave every output unchanged."""
    p, cfg = synth.workload("small320")
    K, n, r, D, eps = cfg.levels, cfg.half_window, cfg.refine_radius, cfg.max_disp, cfg.var_eps
    Lg, Rg = dev(p.left), dev(p.right)
    ref = M.disparity(Lg, Rg, D, K, n, r, eps, with_prior1=True)
    cache = tmp_path / "tune.txt"
    try:
        M.autotune(True, str(cache))
        got = M.disparity(Lg, Rg, D, K, n, r, eps, with_prior1=True)
        table = M.autotune_table()
        again = M.disparity(Lg, Rg, D, K, n, r, eps, with_prior1=True)
    finally:
        M.autotune(False)
    torch.cuda.synchronize()
    for out in (got, again):
        assert torch.equal(ref["disp"], out["disp"]) and torch.equal(ref["cost"], out["cost"])
        assert torch.equal(ref["prior1"], out["prior1"])
    shapes = {(row[4], row[5]) for row in table}
    for k in range(K):
        assert (M.level_dim(240, k), M.level_dim(320, k)) in shapes
    assert all(0 <= row[7] <= 63 and row[8] > 0 for row in table)
    # modes: one full search (mode 0) at the coarsest level, restricted below
    assert {row[0] for row in table} == {0, 1}
    lines = cache.read_text().splitlines()
    assert len(lines) == len(table)
    M.autotune(True, str(cache))  # the cache parses back
    M.autotune(False)
