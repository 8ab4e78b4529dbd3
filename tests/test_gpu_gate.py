"""GPU parity of the confidence gating (Eqs. 5-9) against the FP64 oracle: the
bicubic doubling of the coarser cost, the beta-gated full search, the re-pick
by the 5x5-averaged scores, and the gated hierarchy (through the C ABI)."""
import numpy as np
import pytest

import oracle
from paper_1901_09593_amd import synth
from parity import TOL_ZNCC, cand_bounds

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


def _pair(seed, H, W, s, dtype="u8", noise=4.0):
    return synth.make_pair(seed, H, W, 4, max(1, s // 3), s, True, 0.9, 5.0 if dtype == "u8" else 0.02,
                           noise if dtype == "u8" else noise / 255, dtype)


def _eps(dtype):
    return 0.065 if dtype == "u8" else 1e-6


@pytest.mark.parametrize("Hc,Wc,H,W", [(5, 7, 10, 14), (6, 9, 11, 17), (1, 1, 1, 2), (33, 70, 65, 139)])
def test_upsample_cost_bit_exact(M, Hc, Wc, H, W):
    Cc = (np.random.Generator(np.random.PCG64(Hc * W)).random((Hc, Wc)) * 2 - 1).astype(np.float32)
    got = host(M.upsample_cost(dev(Cc), H, W))
    ref = oracle.bicubic_up(Cc.astype(np.float64), H, W)
    assert np.array_equal(got, ref)


def _check_gated(d, C, L, R, n, Dk, prior, pcost, r, beta, eps):
    """Gated search parity: the same branch per pixel, scores within tolerance,
    the oracle's choice except at near ties."""
    H, W = d.shape
    d_o, C_o, C2_o, full = oracle.match_gated(L, R, n, Dk, prior, pcost.astype(np.float64), r, beta, eps)
    lo_r, hi_r = cand_bounds(H, W, Dk, prior, r)
    lo_f, hi_f = cand_bounds(H, W, Dk, None, r)
    lo, hi = np.where(full, lo_f, lo_r), np.where(full, hi_f, hi_r)
    dg = d.astype(np.int64)
    assert np.all((dg >= lo) & (dg <= hi)), "GPU chose a candidate outside its branch's interval"
    ii, jj = np.nonzero(np.ones((H, W), dtype=bool))
    rho_at = oracle.zncc_many(L, R, n, ii, jj, dg.ravel(), eps).reshape(H, W)
    err = np.abs(C.astype(np.float64) - rho_at)
    assert err.max() <= TOL_ZNCC, err.max()
    mism = dg != d_o
    near = (C_o - C2_o) <= TOL_ZNCC
    assert not (mism & ~near).any(), np.argwhere(mism & ~near)[:5]
    assert np.all(rho_at >= C_o - TOL_ZNCC)
    return {"full_branch": float(full.mean()), "mismatch": float(mism.mean()), "max_dzncc": float(err.max())}


@pytest.mark.parametrize("dtype,H,W,n,D,beta", [("u8", 70, 150, 2, 48, 0.9), ("f32", 45, 131, 3, 40, 0.8),
                                                 ("u8", 37, 70, 1, 20, 2.0), ("u8", 64, 128, 4, 64, -2.0),
                                                 ("u8", 19, 300, 6, 90, 0.95)])
def test_gated_search_matches_oracle(M, dtype, H, W, n, D, beta):
    """Each pixel takes the branch the oracle takes (the doubled cost is the
    same double value) and the branch's winner within the score tolerance."""
    p = _pair(200 + n, H, W, D // 2, dtype)
    eps = _eps(dtype)
    Lg, Rg = dev(p.left), dev(p.right)
    P1L, P1R = M.pyramid(Lg, 2)[1], M.pyramid(Rg, 2)[1]
    prior, pcost = M.match_level(P1L, P1R, n, -(-D // 2), None, 0, eps)
    d, C = M.match_level_gated(Lg, Rg, n, D, prior, pcost, 2, beta, eps)
    st = _check_gated(host(d), host(C), p.left.astype(np.float64), p.right.astype(np.float64), n, D,
                      host(prior), host(pcost), 2, beta, eps)
    print(dtype, H, W, n, D, beta, st)
    if beta > 1:
        assert st["full_branch"] == 1.0
    if beta < -1:
        # nothing gated: the plain restricted search
        d0, C0 = M.match_level(Lg, Rg, n, D, prior, 2, eps)
        assert torch.equal(d0, d) and torch.equal(C0, C)


def _check_repick(d, C, L, R, n, Dk, d1, C1, alpha, eps):
    H, W = d.shape
    picked = ~(C1.astype(np.float64) > alpha)
    assert np.array_equal(d[~picked], d1[~picked]) and np.array_equal(C[~picked], C1[~picked])
    ii, jj = np.nonzero(picked)
    if len(ii) == 0:
        return {"picked": 0.0}
    d_o, C_o, C2_o = oracle.aggregate_pixels(L, R, n, Dk, d1, C1.astype(np.float64), alpha, eps, ii, jj)
    dg = d[ii, jj].astype(np.int64)
    assert np.all((dg >= 0) & (dg <= np.minimum(Dk - 1, jj)))
    e_at = oracle.avg_score_many(L, R, n, ii, jj, dg, eps)
    err = np.abs(C[ii, jj].astype(np.float64) - e_at)
    assert err.max() <= TOL_ZNCC, err.max()
    mism = dg != d_o
    near = (C_o - C2_o) <= TOL_ZNCC
    assert not (mism & ~near).any(), np.argwhere(mism & ~near)[:5]
    assert np.all(e_at >= C_o - TOL_ZNCC)
    return {"picked": float(picked.mean()), "mismatch": float(mism.mean()), "max_dzncc": float(err.max())}


@pytest.mark.parametrize("dtype,H,W,n,D,alpha", [("u8", 70, 150, 2, 48, 0.9), ("f32", 45, 131, 3, 40, 0.95),
                                                  ("u8", 37, 70, 1, 20, 2.0), ("u8", 29, 77, 4, 100, -2.0),
                                                  ("u8", 19, 200, 6, 70, 0.97), ("f32", 8, 64, 5, 33, 0.9)])
def test_repick_matches_oracle(M, dtype, H, W, n, D, alpha):
    """Pixels above alpha keep their values bit for bit; re-picked pixels score
    the oracle's averaged score at their choice and pick the oracle's z except
    at near ties."""
    p = _pair(300 + n, H, W, D // 2, dtype, noise=8.0)
    eps = _eps(dtype)
    Lg, Rg = dev(p.left), dev(p.right)
    d1, C1 = M.match_level(Lg, Rg, n, D, None, 0, eps)
    d, C = M.aggregate_refine(Lg, Rg, n, D, d1, C1, alpha, eps)
    st = _check_repick(host(d), host(C), p.left.astype(np.float64), p.right.astype(np.float64), n, D,
                       host(d1), host(C1), alpha, eps)
    print(dtype, H, W, n, D, alpha, st)
    if alpha > 1:
        assert st["picked"] == 1.0


def test_repick_constant_shift(M):
    """A pure shift: re-picking every pixel recovers it with an averaged score
    of 1 away from the borders."""
    H, W, n, s = 40, 200, 2, 9
    T = synth.texture(np.random.Generator(np.random.PCG64(5)), H, W + s) * 255
    L, R = T[:, :W].astype(np.float32), T[:, s:s + W].astype(np.float32)
    d1 = torch.zeros((H, W), dtype=torch.int16, device="cuda")
    C1 = torch.full((H, W), -1.0, device="cuda")
    d, C = M.aggregate_refine(dev(L), dev(R), n, 32, d1, C1, 0.9, 0.065)
    inner = (slice(n + 2, -n - 2), slice(s + n + 4, -n - 2))
    assert np.all(host(d)[inner] == s)
    assert np.abs(host(C)[inner] - 1.0).max() <= 1e-5


@pytest.mark.parametrize("dtype,K,median", [("u8", 3, False), ("u8", 4, True), ("f32", 3, False)])
def test_gated_hierarchy_equals_level_chain_and_oracle(M, dtype, K, median):
    """The gated forward equals the level-by-level chain of the gating entry
    points (bit for bit), and follows the oracle's gated hierarchy."""
    p = _pair(400 + K, 96, 200, 24, dtype, noise=8.0)
    D, n, r = 64, 2, 1
    eps = _eps(dtype)
    ab = (0.9, 0.9)
    malpha = 0.9 if median else None
    Lg, Rg = dev(p.left), dev(p.right)
    out = M.disparity(Lg, Rg, D, K, n, r, eps, with_prior1=True, gate=ab, median_alpha=malpha)
    PL, PR = M.pyramid(Lg, K), M.pyramid(Rg, K)
    maps, costs = [None] * K, [None] * K
    for k in range(K - 1, -1, -1):
        Lk = Lg if k == 0 else PL[k]
        Rk = Rg if k == 0 else PR[k]
        Dk = -(-D // (1 << k))
        if k == K - 1:
            d1, C1 = M.match_level(Lk, Rk, n, Dk, None, r, eps)
        else:
            d1, C1 = M.match_level_gated(Lk, Rk, n, Dk, maps[k + 1], costs[k + 1], r, ab[1], eps)
        d, C = M.aggregate_refine(Lk, Rk, n, Dk, d1, C1, ab[0], eps)
        if median:
            d = M.median_filter(d, C, malpha)
        maps[k], costs[k] = d, C
    assert torch.equal(maps[0], out["disp"]) and torch.equal(costs[0], out["cost"])
    assert torch.equal(maps[1], out["prior1"])
    ref = oracle.disparity(p.left, p.right, D, K, n, r, eps, gate=ab, median_alpha=malpha)
    mism = float((host(out["disp"]) != ref[0][0]).mean())
    print("gated end-to-end level-0 mismatch rate", mism)
    assert mism < 0.02
    # the gating changes the result; the batched path (and its graph) gives the
    # plain path's
    plain = M.disparity(Lg, Rg, D, K, n, r, eps)
    assert not torch.equal(plain["disp"], out["disp"])
    for flags in (M.FLAG_BATCHED, M.FLAG_BATCHED | M.FLAG_GRAPH):
        got = M.disparity_many([Lg], [Rg], [D], [K], n, r, eps, flags=flags, with_prior1=True, gate=ab,
                               median_alpha=malpha)[0]
        for key in ("disp", "cost", "prior1"):
            assert torch.equal(got[key], out[key]), key


@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_gated_mid1436_level0_sampled(M, dtype):
    """The mid-size workload at full size with the paper's thresholds: level 0's
    gated search and re-pick checked on sampled pixels against the oracle fed the
    GPU's level-1 map and cost.  As float images (the same values), level 0's
    launches hold more workgroups than the two-per-CU pipelined float walk
    takes, so they run the two-barrier walk, and the coarser levels the
    pipelined one."""
    p, cfg = synth.workload("mid1436")
    K, n, r, D, eps = cfg.levels, cfg.half_window, cfg.refine_radius, cfg.max_disp, cfg.var_eps
    ab = (0.9, 0.9)
    if dtype == "f32":
        p.left, p.right = p.left.astype(np.float32), p.right.astype(np.float32)
    Lg, Rg = dev(p.left), dev(p.right)
    PL, PR = M.pyramid(Lg, 2), M.pyramid(Rg, 2)
    out = M.disparity(Lg, Rg, D, K, n, r, eps, with_prior1=True, gate=ab)
    # level 1's cost: re-run level 1's steps from the GPU's level-2 result
    full = M.disparity(PL[1], PR[1], -(-D // 2), K - 1, n, r, eps, gate=ab)
    assert torch.equal(full["disp"], out["prior1"])
    prior, pcost = out["prior1"], full["cost"]
    d1, C1 = M.match_level_gated(Lg, Rg, n, D, prior, pcost, r, ab[1], eps)
    d, C = M.aggregate_refine(Lg, Rg, n, D, d1, C1, ab[0], eps)
    assert torch.equal(d, out["disp"]) and torch.equal(C, out["cost"])
    rng = np.random.Generator(np.random.PCG64(17))
    H, W = p.left.shape
    ii, jj = rng.integers(0, H, 1500), rng.integers(0, W, 1500)
    L64, R64 = p.left.astype(np.float64), p.right.astype(np.float64)
    # gated search at the samples: the branch from the doubled cost, then the
    # branch's oracle search
    up = oracle.bicubic_up(host(pcost).astype(np.float64), H, W)
    fb = ~(up[ii, jj] > ab[1])
    hd1, hC1 = host(d1), host(C1)
    for sel, pri in ((fb, None), (~fb, host(prior))):
        do, Co, C2o = oracle.match_pixels(L64, R64, n, D, pri, r, eps, ii[sel], jj[sel])
        dg = hd1[ii[sel], jj[sel]]
        rho = oracle.zncc_many(L64, R64, n, ii[sel], jj[sel], dg, eps)
        assert np.abs(hC1[ii[sel], jj[sel]] - rho).max() <= TOL_ZNCC
        assert not ((dg != do) & ((Co - C2o) > TOL_ZNCC)).any()
    print("full-search branch at level 0:", float(fb.mean()))
    # re-pick at the samples
    hd, hC = host(d), host(C)
    picked = ~(hC1[ii, jj].astype(np.float64) > ab[0])
    si, sj = ii[picked][:400], jj[picked][:400]
    do, Co, C2o = oracle.aggregate_pixels(L64, R64, n, D, hd1, hC1.astype(np.float64), ab[0], eps, si, sj)
    e_at = oracle.avg_score_many(L64, R64, n, si, sj, hd[si, sj], eps)
    assert np.abs(hC[si, sj] - e_at).max() <= TOL_ZNCC
    assert not ((hd[si, sj] != do) & ((Co - C2o) > TOL_ZNCC)).any()
    print("re-picked at level 0:", float(picked.mean()))
    vis = p.nonocc
    err = np.abs(hd.astype(np.float64) - p.disp)
    print("gated mid1436 bad>2px", float((err[vis] > 2).mean()))


@pytest.mark.parametrize("H,W,D,n", [(1, 1, 4, 2), (2, 3, 5, 1), (1, 70, 30, 3), (70, 1, 8, 2), (9, 130, 1, 6)])
def test_gating_degenerate_shapes(M, H, W, D, n):
    """Single pixels, single rows and columns, one candidate, the largest window:
    both gating steps follow the oracle."""
    rng = np.random.Generator(np.random.PCG64(H * 100 + W))
    L = rng.integers(0, 256, (H, W)).astype(np.uint8)
    R = rng.integers(0, 256, (H, W)).astype(np.uint8)
    Lg, Rg = dev(L), dev(R)
    Hc, Wc = (H + 1) // 2, (W + 1) // 2
    prior = rng.integers(0, max(1, (D + 1) // 2), (Hc, Wc)).astype(np.int16)
    pcost = (rng.random((Hc, Wc)) * 2 - 1).astype(np.float32)
    for beta in (0.0, 2.0):
        d, C = M.match_level_gated(Lg, Rg, n, D, dev(prior), dev(pcost), 1, beta, 0.065)
        _check_gated(host(d), host(C), L.astype(np.float64), R.astype(np.float64), n, D, prior, pcost, 1, beta,
                     0.065)
    d1, C1 = M.match_level(Lg, Rg, n, D, None, 0, 0.065)
    for alpha in (0.3, 2.0):
        d, C = M.aggregate_refine(Lg, Rg, n, D, d1, C1, alpha, 0.065)
        _check_repick(host(d), host(C), L.astype(np.float64), R.astype(np.float64), n, D, host(d1), host(C1),
                      alpha, 0.065)


@pytest.mark.parametrize("dtype", ["f32", "u8"])
def test_gating_pitched_images_and_largest_range(M, dtype):
    """Row-pitched inputs, and a range of 2048 candidates (every tile walks up
    to 2048 candidates through 64 staged chunks; the right-most pixels checked
    against the oracle)."""
    rng = np.random.Generator(np.random.PCG64(77))
    H, W, D, n = 12, 2100, 2048, 2
    base = synth.texture(rng, H, W + 40) * 255
    npt = np.float32 if dtype == "f32" else np.uint8
    if dtype == "u8":
        base = np.clip(np.rint(base), 0, 255)
    wide_L = np.zeros((H, W + 11), npt)
    wide_R = np.zeros((H, W + 11), npt)
    wide_L[:, :W] = base[:, :W]          # a shift of 40: R(x - 40) = L(x)
    wide_R[:, :W] = base[:, 40:40 + W]
    Lg, Rg = dev(wide_L)[:, :W], dev(wide_R)[:, :W]
    assert Lg.stride(0) == W + 11
    d1, C1 = M.match_level(Lg, Rg, n, D, None, 0, 1e-6)
    C1 = torch.where(torch.arange(W, device="cuda")[None, :] % 97 == 0, torch.full_like(C1, -1.0), C1)
    d, C = M.aggregate_refine(Lg, Rg, n, D, d1, C1, 0.9, 1e-6)
    L64, R64 = wide_L[:, :W].astype(np.float64), wide_R[:, :W].astype(np.float64)
    picked = ~(host(C1).astype(np.float64) > 0.9)
    ii, jj = np.nonzero(picked)
    sel = np.argsort(-jj)[:40]  # the largest columns: the longest candidate walks
    ii, jj = ii[sel], jj[sel]
    do, Co, C2o = oracle.aggregate_pixels(L64, R64, n, D, host(d1), host(C1).astype(np.float64), 0.9, 1e-6, ii, jj)
    hd, hC = host(d), host(C)
    e_at = oracle.avg_score_many(L64, R64, n, ii, jj, hd[ii, jj], 1e-6)
    assert np.abs(hC[ii, jj] - e_at).max() <= TOL_ZNCC
    assert not ((hd[ii, jj] != do) & ((Co - C2o) > TOL_ZNCC)).any()
    # the same on contiguous copies
    d2, C2 = M.aggregate_refine(Lg.contiguous(), Rg.contiguous(), n, D, d1, C1, 0.9, 1e-6)
    assert torch.equal(d2, d) and torch.equal(C2, C)


def test_gated_forward_tiny_and_single_level(M):
    """The gated forward on a single level (only the re-pick runs) and on an
    image smaller than one tile, against the oracle's gated hierarchy."""
    for (H, W, D, K) in ((5, 7, 6, 1), (30, 50, 16, 3), (1, 9, 4, 2)):
        rng = np.random.Generator(np.random.PCG64(H + W))
        p = synth.make_pair(H + W, max(H, 8), max(W, 8), 2, 1, max(2, D // 2), False, 1.0, 0.0, 2.0, "u8")
        L, R = np.ascontiguousarray(p.left[:H, :W]), np.ascontiguousarray(p.right[:H, :W])
        out = M.disparity(dev(L), dev(R), D, K, 1, 1, 0.065, gate=(0.9, 0.9))
        ref = oracle.disparity(L, R, D, K, 1, 1, 0.065, gate=(0.9, 0.9))
        mism = float((host(out["disp"]) != ref[0][0]).mean())
        print(H, W, D, K, "mismatch", mism)
        assert mism <= 0.05


@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_paper_parameters_all_options_together(M, dtype):
    """Every plain-path option at once, as the benchmark's paper-parameter row
    runs it (halving windows, refine +-1, pre-blurred level 0, gating and the
    median): the forward against the oracle's hierarchy with the same options,
    and against the level-by-level chain of the entry points."""
    p = _pair(500, 90, 180, 30, dtype, noise=6.0)
    D, K, r = 48, 3, 1
    ns = [5, 2, 1]
    eps = _eps(dtype)
    ab, malpha = (0.9, 0.9), 0.9
    Lg, Rg = dev(p.left), dev(p.right)
    out = M.disparity(Lg, Rg, D, K, ns, r, eps, with_prior1=True, preblur=True, gate=ab, median_alpha=malpha)
    ref = oracle.disparity(p.left, p.right, D, K, ns, r, eps, preblur=True, gate=ab, median_alpha=malpha)
    mism = float((host(out["disp"]) != ref[0][0]).mean())
    print(dtype, "all options: level-0 mismatch rate against the oracle", mism)
    assert mism < 0.02
    # the chain: pyramid of the input, level 0 on the blurred input
    PL, PR = M.pyramid(Lg, K), M.pyramid(Rg, K)
    Lb = dev(oracle.blur(p.left).astype(np.float32))
    Rb = dev(oracle.blur(p.right).astype(np.float32))
    maps, costs = [None] * K, [None] * K
    for k in range(K - 1, -1, -1):
        Lk, Rk = (PL[k], PR[k]) if k > 0 else (Lb, Rb)
        Dk = -(-D // (1 << k))
        if k == K - 1:
            d1, C1 = M.match_level(Lk, Rk, ns[k], Dk, None, r, eps)
        else:
            d1, C1 = M.match_level_gated(Lk, Rk, ns[k], Dk, maps[k + 1], costs[k + 1], r, ab[1], eps)
        d, C = M.aggregate_refine(Lk, Rk, ns[k], Dk, d1, C1, ab[0], eps)
        maps[k], costs[k] = M.median_filter(d, C, malpha), C
    assert torch.equal(maps[1], out["prior1"])
    # level 0 of the chain ran on the oracle's blur (FP64, rounded to float):
    # compare with the oracle's tolerance rule instead of bit for bit
    agree = float((maps[0] == out["disp"]).float().mean())
    print(dtype, "level-0 agreement with the chain on the FP64 blur", agree)
    assert agree > 0.98
