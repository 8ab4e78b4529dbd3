"""Batched forward (one launch per stage for all pairs) and its hipGraph replay
against the plain per-pair path: identical outputs, bit for bit."""
import numpy as np
import pytest

from paper_1901_09593_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PERSISTENT_OFF = ("persistent scheduler disabled: two runs hung on MI355X "
                  "(at the synchronize after the launch) and the cause is not found")


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1901_09593_amd import msibm
    msibm.lib()
    return msibm


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _batch(dtypes, count=5, seed=7, dmin=24):
    """Pairs of assorted sizes and disparity ranges (so level counts differ)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pairs = []
    for i in range(count):
        dtype = dtypes[i % len(dtypes)]
        H = int(rng.integers(40, 260))
        W = int(rng.integers(60, 400))
        D = int(rng.integers(dmin, 160))
        scale = 1.0 if dtype == "u8" else 1.0 / 255
        p = synth.make_pair(100 + i, H, W, 4, 0.05 * D, 0.9 * D, True, 1.0, 0.0, 2.0 * scale, dtype)
        pairs.append((p, D))
    return pairs


def _inputs(pairs):
    L = [dev(p.left) for p, _ in pairs]
    R = [dev(p.right) for p, _ in pairs]
    return L, R, [D for _, D in pairs], [0] * len(pairs)


def _equal(ref, got, tag=""):
    for i, (a, b) in enumerate(zip(ref, got)):
        assert set(a) == set(b)
        for k in a:
            assert torch.equal(a[k], b[k]), (tag, i, k)


@pytest.mark.parametrize("dtypes,n,r,rs", [(("u8",), 4, 2, 0), (("u8",), 3, 3, 0), (("f32",), 5, 2, 0),
                                           (("f32",), 3, 2, 3), (("u8", "f32"), 2, 1, 0),
                                           (("f32",), 6, 4, 4), (("u8",), 1, 0, 0), (("u8",), 5, 1, 0),
                                           (("u8",), 6, 2, 0)])
def test_batched_equals_plain(M, dtypes, n, r, rs):
    pairs = _batch(dtypes, seed=n * 10 + r, dmin=33 if rs else 24)  # soft needs K >= 2
    eps = 0.065 if dtypes == ("u8",) else 1e-6
    L, R, Ds, Ks = _inputs(pairs)
    print("batched call", dtypes, n, r, rs, flush=True)
    plain = M.disparity_many(L, R, Ds, Ks, n, r, eps, soft_radius=rs, with_prior1=True)
    batched = M.disparity_many(L, R, Ds, Ks, n, r, eps, soft_radius=rs, with_prior1=True,
                               flags=M.FLAG_BATCHED)
    torch.cuda.synchronize()
    _equal(plain, batched)


def test_batched_explicit_levels_and_single_pair(M):
    pairs = _batch(("u8",), count=3, seed=11)
    L, R, Ds, _ = _inputs(pairs)
    Ks = [1, 3, 2]
    plain = M.disparity_many(L, R, Ds, Ks, 3, 2, 0.065, with_prior1=True)
    batched = M.disparity_many(L, R, Ds, Ks, 3, 2, 0.065, with_prior1=True, flags=M.FLAG_BATCHED)
    one = M.disparity_many(L[1:2], R[1:2], Ds[1:2], Ks[1:2], 3, 2, 0.065, with_prior1=True,
                           flags=M.FLAG_BATCHED)
    torch.cuda.synchronize()
    _equal(plain, batched)
    _equal(plain[1:2], one)


def test_graph_replay_equals_direct_and_repeats(M):
    pairs = _batch(("u8",), count=6, seed=3)
    L, R, Ds, Ks = _inputs(pairs)
    n, r, eps = 4, 2, 0.065
    ref = M.disparity_many(L, R, Ds, Ks, n, r, eps)
    flags = M.FLAG_BATCHED | M.FLAG_GRAPH
    outs = M.disparity_many(L, R, Ds, Ks, n, r, eps, flags=flags)
    ws = torch.empty(M.workspace_bytes(M._pairs(L, R, Ds, Ks)[0], len(L), M.make_config(n, r, eps, flags=flags)),
                     dtype=torch.uint8, device="cuda")
    for rep in range(4):
        # the same buffers every time: the first call captures, later calls replay;
        # eager work and a synchronisation between replays
        for o in outs:
            for t in o.values():
                t.fill_(-7 if t.dtype == torch.int16 else 7.0)
        ws.fill_(rep)
        M.disparity_many(L, R, Ds, Ks, n, r, eps, flags=flags, workspace=ws, outputs=outs)
        torch.cuda.synchronize()
        _equal(ref, outs, rep)


def test_graph_cache_keys_on_outputs(M):
    pairs = _batch(("f32",), count=3, seed=5, dmin=33)
    L, R, Ds, Ks = _inputs(pairs)
    flags = M.FLAG_BATCHED | M.FLAG_GRAPH
    ref = M.disparity_many(L, R, Ds, Ks, 3, 2, 1e-6, soft_radius=3, with_prior1=True)
    a = M.disparity_many(L, R, Ds, Ks, 3, 2, 1e-6, soft_radius=3, with_prior1=True, flags=flags)
    b = M.disparity_many(L, R, Ds, Ks, 3, 2, 1e-6, soft_radius=3, with_prior1=True, flags=flags)
    torch.cuda.synchronize()
    _equal(ref, a, "a")
    _equal(ref, b, "b")


def test_graph_cache_evicts_least_recently_used(M):
    """More distinct calls than the graph cache holds (64 entries): each new
    call past the limit gives up the least recently replayed graph after its
    last replay ended; every call's output equals the direct path's, and a
    call whose graph was evicted is captured again and still equal."""
    rng = np.random.Generator(np.random.PCG64(11))
    L = torch.from_numpy(rng.integers(0, 256, (40, 72)).astype(np.uint8)).cuda()
    R = torch.from_numpy(rng.integers(0, 256, (40, 72)).astype(np.uint8)).cuda()
    n, r, eps, D, K = 2, 1, 0.065, 16, 2
    ref = M.disparity_many([L], [R], [D], [K], n, r, eps)
    flags = M.FLAG_BATCHED | M.FLAG_GRAPH
    keep = [M.disparity_many([L], [R], [D], [K], n, r, eps, flags=flags) for _ in range(70)]
    torch.cuda.synchronize()
    for i, got in enumerate(keep):
        _equal(ref, got, i)
    first = keep[0]
    for t in first[0].values():
        t.fill_(-5 if t.dtype == torch.int16 else 5.0)
    M.disparity_many([L], [R], [D], [K], n, r, eps, flags=flags, outputs=first)
    torch.cuda.synchronize()
    _equal(ref, first, "recaptured")


@pytest.mark.skip(reason=PERSISTENT_OFF)
@pytest.mark.parametrize("dtype,n,r,rs", [("u8", 4, 2, 0), ("u8", 3, 3, 0), ("f32", 5, 2, 0),
                                          ("f32", 3, 2, 3)])
def test_persistent_equals_plain(M, dtype, n, r, rs):
    pairs = _batch((dtype,), seed=n * 10 + r)
    eps = 0.065 if dtype == "u8" else 1e-6
    L, R, Ds, Ks = _inputs(pairs)
    plain = M.disparity_many(L, R, Ds, Ks, n, r, eps, soft_radius=rs, with_prior1=True)
    pers = M.disparity_many(L, R, Ds, Ks, n, r, eps, soft_radius=rs, with_prior1=True,
                            flags=M.FLAG_PERSISTENT)
    torch.cuda.synchronize()
    _equal(plain, pers)


@pytest.mark.skip(reason=PERSISTENT_OFF)
def test_persistent_graph_replay_repeats(M):
    pairs = _batch(("u8",), count=6, seed=3)
    L, R, Ds, Ks = _inputs(pairs)
    ref = M.disparity_many(L, R, Ds, Ks, 4, 2, 0.065)
    flags = M.FLAG_PERSISTENT | M.FLAG_GRAPH
    outs = M.disparity_many(L, R, Ds, Ks, 4, 2, 0.065, flags=flags)
    for rep in range(4):
        M.disparity_many(L, R, Ds, Ks, 4, 2, 0.065, flags=flags, outputs=outs)
        torch.cuda.synchronize()
        _equal(ref, outs, rep)


def test_batch32_full_size_sampled(M):
    """The 32-pair uneven batch at full size in the launch configuration the
    benchmark times (stage-batched, graph): identical to the per-pair path, and
    level 0 of four pairs (one per level count) checked on sampled pixels against
    the oracle fed the GPU's level-1 map."""
    import oracle
    from parity import check_pixels
    work = synth.batch_workload(32, 1000, workers=8)
    L = [dev(p.left) for p, _ in work]
    R = [dev(p.right) for p, _ in work]
    D = [c.max_disp for _, c in work]
    K = [c.levels for _, c in work]
    n, r, eps = work[0][1].half_window, work[0][1].refine_radius, work[0][1].var_eps
    print("batch32 full size, batched graph", flush=True)
    got = M.disparity_many(L, R, D, K, n, r, eps, with_prior1=True, flags=M.FLAG_BATCHED | M.FLAG_GRAPH)
    ref = M.disparity_many(L, R, D, K, n, r, eps, with_prior1=True)
    torch.cuda.synchronize()
    _equal(ref, got)
    picks = {}
    for i, k in enumerate(K):
        picks.setdefault(k, i)
    rng = np.random.Generator(np.random.PCG64(7))
    for k, i in sorted(picks.items()):
        if k < 2:
            continue
        p = work[i][0]
        H, W = p.left.shape
        ii = rng.integers(0, H, 1500)
        jj = rng.integers(0, W, 1500)
        d, C, p1 = (got[i][x].cpu().numpy() for x in ("disp", "cost", "prior1"))
        st = check_pixels(d, C, p.left, p.right, n, D[i], p1, r, eps, ii, jj)
        print(f"batch32 pair {i} ({W}x{H}, D={D[i]}, K={k})", st)
    # the same batch with the confidence gating and the median (the paper's
    # thresholds): the batched graph equals the per-pair path on every pair
    print("batch32 full size, gated + median, batched graph", flush=True)
    opts = dict(with_prior1=True, gate=(0.9, 0.9), median_alpha=0.9)
    got = M.disparity_many(L, R, D, K, n, r, eps, flags=M.FLAG_BATCHED | M.FLAG_GRAPH, **opts)
    ref = M.disparity_many(L, R, D, K, n, r, eps, **opts)
    torch.cuda.synchronize()
    _equal(ref, got)


def test_batched_median_uneven_pairs_equals_plain(M):
    """The selective median on the batched path, uneven pairs and depths, with
    and without the graph, with a soft level on float pairs: every output equals
    the plain path's."""
    import numpy as np
    from paper_1901_09593_amd import synth
    shapes = [(96, 150, 48, 0), (61, 200, 100, 0), (130, 90, 20, 2)]
    pairs = [synth.make_pair(700 + i, h, w, 3, 2, max(3, D // 2), True, 0.9, 5.0, 4.0, "u8")
             for i, (h, w, D, K) in enumerate(shapes)]
    L = [torch.from_numpy(p.left).cuda() for p in pairs]
    R = [torch.from_numpy(p.right).cuda() for p in pairs]
    Ds = [s[2] for s in shapes]
    Ks = [s[3] for s in shapes]
    plain = M.disparity_many(L, R, Ds, Ks, 3, 2, 0.065, with_prior1=True, median_alpha=0.9)
    for flags in (M.FLAG_BATCHED, M.FLAG_BATCHED | M.FLAG_GRAPH):
        for rep in range(2):
            got = M.disparity_many(L, R, Ds, Ks, 3, 2, 0.065, with_prior1=True, flags=flags, median_alpha=0.9)
            for a, b in zip(got, plain):
                assert torch.equal(a["disp"], b["disp"]) and torch.equal(a["cost"], b["cost"])
                if "prior1" in b:
                    assert torch.equal(a["prior1"], b["prior1"])
    # float pairs with the soft level: the median runs on the hard levels only
    fp = [synth.make_pair(710 + i, 80, 120, 3, 2, 12, True, 0.9, 0.02, 2 / 255, "f32") for i in range(2)]
    Lf = [torch.from_numpy(p.left).cuda() for p in fp]
    Rf = [torch.from_numpy(p.right).cuda() for p in fp]
    plain = M.disparity_many(Lf, Rf, [32, 32], [3, 3], 2, 2, 1e-6, soft_radius=2, tau=0.05, with_prior1=True,
                             median_alpha=0.9)
    got = M.disparity_many(Lf, Rf, [32, 32], [3, 3], 2, 2, 1e-6, soft_radius=2, tau=0.05, with_prior1=True,
                           flags=M.FLAG_BATCHED | M.FLAG_GRAPH, median_alpha=0.9)
    for a, b in zip(got, plain):
        for key in ("disp", "cost", "soft", "prior1"):
            assert torch.equal(a[key], b[key]), key


@pytest.mark.parametrize("median", [False, True])
def test_batched_gating_uneven_pairs_equals_plain(M, median):
    """The confidence gating (with and without the median) on the batched path
    and its graph, uneven pairs and depths (single-level pairs re-pick only):
    every output equals the plain path's."""
    import numpy as np
    from paper_1901_09593_amd import synth
    shapes = [(96, 150, 48, 0), (61, 200, 100, 0), (40, 70, 16, 1), (130, 90, 20, 2)]
    pairs = [synth.make_pair(720 + i, h, w, 3, 2, max(3, D // 2), True, 0.9, 5.0, 6.0, "u8")
             for i, (h, w, D, K) in enumerate(shapes)]
    L = [torch.from_numpy(p.left).cuda() for p in pairs]
    R = [torch.from_numpy(p.right).cuda() for p in pairs]
    Ds = [s[2] for s in shapes]
    Ks = [s[3] for s in shapes]
    ma = 0.9 if median else None
    plain = M.disparity_many(L, R, Ds, Ks, 3, 2, 0.065, with_prior1=True, gate=(0.9, 0.9), median_alpha=ma)
    for flags in (M.FLAG_BATCHED, M.FLAG_BATCHED | M.FLAG_GRAPH):
        for rep in range(2):
            got = M.disparity_many(L, R, Ds, Ks, 3, 2, 0.065, with_prior1=True, flags=flags, gate=(0.9, 0.9),
                                   median_alpha=ma)
            for a, b in zip(got, plain):
                assert torch.equal(a["disp"], b["disp"]) and torch.equal(a["cost"], b["cost"])
                if "prior1" in b:
                    assert torch.equal(a["prior1"], b["prior1"])
    # float pairs with the soft level: the gating runs on the hard levels only
    fp = [synth.make_pair(730 + i, 80, 120, 3, 2, 12, True, 0.9, 0.02, 4 / 255, "f32") for i in range(2)]
    Lf = [torch.from_numpy(p.left).cuda() for p in fp]
    Rf = [torch.from_numpy(p.right).cuda() for p in fp]
    kw = dict(soft_radius=2, tau=0.05, with_prior1=True, gate=(0.9, 0.9), median_alpha=ma)
    plain = M.disparity_many(Lf, Rf, [32, 32], [3, 3], 2, 2, 1e-6, **kw)
    got = M.disparity_many(Lf, Rf, [32, 32], [3, 3], 2, 2, 1e-6, flags=M.FLAG_BATCHED | M.FLAG_GRAPH, **kw)
    for a, b in zip(got, plain):
        for key in ("disp", "cost", "soft", "prior1"):
            assert torch.equal(a[key], b[key]), key
