"""GPU backward of the differentiable finest level against the FP64 oracle and
FP64 central finite differences (through the C ABI and the autograd wrapper)."""
import numpy as np
import pytest

import oracle
from paper_1901_09593_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

REL_TOL = 1e-3


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


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _mask(vis, n):
    """Loss pixels: visible in the right view, at least n pixels from the border."""
    m = vis.copy()
    m[:n, :] = m[-n:, :] = False
    m[:, :n] = m[:, -n:] = False
    return m


def _crop_case(H=180, W=320, seed=0):
    p, cfg = synth.workload("diff960", seed)
    return (np.ascontiguousarray(p.left[:H, :W]), np.ascontiguousarray(p.right[:H, :W]),
            p.disp[:H, :W], p.nonocc[:H, :W], cfg)


@pytest.mark.parametrize("n,rs", [(3, 3), (1, 1), (5, 2), (2, 4), (4, 3), (6, 1), (6, 3)])
def test_backward_matches_oracle(M, n, rs):
    L, R, gt, vis, cfg = _crop_case(96, 200)
    D, K, r, eps, tau = cfg.max_disp, cfg.levels, cfg.refine_radius, cfg.var_eps, cfg.tau
    out = M.disparity(dev(L), dev(R), D, K, n, r, eps, soft_radius=rs, tau=tau)
    p1 = host(out["prior1"])
    g = synth.grad_seed(1, *L.shape)
    gL, gR = M.backward(dev(L), dev(R), out["prior1"], dev(g.astype(np.float32)), D, K, n, r, eps, rs, tau)
    oL, oR = oracle.backward(L, R, n, D, p1, rs, tau, eps, g.astype(np.float32).astype(np.float64))
    eL, eR = rel(host(gL), oL), rel(host(gR), oR)
    print(f"n={n} rs={rs} rel error left {eL:.2e} right {eR:.2e}")
    assert eL <= REL_TOL and eR <= REL_TOL


def test_backward_sum_rules_and_repeatability(M):
    L, R, gt, vis, cfg = _crop_case(120, 256, seed=1)
    D, K, n, r, eps, rs, tau = cfg.max_disp, cfg.levels, cfg.half_window, cfg.refine_radius, \
        cfg.var_eps, cfg.soft_radius, cfg.tau
    out = M.disparity(dev(L), dev(R), D, K, n, r, eps, soft_radius=rs, tau=tau)
    g = dev(synth.grad_seed(2, *L.shape).astype(np.float32))
    a = M.backward(dev(L), dev(R), out["prior1"], g, D, K, n, r, eps, rs, tau)
    b = M.backward(dev(L), dev(R), out["prior1"], g, D, K, n, r, eps, rs, tau)
    for x, y, img in ((a[0], b[0], L), (a[1], b[1], R)):
        xs, ys = host(x).astype(np.float64), host(y).astype(np.float64)
        assert rel(xs, ys) < 1e-5  # only the atomic summation order differs
        scale = np.abs(xs).sum()
        assert abs(xs.sum()) < 1e-4 * scale
        assert abs((xs * img).sum()) < 1e-4 * scale * np.abs(img).max()


def test_backward_against_finite_differences(M):
    """GPU gradient vs FP64 central differences (eps 1e-6) of the oracle forward
    on a small crop pair whose right view is shifted so true matches stay inside."""
    p, cfg = synth.workload("diff960", 0)
    y0, x0, h, w = 200, 400, 40, 48
    s = int(np.floor(p.disp[y0:y0 + h, x0:x0 + w].min())) - 3
    L = np.ascontiguousarray(p.left[y0:y0 + h, x0:x0 + w]).astype(np.float32)
    R = np.ascontiguousarray(p.right[y0:y0 + h, x0 - s:x0 - s + w]).astype(np.float32)
    n, D, K, r, rs, tau, eps = 3, 24, 2, 2, 3, 0.05, cfg.var_eps
    out = M.disparity(dev(L), dev(R), D, K, n, r, eps, soft_radius=rs, tau=tau)
    p1 = host(out["prior1"])
    g = synth.grad_seed(3, h, w)
    gL, gR = M.backward(dev(L), dev(R), out["prior1"], dev(g.astype(np.float32)), D, K, n, r, eps, rs, tau)
    Ld, Rd, gd = L.astype(np.float64), R.astype(np.float64), g.astype(np.float32).astype(np.float64)

    def f(Lx, Rx):
        ds, *_ = oracle.soft_level0(Lx, Rx, n, D, p1, rs, tau, eps)
        return float((gd * ds).sum())

    hstep = 1e-6
    rng = np.random.Generator(np.random.PCG64(4))
    idx = [tuple(x) for x in np.stack([rng.integers(0, h, 300), rng.integers(0, w, 300)], 1)]
    for grad, which in ((host(gL), 0), (host(gR), 1)):
        fd = np.empty(len(idx))
        for k, (i, j) in enumerate(idx):
            e = np.zeros_like(Ld)
            e[i, j] = hstep
            if which == 0:
                fd[k] = (f(Ld + e, Rd) - f(Ld - e, Rd)) / (2 * hstep)
            else:
                fd[k] = (f(Ld, Rd + e) - f(Ld, Rd - e)) / (2 * hstep)
        got = np.array([grad[i, j] for i, j in idx], dtype=np.float64)
        err = rel(got, fd)
        print("view", which, "rel error vs finite differences", err)
        assert err <= REL_TOL


def test_autograd_loss_gradient(M):
    """MsibmFunction + a masked L1 loss in torch, against the oracle's loss
    gradient pushed through the oracle backward."""
    L, R, gt, vis, cfg = _crop_case(96, 192, seed=2)
    D, K, n, r, eps, rs, tau = cfg.max_disp, cfg.levels, cfg.half_window, cfg.refine_radius, \
        cfg.var_eps, cfg.soft_radius, cfg.tau
    Lt = dev(L).requires_grad_(True)
    Rt = dev(R).requires_grad_(True)
    dsoft, dhard = M.MsibmFunction.apply(Lt, Rt, D, K, n, r, eps, rs, tau)
    mask = dev(_mask(vis, n))
    loss = (dsoft - dev(gt.astype(np.float32))).abs()[mask].mean()
    loss.backward()
    p1 = M.disparity(dev(L), dev(R), D, K, n, r, eps, soft_radius=rs, tau=tau)["prior1"]
    ds_o, *_ = oracle.soft_level0(L, R, n, D, host(p1), rs, tau, eps)
    lo, go = oracle.l1_loss(ds_o, gt, oracle.loss_mask(vis, n))
    assert abs(float(loss.detach()) - lo) < 1e-3 * max(1.0, lo)
    oL, oR = oracle.backward(L, R, n, D, host(p1), rs, tau, eps, go)
    eL, eR = rel(host(Lt.grad), oL), rel(host(Rt.grad), oR)
    print("autograd rel error", eL, eR)
    assert eL <= REL_TOL and eR <= REL_TOL


def test_batched_backward_matches_plain_and_oracle(M):
    """Three uneven crops: the batched backward (and its graph replays) against the
    per-pair backward (same arithmetic, only the atomic order differs) and the
    oracle."""
    crops = [(96, 200, 0), (120, 256, 1), (64, 130, 2)]
    L, R, D, K = [], [], [], []
    for h, w, seed in crops:
        l, r_, _, _, cfg = _crop_case(h, w, seed)
        L.append(dev(l))
        R.append(dev(r_))
        D.append(cfg.max_disp)
        K.append(cfg.levels)
    n, r, eps, rs, tau = cfg.half_window, cfg.refine_radius, cfg.var_eps, cfg.soft_radius, cfg.tau
    outs = M.disparity_many(L, R, D, K, n, r, eps, soft_radius=rs, tau=tau, flags=M.FLAG_BATCHED)
    p1 = [o["prior1"] for o in outs]
    g = [dev(synth.grad_seed(5 + i, *x.shape).astype(np.float32)) for i, x in enumerate(L)]
    plain = M.backward_many(L, R, p1, g, D, K, n, r, eps, rs, tau)
    batched = M.backward_many(L, R, p1, g, D, K, n, r, eps, rs, tau, flags=M.FLAG_BATCHED)
    for (a, b), (c, d) in zip(plain, batched):
        assert rel(host(c), host(a)) < 1e-5 and rel(host(d), host(b)) < 1e-5
    flags = M.FLAG_BATCHED | M.FLAG_GRAPH
    gouts = M.backward_many(L, R, p1, g, D, K, n, r, eps, rs, tau, flags=flags)
    for rep in range(3):
        for o in gouts:
            o[0].fill_(5.0)
            o[1].fill_(-5.0)
        M.backward_many(L, R, p1, g, D, K, n, r, eps, rs, tau, flags=flags, outputs=gouts)
        torch.cuda.synchronize()
        for (a, b), (c, d) in zip(plain, gouts):
            assert rel(host(c), host(a)) < 1e-5 and rel(host(d), host(b)) < 1e-5, rep
    i = 2
    oL, oR = oracle.backward(host(L[i]), host(R[i]), n, D[i], host(p1[i]), rs, tau, eps,
                             host(g[i]).astype(np.float64))
    eL, eR = rel(host(batched[i][0]), oL), rel(host(batched[i][1]), oR)
    print("batched backward vs oracle", eL, eR)
    assert eL <= REL_TOL and eR <= REL_TOL


def test_hires2880_full_size_forward_backward(M):
    """The 4 x 2880x1988 forward + backward at full size, in the launch
    configuration the benchmark times (stage-batched, graph): pair 0's soft
    disparities against the oracle fed the GPU's level-1 map; every pair's
    batched gradients against its per-pair ones and against the invariances of
    ZNCC to the offset and scale of each image (properties at any size: the
    oracle's full-size backward takes tens of seconds)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(4) as ex:
        work = list(ex.map(lambda i: synth.workload("hires2880", i), range(4)))
    cfg = work[0][1]
    n, r, eps, rs, tau, D, K = cfg.half_window, cfg.refine_radius, cfg.var_eps, cfg.soft_radius, cfg.tau, \
        cfg.max_disp, cfg.levels
    L = [dev(p.left) for p, _ in work]
    R = [dev(p.right) for p, _ in work]
    Ds, Ks = [D] * 4, [K] * 4
    flags = M.FLAG_BATCHED | M.FLAG_GRAPH
    print("hires2880 full size, batched graph", flush=True)
    outs = M.disparity_many(L, R, Ds, Ks, n, r, eps, soft_radius=rs, tau=tau, flags=flags)
    p1 = [o["prior1"] for o in outs]
    g = [dev(synth.grad_seed(20 + i, *x.shape).astype(np.float32)) for i, x in enumerate(L)]
    grads = M.backward_many(L, R, p1, g, Ds, Ks, n, r, eps, rs, tau, flags=flags)
    plain = M.backward_many(L, R, p1, g, Ds, Ks, n, r, eps, rs, tau)
    for i, ((a, b), (c, d)) in enumerate(zip(grads, plain)):
        for x, y, img in ((a, c, work[i][0].left), (b, d, work[i][0].right)):
            xs = host(x).astype(np.float64)
            assert np.isfinite(xs).all()
            assert rel(xs, host(y)) < 1e-5, i  # only the atomic summation order differs
            scale = np.abs(xs).sum()
            assert abs(xs.sum()) < 1e-4 * scale
            assert abs((xs * img).sum()) < 1e-4 * scale * np.abs(img).max()
    l0, r0, q1 = host(L[0]), host(R[0]), host(p1[0])
    ds_o, dh_o, C_o, C2_o = oracle.soft_level0(l0, r0, n, D, q1, rs, tau, eps)
    err = float(np.abs(host(outs[0]["soft"]).astype(np.float64) - ds_o).max())
    print("hires2880 soft max |dd|", err)
    assert err <= 1e-2


def test_backward_linearity_zero_and_locality(M):
    """The gradient is linear in the upstream gradient g: power-of-two scalings
    of g (2^40 and 2^-40) pass through the per-chunk fixed-point scale, g = 0
    gives exactly zero, and a single-pixel g reaches only that pixel's window
    (left) and its windows at the candidates (right)."""
    L, R, gt, vis, cfg = _crop_case(64, 160, seed=4)
    D, K, n, r, eps, rs, tau = cfg.max_disp, cfg.levels, cfg.half_window, cfg.refine_radius, \
        cfg.var_eps, cfg.soft_radius, cfg.tau
    out = M.disparity(dev(L), dev(R), D, K, n, r, eps, soft_radius=rs, tau=tau)
    g = synth.grad_seed(5, *L.shape).astype(np.float32)

    def bw(gg):
        gL, gR = M.backward(dev(L), dev(R), out["prior1"], dev(gg), D, K, n, r, eps, rs, tau)
        return host(gL).astype(np.float64), host(gR).astype(np.float64)
    aL, aR = bw(g)
    for k in (40, -40):
        bL, bR = bw((g * np.float32(2.0 ** k)).astype(np.float32))
        assert rel(bL * 2.0 ** -k, aL) < 1e-5 and rel(bR * 2.0 ** -k, aR) < 1e-5, k
    zL, zR = bw(np.zeros_like(g))
    assert not zL.any() and not zR.any()
    i, j = 30, 100
    one = np.zeros_like(g)
    one[i, j] = 1.0
    sL, sR = bw(one)
    ys, xs = np.nonzero(sL)
    assert len(ys) > 0
    assert ys.min() >= i - n and ys.max() <= i + n and xs.min() >= j - n and xs.max() <= j + n
    ys, xs = np.nonzero(sR)
    assert len(ys) > 0
    assert ys.min() >= i - n and ys.max() <= i + n and xs.min() >= j - (D - 1) - n and xs.max() <= j + n
