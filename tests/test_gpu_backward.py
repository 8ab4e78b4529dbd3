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


def _crop_case(H=180, W=320, seed=0):
    p, cfg = synth.workload("diff960", seed)
    return (np.ascontiguousarray(p.left[:H, :W]), np.ascontiguousarray(p.right[:H, :W]),
            p.disp[:H, :W], p.nonocc[:H, :W], cfg)


@pytest.mark.parametrize("n,rs", [(3, 3), (1, 1), (5, 2), (5, 3), (2, 4), (4, 3), (6, 1), (6, 3)])
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


def _planar_crop(p, h, w, step=16):
    """First crop (even corner, scanning rows then columns) whose ground truth is
    one exact plane (inside one slanted segment, unclipped) and fully visible."""
    H, W = p.disp.shape
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    A = np.stack([np.ones(h * w), xx.ravel(), yy.ravel()], 1)
    for y0 in range(32, H - h - 32, step):
        for x0 in range(160, W - w - 32, step):
            d = p.disp[y0:y0 + h, x0:x0 + w]
            if not p.nonocc[y0:y0 + h, x0:x0 + w].all():
                continue
            coef, *_ = np.linalg.lstsq(A, d.ravel(), rcond=None)
            if np.abs(A @ coef - d.ravel()).max() < 1e-9:
                return y0, x0
    raise AssertionError("no planar crop")


def test_backward_against_finite_differences(M):
    """The gradient pin of the differentiable workload: on a 64 x 48 crop pair of
    the 960x540 float pair 0, the GPU gradient of the masked mean-L1 loss against
    FP64 central differences (step 1e-6) of the oracle forward at every one of
    the 2 x 3072 inputs.  The left crop lies inside one planar segment; the right
    crop is shifted by s (even, at least the soft radius below the smallest
    doubled prior) so the true matches stay inside it; the prior is the
    full-image run's level-1 map shifted by s / 2 (clipped per pixel by the
    candidate-interval rule)."""
    p, cfg = synth.workload("diff960", 0)
    D, K, n, r, rs, tau, eps = cfg.max_disp, cfg.levels, cfg.half_window, cfg.refine_radius, \
        cfg.soft_radius, cfg.tau, cfg.var_eps
    full = M.disparity(dev(p.left), dev(p.right), D, K, n, r, eps, soft_radius=rs, tau=tau)
    P1 = host(full["prior1"]).astype(np.int64)
    h, w = 48, 64
    y0, x0 = _planar_crop(p, h, w)
    d1 = P1[y0 // 2:(y0 + h) // 2, x0 // 2:(x0 + w) // 2]
    s = 2 * int(d1.min()) - rs - 1          # even: the doubled prior minus rs + 1
    assert s % 2 == 0 and s > 0 and x0 - s >= 0
    p1 = (d1 - s // 2).astype(np.int16)
    Dc = int(2 * p1.max()) + rs + 1          # no candidate clipped by the range
    L = np.ascontiguousarray(p.left[y0:y0 + h, x0:x0 + w])
    R = np.ascontiguousarray(p.right[y0:y0 + h, x0 - s:x0 - s + w])
    gt = p.disp[y0:y0 + h, x0:x0 + w] - s
    mask = synth.loss_mask(np.ones((h, w), bool), n, Dc)
    assert mask.sum() > h * w // 2
    Ld, Rd = L.astype(np.float64), R.astype(np.float64)
    ds_o, *_ = oracle.soft_level0(Ld, Rd, n, Dc, p1, rs, tau, eps)
    loss, gd = oracle.l1_loss(ds_o, gt, mask)
    assert np.abs(ds_o - gt)[mask].min() > 1e-5  # the sign pattern is locally constant
    gL, gR = M.backward(dev(L), dev(R), dev(p1), dev(gd.astype(np.float32)), Dc, K, n, r, eps, rs, tau)
    gd32 = gd.astype(np.float32).astype(np.float64)

    def f(Lx, Rx):
        ds, *_ = oracle.soft_level0(Lx, Rx, n, Dc, p1, rs, tau, eps)
        return float((gd32 * ds).sum())

    hstep = 1e-6

    def column(which, i):
        out = np.empty(w)
        for j in range(w):
            e = np.zeros_like(Ld)
            e[i, j] = hstep
            if which == 0:
                out[j] = (f(Ld + e, Rd) - f(Ld - e, Rd)) / (2 * hstep)
            else:
                out[j] = (f(Ld, Rd + e) - f(Ld, Rd - e)) / (2 * hstep)
        return out
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(16, initializer=oracle.set_threads, initargs=(1,)) as ex:
        fdL = np.stack(list(ex.map(lambda i: column(0, i), range(h))))
        fdR = np.stack(list(ex.map(lambda i: column(1, i), range(h))))
    oracle.set_threads(oracle.num_threads())
    for grad, fd, which in ((host(gL), fdL, "left"), (host(gR), fdR, "right")):
        err = rel(grad.astype(np.float64), fd)
        print(f"crop at ({y0}, {x0}), shift {s}: {which} rel error vs finite differences {err:.2e} "
              f"over {fd.size} inputs")
        assert err <= REL_TOL
    # and the oracle's own gradient agrees with its finite differences
    oL, oR = oracle.backward(Ld, Rd, n, Dc, p1, rs, tau, eps, gd32)
    assert rel(oL, fdL) < 1e-6 and rel(oR, fdR) < 1e-6


def test_autograd_loss_gradient(M):
    """MsibmFunction + a masked L1 loss in torch, against the oracle's loss
    gradient pushed through the oracle backward."""
    L, R, gt, vis, cfg = _crop_case(96, 192, seed=2)
    D, K, n, r, eps, rs, tau = cfg.max_disp, cfg.levels, cfg.half_window, cfg.refine_radius, \
        cfg.var_eps, cfg.soft_radius, cfg.tau
    Lt = dev(L).requires_grad_(True)
    Rt = dev(R).requires_grad_(True)
    dsoft, dhard = M.MsibmFunction.apply(Lt, Rt, D, K, n, r, eps, rs, tau)
    mask = dev(synth.loss_mask(vis, n, D))
    loss = (dsoft - dev(gt.astype(np.float32))).abs()[mask].mean()
    loss.backward()
    p1 = M.disparity(dev(L), dev(R), D, K, n, r, eps, soft_radius=rs, tau=tau)["prior1"]
    ds_o, *_ = oracle.soft_level0(L, R, n, D, host(p1), rs, tau, eps)
    lo, go = oracle.l1_loss(ds_o, gt, synth.loss_mask(vis, n, D))
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


def _band_rows(i0, i1, n, H):
    """Output rows whose gradient comes only from source rows [i0, i1): a source
    row's windows span n rows either side, and clamped reads at the top and
    bottom edges land on rows 0 and H - 1."""
    return (0 if i0 == 0 else i0 + n), (H if i1 >= H else i1 - n)


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
    # gradient rows against the oracle: a band of source rows [i0, i1) fixes the
    # gradient exactly on the rows whose windows reach no other source row
    for i, (i0, i1) in ((0, (980, 1040)), (3, (0, 44))):
        li, ri, qi, gi = host(L[i]), host(R[i]), host(p1[i]), host(g[i]).astype(np.float64)
        oL, oR = oracle.backward(li, ri, n, D, qi, rs, tau, eps, gi, rows=(i0, i1))
        a, b = _band_rows(i0, i1, n, li.shape[0])
        eL = rel(host(grads[i][0])[a:b].astype(np.float64), oL[a:b])
        eR = rel(host(grads[i][1])[a:b].astype(np.float64), oR[a:b])
        print(f"hires2880 pair {i} gradient rows {a}..{b - 1}: rel error left {eL:.2e} right {eR:.2e}")
        assert eL <= REL_TOL and eR <= REL_TOL


def test_diff960x8_full_size_forward_loss_backward(M):
    """The 8 x 960x540 forward, masked mean-L1 loss gradient and backward at full
    size, in the launch configuration the benchmark times (stage-batched,
    graph): every pair's soft disparities against the oracle fed the GPU's
    level-1 map, the loss gradient against the oracle's, and bands of gradient
    rows of three pairs against the oracle's backward of the same upstream
    gradient restricted to the band's source rows."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(8) as ex:
        work = list(ex.map(lambda i: synth.workload("diff960", i), range(8)))
    cfg = work[0][1]
    n, r, eps, rs, tau, D, K = cfg.half_window, cfg.refine_radius, cfg.var_eps, cfg.soft_radius, cfg.tau, \
        cfg.max_disp, cfg.levels
    L = [dev(p.left) for p, _ in work]
    R = [dev(p.right) for p, _ in work]
    gts = [dev(p.disp.astype(np.float32)) for p, _ in work]
    masks = [dev(synth.loss_mask(p.nonocc, n, D)) for p, _ in work]
    Ds, Ks = [D] * 8, [K] * 8
    flags = M.FLAG_BATCHED | M.FLAG_GRAPH
    print("diff960 x 8 full size, batched graph", flush=True)
    outs = M.disparity_many(L, R, Ds, Ks, n, r, eps, soft_radius=rs, tau=tau, flags=flags)
    p1 = [o["prior1"] for o in outs]
    g = [torch.sign(o["soft"] - t) * m / m.sum().clamp(min=1) for o, t, m in zip(outs, gts, masks)]
    grads = M.backward_many(L, R, p1, g, Ds, Ks, n, r, eps, rs, tau, flags=flags)
    for i, (p, _) in enumerate(work):
        li, ri, qi = host(L[i]), host(R[i]), host(p1[i])
        ds_o, *_ = oracle.soft_level0(li, ri, n, D, qi, rs, tau, eps)
        ds = host(outs[i]["soft"]).astype(np.float64)
        err = float(np.abs(ds - ds_o).max())
        mask = synth.loss_mask(p.nonocc, n, D)
        lo, go = oracle.l1_loss(ds_o, p.disp, mask)
        firm = np.abs(ds_o - p.disp) > 1e-2  # the sign is fixed where d_soft is farther than its tolerance
        gi = host(g[i]).astype(np.float64)
        assert np.allclose(gi[firm], go[firm], rtol=1e-6, atol=0), i
        print(f"diff960 pair {i}: soft max |dd| {err:.2e}, loss {lo:.4f}")
        assert err <= 1e-2
        if i in (0, 3, 7):
            i0, i1 = (40, 100) if i != 7 else (470, 540)
            oL, oR = oracle.backward(li, ri, n, D, qi, rs, tau, eps, gi, rows=(i0, i1))
            a, b = _band_rows(i0, i1, n, li.shape[0])
            eL = rel(host(grads[i][0])[a:b].astype(np.float64), oL[a:b])
            eR = rel(host(grads[i][1])[a:b].astype(np.float64), oR[a:b])
            print(f"  gradient rows {a}..{b - 1}: rel error left {eL:.2e} right {eR:.2e}")
            assert eL <= REL_TOL and eR <= REL_TOL


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
