"""The fused forward + masked-L1 loss + backward (msibm_fwd_bwd_l1) against the
separate calls it replaces (forward, the loss gradient formed in torch,
msibm_backward) and against the FP64 oracle, on the plain, the stage-batched
and the graph-replayed paths, at small sizes and at the full 4 x 2880x1988 and
8 x 960x540 sizes."""
import numpy as np
import pytest

import oracle
from paper_1901_09593_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

REL_TOL = 1e-3
# d_soft of the fused kernel against the forward's soft level: both are within
# about 1e-6 of the FP64 scores, summed in another order; the softmax turns a
# score difference into at most (2 r_s / tau) times as much disparity (120 px
# per unit score at r_s = 3, tau = 0.05)
SOFT_TOL = 1e-3


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


def _band_rows(i0, i1, n, H):
    """Gradient rows fixed by source rows [i0, i1) alone: their windows (rows
    within n) reach no source row outside the band."""
    a = 0 if i0 == 0 else i0 + n
    b = H if i1 == H else i1 - n
    return a, b


def _pairs(count, H, W, D, seed0=40):
    out = []
    for i in range(count):
        p = synth.make_pair(seed0 + i, H - 7 * i, W - 11 * i, 5, 0.05 * D, 0.85 * D, True, 0.95, 0.02,
                            2.0 / 255, "f32")
        out.append(p)
    return out


def _separate(M, L, R, gts, masks, Ds, Ks, n, r, eps, rs, tau, flags, soft_for_sign=None):
    """Forward, loss gradient in torch (from `soft_for_sign` when given, so that
    both sides take the same signs), backward."""
    outs = M.disparity_many(L, R, Ds, Ks, n, r, eps, soft_radius=rs, tau=tau, flags=flags)
    soft = soft_for_sign if soft_for_sign is not None else [o["soft"] for o in outs]
    g = [torch.sign(s - t) * m.float() * (1.0 / m.float().sum().clamp(min=1)) for s, t, m in zip(soft, gts, masks)]
    grads = M.backward_many(L, R, [o["prior1"] for o in outs], g, Ds, Ks, n, r, eps, rs, tau, flags=flags)
    return outs, g, grads


@pytest.mark.parametrize("flags_name", ["plain", "batched", "graph"])
def test_fused_equals_separate_calls(M, flags_name):
    flags = {"plain": 0, "batched": M.FLAG_BATCHED, "graph": M.FLAG_BATCHED | M.FLAG_GRAPH}[flags_name]
    n, r, rs, tau, eps = 3, 2, 3, 0.05, 1e-6
    D = 48
    pairs = _pairs(3, 140, 230, D)
    L = [dev(p.left) for p in pairs]
    R = [dev(p.right) for p in pairs]
    gts = [dev(p.disp.astype(np.float32)) for p in pairs]
    masks = [dev(synth.loss_mask(p.nonocc, n, D).astype(np.uint8)) for p in pairs]
    Ds, Ks = [D] * 3, [0, 2, 3]
    print(f"fused vs separate ({flags_name})", flush=True)
    fused = M.fwd_bwd_l1(L, R, gts, masks, Ds, Ks, n, r, eps, rs, tau, flags=flags, with_cost=True)
    if flags & M.FLAG_GRAPH:  # a replay into the same buffers gives the same outputs
        first = [{k: v.clone() for k, v in o.items()} for o in fused]
        for o in fused:
            for t in o.values():
                t.fill_(-3 if t.dtype == torch.int16 else 3.0)
        M.fwd_bwd_l1(L, R, gts, masks, Ds, Ks, n, r, eps, rs, tau, flags=flags, with_cost=True, outputs=fused)
        for a, b in zip(first, fused):
            for k in ("disp", "soft", "prior1", "cost"):
                assert torch.equal(a[k], b[k]), k
            for k in ("grad_left", "grad_right", "loss"):
                assert rel(host(b[k]).astype(np.float64), host(a[k]).astype(np.float64)) < 1e-5, k
    outs, g, grads = _separate(M, L, R, gts, masks, Ds, Ks, n, r, eps, rs, tau, flags,
                               soft_for_sign=[o["soft"] for o in fused])
    for i, (f, o) in enumerate(zip(fused, outs)):
        # levels K-1..1 run the same kernels
        assert torch.equal(f["prior1"], o["prior1"]), i
        # the soft level: the fused kernel sums its windows in another order
        ds = float((f["soft"] - o["soft"]).abs().max())
        mism = float((f["disp"] != o["disp"]).float().mean())
        assert ds <= SOFT_TOL and mism <= 1e-3, (i, ds, mism)
        cnt = float(masks[i].float().sum().clamp(min=1))
        loss = float(((f["soft"] - gts[i]).abs() * masks[i].float()).sum()) / cnt
        assert abs(float(f["loss"]) - loss) <= 1e-5 * max(1.0, loss), (i, float(f["loss"]), loss)
        eL = rel(host(f["grad_left"]).astype(np.float64), host(grads[i][0]).astype(np.float64))
        eR = rel(host(f["grad_right"]).astype(np.float64), host(grads[i][1]).astype(np.float64))
        print(f"pair {i}: soft max diff {ds:.1e}, winner mismatch {mism:.1e}, gradient rel diff {eL:.1e} {eR:.1e}")
        assert eL <= 1e-4 and eR <= 1e-4, (i, eL, eR)


def test_fused_against_oracle(M):
    n, r, rs, tau, eps = 4, 2, 3, 0.05, 1e-6
    p, cfg = synth.workload("diff960", 2)
    H, W = 110, 300
    li, ri = np.ascontiguousarray(p.left[:H, :W]), np.ascontiguousarray(p.right[:H, :W])
    gt = p.disp[:H, :W]
    D = cfg.max_disp
    K = cfg.levels
    mask = synth.loss_mask(p.nonocc[:H, :W], n, D)
    print("fused vs oracle", flush=True)
    f, = M.fwd_bwd_l1([dev(li)], [dev(ri)], [dev(gt.astype(np.float32))], [dev(mask.astype(np.uint8))], [D], [K],
                      n, r, eps, rs, tau)
    q1 = host(f["prior1"])
    ds_o, dh_o, C_o, _ = oracle.soft_level0(li, ri, n, D, q1, rs, tau, eps)
    ds = host(f["soft"]).astype(np.float64)
    assert float(np.abs(ds - ds_o).max()) <= 1e-2
    lo, go = oracle.l1_loss(ds_o, gt, mask)
    assert abs(float(f["loss"]) - lo) <= 1e-2
    # the gradient of the GPU's own loss: the oracle's backward of the same signs
    cnt = max(int(mask.sum()), 1)
    g = np.where(mask, np.sign(ds - gt), 0.0) * np.float64(np.float32(1.0) / np.float32(cnt))
    oL, oR = oracle.backward(li, ri, n, D, q1, rs, tau, eps, g)
    eL, eR = rel(host(f["grad_left"]).astype(np.float64), oL), rel(host(f["grad_right"]).astype(np.float64), oR)
    print(f"fused vs oracle: soft max {np.abs(ds - ds_o).max():.2e}, rel error {eL:.2e} {eR:.2e}")
    assert eL <= REL_TOL and eR <= REL_TOL


def test_fused_empty_mask_gives_zero_gradient(M):
    n, r, rs, tau, eps, D = 3, 2, 3, 0.05, 1e-6, 40
    p, = _pairs(1, 96, 160, D, seed0=77)
    z = np.zeros(p.left.shape, dtype=np.uint8)
    f, = M.fwd_bwd_l1([dev(p.left)], [dev(p.right)], [dev(p.disp.astype(np.float32))], [dev(z)], [D], [0], n, r,
                      eps, rs, tau, flags=M.FLAG_BATCHED)
    assert float(f["loss"]) == 0.0
    assert float(f["grad_left"].abs().max()) == 0.0 and float(f["grad_right"].abs().max()) == 0.0
    o, = M.disparity_many([dev(p.left)], [dev(p.right)], [D], [0], n, r, eps, soft_radius=rs, tau=tau)
    assert float((f["soft"] - o["soft"]).abs().max()) <= SOFT_TOL


def test_fused_hires2880_full_size(M):
    """The 4 x 2880x1988 fused step at full size in the benchmark's launch
    configuration (batched, graph): every pair's loss and gradients against
    the separate batched calls fed the fused step's signs, pair 0's soft
    disparities against the oracle, and bands of gradient rows against the
    oracle's backward restricted to the band's source rows."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(4) as ex:
        work = list(ex.map(lambda i: synth.workload("hires2880", i), range(4)))
    cfg = work[0][1]
    n, r, eps, rs, tau, D, K = cfg.half_window, cfg.refine_radius, cfg.var_eps, cfg.soft_radius, cfg.tau, \
        cfg.max_disp, cfg.levels
    L = [dev(p.left) for p, _ in work]
    R = [dev(p.right) for p, _ in work]
    gts = [dev(p.disp.astype(np.float32)) for p, _ in work]
    masks = [dev(synth.loss_mask(p.nonocc, n, D).astype(np.uint8)) for p, _ in work]
    Ds, Ks = [D] * 4, [K] * 4
    flags = M.FLAG_BATCHED | M.FLAG_GRAPH
    print("hires2880 x 4 fused, batched graph", flush=True)
    fused = M.fwd_bwd_l1(L, R, gts, masks, Ds, Ks, n, r, eps, rs, tau, flags=flags)
    outs, g, grads = _separate(M, L, R, gts, masks, Ds, Ks, n, r, eps, rs, tau, flags,
                               soft_for_sign=[o["soft"] for o in fused])
    for i, (f, o) in enumerate(zip(fused, outs)):
        assert torch.equal(f["prior1"], o["prior1"]), i
        ds = float((f["soft"] - o["soft"]).abs().max())
        print(f"hires2880 pair {i}: fused vs forward soft max diff {ds:.2e}")
        assert ds <= SOFT_TOL, (i, ds)
        for a, b in ((f["grad_left"], grads[i][0]), (f["grad_right"], grads[i][1])):
            assert rel(host(a).astype(np.float64), host(b).astype(np.float64)) < 1e-4, i
    l0, r0, q1 = host(L[0]), host(R[0]), host(fused[0]["prior1"])
    ds_o, *_ = oracle.soft_level0(l0, r0, n, D, q1, rs, tau, eps)
    ds0 = host(fused[0]["soft"]).astype(np.float64)
    assert float(np.abs(ds0 - ds_o).max()) <= 1e-2
    mask0 = synth.loss_mask(work[0][0].nonocc, n, D)
    lo, _ = oracle.l1_loss(ds_o, work[0][0].disp, mask0)
    assert abs(float(fused[0]["loss"]) - lo) <= 1e-2
    for i, (i0, i1) in ((0, (600, 660)), (2, (1940, 1988))):
        li, ri, qi = host(L[i]), host(R[i]), host(fused[i]["prior1"])
        gi = host(g[i]).astype(np.float64)
        oL, oR = oracle.backward(li, ri, n, D, qi, rs, tau, eps, gi, rows=(i0, i1))
        a, b = _band_rows(i0, i1, n, li.shape[0])
        eL = rel(host(fused[i]["grad_left"])[a:b].astype(np.float64), oL[a:b])
        eR = rel(host(fused[i]["grad_right"])[a:b].astype(np.float64), oR[a:b])
        print(f"hires2880 pair {i} fused gradient rows {a}..{b - 1}: rel error left {eL:.2e} right {eR:.2e}")
        assert eL <= REL_TOL and eR <= REL_TOL


def test_fused_diff960x8_full_size(M):
    """The 8 x 960x540 fused step at full size (batched, graph): every pair's
    soft disparities against the oracle fed the GPU's level-1 map, its loss
    against the oracle's loss of those, and bands of gradient rows of two pairs
    against the oracle's backward of the fused step's own loss gradient."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(8) as ex:
        work = list(ex.map(lambda i: synth.workload("diff960", i), range(8)))
    cfg = work[0][1]
    n, r, eps, rs, tau, D, K = cfg.half_window, cfg.refine_radius, cfg.var_eps, cfg.soft_radius, cfg.tau, \
        cfg.max_disp, cfg.levels
    L = [dev(p.left) for p, _ in work]
    R = [dev(p.right) for p, _ in work]
    gts = [dev(p.disp.astype(np.float32)) for p, _ in work]
    mk = [synth.loss_mask(p.nonocc, n, D) for p, _ in work]
    masks = [dev(m.astype(np.uint8)) for m in mk]
    print("diff960 x 8 fused, batched graph", flush=True)
    fused = M.fwd_bwd_l1(L, R, gts, masks, [D] * 8, [K] * 8, n, r, eps, rs, tau,
                         flags=M.FLAG_BATCHED | M.FLAG_GRAPH)
    for i, (p, _) in enumerate(work):
        li, ri, qi = host(L[i]), host(R[i]), host(fused[i]["prior1"])
        ds_o, *_ = oracle.soft_level0(li, ri, n, D, qi, rs, tau, eps)
        ds = host(fused[i]["soft"]).astype(np.float64)
        err = float(np.abs(ds - ds_o).max())
        lo, _ = oracle.l1_loss(ds_o, p.disp, mk[i])
        print(f"diff960 pair {i}: soft max |dd| {err:.2e}, loss {float(fused[i]['loss']):.5f} (oracle {lo:.5f})")
        assert err <= 1e-2 and abs(float(fused[i]["loss"]) - lo) <= 1e-2
        if i in (1, 6):
            cnt = max(int(mk[i].sum()), 1)
            g = np.where(mk[i], np.sign(ds - p.disp), 0.0) * np.float64(np.float32(1.0) / np.float32(cnt))
            i0, i1 = (200, 260) if i == 1 else (0, 50)
            oL, oR = oracle.backward(li, ri, n, D, qi, rs, tau, eps, g, rows=(i0, i1))
            a, b = _band_rows(i0, i1, n, li.shape[0])
            eL = rel(host(fused[i]["grad_left"])[a:b].astype(np.float64), oL[a:b])
            eR = rel(host(fused[i]["grad_right"])[a:b].astype(np.float64), oR[a:b])
            print(f"  fused gradient rows {a}..{b - 1}: rel error left {eL:.2e} right {eR:.2e}")
            assert eL <= REL_TOL and eR <= REL_TOL
