"""GPU parity of the soft output at every level (an extension of the paper):
the pyramid adjoint, the every-level soft forward and the backward through all
levels, against the FP64 oracle (through the C ABI)."""
import numpy as np
import pytest

import oracle
from paper_1901_09593_amd import synth
from parity import check_level

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


@pytest.mark.parametrize("H,W", [(9, 14), (10, 7), (1, 5), (2, 1), (99, 131), (540, 960)])
def test_pyramid_adjoint_matches_oracle_and_accumulates(M, H, W):
    rng = np.random.Generator(np.random.PCG64(H * 1000 + W))
    G = rng.standard_normal(((H + 1) // 2, (W + 1) // 2)).astype(np.float32)
    base = rng.standard_normal((H, W)).astype(np.float32)
    got = host(M.pyramid_adjoint(dev(G), H, W, dev(base)))
    ref = base.astype(np.float64) + oracle.reduce_adjoint(G.astype(np.float64), H, W)
    assert np.abs(got - ref).max() <= 1e-5 * max(1.0, np.abs(ref).max())


def _case(seed=0, H=120, W=200):
    p, cfg = synth.workload("diff960", seed)
    return np.ascontiguousarray(p.left[:H, :W]), np.ascontiguousarray(p.right[:H, :W]), cfg


@pytest.mark.parametrize("K,n,rs", [(3, 3, 3), (4, 2, 1), (2, 1, 2)])
def test_soft_every_level_matches_oracle(M, K, n, rs):
    """Each soft level against the oracle's soft level on the GPU's own pyramid
    images and prior (teacher forcing); the hard maps follow the oracle except
    at near ties."""
    L, R, cfg = _case(K)
    D, eps, tau = 64, cfg.var_eps, cfg.tau
    soft, maps = M.disparity_levels(dev(L), dev(R), D, K, n, eps, rs, tau)
    PL, PR = M.pyramid(dev(L), K), M.pyramid(dev(R), K)
    for k in range(K - 1):
        Lk, Rk = host(PL[k]).astype(np.float64), host(PR[k]).astype(np.float64)
        Dk = -(-D // (1 << k))
        prior = host(maps[k + 1])
        ds_o, dh_o, C_o, C2_o = oracle.soft_level0(Lk, Rk, n, Dk, prior, rs, tau, eps)
        err = np.abs(host(soft[k]).astype(np.float64) - ds_o).max()
        print(f"K={K} level {k}: max |d_soft - oracle| = {err:.2e}")
        assert err <= 1e-2
        check_level(host(maps[k]), None, Lk, Rk, n, Dk, prior, rs, eps, ref=(dh_o, C_o, C2_o))
    # the coarsest map is the full search
    kc = K - 1
    Lc, Rc = host(PL[kc]).astype(np.float64), host(PR[kc]).astype(np.float64)
    check_level(host(maps[kc]), None, Lc, Rc, n, -(-D // (1 << kc)), None, 0, eps)
    # level 0 equals the existing soft level of the plain forward
    out = M.disparity(dev(L), dev(R), D, K, n, rs, eps, soft_radius=rs, tau=tau, with_prior1=True)
    if K >= 3:
        assert torch.equal(out["prior1"], maps[1])
        assert torch.equal(out["soft"], soft[0]) and torch.equal(out["disp"], maps[0])


@pytest.mark.parametrize("K,n,rs,skip", [(3, 3, 3, None), (4, 2, 2, 1), (3, 1, 1, 0)])
def test_backward_every_level_matches_oracle(M, K, n, rs, skip):
    """The gradient through every level (with one level's loss left out in two
    cases) against the oracle's chain of per-level backwards and reduce
    adjoints, the GPU's hard maps held fixed."""
    L, R, cfg = _case(10 + K, 96, 160)
    D, eps, tau = 48, cfg.var_eps, cfg.tau
    soft, maps = M.disparity_levels(dev(L), dev(R), D, K, n, eps, rs, tau)
    rng = np.random.Generator(np.random.PCG64(7 + K))
    grads = [None if k == skip else rng.standard_normal(tuple(soft[k].shape)).astype(np.float32)
             for k in range(K - 1)]
    gL, gR = M.backward_levels(dev(L), dev(R), maps, [None if g is None else dev(g) for g in grads], D, K, n,
                               eps, rs, tau)
    hm = [host(m) for m in maps]
    oL, oR = oracle.backward_levels(L, R, D, K, n, rs, tau, eps, hm,
                                    [None if g is None else g.astype(np.float64) for g in grads] + [None])
    eL, eR = rel(host(gL), oL), rel(host(gR), oR)
    print(f"K={K} n={n} rs={rs} skip={skip}: rel error left {eL:.2e} right {eR:.2e}")
    assert eL <= REL_TOL and eR <= REL_TOL
    # only level 0's loss: the existing single-level backward
    only0 = [grads[0] if grads[0] is not None else rng.standard_normal(tuple(soft[0].shape)).astype(np.float32)]
    only0 += [None] * (K - 2)
    aL, aR = M.backward_levels(dev(L), dev(R), maps, [None if g is None else dev(g) for g in only0], D, K, n,
                               eps, rs, tau)
    bL, bR = M.backward(dev(L), dev(R), maps[1], dev(only0[0]), D, K, n, rs, eps, rs, tau)
    assert rel(host(aL), host(bL)) < 1e-5 and rel(host(aR), host(bR)) < 1e-5


def test_levels_reject_bad_calls(M):
    L = torch.zeros((32, 48), dtype=torch.float32, device="cuda")
    with pytest.raises(M.MsibmError):
        M.disparity_levels(L, L, 16, 1, 2, 1e-6, 1, 0.05)   # K = 1
    with pytest.raises(M.MsibmError):
        M.disparity_levels(L, L, 16, 3, 2, 1e-6, 0, 0.05)   # no soft radius
    Lu = torch.zeros((32, 48), dtype=torch.uint8, device="cuda")
    with pytest.raises(M.MsibmError):
        M.disparity_levels(Lu, Lu, 16, 3, 2, 0.065, 1, 0.05)  # the soft levels take float images


def test_autograd_every_level_loss(M):
    """A loss on all levels' soft outputs through torch autograd equals the
    oracle's gradient of the same loss."""
    L, R, cfg = _case(3, 80, 144)
    D, K, n, rs, eps, tau = 40, 3, 2, 2, cfg.var_eps, cfg.tau
    Lt = dev(L).requires_grad_(True)
    Rt = dev(R).requires_grad_(True)
    softs = M.MsibmLevelsFunction.apply(Lt, Rt, D, K, n, eps, rs, tau)
    loss = sum((w * s).sum() for w, s in zip((1.0, 0.5), softs))
    loss.backward()
    _, maps = M.disparity_levels(dev(L), dev(R), D, K, n, eps, rs, tau)
    grads = [np.full(tuple(s.shape), w) for w, s in zip((1.0, 0.5), softs)] + [None]
    oL, oR = oracle.backward_levels(L, R, D, K, n, rs, tau, eps, [host(m) for m in maps], grads)
    assert rel(host(Lt.grad), oL) <= REL_TOL and rel(host(Rt.grad), oR) <= REL_TOL


@pytest.mark.parametrize("H,W,K", [(1, 1, 2), (3, 2, 3), (200, 300, 8)])
def test_levels_degenerate_and_deepest(M, H, W, K):
    """One pixel, tiny levels, and the deepest pyramid (levels down to 2 x 3):
    the soft levels and the gradient against the oracle."""
    rng = np.random.Generator(np.random.PCG64(H * W + K))
    L = rng.random((H, W)).astype(np.float32)
    R = rng.random((H, W)).astype(np.float32)
    D, n, rs, tau, eps = 40, 1, 1, 0.1, 1e-6
    soft, maps = M.disparity_levels(dev(L), dev(R), D, K, n, eps, rs, tau)
    PL, PR = M.pyramid(dev(L), K), M.pyramid(dev(R), K)
    for k in range(K - 1):
        ds_o = oracle.soft_level0(host(PL[k]).astype(np.float64), host(PR[k]).astype(np.float64), n,
                                  -(-D // (1 << k)), host(maps[k + 1]), rs, tau, eps)[0]
        assert np.abs(host(soft[k]) - ds_o).max() <= 1e-2, k
    grads = [rng.standard_normal(tuple(s.shape)).astype(np.float32) for s in soft]
    gL, gR = M.backward_levels(dev(L), dev(R), maps, [dev(g) for g in grads], D, K, n, eps, rs, tau)
    oL, oR = oracle.backward_levels(L, R, D, K, n, rs, tau, eps, [host(m) for m in maps],
                                    [g.astype(np.float64) for g in grads] + [None])
    scale = max(np.linalg.norm(oL), np.linalg.norm(oR), 1e-12)
    assert np.linalg.norm(host(gL) - oL) <= REL_TOL * scale and np.linalg.norm(host(gR) - oR) <= REL_TOL * scale
