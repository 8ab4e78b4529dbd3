"""Batched persistent launch (and its hipGraph replay) against the plain
per-pair path: identical outputs, bit for bit."""
import numpy as np
import pytest

from paper_1901_09593_amd import synth

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


def _batch(dtype="u8", count=5, seed=7):
    rng = np.random.Generator(np.random.PCG64(seed))
    pairs = []
    for i in range(count):
        H = int(rng.integers(40, 260))
        W = int(rng.integers(60, 400))
        D = int(rng.integers(24, 160))
        scale = 1.0 if dtype == "u8" else 1.0 / 255
        p = synth.make_pair(100 + i, H, W, 4, 0.05 * D, 0.9 * D, True, 1.0, 0.0, 2.0 * scale, dtype)
        pairs.append((p, D))
    return pairs


PERSISTENT_OFF = ("persistent scheduler disabled: two runs hung on MI355X "
                  "(at the synchronize after the launch) and the cause is not found")


@pytest.mark.skip(reason=PERSISTENT_OFF)
@pytest.mark.parametrize("dtype,n,r,rs", [("u8", 4, 2, 0), ("u8", 3, 3, 0), ("f32", 5, 2, 0),
                                          ("f32", 3, 2, 3)])
def test_batched_equals_plain(M, dtype, n, r, rs):
    pairs = _batch(dtype, seed=n * 10 + r)
    eps = 0.065 if dtype == "u8" else 1e-6
    L = [dev(p.left) for p, _ in pairs]
    R = [dev(p.right) for p, _ in pairs]
    Ds = [D for _, D in pairs]
    Ks = [0] * len(pairs)  # automatic level count
    plain = M.disparity_many(L, R, Ds, Ks, n, r, eps, soft_radius=rs, with_prior1=True)
    ws = torch.empty(M.workspace_bytes(M._pairs(L, R, Ds, Ks)[0], len(L),
                                       M.make_config(n, r, eps, rs, flags=M.FLAG_BATCHED)),
                     dtype=torch.uint8, device="cuda")
    print("batched call", dtype, n, r, rs, flush=True)
    batched = M.disparity_many(L, R, Ds, Ks, n, r, eps, soft_radius=rs, with_prior1=True,
                               flags=M.FLAG_BATCHED, workspace=ws)
    torch.cuda.synchronize()
    M.batch_status(L, R, Ds, Ks, n, r, eps, ws, soft_radius=rs)
    for a, b in zip(plain, batched):
        for k in a:
            assert torch.equal(a[k], b[k]), k


@pytest.mark.skip(reason=PERSISTENT_OFF)
def test_graph_replay_equals_direct_and_repeats(M):
    pairs = _batch("u8", count=6, seed=3)
    L = [dev(p.left) for p, _ in pairs]
    R = [dev(p.right) for p, _ in pairs]
    Ds = [D for _, D in pairs]
    Ks = [0] * len(pairs)
    n, r, eps = 4, 2, 0.065
    ref = M.disparity_many(L, R, Ds, Ks, n, r, eps)
    outs = M.disparity_many(L, R, Ds, Ks, n, r, eps, flags=M.FLAG_BATCHED | M.FLAG_GRAPH)
    ws = torch.empty(M.workspace_bytes(M._pairs(L, R, Ds, Ks)[0], len(L),
                                       M.make_config(n, r, eps, flags=M.FLAG_BATCHED | M.FLAG_GRAPH)),
                     dtype=torch.uint8, device="cuda")
    for rep in range(4):
        # the same buffers every time: the first call captures, later calls replay
        for o in outs:
            for t in o.values():
                t.fill_(-7 if t.dtype == torch.int16 else 7.0)
        M.disparity_many(L, R, Ds, Ks, n, r, eps, flags=M.FLAG_BATCHED | M.FLAG_GRAPH,
                         workspace=ws, outputs=outs)
        torch.cuda.synchronize()
        for a, b in zip(ref, outs):
            for k in a:
                assert torch.equal(a[k], b[k]), (rep, k)


def test_batched_rejects_unsupported(M):
    pairs = _batch("u8", count=2)
    L = [dev(p.left) for p, _ in pairs]
    R = [dev(p.right) for p, _ in pairs]
    with pytest.raises(M.MsibmError):
        M.disparity_many(L, R, [32, 32], [0, 0], 2, 2, 0.065, flags=M.FLAG_BATCHED)
