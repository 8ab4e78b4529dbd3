"""The allocation-free entry point (msibm_disparity_noalloc) against the
workspace entry point (msibm_disparity) on the same pairs: both run the same
kernels, so every output must be identical, bit for bit.  Calls follow each
other on the one scratch array of the device, the later ones on smaller pairs,
so a value left over from an earlier call would show."""
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


def _outputs(H, W, K, soft, like=None):
    o = {"disp": torch.full((H, W), -7, dtype=torch.int16, device="cuda"),
         "cost": torch.full((H, W), 7.0, dtype=torch.float32, device="cuda")}
    if K >= 2:
        o["prior1"] = torch.full(((H + 1) // 2, (W + 1) // 2), -7, dtype=torch.int16, device="cuda")
    if soft:
        o["soft"] = torch.full((H, W), 7.0, dtype=torch.float32, device="cuda")
    return o


# (seed, H, W, D, dtype, n, r, soft radius, extra options), larger pairs first
CALLS = [
    (11, 420, 560, 120, "u8", 4, 2, 0, {}),
    (12, 150, 214, 48, "u8", 3, 2, 0, {}),
    (13, 236, 300, 64, "f32", 3, 2, 3, {}),
    (14, 96, 130, 40, "u8", 4, 1, 0, {"median_alpha": 0.9, "gate": (0.9, 0.9)}),
    (15, 61, 77, 24, "f32", 2, 2, 0, {"flags": 8}),
]


def _run(M, seed, H, W, D, dtype, n, r, rs, opts):
    scale = 1.0 if dtype == "u8" else 1.0 / 255
    p = synth.make_pair(seed, H, W, 4, 0.05 * D, 0.9 * D, True, 0.9, 6.0 * scale, 2.0 * scale, dtype)
    eps = 0.065 if dtype == "u8" else 1e-6
    K = synth.auto_levels(D)
    L, R = dev(p.left), dev(p.right)
    print(f"no-alloc pair seed {seed} {H}x{W} {dtype} D={D} K={K} n={n} r={r} rs={rs} {opts}", flush=True)
    flags = opts.get("flags", 0)
    kw = {k: v for k, v in opts.items() if k != "flags"}
    ref = M.disparity_many([L], [R], [D], [K], n, r, eps, soft_radius=rs, tau=0.05, with_prior1=K >= 2,
                           flags=flags, **kw)[0]
    got = M.disparity_noalloc(L, R, D, K, n, r, eps, _outputs(H, W, K, rs > 0), soft_radius=rs, tau=0.05,
                              flags=flags, **kw)
    torch.cuda.synchronize()
    for key in ref:
        assert torch.equal(ref[key], got[key]), (seed, key)


def test_noalloc_equals_workspace_entry_point(M):
    for c in CALLS:
        _run(M, *c)


def test_noalloc_repeats_after_a_smaller_pair(M):
    # the same two pairs again in the opposite order of size: the second, larger
    # call must not see anything of the smaller one's scratch contents
    _run(M, *CALLS[1])
    _run(M, *CALLS[0])


def test_noalloc_rejects_oversized_pair_and_batched_flags(M):
    H, W = 4000, 4000
    L = torch.zeros((H, W), dtype=torch.uint8, device="cuda")
    out = {"disp": torch.empty((H, W), dtype=torch.int16, device="cuda")}
    with pytest.raises(M.MsibmError) as e:
        M.disparity_noalloc(L, L, 64, 2, 4, 2, 0.065, out)
    assert e.value.status == -3
    small = torch.zeros((32, 48), dtype=torch.uint8, device="cuda")
    out = {"disp": torch.empty((32, 48), dtype=torch.int16, device="cuda")}
    with pytest.raises(M.MsibmError) as e:
        M.disparity_noalloc(small, small, 16, 1, 2, 2, 0.065, out, flags=M.FLAG_BATCHED)
    assert e.value.status == -4
