"""The GPU path against the hand-derived worked examples under tests/golden/
(through the C ABI): the scores of the worked ZNCC windows (from the matching
kernel's per-candidate score output), the reduce step, the selective median
and the bicubic doubling.  The expected values are exact rationals; the GPU
computes the scores in FP32 (tolerance 1e-6) and the reduce, median and
doubling exactly for these dyadic inputs."""
import numpy as np
import pytest

from golden_cases import ids, load_cases

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ZNCC = load_cases("zncc_worked.txt")
REDUCE = [c for c in load_cases("pyramid_worked.txt") if c["op"] == "reduce"]
MED = load_cases("median_worked.txt")
BIC = load_cases("bicubic_worked.txt")


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1901_09593_amd import msibm
    msibm.lib()
    return msibm


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("case", ZNCC, ids=ids(ZNCC))
def test_zncc_worked_on_gpu(M, case):
    n = int(case["n"][0])
    i, j = (int(v) for v in case["pixel"])
    z = int(case["z"][0])
    print(f"golden zncc case {case['name']}", flush=True)
    L = dev(case["left"], np.uint8)
    R = dev(case["right"], np.uint8)
    # a full search whose candidates 0..j include z; the score output holds
    # every scored candidate's score
    d, C, V = M.match_level(L, R, n, j + 1, None, var_eps=case["eps"][0], with_costvol=True)
    got = float(host(V)[i, j, z])
    assert got == pytest.approx(case["expect"][0, 0], abs=1e-6)


@pytest.mark.parametrize("case", REDUCE, ids=ids(REDUCE))
def test_reduce_worked_on_gpu(M, case):
    print(f"golden reduce case {case['name']}", flush=True)
    levels = M.pyramid(dev(case["image"], np.float32), 2)
    np.testing.assert_array_equal(host(levels[1]).astype(np.float64), case["expect"])


@pytest.mark.parametrize("case", MED, ids=ids(MED))
def test_median_worked_on_gpu(M, case):
    print(f"golden median case {case['name']}", flush=True)
    out = M.median_filter(dev(case["disp"], np.int16), dev(case["cost"], np.float32), case["alpha"][0])
    np.testing.assert_array_equal(host(out), case["expect"].astype(np.int16))


@pytest.mark.parametrize("case", BIC, ids=ids(BIC))
def test_bicubic_worked_on_gpu(M, case):
    assert case["a"][0] == -0.5  # the method's kernel parameter, fixed in the library
    H, W = (int(v) for v in case["size"])
    print(f"golden bicubic case {case['name']}", flush=True)
    out = M.upsample_cost(dev(case["image"], np.float32), H, W)
    np.testing.assert_array_equal(host(out), case["expect"])
