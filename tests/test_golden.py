"""The oracle against the hand-derived worked examples under tests/golden/.

Each fixture states the definition it follows (section or equation, and the
reading where the paper leaves a choice) and derives its expected values in
exact arithmetic beside them; see tests/golden/README.md for the format.  The
values are exact rationals, so the oracle's FP64 results must agree to a few
units in the last place.
"""
import numpy as np
import pytest

import oracle
from golden_cases import ids, load_cases

ZNCC = load_cases("zncc_worked.txt")
PYR = load_cases("pyramid_worked.txt")
MED = load_cases("median_worked.txt")
BIC = load_cases("bicubic_worked.txt")


def test_fixtures_are_there():
    assert len(ZNCC) == 4 and len(PYR) == 5 and len(MED) == 4 and len(BIC) == 3


@pytest.mark.parametrize("case", ZNCC, ids=ids(ZNCC))
def test_zncc_worked(case):
    n = int(case["n"][0])
    i, j = (int(v) for v in case["pixel"])
    z = int(case["z"][0])
    got = oracle.zncc(case["left"], case["right"], n, i, j, z, case["eps"][0])
    assert got == pytest.approx(case["expect"][0, 0], rel=1e-14, abs=1e-15)


@pytest.mark.parametrize("case", PYR, ids=ids(PYR))
def test_pyramid_worked(case):
    f = {"reduce": oracle.reduce, "blur": oracle.blur}[case["op"]]
    got = f(case["image"])
    assert got.shape == case["expect"].shape
    np.testing.assert_allclose(got, case["expect"], rtol=1e-14, atol=1e-12)


@pytest.mark.parametrize("case", MED, ids=ids(MED))
def test_median_worked(case):
    got = oracle.median_filter(case["disp"].astype(np.int16), case["cost"], case["alpha"][0])
    np.testing.assert_array_equal(got, case["expect"].astype(np.int16))


@pytest.mark.parametrize("case", BIC, ids=ids(BIC))
def test_bicubic_worked(case):
    H, W = (int(v) for v in case["size"])
    got = oracle.bicubic_up(case["image"], H, W, case["a"][0])
    assert got.shape == case["expect"].shape
    np.testing.assert_allclose(got, case["expect"], rtol=1e-14, atol=1e-12)
