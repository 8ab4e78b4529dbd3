"""Comparison helpers shared by the GPU parity tests.

The rule for floating-point winner-take-all outputs: the GPU's score must equal
the oracle's score of the GPU's own choice to within TOL_ZNCC, its choice must be a
valid candidate, and it may differ from the oracle's choice only where the
oracle's best and second-best scores lie within TOL_ZNCC (a near tie), in which
case the GPU's choice still scores within TOL_ZNCC of the oracle's best.
"""
import numpy as np

import oracle

TOL_ZNCC = 1e-4


def cand_bounds(H, W, Dk, prior, r):
    """Per-pixel candidate interval [lo, hi] (numpy restatement of the interval
    definition, used only to check that a GPU choice is a valid candidate)."""
    jj = np.broadcast_to(np.arange(W)[None, :], (H, W))
    top = np.minimum(Dk - 1, jj)
    if prior is None:
        return np.zeros((H, W), dtype=np.int64), top
    ii = np.broadcast_to(np.arange(H)[:, None], (H, W))
    dh = 2 * prior.astype(np.int64)[ii // 2, jj // 2]
    c = np.minimum(dh, jj)
    return np.maximum(0, c - r), np.minimum(top, c + r)


def check_level(d_gpu, C_gpu, L, R, n, Dk, prior, r, eps, tol=TOL_ZNCC, ref=None):
    """Compare one level's GPU output with the oracle on every pixel.

    Returns a dict of statistics (mismatch rate, max score error)."""
    H, W = d_gpu.shape
    d_o, C_o, C2_o = ref if ref is not None else oracle.match_level(L, R, n, Dk, prior, r, eps)
    lo, hi = cand_bounds(H, W, Dk, prior, r)
    dg = d_gpu.astype(np.int64)
    assert np.all((dg >= lo) & (dg <= hi)), "GPU chose an invalid candidate"
    ii, jj = np.nonzero(np.ones((H, W), dtype=bool))
    rho_at = oracle.zncc_many(L, R, n, ii, jj, dg.ravel(), eps).reshape(H, W)
    err = np.abs(C_gpu.astype(np.float64) - rho_at) if C_gpu is not None else np.zeros((H, W))
    assert err.max() <= tol, f"|dZNCC| = {err.max():.3g} > {tol}"
    mism = dg != d_o
    near = (C_o - C2_o) <= tol
    bad = mism & ~near
    assert not bad.any(), f"{bad.sum()} mismatches outside near ties, e.g. {np.argwhere(bad)[:5]}"
    assert np.all(rho_at >= C_o - tol), "GPU choice scores below the best by more than the tolerance"
    return {"mismatch": float(mism.mean()), "near_ties": float(near.mean()),
            "max_dzncc": float(err.max())}


def check_pixels(d_gpu, C_gpu, L, R, n, Dk, prior, r, eps, ii, jj, tol=TOL_ZNCC):
    """check_level on sampled pixels only (large images)."""
    d_o, C_o, C2_o = oracle.match_pixels(L, R, n, Dk, prior, r, eps, ii, jj)
    dg = d_gpu[ii, jj].astype(np.int64)
    H, W = d_gpu.shape
    lo, hi = cand_bounds(H, W, Dk, prior, r)
    assert np.all((dg >= lo[ii, jj]) & (dg <= hi[ii, jj])), "GPU chose an invalid candidate"
    rho_at = oracle.zncc_many(L, R, n, ii, jj, dg, eps)
    err = np.abs(C_gpu[ii, jj].astype(np.float64) - rho_at)
    assert err.max() <= tol, f"|dZNCC| = {err.max():.3g} > {tol}"
    mism = dg != d_o
    near = (C_o - C2_o) <= tol
    assert not (mism & ~near).any(), f"{(mism & ~near).sum()} sampled mismatches outside near ties"
    assert np.all(rho_at >= C_o - tol)
    return {"mismatch": float(mism.mean()), "near_ties": float(near.mean()),
            "max_dzncc": float(err.max())}
