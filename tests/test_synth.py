"""Properties of the seeded synthetic stereo generator (inputs only)."""
import numpy as np

from paper_1901_09593_amd import synth


def test_pair_is_deterministic_and_typed():
    a = synth.make_pair(5, 30, 41, 3, 2, 12, True, 0.9, 8.0, 2.0, "u8")
    b = synth.make_pair(5, 30, 41, 3, 2, 12, True, 0.9, 8.0, 2.0, "u8")
    assert a.left.dtype == np.uint8 and a.right.dtype == np.uint8
    assert np.array_equal(a.left, b.left) and np.array_equal(a.right, b.right)
    f = synth.make_pair(5, 30, 41, 3, 2, 12, True, 1.0, 0.0, 0.01, "f32")
    assert f.left.dtype == np.float32 and 0.0 <= f.left.min() and f.left.max() <= 1.0


def test_warp_ground_truth_is_consistent():
    # without photometric changes the right view holds each visible left pixel
    # at column round(x - d)
    for slanted in (False, True):
        p = synth.make_pair(7, 40, 60, 4, 3, 20, slanted, 1.0, 0.0, 0.0, "u8")
        yy, xx = np.nonzero(p.nonocc)
        xr = np.rint(xx - p.disp[yy, xx]).astype(int)
        assert np.array_equal(p.right[yy, xr], p.left[yy, xx])
        assert 0.5 < p.nonocc.mean() < 1.0


def test_zbuffer_conflict_resolution():
    left = np.array([[10.0, 20.0, 30.0, 40.0, 50.0]])
    disp = np.array([[0.0, 0.0, 0.0, 1.0, 0.0]])  # x=3 -> col 2 competes with x=2 (d=0)
    right, vis = synth.warp_left_to_right(left, disp, np.full((1, 5), -1.0))
    assert right[0, 2] == 40.0 and vis[0, 3] and not vis[0, 2]
    assert right[0, 3] == -1.0  # nothing lands there: fill texture


def test_workload_shapes():
    p, cfg = synth.workload("small320")
    assert p.left.shape == (240, 320) and cfg.max_disp == 64 and cfg.levels == 3
    assert 4 <= p.disp.min() and p.disp.max() <= 60
    shapes = synth.batch_shapes(32)
    assert len(shapes) == 32
    for H, W, D in shapes:
        assert 480 <= H <= 1988 and 640 <= W <= 2880 and 64 <= D <= 400
        K = synth.auto_levels(D)
        assert synth.level_range(D, K - 1) <= 32 and (K == 1 or synth.level_range(D, K - 2) > 32)


def test_texture_statistics():
    t = synth.texture(np.random.Generator(np.random.PCG64(0)), 128, 128)
    assert t.min() == 0.0 and t.max() == 1.0
    # blurred noise: neighbouring pixels correlate, distant ones do not
    c1 = np.corrcoef(t[:, :-1].ravel(), t[:, 1:].ravel())[0, 1]
    c9 = np.corrcoef(t[:, :-9].ravel(), t[:, 9:].ravel())[0, 1]
    assert c1 > 0.7 and abs(c9) < 0.1


def test_loss_mask_keeps_every_candidate_window_inside():
    """Every loss pixel's own window and the right window of every candidate
    z in [0, D-1] lie inside the image; visibility is respected."""
    rng = np.random.Generator(np.random.PCG64(7))
    H, W, n, D = 23, 41, 2, 9
    vis = rng.random((H, W)) > 0.2
    m = synth.loss_mask(vis, n, D)
    ii, jj = np.nonzero(m)
    assert m.any() and not (m & ~vis).any()
    assert ii.min() >= n and ii.max() <= H - 1 - n
    assert jj.max() <= W - 1 - n and (jj - (D - 1) - n).min() >= 0
    # and it is the largest such set: the first admissible column is kept
    j0 = n + D - 1
    assert np.array_equal(m[n:H - n, j0], vis[n:H - n, j0])
