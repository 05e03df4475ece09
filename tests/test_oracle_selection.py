"""Pins of the selection oracle (unprojection, reprojection as a mask, tint).

The unprojection is tied to the projection oracle (eq. 1-2, C code of its own): the
projection of every unprojected point is its pixel's centre at its depth. The
reprojected mask is pinned by hand-placed closed forms, a brute-force loop over
every pixel and point, and the round trip through unprojection. The tint is pinned
by exact products with powers of two.
"""
import math

import numpy as np
import pytest

import synth
from oracle import selection as S
from tests.scenes_by_hand import axis_camera, scene_from


def _depth(seed, H, W, zero_frac=0.1):
    rng = np.random.default_rng(seed)
    d = rng.uniform(1.0, 6.0, (H, W)).astype(np.float32)
    d[rng.random((H, W)) < zero_frac] = 0
    return d


def test_unproject_projects_back_to_pixel_centres(orc):
    cam = synth.make_tiny().view.camera
    H, W = cam.height, cam.width
    mask = synth.brush_mask(W, H, 60.0, 70.0, 30.0)
    keep = synth.sample_keep(3, mask)
    depth = _depth(4, H, W)
    X, pix = S.unproject(cam, mask, keep, depth)
    assert X.shape[0] == int(((mask != 0) & (keep != 0) & (depth > 0)).sum())
    assert np.all(np.diff(pix) > 0)                       # row-major pixel order
    n = X.shape[0]
    sc = scene_from(X, [[math.log(0.01)] * 3] * n, [0.5] * n, dc_rgb=[[0.5] * 3] * n)
    pr = orc.project(sc, cam)
    xs, ys = pix % W, pix // W
    # means are stored as float32: allow the rounding of |X| ~ 4 carried to the pixel
    np.testing.assert_allclose(pr.col("u"), xs + 0.5, atol=2e-3)
    np.testing.assert_allclose(pr.col("v"), ys + 0.5, atol=2e-3)
    np.testing.assert_allclose(pr.col("z"), depth.reshape(-1)[pix], rtol=1e-6)
    # in float64, before the means are rounded, the round trip is exact up to the
    # orthonormality defect of the float32 rotation (R^T stands for R^-1): ~1e-7
    R, t = cam.R.astype(np.float64), cam.t.astype(np.float64)
    defect = np.abs(R.T @ R - np.eye(3)).max()
    assert defect < 1e-6
    m = X @ R.T + t
    np.testing.assert_allclose(cam.fx * m[:, 0] / m[:, 2] + cam.cx, xs + 0.5, atol=1e-5)
    np.testing.assert_allclose(m[:, 2], depth.reshape(-1)[pix], rtol=4 * defect + 1e-12)


def test_unproject_keep_none_and_empty():
    cam = axis_camera(8, 6, 10.0)
    mask = np.ones((6, 8), np.uint8)
    depth = np.full((6, 8), 2.0, np.float32)
    X, pix = S.unproject(cam, mask, None, depth)
    assert X.shape == (48, 3) and list(pix) == list(range(48))
    # axis camera: X = (z (x + 1/2 - cx) / fx, z (y + 1/2 - cy) / fy, z)
    np.testing.assert_allclose(X[9], [2.0 * (1.5 - 4.0) / 10.0, 2.0 * (1.5 - 3.0) / 10.0, 2.0], rtol=1e-15)
    X, pix = S.unproject(cam, np.zeros((6, 8), np.uint8), None, depth)
    assert X.shape == (0, 3)


@pytest.mark.parametrize("q,want", [(1, [8]), (2, [7, 8]), (3, [7, 8, 9]), (2.5, [7, 8, 9]), (4, [6, 7, 8, 9])])
def test_reproject_square_closed_form(q, want):
    # a point on the optical axis projects to (cx, cy) = (8.3, 8.3): square [8.3 - q/2,
    # 8.3 + q/2) holds the pixel centres listed (no centre on an edge)
    cam = axis_camera(16, 16, 20.0, cx=8.3, cy=8.3)
    lo, hi = S.reproject_mask(cam, [[0.0, 0.0, 2.0]], q)
    assert np.array_equal(lo, hi)
    ys, xs = np.nonzero(lo)
    assert sorted(set(xs.tolist())) == want and sorted(set(ys.tolist())) == want
    assert lo.sum() == len(want) ** 2


def test_reproject_centre_on_an_edge_is_in_band():
    # q = 2 around the pixel centre 8.5: the centre 7.5 lies on the closed edge (in),
    # 9.5 on the open edge (out); both are ties that float32 rounding could flip
    cam = axis_camera(16, 16, 20.0, cx=8.5, cy=8.5)
    lo, hi = S.reproject_mask(cam, [[0.0, 0.0, 2.0]], 2)
    assert lo[8, 8] == 1 and lo.sum() == 1
    assert hi[7:10, 7:10].sum() == 9 and hi.sum() == 9
    assert S.reproject_mask_brute(cam, [[0.0, 0.0, 2.0]], 2)[7:9, 7:9].sum() == 4


def test_reproject_depth_test_and_near_plane():
    cam = axis_camera(16, 16, 20.0, cx=8.3, cy=8.3)
    d = np.zeros((16, 16), np.float32)
    d[7, 7] = 1.0        # nearer surface: the point (z = 2) is hidden there
    d[7, 8] = 2.5        # farther surface: drawn
    d[8, 8] = 2.0        # equal depth: a float32 tie, in the band
    lo, hi = S.reproject_mask(cam, [[0.0, 0.0, 2.0]], 3, d, eps=0.0)
    assert lo[7, 7] == 0 and hi[7, 7] == 0
    assert lo[7, 8] == 1 and lo[9, 9] == 1               # depth 0 = no surface: drawn
    assert lo[8, 8] == 0 and hi[8, 8] == 1
    lo, hi = S.reproject_mask(cam, [[0.0, 0.0, 2.0]], 3, d, eps=1e-3)
    assert lo[8, 8] == 1 and lo[7, 7] == 0               # eps = 1e-3 passes the tie
    # behind the near plane (0.2) or behind the camera: nothing
    for z in (0.1, -2.0):
        lo, hi = S.reproject_mask(cam, [[0.0, 0.0, z]], 3)
        assert hi.sum() == 0


def test_reproject_matches_brute_force():
    cam = synth.orbit_camera(24, 20, 60.0, 3.0, 0.4, 0.3)
    rng = np.random.default_rng(9)
    pts = rng.normal(0.0, 0.8, (40, 3))
    d = _depth(10, 20, 24, zero_frac=0.3) * 0.8
    for q, depth, eps in [(1, None, 0.0), (2.5, d, 0.0), (3, d, 0.05), (6, None, 0.0)]:
        lo, hi = S.reproject_mask(cam, pts, q, depth, eps)
        ref = S.reproject_mask_brute(cam, pts, q, depth, eps)
        assert np.all(lo <= ref) and np.all(ref <= hi), q
        assert (hi != lo).sum() <= 2, q
        assert ref.sum() > 0


def test_unproject_then_reproject_is_the_selection():
    """Unit squares of the unprojected points, drawn back into the same view against
    the same depth map, mark exactly the selected pixels."""
    cam = synth.make_tiny().view.camera
    H, W = cam.height, cam.width
    mask = synth.brush_mask(W, H, 64.0, 64.0, 40.0)
    keep = synth.sample_keep(5, mask)
    depth = _depth(6, H, W)
    X, _ = S.unproject(cam, mask, keep, depth)
    lo, hi = S.reproject_mask(cam, X, 1, depth, eps=1e-4)
    want = ((mask != 0) & (keep != 0) & (depth > 0)).astype(np.uint8)
    assert np.array_equal(lo, want) and np.array_equal(hi, want)


def test_tint_exact_products():
    rng = np.random.default_rng(2)
    img = rng.random((5, 7, 3)).astype(np.float32)
    mask = (rng.random((5, 7)) < 0.5).astype(np.uint8)
    out = S.tint(img, mask, (0.5, 2.0, 0.25))
    m = mask.astype(bool)
    np.testing.assert_array_equal(out[m], img[m] * np.float32([0.5, 2.0, 0.25]))   # powers of two: exact
    np.testing.assert_array_equal(out[~m], img[~m])
    t = np.float32([0.3, 0.7, 1.1])
    out = S.tint(img, mask, t)
    np.testing.assert_array_equal(out[m], img[m] * t)    # numpy's float32 product is rounded once too


# ---------------------------------------------------------------------------
# statistical outlier removal (Sec. 3.2, Fig. 2)
# ---------------------------------------------------------------------------
def test_knn_mean_distance_matches_brute_force():
    rng = np.random.default_rng(21)
    X = rng.normal(0, 1, (300, 3))
    X[:5] = X[5]                                    # duplicates: zero distances
    for k in (1, 4, 16, 32):
        np.testing.assert_allclose(S.knn_mean_distance(X, k), S.knn_mean_distance_brute(X, k), rtol=1e-12)
    # fewer points than k: the mean over all the others
    Y = X[:7]
    np.testing.assert_allclose(S.knn_mean_distance(Y, 16), S.knn_mean_distance_brute(Y, 6), rtol=1e-12)


def test_knn_mean_distance_on_a_lattice():
    # interior point of a cubic lattice of spacing s: 6 neighbours at s, 12 at s sqrt(2)
    s = 0.25
    g = np.arange(8) * s
    X = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    D = S.knn_mean_distance(X, 16)
    interior = np.all((X > 1.5 * s) & (X < g[-1] - 1.5 * s), axis=1)
    np.testing.assert_allclose(D[interior], (6 * s + 10 * math.sqrt(2) * s) / 16, rtol=1e-13)
    D6 = S.knn_mean_distance(X, 6)
    np.testing.assert_allclose(D6[interior], s, rtol=1e-13)


def test_outlier_filter_removes_isolated_points_and_is_rigid_invariant():
    s = 0.25
    g = np.arange(8) * s
    X = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    X = np.concatenate([X, [[10.0, 10.0, 10.0], [-8.0, 1.0, 0.5]]])
    keep, flag, D, thr = S.outlier_filter(X, 16, 0.007)
    assert not keep[-1] and not keep[-2]
    interior = np.all((X > 1.5 * s) & (X < g[-1] - 1.5 * s), axis=1)
    assert np.all(keep[interior])
    mu, sd = D.mean(), math.sqrt(((D - D.mean()) ** 2).mean())
    assert thr == pytest.approx(mu + float(np.float32(0.007)) * sd, rel=1e-14)
    # a rotation and a translation change no distance
    th = 0.7
    Rz = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]])
    keep2, _, D2, _ = S.outlier_filter(X @ Rz.T + [3.0, -1.0, 2.0], 16, 0.007)
    np.testing.assert_allclose(D2, D, rtol=1e-12, atol=1e-14)
    assert np.array_equal(keep2, keep)


def test_outlier_filter_degenerate_clouds():
    keep, flag, D, thr = S.outlier_filter(np.zeros((0, 3)))
    assert keep.size == 0
    keep, _, D, _ = S.outlier_filter(np.array([[1.0, 2.0, 3.0]]))
    assert keep.tolist() == [True] and D.tolist() == [0.0]
    keep, _, D, _ = S.outlier_filter(np.ones((5, 3)))     # all coincident: every distance 0, all kept
    assert keep.all() and np.all(D == 0)
