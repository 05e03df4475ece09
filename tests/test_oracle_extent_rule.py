"""Pins of the oracle's second extent rule: the tiles of the 3DGS rasteriser's square
of radius ceil(3 sqrt(lambda_max)) pixels, within which alone a splat reaches pixels.

Pinned by hand-computed rectangles of on-axis Gaussians whose 2D covariance is known
in closed form, by a splat whose alpha >= 1/255 region reaches past its square (the
pixels of the tiles it is not listed in keep the background), and by the definition
of the rule: each tile's pixels composite (eq. 3) exactly the Gaussians that list the
tile, which the default rule's oracle reproduces when given only those Gaussians.
"""
import math

import numpy as np
import pytest

import synth
from tests.scenes_by_hand import axis_camera, scene_from


def _single(orc, s, z, f=40.0, W=64, H=64, tile=(8, 8), opacity=0.9, cx=None, cy=None, rule=1):
    cam = axis_camera(W, H, f, cx=W / 2 + 0.5 if cx is None else cx, cy=H / 2 + 0.5 if cy is None else cy)
    ls = [[math.log(x) for x in s]] if isinstance(s, (tuple, list)) else [[math.log(s)] * 3]
    sc = scene_from([[0.0, 0.0, z]], ls, [opacity], dc_rgb=[[1.0, 0.5, 0.25]])
    return orc.project(sc, cam, tile, extent_rule=rule), cam, sc


@pytest.mark.parametrize("tile,span", [((8, 8), (3, 4)), ((16, 16), (1, 2)), ((32, 32), (0, 1)), ((32, 8), (0, 1))])
def test_isotropic_square_by_hand(orc, tile, span):
    # f s / z = 40 * 0.05 / 2 = 1: Sigma2D = 1.3 I, no spread, so lambda = 1.3 + sqrt(0.1)
    pr, cam, _ = _single(orc, 0.05, 2.0, tile=tile)
    lam = 1.3 + math.sqrt(0.1)
    assert pr.col("sa")[0] == pytest.approx(1.3, rel=1e-6) and pr.col("sb")[0] == pytest.approx(0.0, abs=1e-12)
    r = math.ceil(3 * math.sqrt(lam))
    assert r == 4
    # centre pixel-index coordinate 32 (u = 32.5): x tiles floor(28 / tw) .. floor((36 + tw - 1) / tw) - 1
    tw, th = tile
    tx = (math.floor((32 - r) / tw), math.floor((32 + r + tw - 1) / tw) - 1)
    ty = (math.floor((32 - r) / th), math.floor((32 + r + th - 1) / th) - 1)
    assert tx == span
    assert (pr.col("txlo")[0], pr.col("txhi")[0]) == tx
    assert (pr.col("tylo")[0], pr.col("tyhi")[0]) == ty
    assert pr.col("count")[0] == (tx[1] - tx[0] + 1) * (ty[1] - ty[0] + 1)
    assert pr.col("rule")[0] == 1 and pr.col("flag")[0] == 0


def test_anisotropic_square_uses_the_larger_eigenvalue(orc):
    # axis-aligned: Sigma2D = diag((f sx / z)^2 + 0.3, (f sy / z)^2 + 0.3) = diag(16.3, 0.3625)
    pr, cam, _ = _single(orc, (0.2, 0.0125, 0.01), 2.0, tile=(8, 8))
    a, c = 16.3, 0.3625
    assert pr.col("sa")[0] == pytest.approx(a, rel=1e-6) and pr.col("sc")[0] == pytest.approx(c, rel=1e-5)
    r = math.ceil(3 * math.sqrt(max(a, c)))   # the spread (a - c) / 2 is far above sqrt(0.1)
    assert r == 13
    # a square, not a box: the y span is as wide as the x span
    assert (pr.col("txlo")[0], pr.col("txhi")[0]) == (math.floor((32 - r) / 8), math.floor((32 + r + 7) / 8) - 1)
    assert (pr.col("tylo")[0], pr.col("tyhi")[0]) == (math.floor((32 - r) / 8), math.floor((32 + r + 7) / 8) - 1)
    # the default rule's box is far narrower in y
    pa, _, _ = _single(orc, (0.2, 0.0125, 0.01), 2.0, tile=(8, 8), rule=0)
    assert pa.col("tyhi")[0] - pa.col("tylo")[0] < pr.col("tyhi")[0] - pr.col("tylo")[0]


def test_square_clipped_to_the_grid_and_empty_off_image(orc):
    pr, _, _ = _single(orc, 0.05, 2.0, tile=(16, 16), cx=2.5, cy=62.5)
    assert pr.col("txlo")[0] == 0 and pr.col("tyhi")[0] == 3
    # centre 40 px left of the image: the square (radius 4) misses it
    pr, _, _ = _single(orc, 0.05, 2.0, tile=(16, 16), cx=-40.0)
    assert pr.col("count")[0] == 0 and pr.col("status")[0] == 4
    r = orc.render_image(pr, brute=True)
    assert np.all(r.rgb == 0)


def test_tail_beyond_the_square_is_cut(orc):
    """An opaque splat: alpha >= 1/255 out to q = 2 ln(255 0.99), beyond 3 sqrt(lambda).
    Pixels of tiles it does not list keep the background; the others equal the default
    rule's image."""
    bg = (0.1, 0.2, 0.3)
    # centre at pixel-index coordinate 64.5 (u = 65); f s / z = 10: lambda = 100.3 + sqrt(0.1),
    # radius 31: tiles floor(33.5 / 8) = 4 to floor(102.5 / 8) - 1 = 11, pixels 32..95; the
    # alpha >= 1/255 disc has radius sqrt(2 ln(255 0.99) 100.3) = 33.3, out to 97.8
    kw = dict(W=128, H=128, tile=(8, 8), opacity=0.99, cx=65.0, cy=65.0)
    pr, cam, sc = _single(orc, 0.5, 2.0, **kw)
    pa, _, _ = _single(orc, 0.5, 2.0, rule=0, **kw)
    assert pr.col("txlo")[0] == 4 and pr.col("txhi")[0] == 11
    assert pr.col("tylo")[0] == 4 and pr.col("tyhi")[0] == 11
    rb = orc.render_image(pr, bg=bg, brute=True)
    ra = orc.render_image(pa, bg=bg, brute=True)
    inside = np.zeros((128, 128), bool)
    inside[32:96, 32:96] = True
    np.testing.assert_array_equal(rb.rgb[inside], ra.rgb[inside])
    assert np.all(rb.rgb[~inside] == np.float64(bg))
    # the default rule's image does reach past the square there
    assert (np.abs(ra.rgb[~inside] - np.float64(bg)).max(axis=-1) > 1e-3).sum() > 50


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 8)])
def test_each_tile_composites_exactly_the_gaussians_listing_it(orc, tile):
    w = synth.make_tiny()
    cam = w.view.camera
    sc = w.scene
    pb = orc.project(sc, cam, tile, extent_rule=1)
    rb = orc.render_image(pb, brute=True)
    tw, th = tile
    cnt = pb.col("count")
    lo_x, hi_x, lo_y, hi_y = (pb.col(k) for k in ("txlo", "txhi", "tylo", "tyhi"))
    diff = 0
    for ty in range(-(-cam.height // th)):
        for tx in range(-(-cam.width // tw)):
            listed = np.nonzero((cnt > 0) & (lo_x <= tx) & (tx <= hi_x) & (lo_y <= ty) & (ty <= hi_y))[0]
            x0, y0 = tx * tw, ty * th
            ww, wh = min(tw, cam.width - x0), min(th, cam.height - y0)
            ra = orc.render_windows(orc.project(sc.subset(listed), cam, tile), [(x0, y0, ww, wh)])
            got = rb.rgb[y0:y0 + wh, x0:x0 + ww].reshape(-1, 3)
            np.testing.assert_array_equal(got, ra.rgb)
            np.testing.assert_array_equal(rb.slack[y0:y0 + wh, x0:x0 + ww].reshape(-1), ra.slack)
            full = orc.render_windows(orc.project(sc, cam, tile), [(x0, y0, ww, wh)])
            diff += int((np.abs(full.rgb - got).max(axis=-1) > 1e-6).sum())
    # the square does cut visible tails somewhere in this scene
    assert diff > 0
