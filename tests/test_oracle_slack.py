"""Pins of the oracle's per-pixel `slack` (eq. 3's threshold and termination decisions).

`slack` bounds how far a pixel can move when a float32 evaluation takes one of the
in-band decisions of eq. 3 the other way: an alpha within its rounding band of the
1/255 skip threshold, or a transmittance within its band of the 1e-4 stop level. The
GPU pixel checks pass at tolerance + slack, so a wrong slack would loosen them.

Each case places splats exactly on one pixel centre (there alpha equals the splat's
opacity), puts exactly one or two decisions inside their bands, and checks slack
against the change of the pixel when that decision is taken the other way, obtained
two ways that do not use the slack code: the closed form of the stack, and the
oracle's own compositing of the alternative stack (the splat removed, or its opacity
nudged across the threshold). With no decision in band, slack must be exactly 0.
"""
import math

import numpy as np
import pytest

from tests.scenes_by_hand import Y00, axis_camera, scene_from

THR = 1.0 / 255.0


def _f32(x):
    return float(np.float32(x))


def _pixel(orc, alphas, colors, bg=(0.0, 0.0, 0.0)):
    """The centre pixel of a stack of on-axis splats at increasing depth: (rgb, slack,
    number blended, displayed colours in float64)."""
    k = len(alphas)
    cam = axis_camera(16, 16, 20.0, cx=8.5, cy=8.5)
    sc = scene_from([[0, 0, 1.0 + 0.5 * j] for j in range(k)], [[math.log(0.01)] * 3] * k, alphas, dc_rgb=colors)
    r = orc.render_windows(orc.project(sc, cam), [(8, 8, 1, 1)], bg=bg, brute=True)
    cols = np.maximum(0.0, Y00 * sc.sh_f32()[0:3].astype(np.float64).T + 0.5)
    return r.rgb[0], float(r.slack[0]), int(r.nblend[0]), cols, sc.opacity.astype(np.float64)


def _closed_form(alphas, cols, bg, stop=None):
    """y of eq. 3 for a stack blended in order, skipping alphas below 1/255, stopping
    before index `stop` (None: no stop)."""
    T, y = 1.0, np.zeros(3)
    for j, a in enumerate(alphas):
        if stop is not None and j == stop:
            break
        if a < THR:
            continue
        a = min(a, 0.99)
        y += cols[j] * a * T
        T *= 1.0 - a
    return y + T * np.asarray(bg)


COLS = [[0.9, 0.2, 0.4], [0.1, 0.8, 0.3], [0.5, 0.5, 0.95], [0.7, 0.05, 0.6], [0.3, 0.9, 0.1]]
BG = (0.2, 0.6, 0.35)


def test_no_decision_in_band_gives_zero_slack(orc):
    rng = np.random.default_rng(7)
    for _ in range(40):
        k = int(rng.integers(1, 6))
        alphas = list(rng.uniform(0.02, 0.9, size=k))
        r, s, nb, cols, a = _pixel(orc, alphas, rng.uniform(0, 1, (k, 3)), bg=tuple(rng.uniform(0, 1, 3)))
        assert s == 0.0 and nb == k
    # alphas far below the threshold and a stop far from the 1e-4 level (T 1.25e-4 -> 6.25e-6)
    for alphas in ([0.5, THR * 0.5, 0.3], [0.95, 0.95, 0.95, 0.95], [0.999, 0.5], [0.99, 0.97, 0.5]):
        _, s, _, _, _ = _pixel(orc, alphas, COLS[:len(alphas)], bg=BG)
        assert s == 0.0, alphas


def test_band_edge_of_the_skip_threshold(orc):
    # on the splat centre the alpha band is 1e-5 relative: 2e-6 inside, 2e-5 outside
    for rel, inside in [(-2e-6, True), (2e-6, True), (-2e-5, False), (2e-5, False)]:
        _, s, _, _, _ = _pixel(orc, [0.5, _f32(THR * (1 + rel)), 0.3], COLS[:3], bg=BG)
        assert (s > 0) == inside, (rel, s)


def test_skipped_in_band_splat(orc):
    """alpha just below 1/255: skipped; slack = change if it were blended."""
    a1 = _f32(THR * (1 - 2e-6))
    assert a1 < THR
    y, s, nb, cols, a = _pixel(orc, [0.5, a1, 0.3], COLS[:3], bg=BG)
    assert nb == 2
    # closed form: blending splat 1 adds a1 (1 - a0) (c1 - c2 a2 - bg (1 - a2))
    d = a[1] * (1 - a[0]) * (cols[1] - cols[2] * a[2] - np.asarray(BG) * (1 - a[2]))
    assert s == pytest.approx(np.abs(d).max(), rel=1e-12)
    np.testing.assert_allclose(y, _closed_form(a, cols, BG), rtol=1e-13)
    # the alternative rendered by the oracle: opacity nudged just above the threshold
    y2, _, nb2, _, a2 = _pixel(orc, [0.5, _f32(THR * (1 + 2e-6)), 0.3], COLS[:3], bg=BG)
    assert nb2 == 3
    assert s == pytest.approx(np.abs(y2 - y).max(), rel=1e-5)


def test_blended_in_band_splat(orc):
    """alpha just above 1/255: blended; slack = change if it were skipped (removed)."""
    a1 = _f32(THR * (1 + 2e-6))
    assert a1 >= THR
    y, s, nb, cols, a = _pixel(orc, [0.5, a1, 0.3], COLS[:3], bg=BG)
    assert nb == 3
    d = a[1] * (1 - a[0]) * (cols[1] - cols[2] * a[2] - np.asarray(BG) * (1 - a[2]))
    assert s == pytest.approx(np.abs(d).max(), rel=1e-9)
    y0, s0, _, _, _ = _pixel(orc, [0.5, 0.3], [COLS[0], COLS[2]], bg=BG)
    assert s0 == 0.0
    assert s == pytest.approx(np.abs(y - y0).max(), rel=1e-9)


def _stop_stack(rel):
    # T: 1 -> 0.2 -> 0.002 (0.99, clamped) -> 0.002 (1 - a2) = 1e-4 (1 + rel)
    return [0.8, 0.99, _f32(0.95 - 0.05 * rel)]


def test_blended_at_the_stop_level(orc):
    """T' within its band above 1e-4: the splat is blended; slack = change if the
    pixel stopped before it instead."""
    alphas = _stop_stack(1e-4) + [0.5]   # the last splat takes T to 5e-5: a stop far from the band
    y, s, nb, cols, a = _pixel(orc, alphas, COLS[:4], bg=BG)
    assert nb == 3
    Tk = (1 - a[0]) * (1 - min(a[1], 0.99))
    assert 1e-4 < Tk * (1 - a[2]) < 1.001e-4
    y_stop = _closed_form(a, cols, BG, stop=2)
    assert s == pytest.approx(np.abs(y - y_stop).max(), rel=1e-9)
    # the oracle's own compositing of the two alternatives
    y0, _, nb0, _, _ = _pixel(orc, alphas[:2], COLS[:2], bg=BG)
    assert nb0 == 2 and s == pytest.approx(np.abs(y - y0).max(), rel=1e-9)
    y1, _, nb1, _, _ = _pixel(orc, _stop_stack(-1e-4) + [0.5], COLS[:4], bg=BG)
    assert nb1 == 2 and s == pytest.approx(np.abs(y - y1).max(), rel=1e-9)


def test_stopped_at_the_stop_level(orc):
    """T' within its band below 1e-4: the pixel stops; slack bounds the change if it
    went on (exact with a black background and nothing behind)."""
    y, s, nb, cols, a = _pixel(orc, _stop_stack(-1e-4), COLS[:3])
    assert nb == 2
    Tk = (1 - a[0]) * (1 - min(a[1], 0.99))
    assert s == pytest.approx(np.abs(a[2] * Tk * cols[2]).max(), rel=1e-12)
    y1, _, nb1, _, _ = _pixel(orc, _stop_stack(1e-4), COLS[:3])
    assert nb1 == 3 and s == pytest.approx(np.abs(y1 - y).max(), rel=1e-4)
    # with a background and splats behind, the bound still holds
    alphas = _stop_stack(-1e-4) + [0.6, 0.3]
    y, s, nb, cols, a = _pixel(orc, alphas, COLS, bg=BG)
    y1, _, nb1, _, _ = _pixel(orc, _stop_stack(1e-4) + [0.6, 0.3], COLS, bg=BG)
    assert nb == 2 and nb1 == 3
    assert s >= np.abs(y1 - y).max()
    bound = a[2] * Tk * cols[2] + Tk * (1 - a[2]) * max(cols[3:].max(), max(BG)) + Tk * np.asarray(BG)
    assert s == pytest.approx(bound.max(), rel=1e-9)


def test_two_in_band_decisions_add(orc):
    """slack = max over channels of the sum of the single-decision changes."""
    lo, hi = _f32(THR * (1 - 2e-6)), _f32(THR * (1 + 2e-6))
    alphas = [0.5, lo, 0.3, hi, 0.4]
    y, s, nb, cols, a = _pixel(orc, alphas, COLS, bg=BG)
    assert nb == 4
    y_a, _, _, _, _ = _pixel(orc, [0.5, hi, 0.3, hi, 0.4], COLS, bg=BG)           # splat 1 blended
    y_b, _, _, _, _ = _pixel(orc, [0.5, 0.3, 0.4], [COLS[0], COLS[2], COLS[4]], bg=BG)  # splat 3 skipped
    y_b1, _, _, _, _ = _pixel(orc, [0.5, lo, 0.3, 0.4], [COLS[0], COLS[1], COLS[2], COLS[4]], bg=BG)
    np.testing.assert_array_equal(y_b, y_b1)  # a skipped splat leaves no trace
    expect = (np.abs(y_a - y) + np.abs(y_b - y)).max()
    assert s == pytest.approx(expect, rel=1e-5)
    assert s > max(np.abs(y_a - y).max(), np.abs(y_b - y).max())
