"""Pins of the oracle's rough depth map (Sec. 3.2): the depth of the blended splat at
which the transmittance first falls below tau, 0 where it never does.

Closed forms on hand-placed stacks (the crossing splat for several tau, a strict
threshold, early termination, the alpha threshold and clamp), an identity with the
compositing oracle's own last-blended splat, and monotonicity in tau.
"""
import math

import numpy as np

import synth
from tests.scenes_by_hand import axis_camera, scene_from


def _stack_depth(orc, alphas, depths, tau):
    """Splats centred exactly on pixel (8, 8)'s centre (alpha there = opacity)."""
    k = len(alphas)
    cam = axis_camera(16, 16, 20.0, cx=8.5, cy=8.5)
    sc = scene_from([[0, 0, d] for d in depths], [[math.log(0.01)] * 3] * k, alphas, dc_rgb=[[0.5, 0.5, 0.5]] * k)
    pr = orc.project(sc, cam)
    d, f = orc.depth_windows(pr, [(8, 8, 1, 1)], tau)
    return float(d[0]), int(f[0])


def test_crossing_splat_closed_form(orc):
    # opacity 0.3 four times: T after each = 0.7, 0.49, 0.343, 0.2401
    depths = [1.0, 1.5, 2.0, 2.5]
    for tau, want in [(1.0, 1.0), (0.75, 1.0), (0.7001, 1.0), (0.6999, 1.5), (0.5, 1.5), (0.4, 2.0),
                      (0.3, 2.5), (0.2, 0.0)]:
        d, f = _stack_depth(orc, [0.3] * 4, depths, tau)
        assert d == want, (tau, d)
        assert f == 0, tau


def test_threshold_is_strict(orc):
    # T after the first splat is exactly 1/2 (opacity 0.5 is exact in float32): "lower
    # than" tau = 1/2 happens only at the second splat; the decision is in-band
    d, f = _stack_depth(orc, [0.5, 0.5], [1.0, 3.0], 0.5)
    assert d == 3.0 and f == 1


def test_termination_precludes_crossing(orc):
    a = 0.95
    Ts = [(1 - a) ** k for k in (1, 2, 3)]      # 0.05, 0.0025, 1.25e-4; the fourth would stop
    assert abs(Ts[2] - 1.25e-4) < 1e-9
    d, _ = _stack_depth(orc, [a] * 4, [1.0, 1.5, 2.0, 2.5], 1e-3)
    assert d == 2.0
    d, _ = _stack_depth(orc, [a] * 4, [1.0, 1.5, 2.0, 2.5], 1.2e-4)
    assert d == 0.0   # T stays at 1.25e-4 >= tau: the splat that would cross it is not blended


def test_skipped_and_clamped_splats(orc):
    # opacity 0.9/255 in front is below 1/255 and skipped; 0.999 clamps to 0.99
    d, f = _stack_depth(orc, [0.9 / 255, 0.4, 0.999], [1.0, 2.0, 3.0], 1.0)
    assert d == 2.0 and f == 0
    d, f = _stack_depth(orc, [0.9 / 255, 0.4, 0.999], [1.0, 2.0, 3.0], 0.5)
    assert d == 3.0 and f == 0   # T = 0.6, then 0.006
    d, f = _stack_depth(orc, [0.9 / 255, 0.4, 0.999], [1.0, 2.0, 3.0], 0.005)
    assert d == 0.0 and f == 0   # 0.006 >= 0.005: clamped at 0.99, not at 0.999


def test_last_blended_splat_identity(orc):
    """With tau just above a pixel's final transmittance the crossing splat is the
    compositing oracle's last blended one; just below it, there is none."""
    w = synth.make_tiny()
    cam = w.view.camera
    pr = orc.project(w.scene, cam)
    rng = np.random.default_rng(5)
    xs = rng.integers(0, cam.width, 120)
    ys = rng.integers(0, cam.height, 120)
    wins = [(int(x), int(y), 1, 1) for x, y in zip(xs, ys)]
    r = orc.render_windows(pr, wins)
    z32 = pr.col("z32")
    hits = 0
    for k, win in enumerate(wins):
        if r.last[k] < 0:
            d, _ = orc.depth_windows(pr, [win], 1.0)
            assert d[0] == 0.0
            continue
        hits += 1
        d, _ = orc.depth_windows(pr, [win], r.T[k] * (1 + 1e-9))
        assert d[0] == z32[r.last[k]], k
        d, _ = orc.depth_windows(pr, [win], r.T[k] * (1 - 1e-9))
        assert d[0] == 0.0, k
    assert hits > 60


def test_monotone_in_tau(orc):
    w = synth.make_tiny()
    cam = w.view.camera
    pr = orc.project(w.scene, cam)
    full = [(0, 0, cam.width, cam.height)]
    maps = [orc.depth_windows(pr, full, t)[0] for t in (0.9, 0.5, 0.1)]
    z32 = set(pr.col("z32")[pr.col("status") == 0].tolist())
    for a, b in zip(maps, maps[1:]):
        both = b > 0
        assert np.all(a[both] > 0)              # crossing at a lower tau implies one at a higher tau
        assert np.all(a[both] <= b[both])      # ... no later in the depth order
    for m in maps:
        assert set(m[m > 0].tolist()) <= z32    # every depth is some visible splat's depth
    assert (maps[1] > 0).mean() > 0.2
