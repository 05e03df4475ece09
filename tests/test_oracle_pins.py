"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test names what it pins: scipy's spherical harmonics, exact rational
arithmetic, closed forms of special cases (a single Gaussian's footprint,
stacked transmittance, early termination), invariants of eq. (1), eq. (3) and
eq. (6), brute force, and central finite differences for the gradients.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.special as sps

import synth
from tests.scenes_by_hand import Y00, axis_camera, scene_from


# ---------------------------------------------------------------------------
# eq. (2): SH basis
# ---------------------------------------------------------------------------
def _scipy_real_sh(deg, d):
    """Real SH from scipy's complex Y_l^m (Condon-Shortley phase included):
    m > 0: sqrt2 Re Y_l^m; m < 0: sqrt2 Im Y_l^|m|; m = 0: Y_l^0. Index l^2 + l + m."""
    x, y, z = d
    theta = math.acos(max(-1.0, min(1.0, z)))      # polar
    phi = math.atan2(y, x)                          # azimuth
    out = np.zeros((deg + 1) ** 2)
    for l in range(deg + 1):
        for m in range(-l, l + 1):
            Y = sps.sph_harm_y(l, abs(m), theta, phi)
            if m > 0:
                v = math.sqrt(2.0) * Y.real
            elif m < 0:
                v = math.sqrt(2.0) * Y.imag
            else:
                v = Y.real
            out[l * l + l + m] = v
    return out


def test_sh_basis_matches_scipy(orc):
    rng = np.random.default_rng(11)
    for _ in range(200):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        np.testing.assert_allclose(orc.sh_basis(3, d), _scipy_real_sh(3, d), rtol=0, atol=1e-13)


def test_sh_basis_orthonormal(orc):
    # Gauss-Legendre in cos(theta) (exact to degree 15) x uniform phi (exact for |m| sums < 16)
    xs, ws = np.polynomial.legendre.leggauss(8)
    nphi = 16
    G = np.zeros((16, 16))
    for ct, w in zip(xs, ws):
        st = math.sqrt(1 - ct * ct)
        for j in range(nphi):
            ph = 2 * math.pi * j / nphi
            Y = orc.sh_basis(3, (st * math.cos(ph), st * math.sin(ph), ct))
            G += w * (2 * math.pi / nphi) * np.outer(Y, Y)
    np.testing.assert_allclose(G, np.eye(16), atol=1e-13)


def test_projection_colour_uses_basis_at_view_direction(orc):
    """rgb = max(0, sum_k C_k Y_k(d) + 1/2), d = unit(mu - campos), plane k*3+c (eq. 2),
    with the basis taken from scipy."""
    w = synth.make_mid(n=300)
    sc, cam = w.scene, w.view.camera
    pr = orc.project(sc, cam)
    R = cam.R.astype(np.float64)
    campos = -R.T @ cam.t.astype(np.float64)
    sh = sc.sh_f32().astype(np.float64)
    for i in range(0, 300, 7):
        if pr.col("status")[i] == 1:
            continue
        d = sc.means[:, i].astype(np.float64) - campos
        d /= np.linalg.norm(d)
        Y = _scipy_real_sh(3, d)
        f = np.array([sum(sh[k * 3 + c, i] * Y[k] for k in range(16)) for c in range(3)]) + 0.5
        np.testing.assert_allclose([pr.col("r")[i], pr.col("g")[i], pr.col("b")[i]], np.maximum(f, 0), atol=1e-12)


# ---------------------------------------------------------------------------
# eq. (1): covariance
# ---------------------------------------------------------------------------
def test_covariance_spectrum_and_sign_invariance(orc):
    rng = np.random.default_rng(3)
    n = 64
    ls = rng.normal(-2, 0.7, size=(3, n)).astype(np.float32)
    q = rng.standard_normal((4, n)).astype(np.float32)
    cov = orc.covariance(ls, q)
    cov_neg = orc.covariance(ls, -q)
    np.testing.assert_allclose(cov, cov_neg, rtol=1e-15, atol=0)
    for i in range(n):
        S = np.array([[cov[0, i], cov[1, i], cov[2, i]], [cov[1, i], cov[3, i], cov[4, i]],
                      [cov[2, i], cov[4, i], cov[5, i]]])
        ev = np.sort(np.linalg.eigvalsh(S))
        np.testing.assert_allclose(ev, np.sort(np.exp(2 * ls[:, i].astype(np.float64))), rtol=1e-10)
        np.testing.assert_allclose(np.trace(S), np.exp(2 * ls[:, i].astype(np.float64)).sum(), rtol=1e-12)


def test_covariance_axis_aligned_rotation(orc):
    # a 90 degree turn about z swaps the x and y variances: q = (cos45, 0, 0, sin45)
    ls = np.array([[math.log(0.1)], [math.log(0.3)], [math.log(0.2)]], np.float32)
    q = np.array([[math.cos(math.pi / 4)], [0], [0], [math.sin(math.pi / 4)]], np.float32)
    cov = orc.covariance(ls, q)[:, 0]
    s = np.exp(ls[:, 0].astype(np.float64))
    np.testing.assert_allclose(cov[[0, 3, 5]], [s[1] ** 2, s[0] ** 2, s[2] ** 2], rtol=1e-6)
    np.testing.assert_allclose(cov[[1, 2, 4]], 0, atol=1e-8)


# ---------------------------------------------------------------------------
# depth key: float32 rounding of the exact depth
# ---------------------------------------------------------------------------
def _rn_f32(fr: Fraction) -> float:
    """Round an exact rational to the nearest float32 (ties to even) by bracketing."""
    f = np.float32(float(fr))
    best = None
    for cand in (np.nextafter(f, np.float32(-np.inf)), f, np.nextafter(f, np.float32(np.inf))):
        err = abs(Fraction(float(cand)) - fr)
        key = (err, int(np.array(cand, np.float32).view(np.uint32)) & 1)
        if best is None or key < best[0]:
            best = (key, cand)
    return float(best[1])


def test_depth_is_rn_f32_of_exact_value(orc):
    w = synth.make_mid(n=2000)
    sc, cam = w.scene, w.view.camera
    pr = orc.project(sc, cam)
    R = cam.R.astype(np.float32)
    for i in range(0, 2000, 3):
        fr = sum(Fraction(float(R[2, k])) * Fraction(float(sc.means[k, i])) for k in range(3)) + Fraction(float(cam.t[2]))
        assert pr.col("z32")[i] == _rn_f32(fr)
        assert int(pr.col("z32bits")[i]) == int(np.array(_rn_f32(fr), np.float32).view(np.uint32))


# ---------------------------------------------------------------------------
# single-Gaussian footprint: closed forms of the EWA projection
# ---------------------------------------------------------------------------
def test_isotropic_on_axis_footprint_closed_form(orc):
    f, z, s, sigma = 40.0, 2.0, 0.05, 0.8
    cam = axis_camera(32, 32, f, cx=16.0, cy=16.0)
    sc = scene_from([[0, 0, z]], [[math.log(s)] * 3], [sigma], dc_rgb=[[0.9, 0.5, 0.2]])
    pr = orc.project(sc, cam, (8, 8))
    sf = math.exp(float(np.float32(math.log(s))))
    var = (f * sf / z) ** 2 + 0.3
    np.testing.assert_allclose([pr.col("sa")[0], pr.col("sb")[0], pr.col("sc")[0]], [var, 0, var], rtol=1e-12, atol=1e-14)
    assert pr.col("u")[0] == 16.0 and pr.col("v")[0] == 16.0
    img = orc.render_image(pr, brute=True)
    rgb = Y00 * sc.sh_f32()[0:3, 0].astype(np.float64) + 0.5
    yy, xx = np.mgrid[0:32, 0:32] + 0.5
    G = np.exp(-((xx - 16) ** 2 + (yy - 16) ** 2) / (2 * var))
    a = np.minimum(0.99, float(sc.opacity[0]) * G)
    a[a < 1 / 255] = 0
    np.testing.assert_allclose(img.rgb, a[..., None] * rgb, atol=1e-12)
    np.testing.assert_allclose(img.T, 1 - a, atol=1e-12)
    # extent: alpha >= 1/255 iff r^2 <= var (2 ln(255 sigma)); the box adds 1/64 to that level
    ex = math.sqrt(var * (2 * math.log(255 * float(sc.opacity[0])) + 1 / 64))
    assert pr.col("pxlo")[0] == math.ceil(16 - ex - 0.5) and pr.col("pxhi")[0] == math.floor(16 + ex - 0.5)
    assert pr.col("txlo")[0] == pr.col("pxlo")[0] // 8 and pr.col("txhi")[0] == pr.col("pxhi")[0] // 8
    nt = (pr.col("txhi")[0] - pr.col("txlo")[0] + 1) * (pr.col("tyhi")[0] - pr.col("tylo")[0] + 1)
    assert pr.col("count")[0] == nt


def test_anisotropic_and_off_axis_jacobian(orc):
    f, z = 50.0, 3.0
    cam = axis_camera(64, 48, f)
    sx, sy, sz = 0.02, 0.07, 0.11
    x0 = 0.9  # off axis in x: J picks up -f x/z^2 in its third column
    sc = scene_from([[0, 0, z], [x0, 0, z]], [[math.log(sx), math.log(sy), math.log(sz)]] * 2, [0.5, 0.5],
                    dc_rgb=[[0.5, 0.5, 0.5]] * 2)
    pr = orc.project(sc, cam)
    s = np.exp(np.float32([math.log(sx), math.log(sy), math.log(sz)]).astype(np.float64))
    np.testing.assert_allclose([pr.col("sa")[0], pr.col("sb")[0], pr.col("sc")[0]],
                               [(f * s[0] / z) ** 2 + 0.3, 0, (f * s[1] / z) ** 2 + 0.3], rtol=1e-12, atol=1e-14)
    xm = float(np.float32(x0))
    a = (f / z) ** 2 * s[0] ** 2 + (f * xm / z ** 2) ** 2 * s[2] ** 2 + 0.3
    np.testing.assert_allclose([pr.col("sa")[1], pr.col("sb")[1], pr.col("sc")[1]],
                               [a, 0, (f * s[1] / z) ** 2 + 0.3], rtol=1e-12, atol=1e-14)
    assert abs(pr.col("u")[1] - (f * xm / z + 32)) < 1e-12


def test_frustum_clamp_of_jacobian(orc):
    f, z, W = 50.0, 2.0, 64
    cam = axis_camera(W, W, f)
    lim = 1.3 * (W / 2) / f
    x0 = 3.0 * lim * z  # far outside: the Jacobian uses x = lim z
    sc = scene_from([[x0, 0, z]], [[math.log(0.05)] * 3], [0.5], dc_rgb=[[0.5, 0.5, 0.5]])
    pr = orc.project(sc, cam)
    s = math.exp(float(np.float32(math.log(0.05))))
    a = (f / z) ** 2 * s * s + (f * lim * z / z ** 2) ** 2 * s * s + 0.3
    np.testing.assert_allclose(pr.col("sa")[0], a, rtol=1e-9)


# ---------------------------------------------------------------------------
# eq. (3): compositing
# ---------------------------------------------------------------------------
def _stack(orc, alphas, colors, depths=None, idx_order=None):
    """Splats centred exactly on pixel (8, 8)'s centre; alpha there = sigma."""
    k = len(alphas)
    depths = depths if depths is not None else [1.0 + 0.5 * j for j in range(k)]
    cam = axis_camera(16, 16, 20.0, cx=8.5, cy=8.5)
    sc = scene_from([[0, 0, d] for d in depths], [[math.log(0.01)] * 3] * k, alphas, dc_rgb=colors)
    if idx_order is not None:
        sc = sc.subset(np.asarray(idx_order))
    pr = orc.project(sc, cam)
    return orc.render_windows(pr, [(8, 8, 1, 1)], brute=True), sc


def test_transmittance_is_product(orc):
    alphas = [0.3, 0.55, 0.2, 0.7, 0.1]
    r, sc = _stack(orc, alphas, [[0.25, 0.6, 0.9]] * 5)
    a = sc.opacity.astype(np.float64)
    c = Y00 * sc.sh_f32()[0:3, 0].astype(np.float64) + 0.5
    Tf = np.prod(1 - a)
    np.testing.assert_allclose(r.T[0], Tf, rtol=1e-13)
    np.testing.assert_allclose(r.rgb[0], c * (1 - Tf), rtol=1e-13)
    assert r.nblend[0] == 5


def test_early_termination_three_of_four(orc):
    r, sc = _stack(orc, [0.95] * 4, [[1.0, 0.5, 0.25]] * 4)
    a = float(sc.opacity[0])
    assert r.nblend[0] == 3
    np.testing.assert_allclose(r.T[0], (1 - a) ** 3, rtol=1e-13)
    c = Y00 * sc.sh_f32()[0:3, 0].astype(np.float64) + 0.5
    np.testing.assert_allclose(r.rgb[0], c * (1 - (1 - a) ** 3), rtol=1e-12)
    assert abs(r.T[0] - 1.25e-4) < 1e-9


def test_alpha_clamp(orc):
    r, _ = _stack(orc, [0.999, 0.5], [[1, 1, 1], [0, 0, 0]])
    # 0.999 is clamped to 0.99, then T = 0.01, then 0.5 -> T = 0.005
    np.testing.assert_allclose(r.T[0], 0.01 * 0.5, rtol=1e-6)


def test_front_to_back_order_and_index_invariance(orc):
    cols = [[1, 0, 0], [0, 0, 1]]
    r1, sc = _stack(orc, [0.6, 0.5], cols, depths=[1.0, 2.0])
    r2, _ = _stack(orc, [0.5, 0.6], cols[::-1], depths=[2.0, 1.0])
    np.testing.assert_array_equal(r1.rgb, r2.rgb)
    a0, a1 = float(np.float32(0.6)), float(np.float32(0.5))
    c0 = np.maximum(0, Y00 * sc.sh_f32()[0:3, 0].astype(np.float64) + 0.5)
    c1 = np.maximum(0, Y00 * sc.sh_f32()[0:3, 1].astype(np.float64) + 0.5)
    np.testing.assert_allclose(r1.rgb[0], c0 * a0 + c1 * a1 * (1 - a0), rtol=1e-13, atol=1e-15)


def test_equal_depth_ties_break_by_index(orc):
    cols = [[1, 0, 0], [0, 0, 1]]
    r1, sc1 = _stack(orc, [0.6, 0.5], cols, depths=[2.0, 2.0])
    r2, sc2 = _stack(orc, [0.5, 0.6], cols[::-1], depths=[2.0, 2.0])
    c_red = np.maximum(0, Y00 * sc1.sh_f32()[0:3, 0].astype(np.float64) + 0.5)
    c_blue = np.maximum(0, Y00 * sc1.sh_f32()[0:3, 1].astype(np.float64) + 0.5)
    np.testing.assert_allclose(r1.rgb[0], c_red * 0.6 + c_blue * 0.5 * 0.4, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(r2.rgb[0], c_blue * 0.5 + c_red * 0.6 * 0.5, rtol=1e-6, atol=1e-7)


def test_below_alpha_threshold_contributes_nothing(orc):
    w = synth.make_tiny()
    sc = w.scene
    op = sc.opacity.copy()
    weak = np.arange(0, sc.n, 5)
    op[weak] = np.float32(0.9 / 255)
    sc2 = synth.Scene(sc.means, sc.log_scales, sc.quats, op, sc.sh, sc.sh_degree)
    keep = np.setdiff1d(np.arange(sc.n), weak)
    pr2 = orc.project(sc2, w.view.camera)
    assert np.all(pr2.col("count")[weak] == 0) and np.all(pr2.col("status")[weak] == 3)
    img2 = orc.render_image(pr2, brute=True)
    img3 = orc.render_image(orc.project(sc2.subset(keep), w.view.camera), brute=True)
    np.testing.assert_array_equal(img2.rgb, img3.rgb)


def test_behind_camera_is_culled(orc):
    cam = axis_camera(16, 16, 20.0)
    sc = scene_from([[0, 0, -1.0], [0, 0, 0.1], [0, 0, 0.2], [0, 0, 1.0]], [[math.log(0.05)] * 3] * 4,
                    [0.9] * 4, dc_rgb=[[1, 1, 1]] * 4)
    pr = orc.project(sc, cam)
    # z <= near (0.2 rounded to float32) is culled; float32(0.2) exactly on the plane is culled too
    assert list(pr.col("status")[:3]) == [1, 1, 1] and pr.col("status")[3] == 0


def test_brute_force_equals_windowed(orc):
    w = synth.make_tiny()
    pr = orc.project(w.scene, w.view.camera)
    a = orc.render_image(pr, brute=True)
    b = orc.render_image(pr, brute=False, window=16)
    np.testing.assert_array_equal(a.rgb, b.rgb)
    np.testing.assert_array_equal(a.last, b.last)
    np.testing.assert_array_equal(a.slack, b.slack)


def test_cover_invariant_every_contributing_pixel_is_in_a_listed_tile(orc):
    w = synth.make_tiny()
    cam = w.view.camera
    for tile in [(16, 16), (8, 8), (32, 8)]:
        pr = orc.project(w.scene, cam, tile)
        yy, xx = np.mgrid[0:cam.height, 0:cam.width] + 0.5
        for i in np.nonzero(pr.col("status") == 0)[0][::3]:
            dx, dy = xx - pr.col("u")[i], yy - pr.col("v")[i]
            q = pr.col("ca")[i] * dx * dx + 2 * pr.col("cb")[i] * dx * dy + pr.col("cc")[i] * dy * dy
            hit = pr.col("sigma")[i] * np.exp(-0.5 * q) >= 1 / 255
            ys, xs = np.nonzero(hit)
            assert np.all(xs // tile[0] >= pr.col("txlo")[i]) and np.all(xs // tile[0] <= pr.col("txhi")[i])
            assert np.all(ys // tile[1] >= pr.col("tylo")[i]) and np.all(ys // tile[1] <= pr.col("tyhi")[i])


def test_tiled_lists_reproduce_the_per_pixel_definition(orc):
    """Compositing each pixel over its tile's sorted list (keys, sort, ranges) gives
    the per-pixel full-sort result: tiling is pure acceleration."""
    w = synth.make_tiny()
    cam = w.view.camera
    for tile in [(16, 16), (8, 8), (32, 8)]:
        pr = orc.project(w.scene, cam, tile)
        ref = orc.render_image(pr, brute=True)
        ts, zs, ids = orc.sorted_keys(pr)
        ranges = orc.tile_ranges(ts, pr.tiles_x * pr.tiles_y)
        out = np.zeros((cam.height, cam.width, 3))
        for py in range(0, cam.height, 3):
            for px in range(0, cam.width, 3):
                t = (py // tile[1]) * pr.tiles_x + px // tile[0]
                T, C = 1.0, np.zeros(3)
                for j in ids[ranges[t, 0]:ranges[t, 1]]:
                    dx, dy = px + 0.5 - pr.col("u")[j], py + 0.5 - pr.col("v")[j]
                    q = pr.col("ca")[j] * dx * dx + 2 * pr.col("cb")[j] * dx * dy + pr.col("cc")[j] * dy * dy
                    a = pr.col("sigma")[j] * math.exp(-0.5 * q)
                    if a < 1 / 255:
                        continue
                    a = min(a, 0.99)
                    Tn = T * (1 - a)
                    if Tn < 1e-4:
                        break
                    C += np.array([pr.col("r")[j], pr.col("g")[j], pr.col("b")[j]]) * a * T
                    T = Tn
                out[py, px] = C
                np.testing.assert_allclose(out[py, px], ref.rgb[py, px], rtol=0, atol=1e-13)


# ---------------------------------------------------------------------------
# eq. (6): recolour
# ---------------------------------------------------------------------------
def test_recolor_identity_and_permutation_exact(orc):
    w = synth.make_mid(n=500)
    sh = w.scene.sh_f32()
    mask = np.ones(500, np.uint8)
    out = orc.recolor(sh, mask, np.eye(3), np.zeros(3))
    np.testing.assert_array_equal(out, sh.astype(np.float64))
    P = synth.hue_rotation(120.0)
    out = orc.recolor(sh, mask, P, np.zeros(3))
    for k in range(16):
        np.testing.assert_array_equal(out[k * 3:(k + 1) * 3], P.astype(np.float64) @ sh[k * 3:(k + 1) * 3].astype(np.float64))
    # (r, g, b) -> (b, r, g)
    np.testing.assert_array_equal(out[0], sh[2].astype(np.float64))


def test_recolor_is_affine_map_of_displayed_colour(orc):
    """eval(C')(d) + 1/2 = M (eval(C)(d) + 1/2) + b for any direction, with scipy's basis."""
    rng = np.random.default_rng(5)
    w = synth.make_mid(n=50)
    sh = w.scene.sh_f32().astype(np.float64)
    M = np.eye(3) + 0.3 * rng.standard_normal((3, 3))
    b = rng.uniform(-0.2, 0.2, 3)
    M32, b32 = M.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)
    mask = (rng.random(50) < 0.5).astype(np.uint8)
    out = orc.recolor(sh, mask, M32, b32)
    for i in range(50):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        Y = _scipy_real_sh(3, d)
        f = np.array([sum(sh[k * 3 + c, i] * Y[k] for k in range(16)) for c in range(3)]) + 0.5
        f2 = np.array([sum(out[k * 3 + c, i] * Y[k] for k in range(16)) for c in range(3)]) + 0.5
        exp = M32 @ f + b32 if mask[i] else f
        np.testing.assert_allclose(f2, exp, atol=1e-12)


def test_recolor_diagonal_is_the_papers_tint(orc):
    """M = diag(t), b = 0 gives c* = t c on the displayed DC colour (eq. 6)."""
    t = np.array([0.8, 1.2, 0.5])
    sh = synth.make_tiny().scene.sh_f32()
    out = orc.recolor(sh, np.ones(sh.shape[1], np.uint8), np.diag(t).astype(np.float32), np.zeros(3))
    c = Y00 * sh[0:3].astype(np.float64) + 0.5
    c2 = Y00 * out[0:3] + 0.5
    np.testing.assert_allclose(c2, t.astype(np.float32).astype(np.float64)[:, None] * c, atol=1e-12)


# ---------------------------------------------------------------------------
# selection
# ---------------------------------------------------------------------------
def test_selection_hand_placed(orc):
    f, z = 50.0, 2.0
    cam = axis_camera(64, 64, f)  # centre (32, 32)
    # centres projected at distances 0, 9.5, 10.5 px (in the disk r = 10 or not)
    xs = [0.0, 9.5 * z / f, 10.5 * z / f, 0.0, 0.0]
    cols = [[0.8, 0.2, 0.2], [0.8, 0.2, 0.2], [0.8, 0.2, 0.2], [0.8, 0.2, 0.6], [0.8, 0.2, 0.2]]
    zs = [z, z, z, z, -1.0]
    sc = scene_from([[x, 0, zz] for x, zz in zip(xs, zs)], [[math.log(0.05)] * 3] * 5, [0.5] * 5, dc_rgb=cols)
    sp = synth.SelectParams(32.0, 32.0, 10.0, np.array([0.8, 0.2, 0.25], np.float32), float(np.float32(0.1)))
    mask, flag = orc.select(sc, cam, sp)
    assert list(mask) == [1, 1, 0, 0, 0]
    assert not flag.any()
    pr = orc.project(sc, cam)
    assert pr.col("u")[0] == 32.0 and pr.col("v")[0] == 32.0


def test_selection_counts_on_configs(orc):
    w = synth.make_tiny()
    mask, flag = orc.select(w.scene, w.view.camera, w.view.select)
    assert 0 < mask.sum() < w.scene.n and flag.sum() == 0


# ---------------------------------------------------------------------------
# eq. (8): gradients (central finite differences of the oracle's own forward)
# ---------------------------------------------------------------------------
def _loss_and_state(orc, sc, cam, mask, M, b, g):
    pr = orc.project(sc, cam, mask=mask, M=M, b=b)
    r = orc.render_image(pr, brute=True)
    return float((r.rgb * g).sum()), r, pr


def test_windowed_backward_equals_whole_image(orc):
    """With dL/dy zero outside some windows, visiting only their pixels with the
    per-window candidate lists gives the whole-image backward (pixel order aside)."""
    w = synth.make_diff_fd(n=20000, n_sub=600, size=48)
    sc, cam = w.scene, w.view.camera
    rng = np.random.default_rng(21)
    mask = (rng.random(sc.n) < 0.4).astype(np.uint8)
    M = (np.eye(3) + 0.2 * rng.standard_normal((3, 3))).astype(np.float64)
    pr = orc.project(sc, cam, (16, 16), mask=mask, M=M, b=np.zeros(3))
    wins = [(0, 0, 16, 16), (16, 32, 16, 16), (30, 5, 12, 9)]
    g = np.zeros((cam.height, cam.width, 3))
    for (x0, y0, ww, wh) in wins:
        g[y0:y0 + wh, x0:x0 + ww] = rng.standard_normal((wh, ww, 3))
    full = orc.backward(pr, g, M=M)
    part = orc.backward(pr, g, M=M, windows=wins)
    for a, b in ((full.dsigma, part.dsigma), (full.dc0, part.dc0), (full.dM, part.dM)):
        assert np.allclose(a, b, rtol=1e-12, atol=1e-14 * max(1.0, np.abs(a).max()))
    assert np.abs(full.dsigma).max() > 0 and np.abs(full.dM).max() > 0
    with pytest.raises(ValueError):
        orc.backward(pr, np.ones_like(g), M=M, windows=wins)


def test_gradients_match_central_differences(orc):
    w = synth.make_diff_fd(n=20000, n_sub=96, size=24)
    sc, cam = w.scene, w.view.camera
    rng = np.random.default_rng(9)
    mask = (rng.random(sc.n) < 0.5).astype(np.uint8)
    M = (np.eye(3) + 0.2 * rng.standard_normal((3, 3))).astype(np.float64)
    b = np.zeros(3)
    g = rng.standard_normal((cam.height, cam.width, 3))
    L0, r0, pr0 = _loss_and_state(orc, sc, cam, mask, M, b, g)
    gr = orc.backward(pr0, g, M=M)
    assert np.isfinite(gr.dsigma).all()

    def same_decisions(ra, rb):
        return np.array_equal(ra.nblend, rb.nblend) and np.array_equal(ra.last, rb.last)

    h = 1e-6
    checked = 0
    # recolour matrix
    for k in range(9):
        Mp, Mm = M.copy(), M.copy()
        Mp.flat[k] += h
        Mm.flat[k] -= h
        Lp, rp, _ = _loss_and_state(orc, sc, cam, mask, Mp, b, g)
        Lm, rm, _ = _loss_and_state(orc, sc, cam, mask, Mm, b, g)
        if same_decisions(rp, rm):
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - gr.dM.flat[k]) <= 1e-5 * max(1.0, abs(fd)), (k, fd, gr.dM.flat[k])
            checked += 1
    # opacity and DC, on Gaussians that blend somewhere
    used = np.unique(r0.last[r0.last >= 0])
    for i in used[:12]:
        for which in ("sigma", "dc"):
            for c in ((0,) if which == "sigma" else (0, 1, 2)):
                def perturbed(delta):
                    op = sc.opacity.astype(np.float64).copy()
                    sh = sc.sh.astype(np.float64).copy()
                    if which == "sigma":
                        op[i] += delta
                    else:
                        sh[c, i] += delta
                    s2 = synth.Scene(sc.means, sc.log_scales, sc.quats, op, sh, sc.sh_degree)
                    return _scene64_loss(orc, s2, cam, mask, M, b, g)
                (Lp, rp), (Lm, rm) = perturbed(h), perturbed(-h)
                if not same_decisions(rp, rm):
                    continue
                fd = (Lp - Lm) / (2 * h)
                an = gr.dsigma[i] if which == "sigma" else gr.dc0[c, i]
                assert abs(fd - an) <= 1e-5 * max(1.0, abs(fd)), (which, i, c, fd, an)
                checked += 1
    assert checked >= 30


def _scene64_loss(orc, s2, cam, mask, M, b, g):
    """Loss with double-precision opacity/SH arrays (bypasses float32 storage)."""
    from oracle.oracle import _d, _p, camera, lib, Projection, PCOLS, ICOLS
    import ctypes
    n = s2.n
    means = _d(s2.means)
    cov = orc.covariance(s2.log_scales, s2.quats)
    op = _d(s2.opacity)
    sh = _d(s2.sh)
    f = np.empty((n, len(PCOLS)))
    i = np.empty((n, len(ICOLS)), np.int64)
    mk = np.ascontiguousarray(mask.astype(np.uint8))
    c = camera(cam)
    lib().orc_project(n, _p(means), _p(cov), _p(op), _p(sh), s2.sh_degree, ctypes.byref(c), 16, 16,
                      _p(mk), _p(_d(M).reshape(9)), _p(_d(b)), _p(f), _p(i), 0)
    pr = Projection(f, i, (16, 16), cam.width, cam.height)
    r = orc.render_image(pr, brute=True)
    return float((r.rgb * g).sum()), r


def test_gradient_closed_form_single_splat(orc):
    """One degree-0 Gaussian centred on a pixel: y = alpha max(0, M rgb + b)."""
    cam = axis_camera(8, 8, 20.0, cx=4.5, cy=4.5)
    sc = scene_from([[0, 0, 2.0]], [[math.log(0.01)] * 3], [0.6], dc_rgb=[[0.3, 0.6, 0.9]])
    M = np.array([[0.9, 0.1, 0.0], [0.0, 1.1, 0.2], [0.1, 0.0, 0.8]], np.float32).astype(np.float64)
    b = np.zeros(3)
    pr = orc.project(sc, cam, mask=np.ones(1, np.uint8), M=M, b=b)
    g = np.zeros((8, 8, 3))
    g[4, 4] = [1.0, -2.0, 0.5]
    gr = orc.backward(pr, g, M=M)
    a = float(sc.opacity[0])
    rgb = Y00 * sc.sh_f32()[0:3, 0].astype(np.float64) + 0.5
    np.testing.assert_allclose(gr.dM, a * np.outer(g[4, 4], rgb), rtol=1e-12)
    np.testing.assert_allclose(gr.dsigma[0], g[4, 4] @ (M @ rgb), rtol=1e-12)
    np.testing.assert_allclose(gr.dc0[:, 0], Y00 * a * (M.T @ g[4, 4]), rtol=1e-12)


def test_loss_gradient_definition(orc):
    y = np.random.default_rng(0).random((4, 5, 3))
    t = np.random.default_rng(1).random((4, 5, 3))
    g = orc.loss_l2_grad(y, t)
    h = 1e-7
    y2 = y.copy()
    y2[1, 2, 0] += h
    fd = (orc.loss_l2(y2, t) - orc.loss_l2(y, t)) / h
    assert abs(fd - g[1, 2, 0]) < 1e-6


# ---------------------------------------------------------------------------
# background optimiser pieces (Sec. 3.3 / 4.1): L1 term of eq. 4, gradients of every
# SH band (eq. 2 is linear in the coefficients), the Adam step
# ---------------------------------------------------------------------------
def test_sh_grad_matches_central_differences(orc):
    """dL/dC_{k,c} for bands 1..3 (and DC) against central differences of the oracle's
    own forward, with the fused recolour on half of the Gaussians (the M^T chain)."""
    w = synth.make_diff_fd(n=20000, n_sub=96, size=24)
    sc, cam = w.scene, w.view.camera
    rng = np.random.default_rng(19)
    mask = (rng.random(sc.n) < 0.5).astype(np.uint8)
    M = (np.eye(3) + 0.2 * rng.standard_normal((3, 3))).astype(np.float64)
    b = np.zeros(3)
    g = rng.standard_normal((cam.height, cam.width, 3))
    L0, r0, pr0 = _loss_and_state(orc, sc, cam, mask, M, b, g)
    gr = orc.backward(pr0, g, M=M)
    dsh = orc.sh_grad(sc, cam, pr0, gr, M=M)
    K = (sc.sh_degree + 1) ** 2
    assert dsh.shape == (3 * K, sc.n)
    # the DC planes are the DC gradient of eq. 8's chain
    np.testing.assert_allclose(dsh[0:3], gr.dc0, rtol=1e-12, atol=1e-300)

    def same_decisions(ra, rb):
        return np.array_equal(ra.nblend, rb.nblend) and np.array_equal(ra.last, rb.last)

    h = 1e-6
    checked = 0
    used = np.unique(r0.last[r0.last >= 0])
    for i in used[:10]:
        for k in (1, 3, 6, 11, 15):
            c = int(rng.integers(0, 3))
            def perturbed(delta):
                sh = sc.sh.astype(np.float64).copy()
                sh[k * 3 + c, i] += delta
                s2 = synth.Scene(sc.means, sc.log_scales, sc.quats, sc.opacity.astype(np.float64), sh, sc.sh_degree)
                return _scene64_loss(orc, s2, cam, mask, M, b, g)
            (Lp, rp), (Lm, rm) = perturbed(h), perturbed(-h)
            if not same_decisions(rp, rm):
                continue
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - dsh[k * 3 + c, i]) <= 1e-5 * max(1.0, abs(fd)), (i, k, c, fd, dsh[k * 3 + c, i])
            checked += 1
    assert checked >= 30


def test_loss_l1_gradient_definition(orc):
    y = np.random.default_rng(2).random((4, 5, 3))
    t = np.random.default_rng(3).random((4, 5, 3))
    g = orc.loss_l1_grad(y, t)
    h = 1e-7
    for idx in [(1, 2, 0), (3, 4, 2), (0, 0, 1)]:
        y2 = y.copy()
        y2[idx] += h
        fd = (orc.loss_l1(y2, t) - orc.loss_l1(y, t)) / h
        assert abs(fd - g[idx]) < 1e-6
    assert orc.loss_l1_grad(np.ones(4), np.ones(4)).tolist() == [0.0] * 4   # sign(0) = 0


def test_adam_closed_forms(orc):
    """With a constant gradient the bias-corrected moments equal g and g^2 at every
    step, so each step moves a coefficient by lr g / (|g| + eps): the first step, and
    t steps in a row, in closed form."""
    rng = np.random.default_rng(5)
    p0 = rng.standard_normal(50)
    g = rng.standard_normal(50)
    lr, eps = 0.01, 1e-8
    p, m, v = orc.adam_step(p0, g, np.zeros(50), np.zeros(50), 1, lr, eps=eps)
    np.testing.assert_allclose(p, p0 - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    for step in range(2, 8):
        p, m, v = orc.adam_step(p, g, m, v, step, lr, eps=eps)
    np.testing.assert_allclose(p, p0 - 7 * lr * g / (np.abs(g) + eps), rtol=0, atol=1e-13)


def test_ssim_against_brute_force_windows(orc):
    """The SSIM term of eq. 4 against a direct evaluation: for every pixel and channel,
    explicit 11 x 11 window sums with weights g_i g_j (zero outside the image)."""
    rng = np.random.default_rng(4)
    H, W = 6, 7
    y, t = rng.random((H, W, 3)), rng.random((H, W, 3))
    r = np.arange(11) - 5
    g1 = np.exp(-(r * r) / (2 * 1.5 ** 2))
    g1 /= g1.sum()
    tot = 0.0
    for c in range(3):
        for py in range(H):
            for px in range(W):
                s = np.zeros(5)
                for dy in range(-5, 6):
                    for dx in range(-5, 6):
                        qy, qx = py + dy, px + dx
                        if 0 <= qy < H and 0 <= qx < W:
                            a, b = y[qy, qx, c], t[qy, qx, c]
                            s += g1[dy + 5] * g1[dx + 5] * np.array([a, b, a * a, b * b, a * b])
                mx, mt, exx, ett, ext = s
                sx, st, sxt = exx - mx * mx, ett - mt * mt, ext - mx * mt
                tot += (2 * mx * mt + 1e-4) * (2 * sxt + 9e-4) / ((mx * mx + mt * mt + 1e-4) * (sx + st + 9e-4))
    val, _ = orc.ssim(y, t)
    assert abs(val - tot / (H * W * 3)) < 1e-13


def test_ssim_gradient_and_identity(orc):
    rng = np.random.default_rng(6)
    y, t = rng.random((13, 18, 3)), rng.random((13, 18, 3))
    v, g = orc.ssim(y, t)
    h = 1e-6
    for idx in [(0, 0, 0), (6, 9, 1), (12, 17, 2), (2, 16, 0), (12, 0, 1)]:
        yp, ym = y.copy(), y.copy()
        yp[idx] += h
        ym[idx] -= h
        fd = (orc.ssim(yp, t)[0] - orc.ssim(ym, t)[0]) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-8 * max(1.0, abs(fd)), (idx, fd, g[idx])
    one, g0 = orc.ssim(y, y)
    assert abs(one - 1.0) < 1e-14 and np.abs(g0).max() < 1e-15   # a maximum: value 1, gradient 0
