"""FP64 oracle of the pixel-selection steps around the renderer (Sec. 3.2, 3.3).

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this module. It never imports the HIP
package, and the HIP package never imports it.

- unproject: a 2D selection (mask), thinned by a sampling mask, lifted to world
  points with a per-pixel depth and the camera (Sec. 3.2, 3D selection);
- reproject_mask: a point cloud drawn into a view as screen-space squares of one
  size, depth-tested against that view's rough depth map, giving the view's
  selection mask (Sec. 3.2 and the per-view mask of Sec. 3.3);
- tint: the edit of Sec. 3.3, c* = t c on the pixels the mask marks.

Camera convention (the one of the projection, eq. 1-2): camera point m = R X + t,
pixel coordinates u = fx m_x / m_z + cx, v = fy m_y / m_z + cy; pixel (x, y) has its
centre at (x + 1/2, y + 1/2).

Readings (the paper gives no formulas for these steps):
- the depth of a pixel is its camera-space z (the depth the rough depth map holds);
  pixels with depth 0 (no surface) are not unprojected;
- a square of side q covers the pixels whose centres lie in [u - q/2, u + q/2) x
  [v - q/2, v + q/2) (so an integer q covers q x q pixels);
- the depth test passes where the view's depth map is 0 (no surface) or the point's
  z <= d (1 + eps), eps a relative tolerance; points with z <= znear are not drawn.
"""
from __future__ import annotations

import math

import numpy as np

_EPS32 = 2.0 ** -24


def _cam(cam):
    R = np.asarray(cam.R, np.float64).reshape(3, 3)
    t = np.asarray(cam.t, np.float64).reshape(3)
    return R, t, float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)


def unproject(cam, mask, keep, depth):
    """World points (P, 3) of the pixels with mask, keep and depth > 0, in row-major
    pixel order, and their flat pixel indices. keep None = every pixel."""
    R, t, fx, fy, cx, cy = _cam(cam)
    H, W = cam.height, cam.width
    mask = np.asarray(mask).reshape(H, W) != 0
    sel = mask if keep is None else mask & (np.asarray(keep).reshape(H, W) != 0)
    d = np.asarray(depth, np.float64).reshape(H, W)
    sel = sel & (d > 0)
    ys, xs = np.nonzero(sel)                      # row-major order
    z = d[ys, xs]
    m = np.stack([z * (xs + 0.5 - cx) / fx, z * (ys + 0.5 - cy) / fy, z], axis=1)
    X = (m - t) @ R                               # R^T (m - t), one point per row
    return X, ys * W + xs


def unproject_tolerance(cam, depth_values):
    """Absolute per-coordinate bound for float32 evaluations of unproject: a few
    float32 rounding steps of the camera-space point and of the rotation."""
    R, t, fx, fy, cx, cy = _cam(cam)
    z = np.abs(np.asarray(depth_values, np.float64))
    span = z * (1.0 + (cam.width + abs(cx)) / fx + (cam.height + abs(cy)) / fy) + np.abs(t).sum()
    return 16 * _EPS32 * span


def _project(cam, X):
    R, t, fx, fy, cx, cy = _cam(cam)
    X = np.asarray(X, np.float64).reshape(-1, 3)
    m = X @ R.T + t
    z = m[:, 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        u = fx * m[:, 0] / z + cx
        v = fy * m[:, 1] / z + cy
    # float32 error of m (three products and two sums per row), carried into u, v
    em = 4 * _EPS32 * (np.abs(X) @ np.abs(R).T + np.abs(t))
    with np.errstate(divide="ignore", invalid="ignore"):
        du = 4 * (fx * (em[:, 0] + np.abs(m[:, 0] / z) * em[:, 2]) / np.abs(z) + 4 * _EPS32 * (np.abs(u) + abs(cx)))
        dv = 4 * (fy * (em[:, 1] + np.abs(m[:, 1] / z) * em[:, 2]) / np.abs(z) + 4 * _EPS32 * (np.abs(v) + abs(cy)))
    return u, v, z, du, dv, em[:, 2]


def reproject_mask(cam, points, quad_px, depth=None, eps=0.0):
    """Selection mask of a view (H, W): pixels covered by the square of side quad_px
    around some point's projection that passes the depth test. Returns (lo, hi):
    lo marks pixels covered whatever float32 rounding does, hi those that may be; a
    float32 evaluation lies between them (lo <= mask <= hi)."""
    H, W = cam.height, cam.width
    lo = np.zeros((H, W), np.uint8)
    hi = np.zeros((H, W), np.uint8)
    X = np.asarray(points, np.float64).reshape(-1, 3)
    if X.shape[0] == 0:
        return lo, hi
    u, v, z, du, dv, dz = _project(cam, X)
    zn = float(np.float32(cam.znear))
    front_sure = z > zn + dz + 4 * _EPS32 * zn
    front_may = z > zn - dz - 4 * _EPS32 * zn
    h = 0.5 * float(quad_px)
    dmap = None if depth is None else np.asarray(depth, np.float64).reshape(H, W)
    r = int(math.ceil(h)) + 2
    ok = front_may & np.isfinite(u) & np.isfinite(v)
    X, u, v, z, du, dv, dz, front_sure = X[ok], u[ok], v[ok], z[ok], du[ok], dv[ok], dz[ok], front_sure[ok]
    bx = np.floor(u).astype(np.int64)
    by = np.floor(v).astype(np.int64)
    for oy in range(-r, r + 1):
        y = by + oy
        cy_ = y + 0.5
        # y + 1/2 in [v - h, v + h): exact decision and its float32 band
        ylo, yhi = cy_ - (v - h), (v + h) - cy_
        by_d = dv + 4 * _EPS32 * (np.abs(v) + h)
        yin_sure = (ylo >= by_d) & (yhi > by_d)
        yin_may = (ylo >= -by_d) & (yhi > -by_d)
        for ox in range(-r, r + 1):
            x = bx + ox
            cx_ = x + 0.5
            xlo, xhi = cx_ - (u - h), (u + h) - cx_
            bx_d = du + 4 * _EPS32 * (np.abs(u) + h)
            xin_sure = (xlo >= bx_d) & (xhi > bx_d)
            xin_may = (xlo >= -bx_d) & (xhi > -bx_d)
            inside = (x >= 0) & (x < W) & (y >= 0) & (y < H)
            sure = inside & xin_sure & yin_sure & front_sure
            may = inside & xin_may & yin_may
            if dmap is not None:
                d = np.zeros_like(u)
                d[inside] = dmap[y[inside], x[inside]]
                lim = d * (1.0 + float(np.float32(eps)))
                band = dz + 4 * _EPS32 * lim
                none = d == 0
                sure &= none | (z <= lim - band)
                may &= none | (z <= lim + band)
            lo[y[sure], x[sure]] = 1
            hi[y[may], x[may]] = 1
    return lo, hi


def reproject_mask_brute(cam, points, quad_px, depth=None, eps=0.0):
    """The same covered-pixel set, exact decisions only, by a loop over every pixel and
    every point (tiny inputs)."""
    R, t, fx, fy, cx, cy = _cam(cam)
    H, W = cam.height, cam.width
    out = np.zeros((H, W), np.uint8)
    h = 0.5 * float(quad_px)
    zn = float(np.float32(cam.znear))
    for X in np.asarray(points, np.float64).reshape(-1, 3):
        m = R @ X + t
        if not m[2] > zn:
            continue
        u = fx * m[0] / m[2] + cx
        v = fy * m[1] / m[2] + cy
        for y in range(H):
            for x in range(W):
                if not (u - h <= x + 0.5 < u + h and v - h <= y + 0.5 < v + h):
                    continue
                if depth is not None:
                    d = float(depth[y][x])
                    if d != 0 and not m[2] <= d * (1.0 + float(np.float32(eps))):
                        continue
                out[y, x] = 1
    return out


def tint(image, mask, t):
    """c* = t c (Sec. 3.3) per channel where mask is set, c elsewhere; image (H, W, 3)
    float32. The float32 result is the product of two float32 values rounded once,
    which is the float64 product (exact) rounded to float32."""
    img = np.asarray(image, np.float32)
    m = np.asarray(mask).reshape(img.shape[:-1]) != 0
    prod = (img.astype(np.float64) * np.asarray(t, np.float32).astype(np.float64)).astype(np.float32)
    return np.where(m[..., None], prod, img)


# ---------------------------------------------------------------------------
# Statistical outlier removal of the unprojected cloud (Sec. 3.2, Fig. 2 caption:
# mean distance to 16 neighbours, standard-deviation scale 0.007).
# Reading: D_i = mean Euclidean distance from point i to its k nearest other points
# (all others when there are fewer than k); mu, sigma = mean and population standard
# deviation of D over the cloud; point i is kept iff D_i <= mu + std_ratio * sigma.
# ---------------------------------------------------------------------------
def knn_mean_distance(points, k=16):
    """D_i for every point of a (P, 3) cloud. The k + 1 smallest distances from a point
    to the cloud include its own zero; their sum is the sum of the k smallest distances
    to the other points (a duplicate's zero and the point's own are interchangeable).
    scipy's k-d tree query is the library step."""
    from scipy.spatial import cKDTree
    X = np.asarray(points, np.float64).reshape(-1, 3)
    P = X.shape[0]
    if P <= 1:
        return np.zeros(P)
    kk = min(k, P - 1)
    d, _ = cKDTree(X).query(X, k=kk + 1)
    return d.reshape(P, kk + 1).sum(axis=1) / kk


def knn_mean_distance_brute(points, k=16):
    """The same by sorting every row of the full distance matrix (tiny clouds)."""
    X = np.asarray(points, np.float64).reshape(-1, 3)
    P = X.shape[0]
    if P <= 1:
        return np.zeros(P)
    kk = min(k, P - 1)
    out = np.empty(P)
    for i in range(P):
        dist = np.sqrt(((X - X[i]) ** 2).sum(axis=1))
        dist = np.delete(dist, i)
        out[i] = np.sort(dist)[:kk].mean()
    return out


def outlier_filter(points, k=16, std_ratio=0.007):
    """(keep, flag, D, threshold): keep[i] = D_i <= mu + std_ratio sigma; flag marks the
    points whose D lies within float32 rounding of the threshold."""
    D = knn_mean_distance(points, k)
    if D.size == 0:
        return np.zeros(0, bool), np.zeros(0, bool), D, 0.0
    mu = D.mean()
    sigma = D.std()
    thr = mu + float(np.float32(std_ratio)) * sigma
    keep = D <= thr
    flag = np.abs(D - thr) <= 1e-5 * max(thr, 1e-30) + 1e-30
    return keep, flag, D, thr
