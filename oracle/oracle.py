"""Python face of the FP64 CPU oracle (``recogs_oracle.c``).

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this module. It never imports the HIP
package, and the HIP package never imports it; the two sides meet only in the
seeded arrays produced by ``synth``.

Each function restates one step of the method (paper: ReCoGS, arXiv 2511.18441;
equations cited per function) as a plain definition evaluated in double precision.
Library primitives used as steps: numpy's stable sort for the (tile, depth, index)
order and numpy's cumulative sum for the exclusive scan of tile counts.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "recogs_oracle.c")
# RECOGS_ORACLE_LIB: another build of the same source (the sanitizer run of the host code)
_LIB = os.environ.get("RECOGS_ORACLE_LIB") or os.path.join(_HERE, "liborc.so")

# column layout of the per-Gaussian records (mirrors the enums in recogs_oracle.c)
PCOLS = ["z", "z32", "u", "v", "sa", "sb", "sc", "ca", "cb", "cc", "r", "g", "b",
         "pr", "pg", "pb", "fr", "fg", "fb", "sigma", "qext", "ex", "ey", "det"]
ICOLS = ["status", "pxlo", "pxhi", "pylo", "pyhi", "txlo", "txhi", "tylo", "tyhi",
         "count", "flag", "z32bits", "sel", "rule"]
P = {k: i for i, k in enumerate(PCOLS)}
I = {k: i for i, k in enumerate(ICOLS)}

Y00 = 1.0 / (2.0 * np.sqrt(np.pi))


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP over query windows, strict IEEE doubles)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                        "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Cam(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_double), ("fy", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("R", ctypes.c_double * 9), ("t", ctypes.c_double * 3),
                ("znear", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        vp = ctypes.c_void_p
        i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.orc_sh_basis.argtypes = [i32, f64, f64, f64, vp]
        L.orc_covariance.argtypes = [i64, vp, vp, vp]
        L.orc_project.argtypes = [i64, vp, vp, vp, vp, i32, ctypes.POINTER(_Cam), i32, i32, vp, vp, vp, vp, vp, i32]
        L.orc_select.argtypes = [i64, vp, vp, ctypes.POINTER(_Cam), f64, f64, f64, vp, f64, vp, vp]
        L.orc_recolor.argtypes = [i64, i32, vp, vp, vp, vp, vp]
        L.orc_emit_keys.argtypes = [i64, vp, i32, i64, vp, vp, vp]
        L.orc_emit_keys.restype = i64
        L.orc_render_windows.argtypes = [i64, vp, vp, i32, i32, vp, i64, vp, i32, vp, vp, vp, vp, vp]
        L.orc_depth_windows.argtypes = [i64, vp, vp, i32, i32, f64, i64, vp, vp, vp]
        L.orc_backward.argtypes = [i64, vp, vp, i32, i32, vp, vp, vp, vp, vp, vp, vp]
        L.orc_backward_windows.argtypes = [i64, vp, vp, i32, i32, vp, vp, vp, i64, vp, vp, vp, vp, vp]
        L.orc_ncols.argtypes = [i32]
        L.orc_ncols.restype = i32
        assert L.orc_ncols(0) == len(PCOLS) and L.orc_ncols(1) == len(ICOLS)
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _d(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def camera(cam) -> _Cam:
    c = _Cam()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    for k, v in enumerate(np.asarray(cam.R, np.float32).reshape(9)):
        c.R[k] = float(v)
    for k, v in enumerate(np.asarray(cam.t, np.float32).reshape(3)):
        c.t[k] = float(v)
    c.znear = float(cam.znear)
    return c


# ---------------------------------------------------------------------------
def sh_basis(deg: int, d) -> np.ndarray:
    """Real SH basis values Y_k(d), k < (deg+1)^2, at a unit direction d (eq. 2)."""
    out = np.zeros(16)
    lib().orc_sh_basis(deg, float(d[0]), float(d[1]), float(d[2]), _p(out))
    return out[: (deg + 1) ** 2]


def covariance(log_scales, quats) -> np.ndarray:
    """eq. (1): Sigma = R S S^T R^T; planes xx, xy, xz, yy, yz, zz."""
    ls, q = _d(log_scales), _d(quats)
    n = ls.shape[1]
    out = np.empty((6, n))
    lib().orc_covariance(n, _p(ls), _p(q), _p(out))
    return out


@dataclass
class Projection:
    f: np.ndarray      # (n, len(PCOLS)) float64
    i: np.ndarray      # (n, len(ICOLS)) int64
    tile: tuple
    width: int
    height: int

    def col(self, name):
        return self.f[:, P[name]] if name in P else self.i[:, I[name]]

    @property
    def tiles_x(self):
        return -(-self.width // self.tile[0])

    @property
    def tiles_y(self):
        return -(-self.height // self.tile[1])


def project(scene, cam, tile=(16, 16), cov=None, mask=None, M=None, b=None, extent_rule: int = 0) -> Projection:
    """Per-Gaussian depth, EWA conic, colour (eq. 2, optional fused recolour, eq. 6)
    and tile rectangle (see orc_project): extent_rule 0 = the alpha >= 1/255 box (tiles
    never change a pixel), 1 = the 3DGS rasteriser's ceil(3 sqrt(lambda_max)) square
    (a splat reaches only the pixels of its tiles)."""
    n = scene.n
    means = _d(scene.means)
    if cov is None:
        cov = covariance(scene.log_scales, scene.quats)
    cov = _d(cov)
    op = _d(scene.opacity_f32())
    sh = _d(scene.sh_f32())
    f = np.empty((n, len(PCOLS)))
    i = np.empty((n, len(ICOLS)), dtype=np.int64)
    c = camera(cam)
    mk = Mv = bv = None
    if mask is not None:
        mk = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
        Mv = _d(M).reshape(9)
        bv = _d(b).reshape(3)
    lib().orc_project(n, _p(means), _p(cov), _p(op), _p(sh), scene.sh_degree, ctypes.byref(c),
                      int(tile[0]), int(tile[1]),
                      _p(mk) if mk is not None else None, _p(Mv) if Mv is not None else None,
                      _p(bv) if bv is not None else None, _p(f), _p(i), int(extent_rule))
    return Projection(f, i, tuple(tile), int(cam.width), int(cam.height))


def select(scene, cam, sp):
    """Selection predicate: (mask uint8[n], in-band flag uint8[n])."""
    n = scene.n
    means = _d(scene.means)
    dc = _d(scene.sh_f32()[0:3])
    mask = np.zeros(n, np.uint8)
    flag = np.zeros(n, np.uint8)
    ref = _d(np.asarray(sp.ref, np.float32))
    lib().orc_select(n, _p(means), _p(dc), ctypes.byref(camera(cam)), float(sp.cx), float(sp.cy),
                     float(sp.radius), _p(ref), float(sp.color_radius), _p(mask), _p(flag))
    return mask, flag


def recolor(sh, mask, M, b) -> np.ndarray:
    """Recolour on coefficients (eq. 6 generalised); sh is ([3K], n) float values."""
    sh = _d(sh)
    n = sh.shape[1]
    out = np.empty_like(sh)
    mk = np.ascontiguousarray(np.asarray(mask, np.uint8))
    lib().orc_recolor(n, sh.shape[0] // 3, _p(sh), _p(mk), _p(_d(M).reshape(9)),
                      _p(_d(b).reshape(3)), _p(out))
    return out


def tile_offsets(proj: Projection):
    """Exclusive scan of the per-Gaussian tile counts, and their total K."""
    c = proj.col("count")
    off = np.concatenate([[0], np.cumsum(c)])
    return off[:-1], int(off[-1])


def emit_keys(proj: Projection):
    """(tile, depth bits, index) triplets in emission order."""
    n = proj.f.shape[0]
    K = int(proj.col("count").sum())
    tile = np.empty(K, np.int64)
    zb = np.empty(K, np.int64)
    idx = np.empty(K, np.int64)
    k = lib().orc_emit_keys(n, _p(proj.i), proj.tiles_x, K, _p(tile), _p(zb), _p(idx))
    assert k == K
    return tile, zb, idx


def sorted_keys(proj: Projection):
    """Keys sorted by (tile, float32 depth, index): a stable sort on (tile, depth)."""
    tile, zb, idx = emit_keys(proj)
    order = np.lexsort((idx, zb, tile))
    return tile[order], zb[order], idx[order]


def tile_ranges(tile_sorted: np.ndarray, n_tiles: int) -> np.ndarray:
    """[first, last+1) of each tile in the sorted list; (0, 0) for empty tiles."""
    r = np.zeros((n_tiles, 2), np.int64)
    if tile_sorted.size:
        starts = np.searchsorted(tile_sorted, np.arange(n_tiles), side="left")
        ends = np.searchsorted(tile_sorted, np.arange(n_tiles), side="right")
        nz = ends > starts
        r[nz, 0] = starts[nz]
        r[nz, 1] = ends[nz]
    return r


@dataclass
class PixelResult:
    rgb: np.ndarray     # (npix, 3)
    T: np.ndarray       # (npix,)
    last: np.ndarray    # (npix,) int64, -1 when nothing blended
    nblend: np.ndarray  # (npix,) int64
    slack: np.ndarray   # (npix,)


def render_windows(proj: Projection, windows, bg=(0.0, 0.0, 0.0), brute: bool = False) -> PixelResult:
    """Per-pixel compositing (eq. 3) for the pixels of each window (x0, y0, w, h),
    listed window by window in row-major order."""
    win = np.ascontiguousarray(np.asarray(windows, dtype=np.int32).reshape(-1, 4))
    npix = int((win[:, 2].astype(np.int64) * win[:, 3]).sum())
    rgb = np.empty((npix, 3))
    T = np.empty(npix)
    last = np.empty(npix, np.int64)
    nb = np.empty(npix, np.int64)
    slack = np.empty(npix)
    n = proj.f.shape[0]
    lib().orc_render_windows(n, _p(proj.f), _p(proj.i), proj.width, proj.height, _p(_d(bg)), win.shape[0], _p(win), int(brute),
                             _p(rgb), _p(T), _p(last), _p(nb), _p(slack))
    return PixelResult(rgb, T, last, nb, slack)


def depth_windows(proj: Projection, windows, tau: float = 0.5):
    """Rough depth map (Sec. 3.2) for the pixels of each window: the float32 depth of the
    blended splat whose blending takes the transmittance below tau (0 if it never does),
    and a flag where a float32 evaluation could decide differently. Reading: the paper
    leaves tau unstated; 0.5 makes it the median depth it describes."""
    win = np.ascontiguousarray(np.asarray(windows, dtype=np.int32).reshape(-1, 4))
    npix = int((win[:, 2].astype(np.int64) * win[:, 3]).sum())
    depth = np.empty(npix)
    flag = np.empty(npix, np.int32)
    n = proj.f.shape[0]
    lib().orc_depth_windows(n, _p(proj.f), _p(proj.i), proj.width, proj.height, float(tau), win.shape[0], _p(win),
                            _p(depth), flag.ctypes.data_as(ctypes.c_void_p))
    return depth, flag


def render_image(proj: Projection, bg=(0.0, 0.0, 0.0), brute: bool = False, window: int = 32):
    """Whole image, HWC, via windows of `window` pixels; returns images of each output."""
    W, H = proj.width, proj.height
    wins = [(x, y, min(window, W - x), min(window, H - y))
            for y in range(0, H, window) for x in range(0, W, window)]
    r = render_windows(proj, wins, bg, brute)
    img = np.empty((H, W, 3))
    T = np.empty((H, W))
    last = np.empty((H, W), np.int64)
    nb = np.empty((H, W), np.int64)
    slack = np.empty((H, W))
    o = 0
    for (x, y, w, h) in wins:
        m = w * h
        img[y:y + h, x:x + w] = r.rgb[o:o + m].reshape(h, w, 3)
        T[y:y + h, x:x + w] = r.T[o:o + m].reshape(h, w)
        last[y:y + h, x:x + w] = r.last[o:o + m].reshape(h, w)
        nb[y:y + h, x:x + w] = r.nblend[o:o + m].reshape(h, w)
        slack[y:y + h, x:x + w] = r.slack[o:o + m].reshape(h, w)
        o += m
    return PixelResult(img, T, last, nb, slack)


def loss_l2(y, target) -> float:
    """L = mean over all pixels and channels of (y - t)^2."""
    return float(np.mean((np.asarray(y, np.float64) - np.asarray(target, np.float64)) ** 2))


def loss_l2_grad(y, target, count: Optional[int] = None) -> np.ndarray:
    """dL/dy = 2 (y - t) / count, count = number of pixel channels in the loss."""
    y = np.asarray(y, np.float64)
    count = y.size if count is None else count
    return 2.0 * (y - np.asarray(target, np.float64)) / count


def loss_l1(y, target) -> float:
    """L1 = mean over all pixels and channels of |y - t| (the L1 term of eq. 4; its gradient is in eq. 7)."""
    return float(np.mean(np.abs(np.asarray(y, np.float64) - np.asarray(target, np.float64))))


def loss_l1_grad(y, target, count: Optional[int] = None) -> np.ndarray:
    """dL1/dy = sign(y - t) / count (Sec. 4.1), with sign(0) = 0."""
    y = np.asarray(y, np.float64)
    count = y.size if count is None else count
    return np.sign(y - np.asarray(target, np.float64)) / count


def adam_step(param, grad, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-15):
    """One Adam step (the optimiser that moves the SH coefficients, Sec. 3.3 / 4.1):
    m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2, and with the bias corrections
    m^ = m / (1 - b1^step), v^ = v / (1 - b2^step): p <- p - lr m^ / (sqrt(v^) + eps).
    step counts from 1. Returns (param, m, v), all float64."""
    p, g = np.asarray(param, np.float64), np.asarray(grad, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


SSIM_WINDOW, SSIM_SIGMA, SSIM_C1, SSIM_C2 = 11, 1.5, 0.01 ** 2, 0.03 ** 2


def _ssim_kernel() -> np.ndarray:
    """Normalised 1-D Gaussian of the 11 x 11 SSIM window (sigma 1.5); the 2-D window is
    its outer product."""
    r = np.arange(SSIM_WINDOW) - SSIM_WINDOW // 2
    g = np.exp(-(r * r) / (2.0 * SSIM_SIGMA ** 2))
    return g / g.sum()


def _blur(a: np.ndarray) -> np.ndarray:
    """2-D correlation of an (H, W) array with the window, zero outside the image (the
    window is symmetric, so this is also the convolution)."""
    g = _ssim_kernel()
    h = SSIM_WINDOW // 2
    H, W = a.shape
    p = np.zeros((H + 2 * h, W + 2 * h))
    p[h:h + H, h:h + W] = a
    t = sum(g[k] * p[:, k:k + W] for k in range(SSIM_WINDOW))          # along x
    return sum(g[k] * t[k:k + H, :] for k in range(SSIM_WINDOW))       # along y


def ssim(y, target):
    """Mean SSIM over all pixels and channels of two (H, W, 3) images (the SSIM term of
    eq. 4): per channel, local means, variances and covariance under the 11 x 11 Gaussian
    window (zero padding), S = (2 mu_y mu_t + C1)(2 s_yt + C2) / ((mu_y^2 + mu_t^2 + C1)
    (s_y^2 + s_t^2 + C2)) with C1 = 0.01^2, C2 = 0.03^2. Returns (value, dSSIM/dy).
    The gradient: S depends on y through mu_y = G*y, E_yy = G*(y^2) and E_yt = G*(y t),
    so dS/dy_q = (G * a)_q + 2 y_q (G * b)_q + t_q (G * c)_q with a, b, c the partial
    derivatives of S with respect to those three maps."""
    y = np.asarray(y, np.float64)
    t = np.asarray(target, np.float64)
    H, W, C = y.shape
    total = 0.0
    grad = np.zeros_like(y)
    N = H * W * C
    for c in range(C):
        x, z = y[..., c], t[..., c]
        mx, mz = _blur(x), _blur(z)
        sxx = _blur(x * x) - mx * mx
        szz = _blur(z * z) - mz * mz
        sxz = _blur(x * z) - mx * mz
        l1, l2 = 2 * mx * mz + SSIM_C1, mx * mx + mz * mz + SSIM_C1
        c1, c2 = 2 * sxz + SSIM_C2, sxx + szz + SSIM_C2
        S = l1 * c1 / (l2 * c2)
        total += S.sum()
        dS_dsxz = 2 * l1 / (l2 * c2)
        dS_dsxx = -l1 * c1 / (l2 * c2 * c2)
        dS_dmx = 2 * mz * c1 / (l2 * c2) - l1 * c1 * 2 * mx / (l2 * l2 * c2)
        a = dS_dmx - 2 * mx * dS_dsxx - mz * dS_dsxz      # through mu_x, sigma_x^2 and sigma_xt
        b = dS_dsxx                                       # through E[x^2]
        cc = dS_dsxz                                      # through E[x t]
        grad[..., c] = (_blur(a) + 2 * x * _blur(b) + z * _blur(cc)) / N
    return total / N, grad


@dataclass
class Grads:
    dsigma: np.ndarray   # (n,)
    drgb: np.ndarray     # (n, 3)
    dc0: np.ndarray      # (3, n)
    dM: np.ndarray       # (3, 3)


def backward(proj: Projection, dldy, M=None, bg=(0.0, 0.0, 0.0), windows=None) -> Grads:
    """Gradients of eq. (8) restricted to opacity, SH DC and the recolour matrix.
    With `windows` [(x0, y0, w, h), ...] dL/dy must be zero outside them and only
    their pixels are visited (candidates gathered per window, as for rendering)."""
    n = proj.f.shape[0]
    g = _d(dldy).reshape(proj.height, proj.width, 3)
    Mv = _d(np.eye(3) if M is None else M).reshape(9)
    ds = np.empty(n)
    dr = np.empty((n, 3))
    dc = np.empty((3, n))
    dM = np.empty(9)
    if windows is None:
        lib().orc_backward(n, _p(proj.f), _p(proj.i), proj.width, proj.height, _p(_d(bg)), _p(Mv), _p(g),
                           _p(ds), _p(dr), _p(dc), _p(dM))
    else:
        win = np.ascontiguousarray(np.asarray(windows, dtype=np.int32).reshape(-1, 4))
        inside = np.zeros((proj.height, proj.width), bool)
        for (x0, y0, w, h) in win:
            inside[y0:y0 + h, x0:x0 + w] = True
        if np.any(g[~inside] != 0):
            raise ValueError("dL/dy is nonzero outside the windows")
        lib().orc_backward_windows(n, _p(proj.f), _p(proj.i), proj.width, proj.height, _p(_d(bg)), _p(Mv), _p(g),
                                   len(win), win.ctypes.data_as(ctypes.c_void_p), _p(ds), _p(dr), _p(dc), _p(dM))
    return Grads(ds, dr, dc, dM.reshape(3, 3))


def sh_grad(scene, cam, proj: Projection, grads: Grads, M=None, idx=None) -> np.ndarray:
    """dL/dC for every SH coefficient, planes [3 (deg+1)^2][n] (plane = k * 3 + c, the
    scene's layout). The colour of eq. 2 is linear in the coefficients,
    f_c = sum_k C_{k,c} Y_k(d) with d = (mu - campos) / |mu - campos|, so
    dL/dC_{k,c} = Y_k(d) g_c, where g is the gradient at f: the colour gradient of eq. 8
    masked where max(0, .) clamps and, for Gaussians the fused recolour selected (they
    display M (f + 1/2) + b), multiplied by M^T. Gaussians that reach no pixel get 0.
    With idx, only those Gaussians' columns, [3 (deg+1)^2][len(idx)]."""
    n = proj.f.shape[0]
    cols = np.arange(n) if idx is None else np.asarray(idx, np.int64)
    deg = int(scene.sh_degree)
    K = (deg + 1) ** 2
    Mv = np.eye(3) if M is None else np.asarray(M, np.float64).reshape(3, 3)
    R = np.asarray(cam.R, np.float32).astype(np.float64).reshape(3, 3)
    t = np.asarray(cam.t, np.float32).astype(np.float64)
    campos = -R.T @ t
    means = np.asarray(scene.means, np.float32).astype(np.float64)
    out = np.zeros((3 * K, len(cols)))
    for j, i in enumerate(cols):
        gh = np.array([grads.drgb[i, c] if proj.f[i, P["pr"] + c] > 0 else 0.0 for c in range(3)])
        if not gh.any():
            continue
        g = Mv.T @ gh if proj.i[i, I["sel"]] else gh
        d = means[:, i] - campos
        Y = sh_basis(deg, d / np.linalg.norm(d))
        for k in range(K):
            out[k * 3:(k + 1) * 3, j] = Y[k] * g
    return out
