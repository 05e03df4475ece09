"""Seeded synthetic scenes, cameras and edit parameters.

Every array is drawn from ``numpy.random.default_rng(seed)`` (PCG64). The scenes
are stand-ins for the pre-trained 3D Gaussian Splatting scenes the paper edits
(Sec. 3.1 preliminaries; its MipNeRF360 experiments in Sec. 5 use trained
checkpoints that are not available here), with the parameterisation of eq. (1)
and eq. (2): a mean, a per-axis log-scale, a rotation quaternion (w, x, y, z),
an activated opacity and spherical-harmonic coefficients.

Nothing in this module evaluates the method: covariances, projections, colours
and selections are computed by the HIP library and, independently, by the oracle.
The one constant below, the degree-0 SH basis value, only sets the interval the
DC coefficient is drawn from so that the displayed DC colour is uniform in [0,1].
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# Interval of the DC coefficient: displayed DC colour = coef * Y00 + 1/2 is uniform
# in [0, 1] when coef is uniform in [-1/(2 Y00), 1/(2 Y00)].
_Y00 = 0.28209479177387814
DC_COEF_HALF_RANGE = 0.5 / _Y00

STORAGES = ("f32", "f16", "bf16")


# ----------------------------------------------------------------------------
# storage conversions (round-to-nearest-even)
# ----------------------------------------------------------------------------
def bf16_bits_from_f32(x: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest, ties to even); return the bits."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32)
    bias = ((u >> np.uint32(16)) & np.uint32(1)) + np.uint32(0x7FFF)
    return ((u + bias) >> np.uint32(16)).astype(np.uint16)


def f32_from_bf16_bits(b: np.ndarray) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32)


def f32_to_storage(x: np.ndarray, storage: str) -> np.ndarray:
    if storage == "f32":
        return np.ascontiguousarray(x, dtype=np.float32)
    if storage == "f16":
        return np.ascontiguousarray(x.astype(np.float16))
    if storage == "bf16":
        return bf16_bits_from_f32(x)
    raise ValueError(storage)


def storage_to_f32(a: np.ndarray, storage: str) -> np.ndarray:
    if storage == "f32":
        return np.asarray(a, dtype=np.float32)
    if storage == "f16":
        return np.asarray(a, dtype=np.float16).astype(np.float32)
    if storage == "bf16":
        return f32_from_bf16_bits(a)
    raise ValueError(storage)


# ----------------------------------------------------------------------------
# data containers
# ----------------------------------------------------------------------------
@dataclass
class Camera:
    """Pinhole camera, world->camera (x right, y down, z forward).

    A pixel (px, py) covers [px, px+1) x [py, py+1); its centre is (px+1/2, py+1/2).
    All floating values are float32-representable.
    """
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray          # (3,3) float32, rows are the camera axes in world coordinates
    t: np.ndarray          # (3,) float32, camera-space position of the world origin
    znear: float


@dataclass
class Scene:
    means: np.ndarray       # (3, n) float32 planes x, y, z
    log_scales: np.ndarray  # (3, n) float32
    quats: np.ndarray       # (4, n) float32, (w, x, y, z), unit norm
    opacity: np.ndarray     # (n,) storage dtype, activated opacity in (0, 1)
    sh: np.ndarray          # ((deg+1)^2 * 3, n) storage dtype, plane k*3 + channel
    sh_degree: int
    storage: str = "f32"

    @property
    def n(self) -> int:
        return int(self.means.shape[1])

    def opacity_f32(self) -> np.ndarray:
        return storage_to_f32(self.opacity, self.storage)

    def sh_f32(self) -> np.ndarray:
        return storage_to_f32(self.sh, self.storage)

    def with_storage(self, storage: str) -> "Scene":
        """Same scene with opacity and SH rounded (RNE) from this scene's float32 values."""
        if self.storage != "f32":
            raise ValueError("convert from the float32 form")
        return Scene(self.means, self.log_scales, self.quats,
                     f32_to_storage(self.opacity, storage), f32_to_storage(self.sh, storage),
                     self.sh_degree, storage)

    def subset(self, idx: np.ndarray) -> "Scene":
        return Scene(np.ascontiguousarray(self.means[:, idx]),
                     np.ascontiguousarray(self.log_scales[:, idx]),
                     np.ascontiguousarray(self.quats[:, idx]),
                     np.ascontiguousarray(self.opacity[idx]),
                     np.ascontiguousarray(self.sh[:, idx]), self.sh_degree, self.storage)


@dataclass
class SelectParams:
    """Screen-space disk (centre, radius in pixels) and DC-colour ball (centre, radius)."""
    cx: float
    cy: float
    radius: float
    ref: np.ndarray          # (3,) float32
    color_radius: float


@dataclass
class RecolorParams:
    M: np.ndarray            # (3,3) float32, row-major, acts on RGB column vectors
    b: np.ndarray            # (3,) float32 offset


@dataclass
class View:
    scene: int
    camera: Camera
    select: SelectParams
    recolor: RecolorParams


@dataclass
class Workload:
    name: str
    scenes: List[Scene]
    views: List[View]
    tile: tuple = (16, 16)
    extra: dict = field(default_factory=dict)

    @property
    def scene(self) -> Scene:
        return self.scenes[0]

    @property
    def view(self) -> View:
        return self.views[0]


# ----------------------------------------------------------------------------
# helpers
# ----------------------------------------------------------------------------
def _f32(x) -> float:
    return float(np.float32(x))


def _unit_quats(rng, n) -> np.ndarray:
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q.astype(np.float32)


def _rotation_from_quat(q) -> np.ndarray:
    """Rotation matrix of a unit quaternion (w, x, y, z); used only to orient clusters."""
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def orbit_camera(width: int, height: int, fov_h_deg: float, radius: float,
                 az: float, el: float, znear: float = 0.2) -> Camera:
    """Camera on a sphere of `radius` around the origin, looking at the origin.

    Position C = radius (cos el sin az, sin el, cos el cos az) in a y-up world.
    Camera axes: z_c = -C/|C|, x_c = normalize(z_c x (0,1,0)), y_c = z_c x x_c;
    R has rows (x_c, y_c, z_c) and t = -R C. Square pixels; the horizontal field of
    view sets fx = (W/2)/tan(fov/2); the principal point is the image centre.
    """
    C = radius * np.array([math.cos(el) * math.sin(az), math.sin(el), math.cos(el) * math.cos(az)])
    zc = -C / np.linalg.norm(C)
    xc = np.cross(zc, np.array([0.0, 1.0, 0.0]))
    xc /= np.linalg.norm(xc)
    yc = np.cross(zc, xc)
    R = np.stack([xc, yc, zc]).astype(np.float32)
    t = (-(R.astype(np.float64) @ C)).astype(np.float32)
    fx = _f32((width / 2.0) / math.tan(math.radians(fov_h_deg) / 2.0))
    return Camera(width, height, fx, fx, _f32(width / 2.0), _f32(height / 2.0), R, t, _f32(znear))


def random_orbit(rng, width, height, fov_h_deg, radius, znear=0.2) -> Camera:
    az = rng.uniform(0.0, 2.0 * math.pi)
    el = math.radians(rng.uniform(10.0, 35.0))
    return orbit_camera(width, height, fov_h_deg, radius, az, el, znear)


def hue_rotation(angle_deg: float) -> np.ndarray:
    """Rotation of RGB space by `angle_deg` about the grey axis (1,1,1)/sqrt(3).

    Built in float64 (Rodrigues) and snapped to a 2^-30 grid so that the 120 degree
    case is exactly the cyclic channel permutation (r,g,b) -> (b,r,g).
    """
    th = math.radians(angle_deg)
    k = np.ones(3) / math.sqrt(3.0)
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    M = math.cos(th) * np.eye(3) + math.sin(th) * K + (1 - math.cos(th)) * np.outer(k, k)
    M = np.round(M * 2.0 ** 30) / 2.0 ** 30
    return M.astype(np.float32)


def _sh_planes(rng, n, deg, high_sd) -> np.ndarray:
    K = (deg + 1) ** 2
    sh = np.empty((K * 3, n), dtype=np.float32)
    sh[0:3] = rng.uniform(-DC_COEF_HALF_RANGE, DC_COEF_HALF_RANGE, size=(3, n)).astype(np.float32)
    if K > 1:
        sh[3:] = (high_sd * rng.standard_normal((K * 3 - 3, n), dtype=np.float32))
    return sh


def _sigmoid_normal(rng, n, sd) -> np.ndarray:
    x = sd * rng.standard_normal(n)
    return (1.0 / (1.0 + np.exp(-x))).astype(np.float32)


# ----------------------------------------------------------------------------
# scene families
# ----------------------------------------------------------------------------
def make_scene_tiny_like(rng, n=4096, n_clusters=8) -> Scene:
    """Isotropic clusters: centres U[-1,1]^3, sd 0.2, uniform membership;
    log-scales N(-3.5, 0.5); uniform quaternions; opacity sigmoid(N(0, 1.5));
    SH degree 0 with DC colour U[0,1]^3."""
    centers = rng.uniform(-1.0, 1.0, size=(n_clusters, 3))
    member = rng.integers(0, n_clusters, size=n)
    means = (centers[member] + 0.2 * rng.standard_normal((n, 3))).T.astype(np.float32)
    log_scales = rng.normal(-3.5, 0.5, size=(3, n)).astype(np.float32)
    quats = _unit_quats(rng, n)
    opacity = _sigmoid_normal(rng, n, 1.5)
    sh = _sh_planes(rng, n, 0, 0.0)
    return Scene(np.ascontiguousarray(means), log_scales, quats, opacity, sh, 0, "f32")


def make_scene_mid_like(rng, n: int, deg: int = 3) -> Scene:
    """80 %: 64 anisotropic clusters (centres U[-1.5,1.5]^3, per-axis sd U(0.05,0.4),
    random cluster rotation); 20 %: ground plane x,z ~ U[-2,2], y = -1 + N(0, 0.02).
    Log-scales N(-4.5, 0.6) clipped to [-8, -1]; uniform quaternions; opacity
    sigmoid(N(0, 1.5)); DC colour U[0,1]^3; SH bands 1..deg N(0, 0.05)."""
    n_cl = int(round(0.8 * n))
    n_gp = n - n_cl
    centers = rng.uniform(-1.5, 1.5, size=(64, 3))
    sds = rng.uniform(0.05, 0.4, size=(64, 3))
    rots = np.stack([_rotation_from_quat(q) for q in _unit_quats(rng, 64).T.astype(np.float64)])
    member = rng.integers(0, 64, size=n_cl)
    local = rng.standard_normal((n_cl, 3), dtype=np.float32) * sds[member].astype(np.float32)
    pts_cl = centers[member] + np.einsum("nij,nj->ni", rots[member], local)
    pts_gp = np.empty((n_gp, 3))
    pts_gp[:, 0] = rng.uniform(-2.0, 2.0, size=n_gp)
    pts_gp[:, 2] = rng.uniform(-2.0, 2.0, size=n_gp)
    pts_gp[:, 1] = -1.0 + 0.02 * rng.standard_normal(n_gp)
    means = np.ascontiguousarray(np.concatenate([pts_cl, pts_gp]).T.astype(np.float32))
    log_scales = np.clip(rng.normal(-4.5, 0.6, size=(3, n)), -8.0, -1.0).astype(np.float32)
    quats = _unit_quats(rng, n)
    opacity = _sigmoid_normal(rng, n, 1.5)
    sh = _sh_planes(rng, n, deg, 0.05)
    return Scene(means, log_scales, quats, opacity, sh, deg, "f32")


def _select_ball(rng):
    return rng.uniform(0.2, 0.8, size=3).astype(np.float32)


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------
def make_tiny(seed: int = 0) -> Workload:
    """4,096 Gaussians, SH degree 0, FP32; 128x128, 60 deg FOV, orbit radius 3,
    near 0.2, 16x16 tiles, black background; disk r = 20 px at the centre and
    colour ball 0.35 around (0.8, 0.2, 0.2); recolour = 120 deg hue rotation."""
    rng = np.random.default_rng(seed)
    scene = make_scene_tiny_like(rng)
    cam = random_orbit(rng, 128, 128, 60.0, 3.0)
    sel = SelectParams(64.0, 64.0, 20.0, np.array([0.8, 0.2, 0.2], np.float32), _f32(0.35))
    rec = RecolorParams(hue_rotation(120.0), np.zeros(3, np.float32))
    return Workload("tiny", [scene], [View(0, cam, sel, rec)], (16, 16))


def _affine_recolor(rng, scale=0.2):
    M = (np.eye(3) + scale * rng.standard_normal((3, 3))).astype(np.float32)
    b = rng.uniform(-0.1, 0.1, size=3).astype(np.float32)
    return RecolorParams(M, b)


def make_mid(seed: int = 1, n: int = 200_000) -> Workload:
    """200,000 Gaussians, SH degree 3, FP32; 800x800, 50 deg FOV, orbit radius 4;
    disk r = 120 px at the centre, colour ball 0.3 around a seeded reference;
    recolour M = I + 0.2 N(0,1), b ~ U(-0.1, 0.1)."""
    rng = np.random.default_rng(seed)
    scene = make_scene_mid_like(rng, n)
    cam = random_orbit(rng, 800, 800, 50.0, 4.0)
    sel = SelectParams(400.0, 400.0, 120.0, _select_ball(rng), _f32(0.3))
    rec = _affine_recolor(rng)
    return Workload("mid", [scene], [View(0, cam, sel, rec)], (16, 16))


def make_precision(seed: int = 2, n: int = 1_000_000, storage: str = "f32",
                   width: int = 1920, height: int = 1080) -> Workload:
    """1,000,000 Gaussians generated as the mid scene, SH degree 3; 1920x1080,
    60 deg horizontal FOV, orbit radius 4, 16x16 tiles; the mid scene's selection
    (disk 120 px at the centre) and 3x3 affine recolour. `storage` in f32/f16/bf16
    rounds opacity and SH from the float32 draw. Also draws 64 seeded 32x32 crops."""
    rng = np.random.default_rng(seed)
    scene = make_scene_mid_like(rng, n)
    cam = random_orbit(rng, width, height, 60.0, 4.0)
    sel = SelectParams(_f32(width / 2), _f32(height / 2), 120.0, _select_ball(rng), _f32(0.3))
    rec = _affine_recolor(rng)
    crops = np.stack([rng.integers(0, width - 32 + 1, size=64),
                      rng.integers(0, height - 32 + 1, size=64)], axis=1)
    if storage != "f32":
        scene = scene.with_storage(storage)
    return Workload(f"precision_{storage}", [scene], [View(0, cam, sel, rec)], (16, 16),
                    {"crops": crops})


BATCH_SIZES = (100_000, 250_000, 500_000, 1_000_000, 1_000_000, 1_500_000, 2_000_000, 3_000_000)
BATCH_RES = ((256, 256), (800, 800), (1280, 720), (1920, 1080))


def make_batch(seed_base: int = 3000, sizes=BATCH_SIZES, resolutions=BATCH_RES,
               storage: str = "f16") -> Workload:
    """8 scenes of uneven size generated as the mid scene (seed 3000+s), SH degree 3,
    FP16 storage; 4 views each at 256^2, 800^2, 1280x720, 1920x1080 on seeded orbit
    poses (radius 4, 60 deg horizontal); per view a disk centred uniformly in the
    middle half of the image with r = U[0.05,0.15] min(W,H), colour ball 0.3 around
    a seeded reference, and a hue rotation by a seeded angle."""
    scenes, views = [], []
    for s, n in enumerate(sizes):
        rng = np.random.default_rng(seed_base + s)
        sc = make_scene_mid_like(rng, n)
        scenes.append(sc.with_storage(storage) if storage != "f32" else sc)
        for (w, h) in resolutions:
            cam = random_orbit(rng, w, h, 60.0, 4.0)
            cx = rng.uniform(0.25 * w, 0.75 * w)
            cy = rng.uniform(0.25 * h, 0.75 * h)
            r = rng.uniform(0.05, 0.15) * min(w, h)
            sel = SelectParams(_f32(cx), _f32(cy), _f32(r), _select_ball(rng), _f32(0.3))
            rec = RecolorParams(hue_rotation(rng.uniform(0.0, 360.0)), np.zeros(3, np.float32))
            views.append(View(s, cam, sel, rec))
    return Workload("batch", scenes, views, (16, 16))


def make_diff(seed: int = 4, n: int = 1_000_000, n_views: int = 8,
              width: int = 1280, height: int = 720) -> Workload:
    """1,000,000 Gaussians generated as the mid scene, SH degree 3, FP32; 8 views at
    1280x720 (orbit radius 4, 60 deg horizontal). Selection from view 0 (disk
    r = 0.15 H at the centre, colour ball 0.3) applied in every view. Optimised
    recolour M0 = I + 0.1 N(0,1); target recolour Mt = I + 0.3 N(0,1); target pixel
    noise N(0, 0.01) drawn from `extra['noise_seed']`. For the pixel-selection edit: the
    tint t = (1, 0.6, 0.5) and the seed of the 70% sample of the selected pixels."""
    rng = np.random.default_rng(seed)
    scene = make_scene_mid_like(rng, n)
    cams = [random_orbit(rng, width, height, 60.0, 4.0) for _ in range(n_views)]
    sel = SelectParams(_f32(width / 2), _f32(height / 2), _f32(0.15 * height), _select_ball(rng), _f32(0.3))
    M0 = (np.eye(3) + 0.1 * rng.standard_normal((3, 3))).astype(np.float32)
    Mt = (np.eye(3) + 0.3 * rng.standard_normal((3, 3))).astype(np.float32)
    z = np.zeros(3, np.float32)
    views = [View(0, c, sel, RecolorParams(M0, z)) for c in cams]
    return Workload("diff", [scene], views, (16, 16),
                    {"M_target": Mt, "noise_sd": 0.01, "noise_seed": seed * 1000 + 7,
                     "tint": np.float32([1.0, 0.6, 0.5]), "keep_seed": seed * 1000 + 11})


def make_diff_fd(seed: int = 4, n_sub: int = 4096, size: int = 64, n: int = 1_000_000) -> Workload:
    """Finite-difference subset of the differentiation scene: 4,096 seeded Gaussians
    rendered at 64x64 from view 0's pose (same field of view)."""
    full = make_diff(seed, n)
    rng = np.random.default_rng(seed + 100)
    idx = np.sort(rng.choice(full.scene.n, size=n_sub, replace=False))
    sub = full.scene.subset(idx)
    c = full.view.camera
    cam = Camera(size, size, _f32(c.fx * size / c.width), _f32(c.fx * size / c.width),
                 _f32(size / 2), _f32(size / 2), c.R, c.t, c.znear)
    sel = SelectParams(_f32(size / 2), _f32(size / 2), _f32(0.15 * size), full.view.select.ref,
                       full.view.select.color_radius)
    return Workload("diff_fd", [sub], [View(0, cam, sel, full.view.recolor)], (16, 16),
                    {"M_target": full.extra["M_target"], "noise_sd": 0.01,
                     "noise_seed": full.extra["noise_seed"]})


CONFIG_NAMES = ("tiny", "mid", "precision", "batch", "diff")


def make_config(name: str, **kw) -> Workload:
    return {"tiny": make_tiny, "mid": make_mid, "precision": make_precision,
            "batch": make_batch, "diff": make_diff, "diff_fd": make_diff_fd}[name](**kw)


def target_noise(workload: Workload, shape) -> np.ndarray:
    """Seeded N(0, sd) pixel noise for the differentiation target."""
    rng = np.random.default_rng(workload.extra["noise_seed"])
    return (workload.extra["noise_sd"] * rng.standard_normal(shape)).astype(np.float32)


def random_image(seed: int, shape, scale: float = 1.0) -> np.ndarray:
    """Seeded image-shaped array, e.g. an upstream gradient dL/dy."""
    rng = np.random.default_rng(seed)
    return (scale * rng.standard_normal(shape)).astype(np.float32)


def brush_mask(width: int, height: int, cx: float, cy: float, r: float) -> np.ndarray:
    """A 2D selection as a user's brush would paint it: uint8 (H, W), 1 on the pixels
    whose centres lie in the disk of radius r around (cx, cy)."""
    yy, xx = np.mgrid[0:height, 0:width]
    return (((xx + 0.5 - cx) ** 2 + (yy + 0.5 - cy) ** 2) <= r * r).astype(np.uint8)


def sample_keep(seed: int, mask: np.ndarray, frac: float = 0.7) -> np.ndarray:
    """Uniform sample without replacement of floor(frac * count) of the mask's pixels:
    uint8, 1 on the kept ones (the random draw of the unprojection)."""
    rng = np.random.default_rng(seed)
    flat = np.flatnonzero(np.asarray(mask).reshape(-1))
    keep = np.zeros(np.asarray(mask).size, np.uint8)
    keep[rng.choice(flat, size=int(frac * flat.size), replace=False)] = 1
    return keep.reshape(np.asarray(mask).shape)


def nearby_orbit(cam: Camera, daz: float, del_: float = 0.0) -> Camera:
    """The orbit camera `daz` / `del_` radians of azimuth / elevation away from `cam`
    (same radius, size and field of view), looking at the origin."""
    R = np.asarray(cam.R, np.float64)
    C = -R.T @ np.asarray(cam.t, np.float64)
    r = float(np.linalg.norm(C))
    az = math.atan2(C[0], C[2])
    el = math.asin(C[1] / r)
    fov = 2.0 * math.degrees(math.atan((cam.width / 2.0) / cam.fx))
    return orbit_camera(cam.width, cam.height, fov, r, az + daz, el + del_, cam.znear)
