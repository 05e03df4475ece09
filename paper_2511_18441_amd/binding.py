"""ctypes binding of librecogs.so (include/recogs.h). Argument marshalling only:
every step of the path runs in the HIP library; torch supplies device memory and
the current HIP stream.

The C entry points are exposed under their C names (recogs_select, recogs_recolor,
recogs_render, recogs_render_backward, ...), taking ctypes structs and raw device
pointers; they raise RecogsError on a non-OK status. Helpers below build those
structs from torch tensors and the seeded scene containers.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# RECOGS_LIB: another build of the same sources (the sanitizer run of the host code)
LIB_PATH = os.environ.get("RECOGS_LIB") or os.path.join(_HERE, "librecogs.so")

RECOGS_F32, RECOGS_F16, RECOGS_BF16 = 0, 1, 2
STATUS = {0: "OK", -1: "INVALID", -2: "CAPACITY", -3: "UNSUPPORTED", -4: "HIP"}
STORAGE_CODE = {"f32": RECOGS_F32, "f16": RECOGS_F16, "bf16": RECOGS_BF16}

# every entry point declared in include/recogs.h
ENTRY_POINTS = ("recogs_workspace_bytes", "recogs_workspace_init", "recogs_workspace_readback",
                "recogs_workspace_profile_flush",
                "recogs_workspace_release", "recogs_prepare_covariance", "recogs_select", "recogs_recolor",
                "recogs_render", "recogs_render_backward", "recogs_loss_l2", "recogs_render_backward_sh",
                "recogs_loss_l1", "recogs_adam_step", "recogs_dssim_workspace_bytes", "recogs_loss_dssim",
                "recogs_loss_l1_dssim",
                "recogs_unproject_workspace_bytes", "recogs_unproject", "recogs_reproject_mask", "recogs_tint",
                "recogs_outlier_workspace_bytes", "recogs_remove_outliers", "recogs_render_backward_sh_adam",
                "recogs_workspace_keys_needed", "recogs_unproject_noalloc", "recogs_backward_scratch_bytes",
                "recogs_last_error")


class RecogsError(RuntimeError):
    def __init__(self, fn, status, msg):
        super().__init__(f"{fn} -> {STATUS.get(status, status)}: {msg}")
        self.status = status


class Scene(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("stride", ctypes.c_int64), ("sh_degree", ctypes.c_int32),
                ("storage", ctypes.c_int32), ("means", ctypes.c_void_p), ("cov3d", ctypes.c_void_p),
                ("opacity", ctypes.c_void_p), ("sh", ctypes.c_void_p)]


class Camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3), ("znear", ctypes.c_float)]


class SelectParams(ctypes.Structure):
    _fields_ = [("cx", ctypes.c_float), ("cy", ctypes.c_float), ("radius", ctypes.c_float),
                ("ref", ctypes.c_float * 3), ("color_radius", ctypes.c_float)]


class RenderOpts(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32), ("px_per_thread", ctypes.c_int32),
                ("bg", ctypes.c_float * 3), ("mask", ctypes.c_void_p), ("M", ctypes.c_void_p),
                ("b", ctypes.c_void_p), ("keep_backward_state", ctypes.c_int32), ("profile_stages", ctypes.c_int32),
                ("sort_mode", ctypes.c_int32), ("graph_mode", ctypes.c_int32), ("output_chw", ctypes.c_int32),
                ("depth_map", ctypes.c_void_p), ("depth_tau", ctypes.c_float), ("extent_rule", ctypes.c_int32),
                ("bwd_scratch", ctypes.c_void_p), ("bwd_scratch_bytes", ctypes.c_size_t)]


class Workspace(ctypes.Structure):
    _fields_ = [("base", ctypes.c_void_p), ("bytes", ctypes.c_size_t), ("n_cap", ctypes.c_int64),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("tile_w", ctypes.c_int32),
                ("tile_h", ctypes.c_int32), ("key_capacity", ctypes.c_int64), ("tiles_x", ctypes.c_int32),
                ("tiles_y", ctypes.c_int32)] + \
               [(f, ctypes.c_size_t) for f in (
                   "off_rec", "off_bwd", "off_gpart", "off_zbits", "off_rect", "off_count", "off_offset", "off_scan",
                   "off_keys0", "off_keys1", "off_vals0", "off_vals1", "off_hist", "off_sort_count",
                   "off_ranges", "off_final_T", "off_nproc", "off_header", "off_dkeys0", "off_dkeys1", "off_dvals0",
                   "off_dvals1", "off_dhist", "off_esum", "off_efirst", "scan_chunks", "sort_chunks")] + \
               [("num_keys", ctypes.c_int64), ("num_visible", ctypes.c_int64), ("sort_mode", ctypes.c_int32),
                ("key_bytes", ctypes.c_int32), ("sorted_in_alt", ctypes.c_int32), ("sort_passes", ctypes.c_int32),
                ("depth_passes", ctypes.c_int32), ("key_bits", ctypes.c_int32), ("depth_bits", ctypes.c_int32),
                ("depth_min_bits", ctypes.c_uint32), ("last_n", ctypes.c_int32), ("stage_ms", ctypes.c_float * 9),
                ("stage_ms_sum", ctypes.c_double * 9), ("profiled_frames", ctypes.c_int64),
                ("profile_state", ctypes.c_void_p), ("generation", ctypes.c_int64)]

STAGES = ("preprocess", "scan", "readback", "depth_sort", "emit", "key_sort", "ranges", "tile_sort", "blend")


_lib = None


def lib():
    """Load librecogs.so; raise if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python paper_2511_18441_amd/build.py`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, f32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_float
        P = ctypes.POINTER
        L.recogs_workspace_bytes.argtypes = [i64, i32, i32, i32, i32, i64]
        L.recogs_workspace_bytes.restype = ctypes.c_size_t
        L.recogs_workspace_init.argtypes = [P(Workspace), vp, ctypes.c_size_t, i64, i32, i32, i32, i32, i64]
        L.recogs_workspace_readback.argtypes = [P(Workspace), vp]
        L.recogs_workspace_profile_flush.argtypes = [P(Workspace)]
        L.recogs_workspace_release.argtypes = [P(Workspace)]
        L.recogs_workspace_release.restype = None
        L.recogs_prepare_covariance.argtypes = [vp, vp, vp, i64, i64, vp]
        L.recogs_select.argtypes = [P(Scene), P(Camera), P(SelectParams), vp, vp, vp]
        L.recogs_recolor.argtypes = [P(Scene), vp, vp, vp, vp, i32, vp]
        L.recogs_render.argtypes = [P(Scene), P(Camera), P(RenderOpts), P(Workspace), vp, vp]
        L.recogs_render_backward.argtypes = [P(Scene), P(Camera), P(RenderOpts), P(Workspace), vp, vp, vp, vp, vp, i32,
                                             vp]
        L.recogs_loss_l2.argtypes = [vp, vp, i64, f32, vp, vp, vp]
        L.recogs_render_backward_sh.argtypes = [P(Scene), P(Camera), P(RenderOpts), P(Workspace), vp, vp, vp, vp, vp,
                                                i32, vp]
        L.recogs_workspace_keys_needed.argtypes = [P(Workspace), P(i64), vp]
        L.recogs_backward_scratch_bytes.argtypes = [P(Workspace), P(RenderOpts)]
        L.recogs_backward_scratch_bytes.restype = ctypes.c_size_t
        L.recogs_loss_l1.argtypes = [vp, vp, i64, f32, vp, vp, vp]
        L.recogs_adam_step.argtypes = [vp, vp, vp, vp, i64, f32, f32, f32, f32, i32, vp]
        L.recogs_dssim_workspace_bytes.argtypes = [i32, i32]
        L.recogs_dssim_workspace_bytes.restype = ctypes.c_size_t
        L.recogs_loss_dssim.argtypes = [vp, vp, i32, i32, f32, vp, i32, vp, vp, ctypes.c_size_t, vp]
        L.recogs_loss_l1_dssim.argtypes = [vp, vp, i32, i32, f32, f32, vp, i32, vp, vp, ctypes.c_size_t, vp]
        L.recogs_unproject_workspace_bytes.argtypes = [i32, i32]
        L.recogs_unproject_workspace_bytes.restype = ctypes.c_size_t
        L.recogs_unproject.argtypes = [P(Camera), vp, vp, vp, vp, i64, vp, vp, ctypes.c_size_t, vp]
        L.recogs_unproject_noalloc.argtypes = [P(Camera), vp, vp, vp, vp, i64, vp, vp]
        L.recogs_reproject_mask.argtypes = [P(Camera), vp, i64, i64, f32, vp, f32, vp, vp]
        L.recogs_tint.argtypes = [vp, vp, P(f32), vp, i64, vp]
        L.recogs_render_backward_sh_adam.argtypes = [P(Scene), P(Camera), P(RenderOpts), P(Workspace), vp, vp, vp, vp,
                                                     vp, vp, f32, f32, f32, f32, i32, vp]
        L.recogs_outlier_workspace_bytes.argtypes = [i64]
        L.recogs_outlier_workspace_bytes.restype = ctypes.c_size_t
        L.recogs_remove_outliers.argtypes = [vp, i64, i64, i32, f32, vp, vp, vp, i64, vp, vp, ctypes.c_size_t, vp]
        L.recogs_last_error.restype = ctypes.c_char_p
        for name in ENTRY_POINTS:
            if name not in ("recogs_workspace_bytes", "recogs_last_error", "recogs_workspace_release",
                            "recogs_dssim_workspace_bytes", "recogs_unproject_workspace_bytes",
                            "recogs_outlier_workspace_bytes", "recogs_backward_scratch_bytes"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(fn, status):
    if status != 0:
        raise RecogsError(fn, status, lib().recogs_last_error().decode())
    return status


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream


# ---------------------------------------------------------------------------
# the C entry points under their own names
# ---------------------------------------------------------------------------
def recogs_workspace_bytes(n, width, height, tile_w, tile_h, key_capacity) -> int:
    return int(lib().recogs_workspace_bytes(n, width, height, tile_w, tile_h, key_capacity))


def recogs_workspace_init(ws: Workspace, dev_mem, nbytes, n, width, height, tile_w, tile_h, key_capacity):
    return _check("recogs_workspace_init", lib().recogs_workspace_init(
        ctypes.byref(ws), dev_mem, nbytes, n, width, height, tile_w, tile_h, key_capacity))


def recogs_workspace_readback(ws: Workspace, stream=None):
    return _check("recogs_workspace_readback", lib().recogs_workspace_readback(ctypes.byref(ws), _stream(stream)))


def recogs_workspace_profile_flush(ws: Workspace):
    return _check("recogs_workspace_profile_flush", lib().recogs_workspace_profile_flush(ctypes.byref(ws)))


def recogs_workspace_release(ws: Workspace) -> None:
    lib().recogs_workspace_release(ctypes.byref(ws))


def recogs_prepare_covariance(log_scales, quats, cov3d, n, stride, stream=None):
    return _check("recogs_prepare_covariance", lib().recogs_prepare_covariance(
        log_scales, quats, cov3d, n, stride, _stream(stream)))


def recogs_select(scene: Scene, cam: Camera, params: SelectParams, mask, count, stream=None):
    return _check("recogs_select", lib().recogs_select(ctypes.byref(scene), ctypes.byref(cam), ctypes.byref(params),
                                                       mask, count, _stream(stream)))


def recogs_recolor(scene: Scene, dst_sh, mask, M, b, copy_unselected=0, stream=None):
    return _check("recogs_recolor", lib().recogs_recolor(ctypes.byref(scene), dst_sh, mask, M, b,
                                                         int(copy_unselected), _stream(stream)))


def recogs_render(scene: Scene, cam: Camera, opts: RenderOpts, ws: Workspace, image, stream=None, check=True):
    st = lib().recogs_render(ctypes.byref(scene), ctypes.byref(cam), ctypes.byref(opts), ctypes.byref(ws), image,
                             _stream(stream))
    return _check("recogs_render", st) if check else st


def recogs_render_backward(scene: Scene, cam: Camera, opts: RenderOpts, ws: Workspace, image, dL_dimage,
                           dL_dopacity, dL_dsh_dc, dL_dM, accumulate=0, stream=None):
    return _check("recogs_render_backward", lib().recogs_render_backward(
        ctypes.byref(scene), ctypes.byref(cam), ctypes.byref(opts), ctypes.byref(ws), image, dL_dimage,
        dL_dopacity, dL_dsh_dc, dL_dM, int(accumulate), _stream(stream)))


def recogs_loss_l2(image, target, count, scale, dL_dimage, loss, stream=None):
    return _check("recogs_loss_l2", lib().recogs_loss_l2(image, target, count, float(scale), dL_dimage, loss,
                                                         _stream(stream)))


def recogs_render_backward_sh(scene: Scene, cam: Camera, opts: RenderOpts, ws: Workspace, image, dL_dimage,
                              dL_dopacity, dL_dsh, dL_dM, accumulate=0, stream=None):
    return _check("recogs_render_backward_sh", lib().recogs_render_backward_sh(
        ctypes.byref(scene), ctypes.byref(cam), ctypes.byref(opts), ctypes.byref(ws), image, dL_dimage, dL_dopacity,
        dL_dsh, dL_dM, int(accumulate), _stream(stream)))


def recogs_backward_scratch_bytes(ws: Workspace, opts: RenderOpts) -> int:
    return int(lib().recogs_backward_scratch_bytes(ctypes.byref(ws), ctypes.byref(opts)))


def recogs_workspace_keys_needed(ws: Workspace, stream=None) -> int:
    out = ctypes.c_int64(0)
    _check("recogs_workspace_keys_needed", lib().recogs_workspace_keys_needed(ctypes.byref(ws), ctypes.byref(out),
                                                                              _stream(stream)))
    return int(out.value)


def recogs_render_backward_sh_adam(scene: Scene, cam: Camera, opts: RenderOpts, ws: Workspace, image, dL_dimage,
                                   dL_dopacity, dL_dM, m, v, lr, beta1=0.9, beta2=0.999, eps=1e-15, step=1, stream=None):
    return _check("recogs_render_backward_sh_adam", lib().recogs_render_backward_sh_adam(
        ctypes.byref(scene), ctypes.byref(cam), ctypes.byref(opts), ctypes.byref(ws), image, dL_dimage, dL_dopacity,
        dL_dM, m, v, float(lr), float(beta1), float(beta2), float(eps), int(step), _stream(stream)))


def recogs_loss_l1(image, target, count, scale, dL_dimage, loss, stream=None):
    return _check("recogs_loss_l1", lib().recogs_loss_l1(image, target, count, float(scale), dL_dimage, loss,
                                                         _stream(stream)))


def recogs_adam_step(param, grad, m, v, count, lr, beta1=0.9, beta2=0.999, eps=1e-15, step=1, stream=None):
    return _check("recogs_adam_step", lib().recogs_adam_step(param, grad, m, v, count, float(lr), float(beta1),
                                                             float(beta2), float(eps), int(step), _stream(stream)))


def recogs_unproject_workspace_bytes(width, height) -> int:
    return int(lib().recogs_unproject_workspace_bytes(int(width), int(height)))


def recogs_unproject(cam: Camera, mask, keep, depth, points, capacity, count, workspace, workspace_bytes, stream=None):
    return _check("recogs_unproject", lib().recogs_unproject(ctypes.byref(cam), mask, keep, depth, points, int(capacity),
                                                             count, workspace, int(workspace_bytes), _stream(stream)))


def recogs_unproject_noalloc(cam: Camera, mask, keep, depth, points, capacity, count, stream=None):
    return _check("recogs_unproject_noalloc", lib().recogs_unproject_noalloc(ctypes.byref(cam), mask, keep, depth, points,
                                                                             int(capacity), count, _stream(stream)))


def recogs_reproject_mask(cam: Camera, points, n, stride, quad_px, depth, depth_eps, mask, stream=None):
    return _check("recogs_reproject_mask", lib().recogs_reproject_mask(ctypes.byref(cam), points, int(n), int(stride),
                                                                       float(quad_px), depth, float(depth_eps), mask,
                                                                       _stream(stream)))


def recogs_tint(image, mask, t, out, pixels, stream=None):
    tt = (ctypes.c_float * 3)(*[float(x) for x in t])
    return _check("recogs_tint", lib().recogs_tint(image, mask, tt, out, int(pixels), _stream(stream)))


def unproject(cam, mask, keep, depth, capacity=None):
    """recogs_unproject on device tensors: mask, keep (or None) uint8 (H, W), depth
    float32 (H, W). Returns the points as a (3, count) float32 view of a (3, capacity)
    tensor (capacity defaults to the number of mask pixels) and the selected count."""
    import torch
    c = camera_struct(cam)
    dev = depth.device
    cap = int(mask.numel()) if capacity is None else int(capacity)
    pts = torch.empty((3, max(cap, 1)), dtype=torch.float32, device=dev)
    cnt = torch.zeros(1, dtype=torch.int32, device=dev)
    nb = recogs_unproject_workspace_bytes(cam.width, cam.height)
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    recogs_unproject(c, mask.data_ptr(), keep.data_ptr() if keep is not None else None, depth.data_ptr(),
                     pts.data_ptr(), cap, cnt.data_ptr(), ws.data_ptr(), nb, _stream(None))
    n = int(cnt.item())
    return pts[:, :min(n, cap)], n


def reproject_mask(cam, points, quad_px, depth=None, depth_eps=0.0, mask=None):
    """recogs_reproject_mask of a (3, n) float32 device tensor (any column stride)
    into a uint8 (H, W) mask."""
    import torch
    c = camera_struct(cam)
    if mask is None:
        mask = torch.empty((cam.height, cam.width), dtype=torch.uint8, device=points.device)
    n = points.shape[1]
    stride = points.stride(0) if n > 0 else 0
    if n > 1 and points.stride(1) != 1:
        raise ValueError("points must have unit column stride")
    recogs_reproject_mask(c, points.data_ptr() if n > 0 else None, n, stride, quad_px,
                          depth.data_ptr() if depth is not None else None, depth_eps, mask.data_ptr())
    return mask


def recogs_outlier_workspace_bytes(n) -> int:
    return int(lib().recogs_outlier_workspace_bytes(int(n)))


def recogs_remove_outliers(points, n, stride, k, std_ratio, mean_dist, keep, out_points, out_stride, out_count,
                           workspace, workspace_bytes, stream=None):
    return _check("recogs_remove_outliers", lib().recogs_remove_outliers(
        points, int(n), int(stride), int(k), float(std_ratio), mean_dist, keep, out_points, int(out_stride), out_count,
        workspace, int(workspace_bytes), _stream(stream)))


def remove_outliers(points, k=16, std_ratio=0.007):
    """recogs_remove_outliers of a (3, n) float32 device tensor (unit column stride).
    Returns (kept points (3, m), keep uint8 (n,), mean distances (n,))."""
    import torch
    n = points.shape[1]
    dev = points.device
    if n > 1 and points.stride(1) != 1:
        raise ValueError("points must have unit column stride")
    stride = points.stride(0) if n > 0 else 0
    dmean = torch.empty(max(n, 1), dtype=torch.float32, device=dev)
    keep = torch.empty(max(n, 1), dtype=torch.uint8, device=dev)
    out = torch.empty((3, max(n, 1)), dtype=torch.float32, device=dev)
    cnt = torch.zeros(1, dtype=torch.int32, device=dev)
    nb = recogs_outlier_workspace_bytes(n)
    ws = torch.empty(nb + 256, dtype=torch.uint8, device=dev)
    base = ws.data_ptr()
    aligned = (base + 255) // 256 * 256
    recogs_remove_outliers(points.data_ptr() if n > 0 else None, n, stride, k, std_ratio, dmean.data_ptr(),
                           keep.data_ptr(), out.data_ptr(), max(n, 1), cnt.data_ptr(), aligned, nb)
    m = int(cnt.item())
    return out[:, :m], keep[:n], dmean[:n]


def tint(image, mask, t, out=None):
    """recogs_tint of an (H, W, 3) float32 image with a uint8 (H, W) mask."""
    import torch
    if out is None:
        out = torch.empty_like(image)
    recogs_tint(image.data_ptr(), mask.data_ptr(), t, out.data_ptr(), image.numel() // 3)
    return out


def recogs_dssim_workspace_bytes(width, height) -> int:
    return int(lib().recogs_dssim_workspace_bytes(int(width), int(height)))


def recogs_loss_dssim(image, target, width, height, weight, dL_dimage, accumulate, loss, workspace, workspace_bytes,
                      stream=None):
    return _check("recogs_loss_dssim", lib().recogs_loss_dssim(image, target, int(width), int(height), float(weight),
                                                               dL_dimage, int(accumulate), loss, workspace,
                                                               int(workspace_bytes), _stream(stream)))


def recogs_loss_l1_dssim(image, target, width, height, l1_scale, weight, dL_dimage, accumulate, loss, workspace,
                         workspace_bytes, stream=None):
    return _check("recogs_loss_l1_dssim", lib().recogs_loss_l1_dssim(image, target, int(width), int(height),
                                                                     float(l1_scale), float(weight), dL_dimage,
                                                                     int(accumulate), loss, workspace,
                                                                     int(workspace_bytes), _stream(stream)))


def recogs_last_error() -> str:
    return lib().recogs_last_error().decode()


# ---------------------------------------------------------------------------
# marshalling helpers
# ---------------------------------------------------------------------------
def camera_struct(cam) -> Camera:
    c = Camera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    for k, v in enumerate(np.asarray(cam.R, np.float32).reshape(9)):
        c.R[k] = float(v)
    for k, v in enumerate(np.asarray(cam.t, np.float32).reshape(3)):
        c.t[k] = float(v)
    c.znear = float(cam.znear)
    return c


def select_struct(sp) -> SelectParams:
    p = SelectParams()
    p.cx, p.cy, p.radius = float(sp.cx), float(sp.cy), float(sp.radius)
    for k, v in enumerate(np.asarray(sp.ref, np.float32).reshape(3)):
        p.ref[k] = float(v)
    p.color_radius = float(sp.color_radius)
    return p


def opts_struct(tile=(16, 16), ppt=1, bg=(0.0, 0.0, 0.0), mask=None, M=None, b=None, keep_backward=False,
                profile=False, sort_mode=0, graph_mode=False, chw=False, depth=None, depth_tau=0.5,
                extent_rule=0, bwd_scratch=None) -> RenderOpts:
    o = RenderOpts()
    o.tile_w, o.tile_h = int(tile[0]), int(tile[1])
    o.px_per_thread = int(ppt)
    for k in range(3):
        o.bg[k] = float(bg[k])
    o.mask = mask.data_ptr() if mask is not None else None
    o.M = M.data_ptr() if M is not None else None
    o.b = b.data_ptr() if b is not None else None
    o.keep_backward_state = 1 if keep_backward else 0
    o.profile_stages = int(profile)  # False/True -> 0/1; 2 = accumulate without waiting
    o.sort_mode = int(sort_mode)
    o.graph_mode = 1 if graph_mode else 0
    o.output_chw = 1 if chw else 0
    o.depth_map = depth.data_ptr() if depth is not None else None
    o.depth_tau = float(depth_tau)
    o.extent_rule = int(extent_rule)
    if bwd_scratch is not None:   # a device tensor (e.g. DeviceWorkspace.backward_scratch)
        o.bwd_scratch = bwd_scratch.data_ptr()
        o.bwd_scratch_bytes = bwd_scratch.numel() * bwd_scratch.element_size()
    return o


class DeviceScene:
    """A scene resident in device memory (torch tensors), plus its C view."""

    def __init__(self, scene, device="cuda", stride: Optional[int] = None):
        import torch
        n = scene.n
        self.n = n
        self.stride = n if stride is None else int(stride)
        self.sh_degree = scene.sh_degree
        self.storage = scene.storage
        S = self.stride

        def planes(a, dtype):
            t = torch.zeros((a.shape[0], S), dtype=dtype, device=device)
            if n:
                t[:, :n] = torch.from_numpy(np.ascontiguousarray(a)).to(device)
            return t
        self.means = planes(scene.means, torch.float32)
        self.log_scales = planes(scene.log_scales, torch.float32)
        self.quats = planes(scene.quats, torch.float32)
        tdt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[scene.storage]
        if scene.storage == "bf16":
            op = torch.from_numpy(np.ascontiguousarray(scene.opacity).view(np.int16)).view(torch.bfloat16)
            sh = torch.from_numpy(np.ascontiguousarray(scene.sh).view(np.int16)).view(torch.bfloat16)
        else:
            op = torch.from_numpy(np.ascontiguousarray(scene.opacity))
            sh = torch.from_numpy(np.ascontiguousarray(scene.sh))
        self.opacity = torch.zeros(S, dtype=tdt, device=device)
        self.sh = torch.zeros((sh.shape[0], S), dtype=tdt, device=device)
        if n:
            self.opacity[:n] = op.to(device)
            self.sh[:, :n] = sh.to(device)
        self.cov3d = torch.empty((6, S), dtype=torch.float32, device=device)
        recogs_prepare_covariance(self.log_scales.data_ptr(), self.quats.data_ptr(), self.cov3d.data_ptr(), n, S)

    def c_struct(self, sh=None) -> Scene:
        s = Scene()
        s.n, s.stride, s.sh_degree = self.n, self.stride, self.sh_degree
        s.storage = STORAGE_CODE[self.storage]
        s.means, s.cov3d = self.means.data_ptr(), self.cov3d.data_ptr()
        s.opacity = self.opacity.data_ptr()
        s.sh = (self.sh if sh is None else sh).data_ptr()
        return s


class DeviceWorkspace:
    """Device memory for recogs_render, owned by a torch uint8 tensor."""

    def __init__(self, n, width, height, tile=(16, 16), key_capacity=None, device="cuda"):
        import torch
        self.args = (int(n), int(width), int(height), int(tile[0]), int(tile[1]))
        cap = int(key_capacity if key_capacity is not None else max(1024, 8 * n))
        self.device = device
        self._alloc(cap)

    def _alloc(self, cap):
        import torch
        nbytes = recogs_workspace_bytes(*self.args, cap)
        if nbytes == 0:
            raise RecogsError("recogs_workspace_bytes", -1, "invalid workspace arguments")
        self.release()
        self.mem = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.ws = Workspace()
        recogs_workspace_init(self.ws, self.mem.data_ptr(), nbytes, *self.args, cap)

    def release(self):
        ws = getattr(self, "ws", None)
        if ws is not None and ws.profile_state:
            recogs_workspace_release(ws)

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass

    def readback(self, stream=None):
        """After graph_mode renders: (num_keys, num_visible) of the last one."""
        recogs_workspace_readback(self.ws, stream)
        return int(self.ws.num_keys), int(self.ws.num_visible)

    def blend_time(self):
        """Mean blend milliseconds over the profile_stages=2 renders so far (waits for the
        last one) and their count."""
        recogs_workspace_profile_flush(self.ws)
        n = int(self.ws.profiled_frames)
        return (self.ws.stage_ms_sum[8] / n if n else 0.0), n

    def grow(self, needed):
        self._alloc(int(needed * 1.25) + 1024)

    def backward_scratch(self, tile, ppt):
        """Device scratch for the backward's block form at this tile shape and pixels per
        thread (None where the shape has none), kept for reuse; 256-byte aligned."""
        import torch
        o = opts_struct(tile, ppt)
        nb = recogs_backward_scratch_bytes(self.ws, o)
        if nb == 0:
            return None
        cur = getattr(self, "_bwd", None)
        if cur is None or cur.numel() < nb or cur.data_ptr() % 256:
            self._bwd = torch.empty(nb, dtype=torch.uint8, device=self.device)
        return self._bwd[:nb]

    # views of internal buffers (inspection and tests)
    def view(self, off, count, dtype):
        import torch
        itemsize = torch.empty(0, dtype=dtype).element_size()
        return self.mem[off: off + count * itemsize].view(dtype)

    def keys_sorted(self):
        """Sorted keys: int64 (tile << 32) | depth bits (sort_mode 1) or int32 tile ids (sort_mode 0)."""
        import torch
        K = int(self.ws.num_keys)
        off = self.ws.off_keys1 if self.ws.sorted_in_alt else self.ws.off_keys0
        return self.view(off, K, torch.int64 if self.ws.key_bytes == 8 else torch.int32)

    def vals_sorted(self):
        import torch
        K = int(self.ws.num_keys)
        off = self.ws.off_vals1 if self.ws.sorted_in_alt else self.ws.off_vals0
        return self.view(off, K, torch.int32)

    def counts(self, n):
        import torch
        return self.view(self.ws.off_count, n, torch.int32)

    def offsets(self, n):
        import torch
        return self.view(self.ws.off_offset, n, torch.int32)

    def zbits(self, n):
        import torch
        return self.view(self.ws.off_zbits, n, torch.int32)

    def rects(self, n):
        import torch
        return self.view(self.ws.off_rect, 2 * n, torch.int32).view(n, 2)

    def ranges(self):
        import torch
        T = self.ws.tiles_x * self.ws.tiles_y
        return self.view(self.ws.off_ranges, 2 * T, torch.int32).view(T, 2)

    def final_T(self):
        import torch
        return self.view(self.ws.off_final_T, self.ws.width * self.ws.height, torch.float32).view(
            self.ws.height, self.ws.width)

    def nproc(self):
        import torch
        return self.view(self.ws.off_nproc, self.ws.width * self.ws.height, torch.int32).view(
            self.ws.height, self.ws.width)


def render(dscene: DeviceScene, cam, ws: DeviceWorkspace, tile=(16, 16), ppt=1, bg=(0.0, 0.0, 0.0), mask=None,
           M=None, b=None, keep_backward=False, image=None, sh=None, grow=True, stream=None, profile=False,
           sort_mode=0, graph_mode=False, chw=False, depth=None, depth_tau=0.5, extent_rule=0):
    """recogs_render into a (H, W, 3) float32 tensor ((3, H, W) with chw); grows the
    workspace once when the view needs more tile keys than it holds (eager mode). With
    graph_mode nothing is read back: check ws.readback() (num_keys > key_capacity means
    it overflowed). depth: a (H, W) float32 tensor that receives the rough depth map
    (Sec. 3.2) at threshold depth_tau. extent_rule 1: the 3DGS rasteriser's square."""
    import torch
    c = camera_struct(cam)
    if image is None:
        shape = (3, cam.height, cam.width) if chw else (cam.height, cam.width, 3)
        image = torch.empty(shape, dtype=torch.float32, device=dscene.means.device)
    if depth is not None:
        if tuple(depth.shape) != (cam.height, cam.width) or depth.dtype != torch.float32 or not depth.is_contiguous():
            raise ValueError("depth must be a contiguous float32 (H, W) tensor")
    o = opts_struct(tile, ppt, bg, mask, M, b, keep_backward, profile, sort_mode, graph_mode, chw, depth, depth_tau,
                    extent_rule)
    sc = dscene.c_struct(sh)
    st = recogs_render(sc, c, o, ws.ws, image.data_ptr(), stream, check=False)
    if st == -2 and grow:
        ws.grow(ws.ws.num_keys)
        st = recogs_render(sc, c, o, ws.ws, image.data_ptr(), stream, check=False)
    _check("recogs_render", st)
    return image


# ---------------------------------------------------------------------------
# batched form
# ---------------------------------------------------------------------------
class BatchView(ctypes.Structure):
    _fields_ = [("scene", Scene), ("cam", Camera), ("mask", ctypes.c_void_p), ("M", ctypes.c_void_p),
                ("b", ctypes.c_void_p), ("image", ctypes.c_void_p)]


class BatchWorkspace(ctypes.Structure):
    _fields_ = [("base", ctypes.c_void_p), ("bytes", ctypes.c_size_t), ("nviews", ctypes.c_int32),
                ("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32), ("px_per_thread", ctypes.c_int32),
                ("storage", ctypes.c_int32), ("sh_degree", ctypes.c_int32), ("pairs", ctypes.c_int64),
                ("tiles", ctypes.c_int64), ("key_capacity", ctypes.c_int64), ("tile_bits", ctypes.c_int32),
                ("persistent_blocks", ctypes.c_int32), ("preprocess_blocks", ctypes.c_uint32),
                ("reserved", ctypes.c_int32)] + \
               [(f, ctypes.c_size_t) for f in (
                   "off_views", "off_vtab", "off_rec", "off_zbits", "off_rect", "off_count", "off_offset",
                   "off_dkeys0", "off_dkeys1", "off_dvals0", "off_dvals1", "off_scan", "off_esum", "off_efirst", "off_sort_count",
                   "off_keys0", "off_keys1", "off_vals0", "off_vals1", "off_header", "off_hist", "off_dhist",
                   "off_ranges", "off_order", "scan_chunks")] + \
               [("num_keys", ctypes.c_int64), ("num_visible", ctypes.c_int64), ("overflow", ctypes.c_int32),
                ("sorted_in_alt", ctypes.c_int32)]


BATCH_ENTRY_POINTS = ("recogs_batch_workspace_bytes", "recogs_batch_init", "recogs_render_batch",
                      "recogs_batch_readback")


def _batch_lib():
    L = lib()
    if not getattr(L, "_batch_ready", False):
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        P = ctypes.POINTER
        L.recogs_batch_workspace_bytes.argtypes = [P(BatchView), i32, i32, i32, i64]
        L.recogs_batch_workspace_bytes.restype = ctypes.c_size_t
        L.recogs_batch_init.argtypes = [P(BatchWorkspace), vp, ctypes.c_size_t, P(BatchView), i32, P(RenderOpts), i64]
        L.recogs_batch_init.restype = ctypes.c_int
        L.recogs_render_batch.argtypes = [P(BatchWorkspace), vp]
        L.recogs_render_batch.restype = ctypes.c_int
        L.recogs_batch_readback.argtypes = [P(BatchWorkspace), vp]
        L.recogs_batch_readback.restype = ctypes.c_int
        L._batch_ready = True
    return L


def recogs_batch_workspace_bytes(views, nviews, tile_w, tile_h, key_capacity) -> int:
    return int(_batch_lib().recogs_batch_workspace_bytes(views, nviews, tile_w, tile_h, key_capacity))


def recogs_batch_init(ws: BatchWorkspace, dev_mem, nbytes, views, nviews, opts: RenderOpts, key_capacity):
    return _check("recogs_batch_init", _batch_lib().recogs_batch_init(ctypes.byref(ws), dev_mem, nbytes, views, nviews,
                                                                      ctypes.byref(opts), key_capacity))


def recogs_render_batch(ws: BatchWorkspace, stream=None):
    return _check("recogs_render_batch", _batch_lib().recogs_render_batch(ctypes.byref(ws), _stream(stream)))


def recogs_batch_readback(ws: BatchWorkspace, stream=None):
    return _check("recogs_batch_readback", _batch_lib().recogs_batch_readback(ctypes.byref(ws), _stream(stream)))


class DeviceBatch:
    """A batch of (scene, view) renders: output images (torch tensors), the C view table
    and a workspace. The key capacity, unless given, comes from one dry run (capacity 0:
    the counts are computed, nothing is drawn) times `headroom`."""

    def __init__(self, dscenes, views, tile=(16, 16), ppt=1, bg=(0.0, 0.0, 0.0), key_capacity=None,
                 headroom=1.25, device="cuda", extent_rule=0):
        import torch
        self.dscenes = list(dscenes)
        self.device = device
        self.views_py = list(views)  # (scene index, camera, mask|None, M|None, b|None)
        n = len(self.views_py)
        self.images = [torch.zeros((c.height, c.width, 3), dtype=torch.float32, device=device)
                       for (_, c, *_rest) in self.views_py]
        self.c_views = (BatchView * n)()
        self._keep = []
        for k, (si, cam, mask, M, b) in enumerate(self.views_py):
            bv = self.c_views[k]
            bv.scene = self.dscenes[si].c_struct()
            bv.cam = camera_struct(cam)
            if mask is not None:
                Mc = M.contiguous().reshape(9)
                bc = b.contiguous().reshape(3)
                self._keep += [mask, Mc, bc]
                bv.mask, bv.M, bv.b = mask.data_ptr(), Mc.data_ptr(), bc.data_ptr()
            bv.image = self.images[k].data_ptr()
        self.opts = opts_struct(tile, ppt, bg, extent_rule=extent_rule)
        self.tile, self.ppt = tuple(tile), int(ppt)
        if key_capacity is None:
            self._init(0)
            self.render()
            self.readback()
            key_capacity = int(self.ws.num_keys * headroom) + 1024
        self._init(int(key_capacity))

    def _init(self, cap):
        import torch
        n = len(self.views_py)
        nbytes = recogs_batch_workspace_bytes(self.c_views, n, self.opts.tile_w, self.opts.tile_h, cap)
        if nbytes == 0:
            raise RecogsError("recogs_batch_workspace_bytes", -1, "invalid batch")
        self.mem = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.ws = BatchWorkspace()
        recogs_batch_init(self.ws, self.mem.data_ptr(), nbytes, self.c_views, n, self.opts, cap)

    def render(self, stream=None):
        recogs_render_batch(self.ws, stream)

    def readback(self, stream=None):
        recogs_batch_readback(self.ws, stream)
        return int(self.ws.num_keys), bool(self.ws.overflow)

    def capture_graph(self):
        """A torch.cuda.CUDAGraph (a HIP graph on ROCm) replaying recogs_render_batch."""
        import torch
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.render()  # warm-up on the capture stream
        torch.cuda.current_stream().wait_stream(side)
        with torch.cuda.graph(g):
            self.render()
        return g
