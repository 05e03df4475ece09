"""Benchmark: recolour + render frames/s of a 1,000,000-Gaussian, SH-degree-3 scene at
1920x1080 (32x32 sort tiles, one pixel per blend thread by default) on one MI355X, with
the roofline of the dominant kernel and the FP64 CPU oracle timed beside it.

A step (frame) = recogs_recolor of the selected Gaussians (out of place, from the
pristine SH into the render copy, so frames do not compound the edit) followed by
recogs_render of the edited scene in graph mode (no host synchronisation inside the
frame; the key count is read back once after the timed frames and checked against the
capacity). The eager mode, which reads the key count back in every frame, is timed
too. Inputs are resident in HBM before timing starts.
The timed frames record HIP events between the render's stages on the render stream
(profile mode 2: recorded, never waited on); the dominant kernel's average duration
comes from those events.

Besides the headline (FP32 storage) the same run measures the other forms on the same
GPU: FP16 and BF16 storage of the same scene, the batched form (8 scenes of 0.1M-3M
Gaussians x 4 views, one HIP-graph replay per batch, tile shape and pixels per thread
from the autotuner; beside it the same 32 renders one call at a time), and the
differentiation form (8 views at 1280x720: forward, L2 loss and backward), the SH refit
(eq. 4 loss and its gradient, eq. 7; Adam), the pixel-selection chain (rough depth map, unprojection, outlier
removal, reprojection, tint) and the selection-driven edit loop of Sec. 3.3.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--storage f32|f16|bf16]
                  [--no-cpu-baseline] [--no-forms] [--forms LIST] [--copy-calibration]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "recolor+render frames/s (1M Gaussians, 1080p) and HBM-roofline fraction"
HBM_PEAK_GBS = 8000.0            # MI355X HBM3E
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X fp32 vector (256 CU x 2.4 GHz, packed FMA)
BLEND_FLOPS_PER_EVAL = 23        # dx, dy, exponent (2 mul + 3 fma), test, exp2, clamp, T, weight, 3 fma
SORT_MODE = 0                    # (tile, depth, index) order: 0 depth-first, 2 tile-first; --sort-mode
BWD_FORM = "tile"                # the backward: "tile" (one workgroup per tile) or "block" (a wave per 8x8 block)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_blend_{tw}x{th}_ppt{ppt}_1M_1080p_f32.traffic.txt")
SQ_FILE = os.path.join(ROOT, "profiles", "k_blend_{tw}x{th}_ppt{ppt}_1M_1080p_f32.sq.txt")
LDS_PEAK_BPS = 128.0 * 256 * 2.4e9   # LDS return rate: 128 B per CU per clock (CDNA3's figure), 256 CUs, 2.4 GHz
BLEND_SOURCES = ("paper_2511_18441_amd/csrc/render_device.hpp", "paper_2511_18441_amd/csrc/kernels_render.hip",
                 "paper_2511_18441_amd/csrc/recogs_internal.hpp")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def blend_source_sha1():
    h = hashlib.sha1()
    for p in BLEND_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def recorded_traffic(kernel, tile, ppt):
    """HBM bytes per launch of `kernel` from the committed rocprof counter summary, or
    None when there is none or the blend sources changed since it was taken."""
    path = TRAFFIC_FILE.format(tw=tile[0], th=tile[1], ppt=ppt)
    try:
        kv = dict(l.split(":", 1) for l in open(path).read().splitlines() if ":" in l and not l.startswith("#"))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("kernel") != kernel or kv.get("blend_sources_sha1") != blend_source_sha1():
        return None
    try:
        return int(float(kv["traffic_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def recorded_sq(kernel, tile, ppt):
    """The blend's shader-instruction counters per launch from the committed rocprof
    summary ({name: value}), or None when there is none or the blend sources changed."""
    try:
        kv = dict(l.split(":", 1) for l in open(SQ_FILE.format(tw=tile[0], th=tile[1], ppt=ppt)).read().splitlines()
                  if ":" in l and not l.startswith("#"))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("kernel") != kernel or kv.get("blend_sources_sha1") != blend_source_sha1():
        return None
    try:
        return {k: int(float(v)) for k, v in kv.items() if k not in ("kernel", "blend_sources_sha1")}
    except ValueError:
        return None


def algorithmic_model(st, storage_bytes, deg, keep_bwd=False, sort_mode=0):
    """Bytes (and blend flops) each stage must move for this frame's counts. Sort mode 0:
    depth sort of the V Gaussians with keys, emission in depth order, then 32-bit tile
    keys; mode 2: emission in index order, 32-bit tile keys, then each tile's list
    sorted by depth (list read, depth bits gathered, list written)."""
    N, V, K, S, P, Pd, T, Pix, E, Keff = (st[k] for k in ("N", "V", "K", "S", "passes", "dpasses", "tiles", "pix",
                                                           "evals", "keff"))
    nc = 3 * (deg + 1) ** 2
    b = {
        "recolor": N * 1 + S * nc * storage_bytes * 2,
        "preprocess": N * (12 + 24 + storage_bytes) + V * nc * storage_bytes + V * 48 + N * 16 + (V * 16 if keep_bwd else 0),
        "key_sort": K * 4 + P * K * 16,
        "ranges": K * 4 + T * 8,
        "blend": Keff * 52 + T * 8 + Pix * (20 if keep_bwd else 12),
    }
    if sort_mode == 2:
        b["scan"] = N * 12 + V * 8 + V * 16        # counts, depth bits, offsets; rectangles read, compaction written
        b["emit"] = V * 16 + K * 8
        b["tile_sort"] = K * 12
    else:
        b["scan"] = N * 8 + V * 12
        b["depth_sort"] = V * 4 + Pd * V * 16
        b["emit"] = V * 16 + K * 8
    return b, {"blend": E * BLEND_FLOPS_PER_EVAL}


class Single:
    """One scene + view resident on the GPU, with its selection mask, recolour and
    workspace: a frame is recolour (selected, out of place) + render."""

    def __init__(self, R, w, dev, tile, ppt, chw=False):
        import torch
        self.R, self.w, self.tile, self.ppt, self.chw = R, w, tuple(tile), int(ppt), bool(chw)
        v = w.view
        self.cam = v.camera
        self.n = w.scene.n
        self.d = R.DeviceScene(w.scene, device=dev)
        self.scs = self.d.c_struct()
        self.camc = R.camera_struct(self.cam)
        self.selc = R.select_struct(v.select)
        self.mask = torch.empty(self.n, dtype=torch.uint8, device=dev)
        self.count = torch.empty(1, dtype=torch.int32, device=dev)
        self.select()
        self.M = torch.from_numpy(v.recolor.M.reshape(9)).to(dev)
        self.b = torch.from_numpy(v.recolor.b).to(dev)
        self.render_sh = self.d.sh.clone()
        self.ws = R.DeviceWorkspace(self.n, self.cam.width, self.cam.height, self.tile, key_capacity=16 * self.n,
                                    device=dev)
        shape = (3, self.cam.height, self.cam.width) if self.chw else (self.cam.height, self.cam.width, 3)
        self.image = torch.empty(shape, dtype=torch.float32, device=dev)

    def select(self):
        self.R.recogs_select(self.scs, self.camc, self.selc, self.mask.data_ptr(), self.count.data_ptr())

    def recolor(self):
        self.R.recogs_recolor(self.scs, self.render_sh.data_ptr(), self.mask.data_ptr(), self.M.data_ptr(),
                              self.b.data_ptr(), 0)

    def frame(self, profile=0, graph_mode=True):
        self.recolor()
        self.R.render(self.d, self.cam, self.ws, self.tile, self.ppt, image=self.image, sh=self.render_sh,
                      profile=profile, graph_mode=graph_mode, chw=self.chw, sort_mode=SORT_MODE)

    def timed(self, steps, profile, graph_mode=True):
        """Wall-clock ms per frame over `steps` frames, bracketed by device syncs."""
        import torch
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            self.frame(profile, graph_mode)
        torch.cuda.synchronize()
        return 1000.0 * (time.perf_counter() - t0) / steps

    def event_ms(self, fn, reps):
        import torch
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    def measure(self, steps, warmup):
        """Warm-up; the timed frames, whose blend launches are bracketed by HIP events on
        the render stream (mode 2: recorded, never waited on); the same number of frames
        without any event (overhead check); then a short pass with events between all
        stages (mode 1, waits per frame) for the per-stage breakdown."""
        import numpy as np
        for _ in range(warmup):
            self.frame()
        ws = self.ws.ws
        self.R.recogs_workspace_profile_flush(ws)
        for k in range(len(ws.stage_ms_sum)):
            ws.stage_ms_sum[k] = 0.0
        ws.profiled_frames = 0
        ms = self.timed(steps, 2)
        blend_ms, nfr = self.ws.blend_time()
        k, _ = self.ws.readback()
        if k > self.ws.ws.key_capacity:
            raise RuntimeError(f"the view needs {k} keys, the workspace holds {self.ws.ws.key_capacity}")
        ms_plain = self.timed(steps, 0)
        ms_eager = self.timed(steps, 0, graph_mode=False)
        nprof = max(5, min(20, steps))
        acc = np.zeros(len(ws.stage_ms))
        for _ in range(nprof):
            self.frame(1, graph_mode=False)
            acc += np.array(ws.stage_ms[:])
        stages = dict(zip(self.R.binding.STAGES, (acc / nprof).tolist()))
        stages["recolor"] = self.event_ms(self.recolor, max(10, steps // 2))
        sel_ms = self.event_ms(self.select, max(10, steps // 2))
        return {"ms": ms, "ms_no_events": ms_plain, "ms_eager": ms_eager, "stages": stages, "blend_ms_timed": blend_ms,
                "profiled_frames": nfr, "select_ms": sel_ms}

    def counts(self):
        """Counts of the frame. K, V and the sort passes are those of the timed launch
        shape. The blend's nominal work (`evals`) is fixed independently of that shape:
        per pixel, the entries of its 16x16-tile list (the tiling of the 3DGS rasteriser
        the paper builds on) up to and including its last blended splat, summed over
        pixels; one more render at 16x16 tiles that also writes the per-pixel state
        gives it. `keff` is the per-tile maximum of that count, summed over 16x16 tiles."""
        import torch
        self.R.render(self.d, self.cam, self.ws, self.tile, self.ppt, image=self.image, sh=self.render_sh,
                      sort_mode=SORT_MODE)
        ws = self.ws
        K = int(ws.ws.num_keys)
        cnt = ws.counts(self.n)
        V = int((cnt != 0).sum().item())
        S = int(self.count.item())
        T = ws.ws.tiles_x * ws.ws.tiles_y
        passes, dpasses = int(ws.ws.sort_passes), int(ws.ws.depth_passes)
        ref = self.R.DeviceWorkspace(self.n, self.cam.width, self.cam.height, (16, 16), key_capacity=16 * self.n,
                                     device=self.image.device)
        self.R.render(self.d, self.cam, ref, (16, 16), 1, image=self.image, sh=self.render_sh, keep_backward=True,
                      sort_mode=SORT_MODE)
        nproc = ref.nproc().to(torch.int64)
        E = int(nproc.sum().item())
        Hp, Wp = ref.ws.tiles_y * 16, ref.ws.tiles_x * 16
        npad = torch.zeros((Hp, Wp), dtype=torch.int64, device=nproc.device)
        npad[:self.cam.height, :self.cam.width] = nproc
        keff = int(npad.view(ref.ws.tiles_y, 16, ref.ws.tiles_x, 16).amax(dim=(1, 3)).sum().item())
        del ref
        return dict(N=self.n, V=V, K=K, S=S, passes=passes, dpasses=dpasses, tiles=T,
                    pix=self.cam.width * self.cam.height, evals=E, keff=keff)


def stage_table(stages, bytes_, flops, st):
    if SORT_MODE == 0:
        # the count scan: reduce, rowscan and down (which also does the depth sort's first
        # pass); the emission: offsets and down (its reduce is in the depth sort's last
        # pass, and it counts the key sort's first digit, whose up pass is then skipped)
        launches = {"key_sort": max(0, 3 * st["passes"] - 1), "depth_sort": 3 * st["dpasses"], "scan": 3, "emit": 2}
    else:
        launches = {"key_sort": 3 * st["passes"], "depth_sort": 3 * st["dpasses"]}
    out = {}
    for k, t in stages.items():
        if k == "readback" or k not in bytes_:   # (the stages this sort mode does not run)
            continue
        nl = max(1, launches.get(k, 1))
        ent = {"ms_per_frame": round(t, 4), "launches": nl, "avg_launch_ms": round(t / nl, 4)}
        if k in bytes_ and t > 0:
            ent["alg_bytes"] = int(bytes_[k])
            ent["GBps"] = round(bytes_[k] / (t * 1e-3) / 1e9, 1)
        if k in flops and t > 0:
            ent["TFLOPs"] = round(flops[k] / (t * 1e-3) / 1e12, 2)
        out[k] = ent
    return out, launches


def form_single(R, storage, tile, ppt, steps, warmup, dev):
    import synth
    log(f"bench: form {storage} storage")
    w = synth.make_precision(storage=storage)
    s = Single(R, w, dev, tile, ppt)
    m = s.measure(steps, warmup)
    st = s.counts()
    sb = {"f32": 4, "f16": 2, "bf16": 2}[storage]
    bytes_, _ = algorithmic_model(st, sb, w.scene.sh_degree, sort_mode=SORT_MODE)
    fps = 1000.0 / m["ms"]
    tot = sum(bytes_.values())
    res = {"storage": storage, "frames_per_s": round(fps, 2), "ms_per_frame": round(m["ms"], 4),
           "gaussians_per_s": round(fps * s.n, 1), "blend_ms": round(m["blend_ms_timed"], 4),
           "preprocess_ms": round(m["stages"]["preprocess"], 4), "recolor_ms": round(m["stages"]["recolor"], 4),
           "frame_hbm_frac": round(tot * fps / 1e9 / HBM_PEAK_GBS, 4), "K": st["K"], "V": st["V"]}
    del s
    return res


def form_batch(R, steps, warmup, dev):
    """8 scenes (0.1M..3M Gaussians, FP16, SH 3) x 4 views, each view with its own
    selection and hue rotation fused into the render; one HIP-graph replay per batch."""
    import torch

    import synth
    from paper_2511_18441_amd import autotune
    log("bench: form batch: generating 8 scenes (9.35M Gaussians)")
    w = synth.make_batch()
    dscenes = [R.DeviceScene(sc, device=dev) for sc in w.scenes]
    views = []
    for v in w.views:
        d = dscenes[v.scene]
        mask = torch.zeros(max(d.n, 1), dtype=torch.uint8, device=dev)
        cnt = torch.zeros(1, dtype=torch.int32, device=dev)
        R.recogs_select(d.c_struct(), R.camera_struct(v.camera), R.select_struct(v.select), mask.data_ptr(),
                        cnt.data_ptr())
        views.append((v.scene, v.camera, mask, torch.from_numpy(v.recolor.M.reshape(9).copy()).to(dev),
                      torch.from_numpy(v.recolor.b.copy()).to(dev)))
    log("bench: form batch: autotuning the blend shape")
    tuned = autotune.tune_batch(dscenes, views, reps=3, cache=None)
    tile, ppt = tuple(tuned["tile"]), tuned["ppt"]
    b = R.DeviceBatch(dscenes, views, tile, ppt)
    g = b.capture_graph()
    for _ in range(max(2, warmup // 4)):
        g.replay()
    reps = max(5, steps // 10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g.replay()
    torch.cuda.synchronize()
    ms = 1000.0 * (time.perf_counter() - t0) / reps
    K, ovf = b.readback()
    pairs = sum(dscenes[si].n for (si, *_r) in views)
    pix = sum(c.width * c.height for (_, c, *_r) in views)
    del g, b
    # the same 32 renders, one recogs_render call each (fused recolour, same blend shape)
    log("bench: form batch: the same renders one call at a time")
    wss = {}
    imgs = []
    for (si, cam, mask, M, bb) in views:
        key = (si, cam.width, cam.height)
        if key not in wss:
            wss[key] = R.DeviceWorkspace(dscenes[si].n, cam.width, cam.height, tile, device=dev)
        imgs.append(torch.empty((cam.height, cam.width, 3), dtype=torch.float32, device=dev))

    def singles():
        for k, (si, cam, mask, M, bb) in enumerate(views):
            R.render(dscenes[si], cam, wss[(si, cam.width, cam.height)], tile, ppt, mask=mask, M=M, b=bb,
                     image=imgs[k], sort_mode=SORT_MODE)
    singles()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(max(3, reps // 2)):
        singles()
    torch.cuda.synchronize()
    ms_single = 1000.0 * (time.perf_counter() - t0) / max(3, reps // 2)
    nv = len(views)
    return {"renders_per_batch": nv, "scenes": [d.n for d in dscenes], "storage": "f16", "tile": f"{tile[0]}x{tile[1]}",
            "px_per_thread": ppt, "autotune_ms": {f"{r['tile'][0]}x{r['tile'][1]}p{r['ppt']}": r["ms"]
                                                   for r in tuned["table"]},
            "ms_per_batch": round(ms, 3), "frames_per_s": round(nv * 1000.0 / ms, 1),
            "gaussians_per_s": round(pairs * 1000.0 / ms, 1), "megapixels_per_s": round(pix / ms / 1e3, 1),
            "keys": K, "overflow": ovf,
            "one_call_each": {"ms_per_32_renders": round(ms_single, 3),
                              "frames_per_s": round(nv * 1000.0 / ms_single, 1)}}


DIFF_TILE, DIFF_PPT = (32, 16), 1


def form_diff(R, steps, warmup, dev, tile=DIFF_TILE, ppt=DIFF_PPT):
    """1M Gaussians (FP32, SH 3), 8 views at 1280x720: render with the fused recolour
    (keeping the backward state), L2 loss against a seeded target, backward to the
    opacities, the SH DC coefficients and M, summed over the 8 views (the loss is their
    mean)."""
    import torch

    import synth
    log("bench: form diff: 1M Gaussians, 8 views at 1280x720")
    w = synth.make_diff()
    d = R.DeviceScene(w.scene, device=dev)
    n = d.n
    sc = d.c_struct()
    v0 = w.views[0]
    mask = torch.empty(n, dtype=torch.uint8, device=dev)
    cnt = torch.empty(1, dtype=torch.int32, device=dev)
    R.recogs_select(sc, R.camera_struct(v0.camera), R.select_struct(v0.select), mask.data_ptr(), cnt.data_ptr())
    M = torch.from_numpy(v0.recolor.M.reshape(9).copy()).to(dev)
    Mt = torch.from_numpy(w.extra["M_target"].reshape(9).copy()).to(dev)
    b = torch.zeros(3, dtype=torch.float32, device=dev)
    W, H = v0.camera.width, v0.camera.height
    ws = [R.DeviceWorkspace(n, W, H, tile, device=dev) for _ in w.views]
    targets = []
    for k, v in enumerate(w.views):
        t = R.render(d, v.camera, ws[k], tile, ppt, mask=mask, M=Mt, b=b, sort_mode=SORT_MODE).clone()
        t += torch.from_numpy(synth.random_image(w.extra["noise_seed"] + k, (H, W, 3), w.extra["noise_sd"])).to(dev)
        targets.append(t)
    imgs = [torch.empty((H, W, 3), dtype=torch.float32, device=dev) for _ in w.views]
    dimg = torch.empty((H, W, 3), dtype=torch.float32, device=dev)
    loss = torch.zeros(len(w.views), dtype=torch.float32, device=dev)   # one slot per view
    dop = torch.empty(n, dtype=torch.float32, device=dev)
    ddc = torch.empty((3, n), dtype=torch.float32, device=dev)
    dM = torch.empty(9, dtype=torch.float32, device=dev)
    scale = 1.0 / (len(w.views) * H * W * 3)
    cams = [R.camera_struct(v.camera) for v in w.views]
    o = R.opts_struct(tile, ppt, (0.0, 0.0, 0.0), mask, M, b, keep_backward=True, bwd_scratch=ws[0].backward_scratch(tile, ppt) if BWD_FORM == "block" else None)

    def step(graph=True):
        # graph mode: no host synchronisation in the step (the backward reads the key
        # count on the device); the eager warm-up grows the workspaces if a view needs it
        for k, v in enumerate(w.views):
            R.render(d, v.camera, ws[k], tile, ppt, mask=mask, M=M, b=b, keep_backward=True, image=imgs[k],
                     sort_mode=SORT_MODE, graph_mode=graph)
            R.recogs_loss_l2(imgs[k].data_ptr(), targets[k].data_ptr(), H * W * 3, scale, dimg.data_ptr(),
                             loss.data_ptr() + 4 * k)
            # the loss sums the views: the first view writes the gradients, the others add to them
            R.recogs_render_backward(sc, cams[k], o, ws[k].ws, imgs[k].data_ptr(), dimg.data_ptr(), dop.data_ptr(),
                                     ddc.data_ptr(), dM.data_ptr(), 1 if k else 0)
    step(False)
    for _ in range(max(2, warmup // 4)):
        step()
    reps = max(3, steps // 20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        step()
    torch.cuda.synchronize()
    ms = 1000.0 * (time.perf_counter() - t0) / reps
    # forward alone, for the backward's share
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        for k, v in enumerate(w.views):
            R.render(d, v.camera, ws[k], tile, ppt, mask=mask, M=M, b=b, keep_backward=True, image=imgs[k],
                     sort_mode=SORT_MODE, graph_mode=True)
    torch.cuda.synchronize()
    ms_fwd = 1000.0 * (time.perf_counter() - t0) / reps
    _no_overflow(ws)
    return {"views": len(w.views), "width": W, "height": H, "gaussians": n, "tile": f"{tile[0]}x{tile[1]}", "px_per_thread": ppt,
            "ms_per_step": round(ms, 3), "views_per_s": round(len(w.views) * 1000.0 / ms, 1),
            "forward_ms_per_step": round(ms_fwd, 3), "loss": float(loss.sum().item()),
            "grad_M_norm": float(dM.norm().item()), "grad_opacity_norm": float(dop.norm().item()),
            "grad_dc_norm": float(ddc.norm().item()), "grad_over_views": len(w.views), "backward_form": BWD_FORM}


def form_refit(R, steps, warmup, dev, tile=DIFF_TILE, ppt=DIFF_PPT):
    """SH-only refitting (the background optimiser, Sec. 3.3): 1M Gaussians (FP32, SH 3),
    the 8 views at 1280x720 taken in turn, one per step: render keeping the backward
    state, the loss of eq. 4 (0.8 L1 + 0.2 (1 - SSIM)) against the view recoloured by the
    target matrix (plus seeded noise), the gradient of every SH coefficient, one Adam
    step on all of them, with the two loss terms as two calls and the gradient written
    and read back (`ms_per_step`); `ms_per_step_fused_adam` is the same step with both
    loss terms in one pass and the Adam update inside the SH-gradient pass."""
    import torch

    import synth
    log("bench: form refit: 1M Gaussians, SH-only Adam steps at 1280x720")
    w = synth.make_diff()
    d = R.DeviceScene(w.scene, device=dev)
    n, K = d.n, (w.scene.sh_degree + 1) ** 2
    v0 = w.views[0]
    mask = torch.empty(n, dtype=torch.uint8, device=dev)
    cnt = torch.empty(1, dtype=torch.int32, device=dev)
    R.recogs_select(d.c_struct(), R.camera_struct(v0.camera), R.select_struct(v0.select), mask.data_ptr(), cnt.data_ptr())
    Mt = torch.from_numpy(w.extra["M_target"].reshape(9).copy()).to(dev)
    b = torch.zeros(3, dtype=torch.float32, device=dev)
    W, H = v0.camera.width, v0.camera.height
    ws = R.DeviceWorkspace(n, W, H, tile, device=dev)
    targets = []
    for k, v in enumerate(w.views):
        t = R.render(d, v.camera, ws, tile, ppt, mask=mask, M=Mt, b=b, sort_mode=SORT_MODE).clone()
        t += torch.from_numpy(synth.random_image(w.extra["noise_seed"] + k, (H, W, 3), w.extra["noise_sd"])).to(dev)
        targets.append(t)
    sh = d.sh.clone()
    m, v = torch.zeros_like(sh), torch.zeros_like(sh)
    img = torch.empty((H, W, 3), dtype=torch.float32, device=dev)
    dimg = torch.empty_like(img)
    loss = torch.zeros(len(w.views), dtype=torch.float32, device=dev)
    dop = torch.empty(n, dtype=torch.float32, device=dev)
    dsh = torch.zeros((3 * K, d.stride), dtype=torch.float32, device=dev)
    dM = torch.empty(9, dtype=torch.float32, device=dev)
    cams = [R.camera_struct(v.camera) for v in w.views]
    o = R.opts_struct(tile, ppt, keep_backward=True, bwd_scratch=ws.backward_scratch(tile, ppt) if BWD_FORM == "block" else None)
    sc = d.c_struct(sh)
    cnt_px = H * W * 3
    lam = 0.2
    nb = R.recogs_dssim_workspace_bytes(W, H)
    sws = torch.empty(nb // 4, dtype=torch.float32, device=dev)
    lss = torch.zeros(len(w.views), dtype=torch.float32, device=dev)
    state = {"step": 0}

    def step():
        k = state["step"] % len(w.views)
        state["step"] += 1
        R.render(d, w.views[k].camera, ws, tile, ppt, keep_backward=True, image=img, sh=sh, sort_mode=SORT_MODE,
                 graph_mode=True)
        R.recogs_loss_l1(img.data_ptr(), targets[k].data_ptr(), cnt_px, (1.0 - lam) / cnt_px, dimg.data_ptr(),
                         loss.data_ptr() + 4 * k)
        R.recogs_loss_dssim(img.data_ptr(), targets[k].data_ptr(), W, H, lam, dimg.data_ptr(), 1, lss.data_ptr() + 4 * k,
                            sws.data_ptr(), nb)
        R.recogs_render_backward_sh(sc, cams[k], o, ws.ws, img.data_ptr(), dimg.data_ptr(), dop.data_ptr(),
                                    dsh.data_ptr(), dM.data_ptr())
        R.recogs_adam_step(sh.data_ptr(), dsh.data_ptr(), m.data_ptr(), v.data_ptr(), sh.numel(), 2e-3,
                           step=state["step"])
    lfs = torch.zeros(len(w.views), dtype=torch.float32, device=dev)

    def step_fused():
        # the same step with both loss terms in one pass and the SH backward and the Adam
        # step fused (the gradient does not go through memory)
        k = state["step"] % len(w.views)
        state["step"] += 1
        R.render(d, w.views[k].camera, ws, tile, ppt, keep_backward=True, image=img, sh=sh, sort_mode=SORT_MODE,
                 graph_mode=True)
        R.recogs_loss_l1_dssim(img.data_ptr(), targets[k].data_ptr(), W, H, (1.0 - lam) / cnt_px, lam, dimg.data_ptr(),
                               0, lfs.data_ptr() + 4 * k, sws.data_ptr(), nb)
        R.recogs_render_backward_sh_adam(sc, cams[k], o, ws.ws, img.data_ptr(), dimg.data_ptr(), dop.data_ptr(),
                                         dM.data_ptr(), m.data_ptr(), v.data_ptr(), 2e-3, step=state["step"])
    for _ in range(max(8, warmup)):
        step()
    torch.cuda.synchronize()
    first = float((loss + lss).mean().item())
    reps = max(16, steps // 4)
    t0 = time.perf_counter()
    for _ in range(reps):
        step()
    torch.cuda.synchronize()
    ms = 1000.0 * (time.perf_counter() - t0) / reps
    end = float((loss + lss).mean().item())
    t0 = time.perf_counter()
    for _ in range(reps):
        step_fused()
    torch.cuda.synchronize()
    ms_fused = 1000.0 * (time.perf_counter() - t0) / reps
    _no_overflow([ws])
    return {"views": len(w.views), "width": W, "height": H, "gaussians": n, "sh_coefficients": int(3 * K * n),
            "tile": f"{tile[0]}x{tile[1]}", "px_per_thread": ppt, "backward_form": BWD_FORM, "ms_per_step": round(ms, 3),
            "steps_per_s": round(1000.0 / ms, 1), "steps_timed": reps, "ms_per_step_fused_adam": round(ms_fused, 3),
            "loss": "0.8 L1 + 0.2 (1 - SSIM)", "loss_mean_after_warmup": first, "loss_mean_end": end,
            "loss_mean_after_fused_steps": float(lfs.mean().item())}


def _no_overflow(wss):
    """After graph-mode renders: each workspace's last render held all its keys (a render
    that overflowed draws the background and gives zero gradients)."""
    for ws in wss:
        k, _ = ws.readback()
        if k > ws.ws.key_capacity:
            raise RuntimeError(f"a timed render needed {k} keys, its workspace holds {ws.ws.key_capacity}")


def _event_ms(fn, reps):
    """Mean device time of fn() over reps calls, bracketed by events on the current stream."""
    import torch
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def form_selection(R, steps, warmup, dev, tile=(32, 32), ppt=1):
    """The pixel-selection chain of Sec. 3.2 on the 1M-Gaussian 1920x1080 frame: the
    render with and without the fused rough depth map (tau 0.5), the unprojection of a
    brush selection (disk of radius 378 px, 70% sample), the statistical outlier removal
    (16 neighbours, scale 0.007), and, in a second view 0.3 rad of azimuth away, the
    reprojection of the cloud as a mask (2 px squares, depth test with 1% slack) and the
    tint of that view's image."""
    import torch

    import synth
    log("bench: form selection: depth map, unprojection, outlier removal, reprojection, tint at 1920x1080")
    w = synth.make_precision()
    cam = w.view.camera
    W, H = cam.width, cam.height
    d = R.DeviceScene(w.scene, device=dev)
    ws = R.DeviceWorkspace(d.n, W, H, tile, device=dev)
    img = torch.empty((H, W, 3), dtype=torch.float32, device=dev)
    depth = torch.empty((H, W), dtype=torch.float32, device=dev)
    R.render(d, cam, ws, tile, ppt, image=img, sort_mode=SORT_MODE)     # grows the workspace once if needed
    reps = max(10, steps // 4)
    ms_plain = _event_ms(lambda: R.render(d, cam, ws, tile, ppt, image=img, sort_mode=SORT_MODE), reps)
    ms_depth = _event_ms(lambda: R.render(d, cam, ws, tile, ppt, image=img, depth=depth, depth_tau=0.5,
                                          sort_mode=SORT_MODE), reps)
    mask = torch.from_numpy(synth.brush_mask(W, H, 960.0, 540.0, 378.0)).to(dev)
    keep = torch.from_numpy(synth.sample_keep(41, mask.cpu().numpy())).to(dev)
    c = R.camera_struct(cam)
    cap = int(mask.numel())
    pts = torch.empty((3, cap), dtype=torch.float32, device=dev)
    cnt = torch.zeros(1, dtype=torch.int32, device=dev)
    nb = R.recogs_unproject_workspace_bytes(W, H)
    uws = torch.empty(nb, dtype=torch.uint8, device=dev)

    def unp():
        R.recogs_unproject(c, mask.data_ptr(), keep.data_ptr(), depth.data_ptr(), pts.data_ptr(), cap, cnt.data_ptr(),
                           uws.data_ptr(), nb)
    ms_unp = _event_ms(unp, reps)
    n_pts = int(cnt.item())
    cloud = pts[:, :n_pts].contiguous()
    dmean = torch.empty(n_pts, dtype=torch.float32, device=dev)
    kp = torch.empty(n_pts, dtype=torch.uint8, device=dev)
    out = torch.empty((3, n_pts), dtype=torch.float32, device=dev)
    ocnt = torch.zeros(1, dtype=torch.int32, device=dev)
    onb = R.recogs_outlier_workspace_bytes(n_pts)
    ows = torch.empty(onb, dtype=torch.uint8, device=dev)

    def outl():
        R.recogs_remove_outliers(cloud.data_ptr(), n_pts, n_pts, 16, 0.007, dmean.data_ptr(), kp.data_ptr(),
                                 out.data_ptr(), n_pts, ocnt.data_ptr(), ows.data_ptr(), onb)
    ms_out = _event_ms(outl, reps)
    n_kept = int(ocnt.item())
    cam2 = synth.nearby_orbit(cam, 0.3)
    c2 = R.camera_struct(cam2)
    depth2 = torch.empty((H, W), dtype=torch.float32, device=dev)
    img2 = torch.empty((H, W, 3), dtype=torch.float32, device=dev)
    ws2 = R.DeviceWorkspace(d.n, W, H, tile, device=dev)
    R.render(d, cam2, ws2, tile, ppt, image=img2, depth=depth2, depth_tau=0.5, sort_mode=SORT_MODE)
    vmask = torch.empty((H, W), dtype=torch.uint8, device=dev)
    tinted = torch.empty_like(img2)
    t = [1.0, 0.6, 0.5]

    def rep():
        R.recogs_reproject_mask(c2, out.data_ptr(), n_kept, n_pts, 2.0, depth2.data_ptr(), 0.01, vmask.data_ptr())
    ms_rep = _event_ms(rep, reps)
    ms_tint = _event_ms(lambda: R.recogs_tint(img2.data_ptr(), vmask.data_ptr(), t, tinted.data_ptr(), H * W), reps)
    marked = int(vmask.sum().item())
    return {"width": W, "height": H, "gaussians": d.n, "tile": f"{tile[0]}x{tile[1]}", "px_per_thread": ppt,
            "frame_ms": round(ms_plain, 4), "frame_with_depth_ms": round(ms_depth, 4),
            "depth_overhead_ms": round(ms_depth - ms_plain, 4),
            "selected_pixels": int(mask.sum().item()), "unprojected_points": n_pts, "unproject_ms": round(ms_unp, 4),
            "outlier_kept": n_kept, "outlier_ms": round(ms_out, 4),
            "reproject_ms": round(ms_rep, 4), "reprojected_pixels": marked, "tint_ms": round(ms_tint, 4)}


def form_edit(R, steps, warmup, dev, tile=DIFF_TILE, ppt=DIFF_PPT):
    """The background optimiser of Sec. 3.3 with the selection of Sec. 3.2: 1M Gaussians
    (FP32, SH 3), 8 training views at 1280x720. Once: view 0 rendered with its rough
    depth map, a brush selection (disk of radius 0.15 H at the centre, 70% sample)
    unprojected and cleaned by the outlier removal; the training views' original images
    rendered. Per step (one view, in turn): render the current SH keeping the backward
    state and the rough depth map, draw the cloud into the view as its mask (2 px squares,
    depth test with 1% slack), tint the view's original image there (t = (1, 0.6, 0.5)),
    the loss of eq. 4 against it (both terms in one pass), the gradient of every SH
    coefficient and one Adam step, fused (the gradient goes straight into the update,
    never to memory)."""
    import torch

    import synth
    log("bench: form edit: selection-driven SH refit, 1M Gaussians at 1280x720")
    w = synth.make_diff()
    d = R.DeviceScene(w.scene, device=dev)
    n, K = d.n, (w.scene.sh_degree + 1) ** 2
    v0 = w.views[0]
    W, H = v0.camera.width, v0.camera.height
    ws = R.DeviceWorkspace(n, W, H, tile, device=dev)
    depth = torch.empty((H, W), dtype=torch.float32, device=dev)
    R.render(d, v0.camera, ws, tile, ppt, depth=depth, depth_tau=0.5, sort_mode=SORT_MODE)
    sel = synth.brush_mask(W, H, W / 2, H / 2, 0.15 * H)
    keep = synth.sample_keep(w.extra["keep_seed"], sel)
    cloud, n_sel = R.unproject(v0.camera, torch.from_numpy(sel).to(dev), torch.from_numpy(keep).to(dev), depth)
    cloud, _, _ = R.remove_outliers(cloud.contiguous(), 16, 0.007)
    cloud = cloud.contiguous()
    originals = [R.render(d, v.camera, ws, tile, ppt, sort_mode=SORT_MODE).clone() for v in w.views]
    t = [float(x) for x in w.extra["tint"]]
    sh = d.sh.clone()
    m, v = torch.zeros_like(sh), torch.zeros_like(sh)
    img = torch.empty((H, W, 3), dtype=torch.float32, device=dev)
    target = torch.empty_like(img)
    vmask = torch.empty((H, W), dtype=torch.uint8, device=dev)
    dimg = torch.empty_like(img)
    loss = torch.zeros(len(w.views), dtype=torch.float32, device=dev)
    lss = torch.zeros(len(w.views), dtype=torch.float32, device=dev)
    dop = torch.empty(n, dtype=torch.float32, device=dev)
    dM = torch.empty(9, dtype=torch.float32, device=dev)
    cams = [R.camera_struct(v.camera) for v in w.views]
    o = R.opts_struct(tile, ppt, keep_backward=True, bwd_scratch=ws.backward_scratch(tile, ppt) if BWD_FORM == "block" else None)
    sc = d.c_struct(sh)
    cnt_px = H * W * 3
    lam = 0.2
    nb = R.recogs_dssim_workspace_bytes(W, H)
    sws = torch.empty(nb // 4, dtype=torch.float32, device=dev)
    n_pts = cloud.shape[1]
    marked = torch.zeros(len(w.views), dtype=torch.int64, device=dev)
    state = {"step": 0}

    def step():
        k = state["step"] % len(w.views)
        state["step"] += 1
        R.render(d, w.views[k].camera, ws, tile, ppt, keep_backward=True, image=img, sh=sh, depth=depth, depth_tau=0.5,
                 sort_mode=SORT_MODE, graph_mode=True)
        R.recogs_reproject_mask(cams[k], cloud.data_ptr(), n_pts, n_pts, 2.0, depth.data_ptr(), 0.01, vmask.data_ptr())
        R.recogs_tint(originals[k].data_ptr(), vmask.data_ptr(), t, target.data_ptr(), H * W)
        # eq. 4 in one pass (L1 and SSIM terms; the L1 slots stay zero)
        R.recogs_loss_l1_dssim(img.data_ptr(), target.data_ptr(), W, H, (1.0 - lam) / cnt_px, lam, dimg.data_ptr(), 0,
                               lss.data_ptr() + 4 * k, sws.data_ptr(), nb)
        R.recogs_render_backward_sh_adam(sc, cams[k], o, ws.ws, img.data_ptr(), dimg.data_ptr(), dop.data_ptr(),
                                         dM.data_ptr(), m.data_ptr(), v.data_ptr(), 2e-3, step=state["step"])
    for _ in range(len(w.views)):
        step()
        marked[(state["step"] - 1) % len(w.views)] = vmask.sum()
    torch.cuda.synchronize()
    first = float((loss + lss).mean().item())
    for _ in range(max(0, warmup - len(w.views))):
        step()
    reps = max(16, steps // 4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        step()
    torch.cuda.synchronize()
    ms = 1000.0 * (time.perf_counter() - t0) / reps
    _no_overflow([ws])
    return {"views": len(w.views), "width": W, "height": H, "gaussians": n, "sh_coefficients": int(3 * K * n),
            "tile": f"{tile[0]}x{tile[1]}", "px_per_thread": ppt, "selected_pixels": int(sel.sum()),
            "cloud_points": int(n_pts), "unprojected_points": int(n_sel),
            "marked_pixels_per_view": [int(x) for x in marked.cpu().tolist()],
            "backward_form": BWD_FORM, "ms_per_step": round(ms, 3), "steps_per_s": round(1000.0 / ms, 1), "steps_timed": reps,
            "loss": "0.8 L1 + 0.2 (1 - SSIM) against the tinted view", "loss_mean_first_pass": first,
            "loss_mean_end": float((loss + lss).mean().item())}


def cpu_baseline(w):
    """The oracle as it stands on this host, on one whole frame of the same workload:
    recolour and projection of every Gaussian (one thread), then per-pixel compositing
    of the whole image, window by window (OpenMP over 32x32 windows)."""
    import numpy as np

    import synth
    from oracle import oracle as orc
    orc.lib()
    v = w.view
    t0 = time.perf_counter()
    mask, _ = orc.select(w.scene, v.camera, v.select)
    t1 = time.perf_counter()
    sh2 = orc.recolor(w.scene.sh_f32(), mask, v.recolor.M.astype(np.float64), v.recolor.b.astype(np.float64))
    t2 = time.perf_counter()
    sc2 = synth.Scene(w.scene.means, w.scene.log_scales, w.scene.quats, w.scene.opacity, sh2, w.scene.sh_degree)
    pr = orc.project(sc2, v.camera, (16, 16))
    t3 = time.perf_counter()
    W, H = v.camera.width, v.camera.height
    wins = [(x, y, min(32, W - x), min(32, H - y)) for y in range(0, H, 32) for x in range(0, W, 32)]
    orc.render_windows(pr, wins)
    t4 = time.perf_counter()
    t_frame = t4 - t1
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(1.0 / t_frame, 6), "unit": "frames/s", "cores": cores, "kind": "oracle",
            "sample": (f"one whole {W}x{H} frame of the same workload: recolour ({t2 - t1:.2f} s) and projection "
                       f"({t3 - t2:.2f} s, 1 thread) of all {w.scene.n} Gaussians, per-pixel compositing of "
                       f"{len(wins)} windows ({t4 - t3:.2f} s on {cores} threads); selection ({t1 - t0:.2f} s) "
                       "not counted, as on the GPU"),
            "seconds_measured": round(t4 - t0, 2)}


def main():
    global SORT_MODE, BWD_FORM
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--tile", type=int, nargs=2, default=[32, 32])
    ap.add_argument("--ppt", type=int, default=1)
    ap.add_argument("--sort-mode", type=int, choices=[0, 2], default=SORT_MODE,
                    help="key order of every render: 0 depth-first, 2 tile-first (both graph-capturable)")
    ap.add_argument("--diff-tile", type=int, nargs=2, default=None,
                    help="tile shape of the differentiation form when run alone (--only-form diff)")
    ap.add_argument("--diff-ppt", type=int, default=DIFF_PPT)
    ap.add_argument("--bwd-form", choices=["block", "tile"], default=BWD_FORM,
                    help="backward of the differentiation, refit and edit forms: one workgroup per tile, or one "
                         "wave per 8x8 block (with its scratch)")
    ap.add_argument("--layout", choices=["hwc", "chw"], default="hwc", help="output layout of the timed frame")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the comparison frames (16x16 tiles, the other output layout)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the FP16/BF16, batched, differentiation, refit, "
                    "selection and edit forms")
    ap.add_argument("--forms", default="", help="comma-separated subset of the forms to run (f16, bf16, f32, batch, "
                    "diff, refit, selection, edit); default all")
    ap.add_argument("--only-form", choices=["f16", "bf16", "batch", "diff", "refit"], default=None,
                    help="run only this form and print its JSON (for profiling it)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for rocprof traffic counters)")
    args = ap.parse_args()
    SORT_MODE = args.sort_mode
    BWD_FORM = args.bwd_form
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this path has no multi-GPU form (sharding across GPUs is designed, not built)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2511_18441_amd as R
    import synth

    dev = "cuda:0"
    torch.cuda.set_device(0)
    tile = tuple(args.tile)
    tw, th = tile
    if args.only_form:
        if args.only_form == "batch":
            res = form_batch(R, args.steps, args.warmup, dev)
        elif args.only_form == "refit":
            res = form_refit(R, args.steps, args.warmup, dev)
        elif args.only_form == "diff":
            res = form_diff(R, args.steps, args.warmup, dev,
                            DIFF_TILE if args.diff_tile is None else tuple(args.diff_tile), args.diff_ppt)
        else:
            res = form_single(R, args.only_form, tile, args.ppt, args.steps, args.warmup, dev)
        print(json.dumps({"form": args.only_form, **res}), flush=True)
        return
    log(f"bench: generating 1M-Gaussian scene ({args.storage})")
    w = synth.make_precision(storage=args.storage)
    s = Single(R, w, dev, tile, args.ppt, chw=args.layout == "chw")
    log(f"bench: warmup {args.warmup}, timing {args.steps} frames")
    m = s.measure(args.steps, args.warmup)
    ms = m["ms"]
    fps = 1000.0 / ms
    st = s.counts()
    sb = {"f32": 4, "f16": 2, "bf16": 2}[args.storage]
    bytes_, flops = algorithmic_model(st, sb, w.scene.sh_degree, sort_mode=SORT_MODE)
    per_kernel, launches = stage_table(m["stages"], bytes_, flops, st)
    dom = max(per_kernel, key=lambda k: per_kernel[k]["ms_per_frame"])
    nl = launches.get(dom, 1)
    avg = m["stages"][dom] / nl
    if dom == "blend":
        avg = m["blend_ms_timed"]  # measured over the timed frames themselves
        region = tw % 8 == 0 and th % (8 * args.ppt) == 0
        kname = f"k_blend_region<{tw},{th},{args.ppt}>" if region else f"k_blend<{tw},{th},{args.ppt}>"
        ach = flops["blend"] / (avg * 1e-3) / 1e12
        traffic = recorded_traffic(kname, tile, args.ppt) if args.storage == "f32" else None
        roof = {"bound": "alu", "achieved": round(ach, 3), "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(ach / FP32_VECTOR_PEAK_TFLOPS, 4), "traffic": traffic, "kernel": kname,
                "avg_launch_ms": round(avg, 4), "launches_timed": m["profiled_frames"],
                "work_per_launch": f"{st['evals']} pixel-splat evaluations (16x16-tile lists) x "
                                   f"{BLEND_FLOPS_PER_EVAL} flops",
                "achieved_is": "nominal: the 16x16-tile-list work of the reference rasteriser over the measured time",
                "alg_bytes_per_launch": int(bytes_["blend"]),
                "hbm_GBps_alg": round(bytes_["blend"] / (avg * 1e-3) / 1e9, 1)}
        sq = recorded_sq(kname, tile, args.ppt) if args.storage == "f32" else None
        if sq and "executed_evals_max" in sq:
            # the evaluations the region waves actually execute (64 pixels per wave step,
            # wave steps bounded by the LDS instruction count), from the committed counters
            ex = sq["executed_evals_max"]
            roof["executed_evals_max"] = ex
            roof["achieved_executed_max"] = round(ex * BLEND_FLOPS_PER_EVAL / (avg * 1e-3) / 1e12, 3)
            roof["valu_insts_per_launch"] = sq.get("sq_insts_valu")
            if "lds_load_bytes" in sq:
                # the second limit of the blend: bytes the LDS returns to the lanes (every
                # wave step broadcasts its 36-byte record to 64 lanes), against 128 bytes per
                # CU per clock at the 2.4 GHz peak clock
                lds = sq["lds_load_bytes"] / (avg * 1e-3)
                roof["lds_load_bytes_per_launch"] = sq["lds_load_bytes"]
                roof["lds_TBps"] = round(lds / 1e12, 2)
                roof["lds_frac"] = round(lds / LDS_PEAK_BPS, 4)
        else:
            roof["executed_evals_max"] = None
    else:
        ach = bytes_[dom] / nl / (avg * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom,
                "avg_launch_ms": round(avg, 4), "launches_timed": m["profiled_frames"],
                "work_per_launch": f"{int(bytes_[dom] / nl)} algorithmic bytes"}
    tot_bytes = sum(bytes_.values())
    res = {
        "metric": METRIC, "value": round(fps, 2), "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"1M Gaussians SH deg 3, 1920x1080, {tw}x{th} tiles, {args.storage} storage; "
                               "recolor(selected) + render", "gaussians": s.n, "width": s.cam.width,
                   "height": s.cam.height, "sh_degree": 3, "storage": args.storage, "tile": f"{tw}x{th}",
                   "px_per_thread": args.ppt, "layout": args.layout, "sort_mode": SORT_MODE},
        "gaussians_per_s": round(fps * s.n, 1),
        "frame_hbm_roofline": {"alg_bytes_per_frame": int(tot_bytes),
                               "GBps": round(tot_bytes * fps / 1e9, 1),
                               "frac": round(tot_bytes * fps / 1e9 / HBM_PEAK_GBS, 4)},
        "render_mode": "graph_mode (no host synchronisation in the frame)",
        "ms_per_step_without_blend_events": round(m["ms_no_events"], 4),
        "ms_per_step_eager": round(m["ms_eager"], 4),
        "stage_breakdown": "separate pass with events between all stages (waits per frame)",
        "select_ms": round(m["select_ms"], 4),
        "select_recolor_render_fps": round(1000.0 / (ms + m["select_ms"]), 2),
        "roofline": roof,
        "stages": per_kernel,
        "counts": st,
    }
    del s
    if tuple(tile) != (16, 16) and not args.no_compare:
        # the same frame at the 16x16 tiles of the 3DGS rasteriser (same images, bit for bit)
        log("bench: the same frame at 16x16 tiles, 1 px/thread")
        s16 = Single(R, w, dev, (16, 16), 1)
        m16 = s16.measure(args.steps, args.warmup)
        res["at_16x16_tiles"] = {"px_per_thread": 1, "frames_per_s": round(1000.0 / m16["ms"], 2),
                                 "ms_per_step": round(m16["ms"], 4), "blend_ms": round(m16["blend_ms_timed"], 4),
                                 "stages_ms": {k: round(v, 4) for k, v in m16["stages"].items()}}
        del s16
    if not args.no_compare:
        # the paper's layout experiment (Sec. 4.2): the same frame in the other output layout
        other = "hwc" if args.layout == "chw" else "chw"
        log(f"bench: the same frame with {other.upper()} output")
        sc = Single(R, w, dev, tile, args.ppt, chw=other == "chw")
        mc = sc.measure(args.steps, args.warmup)
        res["output_layout"] = {args.layout: {"frames_per_s": round(fps, 2), "blend_ms": round(m["blend_ms_timed"], 4)},
                                other: {"frames_per_s": round(1000.0 / mc["ms"], 2),
                                        "blend_ms": round(mc["blend_ms_timed"], 4)}}
        del sc
    if args.copy_calibration:
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        res["copy_calibration_bytes"] = 1 << 30
        del src, dst
    if not args.no_forms:
        forms = {}
        only = set(args.forms.split(",")) if args.forms else None

        def want(name):
            return only is None or name in only
        for stg in ("f32", "f16", "bf16"):
            if stg != args.storage and want(stg):
                forms[stg] = form_single(R, stg, tile, args.ppt, args.steps, args.warmup, dev)
        if want("batch"):
            forms["batch"] = form_batch(R, args.steps, args.warmup, dev)
        if want("diff"):
            forms["diff"] = form_diff(R, args.steps, args.warmup, dev)
        if want("refit"):
            forms["refit"] = form_refit(R, args.steps, args.warmup, dev)
        if want("selection"):
            forms["selection"] = form_selection(R, args.steps, args.warmup, dev)
        if want("edit"):
            forms["edit"] = form_edit(R, args.steps, args.warmup, dev)
        res["forms"] = forms
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("bench: oracle CPU baseline")
        res["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
