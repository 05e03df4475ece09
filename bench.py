"""Benchmark: recolour + render frames/s of a 1,000,000-Gaussian, SH-degree-3 scene at
1920x1080 (16x16 tiles) on one MI355X, with the roofline of the dominant kernel and
the FP64 CPU oracle timed beside it.

A step (frame) = recogs_recolor of the selected Gaussians (out of place, from the
pristine SH into the render copy, so frames do not compound the edit) followed by
recogs_render of the edited scene. Inputs are resident in HBM before timing starts.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--storage f32|f16|bf16]
                  [--no-cpu-baseline] [--copy-calibration]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "recolor+render frames/s (1M Gaussians, 1080p) and HBM-roofline fraction"
HBM_PEAK_GBS = 8000.0            # MI355X HBM3E
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X fp32 vector (256 CU x 2.4 GHz)
BLEND_FLOPS_PER_EVAL = 23        # dx, dy, exponent (2 mul + 3 fma), test, exp2, clamp, T, weight, 3 fma


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_model(st, storage_bytes, deg, keep_bwd=False):
    """Bytes (and blend flops) each stage must move for this frame's counts
    (default sort: depth sort of the V Gaussians with keys, then 32-bit tile keys)."""
    N, V, K, S, P, Pd, T, Pix, E, Keff = (st[k] for k in ("N", "V", "K", "S", "passes", "dpasses", "tiles", "pix",
                                                           "evals", "keff"))
    nc = 3 * (deg + 1) ** 2
    b = {
        "recolor": N * 1 + S * nc * storage_bytes * 2,
        "preprocess": N * (12 + 24 + storage_bytes) + V * nc * storage_bytes + V * 48 + N * 16 + (V * 16 if keep_bwd else 0),
        "scan": N * 8 + V * 12,
        "depth_sort": V * 4 + Pd * V * 16,
        "emit": V * 16 + K * 8,
        "key_sort": K * 4 + P * K * 16,
        "ranges": K * 4 + T * 8,
        "blend": Keff * 52 + T * 8 + Pix * 20,
    }
    return b, {"blend": E * BLEND_FLOPS_PER_EVAL}


def cpu_baseline(w, sample_windows=24):
    """The oracle as it stands on this host: recolour + projection of every Gaussian,
    per-pixel compositing of a sample of 32x32 windows, extrapolated to a frame."""
    import numpy as np
    from oracle import oracle as orc
    orc.lib()
    v = w.view
    t0 = time.perf_counter()
    mask, _ = orc.select(w.scene, v.camera, v.select)
    t1 = time.perf_counter()
    sh2 = orc.recolor(w.scene.sh_f32(), mask, v.recolor.M.astype(np.float64), v.recolor.b.astype(np.float64))
    t2 = time.perf_counter()
    import synth
    sc2 = synth.Scene(w.scene.means, w.scene.log_scales, w.scene.quats, w.scene.opacity, sh2, w.scene.sh_degree)
    pr = orc.project(sc2, v.camera, (16, 16))
    t3 = time.perf_counter()
    rng = np.random.default_rng(7)
    W, H = v.camera.width, v.camera.height
    wins = [(int(rng.integers(0, W - 32)), int(rng.integers(0, H - 32)), 32, 32) for _ in range(sample_windows)]
    orc.render_windows(pr, wins)
    t4 = time.perf_counter()
    frac = sample_windows * 32 * 32 / (W * H)
    t_frame = (t2 - t1) + (t3 - t2) + (t4 - t3) / frac
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": 1.0 / t_frame, "unit": "frames/s", "cores": cores, "kind": "oracle",
            "sample": (f"recolour ({t2 - t1:.2f} s) and projection ({t3 - t2:.2f} s, 1 thread) of all "
                       f"{w.scene.n} Gaussians, then per-pixel compositing of {sample_windows} random 32x32 windows "
                       f"({t4 - t3:.2f} s on {cores} threads, {100 * frac:.2f}% of the frame) scaled to the whole frame"),
            "seconds_measured": round(t4 - t0, 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--tile", type=int, nargs=2, default=[16, 16])
    ap.add_argument("--ppt", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for rocprof traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this path has no multi-GPU form (see DESIGN.md, sharding)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2511_18441_amd as R
    import synth

    dev = "cuda:0"
    torch.cuda.set_device(0)
    log(f"bench: generating 1M-Gaussian scene ({args.storage})")
    w = synth.make_precision(storage=args.storage)
    v = w.view
    cam = v.camera
    n = w.scene.n
    sb = {"f32": 4, "f16": 2, "bf16": 2}[args.storage]
    d = R.DeviceScene(w.scene, device=dev)
    scs = d.c_struct()
    camc = R.camera_struct(cam)
    mask = torch.empty(n, dtype=torch.uint8, device=dev)
    count = torch.empty(1, dtype=torch.int32, device=dev)
    R.recogs_select(scs, camc, R.select_struct(v.select), mask.data_ptr(), count.data_ptr())
    M = torch.from_numpy(v.recolor.M.reshape(9)).to(dev)
    bvec = torch.from_numpy(v.recolor.b).to(dev)
    render_sh = d.sh.clone()
    ws = R.DeviceWorkspace(n, cam.width, cam.height, tuple(args.tile), key_capacity=16 * n, device=dev)
    image = torch.empty((cam.height, cam.width, 3), dtype=torch.float32, device=dev)
    tile = tuple(args.tile)

    def step(profile=False):
        R.recogs_recolor(scs, render_sh.data_ptr(), mask.data_ptr(), M.data_ptr(), bvec.data_ptr(), 0)
        R.render(d, cam, ws, tile, args.ppt, image=image, sh=render_sh, profile=profile)

    log("bench: warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"bench: timing {args.steps} frames")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = 1000.0 * (t1 - t0) / args.steps
    ms_ev = ev0.elapsed_time(ev1) / args.steps
    fps = 1000.0 / ms

    # per-stage durations (HIP events recorded by the library on the render stream)
    log("bench: stage profile")
    nprof = max(5, min(20, args.steps))
    stage = np.zeros(8)
    rec_ms = 0.0
    for _ in range(nprof):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        R.recogs_recolor(scs, render_sh.data_ptr(), mask.data_ptr(), M.data_ptr(), bvec.data_ptr(), 0)
        e1.record()
        R.render(d, cam, ws, tile, args.ppt, image=image, sh=render_sh, profile=True)
        torch.cuda.synchronize()
        rec_ms += e0.elapsed_time(e1)
        stage += np.array(ws.ws.stage_ms[:])
    stage /= nprof
    rec_ms /= nprof
    stages = dict(zip(R.binding.STAGES, stage.tolist()))
    stages["recolor"] = rec_ms

    # counts of this frame
    K = int(ws.ws.num_keys)
    cnt = ws.counts(n)
    V = int((cnt != 0).sum().item())
    S = int(count.item())
    P = int(ws.ws.sort_passes)
    Pd = int(ws.ws.depth_passes)
    T = ws.ws.tiles_x * ws.ws.tiles_y
    nproc = ws.nproc().to(torch.int64)
    E = int(nproc.sum().item())
    th, tw = tile[1], tile[0]
    Hp, Wp = ws.ws.tiles_y * th, ws.ws.tiles_x * tw
    npad = torch.zeros((Hp, Wp), dtype=torch.int64, device=dev)
    npad[:cam.height, :cam.width] = nproc
    keff = int(npad.view(ws.ws.tiles_y, th, ws.ws.tiles_x, tw).amax(dim=(1, 3)).sum().item())
    st = dict(N=n, V=V, K=K, S=S, passes=P, dpasses=Pd, tiles=T, pix=cam.width * cam.height, evals=E, keff=keff)
    bytes_, flops = algorithmic_model(st, sb, w.scene.sh_degree)
    launches = {"key_sort": P + 1, "depth_sort": Pd + 1}
    per_kernel = {}
    for k, t in stages.items():
        if k == "readback":
            continue
        nl = launches.get(k, 1)
        ent = {"ms_per_frame": round(t, 4), "launches": nl, "avg_launch_ms": round(t / nl, 4)}
        if k in bytes_ and t > 0:
            ent["alg_bytes"] = int(bytes_[k])
            ent["GBps"] = round(bytes_[k] / (t * 1e-3) / 1e9, 1)
        if k in flops and t > 0:
            ent["TFLOPs"] = round(flops[k] / (t * 1e-3) / 1e12, 2)
        per_kernel[k] = ent
    dom = max((k for k in per_kernel), key=lambda k: per_kernel[k]["ms_per_frame"])
    nl = launches.get(dom, 1)
    avg = stages[dom] / nl
    if dom == "blend":
        ach = flops["blend"] / (avg * 1e-3) / 1e12
        roof = {"kernel": "k_blend<16,16,1>", "bound": "alu", "achieved": round(ach, 3),
                "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(ach / FP32_VECTOR_PEAK_TFLOPS, 4),
                "traffic": None, "avg_launch_ms": round(avg, 4),
                "work_per_launch": f"{E} pixel-splat evaluations x {BLEND_FLOPS_PER_EVAL} flops"}
    else:
        ach = bytes_[dom] / nl / (avg * 1e-3) / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None, "avg_launch_ms": round(avg, 4),
                "work_per_launch": f"{int(bytes_[dom] / nl)} algorithmic bytes"}
    tot_bytes = sum(bytes_.values())
    res = {
        "metric": METRIC, "value": round(fps, 2), "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"1M Gaussians SH deg 3, 1920x1080, 16x16 tiles, {args.storage} storage; "
                               "recolor(selected) + render", "gaussians": n, "width": cam.width,
                   "height": cam.height, "sh_degree": 3, "storage": args.storage, "tile": f"{tw}x{th}",
                   "px_per_thread": args.ppt},
        "gaussians_per_s": round(fps * n, 1),
        "frame_hbm_roofline": {"alg_bytes_per_frame": int(tot_bytes),
                               "GBps": round(tot_bytes * fps / 1e9, 1),
                               "frac": round(tot_bytes * fps / 1e9 / HBM_PEAK_GBS, 4)},
        "ms_per_step_gpu_events": round(ms_ev, 4),
        "roofline": roof,
        "stages": per_kernel,
        "counts": st,
    }
    if args.copy_calibration:
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        res["copy_calibration_bytes"] = 1 << 30
    if not args.no_cpu_baseline:
        log("bench: oracle CPU baseline")
        res["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
