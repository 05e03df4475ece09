"""Shared helpers of the GPU tests: run the HIP path on a seeded workload and pull
its outputs back; run the oracle on the same seeded inputs."""
import numpy as np

import synth


def gpu_run(w, view=0, tile=(16, 16), ppt=1, fused=None, keep_backward=False, key_capacity=None, ws=None,
            dscene=None, bg=(0.0, 0.0, 0.0), sort_mode=0, extent_rule=0):
    """Render view `view` of workload `w` through recogs_render. `fused` = (mask uint8 np, M, b)."""
    import torch
    import paper_2511_18441_amd as R
    v = w.views[view]
    sc = w.scenes[v.scene]
    cam = v.camera
    if dscene is None:
        dscene = R.DeviceScene(sc)
    if ws is None:
        ws = R.DeviceWorkspace(sc.n, cam.width, cam.height, tile, key_capacity)
    mask = M = b = None
    if fused is not None:
        mask = torch.from_numpy(np.asarray(fused[0], np.uint8)).cuda()
        M = torch.from_numpy(np.asarray(fused[1], np.float32).reshape(9)).cuda()
        b = torch.from_numpy(np.asarray(fused[2], np.float32).reshape(3)).cuda()
    img = R.render(dscene, cam, ws, tile, ppt, bg, mask, M, b, keep_backward, sort_mode=sort_mode,
                   extent_rule=extent_rule)
    torch.cuda.synchronize()
    return dict(img=img, ws=ws, dscene=dscene, mask=mask, M=M, b=b, cam=cam, tile=tile, ppt=ppt)


def pull(out, n):
    """Integer outputs of the last render as numpy arrays."""
    ws = out["ws"]
    keys = ws.keys_sorted().cpu().numpy()
    zbits = ws.zbits(n).cpu().numpy().view(np.uint32).astype(np.int64)
    vals = ws.vals_sorted().cpu().numpy().view(np.uint32).astype(np.int64)
    if keys.dtype == np.int64:  # (tile << 32) | depth bits
        keys = keys.view(np.uint64)
        tile = (keys >> np.uint64(32)).astype(np.int64)
        kz = (keys & np.uint64(0xFFFFFFFF)).astype(np.int64)
    else:  # tile ids; the depth comes from the value's Gaussian
        tile = keys.view(np.uint32).astype(np.int64)
        kz = zbits[vals]
    return dict(
        tile=tile, kz=kz,
        img=out["img"].cpu().numpy().astype(np.float64),
        T=ws.final_T().cpu().numpy().astype(np.float64),
        nproc=ws.nproc().cpu().numpy().astype(np.int64),
        counts=ws.counts(n).cpu().numpy().view(np.uint32).astype(np.int64),
        offsets=ws.offsets(n).cpu().numpy().view(np.uint32).astype(np.int64),
        zbits=zbits,
        rects=ws.rects(n).cpu().numpy().view(np.uint32).astype(np.int64),
        vals=vals,
        ranges=ws.ranges().cpu().numpy().view(np.uint32).astype(np.int64),
        K=int(ws.ws.num_keys),
    )


def crop_windows(w, crops, size=32):
    return [(int(x), int(y), size, size) for x, y in crops]


def assert_pixels(gpu_rgb, orc_rgb, slack, tol, what="", max_band_frac=1e-3):
    """|gpu - oracle| <= tol + slack element-wise, and at most max(8, max_band_frac of
    the pixels) whose slack exceeds half the tolerance (so a wrong slack cannot quietly
    loosen the check); return (max err outside band, n in band)."""
    err = np.abs(gpu_rgb - orc_rgb).max(axis=-1)
    bad = err > tol + slack
    assert not bad.any(), (f"{what}: {int(bad.sum())} pixels off by more than {tol} + slack; worst "
                           f"{err[bad].max():.3e} at {np.argwhere(bad)[:5].tolist()}")
    band = slack > 0.5 * tol
    nband = int(band.sum())
    assert nband <= max(8, int(max_band_frac * err.size)), f"{what}: {nband} of {err.size} pixels in band"
    return float(err[~band].max()) if (~band).any() else 0.0, nband
