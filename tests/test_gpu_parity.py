"""Parity of the HIP path (through the C ABI) with the FP64 oracle, per hot-path step.

Integer outputs (selection masks, depth keys, tile rectangles and counts, sorted
order, tile ranges) must match exactly except for decisions the oracle flags as
lying within float32 rounding of their threshold; pixels must match within 2e-3
(float32 path) plus the oracle's per-pixel bound for in-band threshold decisions.
"""
import numpy as np
import pytest

import synth
from tests.gpu_common import assert_pixels, crop_windows, gpu_run, pull

pytestmark = pytest.mark.gpu

TOL_F32 = 2e-3
TOL_F16 = 1e-2


@pytest.fixture(scope="module")
def R():
    import paper_2511_18441_amd as R
    return R


def _oracle(w, orc, tile=(16, 16), fused=None, view=0, cov=None):
    v = w.views[view]
    sc = w.scenes[v.scene]
    if fused is None:
        return orc.project(sc, v.camera, tile, cov=cov)
    return orc.project(sc, v.camera, tile, cov=cov, mask=fused[0], M=fused[1], b=fused[2])


# ---------------------------------------------------------------------------
# covariance (eq. 1), selection, recolour (eq. 6)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("cfg", ["tiny", "mid"])
def test_covariance(R, orc, cfg):
    w = synth.make_tiny() if cfg == "tiny" else synth.make_mid(n=50_000)
    d = R.DeviceScene(w.scene)
    got = d.cov3d[:, : w.scene.n].cpu().numpy().astype(np.float64)
    ref = orc.covariance(w.scene.log_scales, w.scene.quats)
    scale = ref[0] + ref[3] + ref[5]
    assert np.all(np.abs(got - ref) <= 4e-6 * scale + 1e-30)


@pytest.mark.parametrize("cfg,storage", [("tiny", "f32"), ("mid", "f32"), ("mid", "f16"), ("mid", "bf16")])
def test_select(R, orc, cfg, storage):
    import torch
    w = synth.make_tiny() if cfg == "tiny" else synth.make_mid()
    sc = w.scene if storage == "f32" else w.scene.with_storage(storage)
    d = R.DeviceScene(sc)
    mask = torch.empty(sc.n, dtype=torch.uint8, device="cuda")
    count = torch.empty(1, dtype=torch.int32, device="cuda")
    R.recogs_select(d.c_struct(), R.camera_struct(w.view.camera), R.select_struct(w.view.select),
                    mask.data_ptr(), count.data_ptr())
    got = mask.cpu().numpy()
    ref, flag = orc.select(sc, w.view.camera, w.view.select)
    diff = (got != ref)
    assert not (diff & (flag == 0)).any(), np.nonzero(diff & (flag == 0))[0][:10]
    assert int(count.item()) == int(got.sum())
    assert ref.sum() > 0


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("which", ["affine", "hue"])
def test_recolor(R, orc, storage, which):
    import torch
    # the hue case: a ragged count (not a multiple of the 4 mask bytes a thread reads)
    # and a mask that does not start on a 4-byte boundary (read byte by byte)
    w = synth.make_mid(n=60_000 if which == "affine" else 60_003)
    sc = w.scene if storage == "f32" else w.scene.with_storage(storage)
    rng = np.random.default_rng(3)
    maskn = (rng.random(sc.n) < 0.3).astype(np.uint8)
    rec = w.view.recolor if which == "affine" else synth.RecolorParams(synth.hue_rotation(120.0), np.zeros(3, np.float32))
    d = R.DeviceScene(sc)
    if which == "affine":
        mask = torch.from_numpy(maskn).cuda()
    else:
        mbuf = torch.zeros(sc.n + 4, dtype=torch.uint8, device="cuda")
        mbuf[1:sc.n + 1] = torch.from_numpy(maskn).cuda()
        mask = mbuf[1:sc.n + 1]
        assert mask.data_ptr() % 4 == 1
    M = torch.from_numpy(rec.M.reshape(9)).cuda()
    b = torch.from_numpy(rec.b).cuda()
    dst = d.sh.clone()
    R.recogs_recolor(d.c_struct(), dst.data_ptr(), mask.data_ptr(), M.data_ptr(), b.data_ptr(), 0)
    got = dst.float().cpu().numpy().astype(np.float64)
    ref = orc.recolor(sc.sh_f32(), maskn, rec.M.astype(np.float64), rec.b.astype(np.float64))
    if storage == "f32":
        tol = 4e-6 * (1 + np.abs(ref))
    else:
        ulp = {"f16": 2.0 ** -10, "bf16": 2.0 ** -7}[storage]
        tol = ulp * np.maximum(np.abs(ref), 2.0 ** -14) + 4e-6 * (1 + np.abs(ref))
    assert np.all(np.abs(got - ref) <= tol)
    # unselected untouched
    keep = maskn == 0
    assert np.array_equal(got[:, keep], sc.sh_f32()[:, keep].astype(np.float64))
    if which == "hue":  # exact channel permutation (r, g, b) -> (b, r, g) on every band
        sel = maskn == 1
        src = sc.sh_f32().astype(np.float64)
        for k in range(16):
            assert np.array_equal(got[3 * k + 0, sel], src[3 * k + 2, sel])
            assert np.array_equal(got[3 * k + 1, sel], src[3 * k + 0, sel])
    # into a zeroed buffer with the unselected copied over, and in place: the same bits
    dst2 = torch.zeros_like(d.sh)
    R.recogs_recolor(d.c_struct(), dst2.data_ptr(), mask.data_ptr(), M.data_ptr(), b.data_ptr(), 1)
    assert torch.equal(dst2, dst)
    R.recogs_recolor(d.c_struct(), d.sh.data_ptr(), mask.data_ptr(), M.data_ptr(), b.data_ptr(), 0)
    assert torch.equal(d.sh, dst)


# ---------------------------------------------------------------------------
# render steps: preprocess, scan, emit + sort, ranges, blend
# ---------------------------------------------------------------------------
def _check_integer_steps(w, orc, p, pr, n):
    status = pr.col("status")
    flag = pr.col("flag").astype(bool)
    # depth key: float32 rounding of the exact depth
    zmis = (p["zbits"] != pr.col("z32bits")) & (status != 1)
    assert zmis.sum() <= max(2, n // 100_000), int(zmis.sum())
    # tile rectangle and count
    cnt_ref = pr.col("count")
    ok = ~flag & ~zmis
    assert np.array_equal(p["counts"][ok], cnt_ref[ok]), np.nonzero(p["counts"][ok] != cnt_ref[ok])[0][:10]
    has = ok & (cnt_ref > 0)
    r = p["rects"]
    assert np.array_equal(r[has, 0] & 0xFFFF, pr.col("txlo")[has])
    assert np.array_equal(r[has, 0] >> 16, pr.col("txhi")[has])
    assert np.array_equal(r[has, 1] & 0xFFFF, pr.col("tylo")[has])
    assert np.array_equal(r[has, 1] >> 16, pr.col("tyhi")[has])
    # scan: exclusive prefix sum of the counts, total K
    c = p["counts"]
    assert np.array_equal(p["offsets"], np.concatenate([[0], np.cumsum(c)[:-1]]))
    assert p["K"] == int(c.sum())
    # sorted keys: non-decreasing (tile, depth); equal keys in index order (stable)
    tile, zb, vals = p["tile"], p["kz"], p["vals"]
    order_ok = (tile[1:] > tile[:-1]) | ((tile[1:] == tile[:-1]) & ((zb[1:] > zb[:-1]) | ((zb[1:] == zb[:-1]) & (vals[1:] > vals[:-1]))))
    assert order_ok.all()
    assert np.array_equal(zb, p["zbits"][vals])
    # against the oracle's sorted (tile, depth, index) list without flagged Gaussians
    ts, zs, ids = orc.sorted_keys(pr)
    bad = flag | zmis
    keep_o = ~bad[ids]
    keep_g = ~bad[vals]
    assert np.array_equal(tile[keep_g], ts[keep_o])
    assert np.array_equal(zb[keep_g], zs[keep_o])
    assert np.array_equal(vals[keep_g], ids[keep_o])
    # tile ranges: consistent with the GPU's own sorted keys ...
    ntile = p["ranges"].shape[0]
    lo = np.searchsorted(tile, np.arange(ntile), side="left")
    hi = np.searchsorted(tile, np.arange(ntile), side="right")
    prop = np.where((hi > lo)[:, None], np.stack([lo, hi], 1), 0)
    assert np.array_equal(p["ranges"], prop)
    # ... and, per tile not touched by a flagged Gaussian, as long as the oracle's
    ref = orc.tile_ranges(ts, ntile)
    touched = np.zeros(ntile, bool)
    touched[ts[bad[ids]]] = True
    touched[tile[bad[vals]]] = True
    len_g = p["ranges"][:, 1] - p["ranges"][:, 0]
    len_o = ref[:, 1] - ref[:, 0]
    assert np.array_equal(len_g[~touched], len_o[~touched])
    if not bad.any():
        assert np.array_equal(p["ranges"], ref)
    return zmis


@pytest.mark.parametrize("sort_mode", [0, 1, 2])
@pytest.mark.parametrize("cfg", ["tiny", "mid"])
def test_render_full_image(R, orc, cfg, sort_mode):
    w = synth.make_tiny() if cfg == "tiny" else synth.make_mid()
    n = w.scene.n
    out = gpu_run(w, sort_mode=sort_mode, keep_backward=True)
    p = pull(out, n)
    pr = _oracle(w, orc)
    zmis = _check_integer_steps(w, orc, p, pr, n)
    ref = orc.render_image(pr, brute=(cfg == "tiny"))
    err, nband = assert_pixels(p["img"], ref.rgb, ref.slack, TOL_F32, cfg)
    assert err <= TOL_F32
    assert nband <= max(5, p["img"].shape[0] * p["img"].shape[1] // 1000)
    # transmittance, and the last blended splat (the entry nproc - 1 of the pixel's tile
    # list) wherever no threshold decision lies in the rounding band
    assert np.all(np.abs(p["T"] - ref.T) <= TOL_F32 + ref.slack)
    H, W = p["nproc"].shape
    ys, xs = np.mgrid[0:H, 0:W]
    tid = (ys // 16) * ((W + 15) // 16) + xs // 16
    first = p["ranges"][tid, 0].astype(np.int64)
    np_ = p["nproc"]
    gid = np.where(np_ > 0, p["vals"][np.clip(first + np_ - 1, 0, len(p["vals"]) - 1)], -1)
    clean = ref.slack == 0
    assert np.array_equal(gid[clean], ref.last[clean])
    print(f"{cfg}: K={p['K']} max|err| outside band {err:.2e}, in-band pixels {nband}, depth mismatches {int(zmis.sum())}")


@pytest.mark.parametrize("storage,sort_mode,tile,ppt", [("f32", 0, (32, 32), 1), ("f32", 0, (16, 16), 1),
                                                       ("f32", 2, (32, 32), 1), ("f32", 2, (16, 16), 1),
                                                       ("f32", 1, (32, 32), 2), ("f16", 0, (32, 32), 1),
                                                       ("bf16", 0, (16, 16), 1)])
def test_render_1m_1080p_crops(R, orc, storage, sort_mode, tile, ppt):
    """1,000,000 Gaussians, SH degree 3, 1920x1080: integer steps on the whole frame,
    pixels on 64 seeded 32x32 crops (32x32 tiles with 1 pixel per thread is the
    benchmarked launch)."""
    w32 = synth.make_precision()
    w = w32 if storage == "f32" else synth.make_precision(storage=storage)
    n = w.scene.n
    out = gpu_run(w, tile=tile, ppt=ppt, sort_mode=sort_mode)
    p = pull(out, n)
    pr = _oracle(w, orc, tile=tile)
    _check_integer_steps(w, orc, p, pr, n)
    wins = crop_windows(w, w.extra["crops"])
    ref = orc.render_windows(pr, wins)
    got = np.concatenate([p["img"][y:y + 32, x:x + 32].reshape(-1, 3) for (x, y, _, _) in wins])
    err, nband = assert_pixels(got, ref.rgb, ref.slack, TOL_F32, f"{storage} vs oracle on stored inputs")
    if storage != "f32":
        ref32 = orc.render_windows(_oracle(w32, orc, tile=tile), wins)
        err32, _ = assert_pixels(got, ref32.rgb, ref32.slack, TOL_F16, f"{storage} vs oracle on float32 inputs")
        print(f"{storage}: error vs float32-input oracle {err32:.2e}")
    print(f"{storage}: K={p['K']} crops max|err| {err:.2e} in-band {nband}")


def test_fused_recolor_render(R, orc):
    """Selection + fused affine recolour on the mid scene (the displayed colour of the
    selected Gaussians is M (f + 1/2) + b)."""
    w = synth.make_mid()
    mask, _ = orc.select(w.scene, w.view.camera, w.view.select)
    fused = (mask, w.view.recolor.M, w.view.recolor.b)
    out = gpu_run(w, fused=fused)
    p = pull(out, w.scene.n)
    pr = _oracle(w, orc, fused=(mask, w.view.recolor.M.astype(np.float64), w.view.recolor.b.astype(np.float64)))
    ref = orc.render_image(pr)
    assert_pixels(p["img"], ref.rgb, ref.slack, TOL_F32, "fused recolour")


@pytest.mark.parametrize("spread", [0, 100, 3000])
def test_depth_sort_with_few_depth_bits(R, orc, spread):
    """All Gaussians at one depth (no depth bit left for the sort after the count scan's
    pass on the low 8 bits: the emission then makes its own reduce), depths within 100
    float32 steps (the scan's pass covers them) or 3,000 (one more pass): the eager
    render gives the oracle's (tile, depth, index) order and image, the graph-mode render
    (all 32 bits) the eager render's bits."""
    import torch
    from tests.scenes_by_hand import axis_camera, scene_from
    rng = np.random.default_rng(11 + spread)
    n = 2000
    z = np.full(n, np.float32(4.0))
    if spread:
        z = (z.view(np.uint32) + rng.integers(0, spread, n).astype(np.uint32)).view(np.float32)
    means = np.column_stack([rng.uniform(-2.4, 2.4, n), rng.uniform(-2.0, 2.0, n), z.astype(np.float64)])
    sc = scene_from(means, np.log(rng.uniform(0.04, 0.15, (n, 3))), rng.uniform(0.3, 0.95, n),
                    rng.uniform(0.0, 1.0, (n, 3)))
    cam = axis_camera(96, 80, 60.0)
    base = synth.make_tiny()
    w = synth.Workload(f"depths{spread}", [sc], [synth.View(0, cam, base.view.select, base.view.recolor)])
    out = gpu_run(w, keep_backward=True)
    p = pull(out, n)
    pr = _oracle(w, orc)
    _check_integer_steps(w, orc, p, pr, n)
    ref = orc.render_image(pr, brute=True)
    assert_pixels(p["img"], ref.rgb, ref.slack, TOL_F32, f"depth spread {spread}")
    assert int(out["ws"].ws.depth_passes) == {0: 0, 100: 0, 3000: 1}[spread]
    wsg = R.DeviceWorkspace(n, cam.width, cam.height, (16, 16), key_capacity=p["K"] + 1024)
    img = R.render(out["dscene"], cam, wsg, (16, 16), 1, keep_backward=True, graph_mode=True)
    k, _ = wsg.readback()
    assert k == p["K"]
    assert torch.equal(img, out["img"])
    assert torch.equal(wsg.vals_sorted()[:k], out["ws"].vals_sorted()[:k])
    assert torch.equal(wsg.ranges(), out["ws"].ranges())


@pytest.mark.parametrize("deg", [1, 2])
def test_sh_degrees_one_and_two(R, orc, deg):
    """Scenes of SH degree 1 and 2 (eq. 2 sums bands l <= deg): the whole 800x800 image
    with the fused recolour against the oracle, then the gradient of every coefficient
    on the Gaussians that a windowed upstream gradient reaches."""
    import torch
    rng = np.random.default_rng(90 + deg)
    sc = synth.make_scene_mid_like(rng, 60_000, deg=deg)
    base = synth.make_mid(n=1000)
    cam = base.view.camera
    w = synth.Workload(f"deg{deg}", [sc], [synth.View(0, cam, base.view.select, base.view.recolor)])
    mask, _ = orc.select(sc, cam, base.view.select)
    rec = base.view.recolor
    out = gpu_run(w, tile=(32, 32), fused=(mask, rec.M, rec.b), keep_backward=True)
    p = pull(out, sc.n)
    M64, b64 = rec.M.astype(np.float64), rec.b.astype(np.float64)
    pr = orc.project(sc, cam, (32, 32), mask=mask, M=M64, b=b64)
    _check_integer_steps(w, orc, p, pr, sc.n)
    ref = orc.render_image(pr)
    err, nband = assert_pixels(p["img"], ref.rgb, ref.slack, TOL_F32, f"degree {deg}")
    assert mask.sum() > 0
    # every SH coefficient's gradient, upstream gradient on two 32x32 windows
    wins = [(384, 384, 32, 32), (160, 544, 32, 32)]
    rw = orc.render_windows(pr, wins)
    g = np.zeros((cam.height, cam.width, 3), np.float32)
    rg = np.random.default_rng(91)
    o = 0
    for (x0, y0, ww, wh) in wins:
        blk = rg.standard_normal((wh, ww, 3)).astype(np.float32)
        blk[rw.slack[o:o + ww * wh].reshape(wh, ww) > 0] = 0.0
        g[y0:y0 + wh, x0:x0 + ww] = blk
        o += ww * wh
    gr = orc.backward(pr, g.astype(np.float64), M=M64, windows=wins)
    touched = np.nonzero(np.abs(gr.drgb).sum(axis=1) > 0)[0]
    assert len(touched) > 50
    ref_sh = orc.sh_grad(sc, cam, pr, gr, M=M64, idx=touched)
    K = (deg + 1) ** 2
    d = out["dscene"]
    dsh = torch.zeros((3 * K, d.stride), device="cuda")
    t1, t9 = torch.empty(sc.n, device="cuda"), torch.empty(9, device="cuda")
    oo = R.opts_struct((32, 32), 1, (0, 0, 0), out["mask"], out["M"], out["b"], keep_backward=True)
    R.recogs_render_backward_sh(d.c_struct(), R.camera_struct(cam), oo, out["ws"].ws, out["img"].data_ptr(),
                                torch.from_numpy(g).cuda().data_ptr(), t1.data_ptr(), dsh.data_ptr(), t9.data_ptr())
    torch.cuda.synchronize()
    got = dsh[:, touched].cpu().numpy().astype(np.float64)
    scale = np.abs(ref_sh).max()
    assert scale > 0 and np.all(np.abs(got - ref_sh) <= 2e-5 * scale + 1e-4 * np.abs(ref_sh))
    assert np.abs(ref_sh[3:]).max() > 0   # the higher bands carry gradient
    print(f"degree {deg}: max|err| {err:.2e}, in-band {nband}, dSH rel err {np.abs(got - ref_sh).max() / scale:.2e}")


def test_benchmarked_frame_sequence_1m_crops(R, orc):
    """The benchmarked frame at its size: recogs_recolor of the selection out of place
    (from the pristine SH into the render copy) then recogs_render of the recoloured
    coefficients in graph mode, 32x32 tiles, 1 pixel per thread, 1M Gaussians at
    1920x1080; pixels on the 64 seeded crops against the oracle of the recoloured
    projection (eq. 6 in its colour form)."""
    import torch
    w = synth.make_precision()
    v = w.view
    sc = w.scene
    d = R.DeviceScene(sc)
    mask_t = torch.empty(sc.n, dtype=torch.uint8, device="cuda")
    count = torch.empty(1, dtype=torch.int32, device="cuda")
    R.recogs_select(d.c_struct(), R.camera_struct(v.camera), R.select_struct(v.select), mask_t.data_ptr(),
                    count.data_ptr())
    M = torch.from_numpy(v.recolor.M.reshape(9).copy()).cuda()
    b = torch.from_numpy(v.recolor.b.copy()).cuda()
    render_sh = d.sh.clone()
    ws = R.DeviceWorkspace(sc.n, v.camera.width, v.camera.height, (32, 32), key_capacity=16 * sc.n)
    img = torch.empty((v.camera.height, v.camera.width, 3), device="cuda")
    for _ in range(2):   # two frames: the second starts from the first's state
        R.recogs_recolor(d.c_struct(), render_sh.data_ptr(), mask_t.data_ptr(), M.data_ptr(), b.data_ptr(), 0)
        R.render(d, v.camera, ws, (32, 32), 1, image=img, sh=render_sh, graph_mode=True)
    K, _ = ws.readback()
    assert 0 < K <= ws.ws.key_capacity
    torch.cuda.synchronize()
    mask = mask_t.cpu().numpy()
    ref_mask, flag = orc.select(sc, v.camera, v.select)
    assert np.array_equal(mask[flag == 0], ref_mask[flag == 0])
    pr = orc.project(sc, v.camera, (32, 32), mask=mask, M=v.recolor.M.astype(np.float64),
                     b=v.recolor.b.astype(np.float64))
    wins = crop_windows(w, w.extra["crops"])
    ref = orc.render_windows(pr, wins)
    got = np.concatenate([img[y:y + 32, x:x + 32].reshape(-1, 3).cpu().numpy().astype(np.float64)
                          for (x, y, _, _) in wins])
    err, nband = assert_pixels(got, ref.rgb, ref.slack, TOL_F32, "benchmarked frame")
    # the unselected coefficients of the render copy are the pristine ones
    keep = mask == 0
    assert torch.equal(render_sh[:, torch.from_numpy(keep).cuda()], d.sh[:, torch.from_numpy(keep).cuda()])
    print(f"benchmarked frame: K={K}, {int(mask.sum())} selected, crops max|err| {err:.2e}, in-band {nband}")


def test_separate_recolor_then_render_equals_fused(R, orc):
    """recogs_recolor on coefficients then render == render with the fused recolour
    (within float32 rounding), tying eq. (6)'s coefficient form to its colour form."""
    import torch
    w = synth.make_mid(n=100_000)
    mask, _ = orc.select(w.scene, w.view.camera, w.view.select)
    rec = w.view.recolor
    a = gpu_run(w, fused=(mask, rec.M, rec.b))
    d = a["dscene"]
    dst = d.sh.clone()
    R.recogs_recolor(d.c_struct(), dst.data_ptr(), a["mask"].data_ptr(), a["M"].data_ptr(), a["b"].data_ptr(), 0)
    ws = R.DeviceWorkspace(w.scene.n, w.view.camera.width, w.view.camera.height)
    img = R.render(d, w.view.camera, ws, sh=dst)
    torch.cuda.synchronize()
    assert (img - a["img"]).abs().max().item() <= 1e-4


# ---------------------------------------------------------------------------
# invariants
# ---------------------------------------------------------------------------
def test_tile_shape_ppt_and_sort_mode_do_not_change_bits(R):
    w = synth.make_mid(n=100_000)
    base = gpu_run(w, tile=(16, 16), ppt=1)["img"].cpu().numpy()
    for tile in [(16, 16), (8, 8), (32, 8), (32, 16), (32, 32)]:
        for ppt in [1, 2, 4]:
            for mode in [0, 1, 2]:
                img = gpu_run(w, tile=tile, ppt=ppt, sort_mode=mode)["img"].cpu().numpy()
                assert np.array_equal(img, base), (tile, ppt, mode, np.abs(img - base).max())
        # the blend that also writes the backward's per-pixel state draws the same bits
        img = gpu_run(w, tile=tile, ppt=2, keep_backward=True)["img"].cpu().numpy()
        assert np.array_equal(img, base), (tile, "keep_backward")


def test_chw_output_is_the_hwc_image_transposed(R):
    """The CHW layout (the rasteriser's original one, Sec. 4.2) holds the same bits as the
    HWC image, in the region form, the tile form and with the backward state kept; the
    backward refuses a CHW render."""
    import torch
    w = synth.make_mid(n=100_000)
    d = R.DeviceScene(w.scene)
    cam = w.view.camera
    for tile, ppt, keep in [((32, 32), 1, False), ((16, 16), 2, True), ((32, 8), 2, False), ((8, 8), 4, True)]:
        ws = R.DeviceWorkspace(d.n, cam.width, cam.height, tile)
        hwc = R.render(d, cam, ws, tile, ppt, (0.1, 0.2, 0.3), keep_backward=keep).clone()
        chw = R.render(d, cam, ws, tile, ppt, (0.1, 0.2, 0.3), keep_backward=keep, chw=True)
        assert chw.shape == (3, cam.height, cam.width)
        assert torch.equal(chw.permute(1, 2, 0), hwc), (tile, ppt)
    o = R.opts_struct((8, 8), 4, (0.1, 0.2, 0.3), keep_backward=True, chw=True)
    n = d.n
    buf = [torch.empty(n, device="cuda"), torch.empty(3 * n, device="cuda"), torch.empty(9, device="cuda")]
    with pytest.raises(R.RecogsError) as e:
        R.recogs_render_backward(d.c_struct(), R.camera_struct(cam), o, ws.ws, chw.data_ptr(), chw.data_ptr(),
                                 buf[0].data_ptr(), buf[1].data_ptr(), buf[2].data_ptr())
    assert e.value.status == -3


def test_hue_permutation_exact_and_identity_exact(R):
    w = synth.make_mid(n=100_000)
    n = w.scene.n
    ones = np.ones(n, np.uint8)
    plain = gpu_run(w)["img"].cpu().numpy()
    hue = gpu_run(w, fused=(ones, synth.hue_rotation(120.0), np.zeros(3, np.float32)))["img"].cpu().numpy()
    assert np.array_equal(hue[..., 0], plain[..., 2])
    assert np.array_equal(hue[..., 1], plain[..., 0])
    assert np.array_equal(hue[..., 2], plain[..., 1])
    ident = gpu_run(w, fused=(ones, np.eye(3, dtype=np.float32), np.zeros(3, np.float32)))["img"].cpu().numpy()
    assert np.array_equal(ident, plain)


def test_deterministic(R):
    w = synth.make_mid(n=100_000)
    a = gpu_run(w)
    b = gpu_run(w, ws=a["ws"], dscene=a["dscene"])
    assert np.array_equal(a["img"].cpu().numpy(), b["img"].cpu().numpy())


def test_stage_profiling_modes_leave_the_image_unchanged(R):
    import torch
    w = synth.make_mid(n=50_000)
    v = w.view
    d = R.DeviceScene(w.scene)
    ws = R.DeviceWorkspace(d.n, v.camera.width, v.camera.height)
    ref = R.render(d, v.camera, ws, (16, 16), 2).clone()
    img = R.render(d, v.camera, ws, (16, 16), 2, profile=1)
    assert torch.equal(img, ref)
    assert ws.ws.stage_ms[8] > 0 and ws.ws.profiled_frames == 0
    for _ in range(3):
        img = R.render(d, v.camera, ws, (16, 16), 2, profile=2)
    assert torch.equal(img, ref)
    assert ws.ws.profiled_frames == 2  # the third is harvested by the flush
    blend_ms, nfr = ws.blend_time()
    assert nfr == 3 and blend_ms > 0 and ws.ws.stage_ms_sum[0] == 0
    R.recogs_workspace_profile_flush(ws.ws)  # nothing pending: no change
    assert ws.ws.profiled_frames == 3
    ws.release()
    assert not ws.ws.profile_state
    img = R.render(d, v.camera, ws, (16, 16), 2, profile=2)  # recreated on demand
    assert torch.equal(img, ref)
    assert ws.blend_time()[1] == 4


def test_tile_first_order_long_lists(R, orc):
    """Tile lists longer than one workgroup's LDS sort (8,192 keys): 200,000 Gaussians in a
    small view, the per-tile depth sort going through memory; the sorted lists and the
    image equal those of the depth-first order, and the lists the oracle's."""
    import torch
    w = synth.make_mid()
    c = synth.orbit_camera(96, 80, 50.0, 4.0, 0.7, 0.3)
    w1 = synth.Workload("dense", [w.scene], [synth.View(0, c, w.view.select, w.view.recolor)])
    n = w.scene.n
    for tile in [(32, 32), (16, 16)]:
        a = gpu_run(w1, tile=tile, sort_mode=0)
        b = gpu_run(w1, tile=tile, sort_mode=2, dscene=a["dscene"])
        lens = (b["ws"].ranges()[:, 1] - b["ws"].ranges()[:, 0]).cpu().numpy()
        assert lens.max() > 8192 and (lens > 1).sum() > 1, lens.max()
        assert torch.equal(a["img"], b["img"])
        K = int(a["ws"].ws.num_keys)
        assert int(b["ws"].ws.num_keys) == K
        assert torch.equal(a["ws"].vals_sorted()[:K], b["ws"].vals_sorted()[:K])
        assert torch.equal(a["ws"].ranges(), b["ws"].ranges())
        p = pull(b, n)
        pr = orc.project(w.scene, c, tile)
        _check_integer_steps(w1, orc, p, pr, n)
        print(f"{tile}: K={K}, longest list {lens.max()}")


# ---------------------------------------------------------------------------
# edge cases
# ---------------------------------------------------------------------------
def test_empty_scene_and_background(R):
    w = synth.make_tiny()
    empty = w.scene.subset(np.arange(0))
    w0 = synth.Workload("empty", [empty], w.views)
    img = gpu_run(w0, bg=(0.25, 0.5, 0.75))["img"].cpu().numpy()
    assert np.array_equal(img, np.broadcast_to(np.float32([0.25, 0.5, 0.75]), img.shape))


def test_all_behind_camera(R):
    w = synth.make_tiny()
    c = w.view.camera
    # flip the viewing direction: looking away from the scene
    R_ = c.R.copy()
    R_[2] = -R_[2]
    R_[0] = -R_[0]
    behind = synth.Camera(c.width, c.height, c.fx, c.fy, c.cx, c.cy, R_, np.float32([0, 0, -3]), c.znear)
    w1 = synth.Workload("behind", [w.scene], [synth.View(0, behind, w.view.select, w.view.recolor)])
    out = gpu_run(w1)
    assert out["ws"].ws.num_keys == 0
    assert np.array_equal(out["img"].cpu().numpy(), np.zeros((c.height, c.width, 3), np.float32))


@pytest.mark.parametrize("size", [(97, 61), (1, 1), (33, 200)])
def test_ragged_image_sizes(R, orc, size):
    W, H = size
    w = synth.make_tiny()
    c = synth.orbit_camera(W, H, 60.0, 3.0, 0.4, 0.3)
    w1 = synth.Workload("ragged", [w.scene], [synth.View(0, c, w.view.select, w.view.recolor)])
    for tile, mode in [((16, 16), 0), ((32, 8), 0), ((8, 8), 1), ((32, 32), 2), ((8, 8), 2)]:
        out = gpu_run(w1, tile=tile, sort_mode=mode)
        p = pull(out, w.scene.n)
        pr = orc.project(w.scene, c, tile)
        _check_integer_steps(w1, orc, p, pr, w.scene.n)
        ref = orc.render_image(pr, brute=True)
        assert_pixels(p["img"], ref.rgb, ref.slack, TOL_F32, f"{size} {tile}")


def test_capacity_error_reports_needed_keys(R):
    import torch
    w = synth.make_tiny()
    d = R.DeviceScene(w.scene)
    ws = R.DeviceWorkspace(w.scene.n, 128, 128, (16, 16), key_capacity=100)
    img = torch.empty((128, 128, 3), device="cuda")
    with pytest.raises(R.RecogsError) as e:
        R.render(d, w.view.camera, ws, image=img, grow=False)
    assert e.value.status == -2
    need = int(ws.ws.num_keys)
    assert need > 100
    assert R.recogs_workspace_keys_needed(ws.ws) == need
    R.render(d, w.view.camera, ws, image=img, grow=True)
    torch.cuda.synchronize()
    assert int(ws.ws.num_keys) == need
    assert R.recogs_workspace_keys_needed(ws.ws) == need
    # a graph-mode render reads nothing back; the call reports what it needed
    R.render(d, w.view.camera, ws, image=img, graph_mode=True)
    assert R.recogs_workspace_keys_needed(ws.ws) == need


def test_stride_larger_than_n(R, orc):
    w = synth.make_tiny()
    d = R.DeviceScene(w.scene, stride=w.scene.n + 1000)
    out = gpu_run(w, dscene=d)
    pr = orc.project(w.scene, w.view.camera)
    ref = orc.render_image(pr, brute=True)
    assert_pixels(out["img"].cpu().numpy().astype(np.float64), ref.rgb, ref.slack, TOL_F32, "stride")
