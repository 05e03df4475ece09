"""The 3DGS rasteriser's square extent (render option extent_rule = 1) through the C
ABI against the oracle at the same tile shape: under this rule a splat reaches only
the pixels of the tiles that list it, so each tile shape draws its own image and is
compared with the oracle's image for that shape.

Integer steps (tile rectangles, counts, scan, sorted lists, ranges) must match
exactly outside the oracle's rounding bands. Pixels are compared wherever the GPU and
the oracle list the same Gaussians in the pixel's tile: only a Gaussian whose
rectangle edge lies in its rounding band (flagged, and then only where the two
rectangles differ) can list differently.
"""
import numpy as np
import pytest

import synth
from tests.gpu_common import assert_pixels, crop_windows, gpu_run, pull
from tests.test_gpu_parity import TOL_F32, _check_integer_steps

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import paper_2511_18441_amd as R
    return R


def _membership_differs(p, pr, W, H, tile):
    """(H, W) bool: pixels in a tile that the GPU and the oracle list differently for
    some Gaussian (the symmetric difference of the two rectangles)."""
    tw, th = tile
    tx_n, ty_n = -(-W // tw), -(-H // th)
    bad_t = np.zeros((ty_n, tx_n), bool)
    r = p["rects"]
    g = np.stack([r[:, 0] & 0xFFFF, r[:, 0] >> 16, r[:, 1] & 0xFFFF, r[:, 1] >> 16], 1)
    g = np.where((p["counts"] > 0)[:, None], g, np.array([0, -1, 0, -1]))
    o = np.stack([pr.col("txlo"), pr.col("txhi"), pr.col("tylo"), pr.col("tyhi")], 1)
    o = np.where((pr.col("count") > 0)[:, None], o, np.array([0, -1, 0, -1]))
    for i in np.nonzero((g != o).any(axis=1))[0]:
        a = np.zeros((ty_n, tx_n), bool)
        b = np.zeros((ty_n, tx_n), bool)
        a[g[i, 2]:g[i, 3] + 1, g[i, 0]:g[i, 1] + 1] = True
        b[o[i, 2]:o[i, 3] + 1, o[i, 0]:o[i, 1] + 1] = True
        bad_t |= a ^ b
    return np.repeat(np.repeat(bad_t, th, 0), tw, 1)[:H, :W]


@pytest.mark.parametrize("cfg", ["tiny", "mid"])
@pytest.mark.parametrize("tile,ppt", [((16, 16), 1), ((8, 8), 2), ((32, 8), 4), ((32, 32), 1), ((32, 16), 2)])
def test_square_rule_vs_oracle(R, orc, cfg, tile, ppt):
    w = synth.make_tiny() if cfg == "tiny" else synth.make_mid(n=100_000)
    n = w.scene.n
    cam = w.view.camera
    out = gpu_run(w, tile=tile, ppt=ppt, extent_rule=1, bg=(0.1, 0.2, 0.3))
    p = pull(out, n)
    pr = orc.project(w.scene, cam, tile, extent_rule=1)
    _check_integer_steps(w, orc, p, pr, n)
    ref = orc.render_image(pr, bg=(0.1, 0.2, 0.3), brute=(cfg == "tiny"))
    skip = _membership_differs(p, pr, cam.width, cam.height, tile)
    assert skip.mean() < 0.01, skip.mean()
    err, nband = assert_pixels(p["img"][~skip], ref.rgb[~skip], ref.slack[~skip], TOL_F32, f"{cfg} {tile} {ppt}")
    assert err <= TOL_F32
    print(f"{cfg} {tile} ppt {ppt}: K={p['K']} max|err| {err:.2e}, in-band {nband}, "
          f"pixels of differently listed tiles {int(skip.sum())}")


def test_square_rule_differs_from_the_box_and_between_tile_shapes(R):
    """The square cuts visible tails the box keeps, so the two rules and two tile shapes
    under the square draw different images; the box draws the same bits at every shape."""
    w = synth.make_mid(n=100_000)
    a = gpu_run(w, tile=(16, 16), extent_rule=1)["img"].cpu().numpy()
    b = gpu_run(w, tile=(32, 32), extent_rule=1)["img"].cpu().numpy()
    c = gpu_run(w, tile=(16, 16))["img"].cpu().numpy()
    d = gpu_run(w, tile=(32, 32))["img"].cpu().numpy()
    assert np.array_equal(c, d)
    assert not np.array_equal(a, c) and not np.array_equal(a, b)


def test_square_rule_1m_1080p_crops(R, orc):
    """1,000,000 Gaussians at 1920x1080 with the 3DGS rasteriser's 16x16 tiles and its
    extent: whole-frame integer steps, pixels on the 64 seeded 32x32 crops."""
    w = synth.make_precision()
    n = w.scene.n
    tile = (16, 16)
    out = gpu_run(w, tile=tile, extent_rule=1)
    p = pull(out, n)
    pr = orc.project(w.scene, w.view.camera, tile, extent_rule=1)
    _check_integer_steps(w, orc, p, pr, n)
    wins = crop_windows(w, w.extra["crops"])
    ref = orc.render_windows(pr, wins)
    skip = _membership_differs(p, pr, w.view.camera.width, w.view.camera.height, tile)
    got = np.concatenate([p["img"][y:y + 32, x:x + 32].reshape(-1, 3) for (x, y, _, _) in wins])
    keep = ~np.concatenate([skip[y:y + 32, x:x + 32].reshape(-1) for (x, y, _, _) in wins])
    assert keep.mean() > 0.98
    err, nband = assert_pixels(got[keep], ref.rgb[keep], ref.slack[keep], TOL_F32, "1M square rule crops")
    print(f"1M square rule: K={p['K']} crops max|err| {err:.2e}, in-band {nband}, skipped {int((~keep).sum())}")


def test_square_rule_batch_equals_single_renders(R):
    """The batched form under the square rule draws each view as its single render does."""
    import torch
    w = synth.make_batch(seed_base=3100, sizes=(20_000, 50_000, 5_000), resolutions=((64, 64), (200, 120)),
                         storage="f16")
    dscenes = [R.DeviceScene(sc) for sc in w.scenes]
    views = []
    for v in w.views:
        dd = dscenes[v.scene]
        mask = torch.zeros(max(dd.n, 1), dtype=torch.uint8, device="cuda")
        count = torch.zeros(1, dtype=torch.int32, device="cuda")
        R.recogs_select(dd.c_struct(), R.camera_struct(v.camera), R.select_struct(v.select), mask.data_ptr(),
                        count.data_ptr())
        views.append((v.scene, v.camera, mask, torch.from_numpy(v.recolor.M.reshape(9).copy()).cuda(),
                      torch.from_numpy(v.recolor.b.copy()).cuda()))
    for tile, ppt in [((16, 16), 1), ((32, 8), 2)]:
        b = R.DeviceBatch(dscenes, views, tile, ppt, extent_rule=1)
        b.render()
        k, ovf = b.readback()
        assert not ovf
        for vi, (si, cam, mask, M, bb) in enumerate(views):
            ws = R.DeviceWorkspace(dscenes[si].n, cam.width, cam.height, tile)
            one = R.render(dscenes[si], cam, ws, tile, ppt, mask=mask, M=M, b=bb, extent_rule=1)
            assert torch.equal(one, b.images[vi]), (tile, vi)
