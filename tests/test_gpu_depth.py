"""Rough depth map (Sec. 3.2) written by the region blend: parity with the oracle.

Per pixel the depth of the blended splat that takes the transmittance below tau (0
where none does). Where the oracle flags no in-band decision (an alpha near 1/255 or
a transmittance within its float32 band of tau or of the stop threshold) the depth
must be bit-identical to the oracle's float32 depth; flagged pixels must hold 0 or a
visible splat's depth. The depth pass must not change the image or the backward state.
"""
import numpy as np
import pytest

import synth
from tests.gpu_common import crop_windows

pytestmark = pytest.mark.gpu

REGION_SHAPES = [((16, 16), 1), ((16, 16), 2), ((32, 32), 1), ((32, 32), 4), ((8, 8), 1), ((32, 8), 1),
                 ((32, 16), 2)]


@pytest.fixture(scope="module")
def R():
    import paper_2511_18441_amd as R
    return R


def _render(R, d, cam, tile, ppt, tau, keep=False, graph=False, ws=None):
    import torch
    if ws is None:
        ws = R.DeviceWorkspace(d.n, cam.width, cam.height, tile)
    depth = torch.full((cam.height, cam.width), -1.0, device="cuda")   # every pixel must be written
    img = R.render(d, cam, ws, tile, ppt, keep_backward=keep, depth=depth, depth_tau=tau, graph_mode=graph)
    torch.cuda.synchronize()
    return img, depth, ws


def _compare(got, ref, flag, z32, what, max_flagged=0.02):
    got = np.asarray(got, np.float64).reshape(-1)
    ok = flag == 0
    bad = ok & (got != ref)
    assert not bad.any(), (f"{what}: {int(bad.sum())} unflagged pixels differ; first "
                           f"{list(zip(got[bad][:4], ref[bad][:4]))}")
    f = ~ok
    assert np.all((got[f] == 0) | np.isin(got[f], z32)), what
    assert flag.mean() <= max_flagged, (what, flag.mean())
    return int(f.sum())


def _visible_z32(orc, pr):
    return pr.col("z32")[pr.col("status") == 0]


@pytest.mark.parametrize("tile,ppt", REGION_SHAPES)
def test_depth_map_tiny_every_region_shape(R, orc, tile, ppt):
    w = synth.make_tiny()
    cam = w.view.camera
    d = R.DeviceScene(w.scene)
    pr = orc.project(w.scene, cam, tile)
    z = _visible_z32(orc, pr)
    full = [(0, 0, cam.width, cam.height)]
    for tau in (1.0, 0.5, 0.1, 1e-3):
        _, dep, _ = _render(R, d, cam, tile, ppt, tau)
        ref, flag = orc.depth_windows(pr, full, tau)
        _compare(dep.cpu().numpy(), ref, flag, z, f"tiny {tile} {ppt} tau {tau}", max_flagged=0.05)
        if tau == 0.5:
            assert (ref > 0).mean() > 0.2


def test_depth_map_mid_full_image(R, orc):
    w = synth.make_mid()
    cam = w.view.camera
    d = R.DeviceScene(w.scene)
    pr = orc.project(w.scene, cam, (32, 32))
    _, dep, _ = _render(R, d, cam, (32, 32), 1, 0.5)
    ref, flag = orc.depth_windows(pr, crop_windows(w, [(x, y) for y in range(0, 800, 32) for x in range(0, 800, 32)]),
                                  0.5)
    got = np.concatenate([dep.cpu().numpy()[y:y + 32, x:x + 32].reshape(-1)
                          for y in range(0, 800, 32) for x in range(0, 800, 32)])
    nf = _compare(got, ref, flag, _visible_z32(orc, pr), "mid 800x800")
    print(f"mid: {nf} flagged pixels, {(ref > 0).mean():.3f} with a depth")


@pytest.mark.parametrize("tile,ppt,keep", [((32, 32), 1, False), ((16, 16), 2, True)])
def test_depth_map_1m_1080p_crops(R, orc, tile, ppt, keep):
    """1,000,000 Gaussians at 1920x1080 on the 64 seeded 32x32 crops (32x32 tiles with
    1 pixel per thread is the benchmarked launch)."""
    w = synth.make_precision()
    cam = w.view.camera
    d = R.DeviceScene(w.scene)
    _, dep, _ = _render(R, d, cam, tile, ppt, 0.5, keep=keep)
    pr = orc.project(w.scene, cam, tile)
    wins = crop_windows(w, w.extra["crops"])
    ref, flag = orc.depth_windows(pr, wins, 0.5)
    full = dep.cpu().numpy()
    got = np.concatenate([full[y:y + 32, x:x + 32].reshape(-1) for (x, y, _, _) in wins])
    nf = _compare(got, ref, flag, _visible_z32(orc, pr), f"1M 1080p {tile} {ppt}")
    assert np.all(full >= 0)
    print(f"1M: {nf} flagged of {got.size}; {(ref > 0).mean():.3f} with a depth")


def test_depth_pass_leaves_image_and_state_unchanged(R):
    import torch
    w = synth.make_mid(n=100_000)
    cam = w.view.camera
    d = R.DeviceScene(w.scene)
    for tile, ppt in REGION_SHAPES:
        ws = R.DeviceWorkspace(d.n, cam.width, cam.height, tile)
        base = R.render(d, cam, ws, tile, ppt, keep_backward=True).clone()
        T0, n0 = ws.final_T().clone(), ws.nproc().clone()
        img, dep, _ = _render(R, d, cam, tile, ppt, 0.5, keep=True, ws=ws)
        assert torch.equal(img, base), tile
        assert torch.equal(ws.final_T(), T0) and torch.equal(ws.nproc(), n0), tile
        img2, dep2, _ = _render(R, d, cam, tile, ppt, 0.5, keep=False, ws=ws)
        assert torch.equal(img2, base) and torch.equal(dep2, dep), tile
        if tile == (16, 16) and ppt == 1:
            ref_dep = dep
        else:
            assert torch.equal(dep, ref_dep), (tile, ppt)   # the same bits for every region shape


def test_depth_map_in_graph_mode_equals_eager(R):
    import torch
    w = synth.make_mid(n=100_000)
    cam = w.view.camera
    d = R.DeviceScene(w.scene)
    _, a, ws = _render(R, d, cam, (32, 32), 1, 0.5)
    _, b, _ = _render(R, d, cam, (32, 32), 1, 0.5, graph=True, ws=ws)
    assert torch.equal(a, b)


@pytest.mark.parametrize("size", [(97, 61), (1, 1), (33, 200)])
def test_depth_map_ragged_sizes(R, orc, size):
    W, H = size
    w = synth.make_tiny()
    c = synth.orbit_camera(W, H, 60.0, 3.0, 0.4, 0.3)
    d = R.DeviceScene(w.scene)
    for tile, ppt in [((16, 16), 1), ((32, 32), 2)]:
        pr = orc.project(w.scene, c, tile)
        _, dep, _ = _render(R, d, c, tile, ppt, 0.5)
        ref, flag = orc.depth_windows(pr, [(0, 0, W, H)], 0.5)
        _compare(dep.cpu().numpy(), ref, flag, _visible_z32(orc, pr), f"{size} {tile}", max_flagged=0.05)


def test_depth_map_empty_scene_is_zero(R):
    w = synth.make_tiny()
    empty = w.scene.subset(np.arange(0))
    d = R.DeviceScene(empty)
    cam = w.view.camera
    img, dep, _ = _render(R, d, cam, (32, 32), 1, 0.5)
    assert np.array_equal(dep.cpu().numpy(), np.zeros((cam.height, cam.width), np.float32))
