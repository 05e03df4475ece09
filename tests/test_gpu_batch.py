"""Batched form: many uneven (scene, view) renders in one launch sequence, replayed
from a HIP graph, with per-view selection and fused recolour."""
import functools

import numpy as np
import pytest

import synth
from tests.gpu_common import assert_pixels

pytestmark = pytest.mark.gpu

SIZES = (20_000, 50_000, 5_000, 0)
RES = ((64, 64), (200, 120), (320, 180))


@pytest.fixture(scope="module")
def R():
    import paper_2511_18441_amd as R
    return R


@functools.lru_cache(maxsize=None)
def _workload():
    return synth.make_batch(seed_base=3100, sizes=SIZES, resolutions=RES, storage="f16")


def _device(R):
    import torch
    w = _workload()
    dscenes = [R.DeviceScene(sc) for sc in w.scenes]
    views = []
    for v in w.views:
        d = dscenes[v.scene]
        mask = torch.zeros(max(d.n, 1), dtype=torch.uint8, device="cuda")
        count = torch.zeros(1, dtype=torch.int32, device="cuda")
        if d.n:
            R.recogs_select(d.c_struct(), R.camera_struct(v.camera), R.select_struct(v.select), mask.data_ptr(),
                            count.data_ptr())
        M = torch.from_numpy(v.recolor.M.reshape(9).copy()).cuda()
        b = torch.from_numpy(v.recolor.b.copy()).cuda()
        views.append((v.scene, v.camera, mask, M, b))
    return w, dscenes, views


def _singles(R, dscenes, views, tile, ppt, bg=(0.0, 0.0, 0.0)):
    outs = []
    for (si, cam, mask, M, b) in views:
        d = dscenes[si]
        ws = R.DeviceWorkspace(d.n, cam.width, cam.height, tile)
        outs.append(R.render(d, cam, ws, tile, ppt, bg, mask, M, b).clone())
    return outs


@pytest.mark.parametrize("tile,ppt", [((16, 16), 2), ((8, 8), 1), ((32, 8), 4), ((32, 32), 2), ((32, 16), 4)])
def test_batch_equals_single_renders(R, tile, ppt):
    import torch
    w, dscenes, views = _device(R)
    b = R.DeviceBatch(dscenes, views, tile, ppt, bg=(0.1, 0.2, 0.3))
    b.render()
    k, ovf = b.readback()
    assert not ovf and k > 0
    ref = _singles(R, dscenes, views, tile, ppt, bg=(0.1, 0.2, 0.3))
    for i, (a, r) in enumerate(zip(b.images, ref)):
        assert torch.equal(a, r), (i, (a - r).abs().max().item())


def test_batch_graph_replay_matches_eager(R):
    import torch
    w, dscenes, views = _device(R)
    b = R.DeviceBatch(dscenes, views, (16, 16), 2)
    b.render()
    torch.cuda.synchronize()
    eager = [im.clone() for im in b.images]
    g = b.capture_graph()
    for rep in range(3):
        for im in b.images:
            im.fill_(-1.0)
        x = torch.randn(1000, device="cuda")  # unrelated eager work between replays
        (x * 2).sum().item()
        g.replay()
        torch.cuda.synchronize()
        for i, (a, e) in enumerate(zip(b.images, eager)):
            assert torch.equal(a, e), (rep, i)


def test_batch_overflow_sets_flag_and_draws_background(R):
    import torch
    w, dscenes, views = _device(R)
    b = R.DeviceBatch(dscenes, views, (16, 16), 1, bg=(0.25, 0.5, 0.75), key_capacity=10)
    b.render()
    k, ovf = b.readback()
    assert ovf and k > 10
    for im in b.images:
        assert torch.equal(im, torch.tensor([0.25, 0.5, 0.75], device="cuda").expand_as(im))


def test_batch_view_matches_oracle(R, orc):
    w, dscenes, views = _device(R)
    b = R.DeviceBatch(dscenes, views, (16, 16), 2)
    b.render()
    b.readback()
    k = 4  # scene 1 (50,000 Gaussians), 200 x 120
    v = w.views[k]
    sc = w.scenes[v.scene]
    mask = views[k][2].cpu().numpy()[: sc.n]
    pr = orc.project(sc, v.camera, (16, 16), mask=mask, M=v.recolor.M.astype(np.float64),
                     b=v.recolor.b.astype(np.float64))
    ref = orc.render_image(pr)
    got = b.images[k].cpu().numpy().astype(np.float64)
    err, nband = assert_pixels(got, ref.rgb, ref.slack, 2e-3, f"batch view {k}")
    print(f"batch view {k}: max|err| outside band {err:.2e}, in-band pixels {nband}")
    assert mask.sum() > 0


def test_autotune_batch_picks_a_candidate_with_identical_bits(R):
    from paper_2511_18441_amd import autotune
    w, dscenes, views = _device(R)
    cands = (((16, 16), 1), ((32, 32), 2), ((32, 8), 2), ((8, 8), 1))
    res = autotune.tune_batch(dscenes, views, candidates=cands, reps=2, cache=None)
    assert (tuple(res["tile"]), res["ppt"]) in cands
    assert len(res["table"]) == len(cands)


def test_batch_full_size_sampled_views_vs_oracle(R, orc):
    """The batched workload at full size (8 scenes, 9.35M Gaussians, FP16, 32 views of
    mixed resolution, per-view selection and hue rotation) in one launch sequence;
    two views (the 3M-Gaussian scene at 256x256 and a 1M-Gaussian scene at
    1920x1080) checked against the oracle on seeded 32x32 crops."""
    import torch
    w = synth.make_batch()
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
    b = R.DeviceBatch(dscenes, views, (32, 32), 1)
    b.render()
    k, ovf = b.readback()
    assert not ovf and k > 40_000_000
    rng = np.random.default_rng(44)
    for vi in (28, 15):
        v = w.views[vi]
        sc = w.scenes[v.scene]
        cam = v.camera
        mask = views[vi][2].cpu().numpy()[: sc.n]
        pr = orc.project(sc, cam, (32, 32), mask=mask, M=v.recolor.M.astype(np.float64),
                         b=v.recolor.b.astype(np.float64))
        wins = [(int(rng.integers(0, cam.width - 32)), int(rng.integers(0, cam.height - 32)), 32, 32)
                for _ in range(4)]
        ref = orc.render_windows(pr, wins)
        img = b.images[vi].cpu().numpy().astype(np.float64)
        got = np.concatenate([img[y0:y0 + wh, x0:x0 + ww].reshape(-1, 3) for (x0, y0, ww, wh) in wins])
        err, nband = assert_pixels(got, ref.rgb, ref.slack, 2e-3, f"batch view {vi} crops {wins}")
        print(f"batch view {vi}: max|err| outside band {err:.2e}, in-band pixels {nband}")
        assert mask.sum() > 0
