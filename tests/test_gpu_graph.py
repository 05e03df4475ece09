"""Graph mode of the single-view render: no host synchronisation, device-side counts
and capacity decision, capturable in a HIP graph."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import paper_2511_18441_amd as R
    return R


def _setup(R, n=100_000):
    import torch
    w = synth.make_mid(n=n)
    v = w.view
    d = R.DeviceScene(w.scene)
    mask = torch.empty(d.n, dtype=torch.uint8, device="cuda")
    cnt = torch.empty(1, dtype=torch.int32, device="cuda")
    R.recogs_select(d.c_struct(), R.camera_struct(v.camera), R.select_struct(v.select), mask.data_ptr(), cnt.data_ptr())
    M = torch.from_numpy(v.recolor.M.reshape(9).copy()).cuda()
    b = torch.from_numpy(v.recolor.b.copy()).cuda()
    return w, v, d, mask, M, b


@pytest.mark.parametrize("mode", [0, 2])
@pytest.mark.parametrize("tile,ppt", [((16, 16), 2), ((8, 8), 1), ((32, 8), 4), ((32, 32), 2)])
def test_graph_mode_equals_eager(R, tile, ppt, mode):
    import torch
    w, v, d, mask, M, b = _setup(R)
    cam = v.camera
    ws_e = R.DeviceWorkspace(d.n, cam.width, cam.height, tile)
    eager = R.render(d, cam, ws_e, tile, ppt, (0.1, 0.2, 0.3), mask, M, b, sort_mode=mode).clone()  # grows on demand
    ws_g = R.DeviceWorkspace(d.n, cam.width, cam.height, tile, key_capacity=int(ws_e.ws.num_keys) + 1024)
    img = R.render(d, cam, ws_g, tile, ppt, (0.1, 0.2, 0.3), mask, M, b, graph_mode=True, sort_mode=mode)
    k, nv = ws_g.readback()
    assert torch.equal(img, eager)
    assert k == int(ws_e.ws.num_keys) and nv == int(ws_e.ws.num_visible)
    assert int(ws_g.ws.depth_min_bits) == int(ws_e.ws.depth_min_bits)
    assert torch.equal(ws_g.vals_sorted()[:k], ws_e.vals_sorted()[:k])
    assert torch.equal(ws_g.ranges(), ws_e.ranges())


@pytest.mark.parametrize("mode", [0, 2])
def test_graph_mode_captured_recolor_and_render_replays(R, mode):
    import torch
    w, v, d, mask, M, b = _setup(R)
    cam = v.camera
    ws = R.DeviceWorkspace(d.n, cam.width, cam.height, (16, 16))
    sc = d.c_struct()
    sh2 = d.sh.clone()
    img = torch.empty((cam.height, cam.width, 3), dtype=torch.float32, device="cuda")

    def frame():
        R.recogs_recolor(sc, sh2.data_ptr(), mask.data_ptr(), M.data_ptr(), b.data_ptr(), 0)
        R.render(d, cam, ws, (16, 16), 2, image=img, sh=sh2, graph_mode=True, sort_mode=mode)

    frame()
    torch.cuda.synchronize()
    eager = img.clone()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        frame()
    torch.cuda.current_stream().wait_stream(side)
    with torch.cuda.graph(g):
        frame()
    for rep in range(3):
        img.fill_(-1.0)
        sh2.copy_(d.sh)  # pristine colours: the replayed recolour must edit them again
        x = torch.randn(1000, device="cuda")
        (x * 2).sum().item()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(img, eager), rep
    assert ws.readback()[0] > 0


@pytest.mark.parametrize("mode", [0, 2])
def test_graph_mode_overflow_draws_background_and_reports(R, mode):
    import torch
    w, v, d, mask, M, b = _setup(R, n=50_000)
    cam = v.camera
    ws = R.DeviceWorkspace(d.n, cam.width, cam.height, (16, 16), key_capacity=100)
    img = R.render(d, cam, ws, (16, 16), 1, (0.25, 0.5, 0.75), graph_mode=True, sort_mode=mode)
    k, _ = ws.readback()
    assert k > 100
    assert torch.equal(img, torch.tensor([0.25, 0.5, 0.75], device="cuda").expand_as(img))
    with pytest.raises(R.RecogsError):  # a backward of an overflowed render is refused
        o = R.opts_struct(keep_backward=True)
        R.recogs_render_backward(d.c_struct(), R.camera_struct(cam), o, ws.ws, img.data_ptr(), img.data_ptr(),
                                 img.data_ptr(), img.data_ptr(), img.data_ptr())


def test_graph_mode_backward_after_readback_equals_eager(R):
    import torch
    w, v, d, mask, M, b = _setup(R, n=30_000)
    cam = v.camera
    g = torch.from_numpy(synth.random_image(11, (cam.height, cam.width, 3))).cuda()
    out = []
    for gm in (False, True):
        ws = R.DeviceWorkspace(d.n, cam.width, cam.height, (16, 16))
        img = R.render(d, cam, ws, (16, 16), 2, mask=mask, M=M, b=b, keep_backward=True, graph_mode=gm)
        if gm:
            ws.readback()
        dop = torch.empty(d.n, device="cuda")
        ddc = torch.empty((3, d.n), device="cuda")
        dM = torch.empty(9, device="cuda")
        o = R.opts_struct((16, 16), 2, (0, 0, 0), mask, M, b, keep_backward=True)
        R.recogs_render_backward(d.c_struct(), R.camera_struct(cam), o, ws.ws, img.data_ptr(), g.data_ptr(),
                                 dop.data_ptr(), ddc.data_ptr(), dM.data_ptr())
        torch.cuda.synchronize()
        out.append((img.clone(), dop.clone(), ddc.clone(), dM.clone()))
    for a, c in zip(out[0], out[1]):
        assert torch.equal(a, c)
