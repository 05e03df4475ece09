"""Backward of the blend and the fused recolour (eq. 8 restricted to opacity, SH DC
and the recolour matrix) and the L2 loss gradient, through the C ABI, against the
FP64 oracle (whose gradient is itself pinned to central finite differences on the
CPU) and, loosely, against finite differences of the GPU's own float32 forward."""
import functools

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=None)
def _wfd():
    """4,096 seeded Gaussians of the 1M-Gaussian differentiation scene, 64x64 (view 0)."""
    return synth.make_diff_fd()


@pytest.fixture(scope="module")
def R():
    import paper_2511_18441_amd as R
    return R


def _setup(R, orc, w, g_seed=21):
    import torch
    v = w.view
    sc = w.scene
    mask, _ = orc.select(sc, v.camera, v.select)
    M = v.recolor.M
    b = v.recolor.b
    d = R.DeviceScene(sc)
    ws = R.DeviceWorkspace(sc.n, v.camera.width, v.camera.height)
    tm = torch.from_numpy(mask).cuda()
    tM = torch.from_numpy(M.reshape(9).copy()).cuda()
    tb = torch.from_numpy(b.copy()).cuda()
    g = synth.random_image(g_seed, (v.camera.height, v.camera.width, 3))
    return d, ws, tm, tM, tb, mask, M, b, g


def _gpu_grads(R, d, ws, cam, tm, tM, tb, g, tile=(16, 16), ppt=1, blocks=False, graph=False):
    """Render keeping the backward state, then recogs_render_backward; blocks: the
    backward's block form (one wave per 8 x 8 ppt block, with its scratch); graph: the
    render in graph mode, not read back (the backward then reads the key count on the
    device)."""
    import torch
    img = R.render(d, cam, ws, tile, ppt, mask=tm, M=tM, b=tb, keep_backward=True, graph_mode=graph)
    gt = torch.from_numpy(g).cuda()
    n = d.n
    dop = torch.empty(n, device="cuda")
    ddc = torch.empty((3, n), device="cuda")
    dM = torch.empty(9, device="cuda")
    scratch = ws.backward_scratch(tile, ppt) if blocks else None
    assert (scratch is not None) == blocks
    o = R.opts_struct(tile, ppt, (0, 0, 0), tm, tM, tb, keep_backward=True, bwd_scratch=scratch)
    R.recogs_render_backward(d.c_struct(), R.camera_struct(cam), o, ws.ws, img.data_ptr(), gt.data_ptr(),
                             dop.data_ptr(), ddc.data_ptr(), dM.data_ptr())
    torch.cuda.synchronize()
    return img, dop.cpu().numpy().astype(np.float64), ddc.cpu().numpy().astype(np.float64), \
        dM.cpu().numpy().astype(np.float64).reshape(3, 3)


# Gradient tolerance: 2e-5 of the largest entry plus 1e-4 of each entry. The float32
# sums of a few thousand per-pixel terms carry about 1e-6 of the largest; the oracle's
# FP64 gradient is pinned to central differences on the CPU.
GRAD_ABS, GRAD_REL = 2e-5, 1e-4


def _close(got, ref, what, abs_of_max=GRAD_ABS, rel=GRAD_REL):
    scale = max(np.abs(ref).max(), 1e-12)
    err = np.abs(got - ref)
    bad = err > abs_of_max * scale + rel * np.abs(ref)
    assert not bad.any(), f"{what}: {int(bad.sum())} entries off; max err {err.max():.3e} (scale {scale:.3e})"
    return float(err.max() / scale)


@pytest.mark.parametrize("tile,ppt,blocks", [((16, 16), 1, False), ((8, 8), 2, False), ((32, 8), 4, False),
                                             ((32, 32), 2, False), ((32, 16), 1, False), ((16, 16), 1, True),
                                             ((16, 16), 2, True), ((8, 8), 1, True), ((32, 8), 1, True),
                                             ((32, 16), 1, True), ((32, 16), 2, True), ((32, 32), 1, True),
                                             ((32, 32), 4, True)])
def test_backward_vs_oracle(R, orc, tile, ppt, blocks):
    w = _wfd()
    cam = w.view.camera
    d, ws, tm, tM, tb, mask, M, b, g = _setup(R, orc, w)
    pr = orc.project(w.scene, cam, tile, mask=mask, M=M.astype(np.float64), b=b.astype(np.float64))
    ref = orc.render_image(pr, brute=True)
    # pixels with an in-band threshold decision get no upstream gradient on either side
    g = np.where((ref.slack > 0)[..., None], 0.0, g).astype(np.float32)
    assert (ref.slack > 0).mean() < 0.02
    d_ws = R.DeviceWorkspace(w.scene.n, cam.width, cam.height, tile)
    img, dop, ddc, dM = _gpu_grads(R, d, d_ws, cam, tm, tM, tb, g, tile, ppt, blocks)
    gr = orc.backward(pr, g, M=M.astype(np.float64))
    e1 = _close(dop, gr.dsigma, "dL/dopacity")
    e2 = _close(ddc, gr.dc0, "dL/dC0")
    e3 = _close(dM, gr.dM, "dL/dM")
    assert mask.sum() > 0 and np.abs(gr.dM).max() > 0
    print(f"relative max errors: dsigma {e1:.2e} dC0 {e2:.2e} dM {e3:.2e}")


def test_block_form_backward_is_deterministic_and_matches_the_tile_form(R, orc):
    """The block form sums each (Gaussian, tile) gradient's block parts in a fixed order:
    two runs give the same bits; against the tile form it differs by float32 summation
    order only."""
    w = _wfd()
    cam = w.view.camera
    d, ws, tm, tM, tb, mask, M, b, g = _setup(R, orc, w)
    for tile in [(16, 16), (32, 32)]:
        wsx = R.DeviceWorkspace(w.scene.n, cam.width, cam.height, tile)
        a = _gpu_grads(R, d, wsx, cam, tm, tM, tb, g, tile, 1, blocks=True)
        c = _gpu_grads(R, d, wsx, cam, tm, tM, tb, g, tile, 1, blocks=True)
        t = _gpu_grads(R, d, wsx, cam, tm, tM, tb, g, tile, 1, blocks=False)
        for x, y, z in zip(a[1:], c[1:], t[1:]):
            assert np.array_equal(x, y)
            scale = np.abs(z).max()
            assert np.all(np.abs(x - z) <= 1e-5 * scale + 1e-5 * np.abs(z))
    # a scratch of too few bytes is refused
    import torch
    o = R.opts_struct((16, 16), 1, (0, 0, 0), tm, tM, tb, keep_backward=True,
                      bwd_scratch=torch.empty(256, dtype=torch.uint8, device="cuda"))
    img = R.render(d, cam, ws, mask=tm, M=tM, b=tb, keep_backward=True)
    buf = [torch.empty(d.n, device="cuda"), torch.empty((3, d.n), device="cuda"), torch.empty(9, device="cuda")]
    with pytest.raises(R.RecogsError) as e:
        R.recogs_render_backward(d.c_struct(), R.camera_struct(cam), o, ws.ws, img.data_ptr(), img.data_ptr(),
                                 buf[0].data_ptr(), buf[1].data_ptr(), buf[2].data_ptr())
    assert e.value.status == -1


def test_backward_after_graph_render_without_readback(R, orc):
    """After a graph-mode render that is not read back, the backward (tile and block
    forms) gives the bits of the backward of the same render made with a read-back; a
    render that overflowed its key capacity gives zero gradients, with no out-of-bounds
    read of the per-key gradient slots, and its overflow shows in the read-back."""
    import torch
    w = _wfd()
    cam = w.view.camera
    d, ws, tm, tM, tb, mask, M, b, g = _setup(R, orc, w)
    for tile, ppt, blocks in [((16, 16), 1, False), ((32, 16), 1, False), ((8, 8), 2, False), ((16, 16), 1, True)]:
        wsx = R.DeviceWorkspace(w.scene.n, cam.width, cam.height, tile)
        a = _gpu_grads(R, d, wsx, cam, tm, tM, tb, g, tile, ppt, blocks=blocks)
        c = _gpu_grads(R, d, wsx, cam, tm, tM, tb, g, tile, ppt, blocks=blocks, graph=True)
        assert wsx.ws.num_keys == -1   # not read back
        assert torch.equal(a[0], c[0])
        for x, y in zip(a[1:], c[1:]):
            assert np.array_equal(x, y), (tile, ppt, blocks)
    small = R.DeviceWorkspace(w.scene.n, cam.width, cam.height, (16, 16), key_capacity=64)
    img, dop, ddc, dM = _gpu_grads(R, d, small, cam, tm, tM, tb, g, (16, 16), 1, graph=True)
    assert not dop.any() and not ddc.any() and not dM.any()
    k, _ = small.readback()
    assert k > 64


def test_backward_is_deterministic_and_repeatable(R, orc):
    """No atomics: two renders + backwards give the same bits, and a second backward
    on the same render (its per-key scratch overwritten) gives them too."""
    import torch
    w = _wfd()
    cam = w.view.camera
    d, ws, tm, tM, tb, mask, M, b, g = _setup(R, orc, w)
    a = _gpu_grads(R, d, ws, cam, tm, tM, tb, g, (16, 16), 2)
    c = _gpu_grads(R, d, ws, cam, tm, tM, tb, g, (16, 16), 2)
    img = a[0]
    gt = torch.from_numpy(g).cuda()
    n = d.n
    dop = torch.empty(n, device="cuda")
    ddc = torch.empty((3, n), device="cuda")
    dM = torch.empty(9, device="cuda")
    o = R.opts_struct((16, 16), 2, (0, 0, 0), tm, tM, tb, keep_backward=True)
    R.recogs_render_backward(d.c_struct(), R.camera_struct(cam), o, ws.ws, c[0].data_ptr(), gt.data_ptr(),
                             dop.data_ptr(), ddc.data_ptr(), dM.data_ptr())
    torch.cuda.synchronize()
    again = (dop.cpu().numpy().astype(np.float64), ddc.cpu().numpy().astype(np.float64),
             dM.cpu().numpy().astype(np.float64).reshape(3, 3))
    assert torch.equal(a[0], c[0])
    for x, y, z in zip(a[1:], c[1:], again):
        assert np.array_equal(x, y) and np.array_equal(x, z)
    assert np.abs(a[1]).max() > 0


def test_backward_matches_gpu_finite_differences(R, orc):
    """Central differences of the GPU's own float32 loss sum(g * y) w.r.t. M (loose: the
    float32 forward has ~1e-7 relative noise, the step is 1e-2)."""
    import torch
    w = _wfd()
    cam = w.view.camera
    d, ws, tm, tM, tb, mask, M, b, g = _setup(R, orc, w)
    _, _, _, dM = _gpu_grads(R, d, ws, cam, tm, tM, tb, g)
    gt = torch.from_numpy(g).cuda().double()
    h = 1e-2
    for k in range(9):
        vals = []
        for sgn in (1, -1):
            Mp = M.reshape(9).astype(np.float64).copy()
            Mp[k] += sgn * h
            tMp = torch.from_numpy(Mp.astype(np.float32)).cuda()
            img = R.render(d, cam, ws, mask=tm, M=tMp, b=tb)
            vals.append(float((img.double() * gt).sum().item()))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - dM.flat[k]) <= 2e-3 * max(1.0, abs(fd)), (k, fd, dM.flat[k])


def test_autograd_function_matches_direct_backward(R, orc):
    import torch
    w = _wfd()
    cam = w.view.camera
    d, ws, tm, tM, tb, mask, M, b, g = _setup(R, orc, w)
    _, dop, ddc, dM = _gpu_grads(R, d, ws, cam, tm, tM, tb, g)
    # leaves sharing the scene's own storage: the opacity array and its first 3 SH planes
    op = torch.nn.Parameter(d.opacity, requires_grad=True)
    leaf_dc = torch.nn.Parameter(d.sh.narrow(0, 0, 3), requires_grad=True)
    Mt = torch.from_numpy(M.copy()).cuda().requires_grad_(True)
    ws2 = R.DeviceWorkspace(w.scene.n, cam.width, cam.height)
    img = R.RecogsRenderFn.apply(op, leaf_dc, Mt, d, cam, ws2, tm, tb)
    loss = (img * torch.from_numpy(g).cuda()).sum()
    loss.backward()
    np.testing.assert_allclose(op.grad[: d.n].cpu().numpy(), dop, rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(leaf_dc.grad[:, : d.n].cpu().numpy(), ddc, rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(Mt.grad.cpu().numpy(), dM, rtol=1e-5, atol=1e-6)


def test_loss_l2(R, orc):
    import torch
    y = synth.random_image(5, (72, 128, 3))
    t = synth.random_image(6, (72, 128, 3))
    ty, tt = torch.from_numpy(y).cuda(), torch.from_numpy(t).cuda()
    dl = torch.empty_like(ty)
    loss = torch.empty(1, device="cuda")
    cnt = y.size
    R.recogs_loss_l2(ty.data_ptr(), tt.data_ptr(), cnt, 1.0 / cnt, dl.data_ptr(), loss.data_ptr())
    torch.cuda.synchronize()
    ref_loss = orc.loss_l2(y, t)
    ref_g = orc.loss_l2_grad(y, t)
    assert abs(loss.item() - ref_loss) <= 1e-5 * ref_loss
    np.testing.assert_allclose(dl.cpu().numpy(), ref_g, rtol=1e-6, atol=1e-12)
    # arrays that are not 16-byte aligned (one float in) and a count that is not a
    # multiple of 4 take the element-wise path; the loss is overwritten, not added to
    yf, tf = ty.reshape(-1), tt.reshape(-1)
    dlf = torch.zeros(cnt, device="cuda")
    m = cnt - 2
    R.recogs_loss_l2(yf[1:].data_ptr(), tf[1:].data_ptr(), m, 1.0 / m, dlf[1:].data_ptr(), loss.data_ptr())
    torch.cuda.synchronize()
    y1, t1 = y.reshape(-1)[1:1 + m], t.reshape(-1)[1:1 + m]
    assert abs(loss.item() - orc.loss_l2(y1, t1)) <= 1e-5 * orc.loss_l2(y1, t1)
    np.testing.assert_allclose(dlf[1:1 + m].cpu().numpy(), orc.loss_l2_grad(y1, t1), rtol=1e-6, atol=1e-12)
    assert dlf[0].item() == 0.0 and dlf[1 + m].item() == 0.0


def test_backward_without_recolor_and_zero_gradient(R, orc):
    """No fused recolour: dL/dM is zero and dL/dC0 = Y00 gh; a zero upstream gradient
    gives zero gradients."""
    import torch
    w = _wfd()
    cam = w.view.camera
    d = R.DeviceScene(w.scene)
    ws = R.DeviceWorkspace(w.scene.n, cam.width, cam.height)
    img = R.render(d, cam, ws, keep_backward=True)
    n = d.n
    pr = orc.project(w.scene, cam)
    band = orc.render_image(pr, brute=True).slack > 0
    for gz in (False, True):
        g = np.zeros((cam.height, cam.width, 3), np.float32) if gz else synth.random_image(3, (cam.height, cam.width, 3))
        g = np.where(band[..., None], 0.0, g).astype(np.float32)
        gt = torch.from_numpy(g).cuda()
        dop = torch.empty(n, device="cuda")
        ddc = torch.empty((3, n), device="cuda")
        dM = torch.full((9,), 7.0, device="cuda")
        o = R.opts_struct(keep_backward=True)
        R.recogs_render_backward(d.c_struct(), R.camera_struct(cam), o, ws.ws, img.data_ptr(), gt.data_ptr(),
                                 dop.data_ptr(), ddc.data_ptr(), dM.data_ptr())
        torch.cuda.synchronize()
        assert np.all(dM.cpu().numpy() == 0)
        if gz:
            assert np.all(dop.cpu().numpy() == 0) and np.all(ddc.cpu().numpy() == 0)
        else:
            gr = orc.backward(pr, g)
            _close(ddc.cpu().numpy().astype(np.float64), gr.dc0, "dC0 without recolour")


def test_backward_full_size_on_windows_vs_oracle(R, orc):
    """The differentiation workload at full size (1,000,000 Gaussians, 1280x720, view
    0, the fused recolour M0 on the selection): the upstream gradient is nonzero on
    four 32x32 windows only, so the oracle's backward visits just those pixels."""
    import torch
    w = synth.make_diff()
    v = w.view
    cam = v.camera
    sc = w.scene
    mask, _ = orc.select(sc, cam, v.select)
    M = v.recolor.M.astype(np.float64)
    b = v.recolor.b.astype(np.float64)
    pr = orc.project(sc, cam, (32, 16), mask=mask, M=M, b=b)
    wins = [(320, 192, 32, 32), (640, 352, 32, 32), (96, 608, 32, 32), (1152, 64, 32, 32)]
    ref = orc.render_windows(pr, wins)
    rng = np.random.default_rng(33)
    g = np.zeros((cam.height, cam.width, 3), np.float32)
    o = 0
    for (x0, y0, ww, wh) in wins:
        slack = ref.slack[o:o + ww * wh].reshape(wh, ww)
        blk = rng.standard_normal((wh, ww, 3)).astype(np.float32)
        blk[slack > 0] = 0.0   # in-band threshold decisions get no upstream gradient
        g[y0:y0 + wh, x0:x0 + ww] = blk
        o += ww * wh
    gr = orc.backward(pr, g.astype(np.float64), M=M, windows=wins)
    d = R.DeviceScene(sc)
    ws = R.DeviceWorkspace(sc.n, cam.width, cam.height, (32, 16))
    tm = torch.from_numpy(mask).cuda()
    tM = torch.from_numpy(v.recolor.M.reshape(9).copy()).cuda()
    tb = torch.from_numpy(v.recolor.b.copy()).cuda()
    img, dop, ddc, dM = _gpu_grads(R, d, ws, cam, tm, tM, tb, g, (32, 16), 1, blocks=True)
    e1 = _close(dop, gr.dsigma, "dL/dopacity")
    e2 = _close(ddc, gr.dc0, "dL/dC0")
    e3 = _close(dM, gr.dM, "dL/dM")
    assert np.abs(gr.dsigma).max() > 0 and np.abs(gr.dM).max() > 0
    # every SH coefficient, on the Gaussians the windows reach
    K = (sc.sh_degree + 1) ** 2
    o = R.opts_struct((32, 16), 1, (0, 0, 0), tm, tM, tb, keep_backward=True, bwd_scratch=ws.backward_scratch((32, 16), 1))
    gt = torch.from_numpy(g).cuda()
    dsh = torch.zeros((3 * K, d.stride), device="cuda")
    t1, t9 = torch.empty(sc.n, device="cuda"), torch.empty(9, device="cuda")
    R.recogs_render_backward_sh(d.c_struct(), R.camera_struct(cam), o, ws.ws, img.data_ptr(), gt.data_ptr(),
                                t1.data_ptr(), dsh.data_ptr(), t9.data_ptr())
    torch.cuda.synchronize()
    touched = np.nonzero(np.abs(gr.drgb).sum(axis=1) > 0)[0]
    assert len(touched) > 100
    ref_sh = orc.sh_grad(sc, cam, pr, gr, M=M, idx=touched)
    e4 = _close(dsh[:, touched].cpu().numpy().astype(np.float64), ref_sh, "dL/dSH")
    print(f"full size: relative max errors dsigma {e1:.2e} dC0 {e2:.2e} dM {e3:.2e} dSH {e4:.2e} "
          f"({len(touched)} Gaussians)")


def _views_of_subset(w):
    """The finite-difference subset seen from view 0 and two poses a fifth of a radian
    of azimuth either side (64x64 each)."""
    c = w.view.camera
    cams = [c] + [synth.nearby_orbit(c, d) for d in (-0.2, 0.2)]
    # nearby_orbit keeps the field of view; the subset's camera has its own size
    return cams


def test_backward_accumulates_over_views(R, orc):
    """A loss summed over views: render and backward each view in turn, the first
    overwriting, the others adding (accumulate = 1). The sums equal the sum of the
    oracle's per-view gradients, and equal bit for bit the float32 sums of the
    single-view gradients taken in the same order."""
    import torch
    w = _wfd()
    d, ws, tm, tM, tb, mask, M, b, _ = _setup(R, orc, w)
    M64, b64 = M.astype(np.float64), b.astype(np.float64)
    n = d.n
    acc = [torch.full((n,), 7.0, device="cuda"), torch.full((3, n), 7.0, device="cuda"),
           torch.full((9,), 7.0, device="cuda")]
    single = []
    ref = [np.zeros(n), np.zeros((3, n)), np.zeros((3, 3))]
    for k, cam in enumerate(_views_of_subset(w)):
        pr = orc.project(w.scene, cam, (16, 16), mask=mask, M=M64, b=b64)
        r = orc.render_image(pr, brute=True)
        g = synth.random_image(40 + k, (cam.height, cam.width, 3))
        g = np.where((r.slack > 0)[..., None], 0.0, g).astype(np.float32)
        gr = orc.backward(pr, g, M=M64)
        ref[0] += gr.dsigma
        ref[1] += gr.dc0
        ref[2] += gr.dM
        wsk = R.DeviceWorkspace(n, cam.width, cam.height)
        img = R.render(d, cam, wsk, mask=tm, M=tM, b=tb, keep_backward=True)
        gt = torch.from_numpy(g).cuda()
        o = R.opts_struct((16, 16), 1, (0, 0, 0), tm, tM, tb, keep_backward=True)
        R.recogs_render_backward(d.c_struct(), R.camera_struct(cam), o, wsk.ws, img.data_ptr(), gt.data_ptr(),
                                 acc[0].data_ptr(), acc[1].data_ptr(), acc[2].data_ptr(), 1 if k else 0)
        one = [torch.empty(n, device="cuda"), torch.empty((3, n), device="cuda"), torch.empty(9, device="cuda")]
        R.recogs_render_backward(d.c_struct(), R.camera_struct(cam), o, wsk.ws, img.data_ptr(), gt.data_ptr(),
                                 one[0].data_ptr(), one[1].data_ptr(), one[2].data_ptr(), 0)
        single.append(one)
    torch.cuda.synchronize()
    for j in range(3):
        s = single[0][j].clone()
        for one in single[1:]:
            s = s + one[j]
        assert torch.equal(acc[j], s), j
    e1 = _close(acc[0].cpu().numpy().astype(np.float64), ref[0], "summed dL/dopacity")
    e2 = _close(acc[1].cpu().numpy().astype(np.float64), ref[1], "summed dL/dC0")
    e3 = _close(acc[2].cpu().numpy().astype(np.float64).reshape(3, 3), ref[2], "summed dL/dM")
    assert np.abs(ref[2]).max() > 0
    print(f"3 views: relative max errors dsigma {e1:.2e} dC0 {e2:.2e} dM {e3:.2e}")


def test_backward_sh_accumulates(R, orc):
    """recogs_render_backward_sh with accumulate adds every plane (padding columns untouched)."""
    import torch
    w = _wfd()
    d, ws, tm, tM, tb, mask, M, b, g = _setup(R, orc, w)
    cams = _views_of_subset(w)[:2]
    n, K = d.n, (w.scene.sh_degree + 1) ** 2
    d2 = R.DeviceScene(w.scene, stride=n + 100)
    acc = [torch.full((n + 100,), 3.0, device="cuda"), torch.full((3 * K, n + 100), 3.0, device="cuda"),
           torch.full((9,), 3.0, device="cuda")]
    one = []
    for k, cam in enumerate(cams):
        wsk = R.DeviceWorkspace(n, cam.width, cam.height)
        img = R.render(d2, cam, wsk, mask=tm, M=tM, b=tb, keep_backward=True)
        gt = torch.from_numpy(synth.random_image(50 + k, (cam.height, cam.width, 3))).cuda()
        o = R.opts_struct((16, 16), 1, (0, 0, 0), tm, tM, tb, keep_backward=True)
        R.recogs_render_backward_sh(d2.c_struct(), R.camera_struct(cam), o, wsk.ws, img.data_ptr(), gt.data_ptr(),
                                    acc[0].data_ptr(), acc[1].data_ptr(), acc[2].data_ptr(), 1)
        x = [torch.empty(n, device="cuda"), torch.zeros((3 * K, n + 100), device="cuda"), torch.empty(9, device="cuda")]
        R.recogs_render_backward_sh(d2.c_struct(), R.camera_struct(cam), o, wsk.ws, img.data_ptr(), gt.data_ptr(),
                                    x[0].data_ptr(), x[1].data_ptr(), x[2].data_ptr(), 0)
        one.append(x)
    torch.cuda.synchronize()
    assert torch.equal(acc[0][:n], (3.0 + one[0][0]) + one[1][0])
    assert torch.equal(acc[1][:, :n], (3.0 + one[0][1][:, :n]) + one[1][1][:, :n])
    assert torch.equal(acc[2], (3.0 + one[0][2]) + one[1][2])
    assert torch.all(acc[1][:, n:] == 3.0) and torch.all(acc[0][n:] == 3.0)


def test_autograd_refuses_a_workspace_that_rendered_again(R, orc):
    """The backward replays its workspace's per-tile state: a second forward on the same
    workspace makes the first one's backward raise; separate workspaces give the summed
    gradients of the two views."""
    import torch
    w = _wfd()
    d, ws, tm, tM, tb, mask, M, b, g = _setup(R, orc, w)
    cams = _views_of_subset(w)[:2]
    gts = [torch.from_numpy(synth.random_image(60 + k, (c.height, c.width, 3))).cuda() for k, c in enumerate(cams)]
    op = torch.nn.Parameter(d.opacity, requires_grad=True)
    leaf_dc = torch.nn.Parameter(d.sh.narrow(0, 0, 3), requires_grad=True)
    Mt = torch.from_numpy(M.copy()).cuda().requires_grad_(True)
    shared = R.DeviceWorkspace(d.n, cams[0].width, cams[0].height)
    img0 = R.RecogsRenderFn.apply(op, leaf_dc, Mt, d, cams[0], shared, tm, tb)
    img1 = R.RecogsRenderFn.apply(op, leaf_dc, Mt, d, cams[1], shared, tm, tb)
    with pytest.raises(RuntimeError, match="rendered again"):
        ((img0 * gts[0]).sum() + (img1 * gts[1]).sum()).backward()
    op.grad = leaf_dc.grad = Mt.grad = None
    wss = [R.DeviceWorkspace(d.n, c.width, c.height) for c in cams]
    imgs = [R.RecogsRenderFn.apply(op, leaf_dc, Mt, d, c, wk, tm, tb) for c, wk in zip(cams, wss)]
    (sum((im * gt).sum() for im, gt in zip(imgs, gts))).backward()
    ref = [torch.zeros(d.n, device="cuda"), torch.zeros((3, d.n), device="cuda"), torch.zeros(9, device="cuda")]
    for k, cam in enumerate(cams):
        wsk = R.DeviceWorkspace(d.n, cam.width, cam.height)
        img = R.render(d, cam, wsk, mask=tm, M=tM, b=tb, keep_backward=True)
        o = R.opts_struct((16, 16), 1, (0, 0, 0), tm, tM, tb, keep_backward=True)
        R.recogs_render_backward(d.c_struct(), R.camera_struct(cam), o, wsk.ws, img.data_ptr(), gts[k].data_ptr(),
                                 ref[0].data_ptr(), ref[1].data_ptr(), ref[2].data_ptr(), 1 if k else 0)
    torch.cuda.synchronize()
    np.testing.assert_allclose(op.grad[: d.n].cpu().numpy(), ref[0].cpu().numpy(), rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(leaf_dc.grad[:, : d.n].cpu().numpy(), ref[1].cpu().numpy(), rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(Mt.grad.reshape(9).cpu().numpy(), ref[2].cpu().numpy(), rtol=1e-5, atol=1e-6)


def test_backward_full_size_eight_views_accumulated(R, orc):
    """The differentiation workload at full size (1,000,000 Gaussians, 8 views at
    1280x720, fused recolour M0 on view 0's selection): the upstream gradient of each
    view is nonzero on one 32x32 window; the accumulated dsigma, dC0 and dM equal the sum
    of the oracle's windowed per-view gradients."""
    import torch
    w = synth.make_diff()
    sc = w.scene
    v0 = w.views[0]
    mask, _ = orc.select(sc, v0.camera, v0.select)
    M = v0.recolor.M.astype(np.float64)
    b = v0.recolor.b.astype(np.float64)
    d = R.DeviceScene(sc)
    tm = torch.from_numpy(mask).cuda()
    tM = torch.from_numpy(v0.recolor.M.reshape(9).copy()).cuda()
    tb = torch.from_numpy(v0.recolor.b.copy()).cuda()
    tile = (32, 16)
    n = sc.n
    acc = [torch.empty(n, device="cuda"), torch.empty((3, n), device="cuda"), torch.empty(9, device="cuda")]
    ref = [np.zeros(n), np.zeros((3, n)), np.zeros((3, 3))]
    rng = np.random.default_rng(71)
    for k, v in enumerate(w.views):
        cam = v.camera
        pr = orc.project(sc, cam, tile, mask=mask, M=M, b=b)
        win = [(int(rng.integers(0, cam.width - 32)), int(rng.integers(0, cam.height - 32)), 32, 32)]
        r = orc.render_windows(pr, win)
        x0, y0 = win[0][:2]
        g = np.zeros((cam.height, cam.width, 3), np.float32)
        blk = rng.standard_normal((32, 32, 3)).astype(np.float32)
        blk[r.slack.reshape(32, 32) > 0] = 0.0
        g[y0:y0 + 32, x0:x0 + 32] = blk
        gr = orc.backward(pr, g.astype(np.float64), M=M, windows=win)
        ref[0] += gr.dsigma
        ref[1] += gr.dc0
        ref[2] += gr.dM
        ws = R.DeviceWorkspace(n, cam.width, cam.height, tile)
        img = R.render(d, cam, ws, tile, 1, mask=tm, M=tM, b=tb, keep_backward=True)
        o = R.opts_struct(tile, 1, (0, 0, 0), tm, tM, tb, keep_backward=True, bwd_scratch=ws.backward_scratch(tile, 1))
        gt = torch.from_numpy(g).cuda()
        R.recogs_render_backward(d.c_struct(), R.camera_struct(cam), o, ws.ws, img.data_ptr(), gt.data_ptr(),
                                 acc[0].data_ptr(), acc[1].data_ptr(), acc[2].data_ptr(), 1 if k else 0)
        torch.cuda.synchronize()
        del ws
    e1 = _close(acc[0].cpu().numpy().astype(np.float64), ref[0], "8-view dL/dopacity")
    e2 = _close(acc[1].cpu().numpy().astype(np.float64), ref[1], "8-view dL/dC0")
    e3 = _close(acc[2].cpu().numpy().astype(np.float64).reshape(3, 3), ref[2], "8-view dL/dM")
    assert np.abs(ref[0]).max() > 0 and np.abs(ref[2]).max() > 0
    print(f"8 views full size: relative max errors dsigma {e1:.2e} dC0 {e2:.2e} dM {e3:.2e}")


def test_backward_central_differences_h1e3(R, orc):
    """Central differences with step 1e-3 of the GPU's own float32 forward, L = sum(g y)
    on the 4,096-Gaussian 64x64 subset with the fused recolour: every entry of M, 256
    seeded DC coefficients and 256 seeded opacities (Sec. 4.1, eq. 8).

    The image is linear in each of these parameters between discrete decisions (the
    colour is linear in M and C0; alpha, and then y, is linear in one opacity), so the
    difference quotient has no truncation error: it differs from the gradient only by the
    float32 rounding of the two renders. Stencils whose two sides take any decision
    differently (a colour clamp, an alpha crossing 1/255 or 0.99, a pixel stopping at
    another splat) are excluded and counted. Tolerance per stencil: 16 float32 ulps of
    rounding per pixel value, added in quadrature over the pixels the stencil changes,
    divided by the step, plus 1e-4 of the gradient."""
    import torch
    w = _wfd()
    cam = w.view.camera
    d, ws, tm, tM, tb, mask, M, b, g = _setup(R, orc, w)
    M64, b64 = M.astype(np.float64), b.astype(np.float64)
    _, dop, ddc, dM = _gpu_grads(R, d, ws, cam, tm, tM, tb, g)
    pr = orc.project(w.scene, cam, (16, 16), mask=mask, M=M64, b=b64)
    gt = torch.from_numpy(g).cuda().double()
    g2 = torch.from_numpy(g.astype(np.float64) ** 2).cuda()
    h = 1e-3
    ulp = 2.0 ** -23

    def run():
        img = R.render(d, cam, ws, mask=tm, M=tM, b=tb, keep_backward=True)
        return img.double(), ws.nproc().clone()

    def quotient(set_plus, set_minus, restore):
        set_plus()
        yp, npp = run()
        set_minus()
        ym, npm = run()
        restore()
        step = yp - ym
        changed = (step != 0)
        noise = 16 * ulp * torch.sqrt((g2 * (yp * yp + ym * ym) * changed).sum()).item()
        return float((step * gt).sum().item()), noise, bool(torch.equal(npp, npm))

    pre = np.stack([pr.col("pr"), pr.col("pg"), pr.col("pb")], 1)
    f = np.stack([pr.col("fr"), pr.col("fg"), pr.col("fb")], 1)
    vis = pr.col("count") > 0
    sel = (pr.col("sel") == 1) & vis
    checked = excluded = 0
    worst = 0.0

    def check(grad, num, span, noise, same_stops, flips, what):
        nonlocal checked, excluded, worst
        if flips or not same_stops:
            excluded += 1
            return
        fd = num / span
        tol = noise / span + 1e-4 * abs(grad) + 1e-9
        assert abs(fd - grad) <= tol, (what, fd, grad, tol)
        checked += 1
        worst = max(worst, abs(fd - grad) / tol)

    # M (device float32 [9]); a clamp flips where a selected splat's pre-clamp colour crosses 0
    Mv = tM.clone()
    for k in range(9):
        r, c = divmod(k, 3)
        hp = float(np.float32(M.flat[k] + h)) - float(M.flat[k])
        hm = float(np.float32(M.flat[k] - h)) - float(M.flat[k])

        def sp(k=k, hp=hp):
            tM[k] = Mv[k] + hp

        def sm(k=k, hm=hm):
            tM[k] = Mv[k] + hm

        def rs():
            tM.copy_(Mv)
        num, noise, same = quotient(sp, sm, rs)
        flips = np.any(np.sign(pre[sel, r] + hp * f[sel, c]) != np.sign(pre[sel, r] + hm * f[sel, c]))
        check(dM.flat[k], num, hp - hm, noise, same, flips, f"M[{k}]")
    # DC coefficients (float32 planes 0..2 of the SH array)
    rng = np.random.default_rng(81)
    idx = np.nonzero(vis)[0]
    Y00 = 0.28209479177387814
    for i, c in zip(rng.choice(idx, 256, replace=False), rng.integers(0, 3, 256)):
        x0 = float(d.sh[c, i].item())
        hp, hm = float(np.float32(x0 + h)) - x0, float(np.float32(x0 - h)) - x0

        def sp(i=i, c=c, v=x0 + hp):
            d.sh[c, i] = v

        def sm(i=i, c=c, v=x0 + hm):
            d.sh[c, i] = v

        def rs(i=i, c=c, v=x0):
            d.sh[c, i] = v
        num, noise, same = quotient(sp, sm, rs)
        col = (M64[:, c] if sel[i] else np.eye(3)[c]) * Y00
        flips = np.any(np.sign(pre[i] + hp * col) != np.sign(pre[i] + hm * col))
        check(ddc[c, i], num, hp - hm, noise, same, flips, f"C0[{c}, {i}]")
    # opacities: alpha = sigma G(p) at every pixel centre crosses neither 1/255 nor 0.99
    yy, xx = np.mgrid[0:cam.height, 0:cam.width] + 0.5
    cand = idx[(pr.col("sigma")[idx] > 2 * h) & (pr.col("sigma")[idx] < 1 - 2 * h)]
    for i in rng.choice(cand, 256, replace=False):
        x0 = float(d.opacity[i].item())
        hp, hm = float(np.float32(x0 + h)) - x0, float(np.float32(x0 - h)) - x0
        dx, dy = xx - pr.col("u")[i], yy - pr.col("v")[i]
        G = np.exp(-0.5 * (pr.col("ca")[i] * dx * dx + 2 * pr.col("cb")[i] * dx * dy + pr.col("cc")[i] * dy * dy))
        ap, am = (x0 + hp) * G, (x0 + hm) * G
        flips = bool(np.any((ap >= 1 / 255) != (am >= 1 / 255)) or np.any((ap >= 0.99) != (am >= 0.99)))

        def sp(i=i, v=x0 + hp):
            d.opacity[i] = v

        def sm(i=i, v=x0 + hm):
            d.opacity[i] = v

        def rs(i=i, v=x0):
            d.opacity[i] = v
        num, noise, same = quotient(sp, sm, rs)
        check(dop[i], num, hp - hm, noise, same, flips, f"sigma[{i}]")
    total = checked + excluded
    assert total == 9 + 256 + 256 and excluded <= 0.1 * total, (checked, excluded)
    print(f"central differences (h = 1e-3): {checked} stencils within tolerance (worst at {worst:.2f} of it), "
          f"{excluded} excluded for a decision flip")
