"""Pieces of the background optimiser (Sec. 3.3 / 4.1) through the C ABI: the gradient
of every SH coefficient, the L1 and SSIM terms of eq. 4 and the Adam step, against the FP64
oracle (pinned on the CPU by central differences and closed forms); then a few steps of
SH-only refitting toward a recoloured target, which must lower the loss."""
import numpy as np
import pytest

import synth
from tests.test_gpu_backward import _close, _setup, _wfd

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import paper_2511_18441_amd as R
    return R


@pytest.mark.parametrize("tile,ppt", [((16, 16), 1), ((32, 16), 1)])
def test_backward_sh_vs_oracle(R, orc, tile, ppt):
    import torch
    w = _wfd()
    cam = w.view.camera
    d, ws, tm, tM, tb, mask, M, b, g = _setup(R, orc, w)
    pr = orc.project(w.scene, cam, tile, mask=mask, M=M.astype(np.float64), b=b.astype(np.float64))
    ref = orc.render_image(pr, brute=True)
    g = np.where((ref.slack > 0)[..., None], 0.0, g).astype(np.float32)
    ws = R.DeviceWorkspace(w.scene.n, cam.width, cam.height, tile)
    img = R.render(d, cam, ws, tile, ppt, mask=tm, M=tM, b=tb, keep_backward=True)
    gt = torch.from_numpy(g).cuda()
    n, K = d.n, (w.scene.sh_degree + 1) ** 2
    o = R.opts_struct(tile, ppt, (0, 0, 0), tm, tM, tb, keep_backward=True)
    dop, dsh, dM = torch.empty(n, device="cuda"), torch.full((3 * K, d.stride), 7.0, device="cuda"), torch.empty(9, device="cuda")
    R.recogs_render_backward_sh(d.c_struct(), R.camera_struct(cam), o, ws.ws, img.data_ptr(), gt.data_ptr(),
                                dop.data_ptr(), dsh.data_ptr(), dM.data_ptr())
    dop2, ddc, dM2 = torch.empty(n, device="cuda"), torch.empty((3, n), device="cuda"), torch.empty(9, device="cuda")
    R.recogs_render_backward(d.c_struct(), R.camera_struct(cam), o, ws.ws, img.data_ptr(), gt.data_ptr(),
                             dop2.data_ptr(), ddc.data_ptr(), dM2.data_ptr())
    torch.cuda.synchronize()
    # the DC planes, the opacity and M gradients are those of recogs_render_backward, bit for bit
    assert torch.equal(dsh[0:3, :n], ddc) and torch.equal(dop, dop2) and torch.equal(dM, dM2)
    gr = orc.backward(pr, g, M=M.astype(np.float64))
    ref_sh = orc.sh_grad(w.scene, cam, pr, gr, M=M.astype(np.float64))
    got = dsh[:, :n].cpu().numpy().astype(np.float64)
    assert np.isfinite(got).all()
    e = _close(got, ref_sh, "dL/dSH")
    print(f"{tile} ppt {ppt}: dL/dSH rel max err {e:.2e}")


def test_backward_sh_adam_fused_equals_the_two_calls(R, orc):
    """recogs_render_backward_sh_adam gives the bits of recogs_render_backward_sh followed by
    recogs_adam_step on the SH planes, over three steps (with the fused recolour, and a
    plane stride above n whose extra columns stay untouched)."""
    import torch
    w = _wfd()
    cam = w.view.camera
    d, ws, tm, tM, tb, mask, M, b, g = _setup(R, orc, w)
    gt = torch.from_numpy(np.asarray(g, np.float32)).cuda()
    n, K = d.n, (w.scene.sh_degree + 1) ** 2
    o = R.opts_struct((32, 16), 1, (0, 0, 0), tm, tM, tb, keep_backward=True)
    ws = R.DeviceWorkspace(n, cam.width, cam.height, (32, 16))
    d = R.DeviceScene(w.scene, stride=n + 29)          # every plane with 29 spare columns
    base = d.sh.clone()
    base[:, n:] = 0.25                                  # spare columns: must stay as they are
    sh_a, sh_b = base.clone(), base.clone()
    ma, va, mb, vb = (torch.zeros_like(base) for _ in range(4))
    dsh = torch.zeros_like(base)
    dop_a, dop_b = torch.empty(n, device="cuda"), torch.empty(n, device="cuda")
    dM_a, dM_b = torch.empty(9, device="cuda"), torch.empty(9, device="cuda")

    def scene(sh):
        return d.c_struct(sh)
    for step in (1, 2, 3):
        sa = scene(sh_a)
        img = R.render(d, cam, ws, (32, 16), 1, mask=tm, M=tM, b=tb, keep_backward=True, sh=sh_a)
        R.recogs_render_backward_sh(sa, R.camera_struct(cam), o, ws.ws, img.data_ptr(), gt.data_ptr(), dop_a.data_ptr(),
                                    dsh.data_ptr(), dM_a.data_ptr())
        R.recogs_adam_step(sh_a.data_ptr(), dsh.data_ptr(), ma.data_ptr(), va.data_ptr(), sh_a.numel(), 2e-3, step=step)
        sb = scene(sh_b)
        img_b = R.render(d, cam, ws, (32, 16), 1, mask=tm, M=tM, b=tb, keep_backward=True, sh=sh_b)
        assert torch.equal(img, img_b)
        R.recogs_render_backward_sh_adam(sb, R.camera_struct(cam), o, ws.ws, img_b.data_ptr(), gt.data_ptr(),
                                         dop_b.data_ptr(), dM_b.data_ptr(), mb.data_ptr(), vb.data_ptr(), 2e-3,
                                         step=step)
        torch.cuda.synchronize()
        # the separate Adam call also steps the spare columns (with a zero gradient from
        # zero moments: no change), the fused one skips them
        assert torch.equal(sh_a, sh_b) and torch.equal(ma, mb) and torch.equal(va, vb), step
        assert torch.equal(dop_a, dop_b) and torch.equal(dM_a, dM_b), step
    assert torch.equal(sh_b[:, n:], base[:, n:])
    assert not torch.equal(sh_b[:, :n], base[:, :n])
    bad = d.c_struct()
    bad.storage = 1
    with pytest.raises(R.RecogsError) as e:
        R.recogs_render_backward_sh_adam(bad, R.camera_struct(cam), o, ws.ws, img_b.data_ptr(), gt.data_ptr(),
                                         dop_b.data_ptr(), dM_b.data_ptr(), mb.data_ptr(), vb.data_ptr(), 2e-3, step=1)
    assert e.value.status == -3


def test_loss_l1_vs_oracle(R, orc):
    import torch
    y = synth.random_image(7, (72, 128, 3))
    t = synth.random_image(8, (72, 128, 3))
    ty, tt = torch.from_numpy(y).cuda().reshape(-1), torch.from_numpy(t).cuda().reshape(-1)
    cnt = y.size
    loss = torch.empty(1, device="cuda")
    for off, m in ((0, cnt), (1, cnt - 2)):   # 16-byte aligned, then one float in with a ragged count
        dl = torch.zeros(cnt, device="cuda")
        R.recogs_loss_l1(ty[off:].data_ptr(), tt[off:].data_ptr(), m, 1.0 / m, dl[off:].data_ptr(), loss.data_ptr())
        torch.cuda.synchronize()
        y1, t1 = y.reshape(-1)[off:off + m], t.reshape(-1)[off:off + m]
        assert abs(loss.item() - orc.loss_l1(y1, t1)) <= 1e-5 * orc.loss_l1(y1, t1)
        np.testing.assert_allclose(dl[off:off + m].cpu().numpy(), orc.loss_l1_grad(y1, t1), rtol=1e-6, atol=0)


@pytest.mark.parametrize("H,W", [(72, 128), (37, 50)])
def test_dssim_vs_oracle(R, orc, H, W):
    """The SSIM term of eq. 4 and its gradient (written, then accumulated onto an L1
    gradient as eq. 7 combines them), on images whose size is not a multiple of the
    kernels' 16 x 16 tiles."""
    import torch
    y = synth.random_image(9, (H, W, 3))
    t = (0.7 * y + 0.3 * synth.random_image(10, (H, W, 3))).astype(np.float32)   # correlated, as a target is
    ty, tt = torch.from_numpy(y).cuda(), torch.from_numpy(t).cuda()
    nb = R.recogs_dssim_workspace_bytes(W, H)
    ws = torch.empty(nb // 4, device="cuda")
    lam = 0.2
    loss = torch.empty(1, device="cuda")
    dl = torch.full_like(ty, 5.0)
    R.recogs_loss_dssim(ty.data_ptr(), tt.data_ptr(), W, H, lam, dl.data_ptr(), 0, loss.data_ptr(), ws.data_ptr(), nb)
    torch.cuda.synchronize()
    val, g = orc.ssim(y, t)
    assert abs(loss.item() - lam * (1.0 - val)) <= 1e-5
    e = _close(dl.cpu().numpy().astype(np.float64), -lam * g, "dL/dy (SSIM)")
    # the loss is summed in a fixed order: the same bits again (the workspace holding the
    # previous call's partial sums), and the gradient too
    loss2 = torch.empty(1, device="cuda")
    dl2 = torch.empty_like(ty)
    R.recogs_loss_dssim(ty.data_ptr(), tt.data_ptr(), W, H, lam, dl2.data_ptr(), 0, loss2.data_ptr(), ws.data_ptr(), nb)
    torch.cuda.synchronize()
    assert loss2.cpu().numpy().tobytes() == loss.cpu().numpy().tobytes()
    assert torch.equal(dl2, dl)
    # eq. 4: (1 - lambda) L1 + lambda (1 - SSIM); eq. 7: the SSIM gradient added to the L1 one
    n = y.size
    l1 = torch.empty(1, device="cuda")
    R.recogs_loss_l1(ty.data_ptr(), tt.data_ptr(), n, (1 - lam) / n, dl.data_ptr(), l1.data_ptr())
    R.recogs_loss_dssim(ty.data_ptr(), tt.data_ptr(), W, H, lam, dl.data_ptr(), 1, loss.data_ptr(), ws.data_ptr(), nb)
    torch.cuda.synchronize()
    ref = (1 - lam) * orc.loss_l1_grad(y, t) - lam * g
    e2 = _close(dl.cpu().numpy().astype(np.float64), ref, "dL/dy (eq. 7)")
    assert abs(l1.item() - (1 - lam) * orc.loss_l1(y, t)) <= 1e-5
    print(f"{H}x{W}: SSIM {val:.6f}, gradient rel err {e:.2e}, eq. 7 gradient rel err {e2:.2e}")
    # both terms in one pass: the two calls' gradient bits, written or added; the loss
    # against the oracle, and the same bits on every run (both sums in a fixed order)
    dlf = torch.empty_like(ty)
    lf = torch.empty(1, device="cuda")
    R.recogs_loss_l1_dssim(ty.data_ptr(), tt.data_ptr(), W, H, (1 - lam) / n, lam, dlf.data_ptr(), 0, lf.data_ptr(),
                           ws.data_ptr(), nb)
    torch.cuda.synchronize()
    assert torch.equal(dlf, dl)
    assert abs(lf.item() - ((1 - lam) * orc.loss_l1(y, t) + lam * (1.0 - val))) <= 1e-5
    lf2 = torch.empty(1, device="cuda")
    dacc = torch.full_like(ty, 0.25)
    R.recogs_loss_l1_dssim(ty.data_ptr(), tt.data_ptr(), W, H, (1 - lam) / n, lam, dacc.data_ptr(), 1, lf2.data_ptr(),
                           ws.data_ptr(), nb)
    torch.cuda.synchronize()
    assert lf2.cpu().numpy().tobytes() == lf.cpu().numpy().tobytes()
    assert torch.equal(dacc, torch.full_like(ty, 0.25) + dlf)


def test_adam_vector_and_scalar_paths_agree(R):
    """16-byte-aligned arrays take the four-per-thread path (with a scalar tail),
    misaligned ones the scalar path: the per-value arithmetic, and so the bits, agree."""
    import torch
    rng = np.random.default_rng(4)
    n = 1031
    p0, g0 = rng.standard_normal(n).astype(np.float32), rng.standard_normal(n).astype(np.float32)
    outs = []
    for off in (0, 1):
        buf = [torch.zeros(n + 1, device="cuda") for _ in range(4)]
        p, g, m, v = (b[off:off + n] for b in buf)
        p.copy_(torch.from_numpy(p0))
        g.copy_(torch.from_numpy(g0))
        for step in (1, 2, 3):
            R.recogs_adam_step(p.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(), n, 1e-3, 0.9, 0.999, 1e-15, step)
        outs.append([t.cpu().numpy() for t in (p, m, v)])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_adam_vs_oracle(R, orc):
    import torch
    rng = np.random.default_rng(3)
    n = 100_003
    p0 = rng.standard_normal(n).astype(np.float32)
    p, m, v = torch.from_numpy(p0).cuda(), torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    rp, rm, rv = p0.astype(np.float64), np.zeros(n), np.zeros(n)
    mabs = np.zeros(n)   # the same recurrence over |g|: the scale of m's float32 rounding
    for step in range(1, 6):
        g = (rng.standard_normal(n) * 10.0 ** rng.integers(-3, 1, n)).astype(np.float32)
        R.recogs_adam_step(p.data_ptr(), torch.from_numpy(g).cuda().data_ptr(), m.data_ptr(), v.data_ptr(), n, 1e-3,
                           0.9, 0.999, 1e-15, step)
        # the same hyperparameter values the C ABI receives (float32)
        f = lambda x: float(np.float32(x))  # noqa: E731
        rp, rm, rv = orc.adam_step(rp, g, rm, rv, step, f(1e-3), f(0.9), f(0.999), f(1e-15))
        mabs = 0.9 * mabs + 0.1 * np.abs(g.astype(np.float64))
    torch.cuda.synchronize()
    np.testing.assert_allclose(p.cpu().numpy(), rp, rtol=0, atol=2e-6)
    # m can cancel to near zero: bound its error by a few float32 ulps of the terms' magnitude
    assert np.all(np.abs(m.cpu().numpy() - rm) <= 1e-6 * mabs + 1e-12)
    np.testing.assert_allclose(v.cpu().numpy(), rv, rtol=1e-5, atol=0)
    with pytest.raises(R.RecogsError):
        R.recogs_adam_step(p.data_ptr(), p.data_ptr(), m.data_ptr(), v.data_ptr(), n, 1e-3, step=0)


def test_sh_refit_lowers_the_l1_loss(R, orc):
    """SH-only refitting (geometry frozen, Sec. 3.3): the target is the same view with
    the selection recoloured by another matrix; Adam steps on the SH coefficients
    driven by the loss of eq. 4 must bring the render toward it (L1 distance tracked)."""
    import torch
    w = _wfd()
    cam = w.view.camera
    d, ws, tm, tM, tb, mask, M, b, g = _setup(R, orc, w)
    Mt = torch.from_numpy(w.extra["M_target"].reshape(9).copy()).cuda()
    target = R.render(d, cam, ws, mask=tm, M=Mt, b=tb).clone()
    n, K = d.n, (w.scene.sh_degree + 1) ** 2
    sh = d.sh.clone()                       # the coefficients being refitted (f32 planes)
    m, v = torch.zeros_like(sh), torch.zeros_like(sh)
    dl, loss = torch.empty_like(target), torch.empty(1, device="cuda")
    dop, dsh, dM = torch.empty(n, device="cuda"), torch.zeros((3 * K, d.stride), device="cuda"), torch.empty(9, device="cuda")
    o = R.opts_struct((16, 16), 1, keep_backward=True)
    cnt = target.numel()
    losses = []
    lam = 0.2
    nb = R.recogs_dssim_workspace_bytes(cam.width, cam.height)
    sws = torch.empty(nb // 4, device="cuda")
    ls = torch.empty(1, device="cuda")
    for step in range(1, 31):
        img = R.render(d, cam, ws, keep_backward=True, sh=sh)
        # eq. 4: (1 - lambda) L1 + lambda (1 - SSIM)
        R.recogs_loss_l1(img.data_ptr(), target.data_ptr(), cnt, 1.0 / cnt, dl.data_ptr(), loss.data_ptr())
        R.recogs_loss_l1(img.data_ptr(), target.data_ptr(), cnt, (1 - lam) / cnt, dl.data_ptr(), ls.data_ptr())
        R.recogs_loss_dssim(img.data_ptr(), target.data_ptr(), cam.width, cam.height, lam, dl.data_ptr(), 1,
                            ls.data_ptr(), sws.data_ptr(), nb)
        R.recogs_render_backward_sh(d.c_struct(sh), R.camera_struct(cam), o, ws.ws, img.data_ptr(), dl.data_ptr(),
                                    dop.data_ptr(), dsh.data_ptr(), dM.data_ptr())
        R.recogs_adam_step(sh.data_ptr(), dsh.data_ptr(), m.data_ptr(), v.data_ptr(), sh.numel(), 2e-3, step=step)
        losses.append(loss.item())
    print("L1 loss over the refit:", [round(x, 5) for x in losses[::5]], round(losses[-1], 5))
    assert losses[-1] < 0.5 * losses[0]


def test_backward_sh_adam_fused_at_full_size(R):
    """The benchmarked refit step's size (1M Gaussians, SH degree 3, 1280x720, 32x16 tiles,
    1 px/thread): the fused step and the two calls agree bit for bit over two steps."""
    import torch
    w = synth.make_diff()
    v0 = w.views[0]
    cam = v0.camera
    d = R.DeviceScene(w.scene)
    n = d.n
    ws = R.DeviceWorkspace(n, cam.width, cam.height, (32, 16))
    o = R.opts_struct((32, 16), 1, keep_backward=True)
    H, W = cam.height, cam.width
    target = torch.from_numpy(synth.random_image(61, (H, W, 3), 0.5) + np.float32(0.5)).cuda()
    dimg = torch.empty((H, W, 3), device="cuda")
    loss = torch.empty(1, device="cuda")
    sh_a, sh_b = d.sh.clone(), d.sh.clone()
    ma, va, mb, vb = (torch.zeros_like(sh_a) for _ in range(4))
    dsh = torch.zeros_like(sh_a)
    dop, dM = torch.empty(n, device="cuda"), torch.empty(9, device="cuda")
    for step in (1, 2):
        for sh, fused in ((sh_a, False), (sh_b, True)):
            img = R.render(d, cam, ws, (32, 16), 1, keep_backward=True, sh=sh)
            R.recogs_loss_l1(img.data_ptr(), target.data_ptr(), img.numel(), 1.0 / img.numel(), dimg.data_ptr(),
                             loss.data_ptr())
            if fused:
                R.recogs_render_backward_sh_adam(d.c_struct(sh), R.camera_struct(cam), o, ws.ws, img.data_ptr(),
                                                 dimg.data_ptr(), dop.data_ptr(), dM.data_ptr(), mb.data_ptr(),
                                                 vb.data_ptr(), 2e-3, step=step)
            else:
                R.recogs_render_backward_sh(d.c_struct(sh), R.camera_struct(cam), o, ws.ws, img.data_ptr(),
                                            dimg.data_ptr(), dop.data_ptr(), dsh.data_ptr(), dM.data_ptr())
                R.recogs_adam_step(sh.data_ptr(), dsh.data_ptr(), ma.data_ptr(), va.data_ptr(), sh.numel(), 2e-3,
                                   step=step)
        torch.cuda.synchronize()
        assert torch.equal(sh_a, sh_b) and torch.equal(ma, mb) and torch.equal(va, vb), step
    assert not torch.equal(sh_a, d.sh)
