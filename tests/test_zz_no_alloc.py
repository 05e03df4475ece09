"""recogs_unproject_noalloc, the unprojection for callers that cannot allocate, against
recogs_unproject (its workspace form) on the same inputs: two calls in a row, the second
on a smaller image, each equal bit for bit in count and points."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import paper_2511_18441_amd as R
    return R


def _inputs(seed, W, H):
    rng = np.random.default_rng(seed)
    cam = synth.orbit_camera(W, H, 60.0, 4.0, rng.uniform(0, 6.28), rng.uniform(0.2, 0.6))
    mask = synth.brush_mask(W, H, W * rng.uniform(0.3, 0.7), H * rng.uniform(0.3, 0.7), 0.3 * min(W, H))
    keep = synth.sample_keep(seed + 1, mask)
    depth = rng.uniform(1.0, 6.0, size=(H, W)).astype(np.float32)
    depth[rng.random((H, W)) < 0.15] = 0.0
    return cam, mask, keep, depth


def _run(R, cam, mask, keep, depth, noalloc):
    import torch
    tm, tk, td = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (mask, keep, depth))
    cap = int(mask.sum())
    pts = torch.full((3, max(cap, 1)), -1.0, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    c = R.camera_struct(cam)
    if noalloc:
        R.recogs_unproject_noalloc(c, tm.data_ptr(), tk.data_ptr(), td.data_ptr(), pts.data_ptr(), cap, cnt.data_ptr())
    else:
        nb = R.recogs_unproject_workspace_bytes(cam.width, cam.height)
        ws = torch.empty(nb // 4 + 1, dtype=torch.int32, device="cuda")
        R.recogs_unproject(c, tm.data_ptr(), tk.data_ptr(), td.data_ptr(), pts.data_ptr(), cap, cnt.data_ptr(),
                           ws.data_ptr(), nb)
    torch.cuda.synchronize()
    return int(cnt.item()), pts.cpu().numpy()


def test_noalloc_unprojection_equals_the_workspace_form(R):
    for seed, (W, H) in [(5, (1920, 1080)), (6, (333, 201))]:   # the second call is smaller
        cam, mask, keep, depth = _inputs(seed, W, H)
        n0, p0 = _run(R, cam, mask, keep, depth, noalloc=False)
        n1, p1 = _run(R, cam, mask, keep, depth, noalloc=True)
        assert n0 == n1 and n0 > 1000, (W, H, n0, n1)
        assert np.array_equal(p0, p1), (W, H)
        print(f"{W}x{H}: {n1} points, same bits as recogs_unproject")


def test_noalloc_unprojection_refuses_images_beyond_its_scratch(R):
    cam = synth.orbit_camera(8193, 8192, 60.0, 4.0, 0.0, 0.3)
    with pytest.raises(R.RecogsError) as e:
        R.recogs_unproject_noalloc(R.camera_struct(cam), 256, 0, 256, 256, 10, 256)
    assert e.value.status == -1 and "scratch" in R.recogs_last_error()
