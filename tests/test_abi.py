"""The C-ABI library: exports, struct layout and host-side argument errors (no GPU)."""
import ctypes
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "recogs.h")


@pytest.fixture(scope="module")
def R():
    import paper_2511_18441_amd as R
    return R


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(recogs_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_function_is_exported(R):
    names = declared_functions()
    assert len(names) >= 12
    out = subprocess.run(["nm", "-D", "--defined-only", R.binding.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r" T (recogs_[a-z0-9_]+)", out))
    assert set(names) <= exported, set(names) - exported
    assert set(R.ENTRY_POINTS) | set(R.BATCH_ENTRY_POINTS) == set(names)


PROBE = r"""
#include <stddef.h>
#include <stdio.h>
#include "recogs.h"
#define S(T) printf(#T " %zu\n", sizeof(T));
#define O(T, f) printf(#T "." #f " %zu\n", offsetof(T, f));
int main(void) {
  S(recogs_scene) S(recogs_camera) S(recogs_select_params) S(recogs_render_opts) S(recogs_workspace)
  S(recogs_batch_view) S(recogs_batch_workspace)
  O(recogs_render_opts, mask) O(recogs_render_opts, sort_mode) O(recogs_render_opts, depth_map)
  O(recogs_render_opts, depth_tau) O(recogs_render_opts, extent_rule) O(recogs_render_opts, bwd_scratch)
  O(recogs_render_opts, bwd_scratch_bytes)
  O(recogs_workspace, off_rec) O(recogs_workspace, num_keys) O(recogs_workspace, stage_ms)
  O(recogs_workspace, generation)
  O(recogs_batch_workspace, pairs) O(recogs_batch_workspace, off_views) O(recogs_batch_workspace, num_keys)
  O(recogs_batch_view, image)
  return 0;
}
"""


def test_struct_layout_matches_binding(R):
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "probe.c")
        exe = os.path.join(d, "probe")
        open(src, "w").write(PROBE)
        subprocess.run(["gcc", "-std=c11", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                        "-I", "/opt/rocm/include", src, "-o", exe], check=True)
        lines = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    got = dict(l.rsplit(" ", 1) for l in lines if l)
    C = {"recogs_scene": R.Scene, "recogs_camera": R.Camera, "recogs_select_params": R.SelectParams,
         "recogs_render_opts": R.RenderOpts, "recogs_workspace": R.Workspace, "recogs_batch_view": R.BatchView,
         "recogs_batch_workspace": R.BatchWorkspace}
    for name, cls in C.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
    for key, v in got.items():
        if "." in key:
            t, f = key.split(".")
            assert getattr(C[t], f).offset == int(v), key


class _Ptr:
    """Stands in for a device tensor: only its address is read."""

    def __init__(self, addr):
        self.addr = addr

    def data_ptr(self):
        return self.addr


class _Buf(_Ptr):
    """A device byte buffer stand-in: address and size."""

    def __init__(self, addr, nbytes):
        super().__init__(addr)
        self.nbytes = nbytes

    def numel(self):
        return self.nbytes

    def element_size(self):
        return 1


def test_host_argument_errors_before_any_launch(R):
    B = R.binding
    cam = B.Camera()
    cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy = 64, 64, 50.0, 50.0, 32.0, 32.0
    cam.R[0] = cam.R[4] = cam.R[8] = 1.0
    sc = B.Scene()
    sc.n, sc.stride, sc.sh_degree, sc.storage = 0, 0, 0, 0
    ws = B.Workspace()
    opts = B.opts_struct((16, 16), 1)

    def status(fn, *a):
        with pytest.raises(R.RecogsError) as e:
            fn(*a)
        assert R.recogs_last_error() != ""
        return e.value.status

    # workspace not initialised
    assert status(B.recogs_render, sc, cam, opts, ws, 1, 0) == -1
    # unsupported tile shape / pixels per thread
    assert status(B.recogs_render, sc, cam, B.opts_struct((16, 8), 1), ws, 1, 0) == -3
    assert status(B.recogs_render, sc, cam, B.opts_struct((16, 16), 3), ws, 1, 0) == -3
    # output layout flag and extent rule outside {0, 1}
    o_bad = B.opts_struct((16, 16), 1)
    o_bad.output_chw = 2
    assert status(B.recogs_render, sc, cam, o_bad, ws, 1, 0) == -1
    assert status(B.recogs_render, sc, cam, B.opts_struct((16, 16), 1, extent_rule=2), ws, 1, 0) == -1
    assert status(B.recogs_render, sc, cam, B.opts_struct((16, 16), 1, extent_rule=-1), ws, 1, 0) == -1
    # key count of a workspace: not initialised; before any render it is 0 without a device access
    with pytest.raises(R.RecogsError) as e:
        B.recogs_workspace_keys_needed(ws, 0)
    assert e.value.status == -1
    fake = B.Workspace()
    fake.base, fake.width, fake.height, fake.tile_w, fake.tile_h = 256, 64, 64, 16, 16
    assert B.recogs_workspace_keys_needed(fake, 0) == 0
    # backward: accumulate outside {0, 1}, refused before any launch (an empty scene's
    # workspace state, faked on the host)
    ok = B.opts_struct((16, 16), 1, keep_backward=True)
    assert status(B.recogs_render_backward, sc, cam, ok, fake, 8, 8, 8, 8, 8, 2, 0) == -1
    assert "accumulate" in R.recogs_last_error()
    assert status(B.recogs_render_backward_sh, sc, cam, ok, fake, 8, 8, 8, 8, 8, -1, 0) == -1
    assert status(B.recogs_render_backward, sc, cam, B.opts_struct((16, 16), 1), fake, 8, 8, 8, 8, 8, 0, 0) == -1
    # the block form's scratch: its size, and a scratch too small or misaligned refused
    # (per block of a tile: a float4 per key of capacity, 256-byte rounded, then a 16-byte
    # flag word per 64 keys and per tile, plus two)
    fake.key_capacity, fake.tiles_x, fake.tiles_y = 1000, 4, 4
    assert R.recogs_backward_scratch_bytes(fake, B.opts_struct((16, 16), 1)) == 16 * 4 * 1000 + 16 * 4 * (15 + 16 + 2)
    assert R.recogs_backward_scratch_bytes(fake, B.opts_struct((32, 32), 1)) == 16 * 16 * 1000 + 16 * 16 * (15 + 16 + 2)
    assert R.recogs_backward_scratch_bytes(fake, B.opts_struct((32, 16), 2)) == 16 * 4 * 1000 + 16 * 4 * (15 + 16 + 2)
    fake.key_capacity = 1001
    assert R.recogs_backward_scratch_bytes(fake, B.opts_struct((16, 16), 1)) == 64256 + 16 * 4 * (15 + 16 + 2)
    assert R.recogs_backward_scratch_bytes(fake, B.opts_struct((32, 8), 2)) == 0   # no block form
    small = B.opts_struct((16, 16), 1, keep_backward=True, bwd_scratch=_Buf(512, 100))
    assert status(B.recogs_render_backward, sc, cam, small, fake, 8, 8, 8, 8, 8, 0, 0) == -1
    assert "bwd_scratch" in R.recogs_last_error()
    odd = B.opts_struct((16, 16), 1, keep_backward=True, bwd_scratch=_Buf(520, 1 << 20))
    assert status(B.recogs_render_backward, sc, cam, odd, fake, 8, 8, 8, 8, 8, 0, 0) == -1
    # rough depth map: threshold outside (0, 1], a tile form without one wave per region
    dep = 64  # any non-NULL device address: the options are refused before any launch
    assert status(B.recogs_render, sc, cam, B.opts_struct((16, 16), 1, depth=_Ptr(dep), depth_tau=0.0), ws, 1, 0) == -1
    assert status(B.recogs_render, sc, cam, B.opts_struct((16, 16), 1, depth=_Ptr(dep), depth_tau=1.5), ws, 1, 0) == -1
    assert status(B.recogs_render, sc, cam, B.opts_struct((32, 8), 2, depth=_Ptr(dep)), ws, 1, 0) == -3
    assert status(B.recogs_render, sc, cam, B.opts_struct((8, 8), 4, depth=_Ptr(dep)), ws, 1, 0) == -3
    # selection steps
    assert R.recogs_unproject_workspace_bytes(0, 5) == 0 and R.recogs_unproject_workspace_bytes(64, 64) >= 4 * 5
    nb = R.recogs_unproject_workspace_bytes(64, 64)
    assert status(B.recogs_unproject, cam, 8, 0, 8, 8, -1, 8, 256, nb, 0) == -1          # capacity < 0
    assert status(B.recogs_unproject, cam, 0, 0, 8, 8, 10, 8, 256, nb, 0) == -1          # mask NULL
    assert status(B.recogs_unproject, cam, 8, 0, 8, 8, 10, 8, 256, nb - 1, 0) == -1      # workspace too small
    assert status(B.recogs_unproject, cam, 8, 0, 8, 8, 10, 8, 258, nb, 0) == -1          # workspace misaligned
    assert status(B.recogs_reproject_mask, cam, 8, 10, 5, 2.0, 0, 0.0, 8, 0) == -1       # stride < n
    assert status(B.recogs_reproject_mask, cam, 8, 10, 10, 0.0, 0, 0.0, 8, 0) == -1      # quad_px 0
    assert status(B.recogs_reproject_mask, cam, 8, 10, 10, 65.0, 0, 0.0, 8, 0) == -1     # quad_px > 64
    assert status(B.recogs_reproject_mask, cam, 8, 10, 10, 2.0, 0, -1.0, 8, 0) == -1     # depth_eps < 0
    assert status(B.recogs_reproject_mask, cam, 8, 10, 10, 2.0, 0, 0.0, 0, 0) == -1      # mask NULL
    big = B.Camera()
    big.width, big.height, big.fx, big.fy, big.cx, big.cy = 8193, 8192, 50.0, 50.0, 32.0, 32.0
    big.R[0] = big.R[4] = big.R[8] = 1.0
    assert status(B.recogs_unproject_noalloc, big, 8, 0, 8, 8, 10, 8, 0) == -1          # beyond the fixed scratch
    assert "scratch" in R.recogs_last_error()
    assert status(B.recogs_unproject_noalloc, cam, 0, 0, 8, 8, 10, 8, 0) == -1          # mask NULL
    assert status(B.recogs_tint, 8, 8, (1.0, float("nan"), 1.0), 8, 10, 0) == -1
    assert status(B.recogs_tint, 0, 8, (1.0, 1.0, 1.0), 8, 10, 0) == -1
    # outlier removal
    nb = R.recogs_outlier_workspace_bytes(100)
    assert nb > 0 and R.recogs_outlier_workspace_bytes(-1) == 0
    assert status(B.recogs_remove_outliers, 8, 100, 50, 16, 0.007, 8, 8, 0, 0, 8, 256, nb, 0) == -1   # stride < n
    assert status(B.recogs_remove_outliers, 8, 100, 100, 12, 0.007, 8, 8, 0, 0, 8, 256, nb, 0) == -3  # k
    assert status(B.recogs_remove_outliers, 8, 100, 100, 16, -1.0, 8, 8, 0, 0, 8, 256, nb, 0) == -1   # ratio < 0
    assert status(B.recogs_remove_outliers, 8, 100, 100, 16, 0.007, 8, 8, 8, 50, 8, 256, nb, 0) == -1  # out_stride
    assert status(B.recogs_remove_outliers, 8, 100, 100, 16, 0.007, 8, 8, 0, 0, 8, 256, nb - 1, 0) == -1
    assert status(B.recogs_remove_outliers, 8, 100, 100, 16, 0.007, 8, 8, 0, 0, 8, 128, nb, 0) == -1  # misaligned
    assert status(B.recogs_remove_outliers, 0, 100, 100, 16, 0.007, 8, 8, 0, 0, 8, 256, nb, 0) == -1  # NULL points
    # invalid scene fields
    bad = B.Scene()
    bad.n, bad.stride, bad.sh_degree = 10, 5, 0
    assert status(B.recogs_select, bad, cam, B.SelectParams(), 1, 1, 0) == -1
    bad.stride, bad.sh_degree = 10, 4
    assert status(B.recogs_select, bad, cam, B.SelectParams(), 1, 1, 0) == -1
    bad.sh_degree, bad.storage = 0, 7
    assert status(B.recogs_select, bad, cam, B.SelectParams(), 1, 1, 0) == -1
    bad.storage = 0
    assert status(B.recogs_select, bad, cam, B.SelectParams(), 1, 1, 0) == -1  # null pointers with n > 0
    # invalid camera
    cam2 = B.Camera()
    assert status(B.recogs_select, sc, cam2, B.SelectParams(), 1, 1, 0) == -1
    # half a fused recolour
    o2 = B.opts_struct((16, 16), 1)
    o2.mask = 8
    assert status(B.recogs_render, sc, cam, o2, ws, 1, 0) == -1
    # workspace sizing and carving
    assert R.recogs_workspace_bytes(-1, 64, 64, 16, 16, 10) == 0
    assert R.recogs_workspace_bytes(10, 64, 64, 16, 8, 10) == 0
    need = R.recogs_workspace_bytes(100, 64, 64, 16, 16, 1000)
    assert need > 0
    assert status(R.recogs_workspace_init, ws, 256, need - 1, 100, 64, 64, 16, 16, 1000) == -1
    assert status(R.recogs_workspace_init, ws, 257, need, 100, 64, 64, 16, 16, 1000) == -1
    # loss
    assert status(B.recogs_loss_l2, 0, 0, 10, 1.0, 0, 0, 0) == -1
    assert status(B.recogs_loss_l1, 0, 0, 10, 1.0, 0, 0, 0) == -1
    assert status(B.recogs_loss_l1, 0, 0, -1, 1.0, 0, 0, 0) == -1
    # 9 floats per pixel, then 2 x 3 per 16 x 16 tile (partial sums of S and of |y - t|)
    assert R.recogs_dssim_workspace_bytes(0, 10) == 0 and R.recogs_dssim_workspace_bytes(4, 5) == 4 * (9 * 20 + 6)
    assert R.recogs_dssim_workspace_bytes(33, 17) == 4 * (9 * 33 * 17 + 6 * 3 * 2)
    assert status(B.recogs_loss_dssim, 0, 0, 0, 8, 0.2, 0, 0, 0, 0, 0, 0) == -1           # width 0
    assert status(B.recogs_loss_dssim, 8, 8, 4, 5, 0.2, 8, 0, 8, 8, 4 * (9 * 20 + 6) - 1, 0) == -1  # workspace too small
    # (image, target, width, height, l1_scale, weight, dL, accumulate, loss, workspace, bytes, stream)
    assert status(B.recogs_loss_l1_dssim, 8, 8, 0, 5, 0.1, 0.2, 8, 0, 8, 8, 10 ** 6, 0) == -1       # width 0
    assert status(B.recogs_loss_l1_dssim, 8, 8, 4, 5, 0.1, 0.2, 8, 2, 8, 8, 10 ** 6, 0) == -1       # accumulate 2
    assert status(B.recogs_loss_l1_dssim, 8, 0, 4, 5, 0.1, 0.2, 8, 0, 8, 8, 10 ** 6, 0) == -1       # NULL target
    assert status(B.recogs_loss_l1_dssim, 8, 8, 4, 5, 0.1, 0.2, 8, 0, 8, 8, 4 * (9 * 20 + 6) - 1, 0) == -1
    assert status(B.recogs_loss_l1_dssim, 8, 8, 4, 5, 0.1, 0.2, 8, 0, 8, 10, 10 ** 6, 0) == -1      # workspace alignment
        # (param, grad, m, v, count, lr, beta1, beta2, eps, step, stream)
    assert status(B.recogs_adam_step, 0, 0, 0, 0, 10, 1e-3, 0.9, 0.999, 1e-15, 1, 0) == -1  # NULL arrays
    assert status(B.recogs_adam_step, 0, 0, 0, 0, 0, 1e-3, 0.9, 0.999, 1e-15, 0, 0) == -1   # step counts from 1
    assert status(B.recogs_adam_step, 0, 0, 0, 0, 0, 1e-3, 1.0, 0.999, 1e-15, 1, 0) == -1   # beta outside [0, 1)
    # batch: empty, and mixed storage
    views = (B.BatchView * 2)()
    assert R.recogs_batch_workspace_bytes(views, 0, 16, 16, 10) == 0
    for k in range(2):
        views[k].scene = sc
        views[k].cam = cam
        views[k].image = 64
    views[1].scene.storage = 1
    assert R.recogs_batch_workspace_bytes(views, 2, 16, 16, 10) == 0
    bw = B.BatchWorkspace()
    assert status(R.recogs_batch_init, bw, 256, 1 << 20, views, 2, opts, 10) == -3
    views[1].scene.storage = 0
    assert status(R.recogs_batch_init, bw, 256, 1 << 20, views, 2, B.opts_struct((16, 16), 1, depth=_Ptr(64)), 10) == -3
    assert status(R.recogs_render_batch, bw, 0) == -1
