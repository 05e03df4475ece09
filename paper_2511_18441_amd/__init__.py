"""MI355X-native select / recolour / splat-render path of ReCoGS (arXiv 2511.18441).

The compute path is librecogs.so (hand-written HIP for gfx950, C ABI in
include/recogs.h); this package is its ctypes binding plus a torch.autograd.Function
over the hand-written backward. Importing it loads the library and fails loudly if it
has not been built.
"""
from .binding import (  # noqa: F401
    ENTRY_POINTS, RecogsError, DeviceScene, DeviceWorkspace, Scene, Camera, SelectParams, RenderOpts, Workspace,
    camera_struct, select_struct, opts_struct, render, lib,
    recogs_workspace_bytes, recogs_workspace_init, recogs_workspace_readback, recogs_workspace_profile_flush, recogs_workspace_release,
    recogs_prepare_covariance, recogs_select, recogs_recolor,
    recogs_render, recogs_render_backward, recogs_loss_l2, recogs_render_backward_sh, recogs_loss_l1,
    recogs_adam_step, recogs_dssim_workspace_bytes, recogs_loss_dssim, recogs_loss_l1_dssim, recogs_last_error,
    recogs_unproject_workspace_bytes, recogs_unproject, recogs_reproject_mask, recogs_tint, unproject, reproject_mask, tint,
    recogs_outlier_workspace_bytes, recogs_remove_outliers, remove_outliers, recogs_render_backward_sh_adam,
    recogs_workspace_keys_needed, recogs_unproject_noalloc, recogs_backward_scratch_bytes,
    BATCH_ENTRY_POINTS, BatchView, BatchWorkspace, DeviceBatch, recogs_batch_workspace_bytes, recogs_batch_init,
    recogs_render_batch, recogs_batch_readback,
)

lib()

try:  # the autograd wrapper needs torch
    from .autograd import RecogsRenderFn  # noqa: F401
except ImportError:  # pragma: no cover
    pass
