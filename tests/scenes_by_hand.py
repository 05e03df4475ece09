"""Hand-placed scenes and cameras for closed-form tests (no method arithmetic here)."""
import numpy as np

from synth import Camera, Scene

Y00 = 0.28209479177387814


def axis_camera(W=32, H=32, f=40.0, cx=None, cy=None, R=None, t=None, znear=0.2):
    """Camera at the world origin looking down +z (R = I, t = 0) unless given."""
    return Camera(W, H, float(np.float32(f)), float(np.float32(f)),
                  float(np.float32(W / 2 if cx is None else cx)), float(np.float32(H / 2 if cy is None else cy)),
                  np.eye(3, dtype=np.float32) if R is None else np.asarray(R, np.float32),
                  np.zeros(3, np.float32) if t is None else np.asarray(t, np.float32),
                  float(np.float32(znear)))


def scene_from(means, log_scales, opacity, dc_rgb=None, quats=None, sh=None, deg=0):
    """means (n,3), log_scales (n,3), opacity (n,), dc_rgb (n,3) displayed DC colour."""
    means = np.asarray(means, np.float64).reshape(-1, 3)
    n = means.shape[0]
    ls = np.asarray(log_scales, np.float64).reshape(n, 3)
    q = np.tile([1.0, 0, 0, 0], (n, 1)) if quats is None else np.asarray(quats, np.float64).reshape(n, 4)
    if sh is None:
        K = (deg + 1) ** 2
        sh = np.zeros((K * 3, n))
        rgb = np.asarray(dc_rgb, np.float64).reshape(n, 3)
        sh[0:3] = ((rgb - 0.5) / Y00).T
    return Scene(np.ascontiguousarray(means.T.astype(np.float32)), np.ascontiguousarray(ls.T.astype(np.float32)),
                 np.ascontiguousarray(q.T.astype(np.float32)), np.asarray(opacity, np.float32).reshape(n),
                 np.ascontiguousarray(np.asarray(sh, np.float32)), deg, "f32")
