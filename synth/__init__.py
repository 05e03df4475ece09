"""Seeded synthetic inputs shared by the HIP path's tests/bench and the CPU oracle.

This package draws random numbers and packs them into arrays. It performs none of
the rendering, selection or recolor arithmetic; both sides consume its arrays.
"""
from .scenes import (  # noqa: F401
    Camera, Scene, SelectParams, RecolorParams, View, Workload, target_noise, random_image,
    make_tiny, make_mid, make_precision, make_batch, make_diff, make_diff_fd,
    orbit_camera, hue_rotation, make_scene_mid_like, make_scene_tiny_like,
    bf16_bits_from_f32, f32_from_bf16_bits, storage_to_f32, f32_to_storage,
    CONFIG_NAMES, make_config, brush_mask, sample_keep, nearby_orbit,
)
