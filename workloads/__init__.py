"""Seeded synthetic inputs for the splatting renderer.

This package only draws random numbers and lays them out: Gaussian scenes,
pinhole cameras and poses, target images and upstream gradients.  It contains
none of the renderer's arithmetic, so both the CPU oracle and the GPU path can
consume the same arrays without sharing any of the method's code.
"""
from .scenes import (  # noqa: F401
    Camera,
    Scene,
    random_scene,
    needle_scene,
    room_scene,
    tracking_scene,
    camera_small,
    camera_replica,
    camera_tum,
    camera_tum_coarse,
    camera_quarter_tum,
    camera_hyp_half,
    camera_tracking,
    se3_exp,
    perturb_pose,
    tracking_start,
    noisy_targets,
    mapping_views,
    hypothesis_views,
    upstream_grads,
    random_targets,
    loss_images,
    expansion_images,
    room_depth,
    with_sh,
    subset,
)
