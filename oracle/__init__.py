"""CPU FP64 oracle of the tile-based splatting renderer.

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.
"""
from .splat import (  # noqa: F401
    Config, TILE, GRAD2D_FIELDS, AMBIG_ALPHA, AMBIG_T, AMBIG_BIN,
    quat_to_rotmat, quat_to_rotmat_grads, covariance_3d, project, tile_lists, tile_alpha_max,
    render, backward_2d, sigma2d_backward, select_reliable, backward_params, render_backward, l1_loss, f32,
    l1_pixel_loss, loss_median, loss_cap, sh_basis, SH_C0, SH_C1,
)
from .pose import se3_exp, se3_left_jacobian, pose_xi_grad, apply_xi, pose_from_qt  # noqa: F401,E402
