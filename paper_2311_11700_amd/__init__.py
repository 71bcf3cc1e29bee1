"""MI355X (gfx950) differentiable tile-based Gaussian splatting renderer.

The rendering hot path of GS-SLAM (arXiv 2311.11700): projection (Eq. 3),
tile binning and depth sort, front-to-back colour/depth compositing
(Eq. 4-5), L1 loss (Eq. 6/10) and the backward pass to every Gaussian
parameter and the se(3) camera pose -- all in hand-written HIP kernels
behind the C ABI of include/gsr.h.  This package is the ctypes binding.
"""
from ._abi import (  # noqa: F401
    GSR_FULL_RECT, GSR_GAUSS_GRAD, GSR_POSE_GRAD, GSR_PAPER_POSE_APPROX, GSR_GRAD_OVERWRITE,
    GSR_OK, GSR_E_INVALID, GSR_E_CAPACITY, GSR_E_HIP, GSR_E_UNSUPPORTED, GSR_E_STATE, GSR_NOALLOC_SCRATCH_BYTES,
    load, exported_symbols, LIB_PATH,
)
from .renderer import (  # noqa: F401
    Config, Gaussians, GsrError, Renderer, pack_cameras, render, split_views,
)
