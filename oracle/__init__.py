"""FP64 CPU oracle for the anchor-Gaussian render hot path (test infrastructure).

This package is test infrastructure. Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path (the HIP library
and its Python binding) never does, and this package imports nothing from the
product path.

It is a plain, slow, direct transcription of what the paper's method computes,
in float64 with PyTorch CPU ops:

* ``decode``      anchor -> k neural Gaussians through five two-layer head MLPs
                  (Sec. 3.3, Eq. 8 and Eq. 9, MLP details in the appendix);
* ``project``     3D Gaussians -> 2D conics with the EWA Jacobian (Sec. 3.1,
                  Eq. 2) and the tight footprint / tile rectangle;
* ``binning``     per-tile depth-ordered lists (tile-based rasteriser the paper
                  follows, Sec. 2 and Sec. 3.1);
* ``composite``   front-to-back alpha compositing of colour, depth, the opacity
                  sum (Eq. 3) and the low-dimensional feature (Eq. 10);
* ``uncertainty`` the multi-modal tracking residual (Sec. 3.2, Eq. 6) and
                  the per-pixel uncertainty and motion mask (Sec. 3.4, Eq. 15);
* ``feature``     the feature lift F_m and the cosine distillation loss
                  (Sec. 3.3, Eq. 11 and Eq. 12);
* ``anchors``     the probabilistic anchor update (Sec. 3.3, Eq. 7);
* ``mapping``     the mapping losses: SSIM geometric loss (Sec. 3.1, Eq. 4),
                  the uncertainty MLP F_u and its loss (Sec. 3.2 Eq. 5,
                  Sec. 3.3 Eq. 13), the motion mask and the total loss with
                  the mean-scale term (Sec. 3.3, Eq. 14);
* ``render``      the whole path, with the backward pass as the vector-Jacobian
                  product of the forward definition (torch autograd in float64)
                  and the SE(3) pose gradient.

Readings of the paper where it is silent are listed in ``oracle.readings``.
Parity pins (closed forms, invariants, brute force, finite differences) live
in ``tests/test_oracle_*.py``.
"""
from .readings import (RenderOpts, READINGS, RESIDUAL_READINGS, FEATURE_READINGS, ANCHOR_READINGS,  # noqa: F401
                       MAPPING_READINGS)
from .geometry import quat_to_rotmat, se3_exp, pose_cw, camera_center  # noqa: F401
from .decode import decode, bf16_hidden_margin, bf16_flip_bound, HEAD_ORDER  # noqa: F401
from .project import project  # noqa: F401
from .binning import bin_and_sort  # noqa: F401
from .composite import composite_tile, composite_bruteforce  # noqa: F401
from .render import render, render_scene, gaussians_from_plain, Leaves  # noqa: F401
from .uncertainty import box3, cosine, residual, uncertainty, RESIDUAL_WEIGHTS  # noqa: F401
from .feature import upsample, lift, cosine_map, distill, relu_margin  # noqa: F401
from .anchors import anchor_update  # noqa: F401
from .mapping import (gaussian_filter, ssim_map, pixel_loss, mapping_loss, mean_scale,  # noqa: F401
                      uncertainty_mlp, uncertainty_loss, uncertainty_flip_bound, MAPPING_WEIGHTS)
