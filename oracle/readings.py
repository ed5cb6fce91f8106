"""Render options and the readings taken where the paper is silent.

Test infrastructure (see the package docstring).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Tuple


@dataclass
class RenderOpts:
    tile: int = 16                 # square screen tiles (pixels per side)
    n_feat: int = 16               # low-dimensional feature channels N_l (0 = none)
    alpha_min: float = 1.0 / 255.0  # a Gaussian with alpha below this is skipped
    alpha_max: float = 0.99         # alpha is clamped to at most this
    T_min: float = 1e-4             # compositing stops before T would fall below this
    dilation: float = 0.3           # added to the 2D covariance diagonal (px^2)
    znear: float = 0.2              # camera-space depth below which a Gaussian is culled
    fov_clamp: float = 1.3          # Jacobian evaluated with x/z clamped to +-fov_clamp*W/(2 fx); 0 = off
    bg: Tuple[float, float, float] = field(default=(0.0, 0.0, 0.0))
    extent_mode: int = 0            # 0: tight alpha_min box; 1: 3-sigma square (vanilla 3DGS)


# Each reading: where the paper is silent, ambiguous or garbled, and what is taken.
READINGS = (
    "Eq.2 writes the 4x4 pose inverse around a 3x3 covariance: W is read as the rotation of T_wc^-1.",
    "Eq.3 names the opacity sum 'accumulated transmittance'; the rendered 'alpha' is that sum, "
    "sum_i sigma_i prod_{j<i}(1-sigma_j), which equals 1 - T_final.",
    "sigma_i of Eq.3 is alpha_i = min(alpha_max, o_i exp(-1/2 d^T Sigma'^-1 d)).",
    "Unstated constants follow the vanilla 3DGS rasteriser the paper says it follows: alpha_min 1/255, "
    "alpha_max 0.99, T_min 1e-4, dilation 0.3 px^2, znear 0.2, Jacobian clamp 1.3, 16x16 tiles.",
    "Termination is exclusive: the Gaussian that would take T below T_min is not composited, and the "
    "pixel stops there.",
    "Footprint is the exact axis-aligned box of the ellipse where alpha >= alpha_min, so tiled "
    "compositing equals per-pixel brute force and does not depend on the tile size. The vanilla "
    "rasteriser's footprint (a square of half side ceil(3 sqrt(lambda_max)), lambda_max = mid + "
    "sqrt(max(0.1, mid^2 - det)), mid = (a + c)/2 of the dilated 2D covariance) is an option.",
    "Pixel (px, py) is evaluated at the integer point (px, py); cx = (W-1)/2 in the workloads.",
    "z_i is the camera-space depth of the Gaussian centre; rendered depth is not normalised by alpha; "
    "background is zero unless bg is set (colour only).",
    "Gaussians at exactly equal float32 depth in one tile are ordered by ascending index.",
    "Quaternions are (w, x, y, z), normalised inside the projection; gradients are w.r.t. the raw input.",
    "Five separate head MLPs in->32->k*m (opacity, colour, scale, rotation with ReLU; feature with "
    "SoftPlus); outputs: opacity=sigmoid, colour=sigmoid, scale=l_s*sigmoid, rotation raw, feature raw.",
    "Decoder input is [anchor feature (32), unit view direction (3)] (35 wide); mean = x_v + l_o*O_vi.",
    "Scene-variant decoders append the anchor-camera distance |x_v - c| (unnormalised, metres; 36 wide) "
    "and then the temporal embedding (sin pi t, cos pi t) (38 wide) to every head's input; t is the "
    "frame time of the view, given by the caller.",
    "Pose gradient is w.r.t. xi=(rho,phi) under T_cw <- Exp(xi) T_cw and includes the camera-centre "
    "path through the decoder's view direction.",
    "A Gaussian is culled when o <= alpha_min (no pixel can reach alpha_min), when t_z <= znear, "
    "when det(Sigma') <= 0, or when its tile rectangle is empty.",
)


# Readings for the tracking residual and uncertainty (Sec. 3.2 Eq. 6, Sec. 3.4 Eq. 15).
RESIDUAL_READINGS = (
    "Eq.6 names its mask (T~ < 0.1) after the 'accumulated transmittance' but says it keeps low-opacity "
    "regions out: a pixel contributes when its remaining transmittance 1 - alpha (alpha = the opacity "
    "sum of Eq.3) is below 0.1.",
    "|C~ - C| is the L1 norm over the three colour channels (their sum of absolute differences).",
    "The 3x3 box filter of the observed depth averages the pixel and its neighbours inside the image "
    "(no padding values); no pixel is treated as missing depth.",
    "cos(F, F^) divides by the product of the two norms bounded below by 1e-12; the feature term is "
    "min(1, 1 - cos).",
    "Eq.15 is minimised pixel by pixel: sigma = max(sigma_min, sqrt(2R)), the exact minimiser of "
    "1/2 (R/sigma^2 + log sigma) over sigma >= sigma_min (sigma_min = 1e-3 keeps R = 0 finite).",
    "The tracking motion mask threshold is unstated: the mapping mask's criterion 2 sigma^2 > 1 (Eq.14) "
    "is used, i.e. dynamic where 4R > 1 above the floor.",
    "Residual weights (lambda_1^t, lambda_2^t, lambda_3^t) = (0.25, 0.7, 0.1) from the appendix.",
    "The tracking optimiser is unstated: Adam on the pose twist (lr 5e-4), the twist folded into the pose "
    "after every step; the colour and depth terms of a weighted L1 residual carry lambda_1^t and "
    "lambda_2^t, with per-pixel weights standing in for the uncertainty mask.",
)


# Readings for the feature lift and the distillation loss (Sec. 3.3, Eq. 11, Eq. 12).
FEATURE_READINGS = (
    "F_m is a per-pixel MLP: the appendix's 'Convolution -> ReLU -> Convolution' with a 128-wide hidden "
    "layer is read as 1x1 convolutions 16 -> 128 -> N_h (a 'shallow MLP' lifting each pixel's feature).",
    "N_h is unstated: 384, the width of DINOv2 ViT-S/14 features, as a parameter.",
    "DINO features live on the patch grid (34 x 46 patches of 14 px for a 476 x 644 crop of a 640 x 480 "
    "frame) and are upsampled bilinearly to the image with half-pixel sample centres, clamped at the "
    "borders (the usual align-corners-off convention).",
    "Eq.12's sum over i = 0..N_d divided by N_d is the mean over the image's pixels (feature vectors) of "
    "1 - cos(F, F^).",
    "cos divides by the product of the norms bounded below by 1e-12, as in the tracking residual.",
)


# Readings for the probabilistic anchor update (Sec. 3.3, Eq. 7).
ANCHOR_READINGS = (
    "Eq.7's factor P(n)/P(n) is read as the prior odds P(n)/(1 - P(n)), the occupancy-mapping form the "
    "paper cites: the log-odds of the posterior are those of the observation plus those of the previous "
    "estimate minus those of the prior.",
    "The observation model P(n | z_t) is not stated: it is an input per anchor.",
    "Clamping bounds and the pruning level are not stated: options, by default no clamping [0, 1] and no "
    "pruning.",
)


# Readings for the mapping losses (Sec. 3.1 Eq. 4, Sec. 3.2 Eq. 5, Sec. 3.3 Eq. 13 and Eq. 14).
MAPPING_READINGS = (
    "The appendix lists five values {0.8, 0.6, 1.0, 0.4, 0.01} for six names {lambda, lambda_1 .. lambda_5}: "
    "they are read in order (lambda 0.8, lambda_1 0.6, lambda_2 1.0, lambda_3 0.4, lambda_4 0.01) and "
    "lambda_5, left without a value, is an option with default 0.01.",
    "The squared norms of Eq.4 are per pixel (the colour one summed over the three channels) and the loss "
    "is their mean over the pixels; SSIM(C~, C) is the mean over channels and pixels of the structural-"
    "similarity map with the vanilla 3DGS window: 11 x 11 Gaussian, sigma 1.5, zero padding, "
    "C1 = 0.01^2, C2 = 0.03^2.",
    "Eq.14 writes M(L_g + lambda_4 L_d) with M = [2 sigma^2 > 1] true on dynamic pixels; the loss is read as "
    "gating out the dynamic pixels, i.e. weighting each pixel's terms by 1 - M, then averaging over all "
    "pixels.",
    "s_bar is the mean over Gaussians and axes of the linear (post-activation) scale.",
    "F_u (Conv -> ReLU -> Conv -> SoftPlus, hidden 128) is a per-pixel MLP N_h -> 128 -> 1 on the DINO "
    "feature bilinearly upsampled to the pixel (the F of Eq.12); sigma = sigma_min + its output with "
    "sigma_min = 1e-3, which keeps L_u bounded below where R = 0.",
    "R in Eq.5 is the residual of Eq.6 (the same weights as tracking), taken as a constant: L_u's "
    "gradient reaches only F_u's parameters, L's only the Gaussians (and F_m), which is how the two "
    "gradient flows are kept separate; M is formed from F_u's sigma before F_u's update.",
)
