"""FP64 oracle of the mapping loss (Sec. 3.1, submap update: Eq. 3 to Eq. 5).

TEST INFRASTRUCTURE ONLY (see the package docstring): never imported by the
product path.

The submap-update loss weighs a colour term, a depth term and an isotropic
regulariser (Eq. 3); the colour term mixes L1 and SSIM (Eq. 4); the
regulariser pulls each Gaussian's three scales towards their mean (Eq. 5).
The supplement sets the three weights of Eq. 3 to 1.  What the paper leaves
open is fixed by these readings:

  R26 SSIM is the windowed index of Wang et al. (2004) with an 11 x 11
      Gaussian window of standard deviation 1.5 (weights normalised to sum
      to 1), zero padding outside the image, C1 = 0.01^2 and C2 = 0.03^2
      (dynamic range 1), moments taken as E[xy] - mu_x mu_y, evaluated per
      colour channel; SSIM(I^, I) is the mean of the index over the three
      channels and every pixel.
  R27 lambda_SSIM = 0.2 (the paper gives none; this is the usual 3DGS value).
  R28 the L1 parts of the colour and depth terms follow R15: the mean over
      the pixels with target depth > 0 of sum_c |C^ - C| and of |D^ - D|.
  R29 the regulariser's |.|_1 is summed over the three axes and averaged over
      the K Gaussians, on the scales s = exp(log_scale); the mean s-bar is the
      arithmetic mean of the three scales and is differentiated through.
"""

from __future__ import annotations

import math

import numpy as np
import torch
import torch.nn.functional as F

F64 = torch.float64

SSIM_RADIUS = 5
SSIM_SIGMA = 1.5
SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2
LAMBDA_SSIM = 0.2


def ssim_window() -> torch.Tensor:
    """The 11 normalised 1D Gaussian weights (R26); the 2D window is their
    outer product."""
    k = torch.arange(-SSIM_RADIUS, SSIM_RADIUS + 1, dtype=F64)
    g = torch.exp(-(k * k) / (2.0 * SSIM_SIGMA ** 2))
    return g / g.sum()


def ssim_map(x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    """Per-pixel SSIM index of two [C, H, W] images (R26), float64, by 2D
    convolution with the zero-padded window; differentiable."""
    g = ssim_window()
    w2 = torch.outer(g, g)[None, None]
    c = x.shape[0]
    xx, yy = x.to(F64)[:, None], y.to(F64)[:, None]

    def blur(t):
        return F.conv2d(t, w2, padding=SSIM_RADIUS).reshape(c, *x.shape[1:])

    mx, my = blur(xx), blur(yy)
    sxx = blur(xx * xx) - mx * mx
    syy = blur(yy * yy) - my * my
    sxy = blur(xx * yy) - mx * my
    num = (2.0 * mx * my + SSIM_C1) * (2.0 * sxy + SSIM_C2)
    den = (mx * mx + my * my + SSIM_C1) * (sxx + syy + SSIM_C2)
    return num / den


def loss_mapping(rgb, depth, tgt_rgb, tgt_depth, lambda_ssim: float = LAMBDA_SSIM, lambda_color: float = 1.0,
                 lambda_depth: float = 1.0):
    """Image part of the mapping loss (Eq. 3 without the regulariser, Eq. 4,
    R26-R28) for one render: rgb [3,H,W], depth [H,W].

    L = lc ((1 - ls) L1_rgb + ls (1 - SSIM)) + ld L1_depth.  The L1 means are
    0 when no pixel has a target depth; the SSIM term is not masked."""
    valid = (torch.as_tensor(tgt_depth) > 0).to(F64)
    cnt = valid.sum()
    tr, td = torch.as_tensor(tgt_rgb, dtype=F64), torch.as_tensor(tgt_depth, dtype=F64)
    if cnt.item() > 0:
        l1_rgb = (torch.abs(rgb - tr).sum(0) * valid).sum() / cnt
        l1_depth = (torch.abs(depth - td) * valid).sum() / cnt
    else:
        l1_rgb = rgb.sum() * 0.0
        l1_depth = depth.sum() * 0.0
    ssim = ssim_map(rgb, tr).mean()
    return lambda_color * ((1.0 - lambda_ssim) * l1_rgb + lambda_ssim * (1.0 - ssim)) + lambda_depth * l1_depth


def loss_isotropic(log_scale: torch.Tensor, lambda_reg: float = 1.0) -> torch.Tensor:
    """Isotropic regulariser (Eq. 5, R29) of one submap: log_scale [K, 3]."""
    s = torch.exp(log_scale.to(F64))
    if s.shape[0] == 0:
        return s.sum() * 0.0
    sbar = s.mean(dim=1, keepdim=True)
    return lambda_reg * torch.abs(s - sbar).sum(dim=1).mean()


def ssim_brute_force(x: np.ndarray, y: np.ndarray, ch: int, i: int, j: int) -> float:
    """SSIM index of one pixel (row i, column j) of channel ch, from explicit
    window sums in pure Python (small images only)."""
    g = [math.exp(-(k * k) / (2.0 * SSIM_SIGMA ** 2)) for k in range(-SSIM_RADIUS, SSIM_RADIUS + 1)]
    tot = sum(g)
    g = [v / tot for v in g]
    h, w = x.shape[1], x.shape[2]
    mx = my = exx = eyy = exy = 0.0
    for a in range(-SSIM_RADIUS, SSIM_RADIUS + 1):
        for b in range(-SSIM_RADIUS, SSIM_RADIUS + 1):
            r, c = i + a, j + b
            if 0 <= r < h and 0 <= c < w:
                wt = g[a + SSIM_RADIUS] * g[b + SSIM_RADIUS]
                xv, yv = float(x[ch, r, c]), float(y[ch, r, c])
                mx += wt * xv
                my += wt * yv
                exx += wt * xv * xv
                eyy += wt * yv * yv
                exy += wt * xv * yv
    vx, vy, cxy = exx - mx * mx, eyy - my * my, exy - mx * my
    return ((2 * mx * my + SSIM_C1) * (2 * cxy + SSIM_C2)) / ((mx * mx + my * my + SSIM_C1) * (vx + vy + SSIM_C2))
