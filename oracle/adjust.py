"""FP64 oracle of the globally consistent map adjustment (Sec. 3.3, Eq. 8).

TEST INFRASTRUCTURE ONLY (see the package docstring): never imported by the
product path.

After pose-graph optimisation every submap i receives a rigid correction
T_c = [R_c | t_c].  Its keyframe poses are left-multiplied by T_c, its
Gaussian means map to R_c mu + t_c and its covariances to R_c Sigma R_c^T.
Scales, opacities and colours are unchanged.

  R30 keyframe poses are camera-to-world, so the correction (expressed in the
      world frame) is applied on the left: T_j <- T_c T_j, as Eq. 8 writes.
"""

from __future__ import annotations

import numpy as np
import torch

from . import raster

F64 = torch.float64


def adjust_gaussians(mean: torch.Tensor, log_scale: torch.Tensor, quat: torch.Tensor, T: np.ndarray):
    """Means [N,3] and covariances [N,3,3] of one submap after the correction
    T ([3,4] or [4,4], rotation block R_c, translation t_c)."""
    T = torch.as_tensor(np.asarray(T, np.float64))
    Rc, tc = T[:3, :3], T[:3, 3]
    sigma = raster.covariance3d(log_scale.to(F64), quat.to(F64))
    return mean.to(F64) @ Rc.T + tc, Rc @ sigma @ Rc.T


def adjust_poses(c2w: np.ndarray, T: np.ndarray) -> np.ndarray:
    """Keyframe poses [k,4,4] (or [k,3,4]) after the correction: T_c T_j."""
    c2w = np.asarray(c2w, np.float64)
    k = c2w.shape[0]
    full = np.tile(np.eye(4), (k, 1, 1))
    full[:, :3, :] = c2w[:, :3, :]
    Tf = np.eye(4)
    Tf[:3, :] = np.asarray(T, np.float64)[:3, :]
    return Tf[None] @ full
