"""Shared helpers of the GPU parity tests: move seeded inputs to the device,
turn oracle outputs into the projected-record layout, and compare."""

from __future__ import annotations

import numpy as np
import torch

from oracle import raster as R

F64 = torch.float64


def oracle_camera(cam: dict) -> R.Camera:
    return R.Camera(**cam)


def oracle_render(gauss_np: dict, cam: dict, w2c, pose=None, requires_grad=False, bg=None, tiles_subset=None,
                  with_margins=True):
    g = R.to_f64(gauss_np, requires_grad=requires_grad)
    pose_t = None
    if pose is not None:
        pose_t = torch.as_tensor(np.asarray(pose, np.float64)).clone().requires_grad_(requires_grad)
    out = R.render(g, oracle_camera(cam), torch.as_tensor(np.asarray(w2c, np.float64)), pose_t,
                   bg=None if bg is None else torch.as_tensor(np.asarray(bg, np.float64)), tiles_subset=tiles_subset,
                   with_margins=with_margins)
    return g, pose_t, out


def records_from_oracle(pr: dict, gauss_np: dict) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """FP32 projected records (ls_projected layout) from an oracle projection."""
    n = len(pr["radius"])
    rec = np.zeros((n, 12), np.float32)
    rec[:, 0] = pr["u32"]
    rec[:, 1] = pr["v32"]
    conic = pr["conic"].detach().numpy()
    rec[:, 2] = conic[:, 0]
    rec[:, 3] = conic[:, 1]
    rec[:, 4] = conic[:, 2]
    rec[:, 5] = (1.0 / (1.0 + np.exp(-np.asarray(gauss_np["opacity_logit"], np.float64)))).astype(np.float32)
    rec[:, 6] = pr["z32"]
    rec[:, 8:11] = np.asarray(gauss_np["rgb"], np.float32).T
    culled = pr["radius"] == 0
    rec[culled] = 0.0
    return rec, pr["radius"].astype(np.int32), pr["tiles"].astype(np.int32)


def rel_err(a, b) -> float:
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a - b))


def image_close(gpu, ora, mask=None, tol=1e-4):
    """|gpu - ora| <= tol * max(|ora|, 1) on the masked pixels; returns the
    number of violations."""
    gpu = np.asarray(gpu, np.float64)
    ora = np.asarray(ora, np.float64)
    bad = np.abs(gpu - ora) > tol * np.maximum(np.abs(ora), 1.0)
    if mask is not None:
        bad &= mask
    return int(bad.sum())
