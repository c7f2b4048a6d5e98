"""Pair registration through the C ABI (3DGS registration, Sec. 3.2).

`keyframe_targets` renders a submap at its own keyframes with the rasterizer
(the synthetic stand-in for the keyframes' RGB-D measurements);
`register_pair` hands one pair to ls_register_pair and returns the fused
T_{P->Q}, the per-view estimates and residuals (and exposure coefficients
when they are optimised).
"""

from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import lib as L
from .render import GaussianSet, RenderBatch, _stream


def inv_rigid(t: np.ndarray) -> np.ndarray:
    out = np.eye(4)
    out[:3, :3] = t[:3, :3].T
    out[:3, 3] = -t[:3, :3].T @ t[:3, 3]
    return out


def keyframe_targets(g: GaussianSet, cam: dict, c2ws: np.ndarray):
    """Renders `g` at each camera-to-world pose: returns rgb [V,3,H,W] and
    depth [V,H,W] device tensors."""
    jobs = [(g, cam, inv_rigid(np.asarray(c, np.float64))[:3]) for c in c2ws]
    b = RenderBatch(jobs)
    b.project()
    b.bin_sort()
    b.render_fwd()
    H, W = cam["height"], cam["width"]
    rgb = b.rgb.view(len(jobs), 3, H, W).clone()
    depth = b.depth.view(len(jobs), H, W).clone()
    b.close()
    return rgb, depth


def default_params(iters=200, lr_rot=0.015, lr_trans=0.005, exit_rel_tol=0.0, exit_patience=0, loss="l1",
                   lambda_c=0.6, inlier_k=50.0, alpha_power=3, exposure=False,
                   lr_exposure=0.1, joint=False, top_k=0, exit_mode="loss") -> L.ls_reg_params:
    """Registration settings: real-data learning rates of the paper's
    loop-closure table by default; early exit off unless exit_patience > 0.
    loss "l1" (the default) is the registration loss of Sec. 3.2, the plain
    unmasked colour + depth L1; "tracking" is Eq. 2 with the supplement's
    alpha and inlier masks (lambda_c of the real-data column of the
    per-dataset table), a variant.  exposure: per-view exposure
    coefficients (gain and offset of the rendered colour) optimised with the
    pose at lr_exposure (the supplement's 0.1).  joint: one transform shared
    by all views instead of per-view estimates and their fusion (a
    comparison; ls_register_pair only).  top_k: keyframes kept per direction
    (0: all), ranked by rendered co-visibility (ls_register_pair only).
    exit_mode: "loss" (plateau of the loss, exit_rel_tol relative) or "step"
    (Adam step below exit_rel_tol learning rates) when exit_patience > 0."""
    if loss not in ("tracking", "l1"):
        raise ValueError(f"loss must be 'tracking' or 'l1', not {loss!r}")
    if exit_mode not in ("loss", "step"):
        raise ValueError(f"exit_mode must be 'loss' or 'step', not {exit_mode!r}")
    return L.ls_reg_params(iters, lr_rot, lr_trans, 0.9, 0.999, 1e-8, exit_rel_tol, exit_patience,
                           1 if loss == "tracking" else 0, L.ls_loss_params(lambda_c, inlier_k, alpha_power, 0),
                           1 if exposure else 0, lr_exposure, 1 if joint else 0, 1 if exit_mode == "step" else 0,
                           int(top_k))


def make_pair(P: GaussianSet, Q: GaussianSet, cam: dict, c2w_p, c2w_q, rgbP, depthP, rgbQ, depthQ):
    """Builds an ls_pair; the returned host arrays must outlive the call."""
    hp = np.ascontiguousarray(np.asarray(c2w_p, np.float64)[:, :3, :].reshape(-1, 12), np.float32)
    hq = np.ascontiguousarray(np.asarray(c2w_q, np.float64)[:, :3, :].reshape(-1, 12), np.float32)
    pair = L.ls_pair()
    pair.P = P.to_c()
    pair.Q = Q.to_c()
    pair.vP, pair.vQ = len(hp), len(hq)
    pair.rgbP, pair.depthP = rgbP.data_ptr(), depthP.data_ptr()
    pair.rgbQ, pair.depthQ = rgbQ.data_ptr(), depthQ.data_ptr()
    pair.c2wP = hp.ctypes.data_as(C.c_void_p)
    pair.c2wQ = hq.ctypes.data_as(C.c_void_p)
    pair.K = L.ls_intrinsics(cam["fx"], cam["fy"], cam["cx"], cam["cy"], cam["width"], cam["height"])
    return pair, (hp, hq, rgbP, depthP, rgbQ, depthQ)


_WORK = {}  # device -> grow-only workspace tensor of ls_register_pair


def _workspace(device: int, nbytes: int) -> torch.Tensor:
    w = _WORK.get(device)
    if w is None or w.numel() < nbytes:
        _WORK.pop(device, None)
        w = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=f"cuda:{device}")
        assert w.data_ptr() % 256 == 0
        _WORK[device] = w
    return w


def register_pair(P: GaussianSet, Q: GaussianSet, cam: dict, c2w_p, c2w_q, rgbP, depthP, rgbQ, depthQ,
                  params: L.ls_reg_params | None = None, capacity: int | None = None):
    """Runs ls_register_pair in a workspace kept per device (grown, never
    shrunk, so a stream of pairs allocates only when one needs more than any
    before).  The tile-instance capacity starts at 6 instances per rendered
    Gaussian (or `capacity`); when the call reports more are needed it is
    re-run with 1.5x the reported count.  Returns dict(T [4,4] float64,
    per_view [V,4,4], residual [V], status, iters, exposure, capacity)."""
    params = params or default_params()
    pair, keep = make_pair(P, Q, cam, c2w_p, c2w_q, rgbP, depthP, rgbQ, depthQ)
    nv = pair.vP + pair.vQ
    items = pair.vP * pair.Q.n + pair.vQ * pair.P.n
    cap = int(capacity) if capacity is not None else max(4096, 6 * items)
    per_view = np.zeros((nv, 12), np.float32)
    resid = np.zeros(nv, np.float32)
    expo = np.zeros((nv, 2), np.float32)
    dev = torch.cuda.current_device()
    for _ in range(4):
        res = L.ls_reg_result()
        res.per_view_T = per_view.ctypes.data_as(C.c_void_p)
        res.residual = resid.ctypes.data_as(C.c_void_p)
        res.exposure = expo.ctypes.data_as(C.c_void_p)
        need = L.ls_register_workspace_size(pair, params, cap)
        work = _workspace(dev, need)
        st = L.ls_register_pair(pair, params, work.data_ptr(), work.numel(), cap, res, _stream(),
                                raise_on_error=False)
        if st == L.LS_ERR_CAPACITY and res.instances_required > 0:
            cap = min(int(res.instances_required * 1.5) + 4096, 2**31 - 1)
            continue
        L.check(st)
        break
    else:
        raise L.LsError(L.LS_ERR_CAPACITY, "tile-instance capacity kept overflowing")
    T = np.eye(4)
    T[:3, :] = np.asarray(res.T_PQ, np.float64).reshape(3, 4)
    pv = np.tile(np.eye(4), (nv, 1, 1))
    pv[:, :3, :] = per_view.reshape(nv, 3, 4)
    del keep
    return dict(T=T, per_view=pv, residual=resid.astype(np.float64), status=res.status, iters=res.iters_done,
                exposure=expo.astype(np.float64) if params.exposure else None, capacity=cap)


def fuse_estimates(estimates, residuals, reverse) -> np.ndarray:
    """Host-only Eq. 7 fusion in the library (no GPU needed)."""
    n = len(estimates)
    est = np.ascontiguousarray(np.asarray(estimates, np.float64)[:, :3, :].reshape(n, 12))
    res = np.ascontiguousarray(np.asarray(residuals, np.float64))
    rev = np.ascontiguousarray(np.asarray(reverse, np.int32))
    out = np.zeros(12, np.float64)
    L.ls_fuse_estimates(est.ctypes.data_as(C.c_void_p), res.ctypes.data_as(C.c_void_p),
                        rev.ctypes.data_as(C.c_void_p), n, out.ctypes.data_as(C.c_void_p))
    T = np.eye(4)
    T[:3, :] = out.reshape(3, 4)
    return T


def rotation_error_deg(R, R_gt) -> float:
    c = (np.trace(np.asarray(R)[:3, :3] @ np.asarray(R_gt)[:3, :3].T) - 1.0) / 2.0
    return float(np.degrees(np.arccos(np.clip(c, -1.0, 1.0))))


def translation_error_cm(T, T_gt) -> float:
    return float(100.0 * np.linalg.norm(np.asarray(T)[:3, 3] - np.asarray(T_gt)[:3, 3]))
