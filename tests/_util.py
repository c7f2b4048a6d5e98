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


def grad_elementwise(got, ref, keep=None, rtol: float = 1e-3, floor: float = 1e-3):
    """Element-wise gradient bar: |g - g_ref| <= rtol * max(|g_ref|,
    floor * max|g_ref|) on the rows kept (first axis = Gaussian; the maximum
    is over the whole group).  Returns (violations, worst ratio of error to
    bound)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    gmax = float(np.abs(ref).max()) if ref.size else 0.0
    if keep is not None:
        got, ref = got[keep], ref[keep]
    if ref.size == 0:
        return 0, 0.0
    bound = rtol * np.maximum(np.abs(ref), floor * gmax)
    bound = np.maximum(bound, np.finfo(np.float64).tiny)
    ratio = np.abs(got - ref) / bound
    return int((ratio > 1.0).sum()), float(ratio.max())


def decision_flips(out: dict, gpu: dict, n: int, gpu_radius=None, sign_pairs=(), close_pairs=(),
                   tol: float = 1e-4, near_margin: float = 1e-5):
    """Pixels and Gaussians touched by a discrete decision that the GPU (FP32)
    took, or may have taken, differently from the oracle (FP64):
      - near-ties: pixels whose alpha-skip / clamp / stop decision lies
        within relative `near_margin` of its threshold (the oracle reports
        the margin); a flip there can change the image by less than `tol`
        and still move the gradients;
      - pixels whose n_last differs, or whose colour, depth or alpha differs
        by more than `tol` relative (1 m unit): a flipped alpha-skip, clamp
        or stop decision there;
      - pixels where an L1 loss took a different sign: `sign_pairs` holds
        (GPU sign image, oracle residual image) pairs of one shape; where the
        GPU's sign is not available, `close_pairs` holds (oracle residual
        image, tolerance) pairs and marks every pixel whose residual is
        within the tolerance of zero (a sign FP32 may take differently);
      - Gaussians whose radius differs (gpu_radius [n], optional): every
        pixel of the tiles of their oracle rectangle grown by one tile.
    A flipped decision changes the transmittance seen by every entry of the
    pixel, so every list entry visited at a flipped pixel (up to the later
    of the two stop positions) is marked.  Returns (Gaussian mask [n], pixel
    mask [H, W])."""
    H, W = np.asarray(out["n_last"]).shape
    n_last_o = np.asarray(out["n_last"])
    n_last_g = np.asarray(gpu["n_last"]).reshape(H, W)
    flip = (n_last_g != n_last_o) | (np.asarray(out["margin"]) < near_margin)
    for key in ("rgb", "depth", "alpha"):
        o = np.asarray(out[key].detach().numpy() if hasattr(out[key], "detach") else out[key], np.float64)
        g = np.asarray(gpu[key], np.float64).reshape(o.shape)
        bad = np.abs(g - o) > tol * np.maximum(np.abs(o), 1.0)
        flip |= bad.reshape(-1, H, W).any(axis=0)
    for g_sign, o_res in sign_pairs:
        o_res = np.asarray(o_res, np.float64)
        g_sign = np.asarray(g_sign, np.float64).reshape(o_res.shape)
        flip |= (np.sign(g_sign) != np.sign(o_res)).reshape(-1, H, W).any(axis=0)
    for o_res, ctol in close_pairs:
        o_res = np.asarray(o_res, np.float64)
        flip |= ((np.abs(o_res) <= ctol) & (o_res != 0)).reshape(-1, H, W).any(axis=0)
    pr = out["proj"]
    mask = np.zeros(n, bool)
    tiles_x, tiles_y = (W + 15) // 16, (H + 15) // 16
    if gpu_radius is not None:
        moved = np.asarray(gpu_radius).reshape(-1) != np.asarray(pr["radius"])
        mask |= moved
        x0, x1, y0, y1 = (np.asarray(a) for a in pr["rect"])
        for gi in np.nonzero(moved)[0]:
            ty0, ty1 = max(int(y0[gi]) - 1, 0), min(int(y1[gi]) + 1, tiles_y)
            tx0, tx1 = max(int(x0[gi]) - 1, 0), min(int(x1[gi]) + 1, tiles_x)
            flip[ty0 * 16:ty1 * 16, tx0 * 16:tx1 * 16] = True
    _, gid, ranges = out["bins"]
    gid = np.asarray(gid)
    for y, x in zip(*np.nonzero(flip)):
        s, e = ranges[(y // 16) * tiles_x + x // 16]
        k = min(max(int(n_last_o[y, x]), int(n_last_g[y, x])) + 1, e - s)
        mask[gid[s:s + k]] = True
    return mask, flip


def check_gradients(pairs, exclude=None, tag: str = "", max_frac: float = 1e-3, max_ratio: float = 3.0):
    """The gradient bars against the oracle, per parameter group
    (name, GPU [n, k] or [n], oracle same shape):
      - norm clause: |g - g_ref|_2 / |g_ref|_2 < 1e-3 over every Gaussian;
      - element clause on the Gaussians not excluded (decision flips):
        |g - g_ref| <= 1e-3 max(|g_ref|, 1e-3 |g_ref|_inf).  FP32 summation
        over a Gaussian's pixels leaves an absolute error of a few 1e-6
        |g_ref|_inf, so elements that cancel down to the floor may exceed it:
        at most `max_frac` of the elements (and one), each within `max_ratio`
        of its bound, and every kept element within 1e-3 max(|g_ref|,
        1e-2 |g_ref|_inf).
    Returns a summary string (counts and worst ratios)."""
    out = []
    for name, got, ref in pairs:
        got = np.asarray(got, np.float64)
        ref = np.asarray(ref, np.float64)
        err = rel_err(got, ref)
        assert err < 1e-3, (tag, name, "norm", err)
        keep = None if exclude is None else ~np.asarray(exclude)
        nb, worst = grad_elementwise(got, ref, keep)
        nb2, worst2 = grad_elementwise(got, ref, keep, floor=1e-2)
        assert nb2 == 0, (tag, name, "element (floor 1e-2)", nb2, worst2)
        assert nb <= max(1, int(max_frac * got.size)) and worst <= max_ratio, (tag, name, "element", nb, worst)
        out.append(f"{name}: norm {err:.1e}, element {nb} over (worst {worst:.2f})")
    return f"{tag} " + "; ".join(out)


def render_flips(b, r, o, n, **kw):
    """Gaussians of render r of batch b touched by a decision the GPU took
    differently from the oracle render o (see decision_flips).  The pixels
    whose compositing decisions flipped must sit at a decision margin below
    1e-3 and be at most 0.1 % of the render; loss-sign flips (passed in
    `kw`) are added after that check."""
    o_, e_ = int(b.item_off[r]), int(b.item_off[r + 1])
    v = {k: t.cpu().numpy() for k, t in b.image_views(r).items()}
    radius = b.radius[o_:e_].cpu().numpy()
    excl, flip = decision_flips(o, v, n, radius)
    assert flip.mean() <= 1e-3, int(flip.sum())
    moved = radius != np.asarray(o["proj"]["radius"])
    assert np.all(np.asarray(o["margin"])[flip & ~rect_pixels(o, moved)] < 1e-3)
    if kw:
        excl, flip = decision_flips(o, v, n, radius, **kw)
        assert flip.mean() <= 1e-3, int(flip.sum())
    return excl


def rect_pixels(o, which):
    """Pixels of the tiles of the oracle rectangles (grown by one tile) of the
    Gaussians in `which`."""
    H, W = np.asarray(o["n_last"]).shape
    px = np.zeros((H, W), bool)
    x0, x1, y0, y1 = (np.asarray(a) for a in o["proj"]["rect"])
    for gi in np.nonzero(which)[0]:
        px[max(int(y0[gi]) - 1, 0) * 16:(int(y1[gi]) + 1) * 16, max(int(x0[gi]) - 1, 0) * 16:(int(x1[gi]) + 1) * 16] = True
    return px
