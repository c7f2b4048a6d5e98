"""FP64 oracle of the differentiable 3D-Gaussian-splat rasterizer.

TEST INFRASTRUCTURE ONLY (see the package docstring): never imported by the
product path.

The paper (Sec. 3.1, Eq. 1) represents a submap as a set of Gaussians with a
mean, a covariance, an opacity and an RGB colour, renders colour and depth from
a pose (Sec. 3.1 tracking loss, Eq. 2; Sec. 3.2 registration), and inherits the
rasterizer itself from 3D Gaussian Splatting.  The paper does not spell out the
rendering steps, so each step below is a stated reading, numbered R1-R17
(one choice each where the paper is silent):

  R1  opacity  o = sigmoid(opacity_logit)
  R2  colour   c = rgb (SH degree 0, no clamp; the paper drops SH, Sec. 3.3)
  R3  Sigma = M M^T,  M = R(q/|q|) diag(exp(log_scale)),  q = (w, x, y, z)
  R4  pose     a rigid correction Delta = (q_d, t_d) applied in the camera
               frame of the render after its world-to-camera transform:
               p = R(q_d)(R_cw mu + t_cw) + t_d.  This is the supplement's
               tracking parametrisation (the submap moved by the inverse
               relative pose, rendered from the previous camera).
  R5  exact EWA Jacobian, no off-axis clamp
  R6  2D low-pass dilation  +EPS_2D * I  (0.3 px^2)
  R7  pixel (i, j) sampled at (i + 0.5, j + 0.5)
  R8  near plane  z > NEAR_Z = 0.2 m
  R9  radius  r = ceil(3 sqrt(lambda_max))   (decided in FP32)
  R10 16x16 tiles, rect [floor((u-r)/16), floor((u+r)/16)+1) clamped (FP32)
  R11 list order (tile, float32 depth bits, Gaussian index)
  R12 alpha = min(ALPHA_MAX, o exp(-s)); skip if alpha < ALPHA_MIN; stop
      *before* the entry whose compositing would take T below T_STOP
  R13 background 0 unless given; R14 depth = sum w z (not normalised)
  R15 loss = mean over pixels with target depth > 0 of sum_c|C-C*| + |D-D*|
  R16 d|x|/dx = sign(x) with sign(0) = 0 (torch.abs)
  R17 no gradient through the alpha clamp when it is active
  R24 tracking loss (Eq. 2 with the supplement's masks), per render:
        L = (1/|Omega|) sum_{p in Omega} M_in M_a (lc sum_c|C-C*| + (1-lc)|D-D*|)
      Omega = pixels with target depth > 0 (pixels without a valid depth
      measurement are excluded); M_a = alpha^k (k = 3, a per-pixel weight,
      no gradient flows through it); M_in = [e <= K_IN * median(e)], e =
      |D - D*| over Omega, K_IN = 50, the median being the lower one (the
      element of rank floor((n-1)/2) in ascending order).  The normalisation
      by |Omega| instead of a plain sum leaves Adam's steps unchanged and
      keeps residuals of views with different coverage comparable.  e, the
      median and the inlier test are evaluated in FP32 on FP32 inputs, the
      precision of the GPU path, since they decide a mask.

Decisions that turn floating point into integers or control flow (radius,
tile rect, cull, list order) are taken in FP32 on FP32-rounded inputs, the
precision the GPU kernels use; margins to each decision are reported so that
tests can tell a genuine mismatch from a rounding near-tie.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

F64 = torch.float64

NEAR_Z = 0.2
EPS_2D = 0.3
TILE = 16
# Thresholds are the FP32 values of the stated constants, used on both sides.
ALPHA_MIN = float(np.float32(1.0 / 255.0))
ALPHA_MAX = float(np.float32(0.99))
T_STOP = float(np.float32(1e-4))


@dataclass
class Camera:
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    @property
    def tiles_x(self) -> int:
        return (self.width + TILE - 1) // TILE

    @property
    def tiles_y(self) -> int:
        return (self.height + TILE - 1) // TILE


def quat_to_rotmat(q: torch.Tensor) -> torch.Tensor:
    """Rotation matrix of the unit quaternion q/|q|, q = (w, x, y, z).

    Standard Hamilton convention: R v = q v q*.
    """
    q = q / torch.linalg.norm(q, dim=-1, keepdim=True)
    w, x, y, z = q.unbind(-1)
    r = torch.stack(
        [
            1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
            2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
            2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y),
        ],
        dim=-1,
    )
    return r.reshape(q.shape[:-1] + (3, 3))


def identity_pose() -> torch.Tensor:
    return torch.tensor([1.0, 0, 0, 0, 0, 0, 0], dtype=F64)


def covariance3d(log_scale: torch.Tensor, quat: torch.Tensor) -> torch.Tensor:
    """Sigma = R S S^T R^T with S = diag(exp(log_scale)) (reading R3; the paper
    names Sigma and per-axis scales s_k, Sec. 3.1 Eq. 1 and Eq. 5)."""
    m = quat_to_rotmat(quat) * torch.exp(log_scale)[..., None, :]
    return m @ m.transpose(-1, -2)


def camera_transform(w2c: torch.Tensor, pose: torch.Tensor):
    """Effective world-to-camera (W, t) = Delta o w2c (reading R4)."""
    r_cw, t_cw = w2c[:, :3], w2c[:, 3]
    r_d = quat_to_rotmat(pose[:4])
    return r_d @ r_cw, r_d @ t_cw + pose[4:7]


def _f32(x) -> np.ndarray:
    return np.asarray(x.detach().numpy() if torch.is_tensor(x) else x, dtype=np.float64).astype(np.float32)


def radius_f32(a32: np.ndarray, b32: np.ndarray, c32: np.ndarray) -> np.ndarray:
    """r = ceil(3 sqrt(lambda_max)) of [[a, b], [b, c]], in FP32 (R9)."""
    half = np.float32(0.5)
    mid = half * (a32 + c32)
    hd = half * (a32 - c32)
    lam = mid + np.sqrt(hd * hd + b32 * b32)
    return np.ceil(np.float32(3.0) * np.sqrt(lam)).astype(np.int64)


def tile_rect_f32(u32: np.ndarray, v32: np.ndarray, radius: np.ndarray, cam: Camera):
    """Conservative tile rectangle [x0, x1) x [y0, y1) in tile units (R10).

    Computed in FP32 from FP32 centres and the integer radius, clamped to the
    tile grid.  Returns int64 arrays (x0, x1, y0, y1).
    """
    r32 = radius.astype(np.float32)
    inv = np.float32(1.0 / TILE)
    x0 = np.floor((u32 - r32) * inv).astype(np.int64)
    x1 = np.floor((u32 + r32) * inv).astype(np.int64) + 1
    y0 = np.floor((v32 - r32) * inv).astype(np.int64)
    y1 = np.floor((v32 + r32) * inv).astype(np.int64) + 1
    tx, ty = cam.tiles_x, cam.tiles_y
    return (np.clip(x0, 0, tx), np.clip(x1, 0, tx), np.clip(y0, 0, ty), np.clip(y1, 0, ty))


def project(mean, log_scale, quat, cam: Camera, w2c, pose=None):
    """Per-Gaussian EWA projection (readings R3-R10).

    mean [N,3], log_scale [N,3], quat [N,4] (float64 tensors, may require
    grad); w2c [3,4]; pose [7] (q_w, q_x, q_y, q_z, t_x, t_y, t_z) or None.

    Returns a dict of float64 tensors u, v, conic [N,3] (A, B, C with
    sigma = A dx^2/2 + B dx dy + C dy^2/2), depth z, the camera-space point
    p [N,3] and covariance, plus NumPy decision outputs: radius (int64,
    0 = culled), tiles (count), rect, and FP32 copies u32, v32, z32 that the
    binning uses.  `margin_px` is the distance, in pixels, of the radius and
    tile-rect decisions to their nearest flip.
    """
    if pose is None:
        pose = identity_pose()
    w, t = camera_transform(torch.as_tensor(w2c, dtype=F64), pose)
    p = mean @ w.T + t
    sigma_c = w @ covariance3d(log_scale, quat) @ w.T
    x, y, z = p.unbind(-1)
    n = mean.shape[0]
    zero = torch.zeros_like(z)
    j = torch.stack(
        [
            torch.stack([cam.fx / z, zero, -cam.fx * x / (z * z)], -1),
            torch.stack([zero, cam.fy / z, -cam.fy * y / (z * z)], -1),
        ],
        -2,
    )  # [N,2,3]
    s2 = j @ sigma_c @ j.transpose(-1, -2) + EPS_2D * torch.eye(2, dtype=F64)
    a, b, c = s2[:, 0, 0], s2[:, 0, 1], s2[:, 1, 1]
    det = a * c - b * b
    conic = torch.stack([c / det, -b / det, a / det], -1)
    u = cam.fx * x / z + cam.cx
    v = cam.fy * y / z + cam.cy

    # ---- decisions, taken in FP32 on FP32-rounded values (R8-R10)
    a32, b32, c32 = _f32(a), _f32(b), _f32(c)
    z32 = _f32(z)
    u32, v32 = _f32(u), _f32(v)
    with np.errstate(invalid="ignore", over="ignore"):
        det32 = a32 * c32 - b32 * b32
        visible = (z32 > np.float32(NEAR_Z)) & (det32 > 0)
        radius = np.where(visible, radius_f32(a32, b32, c32), 0)
    x0, x1, y0, y1 = tile_rect_f32(u32, v32, radius, cam)
    tiles = np.where(radius > 0, np.maximum(x1 - x0, 0) * np.maximum(y1 - y0, 0), 0)
    radius = np.where(tiles > 0, radius, 0)
    tiles = np.where(radius > 0, tiles, 0)

    # ---- margins (float64) of the integer decisions
    with torch.no_grad(), np.errstate(invalid="ignore", over="ignore"):
        a64, b64, c64 = a.numpy(), b.numpy(), c.numpy()
        lam = 0.5 * (a64 + c64) + np.sqrt((0.5 * (a64 - c64)) ** 2 + b64 * b64)
        r_real = 3.0 * np.sqrt(np.maximum(lam, 0.0))
        m_r = np.abs(r_real - np.round(r_real))
        u64, v64 = u.numpy(), v.numpy()
        m_rect = np.full(n, np.inf)
        for e in (u64 - radius, u64 + radius, v64 - radius, v64 + radius):
            m_rect = np.minimum(m_rect, np.abs(e - TILE * np.round(e / TILE)))
        m_near = np.abs(z.numpy() - NEAR_Z)
    margin_px = np.minimum(np.minimum(m_r, m_rect), m_near * cam.fx)
    return dict(
        u=u, v=v, conic=conic, depth=z, p=p, cov2d=s2, cov_cam=sigma_c,
        radius=radius.astype(np.int64), tiles=tiles.astype(np.int64),
        rect=(x0, x1, y0, y1), u32=u32, v32=v32, z32=z32, margin_px=margin_px,
    )


def bin_sort(u32, v32, z32, radius, cam: Camera):
    """Tile binning and ordering of one render (R10, R11).

    Inputs are FP32 centres/depths and integer radii (0 = culled).  Every
    Gaussian is listed in every tile of its rect; the list is ordered by
    (tile index, FP32 depth bit pattern, Gaussian index) - for positive depths
    the bit pattern orders like the value.  Returns (tile_of, gid, ranges)
    with ranges[t] = [start, end) into the sorted list.
    """
    u32 = np.asarray(u32, np.float32)
    v32 = np.asarray(v32, np.float32)
    z32 = np.asarray(z32, np.float32)
    radius = np.asarray(radius, np.int64)
    x0, x1, y0, y1 = tile_rect_f32(u32, v32, radius, cam)
    tiles_out, gids_out, keys_out = [], [], []
    zbits = z32.view(np.uint32)
    for g in np.nonzero(radius > 0)[0]:
        for ty in range(y0[g], y1[g]):
            for tx in range(x0[g], x1[g]):
                tiles_out.append(ty * cam.tiles_x + tx)
                gids_out.append(g)
                keys_out.append(zbits[g])
    tile_of = np.asarray(tiles_out, np.int64)
    gid = np.asarray(gids_out, np.int64)
    key = np.asarray(keys_out, np.uint64)
    order = np.lexsort((gid, key, tile_of))
    tile_of, gid = tile_of[order], gid[order]
    ntiles = cam.tiles_x * cam.tiles_y
    ranges = np.zeros((ntiles, 2), np.int64)
    if len(tile_of):
        starts = np.searchsorted(tile_of, np.arange(ntiles), side="left")
        ends = np.searchsorted(tile_of, np.arange(ntiles), side="right")
        ranges[:, 0] = np.where(ends > starts, starts, 0)
        ranges[:, 1] = np.where(ends > starts, ends, 0)
    return tile_of, gid, ranges


def composite(u, v, conic, opacity, rgb, depth, gid, ranges, cam: Camera, bg=None, with_margins=True,
              tiles_subset=None, with_decisions=False):
    """Front-to-back alpha compositing over each tile's ordered list (R7, R12-R14).

    u, v, depth [N], conic [N,3], opacity [N], rgb [N,3]: float64 tensors
    (differentiable).  gid/ranges from bin_sort.  For every pixel the entries
    of its tile's list are visited in order:
        s = A dx^2/2 + B dx dy + C dy^2/2 with d = pixel centre - (u, v)
        skip if s < 0;  alpha = min(ALPHA_MAX, o exp(-s));  skip if alpha < ALPHA_MIN
        stop before this entry if T (1 - alpha) < T_STOP
        else w = alpha T;  C += w c;  D += w z;  T *= (1 - alpha)
    Returns rgb [3,H,W], depth [H,W], alpha = 1 - T_final [H,W], T_final,
    n_last [H,W] (entries visited before the stop, or the list length), and
    the per-pixel relative margin of the alpha/clamp/stop decisions (NumPy).

    `tiles_subset` restricts the work to the listed tile indices (other pixels
    are left at their background values); used for sampled checks at size.

    `with_decisions` adds "decisions": every discrete choice of the loop (per
    tile, per pixel and list entry: skipped, clamped at ALPHA_MAX, composited)
    packed into one byte string, so that two renders can be checked for the
    same decisions (finite differences must not straddle a threshold).
    """
    if bg is None:
        bg = torch.zeros(3, dtype=F64)
    bg = torch.as_tensor(bg, dtype=F64)
    W, H = cam.width, cam.height
    tx_n = cam.tiles_x
    n_last = np.zeros((H, W), np.int64)
    margin = np.full((H, W), np.inf)
    img_rgb = bg[:, None, None].expand(3, H, W).clone()
    img_d = torch.zeros(H, W, dtype=F64)
    img_t = torch.ones(H, W, dtype=F64)
    rows_rgb, rows_d, rows_t, idx_y, idx_x = [], [], [], [], []
    decisions = []
    tiles = range(cam.tiles_x * cam.tiles_y) if tiles_subset is None else tiles_subset
    for t in tiles:
        ty, tx = divmod(int(t), tx_n)
        ys = np.arange(ty * TILE, min((ty + 1) * TILE, H))
        xs = np.arange(tx * TILE, min((tx + 1) * TILE, W))
        if len(ys) == 0 or len(xs) == 0:
            continue
        yy, xx = np.meshgrid(ys, xs, indexing="ij")
        yy, xx = yy.ravel(), xx.ravel()
        s, e = ranges[t]
        ids = torch.as_tensor(np.asarray(gid[s:e], np.int64))
        k = len(ids)
        px = torch.as_tensor(xx + 0.5, dtype=F64)[:, None]
        py = torch.as_tensor(yy + 0.5, dtype=F64)[:, None]
        if k == 0:
            c_t = bg[None, :].expand(len(xx), 3)
            d_t = torch.zeros(len(xx), dtype=F64)
            t_t = torch.ones(len(xx), dtype=F64)
            n_last[yy, xx] = 0
        else:
            dx = px - u[ids][None, :]
            dy = py - v[ids][None, :]
            ca, cb, cc = conic[ids, 0][None, :], conic[ids, 1][None, :], conic[ids, 2][None, :]
            sig = 0.5 * (ca * dx * dx + cc * dy * dy) + cb * dx * dy
            gval = opacity[ids][None, :] * torch.exp(-sig)
            alpha = torch.clamp(gval, max=ALPHA_MAX)
            with torch.no_grad():
                skip = (sig < 0) | (alpha < ALPHA_MIN)
                a_np = torch.where(skip, torch.zeros_like(alpha), alpha).numpy()
                one_m = 1.0 - a_np
                t_after = np.cumprod(one_m, axis=1)          # T after entry k (if composited)
                t_before = np.concatenate([np.ones((len(xx), 1)), t_after[:, :-1]], axis=1)
                stop = (~skip.numpy()) & (t_after < T_STOP)
                has_stop = stop.any(axis=1)
                first = np.where(has_stop, stop.argmax(axis=1), k)
                keep = (np.arange(k)[None, :] < first[:, None]) & (~skip.numpy())
                n_last[yy, xx] = first
                if with_decisions:
                    decisions.append(np.packbits(np.stack([skip.numpy(), (gval >= ALPHA_MAX).numpy(), keep])).tobytes())
                if with_margins:
                    visited = np.arange(k)[None, :] <= np.minimum(first, k - 1)[:, None]
                    g_np = gval.numpy()
                    ok_sig = sig.numpy() >= 0
                    m1 = np.where(ok_sig, np.abs(g_np - ALPHA_MIN) / ALPHA_MIN, np.inf)
                    m2 = np.where(ok_sig, np.abs(g_np - ALPHA_MAX) / ALPHA_MAX, np.inf)
                    m3 = np.where((~skip.numpy()), np.abs(t_before * one_m - T_STOP) / T_STOP, np.inf)
                    mm = np.where(visited, np.minimum(np.minimum(m1, m2), m3), np.inf)
                    margin[yy, xx] = mm.min(axis=1)
            keep_t = torch.as_tensor(keep)
            a_eff = torch.where(keep_t, alpha, torch.zeros_like(alpha))
            one_minus = 1.0 - a_eff
            t_incl = torch.cumprod(one_minus, dim=1)
            t_excl = torch.cat([torch.ones(len(xx), 1, dtype=F64), t_incl[:, :-1]], dim=1)
            wgt = a_eff * t_excl
            t_t = t_incl[:, -1]
            c_t = wgt @ rgb[ids] + t_t[:, None] * bg[None, :]
            d_t = wgt @ depth[ids]
        rows_rgb.append(c_t)
        rows_d.append(d_t)
        rows_t.append(t_t)
        idx_y.append(yy)
        idx_x.append(xx)
    if rows_rgb:
        yy = torch.as_tensor(np.concatenate(idx_y))
        xx = torch.as_tensor(np.concatenate(idx_x))
        c_all = torch.cat(rows_rgb, 0)
        d_all = torch.cat(rows_d, 0)
        t_all = torch.cat(rows_t, 0)
        img_rgb = _scatter_rgb(img_rgb, yy, xx, c_all)
        img_d = img_d.index_put((yy, xx), d_all)
        img_t = img_t.index_put((yy, xx), t_all)
    img_a = 1.0 - img_t
    out = dict(rgb=img_rgb, depth=img_d, alpha=img_a, T_final=img_t, n_last=n_last, margin=margin)
    if with_decisions:
        out["decisions"] = b"".join(decisions)
    return out


def _scatter_rgb(img, yy, xx, vals):
    chans = [img[ch].index_put((yy, xx), vals[:, ch]) for ch in range(3)]
    return torch.stack(chans, 0)


def render(gauss: dict, cam: Camera, w2c, pose=None, bg=None, tiles_subset=None, with_margins=True,
           with_decisions=False):
    """Full render of one job: project -> bin -> composite.

    gauss: dict of float64 tensors mean [N,3], log_scale [N,3], quat [N,4],
    opacity_logit [N], rgb [N,3].  Returns composite()'s dict plus the
    projection dict under "proj" and the binning under "bins".
    """
    pr = project(gauss["mean"], gauss["log_scale"], gauss["quat"], cam, w2c, pose)
    tile_of, gid, ranges = bin_sort(pr["u32"], pr["v32"], pr["z32"], pr["radius"], cam)
    opacity = torch.sigmoid(gauss["opacity_logit"])
    out = composite(pr["u"], pr["v"], pr["conic"], opacity, gauss["rgb"], pr["depth"], gid, ranges, cam,
                    bg=bg, tiles_subset=tiles_subset, with_margins=with_margins, with_decisions=with_decisions)
    out["proj"] = pr
    out["bins"] = (tile_of, gid, ranges)
    return out


def loss_l1(rgb, depth, tgt_rgb, tgt_depth):
    """Registration/tracking photometric + geometric L1 (R15, R16).

    L = (1/|Omega|) sum_{p in Omega} (sum_c |C_c - C*_c| + |D - D*|),
    Omega = pixels whose target depth is > 0.  Returns 0 when Omega is empty.
    """
    valid = (torch.as_tensor(tgt_depth) > 0).to(F64)
    cnt = valid.sum()
    if cnt.item() == 0:
        return (rgb.sum() + depth.sum()) * 0.0
    per_px = (torch.abs(rgb - tgt_rgb)).sum(0) + torch.abs(depth - tgt_depth)
    return (per_px * valid).sum() / cnt


def lower_median_f32(x: np.ndarray) -> np.float32:
    """Element of rank floor((n-1)/2) of the ascending order of x (float32);
    0 for an empty array."""
    x = np.sort(np.asarray(x, np.float32).ravel())
    return x[(x.size - 1) // 2] if x.size else np.float32(0.0)


def tracking_masks(alpha, depth, tgt_depth, alpha_power: int = 3, inlier_k: float = 50.0):
    """Per-pixel weight M_in * M_a * [p in Omega] of R24 (float64, constant),
    the FP32 median depth error and |Omega|.  alpha_power = 0 drops M_a;
    inlier_k <= 0 drops M_in."""
    d32 = np.asarray(torch.as_tensor(depth).detach().cpu().numpy(), np.float32)
    t32 = np.asarray(torch.as_tensor(tgt_depth).detach().cpu().numpy(), np.float32)
    valid = t32 > 0
    err = np.abs(d32 - t32)
    med = lower_median_f32(err[valid])
    mask = valid.copy()
    if inlier_k > 0:
        mask &= err <= np.float32(inlier_k) * med
    w = torch.as_tensor(mask.astype(np.float64))
    if alpha_power > 0:
        w = w * torch.as_tensor(alpha).detach().to(F64) ** alpha_power
    return w, float(med), int(valid.sum())


def loss_tracking(rgb, depth, alpha, tgt_rgb, tgt_depth, lambda_c: float = 0.6, alpha_power: int = 3,
                  inlier_k: float = 50.0):
    """Tracking / keyframe-localisation loss of R24 (Eq. 2 with its masks);
    rgb [3,H,W], depth and alpha [H,W].  Returns (loss, median depth error)."""
    w, med, n = tracking_masks(alpha, depth, tgt_depth, alpha_power, inlier_k)
    if n == 0:
        return (rgb.sum() + depth.sum()) * 0.0, med
    per_px = lambda_c * torch.abs(rgb - tgt_rgb).sum(0) + (1.0 - lambda_c) * torch.abs(depth - tgt_depth)
    return (w * per_px).sum() / n, med


def to_f64(gauss_np: dict, requires_grad=False) -> dict:
    """Convert a SoA NumPy Gaussian set ([3,N] etc.) to the oracle's AoS float64 tensors."""
    out = {
        "mean": torch.as_tensor(np.asarray(gauss_np["mean"], np.float64).T.copy()),
        "log_scale": torch.as_tensor(np.asarray(gauss_np["log_scale"], np.float64).T.copy()),
        "quat": torch.as_tensor(np.asarray(gauss_np["quat"], np.float64).T.copy()),
        "opacity_logit": torch.as_tensor(np.asarray(gauss_np["opacity_logit"], np.float64).copy()),
        "rgb": torch.as_tensor(np.asarray(gauss_np["rgb"], np.float64).T.copy()),
    }
    if requires_grad:
        for v in out.values():
            v.requires_grad_(True)
    return out


def brute_force_pixel(gauss: dict, cam: Camera, w2c, pose, px: int, py: int, bg=None):
    """Plain per-pixel compositing with a Python loop (pin for the tiled path).

    Lists every Gaussian whose tile rect contains the pixel's tile, orders the
    list by (FP32 depth, index) and composites it entry by entry in float64.
    Returns (rgb[3], depth, T_final, n_last).
    """
    with torch.no_grad():
        pr = project(gauss["mean"], gauss["log_scale"], gauss["quat"], cam, w2c, pose)
        x0, x1, y0, y1 = pr["rect"]
        tx, ty = px // TILE, py // TILE
        cand = [g for g in range(len(pr["radius"]))
                if pr["radius"][g] > 0 and x0[g] <= tx < x1[g] and y0[g] <= ty < y1[g]]
        cand.sort(key=lambda g: (float(pr["z32"][g]), g))
        opac = torch.sigmoid(gauss["opacity_logit"]).numpy()
        rgbs = gauss["rgb"].numpy()
        T = 1.0
        col = [0.0, 0.0, 0.0]
        dep = 0.0
        n_last = len(cand)
        for i, g in enumerate(cand):
            dx = px + 0.5 - float(pr["u"][g])
            dy = py + 0.5 - float(pr["v"][g])
            A, B, C = (float(val) for val in pr["conic"][g])
            s = 0.5 * (A * dx * dx + C * dy * dy) + B * dx * dy
            if s < 0:
                continue
            a = min(ALPHA_MAX, float(opac[g]) * math.exp(-s))
            if a < ALPHA_MIN:
                continue
            if T * (1 - a) < T_STOP:
                n_last = i
                break
            w = a * T
            for ch in range(3):
                col[ch] += w * float(rgbs[g, ch])
            dep += w * float(pr["depth"][g])
            T *= 1 - a
        if bg is not None:
            col = [col[ch] + T * float(bg[ch]) for ch in range(3)]
        return col, dep, T, n_last
