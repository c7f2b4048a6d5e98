"""Seeded synthetic inputs shaped like the paper's RGB-D workloads.

This module only draws random numbers and lays them out; it holds none of the
rendering or registration arithmetic, so both the GPU path and the CPU oracle
can take their inputs from it.  Every array is float32, structure-of-arrays:
mean [3,N], log_scale [3,N], quat [4,N] (w, x, y, z, unnormalised),
opacity_logit [N], rgb [3,N].

The paper's datasets (Replica, TUM-RGBD, ScanNet, ScanNet++) are not used;
these generators stand in for them with the Gaussian counts the paper reports
(about 0.2-0.33 M per scene, supplement table of Gaussian counts) and its
per-frame motion scale (supplement table of average frame motion).
"""

from __future__ import annotations

import math

import numpy as np


def camera(fx, fy, cx, cy, width, height) -> dict:
    return dict(fx=float(fx), fy=float(fy), cx=float(cx), cy=float(cy), width=int(width), height=int(height))


def identity_w2c() -> np.ndarray:
    return np.concatenate([np.eye(3), np.zeros((3, 1))], 1).astype(np.float32)


def identity_pose() -> np.ndarray:
    return np.array([1, 0, 0, 0, 0, 0, 0], np.float32)


def gaussians_in_box(rng: np.random.Generator, n: int, lo, hi, log_scale_mu=math.log(0.02),
                     log_scale_sd=0.3) -> dict:
    """N Gaussians with means uniform in the box [lo, hi] (metres), log-scales
    N(log 0.02, 0.3), random unit quaternions (normalised N(0, I4) draws),
    opacity logits N(0, 1) and RGB U[0, 1]."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    mean = lo[:, None] + (hi - lo)[:, None] * rng.random((3, n))
    log_scale = rng.normal(log_scale_mu, log_scale_sd, (3, n))
    q = rng.normal(0.0, 1.0, (4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    opacity_logit = rng.normal(0.0, 1.0, n)
    rgb = rng.random((3, n))
    return dict(
        mean=mean.astype(np.float32), log_scale=log_scale.astype(np.float32), quat=q.astype(np.float32),
        opacity_logit=opacity_logit.astype(np.float32), rgb=rgb.astype(np.float32),
    )


def random_axis(rng: np.random.Generator) -> np.ndarray:
    a = rng.normal(0.0, 1.0, 3)
    return a / np.linalg.norm(a)


def axis_angle_pose(axis, angle_rad: float, trans) -> np.ndarray:
    """Pose 7-vector (q_w, q_x, q_y, q_z, t_x, t_y, t_z) of a rotation by
    `angle_rad` about the unit `axis` and a translation."""
    axis = np.asarray(axis, np.float64)
    h = 0.5 * angle_rad
    q = np.concatenate([[math.cos(h)], math.sin(h) * axis])
    return np.concatenate([q, np.asarray(trans, np.float64)]).astype(np.float32)


def perturbation(rng: np.random.Generator, deg: float, metres: float) -> np.ndarray:
    """A rotation of `deg` degrees about a random axis plus a translation of
    `metres` in a random direction, as a pose 7-vector."""
    return axis_angle_pose(random_axis(rng), math.radians(deg), metres * random_axis(rng))


def scene_small(seed: int = 0, n: int = 4096) -> dict:
    """Plain single-view workload: 4,096 Gaussians in a 2 m cube centred
    2.5 m in front of an identity camera, 160x120 pinhole, f = 150, and a
    target pose perturbed by 2 deg / 3 cm."""
    rng = np.random.default_rng(seed)
    g = gaussians_in_box(rng, n, (-1.0, -1.0, 1.5), (1.0, 1.0, 3.5))
    return dict(gauss=g, cam=camera(150, 150, 80, 60, 160, 120), w2c=identity_w2c(),
                target_pose=perturbation(rng, 2.0, 0.03))


def scene_room_volume(seed: int = 1, n: int = 200_000) -> dict:
    """Tracking/mapping-shaped workload: 200k Gaussians in a 6 x 3 x 4 m
    room-shaped box in front of the camera (x in [-3, 3], y in [-1.5, 1.5],
    z in [0.5, 4.5]), 1200x680 pinhole, f = 600, target pose 2 deg / 3 cm."""
    rng = np.random.default_rng(seed)
    g = gaussians_in_box(rng, n, (-3.0, -1.5, 0.5), (3.0, 1.5, 4.5))
    return dict(gauss=g, cam=camera(600, 600, 600, 340, 1200, 680), w2c=identity_w2c(),
                target_pose=perturbation(rng, 2.0, 0.03))


def scene_tiny(seed: int, n: int, width: int, height: int, f: float, depth_range=(1.5, 3.0),
               half_extent=0.8, log_scale_mu=math.log(0.05)) -> dict:
    """Small scene for brute-force and finite-difference checks."""
    rng = np.random.default_rng(seed)
    zc = 0.5 * (depth_range[0] + depth_range[1])
    hz = 0.5 * (depth_range[1] - depth_range[0])
    g = gaussians_in_box(rng, n, (-half_extent, -half_extent, zc - hz), (half_extent, half_extent, zc + hz),
                         log_scale_mu=log_scale_mu)
    return dict(gauss=g, cam=camera(f, f, width / 2, height / 2, width, height), w2c=identity_w2c(),
                target_pose=perturbation(rng, 2.0, 0.03))


def random_image_grads(rng: np.random.Generator, n_pix: int, scale=1.0) -> dict:
    """Upstream gradients dL/d(rgb [3,P], depth [P], alpha [P]) for backward tests."""
    return dict(
        rgb=(scale * rng.normal(0.0, 1.0, (3, n_pix))).astype(np.float32),
        depth=(scale * rng.normal(0.0, 1.0, n_pix)).astype(np.float32),
        alpha=(scale * rng.normal(0.0, 1.0, n_pix)).astype(np.float32),
    )


def look_at_c2w(position, target, up=(0.0, 1.0, 0.0)) -> np.ndarray:
    """Camera-to-world 4x4 of a camera at `position` looking at `target`
    (camera axes: x right, y down, z forward; world y up)."""
    position = np.asarray(position, np.float64)
    z = np.asarray(target, np.float64) - position
    z /= np.linalg.norm(z)
    x = np.cross(z, np.asarray(up, np.float64))
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    out = np.eye(4)
    out[:3, 0], out[:3, 1], out[:3, 2], out[:3, 3] = x, y, z, position
    return out


def _smooth_colour(rng: np.random.Generator, pts: np.ndarray, n_waves=8, wl=(0.3, 2.0), noise=0.05):
    """RGB from a sum of random plane waves (wavelengths `wl` metres) plus
    N(0, noise) per Gaussian; pts [3,N]."""
    out = np.zeros((3, pts.shape[1]))
    for ch in range(3):
        acc = np.zeros(pts.shape[1])
        for _ in range(n_waves):
            k = random_axis(rng) * (2 * math.pi / rng.uniform(*wl))
            acc += np.sin(k @ pts + rng.uniform(0, 2 * math.pi))
        out[ch] = 0.5 + 0.5 * acc / math.sqrt(n_waves)
    out += rng.normal(0.0, noise, out.shape)
    return out


def room_faces(rng: np.random.Generator, half=(3.0, 1.5, 2.0), boxes=4) -> list:
    """Faces (centre, u-axis half, v-axis half, normal) of the inner shell of a
    box room (6 x 3 x 4 m by default) and of `boxes` random boxes inside it."""
    half = np.asarray(half, np.float64)
    faces = []
    for ax in range(3):
        for sgn in (-1.0, 1.0):
            c = np.zeros(3)
            c[ax] = sgn * half[ax]
            o = [a for a in range(3) if a != ax]
            eu = np.zeros(3)
            eu[o[0]] = half[o[0]]
            ev = np.zeros(3)
            ev[o[1]] = half[o[1]]
            nrm = np.zeros(3)
            nrm[ax] = 1.0
            faces.append((c, eu, ev, nrm))
    for _ in range(boxes):
        bc = rng.uniform(-0.6, 0.6, 3) * half
        bc[1] = -half[1] + rng.uniform(0.3, 0.8)
        bh = rng.uniform(0.2, 0.5, 3)
        for ax in range(3):
            for sgn in (-1.0, 1.0):
                c = bc.copy()
                c[ax] += sgn * bh[ax]
                o = [a for a in range(3) if a != ax]
                eu = np.zeros(3)
                eu[o[0]] = bh[o[0]]
                ev = np.zeros(3)
                ev[o[1]] = bh[o[1]]
                nrm = np.zeros(3)
                nrm[ax] = 1.0
                faces.append((c, eu, ev, nrm))
    return faces


def face_points(rng: np.random.Generator, faces: list, n: int, jitter=0.01) -> np.ndarray:
    """n points uniform by area over `faces`, jittered along the normal; [3,n]."""
    areas = np.array([4 * np.linalg.norm(f[1]) * np.linalg.norm(f[2]) for f in faces])
    which = rng.choice(len(faces), size=n, p=areas / areas.sum())
    pts = np.zeros((3, n))
    for i, (c, eu, ev, nrm) in enumerate(faces):
        m = which == i
        k = int(m.sum())
        a = rng.uniform(-1, 1, k)
        b = rng.uniform(-1, 1, k)
        pts[:, m] = (c[:, None] + eu[:, None] * a + ev[:, None] * b + nrm[:, None] * rng.normal(0, jitter, k))
    return pts


def room_points(rng: np.random.Generator, n: int, half=(3.0, 1.5, 2.0), boxes=4, jitter=0.01) -> np.ndarray:
    """Points on the inner shell of a box room (6 x 3 x 4 m by default) plus
    the surfaces of `boxes` random boxes inside it, jittered along the normal."""
    return face_points(rng, room_faces(rng, half, boxes), n, jitter)


def in_view(pts: np.ndarray, c2ws, cam: dict, margin_px: float, z_near: float = 0.2) -> np.ndarray:
    """Mask of the points [3,N] that project into any of the cameras' images
    grown by `margin_px` on every side, in front of z_near (a pinhole
    frustum test; occlusion is ignored, so it over-approximates what a camera
    sees)."""
    out = np.zeros(pts.shape[1], bool)
    for c in c2ws:
        c = np.asarray(c, np.float64)
        p = c[:3, :3].T @ (pts - c[:3, 3:4])
        z = p[2]
        ok = z > z_near
        zs = np.where(ok, z, 1.0)
        u = cam["fx"] * p[0] / zs + cam["cx"]
        v = cam["fy"] * p[1] / zs + cam["cy"]
        out |= ok & (u >= -margin_px) & (u <= cam["width"] + margin_px) & (v >= -margin_px) & \
            (v <= cam["height"] + margin_px)
    return out


def pose_matrix4(pose: np.ndarray) -> np.ndarray:
    """4x4 rigid matrix of a (w, x, y, z, tx, ty, tz) pose vector."""
    w, x, y, z = pose[:4].astype(np.float64) / np.linalg.norm(pose[:4])
    t = np.eye(4)
    t[:3, :3] = [
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ]
    t[:3, 3] = pose[4:7]
    return t


def in_frame(pose: np.ndarray, g: dict) -> dict:
    """Gaussians moved rigidly by a (w, x, y, z, tx, ty, tz) pose: means mapped,
    quaternions left-multiplied by the pose's (scales, opacities, colours
    unchanged)."""
    t = pose_matrix4(pose)
    w, x, y, z = pose[:4].astype(np.float64) / np.linalg.norm(pose[:4])
    out = dict(g)
    out["mean"] = (t[:3, :3] @ g["mean"].astype(np.float64) + t[:3, 3:4]).astype(np.float32)
    qq = g["quat"].astype(np.float64)
    out["quat"] = np.stack([
        w * qq[0] - x * qq[1] - y * qq[2] - z * qq[3],
        w * qq[1] + x * qq[0] + y * qq[3] - z * qq[2],
        w * qq[2] - x * qq[3] + y * qq[0] + z * qq[1],
        w * qq[3] + x * qq[2] - y * qq[1] + z * qq[0],
    ]).astype(np.float32)
    return out


def registration_pair(seed: int, n_p: int, n_q: int, shared_frac: float = 0.6, views_p: int = 8,
                      views_q: int = 8, width: int = 640, height: int = 480, f: float = 500.0,
                      rot_deg_max: float = 10.0, trans_max: float = 0.3, half=(3.0, 1.5, 2.0),
                      log_scale_mu=math.log(0.02), fixed_gt=None, layout: str = "x_split",
                      view_margin_px: float = 64.0) -> dict:
    """Two overlapping submaps of one synthetic room and their keyframes.

    P is kept in the world frame; Q is expressed in its own frame through the
    ground-truth T_gt (rotation about a random axis by U[0, rot_deg_max] deg,
    translation of length U[0, trans_max] m), so x_Q = T_gt x_P.  Keyframe
    poses are camera-to-world in the submap's own frame.  Targets (the
    submaps rendered at their own keyframes) are made by the caller with the
    renderer.  Two layouts:

    "x_split": the room's points are ordered along x; the lowest (n_p - S)
    belong to P only, the highest (n_q - S) to Q only and the
    S = shared_frac * (n_p + n_q) / 2 in between (at most min(n_p, n_q)) to
    both.  Keyframes: cameras near the room centre, each looking at a point
    of the shared band.  When one submap is much smaller than the other, the
    shared band is a thin x-slab and the keyframes also see content that
    only one submap holds.

    "views": keyframes first, then the split.  Every keyframe of either
    submap stands near the room centre and looks at a point of one wall (a
    random x or z wall) between knee and head height, so views hold that
    wall, the floor near it and any box in front of it.  The shared
    Gaussians are S = min(shared_frac * (n_p + n_q) / 2, 0.8 min(n_p, n_q))
    points drawn over the part of the room inside some keyframe's frustum
    (image grown by `view_margin_px`); the unshared ones are drawn over the
    rest of the room, ordered along the wall and split into P's side and
    Q's side.  So every keyframe of either submap sees only Gaussians that
    both submaps hold: each view's target is reproduced by the other submap
    at the true transform.
    """
    if layout not in ("x_split", "views"):
        raise ValueError(f"layout must be 'x_split' or 'views', not {layout!r}")
    rng = np.random.default_rng(seed)
    cam = camera(f, f, width / 2, height / 2, width, height)
    if layout == "views":
        return _pair_views(rng, n_p, n_q, shared_frac, views_p, views_q, cam, rot_deg_max, trans_max,
                           np.asarray(half, np.float64), log_scale_mu, fixed_gt, view_margin_px)
    s = int(round(shared_frac * (n_p + n_q) / 2))
    s = min(s, n_p, n_q)
    n_w = n_p + n_q - s
    pts = room_points(rng, n_w, half=half)
    order = np.argsort(pts[0], kind="stable")
    pts = pts[:, order]
    g = gaussians_in_box(rng, n_w, (0, 0, 0), (1, 1, 1), log_scale_mu=log_scale_mu)
    g["mean"] = pts.astype(np.float32)
    g["rgb"] = _smooth_colour(rng, pts).astype(np.float32)
    idx_p = np.arange(0, n_p)
    idx_q = np.arange(n_w - n_q, n_w)
    gt = _ground_truth(rng, rot_deg_max, trans_max, fixed_gt)
    t_gt = pose_matrix4(gt)
    P = {k: v[..., idx_p].copy() for k, v in g.items()}
    Q = in_frame(gt, {k: v[..., idx_q].copy() for k, v in g.items()})
    band = pts[:, n_w - n_q:n_p] if n_p > n_w - n_q else pts
    half = np.asarray(half)

    def keyframes(k):
        out = []
        for _ in range(k):
            pos = rng.uniform(-0.35, 0.35, 3) * half
            tgt = band[:, rng.integers(band.shape[1])]
            if np.linalg.norm(tgt - pos) < 1.0:
                tgt = pos + (tgt - pos) / max(np.linalg.norm(tgt - pos), 1e-6) * 1.5
            out.append(look_at_c2w(pos, tgt))
        return out

    kf_p = keyframes(views_p)
    kf_q = [t_gt @ c for c in keyframes(views_q)]
    return dict(P=P, Q=Q, kf_p=np.stack(kf_p).astype(np.float64), kf_q=np.stack(kf_q).astype(np.float64),
                T_gt=t_gt, cam=cam, shared=s)


def _ground_truth(rng, rot_deg_max, trans_max, fixed_gt):
    if fixed_gt is not None:
        return np.asarray(fixed_gt, np.float32)
    ang = math.radians(rng.uniform(0.0, rot_deg_max))
    return axis_angle_pose(random_axis(rng), ang, rng.uniform(0.0, trans_max) * random_axis(rng))


def _pair_views(rng, n_p, n_q, shared_frac, views_p, views_q, cam, rot_deg_max, trans_max, half, log_scale_mu,
                fixed_gt, margin_px) -> dict:
    """The "views" layout of registration_pair."""
    s = int(round(min(shared_frac * (n_p + n_q) / 2, 0.8 * min(n_p, n_q))))
    n_w = n_p + n_q - s
    faces = room_faces(rng, half)
    ax = (0, 2)[int(rng.integers(2))]           # the wall the keyframes look at: an x or a z wall
    sgn = (-1.0, 1.0)[int(rng.integers(2))]
    along = 2 if ax == 0 else 0                 # horizontal axis within that wall

    def keyframes(k):
        out = []
        for _ in range(k):
            pos = rng.uniform(-0.35, 0.35, 3) * half
            pos[ax] -= sgn * 0.2 * half[ax]     # a step back from the wall
            tgt = np.zeros(3)
            tgt[ax] = sgn * half[ax]
            tgt[along] = rng.uniform(-0.5, 0.5) * half[along]
            tgt[1] = rng.uniform(-0.9, 0.2) * half[1]
            out.append(look_at_c2w(pos, tgt))
        return out

    kf_p = keyframes(views_p)
    kf_q_world = keyframes(views_q)
    seen, unseen = [], []
    n_seen = n_unseen = 0
    while n_seen < s or n_unseen < n_w - s:
        pool = face_points(rng, faces, max(4 * n_w, 4096))
        m = in_view(pool, kf_p + kf_q_world, cam, margin_px)
        seen.append(pool[:, m])
        unseen.append(pool[:, ~m])
        n_seen += int(m.sum())
        n_unseen += int((~m).sum())
    shared = np.concatenate(seen, 1)[:, :s]
    rest = np.concatenate(unseen, 1)[:, :n_w - s]
    rest = rest[:, np.argsort(rest[along], kind="stable")]
    pts = np.concatenate([rest[:, :n_p - s], shared, rest[:, n_p - s:]], 1)
    g = gaussians_in_box(rng, n_w, (0, 0, 0), (1, 1, 1), log_scale_mu=log_scale_mu)
    g["mean"] = pts.astype(np.float32)
    g["rgb"] = _smooth_colour(rng, pts).astype(np.float32)
    gt = _ground_truth(rng, rot_deg_max, trans_max, fixed_gt)
    t_gt = pose_matrix4(gt)
    P = {k: v[..., :n_p].copy() for k, v in g.items()}
    Q = in_frame(gt, {k: v[..., n_w - n_q:].copy() for k, v in g.items()})
    kf_q = [t_gt @ c for c in kf_q_world]
    return dict(P=P, Q=Q, kf_p=np.stack(kf_p).astype(np.float64), kf_q=np.stack(kf_q).astype(np.float64),
                T_gt=t_gt, cam=cam, shared=s)


def pair_set(seed: int, n_pairs: int, n_min: int = 20_000, n_max: int = 300_000, views_min: int = 4,
             views_max: int = 12, layout: str = "views") -> list:
    """Specs of a batch of registration pairs: per submap a Gaussian count
    log-uniform in [n_min, n_max] and a keyframe count uniform in
    {views_min..views_max}; each pair gets its own seed (hence its own room,
    split and ground-truth transform) and the submap layout `layout` of
    registration_pair."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_pairs):
        n_p, n_q = (int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max))))) for _ in range(2))
        v_p, v_q = (int(rng.integers(views_min, views_max + 1)) for _ in range(2))
        out.append(dict(seed=int(seed * 1000 + k), n_p=n_p, n_q=n_q, views_p=v_p, views_q=v_q, layout=layout))
    return out


def request_stream(seed: int, n_requests: int, rate_per_s: float, median_n: int = 100_000, sigma: float = 0.8,
                   n_cap: int = 500_000, n_floor: int = 5_000, views_min: int = 4, views_max: int = 12,
                   resolutions=((640, 480, 500.0), (1200, 680, 600.0))) -> list:
    """A serving stream: Poisson arrivals at `rate_per_s` (exponential gaps),
    submap sizes lognormal(median, sigma) clipped to [n_floor, n_cap], views
    uniform in {views_min..views_max}, resolution drawn from `resolutions`."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(n_requests):
        t += float(rng.exponential(1.0 / rate_per_s))
        n_p, n_q = (int(np.clip(round(median_n * math.exp(sigma * rng.normal())), n_floor, n_cap)) for _ in range(2))
        v_p, v_q = (int(rng.integers(views_min, views_max + 1)) for _ in range(2))
        w, h, f = resolutions[int(rng.integers(len(resolutions)))]
        out.append(dict(arrival=t, seed=int(seed * 100000 + k), n_p=n_p, n_q=n_q, views_p=v_p, views_q=v_q,
                        width=int(w), height=int(h), f=float(f), layout="views"))
    return out

