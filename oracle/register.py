"""FP64 oracle of 3DGS registration as keyframe localisation (paper Sec. 3.2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings (the paper leaves these open):
  R18 optimiser: Adam with beta1 = 0.9, beta2 = 0.999, eps = 1e-8 and bias
      correction; the rotation (unnormalised quaternion) and the translation
      get their own learning rates (supplement, loop-closure hyper-parameter
      table: 0.003 / 0.001 synthetic-like, 0.015 / 0.005 real-like)
  R19 iteration count: a parameter (200 in the single-pair workload)
  R20 residual eps_i: the unmasked colour + depth L1 of R15 at the final
      pose, from one extra forward, whichever loss drove the optimisation:
      the residual rates how well the moved viewpoint explains its whole
      observation (Sec. 3.2).  A masked residual would rate a view that
      drifted off the other submap (alpha ~ 0, masked loss ~ 0) best.
  R21 weight 1 / max(eps_i, 1e-12)
  R22 translation: weighted mean of the P->Q translations, the Q->P
      estimates inverted first
  R33 joint registration (optional comparison, not the paper's estimator):
      one T = T_{P->Q} (unnormalised quaternion and translation, starting
      at identity) shared by all views.  View i's camera-frame correction is
      Delta_i = C_i^-1 T^-1 C_i for a keyframe of P and C_i^-1 T C_i for one
      of Q (C_i its camera-to-world pose), the objective is the sum of the
      views' losses and T takes the Adam steps (lr_rot for q, lr_trans for
      t); the estimate is T itself, with no Eq. 7 fusion.
  R23 exposure coefficients (supplement, 3DGS registration; optional): per
      view an affine brightness map of the rendered colour,
      C' = exp(a) C + b with scalars a, b shared by the three channels,
      starting at a = b = 0 and optimised with the pose by Adam (learning
      rate 0.1, the supplement's table; same step count and moments rule).
      The loss and the residual of R20 see C'.  The paper names exposure
      coefficients but not their form; this gain/offset form is the reading.

Per-view problem (Sec. 3.2, keyframe localisation).  For keyframe i of P with
camera-to-world pose T_i (in P's frame) and measurements (I, D)_i, the
submap Q is rendered with world-to-camera Delta o T_i^-1 and Delta (starting
at identity) is optimised with Q held fixed.  The keyframe's pose in Q is
T_i^q = T_i Delta^-1, so the estimate of T_{P->Q} = T_i^q T_i^-1 is
E_i = T_i Delta^-1 T_i^-1.  Keyframes of Q rendering P give estimates of
T_{Q->P} the same way.

Fusion (Eq. 7): R_bar = argmin_R sum_i w_i ||R - R~_i||_F^2 with R~_i = R_i
for P->Q estimates and R_i^-1 for Q->P ones.  Its closed form is the
projection of M = sum_i w_i R~_i onto SO(3): M = U S V^T,
R_bar = U diag(1, 1, det(U V^T)) V^T.
"""

from __future__ import annotations

import math

import numpy as np
import torch

from . import raster

F64 = torch.float64


def adam_step(param, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update in place on float64 tensors; `step` counts from 1."""
    with torch.no_grad():
        m.mul_(beta1).add_((1 - beta1) * grad)
        v.mul_(beta2).add_((1 - beta2) * grad * grad)
        m_hat = m / (1 - beta1 ** step)
        v_hat = v / (1 - beta2 ** step)
        param.sub_(lr * m_hat / (torch.sqrt(v_hat) + eps))


def pose_matrix(pose7) -> np.ndarray:
    """4x4 rigid transform of a pose 7-vector (q_w, q_x, q_y, q_z, t)."""
    p = torch.as_tensor(np.asarray(pose7, np.float64))
    out = np.eye(4)
    out[:3, :3] = raster.quat_to_rotmat(p[:4]).numpy()
    out[:3, 3] = p[4:7].numpy()
    return out


def inv_rigid(t: np.ndarray) -> np.ndarray:
    out = np.eye(4)
    out[:3, :3] = t[:3, :3].T
    out[:3, 3] = -t[:3, :3].T @ t[:3, 3]
    return out


def view_loss(out: dict, tgt_rgb, tgt_depth, loss):
    """The localisation loss of one render: loss None -> plain L1 (R15);
    else a dict of loss_tracking's keyword arguments -> R24."""
    if loss is None:
        return raster.loss_l1(out["rgb"], out["depth"], tgt_rgb, tgt_depth)
    return raster.loss_tracking(out["rgb"], out["depth"], out["alpha"], tgt_rgb, tgt_depth, **loss)[0]


def localise_view(gauss: dict, cam: raster.Camera, c2w: np.ndarray, tgt_rgb, tgt_depth, iters: int,
                  lr_rot: float, lr_trans: float, beta1=0.9, beta2=0.999, eps=1e-8, loss=None,
                  lr_exposure: float | None = None, return_exposure: bool = False):
    """Optimise the camera-frame correction Delta of one keyframe (R18-R20),
    and with lr_exposure set its exposure coefficients (a, b) too (R23).

    gauss: the *other* submap (float64 tensors, held fixed); c2w: the
    keyframe's camera-to-world pose in its own submap; targets [3,H,W], [H,W];
    loss: None (plain L1) or loss_tracking's keyword arguments (R24).
    Returns (Delta as a pose 7-vector, residual eps, loss history), plus (a, b)
    when return_exposure.
    """
    w2c = torch.as_tensor(inv_rigid(np.asarray(c2w, np.float64))[:3, :])
    fixed = {k: v.detach() for k, v in gauss.items()}
    q = torch.tensor([1.0, 0.0, 0.0, 0.0], dtype=F64, requires_grad=True)
    t = torch.zeros(3, dtype=F64, requires_grad=True)
    mq, vq = torch.zeros(4, dtype=F64), torch.zeros(4, dtype=F64)
    mt, vt = torch.zeros(3, dtype=F64), torch.zeros(3, dtype=F64)
    tgt_rgb = torch.as_tensor(np.asarray(tgt_rgb, np.float64))
    tgt_depth = torch.as_tensor(np.asarray(tgt_depth, np.float64))
    ab = torch.zeros(2, dtype=F64, requires_grad=lr_exposure is not None)
    mab, vab = torch.zeros(2, dtype=F64), torch.zeros(2, dtype=F64)

    def exposed(out):
        if lr_exposure is None:
            return out
        return dict(out, rgb=torch.exp(ab[0]) * out["rgb"] + ab[1])

    params = [q, t] + ([ab] if lr_exposure is not None else [])
    hist = []
    for it in range(1, iters + 1):
        out = exposed(raster.render(fixed, cam, w2c, torch.cat([q, t]), with_margins=False))
        val = view_loss(out, tgt_rgb, tgt_depth, loss)
        # an empty render (nothing in front of the camera) does not depend on the pose
        grads = torch.autograd.grad(val, params, allow_unused=True) if val.requires_grad else [None] * len(params)
        gq = torch.zeros(4, dtype=F64) if grads[0] is None else grads[0]
        gt = torch.zeros(3, dtype=F64) if grads[1] is None else grads[1]
        adam_step(q, gq, mq, vq, it, lr_rot, beta1, beta2, eps)
        adam_step(t, gt, mt, vt, it, lr_trans, beta1, beta2, eps)
        if lr_exposure is not None:
            gab = torch.zeros(2, dtype=F64) if grads[2] is None else grads[2]
            adam_step(ab, gab, mab, vab, it, lr_exposure, beta1, beta2, eps)
        hist.append(float(val.detach()))
    with torch.no_grad():
        out = exposed(raster.render(fixed, cam, w2c, torch.cat([q, t]), with_margins=False))
        resid = float(raster.loss_l1(out["rgb"], out["depth"], tgt_rgb, tgt_depth))
    if return_exposure:
        return torch.cat([q, t]).detach().numpy(), resid, hist, ab.detach().numpy().copy()
    return torch.cat([q, t]).detach().numpy(), resid, hist


def view_estimate(c2w: np.ndarray, delta7) -> np.ndarray:
    """E = T_i Delta^-1 T_i^-1: the source-to-target transform implied by one
    keyframe localisation (Sec. 3.2, T_{P->Q} = T_i^q T_i^-1)."""
    c2w = np.asarray(c2w, np.float64)
    return c2w @ inv_rigid(pose_matrix(delta7)) @ inv_rigid(c2w)


def fuse(estimates, residuals, reverse) -> np.ndarray:
    """Weighted rotation averaging (Eq. 7) and weighted translation mean.

    estimates: list of 4x4 transforms; residuals: eps_i; reverse[i] True for
    a Q->P estimate (inverted before averaging).  Returns the 4x4 T_bar.
    """
    m = np.zeros((3, 3))
    tsum = np.zeros(3)
    wsum = 0.0
    for e, r, rev in zip(estimates, residuals, reverse):
        w = 1.0 / max(float(r), 1e-12)
        e = inv_rigid(e) if rev else np.asarray(e, np.float64)
        m += w * e[:3, :3]
        tsum += w * e[:3, 3]
        wsum += w
    u, _, vt = np.linalg.svd(m)
    d = np.sign(np.linalg.det(u @ vt))
    out = np.eye(4)
    out[:3, :3] = u @ np.diag([1.0, 1.0, d]) @ vt
    out[:3, 3] = tsum / wsum
    return out


def register_pair(P: dict, Q: dict, views_p, views_q, cam: raster.Camera, iters: int, lr_rot: float,
                  lr_trans: float, loss=None, lr_exposure: float | None = None):
    """Full pair registration: every keyframe of P localised in Q and every
    keyframe of Q in P, then fused (Sec. 3.2); with lr_exposure set, each
    view also fits its exposure coefficients (R23).

    P, Q: float64 Gaussian dicts; views_*: lists of (c2w 4x4, rgb [3,H,W],
    depth [H,W]).  Returns (T_bar 4x4, per-view estimates, residuals).
    """
    ests, res, rev = [], [], []
    for views, other, reverse in ((views_p, Q, False), (views_q, P, True)):
        for c2w, rgb, dep in views:
            d, r, _ = localise_view(other, cam, c2w, rgb, dep, iters, lr_rot, lr_trans, loss=loss,
                                    lr_exposure=lr_exposure)
            ests.append(view_estimate(c2w, d))
            res.append(r)
            rev.append(reverse)
    return fuse(ests, res, rev), ests, res


def _quat_mul(a, b):
    """Hamilton product of (w, x, y, z) quaternions (torch, differentiable)."""
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return torch.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                        w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def _quat_of(rot: np.ndarray) -> torch.Tensor:
    from scipy.spatial.transform import Rotation

    q = Rotation.from_matrix(np.asarray(rot, np.float64)).as_quat()  # x, y, z, w
    return torch.as_tensor([q[3], q[0], q[1], q[2]], dtype=F64)


def joint_delta(T7: torch.Tensor, c2w: np.ndarray, reverse: bool) -> torch.Tensor:
    """Delta_i of R33 as a pose 7-vector, differentiable in T7."""
    T7 = T7.to(F64)
    q = T7[:4] / torch.linalg.norm(T7[:4])
    t = T7[4:7]
    conj = torch.tensor([1.0, -1.0, -1.0, -1.0], dtype=F64)
    qc = _quat_of(np.asarray(c2w)[:3, :3])
    Rc = torch.as_tensor(np.asarray(c2w, np.float64)[:3, :3])
    tc = torch.as_tensor(np.asarray(c2w, np.float64)[:3, 3])
    Rt = raster.quat_to_rotmat(q)
    if reverse:  # keyframe of Q: Delta = C^-1 T C
        qd = _quat_mul(_quat_mul(qc * conj, q), qc)
        td = Rc.T @ (Rt @ tc + t - tc)
    else:  # keyframe of P: Delta = C^-1 T^-1 C
        qd = _quat_mul(_quat_mul(qc * conj, q * conj), qc)
        td = Rc.T @ (Rt.T @ (tc - t) - tc)
    return torch.cat([qd, td])


def register_pair_joint(P: dict, Q: dict, views_p, views_q, cam: raster.Camera, iters: int, lr_rot: float,
                        lr_trans: float, loss=None, beta1=0.9, beta2=0.999, eps=1e-8):
    """R33: one shared T_{P->Q} optimised over every view's loss.  Returns
    (T 4x4, residuals of the views at the final T)."""
    T7 = torch.tensor([1.0, 0, 0, 0, 0, 0, 0], dtype=F64, requires_grad=True)
    m, v = torch.zeros(7, dtype=F64), torch.zeros(7, dtype=F64)
    views = [(c2w, rgb, dep, other, rev) for vs, other, rev in ((views_p, Q, False), (views_q, P, True))
             for c2w, rgb, dep in vs]
    prepared = []
    for c2w, rgb, dep, other, rev in views:
        w2c = torch.as_tensor(inv_rigid(np.asarray(c2w, np.float64))[:3, :])
        prepared.append((c2w, w2c, torch.as_tensor(np.asarray(rgb, np.float64)),
                         torch.as_tensor(np.asarray(dep, np.float64)), {k: x.detach() for k, x in other.items()}, rev))
    for it in range(1, iters + 1):
        total = None
        for c2w, w2c, rgb, dep, other, rev in prepared:
            out = raster.render(other, cam, w2c, joint_delta(T7, c2w, rev), with_margins=False)
            val = view_loss(out, rgb, dep, loss)
            total = val if total is None else total + val
        (g,) = torch.autograd.grad(total, [T7], allow_unused=True) if total.requires_grad else (None,)
        g = torch.zeros(7, dtype=F64) if g is None else g
        with torch.no_grad():
            m[:4] = beta1 * m[:4] + (1 - beta1) * g[:4]
            m[4:] = beta1 * m[4:] + (1 - beta1) * g[4:]
            v.mul_(beta2).add_((1 - beta2) * g * g)
            mh, vh = m / (1 - beta1 ** it), v / (1 - beta2 ** it)
            lr = torch.tensor([lr_rot] * 4 + [lr_trans] * 3, dtype=F64)
            T7.sub_(lr * mh / (torch.sqrt(vh) + eps))
    res = []
    with torch.no_grad():
        for c2w, w2c, rgb, dep, other, rev in prepared:
            out = raster.render(other, cam, w2c, joint_delta(T7, c2w, rev), with_margins=False)
            res.append(float(raster.loss_l1(out["rgb"], out["depth"], rgb, dep)))
    return pose_matrix(T7.detach().numpy()), res


def rotation_error_deg(r: np.ndarray, r_gt: np.ndarray) -> float:
    c = (np.trace(np.asarray(r)[:3, :3] @ np.asarray(r_gt)[:3, :3].T) - 1.0) / 2.0
    return math.degrees(math.acos(min(1.0, max(-1.0, c))))


def translation_error_cm(t: np.ndarray, t_gt: np.ndarray) -> float:
    return 100.0 * float(np.linalg.norm(np.asarray(t, np.float64) - np.asarray(t_gt, np.float64)))
