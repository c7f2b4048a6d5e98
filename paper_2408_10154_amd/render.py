"""PyTorch-facing wrapper of the rasterizer C ABI.

PyTorch supplies device memory and the current HIP stream; every step of
the computation runs in libloopsplat.so.  `RenderBatch` owns the buffers of
one batch of render jobs and exposes the C calls one to one; `render()` is a
torch.autograd.Function over a batch whose backward is ls_render_bwd.
"""

from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import lib as L


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclass
class GaussianSet:
    """Device SoA Gaussians: mean [3,N], log_scale [3,N], quat [4,N],
    opacity_logit [N], rgb [3,N] (float32, contiguous)."""

    mean: torch.Tensor
    log_scale: torch.Tensor
    quat: torch.Tensor
    opacity_logit: torch.Tensor
    rgb: torch.Tensor

    FIELDS = ("mean", "log_scale", "quat", "opacity_logit", "rgb")

    @property
    def n(self) -> int:
        return int(self.opacity_logit.shape[0])

    @classmethod
    def from_numpy(cls, g: dict, device="cuda") -> "GaussianSet":
        return cls(**{k: torch.as_tensor(np.ascontiguousarray(g[k], np.float32), device=device) for k in cls.FIELDS})

    def tensors(self):
        return [getattr(self, k) for k in self.FIELDS]

    def zeros_like(self) -> "GaussianSet":
        return GaussianSet(*[torch.zeros_like(t) for t in self.tensors()])

    def to_c(self) -> L.ls_gaussians:
        for t in self.tensors():
            if t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda:
                raise ValueError("Gaussian arrays must be contiguous float32 device tensors")
        return L.ls_gaussians(self.n, *[t.data_ptr() for t in self.tensors()])

    def grads_c(self) -> L.ls_gaussian_grads:
        return L.ls_gaussian_grads(*[t.data_ptr() for t in self.tensors()])


class RenderBatch:
    """R render jobs sharing one set of launches.

    jobs: list of (GaussianSet, camera dict fx fy cx cy width height,
    w2c [3,4]).  `capacity` is the tile-instance capacity; with
    `auto_grow` (default) bin_sort() reads the instance count back and grows
    the buffers and re-bins when it overflows (one host sync per call).
    """

    def __init__(self, jobs, capacity: int | None = None, auto_grow: bool = True, device="cuda"):
        self.lib = L.load()
        self.device = torch.device(device)
        self.gsets = [j[0] for j in jobs]
        self.cams = [dict(j[1]) for j in jobs]
        arr = (L.ls_render_job * len(jobs))()
        for i, (g, cam, w2c) in enumerate(jobs):
            arr[i].g = g.to_c()
            arr[i].K = L.ls_intrinsics(cam["fx"], cam["fy"], cam["cx"], cam["cy"], cam["width"], cam["height"])
            w = np.asarray(w2c, np.float64).reshape(3, 4).astype(np.float32).ravel()
            for k in range(12):
                arr[i].w2c[k] = float(w[k])
        self._jobs_c = arr
        self.h = L.ls_batch_create(arr, len(jobs))
        info = L.ls_batch_query(self.h, 0)
        self.R, self.M, self.T, self.P = info.renders, info.items, info.tiles, info.pixels
        self.item_off = np.zeros(self.R + 1, np.int64)
        self.pix_off = np.zeros(self.R + 1, np.int64)
        self.tile_off = np.zeros(self.R + 1, np.int32)
        L.ls_batch_offsets(self.h, self.item_off.ctypes.data_as(C.c_void_p), self.pix_off.ctypes.data_as(C.c_void_p),
                           self.tile_off.ctypes.data_as(C.c_void_p))
        dev = self.device
        self.rec = torch.zeros(max(self.M, 1), L.REC_FLOATS, dtype=torch.float32, device=dev)
        self.radius = torch.zeros(max(self.M, 1), dtype=torch.int32, device=dev)
        self.tiles = torch.zeros(max(self.M, 1), dtype=torch.int32, device=dev)
        self.aux = torch.zeros(max(self.M, 1), 12, dtype=torch.float32, device=dev)
        self.proj = L.ls_projected(self.rec.data_ptr(), self.radius.data_ptr(), self.tiles.data_ptr(),
                                   self.aux.data_ptr())
        self.rgb = torch.zeros(3 * self.P, dtype=torch.float32, device=dev)
        self.depth = torch.zeros(self.P, dtype=torch.float32, device=dev)
        self.alpha = torch.zeros(self.P, dtype=torch.float32, device=dev)
        self.T_final = torch.zeros(self.P, dtype=torch.float32, device=dev)
        self.n_last = torch.zeros(self.P, dtype=torch.int32, device=dev)
        self.image = L.ls_image(self.rgb.data_ptr(), self.depth.data_ptr(), self.alpha.data_ptr(),
                                self.T_final.data_ptr(), self.n_last.data_ptr())
        self.count = torch.zeros(4, dtype=torch.int32, device=dev)
        self.range = torch.zeros(max(self.T, 1), 2, dtype=torch.int32, device=dev)
        self.auto_grow = auto_grow
        self.capacity = 0
        self._alloc_bins(capacity if capacity is not None else max(1024, 16 * self.M))

    # ------------------------------------------------------------ buffers
    def _alloc_bins(self, capacity: int):
        capacity = int(capacity)
        info = L.ls_batch_query(self.h, capacity)
        dev = self.device
        self.capacity = capacity
        self.tile_of = torch.zeros(max(capacity, 1), dtype=torch.int32, device=dev)
        self.item = torch.zeros(max(capacity, 1), dtype=torch.int32, device=dev)
        self.work = torch.zeros(int(info.workspace_bytes) + 256, dtype=torch.uint8, device=dev)
        wp = (self.work.data_ptr() + 255) // 256 * 256
        self.bins = L.ls_bins(capacity, self.tile_of.data_ptr(), self.item.data_ptr(), self.range.data_ptr(),
                              self.count.data_ptr(), wp)

    def close(self):
        if getattr(self, "h", None) is not None:
            L.ls_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ C calls
    def _check_pose(self, pose):
        if pose is not None:
            if pose.dtype != torch.float32 or not pose.is_cuda or not pose.is_contiguous() or pose.numel() != 7 * self.R:
                raise ValueError(f"pose must be a contiguous float32 device tensor of {7 * self.R} values")

    def _check_dev(self, t, numel, dtype=torch.float32, name="tensor"):
        if t is None:
            return
        if t.dtype != dtype or not t.is_cuda or not t.is_contiguous() or t.numel() != numel:
            raise ValueError(f"{name} must be a contiguous {dtype} device tensor of {numel} values")

    def project(self, pose: torch.Tensor | None = None):
        self._check_pose(pose)
        L.ls_project(self.h, _ptr(pose), self.proj, _stream())

    def bin_sort(self):
        L.ls_bin_sort(self.h, self.proj, self.bins, _stream())
        if self.auto_grow:
            cnt = self.count.cpu()
            if int(cnt[1]) != 0:
                self._alloc_bins(int(int(cnt[2]) * 1.25) + 1024)
                L.ls_bin_sort(self.h, self.proj, self.bins, _stream())

    def instances(self) -> int:
        return int(self.count[0].item())

    def render_fwd(self, bg=None):
        bgc = (C.c_float * 3)(*bg) if bg is not None else None
        L.ls_render_fwd(self.h, self.proj, self.bins, bgc, self.image, _stream())

    def render_bwd(self, up_rgb=None, up_depth=None, up_alpha=None, scale=None, grads=None, pose=None,
                   pose_grad=None, bg=None):
        self._check_pose(pose)
        self._check_dev(pose_grad, 7 * self.R, name="pose_grad")
        self._check_dev(up_rgb, 3 * self.P, name="up_rgb")
        self._check_dev(up_depth, self.P, name="up_depth")
        self._check_dev(up_alpha, self.P, name="up_alpha")
        self._check_dev(scale, self.R, name="scale")
        if grads is not None:
            if len(grads) != self.R:
                raise ValueError("need one gradient set per render")
            for g, gs in zip(grads, self.gsets):
                for t, ref in zip(g.tensors(), gs.tensors()):
                    self._check_dev(t, ref.numel(), name="gradient")
        up = L.ls_image_grad(*[None if t is None else t.data_ptr() for t in (up_rgb, up_depth, up_alpha, scale)])
        garr = None
        if grads is not None:
            garr = (L.ls_gaussian_grads * self.R)(*[g.grads_c() for g in grads])
        bgc = (C.c_float * 3)(*bg) if bg is not None else None
        L.ls_render_bwd(self.h, _ptr(pose), self.proj, self.bins, bgc, self.image, up, garr, _ptr(pose_grad),
                        _stream())

    def render_bwd_tiles(self, up_rgb=None, up_depth=None, up_alpha=None, scale=None, bg=None, pose=None,
                         pose_only=False):
        self._check_pose(pose)
        self._check_dev(up_rgb, 3 * self.P, name="up_rgb")
        self._check_dev(up_depth, self.P, name="up_depth")
        self._check_dev(up_alpha, self.P, name="up_alpha")
        self._check_dev(scale, self.R, name="scale")
        up = L.ls_image_grad(*[None if t is None else t.data_ptr() for t in (up_rgb, up_depth, up_alpha, scale)])
        bgc = (C.c_float * 3)(*bg) if bg is not None else None
        L.ls_render_bwd_tiles(self.h, _ptr(pose), self.proj, self.bins, bgc, self.image, up,
                              L.BWD_POSE_ONLY if pose_only else 0, _stream())

    def render_bwd_tiles_l1(self, tgt_rgb, tgt_depth, inv_count, bg=None, pose=None, pose_only=False):
        """loss_l1 + render_bwd_tiles fused: the L1 gradient is formed inside
        the backward from the batch's images and the targets; inv_count is
        loss_l1's grad_scale for the same targets.  loss_l1_tiles() gives the
        loss afterwards."""
        self._check_pose(pose)
        self._check_dev(tgt_rgb, 3 * self.P, name="tgt_rgb")
        self._check_dev(tgt_depth, self.P, name="tgt_depth")
        self._check_dev(inv_count, self.R, name="inv_count")
        bgc = (C.c_float * 3)(*bg) if bg is not None else None
        L.ls_render_bwd_tiles_l1(self.h, _ptr(pose), self.proj, self.bins, bgc, self.image, _ptr(tgt_rgb),
                                 _ptr(tgt_depth), _ptr(inv_count), L.BWD_POSE_ONLY if pose_only else 0, _stream())

    def loss_l1_tiles(self, loss=None):
        """The L1 loss per render of the last render_bwd_tiles_l1."""
        loss = torch.zeros(self.R, dtype=torch.float32, device=self.device) if loss is None else loss
        self._check_dev(loss, self.R, name="loss")
        L.ls_loss_l1_tiles(self.h, self.bins, _ptr(loss), _stream())
        return loss

    def render_bwd_project(self, grads=None, pose=None, pose_grad=None, pose_only=False):
        self._check_pose(pose)
        self._check_dev(pose_grad, 7 * self.R, name="pose_grad")
        garr = None
        if grads is not None:
            if len(grads) != self.R:
                raise ValueError("need one gradient set per render")
            garr = (L.ls_gaussian_grads * self.R)(*[g.grads_c() for g in grads])
        L.ls_render_bwd_project(self.h, _ptr(pose), self.proj, self.bins, garr, _ptr(pose_grad),
                                L.BWD_POSE_ONLY if pose_only else 0, _stream())

    def render_bwd_project_adam(self, adam, step: int, pose=None, pose_grad=None, pose_adam=None, beta1=0.9,
                                beta2=0.999, eps=1e-8):
        """render_bwd_project with the Adam step fused: adam is one
        (moments, rates) entry per render, each a dict name -> (m, v, lr) over
        mean, log_scale, quat, opacity_logit and rgb (m, v device tensors
        shaped like the parameter); the batch's Gaussian sets are updated in
        place.  The pose gradient is accumulated into pose_grad; with
        pose_adam = (m, v, lr_rot, lr_trans) ([R, 7] moments) the poses take
        their step too (pose_grad consumed)."""
        self._check_pose(pose)
        self._check_dev(pose_grad, 7 * self.R, name="pose_grad")
        pa = None
        if pose_adam is not None:
            pm, pv, lr_rot, lr_trans = pose_adam
            self._check_dev(pm, 7 * self.R, name="pose moment")
            self._check_dev(pv, 7 * self.R, name="pose moment")
            pa = C.byref(L.ls_pose_adam(pm.data_ptr(), pv.data_ptr(), float(lr_rot), float(lr_trans)))
        if len(adam) != self.R:
            raise ValueError("need one Adam state per render")
        arr = (L.ls_gaussian_adam * self.R)()
        for r, (st, gs) in enumerate(zip(adam, self.gsets)):
            for name, ref in zip(("mean", "log_scale", "quat", "opacity_logit", "rgb"), gs.tensors()):
                m, v, lr = st[name]
                self._check_dev(m, ref.numel(), name="moment")
                self._check_dev(v, ref.numel(), name="moment")
                setattr(arr[r], name, L.ls_adam_array(m.data_ptr(), v.data_ptr(), float(lr)))
        L.ls_render_bwd_project_adam(self.h, _ptr(pose), self.proj, self.bins, arr, pa, int(step), beta1, beta2, eps,
                                     _ptr(pose_grad), _stream())

    def render_stats(self):
        """(entries evaluated, entries composited) of the last forward (syncs)."""
        st = torch.zeros(2, dtype=torch.int64, device=self.device)
        L.ls_render_stats(self.h, self.proj, self.bins, self.image, _ptr(st), _stream())
        v = st.cpu().numpy()
        return int(v[0]), int(v[1])

    def loss_l1(self, tgt_rgb, tgt_depth, loss=None, grad_rgb=None, grad_depth=None, grad_scale=None):
        dev = self.device
        loss = torch.zeros(self.R, dtype=torch.float32, device=dev) if loss is None else loss
        grad_rgb = torch.empty_like(self.rgb) if grad_rgb is None else grad_rgb
        grad_depth = torch.empty_like(self.depth) if grad_depth is None else grad_depth
        grad_scale = torch.zeros(self.R, dtype=torch.float32, device=dev) if grad_scale is None else grad_scale
        self._check_dev(tgt_rgb, 3 * self.P, name="tgt_rgb")
        self._check_dev(tgt_depth, self.P, name="tgt_depth")
        for t, n in ((loss, self.R), (grad_rgb, 3 * self.P), (grad_depth, self.P), (grad_scale, self.R)):
            self._check_dev(t, n)
        L.ls_loss_l1(self.h, self.image, _ptr(tgt_rgb), _ptr(tgt_depth), _ptr(loss), _ptr(grad_rgb), _ptr(grad_depth),
                     _ptr(grad_scale), _stream())
        return loss, grad_rgb, grad_depth, grad_scale

    def loss_tracking(self, tgt_rgb, tgt_depth, lambda_c=0.6, inlier_k=50.0, alpha_power=3, pred=None, loss=None,
                      median=None, grad_rgb=None, grad_depth=None, grad_scale=None):
        """Tracking loss with masks on the batch's images, or on `pred` =
        (rgb, depth, alpha) device tensors laid out like them."""
        dev = self.device
        img = self.image
        if pred is not None:
            for t, n in zip(pred, (3 * self.P, self.P, self.P)):
                self._check_dev(t, n)
            img = L.ls_image(pred[0].data_ptr(), pred[1].data_ptr(), pred[2].data_ptr(), None, None)
        loss = torch.zeros(self.R, dtype=torch.float32, device=dev) if loss is None else loss
        median = torch.zeros(self.R, dtype=torch.float32, device=dev) if median is None else median
        grad_rgb = torch.empty_like(self.rgb) if grad_rgb is None else grad_rgb
        grad_depth = torch.empty_like(self.depth) if grad_depth is None else grad_depth
        grad_scale = torch.zeros(self.R, dtype=torch.float32, device=dev) if grad_scale is None else grad_scale
        self._check_dev(tgt_rgb, 3 * self.P, name="tgt_rgb")
        self._check_dev(tgt_depth, self.P, name="tgt_depth")
        for t, n in ((loss, self.R), (median, self.R), (grad_rgb, 3 * self.P), (grad_depth, self.P),
                     (grad_scale, self.R)):
            self._check_dev(t, n)
        prm = L.ls_loss_params(float(lambda_c), float(inlier_k), int(alpha_power), 0)
        L.ls_loss_tracking(self.h, img, _ptr(tgt_rgb), _ptr(tgt_depth), prm, _ptr(loss), _ptr(median),
                           _ptr(grad_rgb), _ptr(grad_depth), _ptr(grad_scale), _stream())
        return loss, median, grad_rgb, grad_depth, grad_scale

    def loss_mapping(self, tgt_rgb, tgt_depth, lambda_ssim=0.2, lambda_color=1.0, lambda_depth=1.0, loss=None,
                     grad_rgb=None, grad_depth=None, grad_scale=None):
        """Image part of the submap-update loss (L1 + SSIM colour term and L1
        depth term) on the batch's images; the gradients come fully weighted
        and grad_scale is 1."""
        dev = self.device
        loss = torch.zeros(self.R, dtype=torch.float32, device=dev) if loss is None else loss
        grad_rgb = torch.empty_like(self.rgb) if grad_rgb is None else grad_rgb
        grad_depth = torch.empty_like(self.depth) if grad_depth is None else grad_depth
        grad_scale = torch.zeros(self.R, dtype=torch.float32, device=dev) if grad_scale is None else grad_scale
        self._check_dev(tgt_rgb, 3 * self.P, name="tgt_rgb")
        self._check_dev(tgt_depth, self.P, name="tgt_depth")
        for t, n in ((loss, self.R), (grad_rgb, 3 * self.P), (grad_depth, self.P), (grad_scale, self.R)):
            self._check_dev(t, n)
        prm = L.ls_mapping_params(float(lambda_ssim), float(lambda_color), float(lambda_depth), 0)
        L.ls_loss_mapping(self.h, self.image, _ptr(tgt_rgb), _ptr(tgt_depth), prm, _ptr(loss), _ptr(grad_rgb),
                          _ptr(grad_depth), _ptr(grad_scale), _stream())
        return loss, grad_rgb, grad_depth, grad_scale

    # ------------------------------------------------------------ views
    def image_views(self, r: int):
        cam = self.cams[r]
        H, W = cam["height"], cam["width"]
        p0 = int(self.pix_off[r])
        return dict(
            rgb=self.rgb[3 * p0: 3 * p0 + 3 * H * W].view(3, H, W),
            depth=self.depth[p0: p0 + H * W].view(H, W),
            alpha=self.alpha[p0: p0 + H * W].view(H, W),
            T_final=self.T_final[p0: p0 + H * W].view(H, W),
            n_last=self.n_last[p0: p0 + H * W].view(H, W),
        )


def loss_isotropic(log_scale: torch.Tensor, lambda_reg: float = 1.0, loss=None, grad=None, work=None):
    """Isotropic scale regulariser of one Gaussian set: log_scale [3, n]
    device tensor; grad (same shape) is accumulated when given."""
    if log_scale.dim() != 2 or log_scale.shape[0] != 3 or not log_scale.is_contiguous() or not log_scale.is_cuda:
        raise ValueError("log_scale must be a contiguous [3, n] device tensor")
    n = log_scale.shape[1]
    dev = log_scale.device
    loss = torch.zeros(1, dtype=torch.float32, device=dev) if loss is None else loss
    work = torch.empty(L.LS_ISOTROPIC_WORK_FLOATS, dtype=torch.float32, device=dev) if work is None else work
    if grad is not None and (grad.shape != log_scale.shape or not grad.is_contiguous()):
        raise ValueError("grad must match log_scale")
    L.ls_loss_isotropic(_ptr(log_scale), n, float(lambda_reg), _ptr(loss), _ptr(grad), _ptr(work), _stream())
    return loss


def adjust_submaps(subs):
    """Applies pose-graph corrections in place (map adjustment): subs is a
    list of (GaussianSet, c2w, T) with c2w a contiguous device tensor
    [k, 12] (row-major 3x4 camera-to-world keyframe poses) or None, and T
    the submap's correction as a 3x4 or 4x4 array."""
    arr = (L.ls_submap_adjust * max(len(subs), 1))()
    for k, (g, c2w, T) in enumerate(subs):
        T = np.asarray(T, np.float64)[:3, :4]
        if c2w is not None and (not c2w.is_cuda or not c2w.is_contiguous() or c2w.dim() != 2 or c2w.shape[1] != 12):
            raise ValueError("c2w must be a contiguous [k, 12] device tensor")
        arr[k] = L.ls_submap_adjust(g.n, 0 if c2w is None else c2w.shape[0], g.mean.data_ptr(), g.quat.data_ptr(),
                                    None if c2w is None else c2w.data_ptr(),
                                    (C.c_float * 12)(*[float(v) for v in T.reshape(-1)]))
    L.ls_adjust_submaps(arr, len(subs), _stream())


def overlap_ratio(p_mean: torch.Tensor, q_mean: torch.Tensor, T, tau: float, work=None):
    """Geometric overlap ratio of two Gaussian sets (means [3, n] device
    tensors) under the estimate T (3x4 or 4x4) of T_{P->Q}: returns
    (ratio, reciprocal pairs, pairs closer than tau, nn_pq, nn_qp); the two
    counts are read back to the host."""
    for t in (p_mean, q_mean):
        if t.dim() != 2 or t.shape[0] != 3 or not t.is_contiguous() or not t.is_cuda:
            raise ValueError("means must be contiguous [3, n] device tensors")
    n_p, n_q = p_mean.shape[1], q_mean.shape[1]
    dev = p_mean.device
    need = L.ls_overlap_workspace_size(n_p, n_q)
    if work is None or work.numel() < need:
        work = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    nn_pq = torch.empty(n_p, dtype=torch.int32, device=dev)
    nn_qp = torch.empty(n_q, dtype=torch.int32, device=dev)
    counts = torch.empty(2, dtype=torch.int32, device=dev)
    Tc = (C.c_float * 12)(*[float(v) for v in np.asarray(T, np.float64)[:3, :4].reshape(-1)])
    L.ls_overlap_ratio(_ptr(p_mean), n_p, _ptr(q_mean), n_q, Tc, float(tau), _ptr(nn_pq), _ptr(nn_qp), _ptr(counts),
                       _ptr(work), work.numel(), _stream())
    pairs, inliers = (int(v) for v in counts.cpu())
    return (inliers / pairs if pairs else 0.0), pairs, inliers, nn_pq, nn_qp


def prune_gaussians(g: "GaussianSet", o_thre: float, extra=(), work=None):
    """Opacity pruning of a Gaussian set (supplement, submap update): returns
    (GaussianSet of the kept Gaussians, kept indices [k] int32 device tensor,
    compacted extra arrays).  `extra` holds further [c, n] (or [n]) float32
    device tensors compacted with the same selection (e.g. optimiser moments).
    The kept count is read back to the host."""
    n = g.n
    dev = g.mean.device
    srcs = [getattr(g, k) for k in GaussianSet.FIELDS] + list(extra)
    if len(srcs) > L.LS_PRUNE_MAX_ARRAYS:
        raise ValueError(f"at most {L.LS_PRUNE_MAX_ARRAYS} arrays per call")
    dsts = [torch.empty_like(t) for t in srcs]
    arr = (L.ls_prune_array * len(srcs))()
    for i, (a, b) in enumerate(zip(srcs, dsts)):
        if a.dtype != torch.float32 or not a.is_contiguous() or a.shape[-1] != n:
            raise ValueError("arrays must be contiguous float32 [c, n] or [n]")
        arr[i] = L.ls_prune_array(a.data_ptr(), b.data_ptr(), 1 if a.dim() == 1 else a.shape[0], 0)
    kept = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    count = torch.empty(1, dtype=torch.int32, device=dev)
    need = L.ls_prune_workspace_size(n)
    if work is None or work.numel() < need:
        work = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
    L.ls_prune_gaussians(_ptr(g.opacity_logit), n, float(o_thre), arr, len(srcs), _ptr(kept), _ptr(count),
                         _ptr(work), work.numel(), _stream())
    k = int(count.item())
    views = [(d.view(-1)[: d.shape[0] * k].view(d.shape[0], k) if d.dim() == 2 else d[:k]) for d in dsts]
    out = GaussianSet(*views[:5])
    return out, kept[:k], views[5:]


def adam(groups, step: int, beta1=0.9, beta2=0.999, eps=1e-8, zero_grad=True):
    """Fused Adam over (param, grad, m, v, lr) tuples of float32 device tensors."""
    for i in range(0, len(groups), 16):
        chunk = groups[i: i + 16]
        arr = (L.ls_adam_group * len(chunk))(*[
            L.ls_adam_group(p.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(), p.numel(), lr)
            for (p, g, m, v, lr) in chunk])
        L.ls_adam(arr, len(chunk), step, beta1, beta2, eps, 1 if zero_grad else 0, _stream())


class _RenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, batch: RenderBatch, bg, pose, *params):
        batch.project(pose)
        batch.bin_sort()
        batch.render_fwd(bg)
        ctx.batch = batch
        ctx.bg = bg
        ctx.save_for_backward(pose if pose is not None else torch.empty(0))
        ctx.has_pose = pose is not None
        return batch.rgb.clone(), batch.depth.clone(), batch.alpha.clone()

    @staticmethod
    def backward(ctx, g_rgb, g_depth, g_alpha):
        batch = ctx.batch
        (pose,) = ctx.saved_tensors
        pose = pose if ctx.has_pose else None
        want_g = any(ctx.needs_input_grad[3:])
        grads = [g.zeros_like() for g in batch.gsets] if want_g else None
        # renders that share a Gaussian set share one gradient set
        if grads is not None:
            seen = {}
            for i, g in enumerate(batch.gsets):
                key = g.mean.data_ptr()
                if key in seen:
                    grads[i] = grads[seen[key]]
                else:
                    seen[key] = i
        pose_grad = torch.zeros_like(pose) if (pose is not None and ctx.needs_input_grad[2]) else None
        batch.render_bwd(
            up_rgb=None if g_rgb is None else g_rgb.contiguous(),
            up_depth=None if g_depth is None else g_depth.contiguous(),
            up_alpha=None if g_alpha is None else g_alpha.contiguous(),
            grads=grads, pose=pose, pose_grad=pose_grad, bg=ctx.bg)
        out = [None, None, pose_grad]
        uniq = []
        seen_ptr = set()
        for g in (grads or []):
            if id(g) in seen_ptr:
                continue
            seen_ptr.add(id(g))
            uniq.append(g)
        if grads is None:
            out += [None] * (len(ctx.needs_input_grad) - 3)
        else:
            for g in uniq:
                out += g.tensors()
        return tuple(out)


def render(batch: RenderBatch, pose: torch.Tensor | None = None, bg=None):
    """Differentiable render of every job of `batch`.  Returns flat (rgb [3P],
    depth [P], alpha [P]); gradients flow to `pose` ([R,7]) and to the
    Gaussian tensors of the batch's distinct Gaussian sets."""
    params = []
    seen = set()
    for g in batch.gsets:
        if g.mean.data_ptr() in seen:
            continue
        seen.add(g.mean.data_ptr())
        params += g.tensors()
    return _RenderFn.apply(batch, bg, pose, *params)
