"""ctypes binding of libloopsplat.so (argument marshalling only).

The structures mirror include/loopsplat.h field for field.  `load()` opens the
in-tree library and raises if it has not been built - there is no fallback
implementation.  Every `ls_*` function here has the C function's name and
arguments and raises `LsError` on a negative status.
"""

from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libloopsplat.so")

LS_OK = 0
LS_NOT_READY = 1
LS_ERR_INVALID = -1
LS_ERR_CAPACITY = -2
LS_ERR_BUDGET = -3
LS_ERR_HIP = -4
LS_ERR_NONFINITE = -5
REC_FLOATS = 12
BWD_POSE_ONLY = 1
TILE = 16


class LsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"loopsplat status {status}: {msg}")
        self.status = status


class ls_gaussians(C.Structure):
    _fields_ = [("n", C.c_int32), ("mean", C.c_void_p), ("log_scale", C.c_void_p), ("quat", C.c_void_p),
                ("opacity_logit", C.c_void_p), ("rgb", C.c_void_p)]


class ls_intrinsics(C.Structure):
    _fields_ = [("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
                ("width", C.c_int32), ("height", C.c_int32)]


class ls_render_job(C.Structure):
    _fields_ = [("g", ls_gaussians), ("K", ls_intrinsics), ("w2c", C.c_float * 12)]


class ls_batch_info(C.Structure):
    _fields_ = [("renders", C.c_int32), ("items", C.c_int64), ("tiles", C.c_int32), ("pixels", C.c_int64),
                ("workspace_bytes", C.c_size_t)]


class ls_projected(C.Structure):
    _fields_ = [("rec", C.c_void_p), ("radius", C.c_void_p), ("tiles", C.c_void_p), ("aux", C.c_void_p)]


class ls_bins(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("tile_of", C.c_void_p), ("item", C.c_void_p), ("range", C.c_void_p),
                ("count", C.c_void_p), ("work", C.c_void_p)]


class ls_image(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("depth", C.c_void_p), ("alpha", C.c_void_p), ("T_final", C.c_void_p),
                ("n_last", C.c_void_p)]


class ls_image_grad(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("depth", C.c_void_p), ("alpha", C.c_void_p), ("scale", C.c_void_p)]


class ls_gaussian_grads(C.Structure):
    _fields_ = [("mean", C.c_void_p), ("log_scale", C.c_void_p), ("quat", C.c_void_p),
                ("opacity_logit", C.c_void_p), ("rgb", C.c_void_p)]


class ls_pair(C.Structure):
    _fields_ = [("P", ls_gaussians), ("Q", ls_gaussians), ("vP", C.c_int32), ("vQ", C.c_int32),
                ("rgbP", C.c_void_p), ("depthP", C.c_void_p), ("c2wP", C.c_void_p),
                ("rgbQ", C.c_void_p), ("depthQ", C.c_void_p), ("c2wQ", C.c_void_p), ("K", ls_intrinsics)]


class ls_loss_params(C.Structure):
    _fields_ = [("lambda_c", C.c_float), ("inlier_k", C.c_float), ("alpha_power", C.c_int32), ("pad", C.c_int32)]


class ls_mapping_params(C.Structure):
    _fields_ = [("lambda_ssim", C.c_float), ("lambda_color", C.c_float), ("lambda_depth", C.c_float),
                ("pad", C.c_int32)]


class ls_submap_adjust(C.Structure):
    _fields_ = [("n", C.c_int32), ("n_poses", C.c_int32), ("mean", C.c_void_p), ("quat", C.c_void_p),
                ("c2w", C.c_void_p), ("T", C.c_float * 12)]


class ls_reg_params(C.Structure):
    _fields_ = [("iters", C.c_int32), ("lr_rot", C.c_float), ("lr_trans", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("adam_eps", C.c_float), ("exit_rel_tol", C.c_float),
                ("exit_patience", C.c_int32), ("loss_kind", C.c_int32), ("track", ls_loss_params),
                ("exposure", C.c_int32), ("lr_exposure", C.c_float), ("joint", C.c_int32), ("exit_mode", C.c_int32),
                ("top_k", C.c_int32)]


class ls_prune_array(C.Structure):
    _fields_ = [("src", C.c_void_p), ("dst", C.c_void_p), ("components", C.c_int32), ("pad", C.c_int32)]


class ls_reg_result(C.Structure):
    _fields_ = [("T_PQ", C.c_float * 12), ("per_view_T", C.c_void_p), ("residual", C.c_void_p),
                ("status", C.c_int32), ("iters_done", C.c_int32), ("exposure", C.c_void_p),
                ("instances_required", C.c_int64), ("workspace_required", C.c_int64)]


class ls_server_params(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_size_t), ("max_slots", C.c_int32), ("chunk_iters", C.c_int32),
                ("instance_headroom", C.c_float), ("use_graphs", C.c_int32), ("max_active_pixels", C.c_int64)]


class ls_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64), ("epochs", C.c_int64),
                ("iterations", C.c_int64), ("graph_replays", C.c_int64), ("overflow_retries", C.c_int64),
                ("peak_bytes", C.c_int64), ("active", C.c_int32), ("waiting", C.c_int32),
                ("peak_active", C.c_int32), ("pad", C.c_int32)]


class ls_adam_group(C.Structure):
    _fields_ = [("param", C.c_void_p), ("grad", C.c_void_p), ("m", C.c_void_p), ("v", C.c_void_p),
                ("n", C.c_int64), ("lr", C.c_float)]


class ls_adam_array(C.Structure):
    _fields_ = [("m", C.c_void_p), ("v", C.c_void_p), ("lr", C.c_float)]


class ls_gaussian_adam(C.Structure):
    _fields_ = [("mean", ls_adam_array), ("log_scale", ls_adam_array), ("quat", ls_adam_array),
                ("opacity_logit", ls_adam_array), ("rgb", ls_adam_array)]


class ls_pose_adam(C.Structure):
    _fields_ = [("m", C.c_void_p), ("v", C.c_void_p), ("lr_rot", C.c_float), ("lr_trans", C.c_float)]


LS_ADAM_FUSED_MAX_RENDERS = 16  # renders one ls_render_bwd_project_adam call steps
LS_ISOTROPIC_WORK_FLOATS = 256  # scratch floats of ls_loss_isotropic
LS_OVERLAP_NOALLOC_MAX_POINTS = 524288  # points per set taken by ls_overlap_ratio_noalloc
LS_OVERLAP_NOALLOC_BYTES = 40 << 20     # its static per-device scratch array
LS_PRUNE_MAX_ARRAYS = 16                # arrays one ls_prune_gaussians call compacts

_P = C.c_void_p
_PROTOS = {
    "ls_last_error": (C.c_char_p, []),
    "ls_version": (C.c_int32, []),
    "ls_struct_size": (C.c_int64, [C.c_char_p]),
    "ls_batch_create": (C.c_int32, [C.POINTER(ls_render_job), C.c_int32, C.POINTER(_P)]),
    "ls_batch_destroy": (C.c_int32, [_P]),
    "ls_batch_query": (C.c_int32, [_P, C.c_int64, C.POINTER(ls_batch_info)]),
    "ls_batch_offsets": (C.c_int32, [_P, _P, _P, _P]),
    "ls_project": (C.c_int32, [_P, _P, C.POINTER(ls_projected), _P]),
    "ls_bin_sort": (C.c_int32, [_P, C.POINTER(ls_projected), C.POINTER(ls_bins), _P]),
    "ls_render_fwd": (C.c_int32, [_P, C.POINTER(ls_projected), C.POINTER(ls_bins), _P, C.POINTER(ls_image), _P]),
    "ls_render_bwd": (C.c_int32, [_P, _P, C.POINTER(ls_projected), C.POINTER(ls_bins), _P, C.POINTER(ls_image),
                                  C.POINTER(ls_image_grad), _P, _P, _P]),
    "ls_render_bwd_tiles": (C.c_int32, [_P, _P, C.POINTER(ls_projected), C.POINTER(ls_bins), _P, C.POINTER(ls_image),
                                        C.POINTER(ls_image_grad), C.c_uint32, _P]),
    "ls_render_bwd_tiles_l1": (C.c_int32, [_P, _P, C.POINTER(ls_projected), C.POINTER(ls_bins), _P,
                                           C.POINTER(ls_image), _P, _P, _P, C.c_uint32, _P]),
    "ls_loss_l1_tiles": (C.c_int32, [_P, C.POINTER(ls_bins), _P, _P]),
    "ls_render_bwd_project": (C.c_int32, [_P, _P, C.POINTER(ls_projected), C.POINTER(ls_bins), _P, _P, C.c_uint32,
                                          _P]),
    "ls_render_bwd_project_adam": (C.c_int32, [_P, _P, C.POINTER(ls_projected), C.POINTER(ls_bins),
                                               C.POINTER(ls_gaussian_adam), C.POINTER(ls_pose_adam), C.c_int32,
                                               C.c_float, C.c_float, C.c_float, _P, _P]),
    "ls_render_stats": (C.c_int32, [_P, C.POINTER(ls_projected), C.POINTER(ls_bins), C.POINTER(ls_image), _P, _P]),
    "ls_loss_l1": (C.c_int32, [_P, C.POINTER(ls_image), _P, _P, _P, _P, _P, _P, _P]),
    "ls_loss_tracking": (C.c_int32, [_P, C.POINTER(ls_image), _P, _P, C.POINTER(ls_loss_params), _P, _P, _P, _P, _P,
                                     _P]),
    "ls_loss_mapping": (C.c_int32, [_P, C.POINTER(ls_image), _P, _P, C.POINTER(ls_mapping_params), _P, _P, _P,
                                    _P, _P]),
    "ls_loss_isotropic": (C.c_int32, [_P, C.c_int64, C.c_float, _P, _P, _P, _P]),
    "ls_adjust_submaps": (C.c_int32, [C.POINTER(ls_submap_adjust), C.c_int32, _P]),
    "ls_overlap_workspace_size": (C.c_size_t, [C.c_int32, C.c_int32]),
    "ls_overlap_ratio": (C.c_int32, [_P, C.c_int32, _P, C.c_int32, C.POINTER(C.c_float), C.c_float, _P, _P, _P, _P,
                                     C.c_size_t, _P]),
    "ls_prune_workspace_size": (C.c_size_t, [C.c_int32]),
    "ls_prune_gaussians": (C.c_int32, [_P, C.c_int32, C.c_float, C.POINTER(ls_prune_array), C.c_int32, _P, _P, _P,
                                       C.c_size_t, _P]),
    "ls_overlap_ratio_noalloc": (C.c_int32, [_P, C.c_int32, _P, C.c_int32, C.POINTER(C.c_float), C.c_float, _P, _P,
                                             _P, _P]),
    "ls_adam": (C.c_int32, [C.POINTER(ls_adam_group), C.c_int32, C.c_int32, C.c_float, C.c_float, C.c_float,
                            C.c_int32, _P]),
    "ls_fill_i32": (C.c_int32, [_P, C.c_int64, C.c_int32, _P]),
    "ls_register_workspace_size": (C.c_int32, [C.POINTER(ls_pair), C.POINTER(ls_reg_params), C.c_int64,
                                               C.POINTER(C.c_size_t)]),
    "ls_register_pair": (C.c_int32, [C.POINTER(ls_pair), C.POINTER(ls_reg_params), _P, C.c_size_t, C.c_int64,
                                     C.POINTER(ls_reg_result), _P]),
    "ls_fuse_estimates": (C.c_int32, [_P, _P, _P, C.c_int32, _P]),
    "ls_server_create": (C.c_int32, [C.POINTER(ls_server_params), C.POINTER(_P)]),
    "ls_register_submit": (C.c_int32, [_P, C.POINTER(ls_pair), C.POINTER(ls_reg_params), _P, C.POINTER(C.c_uint64)]),
    "ls_register_poll": (C.c_int32, [_P, C.c_uint64, C.POINTER(ls_reg_result), _P]),
    "ls_server_get_stats": (C.c_int32, [_P, C.POINTER(ls_server_stats)]),
    "ls_server_destroy": (C.c_int32, [_P]),
}

_lib = None


def load():
    """Open libloopsplat.so (once).  Raises if it is missing: build it with
    `python -m paper_2408_10154_amd.build`."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2408_10154_amd.build`")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in _PROTOS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def declared_functions():
    return sorted(_PROTOS)


def check(status: int) -> int:
    if status < 0:
        raise LsError(status, load().ls_last_error().decode(errors="replace"))
    return status


def _call(name, *args):
    return check(getattr(load(), name)(*args))


# Thin wrappers with the C names -------------------------------------------

def ls_batch_create(jobs, R):
    h = C.c_void_p()
    _call("ls_batch_create", jobs, R, C.byref(h))
    return h


def ls_batch_destroy(h):
    return _call("ls_batch_destroy", h)


def ls_batch_query(h, capacity):
    info = ls_batch_info()
    _call("ls_batch_query", h, capacity, C.byref(info))
    return info


def ls_batch_offsets(h, item_off, pix_off, tile_off):
    return _call("ls_batch_offsets", h, item_off, pix_off, tile_off)


def ls_project(h, pose, proj, stream):
    return _call("ls_project", h, pose, C.byref(proj), stream)


def ls_bin_sort(h, proj, bins, stream):
    return _call("ls_bin_sort", h, C.byref(proj), C.byref(bins), stream)


def ls_render_fwd(h, proj, bins, bg, img, stream):
    return _call("ls_render_fwd", h, C.byref(proj), C.byref(bins), bg, C.byref(img), stream)


def ls_render_bwd(h, pose, proj, bins, bg, fwd, up, grads, pose_grad, stream):
    return _call("ls_render_bwd", h, pose, C.byref(proj), C.byref(bins), bg, C.byref(fwd), C.byref(up), grads,
                 pose_grad, stream)


def ls_render_bwd_tiles(h, pose, proj, bins, bg, fwd, up, flags, stream):
    return _call("ls_render_bwd_tiles", h, pose, C.byref(proj), C.byref(bins), bg, C.byref(fwd), C.byref(up), flags,
                 stream)


def ls_render_bwd_tiles_l1(h, pose, proj, bins, bg, fwd, tgt_rgb, tgt_depth, inv_count, flags, stream):
    return _call("ls_render_bwd_tiles_l1", h, pose, C.byref(proj), C.byref(bins), bg, C.byref(fwd), tgt_rgb,
                 tgt_depth, inv_count, flags, stream)


def ls_loss_l1_tiles(h, bins, loss, stream):
    return _call("ls_loss_l1_tiles", h, C.byref(bins), loss, stream)


def ls_render_bwd_project(h, pose, proj, bins, grads, pose_grad, flags, stream):
    return _call("ls_render_bwd_project", h, pose, C.byref(proj), C.byref(bins), grads, pose_grad, flags, stream)


def ls_render_bwd_project_adam(h, pose, proj, bins, adam, pose_adam, step, beta1, beta2, eps, pose_grad, stream):
    return _call("ls_render_bwd_project_adam", h, pose, C.byref(proj), C.byref(bins), adam, pose_adam, step, beta1,
                 beta2, eps, pose_grad, stream)


def ls_render_stats(h, proj, bins, fwd, stats, stream):
    return _call("ls_render_stats", h, C.byref(proj), C.byref(bins), C.byref(fwd), stats, stream)


def ls_loss_l1(h, pred, tgt_rgb, tgt_depth, loss, grad_rgb, grad_depth, grad_scale, stream):
    return _call("ls_loss_l1", h, C.byref(pred), tgt_rgb, tgt_depth, loss, grad_rgb, grad_depth, grad_scale, stream)


def ls_loss_tracking(h, pred, tgt_rgb, tgt_depth, prm, loss, median, grad_rgb, grad_depth, grad_scale, stream):
    return _call("ls_loss_tracking", h, C.byref(pred), tgt_rgb, tgt_depth, C.byref(prm), loss, median, grad_rgb,
                 grad_depth, grad_scale, stream)


def ls_loss_mapping(h, pred, tgt_rgb, tgt_depth, prm, loss, grad_rgb, grad_depth, grad_scale, stream):
    return _call("ls_loss_mapping", h, C.byref(pred), tgt_rgb, tgt_depth, C.byref(prm), loss, grad_rgb, grad_depth,
                 grad_scale, stream)


def ls_loss_isotropic(log_scale, n, lambda_reg, loss, grad_log_scale, work, stream):
    return _call("ls_loss_isotropic", log_scale, n, lambda_reg, loss, grad_log_scale, work, stream)


def ls_adjust_submaps(subs, count, stream):
    return _call("ls_adjust_submaps", subs, count, stream)


def ls_overlap_workspace_size(np_, nq):
    return load().ls_overlap_workspace_size(np_, nq)


def ls_overlap_ratio(p_mean, np_, q_mean, nq, T, tau, nn_pq, nn_qp, counts, work, work_bytes, stream):
    return _call("ls_overlap_ratio", p_mean, np_, q_mean, nq, T, tau, nn_pq, nn_qp, counts, work, work_bytes, stream)


def ls_prune_workspace_size(n):
    return load().ls_prune_workspace_size(n)


def ls_prune_gaussians(logit, n, o_thre, arrays, narrays, kept, count, work, work_bytes, stream):
    return _call("ls_prune_gaussians", logit, n, o_thre, arrays, narrays, kept, count, work, work_bytes, stream)


def ls_overlap_ratio_noalloc(p_mean, np_, q_mean, nq, T, tau, nn_pq, nn_qp, counts, stream):
    return _call("ls_overlap_ratio_noalloc", p_mean, np_, q_mean, nq, T, tau, nn_pq, nn_qp, counts, stream)


def ls_adam(groups, ngroups, step, beta1, beta2, eps, zero_grad, stream):
    return _call("ls_adam", groups, ngroups, step, beta1, beta2, eps, zero_grad, stream)


def ls_register_workspace_size(pair, prm, capacity):
    out = C.c_size_t(0)
    _call("ls_register_workspace_size", C.byref(pair), C.byref(prm), int(capacity), C.byref(out))
    return int(out.value)


def ls_register_pair(pair, prm, work, work_bytes, capacity, result, stream, raise_on_error=True):
    st = getattr(load(), "ls_register_pair")(C.byref(pair), C.byref(prm), work, work_bytes, int(capacity),
                                             C.byref(result), stream)
    return check(st) if raise_on_error else st


def ls_fuse_estimates(est, resid, reverse, n, out):
    return _call("ls_fuse_estimates", est, resid, reverse, n, out)


def ls_fill_i32(ptr, count, value, stream):
    return _call("ls_fill_i32", ptr, count, value, stream)
