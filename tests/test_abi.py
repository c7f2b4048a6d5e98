"""The C-ABI library loads on a CPU-only host, exports every function that
include/loopsplat.h declares, and its struct layouts match the binding.
No compute call is made (there is no GPU here)."""

import ctypes as C
import os
import re

import pytest

from paper_2408_10154_amd import lib as L
from paper_2408_10154_amd import register as REG

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h")]


def declared():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(ls_[a-z0-9_]+)\s*\(", text, re.M):
            names.add(m.group(1))
    return names


def test_header_declares_the_boundary():
    names = declared()
    for must in ["ls_project", "ls_bin_sort", "ls_render_fwd", "ls_render_bwd"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = L.load()
    missing = [n for n in sorted(declared()) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    assert set(L.declared_functions()) == declared()


@pytest.mark.parametrize("name", ["ls_prune_array", "ls_loss_params", "ls_mapping_params", "ls_submap_adjust", "ls_pair", "ls_reg_params", "ls_reg_result", "ls_server_params", "ls_server_stats", "ls_gaussians", "ls_intrinsics", "ls_render_job", "ls_batch_info", "ls_projected",
                                  "ls_bins", "ls_image", "ls_image_grad", "ls_gaussian_grads", "ls_adam_group",
                                  "ls_adam_array", "ls_gaussian_adam", "ls_pose_adam"])
def test_struct_layouts_match(name):
    lib = L.load()
    assert lib.ls_struct_size(name.encode()) == C.sizeof(getattr(L, name))


def test_invalid_arguments_are_rejected_without_a_device():
    lib = L.load()
    h = C.c_void_p()
    assert lib.ls_batch_create(None, 0, C.byref(h)) == L.LS_ERR_INVALID
    assert b"R >= 1" in lib.ls_last_error()
    job = (L.ls_render_job * 1)()
    job[0].K = L.ls_intrinsics(100.0, 100.0, 8.0, 8.0, 0, 16)  # zero width
    assert lib.ls_batch_create(job, 1, C.byref(h)) == L.LS_ERR_INVALID
    job[0].K = L.ls_intrinsics(100.0, 100.0, 8.0, 8.0, 16, 16)
    job[0].g.n = 5  # n > 0 with NULL arrays
    assert lib.ls_batch_create(job, 1, C.byref(h)) == L.LS_ERR_INVALID
    assert lib.ls_adam(None, 0, 1, 0.9, 0.999, 1e-8, 0, None) == L.LS_ERR_INVALID
    grp = (L.ls_adam_group * 1)()
    assert lib.ls_adam(grp, 1, 0, 0.9, 0.999, 1e-8, 0, None) == L.LS_ERR_INVALID  # step 0
    assert lib.ls_fill_i32(None, 4, 0, None) == L.LS_ERR_INVALID
    assert lib.ls_render_bwd_project_adam(None, None, None, None, None, None, 1, 0.9, 0.999, 1e-8, None,
                                          None) == L.LS_ERR_INVALID
    assert lib.ls_render_bwd_tiles_l1(None, None, None, None, None, None, None, None, None, 0, None) == L.LS_ERR_INVALID
    assert lib.ls_loss_l1_tiles(None, None, None, None) == L.LS_ERR_INVALID
    assert lib.ls_loss_isotropic(None, -1, 1.0, None, None, None, None) == L.LS_ERR_INVALID
    assert lib.ls_loss_isotropic(None, 4, 1.0, None, None, None, None) == L.LS_ERR_INVALID  # NULL arrays
    sub = L.ls_submap_adjust(0, 0, None, None, None, (C.c_float * 12)(2, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0))
    assert lib.ls_adjust_submaps(C.byref(sub), 1, None) == L.LS_ERR_INVALID  # not a rotation
    assert b"rigid" in lib.ls_last_error()
    sub = L.ls_submap_adjust(5, 0, None, None, None, (C.c_float * 12)(1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0))
    assert lib.ls_adjust_submaps(C.byref(sub), 1, None) == L.LS_ERR_INVALID  # NULL arrays
    assert lib.ls_adjust_submaps(None, -1, None) == L.LS_ERR_INVALID
    T = (C.c_float * 12)(1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0)
    fake = C.c_void_p(256)  # never dereferenced: the calls fail validation first
    assert lib.ls_overlap_ratio(fake, 4, fake, 4, T, 0.0, fake, fake, fake, fake, 1 << 30, None) == L.LS_ERR_INVALID
    assert lib.ls_overlap_ratio(fake, 4, fake, 4, T, 0.1, fake, fake, fake, fake, 0, None) == L.LS_ERR_CAPACITY
    assert lib.ls_overlap_workspace_size(1000, 2000) > 0 and lib.ls_overlap_workspace_size(-1, 5) == 0
    prm = L.ls_mapping_params(1.5, 1.0, 1.0, 0)  # lambda_ssim outside [0, 1]
    assert lib.ls_loss_mapping(None, None, None, None, C.byref(prm), None, None, None, None, None) == L.LS_ERR_INVALID
    assert lib.ls_struct_size(b"no_such_struct") == -1
    with pytest.raises(L.LsError):
        L.check(L.LS_ERR_INVALID)


def test_register_pair_rejects_bad_parameters_before_touching_a_device():
    lib = L.load()
    pair = L.ls_pair()
    prm = L.ls_reg_params(0, 0.01, 0.01, 0.9, 0.999, 1e-8)  # iters = 0
    res = L.ls_reg_result()
    assert lib.ls_register_pair(C.byref(pair), C.byref(prm), None, 0, 0, C.byref(res), None) == L.LS_ERR_INVALID
    prm.iters = 10
    assert lib.ls_register_pair(C.byref(pair), C.byref(prm), None, 0, 0, C.byref(res),
                                None) == L.LS_ERR_INVALID  # no views
    assert lib.ls_fuse_estimates(None, None, None, 0, None) == L.LS_ERR_INVALID


def _host_pair(vp=3, vq=2, n_p=1000, n_q=700, w=64, h=48):
    """An ls_pair whose device pointers are placeholders: only host-side
    calls may see it."""
    fake = 256
    pair = L.ls_pair()
    pair.P = L.ls_gaussians(n_p, fake, fake, fake, fake, fake)
    pair.Q = L.ls_gaussians(n_q, fake, fake, fake, fake, fake)
    pair.vP, pair.vQ = vp, vq
    pair.rgbP = pair.depthP = pair.rgbQ = pair.depthQ = fake
    eye = [1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0]
    keep = [(C.c_float * (12 * vp))(*(eye * vp)), (C.c_float * (12 * vq))(*(eye * vq))]
    pair.c2wP = C.cast(keep[0], C.c_void_p)
    pair.c2wQ = C.cast(keep[1], C.c_void_p)
    pair.K = L.ls_intrinsics(50.0, 50.0, w / 2, h / 2, w, h)
    return pair, keep


def test_register_workspace_query_without_a_device():
    """ls_register_workspace_size is host-only: it grows with the instance
    capacity (8 bytes per instance plus the sort buffers), with the views and
    with the Gaussians, rejects what ls_register_pair rejects, and the pair
    call itself refuses a short workspace before any device work, reporting
    the bytes it needs."""
    pair, keep = _host_pair()
    prm = L.ls_reg_params(10, 0.01, 0.01, 0.9, 0.999, 1e-8)
    b0 = L.ls_register_workspace_size(pair, prm, 0)
    b1 = L.ls_register_workspace_size(pair, prm, 100_000)
    b2 = L.ls_register_workspace_size(pair, prm, 200_000)
    assert 0 < b0 < b1 < b2 and b2 - b1 >= 8 * 100_000
    more_views, k2 = _host_pair(vp=6)
    assert L.ls_register_workspace_size(more_views, prm, 100_000) > b1
    more_g, k3 = _host_pair(n_q=5000)
    assert L.ls_register_workspace_size(more_g, prm, 100_000) > b1
    lib = L.load()
    out = C.c_size_t(0)
    assert lib.ls_register_workspace_size(C.byref(pair), C.byref(prm), -1, C.byref(out)) == L.LS_ERR_INVALID
    bad = L.ls_reg_params(0, 0.01, 0.01, 0.9, 0.999, 1e-8)
    assert lib.ls_register_workspace_size(C.byref(pair), C.byref(bad), 10, C.byref(out)) == L.LS_ERR_INVALID
    res = L.ls_reg_result()
    assert lib.ls_register_pair(C.byref(pair), C.byref(prm), C.c_void_p(256), 1024, 100_000, C.byref(res),
                                None) == L.LS_ERR_CAPACITY
    assert res.workspace_required == b1 and res.instances_required == 0


def test_server_rejects_bad_parameters_without_a_device():
    lib = L.load()
    h = C.c_void_p()
    prm = L.ls_server_params(1 << 30, 0, 16, 1.5, 1)  # max_slots = 0
    assert lib.ls_server_create(C.byref(prm), C.byref(h)) == L.LS_ERR_INVALID
    prm = L.ls_server_params(1 << 30, 4, 16, 0.1, 1)  # headroom < 0.25
    assert lib.ls_server_create(C.byref(prm), C.byref(h)) == L.LS_ERR_INVALID
    prm = L.ls_server_params(1 << 30, 4, 16, 1.5, 1, -1)  # negative pixel cap
    assert lib.ls_server_create(C.byref(prm), C.byref(h)) == L.LS_ERR_INVALID
    assert lib.ls_register_poll(None, 1, None, None) == L.LS_ERR_INVALID
    assert lib.ls_server_destroy(None) == L.LS_OK


def test_register_pair_rejects_bad_loss_parameters_before_touching_a_device():
    """A structurally valid pair whose loss settings are out of range is
    refused before any device call."""
    import numpy as np

    lib = L.load()
    c2w = np.eye(4, dtype=np.float32)[:3].reshape(-1).copy()
    dummy = np.zeros(16, np.float32)
    pair = L.ls_pair()
    pair.vP, pair.vQ = 1, 0
    pair.rgbP = pair.depthP = dummy.ctypes.data
    pair.c2wP = c2w.ctypes.data
    pair.K = L.ls_intrinsics(10.0, 10.0, 2.0, 2.0, 4, 4)
    res = L.ls_reg_result()
    for kind, track in ((2, L.ls_loss_params(0.6, 50.0, 3, 0)), (1, L.ls_loss_params(1.5, 50.0, 3, 0)),
                        (1, L.ls_loss_params(0.6, float("nan"), 3, 0)), (1, L.ls_loss_params(0.6, 50.0, -1, 0))):
        prm = L.ls_reg_params(10, 0.01, 0.01, 0.9, 0.999, 1e-8, 0.0, 0, kind, track)
        assert lib.ls_register_pair(C.byref(pair), C.byref(prm), None, 0, 0, C.byref(res), None) == L.LS_ERR_INVALID
    # exposure coefficients: flag out of range, or a bad learning rate
    good = L.ls_loss_params(0.6, 50.0, 3, 0)
    for expo, lr in ((2, 0.1), (-1, 0.1), (1, -0.1), (1, float("inf"))):
        prm = L.ls_reg_params(10, 0.01, 0.01, 0.9, 0.999, 1e-8, 0.0, 0, 1, good, expo, lr)
        assert lib.ls_register_pair(C.byref(pair), C.byref(prm), None, 0, 0, C.byref(res), None) == L.LS_ERR_INVALID
    # joint registration: flag out of range, or combined with exposure or early exit
    for expo, joint, patience in ((0, 2, 0), (1, 1, 0), (0, 1, 5)):
        prm = L.ls_reg_params(10, 0.01, 0.01, 0.9, 0.999, 1e-8, 0.0, patience, 1, good, expo, 0.1, joint)
        assert lib.ls_register_pair(C.byref(pair), C.byref(prm), None, 0, 0, C.byref(res), None) == L.LS_ERR_INVALID
    # early-exit rule out of range; negative top-k
    for mode, top_k in ((2, 0), (-1, 0), (0, -1)):
        prm = L.ls_reg_params(10, 0.01, 0.01, 0.9, 0.999, 1e-8, 0.1, 5, 1, good, 0, 0.1, 0, mode, top_k)
        assert lib.ls_register_pair(C.byref(pair), C.byref(prm), None, 0, 0, C.byref(res), None) == L.LS_ERR_INVALID
    with pytest.raises(ValueError):
        REG.default_params(10, exit_rel_tol=0.1, exit_patience=5, exit_mode="plateau")


def test_overlap_noalloc_limits_without_a_device():
    """The static scratch of ls_overlap_ratio_noalloc holds the workspace of
    every size it accepts, and larger or invalid requests are refused before
    any device call."""
    lib = L.load()
    assert L.LS_OVERLAP_NOALLOC_BYTES % 256 == 0
    mx = L.LS_OVERLAP_NOALLOC_MAX_POINTS
    for a in (0, 1, 63, 64, 65, 4097, 131071, 200003, mx - 1, mx):
        for b in (0, 1, 777, 65536, mx):
            assert L.ls_overlap_workspace_size(a, b) <= L.LS_OVERLAP_NOALLOC_BYTES, (a, b)
    T = (C.c_float * 12)(1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0)
    fake = C.c_void_p(256)  # never dereferenced: the checks fail first
    assert lib.ls_overlap_ratio_noalloc(fake, mx + 1, fake, 10, T, C.c_float(0.2), fake, fake, fake,
                                        None) == L.LS_ERR_CAPACITY
    assert b"LS_OVERLAP_NOALLOC_MAX_POINTS" in lib.ls_last_error()
    assert lib.ls_overlap_ratio_noalloc(fake, 10, fake, mx + 1, T, C.c_float(0.2), fake, fake, fake,
                                        None) == L.LS_ERR_CAPACITY
    assert lib.ls_overlap_ratio_noalloc(None, 10, fake, 10, T, C.c_float(0.2), fake, fake, fake,
                                        None) == L.LS_ERR_INVALID
    assert lib.ls_overlap_ratio_noalloc(fake, 10, fake, 10, T, C.c_float(0.0), fake, fake, fake,
                                        None) == L.LS_ERR_INVALID


def test_prune_rejects_bad_arguments_without_a_device():
    lib = L.load()
    fake = C.c_void_p(256)
    arr = (L.ls_prune_array * 1)(L.ls_prune_array(256, 512, 3, 0))
    assert L.ls_prune_workspace_size(-1) == 0 and L.ls_prune_workspace_size(0) > 0
    assert L.ls_prune_workspace_size(10_000) >= L.ls_prune_workspace_size(100)
    for n, o, narr, work_bytes, expect in ((-1, 0.5, 1, 1 << 20, L.LS_ERR_INVALID), (10, 0.0, 1, 1 << 20, L.LS_ERR_INVALID),
                                           (10, 1.0, 1, 1 << 20, L.LS_ERR_INVALID), (10, 0.5, 17, 1 << 20, L.LS_ERR_INVALID),
                                           (10_000_000, 0.5, 1, 16, L.LS_ERR_CAPACITY)):
        assert lib.ls_prune_gaussians(fake, n, C.c_float(o), arr, narr, fake, fake, fake, work_bytes,
                                      None) == expect, (n, o, narr)
    bad = (L.ls_prune_array * 1)(L.ls_prune_array(256, 512, -1, 0))
    assert lib.ls_prune_gaussians(fake, 10, C.c_float(0.5), bad, 1, fake, fake, fake, 1 << 20, None) == L.LS_ERR_INVALID
