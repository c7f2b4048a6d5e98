"""Pins of the FP64 rasterizer oracle against closed forms, library routines,
invariants and brute force.  CPU only."""

import math

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

from oracle import raster as R
from paper_2408_10154_amd import synth

F64 = torch.float64


def one_gaussian(mean, log_scale, quat=(1, 0, 0, 0), opacity_logit=8.0, rgb=(0.2, 0.5, 0.9)):
    g = dict(
        mean=np.asarray(mean, np.float64).reshape(3, -1),
        log_scale=np.asarray(log_scale, np.float64).reshape(3, -1),
        quat=np.asarray(quat, np.float64).reshape(4, -1),
        opacity_logit=np.asarray([opacity_logit], np.float64).reshape(-1),
        rgb=np.asarray(rgb, np.float64).reshape(3, -1),
    )
    return g


def stack_gaussians(gs):
    return {k: np.concatenate([g[k] for g in gs], axis=-1) for k in gs[0]}


def w2c_eye():
    return torch.as_tensor(np.concatenate([np.eye(3), np.zeros((3, 1))], 1))


# ---------------------------------------------------------------- projection


def test_quaternion_matches_scipy():
    rng = np.random.default_rng(5)
    q = rng.normal(size=(64, 4)) * rng.uniform(0.2, 3.0, size=(64, 1))  # unnormalised
    ours = R.quat_to_rotmat(torch.as_tensor(q)).numpy()
    ref = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()  # scipy takes (x, y, z, w)
    np.testing.assert_allclose(ours, ref, atol=1e-12)


@pytest.mark.parametrize("x", [0.0, 0.35, -0.6])
def test_axis_aligned_projected_covariance_closed_form(x):
    """R = I, camera = I at (x, 0, z):
    Sigma2D = diag((f/z)^2 sx^2 + (f x / z^2)^2 sz^2 + eps, (f/z)^2 sy^2 + eps)."""
    f, z = 300.0, 2.5
    sx, sy, sz = 0.05, 0.02, 0.08
    g = R.to_f64(one_gaussian([x, 0.0, z], np.log([sx, sy, sz])))
    cam = R.Camera(f, f, 64, 48, 128, 96)
    pr = R.project(g["mean"], g["log_scale"], g["quat"], cam, w2c_eye())
    cov = pr["cov2d"][0].numpy()
    expect_a = (f / z) ** 2 * sx**2 + (f * x / z**2) ** 2 * sz**2 + R.EPS_2D
    expect_c = (f / z) ** 2 * sy**2 + R.EPS_2D
    np.testing.assert_allclose(cov, [[expect_a, 0.0], [0.0, expect_c]], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(pr["u"].numpy(), [f * x / z + 64], rtol=1e-14)
    # conic is the inverse of the 2D covariance, laid out (A, B, C)
    A, B, C = pr["conic"][0].numpy()
    np.testing.assert_allclose(np.array([[A, B], [B, C]]) @ cov, np.eye(2), atol=1e-12)


def test_rotated_gaussian_swaps_axes():
    """90 deg about the optical axis swaps the x and y extents (pins the
    quaternion order w, x, y, z and the R S S^T R^T form)."""
    f, z = 300.0, 2.0
    sx, sy, sz = 0.06, 0.02, 0.03
    h = math.radians(45.0)
    g = R.to_f64(one_gaussian([0.0, 0.0, z], np.log([sx, sy, sz]), quat=[math.cos(h), 0, 0, math.sin(h)]))
    cam = R.Camera(f, f, 64, 48, 128, 96)
    cov = R.project(g["mean"], g["log_scale"], g["quat"], cam, w2c_eye())["cov2d"][0].numpy()
    np.testing.assert_allclose(cov, np.diag([(f / z * sy) ** 2 + R.EPS_2D, (f / z * sx) ** 2 + R.EPS_2D]),
                               rtol=1e-12, atol=1e-12)


def test_cull_near_plane_and_offscreen():
    g = R.to_f64(stack_gaussians([
        one_gaussian([0.0, 0.0, 0.15], np.log([0.02] * 3)),   # in front of the near plane
        one_gaussian([0.0, 0.0, -2.0], np.log([0.02] * 3)),   # behind the camera
        one_gaussian([50.0, 0.0, 2.0], np.log([0.02] * 3)),   # far off-screen
        one_gaussian([0.0, 0.0, 2.0], np.log([0.02] * 3)),    # visible
    ]))
    cam = R.Camera(100, 100, 32, 32, 64, 64)
    pr = R.project(g["mean"], g["log_scale"], g["quat"], cam, w2c_eye())
    assert list(pr["radius"] > 0) == [False, False, False, True]
    assert list(pr["tiles"] > 0) == [False, False, False, True]


def test_radius_is_three_sigma_ceil():
    f, z, s = 200.0, 2.0, 0.05
    g = R.to_f64(one_gaussian([0.0, 0.0, z], np.log([s, s, s])))
    cam = R.Camera(f, f, 32, 32, 64, 64)
    pr = R.project(g["mean"], g["log_scale"], g["quat"], cam, w2c_eye())
    sd = math.sqrt((f / z * s) ** 2 + R.EPS_2D)
    assert pr["radius"][0] == math.ceil(3 * sd)


def test_tile_rect_worked_cases():
    cam = R.Camera(100, 100, 40, 40, 80, 70)  # 5 x 5 tiles
    u = np.array([24.0, 24.0, 0.5, 79.0], np.float32)
    v = np.array([24.0, 8.0, 0.5, 69.0], np.float32)
    r = np.array([8, 7, 3, 20])
    x0, x1, y0, y1 = R.tile_rect_f32(u, v, r, cam)
    # [16, 32] touches tiles 1 and 2 (conservative at the right edge)
    assert (x0[0], x1[0], y0[0], y1[0]) == (1, 3, 1, 3)
    # [17, 31] stays inside tile 1; in y [1, 15] stays in tile 0
    assert (x0[1], x1[1], y0[1], y1[1]) == (1, 2, 0, 1)
    # clamped at the image origin
    assert (x0[2], x1[2], y0[2], y1[2]) == (0, 1, 0, 1)
    # clamped at the far edge (5 tiles each way)
    assert (x0[3], x1[3], y0[3], y1[3]) == (3, 5, 3, 5)


# ---------------------------------------------------------------- binning


def test_bin_sort_matches_brute_force_with_ties():
    sc = synth.scene_tiny(3, 300, 96, 64, 120.0)
    cam = R.Camera(**sc["cam"])
    g = R.to_f64(sc["gauss"])
    pr = R.project(g["mean"], g["log_scale"], g["quat"], cam, w2c_eye())
    z32 = pr["z32"].copy()
    z32[10:40] = z32[10]  # deliberate equal-depth ties
    z32[200:260:3] = np.float32(2.25)
    tile_of, gid, ranges = R.bin_sort(pr["u32"], pr["v32"], z32, pr["radius"], cam)
    x0, x1, y0, y1 = pr["rect"]
    for t in range(cam.tiles_x * cam.tiles_y):
        ty, tx = divmod(t, cam.tiles_x)
        members = [i for i in range(len(z32)) if pr["radius"][i] > 0 and x0[i] <= tx < x1[i] and y0[i] <= ty < y1[i]]
        members.sort(key=lambda i: (float(z32[i]), i))
        s, e = ranges[t]
        assert list(gid[s:e]) == members
        assert np.all(tile_of[s:e] == t)
    assert len(gid) == int(pr["tiles"].sum())


# ---------------------------------------------------------------- compositing


def test_single_opaque_gaussian_exact_colour():
    """o exp(-s) >= 0.99 at a pixel => C = 0.99 c + 0.01 bg, D = 0.99 z, A = 0.99."""
    cam = R.Camera(200, 200, 32, 32, 64, 64)
    z = 2.0
    g = R.to_f64(one_gaussian([0.0, 0.0, z], np.log([0.05] * 3), opacity_logit=9.0, rgb=(0.2, 0.5, 0.9)))
    bg = torch.tensor([0.1, 0.3, 0.7], dtype=F64)
    out = R.render(g, cam, w2c_eye(), bg=bg)
    # the pixel whose centre is the projected centre (32, 32) is pixel index 31.5 -> use (31, 31): s tiny
    a = R.ALPHA_MAX
    np.testing.assert_allclose(out["rgb"][:, 31, 31].numpy(), a * np.array([0.2, 0.5, 0.9]) + (1 - a) * bg.numpy(),
                               rtol=1e-12)
    np.testing.assert_allclose(out["depth"][31, 31].item(), a * z, rtol=1e-12)
    np.testing.assert_allclose(out["alpha"][31, 31].item(), a, rtol=1e-12)


def test_faint_gaussian_is_skipped_but_counted():
    cam = R.Camera(200, 200, 32, 32, 64, 64)
    g = R.to_f64(one_gaussian([0.0, 0.0, 2.0], np.log([0.05] * 3), opacity_logit=-7.0))
    bg = torch.tensor([0.1, 0.3, 0.7], dtype=F64)
    out = R.render(g, cam, w2c_eye(), bg=bg)
    np.testing.assert_allclose(out["rgb"][:, 31, 31].numpy(), bg.numpy(), rtol=0, atol=0)
    assert out["alpha"][31, 31].item() == 0.0
    assert out["n_last"][31, 31] == 1


def test_two_gaussians_order_by_depth():
    """C = a1 c1 + (1 - a1) a2 c2, and swapping depths swaps the order."""
    cam = R.Camera(200, 200, 32, 32, 64, 64)
    o1, o2 = 0.6, 0.7
    c1, c2 = np.array([1.0, 0.0, 0.0]), np.array([0.0, 0.0, 1.0])
    lg = lambda o: math.log(o / (1 - o))  # noqa: E731
    # centres project exactly onto pixel centre (31.5, 31.5): x = (31.5 - 32) z / f
    def mk(z, o, c):
        return one_gaussian([-0.5 * z / 200, -0.5 * z / 200, z], np.log([0.05] * 3), opacity_logit=lg(o), rgb=c)
    out = R.render(R.to_f64(stack_gaussians([mk(2.0, o1, c1), mk(3.0, o2, c2)])), cam, w2c_eye())
    np.testing.assert_allclose(out["rgb"][:, 31, 31].numpy(), o1 * c1 + (1 - o1) * o2 * c2, rtol=1e-12)
    out = R.render(R.to_f64(stack_gaussians([mk(3.0, o1, c1), mk(2.0, o2, c2)])), cam, w2c_eye())
    np.testing.assert_allclose(out["rgb"][:, 31, 31].numpy(), o2 * c2 + (1 - o2) * o1 * c1, rtol=1e-12)


def test_stop_before_transmittance_floor():
    """alpha 0.99, 0.5, 0.99 at one pixel: T goes 1 -> 0.01 -> 0.005, and the
    third entry would take it to 5e-5 < 1e-4, so compositing stops before it."""
    cam = R.Camera(200, 200, 32, 32, 64, 64)
    lg = lambda o: math.log(o / (1 - o))  # noqa: E731
    cs = [np.array([1.0, 0, 0]), np.array([0, 1.0, 0]), np.array([0, 0, 1.0])]
    gs = [one_gaussian([-0.5 * z / 200, -0.5 * z / 200, z], np.log([0.05] * 3), opacity_logit=ol, rgb=c)
          for z, ol, c in zip([2.0, 2.5, 3.0], [12.0, lg(0.5), 12.0], cs)]
    out = R.render(R.to_f64(stack_gaussians(gs)), cam, w2c_eye())
    a = R.ALPHA_MAX
    assert out["n_last"][31, 31] == 2
    np.testing.assert_allclose(out["rgb"][:, 31, 31].numpy(), a * cs[0] + (1 - a) * 0.5 * cs[1], rtol=1e-9)
    np.testing.assert_allclose(out["T_final"][31, 31].item(), (1 - a) * 0.5, rtol=1e-12)


def test_transmittance_invariants_small_scene():
    """with every colour 1 and bg 0, C = sum w = 1 - T_final = alpha;
    T_final >= T_STOP; alpha within [0, 1 - T_STOP]."""
    sc = synth.scene_small(0, n=600)
    cam = R.Camera(**sc["cam"])
    g = R.to_f64(sc["gauss"])
    g["rgb"] = torch.ones_like(g["rgb"])
    out = R.render(g, cam, torch.as_tensor(sc["w2c"], dtype=F64))
    for ch in range(3):
        np.testing.assert_allclose(out["rgb"][ch].numpy(), out["alpha"].numpy(), atol=1e-12)
    assert out["T_final"].min().item() >= R.T_STOP
    assert out["alpha"].min().item() >= 0.0
    assert out["alpha"].max().item() <= 1 - R.T_STOP


def test_tiled_composite_equals_brute_force():
    """the tiled path equals a per-pixel Python loop over a globally sorted
    candidate list, on every pixel of a small image."""
    sc = synth.scene_tiny(7, 150, 40, 32, 60.0)
    cam = R.Camera(**sc["cam"])
    g = R.to_f64(sc["gauss"])
    pose = torch.as_tensor(sc["target_pose"], dtype=F64)
    bg = [0.05, 0.1, 0.2]
    out = R.render(g, cam, torch.as_tensor(sc["w2c"], dtype=F64), pose, bg=torch.tensor(bg, dtype=F64))
    for py in range(cam.height):
        for px in range(cam.width):
            col, dep, T, n_last = R.brute_force_pixel(g, cam, sc["w2c"], pose, px, py, bg=bg)
            np.testing.assert_allclose(out["rgb"][:, py, px].numpy(), col, rtol=1e-11, atol=1e-13)
            np.testing.assert_allclose(out["depth"][py, px].item(), dep, rtol=1e-11, atol=1e-13)
            np.testing.assert_allclose(out["T_final"][py, px].item(), T, rtol=1e-11)
            assert out["n_last"][py, px] == n_last


def quat_mul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([
        w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
        w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
        w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
        w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2,
    ])


def test_moving_gaussians_equals_moving_camera():
    """transforming every Gaussian by T (mean R mu + t, quaternion q_T q)
    and rendering with w2c equals rendering the originals with w2c o T.
    Also: a pose correction Delta equals the camera Delta o w2c."""
    sc = synth.scene_tiny(11, 200, 48, 40, 70.0)
    cam = R.Camera(**sc["cam"])
    gnp = {k: v.astype(np.float64) for k, v in sc["gauss"].items()}
    tpose = synth.perturbation(np.random.default_rng(1), 7.0, 0.1).astype(np.float64)
    qn = tpose[:4] / np.linalg.norm(tpose[:4])
    rot = Rotation.from_quat(qn[[1, 2, 3, 0]]).as_matrix()
    moved = dict(gnp)
    moved["mean"] = rot @ gnp["mean"] + tpose[4:, None]
    moved["quat"] = np.stack([quat_mul(qn, gnp["quat"][:, i]) for i in range(gnp["quat"].shape[1])], 1)
    w2c = np.concatenate([np.eye(3), np.zeros((3, 1))], 1)
    w2c_t = np.concatenate([rot, tpose[4:, None]], 1)  # w2c o T with w2c = I
    a = R.render(R.to_f64(moved), cam, torch.as_tensor(w2c))
    b = R.render(R.to_f64(gnp), cam, torch.as_tensor(w2c_t))
    c = R.render(R.to_f64(gnp), cam, torch.as_tensor(w2c), torch.as_tensor(tpose))
    for x, y in ((a, b), (b, c)):
        np.testing.assert_allclose(x["rgb"].numpy(), y["rgb"].numpy(), atol=1e-9)
        np.testing.assert_allclose(x["depth"].numpy(), y["depth"].numpy(), atol=1e-9)


# ---------------------------------------------------------------- loss + gradients


def test_loss_matches_library_l1_and_is_zero_at_identity():
    """target rendered by the same renderer at the same pose -> L = 0 and a
    zero pose gradient; and L equals torch's summed L1 over valid pixels / count."""
    sc = synth.scene_tiny(2, 120, 32, 24, 40.0)
    cam = R.Camera(**sc["cam"])
    g = R.to_f64(sc["gauss"])
    w2c = torch.as_tensor(sc["w2c"], dtype=F64)
    tgt = R.render(g, cam, w2c)
    pose = R.identity_pose().requires_grad_(True)
    out = R.render(g, cam, w2c, pose)
    loss = R.loss_l1(out["rgb"], out["depth"], tgt["rgb"].detach(), tgt["depth"].detach())
    loss.backward()
    assert loss.item() == 0.0
    assert torch.all(pose.grad == 0)

    rng = np.random.default_rng(0)
    pr = torch.as_tensor(rng.random((3, 24, 32)))
    pd = torch.as_tensor(rng.random((24, 32)) * 3)
    tr = torch.as_tensor(rng.random((3, 24, 32)))
    td = torch.as_tensor(np.where(rng.random((24, 32)) < 0.3, 0.0, rng.random((24, 32)) * 3))
    valid = td > 0
    ref = (torch.nn.functional.l1_loss(pr[:, valid], tr[:, valid], reduction="sum")
           + torch.nn.functional.l1_loss(pd[valid], td[valid], reduction="sum")) / valid.sum()
    np.testing.assert_allclose(R.loss_l1(pr, pd, tr, td).item(), ref.item(), rtol=1e-14)


def _track_case():
    """1x4 image, hand-checked: target depth (1, 2, 0, 4) -> Omega = {0, 1, 3};
    depth errors (0.5, 0.25, -, 6.0) (exact in binary); alpha (1, 0.5, 1, 1);
    colour residual sums (0.6, 3, -, 0.5)."""
    rgb = torch.zeros(3, 1, 4, dtype=F64)
    tgt_rgb = torch.tensor([[[0.1, 1.0, 0.7, 0.0]], [[0.2, 1.0, 0.7, 0.0]], [[0.3, 1.0, 0.7, 0.5]]], dtype=F64)
    depth = torch.tensor([[1.5, 2.25, 7.0, 10.0]], dtype=F64)
    tgt_depth = torch.tensor([[1.0, 2.0, 0.0, 4.0]], dtype=F64)
    alpha = torch.tensor([[1.0, 0.5, 1.0, 1.0]], dtype=F64)
    return rgb, depth, alpha, tgt_rgb, tgt_depth


def test_tracking_loss_hand_values():
    """Eq. 2 with the supplement's masks on a hand-computed case (lambda_c = 0.6):
    per-pixel terms 0.6 * 0.6 + 0.4 * 0.5 = 0.56, 0.6 * 3 + 0.4 * 0.25 = 1.9
    (alpha^3 = 1/8 -> 0.2375), 0.6 * 0.5 + 0.4 * 6 = 2.7; median error 0.5."""
    rgb, depth, alpha, tr, td = _track_case()
    loss, med = R.loss_tracking(rgb, depth, alpha, tr, td, lambda_c=0.6, alpha_power=3, inlier_k=50.0)
    assert med == 0.5
    np.testing.assert_allclose(loss.item(), (0.56 + 0.2375 + 2.7) / 3, rtol=1e-13)
    # K = 10: threshold 5 drops the pixel with error 6 (|Omega| stays 3)
    loss, _ = R.loss_tracking(rgb, depth, alpha, tr, td, lambda_c=0.6, alpha_power=3, inlier_k=10.0)
    np.testing.assert_allclose(loss.item(), (0.56 + 0.2375) / 3, rtol=1e-13)
    # masks off
    loss, _ = R.loss_tracking(rgb, depth, alpha, tr, td, lambda_c=0.6, alpha_power=0, inlier_k=0.0)
    np.testing.assert_allclose(loss.item(), (0.56 + 1.9 + 2.7) / 3, rtol=1e-13)
    # lambda_c = 1: colour only; 0: depth only
    loss, _ = R.loss_tracking(rgb, depth, alpha, tr, td, lambda_c=1.0, alpha_power=0, inlier_k=0.0)
    np.testing.assert_allclose(loss.item(), (0.6 + 3.0 + 0.5) / 3, rtol=1e-13)
    loss, _ = R.loss_tracking(rgb, depth, alpha, tr, td, lambda_c=0.0, alpha_power=0, inlier_k=0.0)
    np.testing.assert_allclose(loss.item(), (0.5 + 0.25 + 6.0) / 3, rtol=1e-13)
    # no valid pixel -> 0
    loss, _ = R.loss_tracking(rgb, depth, alpha, tr, td * 0.0)
    assert loss.item() == 0.0


def test_lower_median_hand_values():
    assert R.lower_median_f32(np.array([0.4, 0.1, 0.3, 0.2])) == np.float32(0.2)
    assert R.lower_median_f32(np.array([5.0, 1.0, 3.0])) == np.float32(3.0)
    assert R.lower_median_f32(np.array([2.0])) == np.float32(2.0)
    assert R.lower_median_f32(np.array([])) == np.float32(0.0)
    assert R.lower_median_f32(np.array([0.0, 0.0, 7.0, 7.0])) == np.float32(0.0)


def test_tracking_loss_reduces_to_l1_and_ignores_gross_outliers():
    """Without masks and with lambda_c = 1/2 the tracking loss is half the
    plain L1 (itself pinned to torch's l1_loss above); a pixel whose depth
    error exceeds 50x the median leaves the numerator unchanged."""
    rng = np.random.default_rng(3)
    pr = torch.as_tensor(rng.random((3, 24, 32)))
    pd = torch.as_tensor(rng.random((24, 32)) * 3 + 0.5)
    tr = torch.as_tensor(rng.random((3, 24, 32)))
    td = torch.as_tensor(np.where(rng.random((24, 32)) < 0.3, 0.0, pd.numpy() + rng.normal(0, 0.01, (24, 32))))
    one = torch.ones(24, 32, dtype=F64)
    lt, _ = R.loss_tracking(pr, pd, one, tr, td, lambda_c=0.5, alpha_power=0, inlier_k=0.0)
    np.testing.assert_allclose(lt.item(), 0.5 * R.loss_l1(pr, pd, tr, td).item(), rtol=1e-13)
    base, med = R.loss_tracking(pr, pd, one, tr, td, lambda_c=0.6)
    n = int((td > 0).sum())
    j = int(np.argmax(td.numpy().ravel() > 0))
    pd2 = pd.clone().view(-1)
    pd2[j] = td.view(-1)[j] + 100.0 * med + 1.0        # a gross depth outlier
    pd2 = pd2.view(24, 32)
    out, med2 = R.loss_tracking(pr, pd2, one, tr, td, lambda_c=0.6)
    y, x = divmod(j, 32)
    term_j = 0.6 * torch.abs(pr[:, y, x] - tr[:, y, x]).sum() + 0.4 * torch.abs(pd[y, x] - td[y, x])
    np.testing.assert_allclose(out.item() * n, base.item() * n - term_j.item(), rtol=1e-10)


def test_tracking_loss_gradient_matches_central_differences():
    """Away from the mask thresholds the masks are constant, and the gradient
    w.r.t. the rendered colour and depth matches central differences."""
    rng = np.random.default_rng(5)
    pr = torch.as_tensor(rng.random((3, 6, 8)), dtype=F64).requires_grad_(True)
    pd = torch.as_tensor(rng.random((6, 8)) + 1.0, dtype=F64).requires_grad_(True)
    al = torch.as_tensor(rng.random((6, 8)), dtype=F64)
    tr = torch.as_tensor(rng.random((3, 6, 8)), dtype=F64)
    td = torch.as_tensor(np.where(rng.random((6, 8)) < 0.2, 0.0, rng.random((6, 8)) + 1.0), dtype=F64)
    al.requires_grad_(True)
    loss, _ = R.loss_tracking(pr, pd, al, tr, td, lambda_c=0.6)
    g_rgb, g_d, g_a = torch.autograd.grad(loss, [pr, pd, al], allow_unused=True)
    assert g_a is None or torch.all(g_a == 0)     # M_a is a weight: no gradient through alpha
    al = al.detach()
    h = 1e-7
    for (c, y, x) in ((0, 1, 2), (2, 4, 7), (1, 0, 0)):
        a, b = pr.detach().clone(), pr.detach().clone()
        a[c, y, x] += h
        b[c, y, x] -= h
        fd = (R.loss_tracking(a, pd.detach(), al, tr, td)[0] - R.loss_tracking(b, pd.detach(), al, tr, td)[0]) / (2 * h)
        np.testing.assert_allclose(g_rgb[c, y, x].item(), fd.item(), rtol=1e-5, atol=1e-9)
    for (y, x) in ((1, 2), (5, 5), (3, 0)):
        a, b = pd.detach().clone(), pd.detach().clone()
        a[y, x] += h
        b[y, x] -= h
        fd = (R.loss_tracking(pr.detach(), a, al, tr, td)[0] - R.loss_tracking(pr.detach(), b, al, tr, td)[0]) / (2 * h)
        np.testing.assert_allclose(g_d[y, x].item(), fd.item(), rtol=1e-5, atol=1e-9)


def _fd_scene():
    sc = synth.scene_tiny(21, 8, 32, 32, 50.0, half_extent=0.5, log_scale_mu=math.log(0.08))
    cam = R.Camera(**sc["cam"])
    return sc, cam


def test_autograd_matches_central_differences():
    """FP64 analytic gradient (autograd of the forward) vs central
    differences, h = 1e-6, on 8 Gaussians at 32x32: every sampled component
    within 1e-6 relative, |fd - g| <= 1e-6 max(|g|, 1e-3 max|g_group|).  A
    sample is rejected when any discrete decision (radius, tile rectangle,
    list order, per-entry skip / clamp / composite, stop position) differs
    between the base point and either side of the step."""
    sc, cam = _fd_scene()
    rng = np.random.default_rng(3)
    wr = torch.as_tensor(rng.normal(size=(3, 32, 32)))
    wd = torch.as_tensor(rng.normal(size=(32, 32)))
    wa = torch.as_tensor(rng.normal(size=(32, 32)))
    w2c = torch.as_tensor(sc["w2c"], dtype=F64)
    base_pose = torch.as_tensor(sc["target_pose"], dtype=F64)

    def f(gd, pose):
        out = R.render(gd, cam, w2c, pose, with_margins=False, with_decisions=True)
        val = (out["rgb"] * wr).sum() + (out["depth"] * wd).sum() + (out["alpha"] * wa).sum()
        dec = (out["decisions"], out["n_last"].tobytes(), out["proj"]["radius"].tobytes(),
               np.asarray(out["proj"]["rect"]).tobytes(), np.asarray(out["bins"][1]).tobytes())
        return val, dec

    g = R.to_f64(sc["gauss"], requires_grad=True)
    pose = base_pose.clone().requires_grad_(True)
    val, dec0 = f(g, pose)
    val.backward()
    grads = {k: v.grad.numpy().copy() for k, v in g.items()}
    grads["pose"] = pose.grad.numpy().copy()

    h = 1e-6
    checked = rejected = 0
    for name in ["mean", "log_scale", "quat", "opacity_logit", "rgb", "pose"]:
        base = (base_pose.numpy() if name == "pose" else R.to_f64(sc["gauss"])[name].numpy()).copy()
        scale = 1e-3 * float(np.abs(grads[name]).max())
        assert scale > 0, name
        for idx in rng.choice(base.size, size=min(base.size, 10), replace=False):
            vals, decs = [], []
            for sgn in (+1, -1):
                gd = {k: v.detach().clone() for k, v in R.to_f64(sc["gauss"]).items()}
                pz = base_pose.clone()
                arr = base.copy().reshape(-1)
                arr[idx] += sgn * h
                if name == "pose":
                    pz = torch.as_tensor(arr.reshape(base.shape))
                else:
                    gd[name] = torch.as_tensor(arr.reshape(base.shape))
                v, d = f(gd, pz)
                vals.append(v.item())
                decs.append(d)
            if decs[0] != dec0 or decs[1] != dec0:
                rejected += 1
                continue
            fd = (vals[0] - vals[1]) / (2 * h)
            an = grads[name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(abs(an), scale), (name, idx, fd, an)
            checked += 1
    assert checked >= 40 and rejected <= 5, (checked, rejected)
