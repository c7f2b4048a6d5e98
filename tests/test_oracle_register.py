"""Pins of the registration oracle: Adam against torch.optim.Adam, the
rotation-averaging closed forms, the estimate composition, and recovery of a
known rigid transform on a tiny scene.  CPU only."""

import math

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

from oracle import raster as R
from oracle import register as G
from paper_2408_10154_amd import synth

F64 = torch.float64


def rigid(axis, deg, t):
    out = np.eye(4)
    out[:3, :3] = Rotation.from_rotvec(np.asarray(axis, float) / np.linalg.norm(axis) * math.radians(deg)).as_matrix()
    out[:3, 3] = t
    return out


def test_adam_matches_torch_optim():
    rng = np.random.default_rng(0)
    p0 = rng.normal(size=7)
    ours = torch.tensor(p0.copy())
    ref = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.Adam([ref], lr=0.01, betas=(0.9, 0.999), eps=1e-8)
    m, v = torch.zeros(7, dtype=F64), torch.zeros(7, dtype=F64)
    for step in range(1, 31):
        g = torch.as_tensor(rng.normal(size=7))
        G.adam_step(ours, g, m, v, step, 0.01)
        opt.zero_grad()
        ref.grad = g.clone()
        opt.step()
    np.testing.assert_allclose(ours.numpy(), ref.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_fuse_identical_estimates():
    e = rigid([1, 2, 3], 8.0, [0.1, -0.2, 0.05])
    out = G.fuse([e, e, G.inv_rigid(e)], [0.5, 0.1, 2.0], [False, False, True])
    np.testing.assert_allclose(out, e, atol=1e-12)


@pytest.mark.parametrize("w1,w2", [(1.0, 1.0), (1.0, 3.0), (5.0, 0.5)])
def test_fuse_same_axis_weighted_closed_form(w1, w2):
    """Two rotations about one axis, angles a1 and a2, weights w1 and w2: the
    chordal weighted mean is the rotation about that axis by
    atan2(w1 sin a1 + w2 sin a2, w1 cos a1 + w2 cos a2) (midpoint for equal
    weights).  The translation is the weighted mean."""
    axis = np.array([0.3, -0.5, 0.8])
    a1, a2 = 4.0, 18.0
    t1, t2 = np.array([0.1, 0.0, 0.3]), np.array([-0.2, 0.4, 0.1])
    e1, e2 = rigid(axis, a1, t1), rigid(axis, a2, t2)
    out = G.fuse([e1, e2], [1.0 / w1, 1.0 / w2], [False, False])
    r1, r2 = math.radians(a1), math.radians(a2)
    expect = math.degrees(math.atan2(w1 * math.sin(r1) + w2 * math.sin(r2), w1 * math.cos(r1) + w2 * math.cos(r2)))
    np.testing.assert_allclose(out[:3, :3], rigid(axis, expect, [0, 0, 0])[:3, :3], atol=1e-12)
    np.testing.assert_allclose(out[:3, 3], (w1 * t1 + w2 * t2) / (w1 + w2), atol=1e-12)
    # the same estimates handed in as reverse-direction (inverted) ones give the same result
    back = G.fuse([G.inv_rigid(e1), G.inv_rigid(e2)], [1.0 / w1, 1.0 / w2], [True, True])
    np.testing.assert_allclose(back, out, atol=1e-12)


def test_fuse_zero_residual_dominates():
    e1, e2 = rigid([0, 0, 1], 5.0, [0.1, 0, 0]), rigid([1, 0, 0], 30.0, [0, 1, 0])
    out = G.fuse([e1, e2], [0.0, 1.0], [False, False])
    np.testing.assert_allclose(out, e1, atol=1e-9)


def test_view_estimate_composition():
    """Delta = T_i^-1 T^-1 T_i, the exact keyframe correction when Q = T P,
    gives back T from E = T_i Delta^-1 T_i^-1."""
    t_true = rigid([0.2, 1.0, -0.3], 9.0, [0.2, -0.1, 0.25])
    c2w = rigid([1.0, 0.2, 0.1], 35.0, [0.4, 0.1, -0.3])
    delta = G.inv_rigid(c2w) @ G.inv_rigid(t_true) @ c2w
    q = Rotation.from_matrix(delta[:3, :3]).as_quat()  # x, y, z, w
    d7 = np.concatenate([[q[3]], q[:3], delta[:3, 3]])
    np.testing.assert_allclose(G.view_estimate(c2w, d7), t_true, atol=1e-12)


def _tiny_pair(seed, deg, metres):
    return synth.registration_pair(seed, 1500, 1500, shared_frac=1.0, views_p=1, views_q=1, width=64, height=48,
                                   f=45, half=(1.0, 0.6, 0.8), log_scale_mu=math.log(0.05), rot_deg_max=deg,
                                   trans_max=metres)


def _targets(g, cam, kfs):
    out = []
    for c2w in kfs:
        o = R.render(g, cam, torch.as_tensor(G.inv_rigid(c2w)[:3]), with_margins=False)
        out.append((c2w, o["rgb"].detach().numpy(), o["depth"].detach().numpy()))
    return out


def test_exact_correction_gives_zero_loss():
    """With every Gaussian shared, rendering Q from keyframe i of P with the
    exact correction reproduces P's render up to rounding."""
    d = _tiny_pair(4, 8.0, 0.2)
    cam = R.Camera(**d["cam"])
    P, Q = R.to_f64(d["P"]), R.to_f64(d["Q"])
    (c2w, rgb, dep), = _targets(P, cam, d["kf_p"])
    delta = G.inv_rigid(c2w) @ G.inv_rigid(d["T_gt"]) @ c2w
    q = Rotation.from_matrix(delta[:3, :3]).as_quat()
    d7 = torch.as_tensor(np.concatenate([[q[3]], q[:3], delta[:3, 3]]))
    out = R.render(Q, cam, torch.as_tensor(G.inv_rigid(c2w)[:3]), d7, with_margins=False)
    np.testing.assert_allclose(out["rgb"].detach().numpy(), rgb, atol=2e-5)
    np.testing.assert_allclose(out["depth"].detach().numpy(), dep, atol=2e-5)


@pytest.mark.parametrize("loss", [None, dict(lambda_c=0.6, alpha_power=3, inlier_k=50.0)],
                         ids=["plain_l1", "tracking_eq2"])
def test_recovers_known_transform_tiny_scene(loss):
    """Both directions localised, 100 Adam steps each, fused: the transform
    is recovered to < 0.5 deg and < 1 cm, with the plain L1 and with the
    masked tracking loss."""
    d = _tiny_pair(4, 2.0, 0.03)
    cam = R.Camera(**d["cam"])
    P, Q = R.to_f64(d["P"]), R.to_f64(d["Q"])
    t_bar, ests, res = G.register_pair(P, Q, _targets(P, cam, d["kf_p"]), _targets(Q, cam, d["kf_q"]), cam, 100,
                                       0.003, 0.001, loss=loss)
    assert G.rotation_error_deg(t_bar, d["T_gt"]) < 0.5
    assert G.translation_error_cm(t_bar[:3, 3], d["T_gt"][:3, 3]) < 1.0
    assert all(r >= 0 for r in res)


def test_residual_is_the_unmasked_l1_whatever_the_loss():
    """With the pose frozen (zero learning rates) the residual of a view is the
    plain L1 of its render at identity, also when the masked tracking loss
    drives the optimisation; a view that sees nothing of the other submap
    (alpha = 0 everywhere) gets the mean absolute measurement as residual,
    not the zero of its masked loss."""
    d = _tiny_pair(4, 2.0, 0.03)
    cam = R.Camera(**d["cam"])
    P, Q = R.to_f64(d["P"]), R.to_f64(d["Q"])
    (c2w, rgb, dep), = _targets(P, cam, d["kf_p"])
    track = dict(lambda_c=0.6, alpha_power=3, inlier_k=50.0)
    _, resid, hist = G.localise_view(Q, cam, c2w, rgb, dep, 1, 0.0, 0.0, loss=track)
    out = R.render(Q, cam, torch.as_tensor(G.inv_rigid(c2w)[:3]), R.identity_pose(), with_margins=False)
    l1 = float(R.loss_l1(out["rgb"], out["depth"], torch.as_tensor(rgb), torch.as_tensor(dep)))
    assert resid == pytest.approx(l1, rel=1e-12)
    assert hist[0] != pytest.approx(l1, rel=1e-3)          # the masked loss is a different number
    # the camera moved 1 km along its viewing axis: every Gaussian is behind it
    away = np.array(c2w, np.float64)
    away[:3, 3] += 1000.0 * away[:3, 2]
    _, resid, hist = G.localise_view(Q, cam, away, rgb, dep, 1, 0.0, 0.0, loss=track)
    valid = dep > 0
    expect = (np.abs(rgb).sum(0)[valid].sum() + np.abs(dep)[valid].sum()) / valid.sum()
    assert hist[0] == 0.0 and resid == pytest.approx(expect, rel=1e-12)


def _exposed_target(seed, a_true, b_true):
    d = _tiny_pair(seed, 2.0, 0.03)
    cam = R.Camera(**d["cam"])
    P = R.to_f64(d["P"])
    (c2w, rgb, dep), = _targets(P, cam, d["kf_p"])
    return d, cam, P, c2w, math.exp(a_true) * rgb + b_true, dep


def test_exposure_recovers_a_known_gain_and_offset():
    """R23: the keyframe's own submap rendered at its exact pose, but with the
    colours under a known exposure (gain 1.2, offset 0.03).  With exposure
    coefficients the view recovers them (a to 0.02, b to 0.01) and stays at
    the identity pose (< 0.3 cm); without them the pose drifts to absorb the
    brightness change and the residual is 20x larger."""
    a0, b0 = math.log(1.2), 0.03
    d, cam, P, c2w, rgb, dep = _exposed_target(4, a0, b0)
    pose_e, res_e, _, ab = G.localise_view(P, cam, c2w, rgb, dep, 100, 0.003, 0.001, lr_exposure=0.1,
                                           return_exposure=True)
    pose_n, res_n, _ = G.localise_view(P, cam, c2w, rgb, dep, 100, 0.003, 0.001)
    assert abs(ab[0] - a0) < 0.02 and abs(ab[1] - b0) < 0.01, ab
    assert np.linalg.norm(pose_e[4:]) < 0.003
    assert res_n > 20 * res_e


def test_exposure_with_zero_learning_rate_is_the_plain_path():
    """a = b = 0 held fixed: exp(0) C + 0 = C, so every step equals the
    localisation without exposure coefficients, bit for bit."""
    d, cam, P, c2w, rgb, dep = _exposed_target(5, 0.1, 0.02)
    a = G.localise_view(P, cam, c2w, rgb, dep, 15, 0.003, 0.001, lr_exposure=0.0, return_exposure=True)
    b = G.localise_view(P, cam, c2w, rgb, dep, 15, 0.003, 0.001)
    np.testing.assert_array_equal(a[0], b[0])
    assert a[1] == b[1] and a[2] == b[2] and np.all(a[3] == 0.0)


def test_exposure_gradient_matches_finite_differences():
    """d loss / d(a, b) of the exposed render (autograd) against central
    differences, away from the L1 kinks of the unmasked loss."""
    d, cam, P, c2w, rgb, dep = _exposed_target(6, 0.15, 0.05)
    out = R.render(P, cam, torch.as_tensor(G.inv_rigid(c2w)[:3]), with_margins=False)
    C = out["rgb"].detach()
    tr, td = torch.as_tensor(rgb), torch.as_tensor(dep)

    def f(ab):
        return R.loss_l1(torch.exp(ab[0]) * C + ab[1], out["depth"].detach(), tr, td)

    ab = torch.tensor([0.05, 0.01], dtype=torch.float64, requires_grad=True)
    (g,) = torch.autograd.grad(f(ab), [ab])
    for k in range(2):
        e = torch.zeros(2, dtype=torch.float64)
        e[k] = 1e-7
        fd = (float(f(ab.detach() + e)) - float(f(ab.detach() - e))) / 2e-7
        np.testing.assert_allclose(float(g[k]), fd, rtol=1e-5)


def test_joint_delta_is_the_view_correction_of_the_shared_transform():
    """R33: at T = T_gt, Delta_i of a P keyframe is the exact correction
    C^-1 T^-1 C (so its view estimate is T_gt) and that of a Q keyframe gives
    the estimate T_gt^-1; identity T gives identity corrections."""
    d = _tiny_pair(4, 8.0, 0.2)
    T = d["T_gt"]
    q = Rotation.from_matrix(T[:3, :3]).as_quat()
    T7 = torch.as_tensor(np.concatenate([[q[3]], q[:3], T[:3, 3]]))
    for c2w, rev, want in ((d["kf_p"][0], False, T), (d["kf_q"][0], True, G.inv_rigid(T))):
        dl = G.joint_delta(T7, c2w, rev).numpy()
        np.testing.assert_allclose(G.view_estimate(c2w, dl), want, atol=1e-12)
        ident = G.joint_delta(torch.as_tensor([1.0, 0, 0, 0, 0, 0, 0]), c2w, rev).numpy()
        np.testing.assert_allclose(G.pose_matrix(ident), np.eye(4), atol=1e-12)


def test_joint_registration_recovers_a_known_transform():
    """R33 on the tiny room: one shared transform over both keyframes,
    100 Adam steps, recovers the known 2 deg / 3 cm transform."""
    d = _tiny_pair(4, 2.0, 0.03)
    cam = R.Camera(**d["cam"])
    P, Q = R.to_f64(d["P"]), R.to_f64(d["Q"])
    T, res = G.register_pair_joint(P, Q, _targets(P, cam, d["kf_p"]), _targets(Q, cam, d["kf_q"]), cam, 100,
                                   0.003, 0.001)
    assert G.rotation_error_deg(T, d["T_gt"]) < 0.5
    assert G.translation_error_cm(T[:3, 3], d["T_gt"][:3, 3]) < 1.0
    assert len(res) == 2 and all(r >= 0 for r in res)


@pytest.mark.parametrize("deg", [0.0, 0.5, 1.0, 90.0, 179.0])
def test_rotation_error_degrees_of_known_rotations(deg):
    """O13: the rotation error of R against R_gt is the angle of R R_gt^T in
    degrees.  Pinned by R = R_gt R(axis, deg) for a non-trivial R_gt (a
    missing transpose, radians or a half angle each fail), both argument
    orders, and the package's reporting helper agreeing."""
    from paper_2408_10154_amd import register as REG

    gt = rigid([0.2, -1.0, 0.4], 37.0, [0.0, 0.0, 0.0])
    for axis in ([1, 0, 0], [0.3, 0.5, -0.8]):
        est = gt @ rigid(axis, deg, [0.0, 0.0, 0.0])
        assert abs(G.rotation_error_deg(est, gt) - deg) < 1e-6
        assert abs(G.rotation_error_deg(gt, est) - deg) < 1e-6
        assert abs(REG.rotation_error_deg(est, gt) - deg) < 1e-6
        est2 = rigid(axis, deg, [0.0, 0.0, 0.0]) @ gt
        assert abs(G.rotation_error_deg(est2, gt) - deg) < 1e-6


@pytest.mark.parametrize("offset_m,expect_cm", [((0.0, 0.0, 0.0), 0.0), ((0.03, 0.04, 0.0), 5.0),
                                                ((-0.002, 0.0, 0.0), 0.2), ((0.1, -0.2, 0.2), 30.0)])
def test_translation_error_centimetres_of_known_offsets(offset_m, expect_cm):
    """O13: the translation error is |t - t_gt| in centimetres (metres in,
    a factor 100 out), pinned by offsets with exact norms."""
    from paper_2408_10154_amd import register as REG

    gt = rigid([1, 2, 3], 5.0, [0.4, -0.1, 1.2])
    est = gt.copy()
    est[:3, 3] += np.asarray(offset_m)
    assert abs(G.translation_error_cm(est[:3, 3], gt[:3, 3]) - expect_cm) < 1e-9
    assert abs(REG.translation_error_cm(est, gt) - expect_cm) < 1e-9
