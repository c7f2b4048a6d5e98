"""Pins of the FP64 map-adjustment oracle (Sec. 3.3, Eq. 8, reading R30):
special cases, composition, a library rotation composition and the
rendering invariance of a rigidly moved scene and camera.  CPU only."""

import numpy as np
import torch
from scipy.spatial.transform import Rotation

from oracle import adjust as A
from oracle import raster as R
from paper_2408_10154_amd import synth

F64 = torch.float64


def _rigid(seed, deg=25.0, metres=0.4):
    rng = np.random.default_rng(seed)
    T = np.eye(4)
    T[:3, :3] = Rotation.from_rotvec(rng.normal(size=3) / np.sqrt(3) * np.deg2rad(deg)).as_matrix()
    T[:3, 3] = rng.uniform(-metres, metres, 3)
    return T


def _gauss(seed, n=40):
    g = R.to_f64(synth.scene_tiny(seed, n, 32, 24, 30.0)["gauss"])
    return g["mean"], g["log_scale"], g["quat"]


def test_identity_and_pure_translation():
    mean, ls, q = _gauss(1)
    m1, s1 = A.adjust_gaussians(mean, ls, q, np.eye(4))
    np.testing.assert_allclose(m1.numpy(), mean.numpy(), rtol=0, atol=0)
    np.testing.assert_allclose(s1.numpy(), R.covariance3d(ls, q).numpy(), rtol=1e-15, atol=1e-18)
    T = np.eye(4)
    T[:3, 3] = [0.3, -0.2, 1.5]
    m2, s2 = A.adjust_gaussians(mean, ls, q, T)
    np.testing.assert_allclose(m2.numpy(), mean.numpy() + [0.3, -0.2, 1.5], rtol=1e-15)
    np.testing.assert_allclose(s2.numpy(), R.covariance3d(ls, q).numpy(), rtol=1e-15, atol=1e-18)


def test_composition_of_two_corrections():
    mean, ls, q = _gauss(2)
    Ta, Tb = _rigid(3), _rigid(4)
    ma, sa = A.adjust_gaussians(mean, ls, q, Ta)
    mb, sb = A.adjust_gaussians(mean, ls, q, Tb @ Ta)
    # second correction applied to the once-corrected means and covariances
    m2 = ma @ torch.as_tensor(Tb[:3, :3]).T + torch.as_tensor(Tb[:3, 3])
    s2 = torch.as_tensor(Tb[:3, :3]) @ sa @ torch.as_tensor(Tb[:3, :3]).T
    np.testing.assert_allclose(mb.numpy(), m2.numpy(), atol=1e-14)
    np.testing.assert_allclose(sb.numpy(), s2.numpy(), atol=1e-16)
    poses = np.stack([_rigid(10 + k) for k in range(3)])
    np.testing.assert_allclose(A.adjust_poses(poses, Tb @ Ta), A.adjust_poses(A.adjust_poses(poses, Ta), Tb),
                               atol=1e-14)


def test_covariance_matches_library_rotation_composition():
    """Sigma' equals the covariance of the rotated Gaussian written with the
    composed rotation R_c R(q) (scipy), and keeps its eigenvalues."""
    mean, ls, q = _gauss(5)
    T = _rigid(6)
    _, s1 = A.adjust_gaussians(mean, ls, q, T)
    qn = q.numpy() / np.linalg.norm(q.numpy(), axis=1, keepdims=True)
    rot = Rotation.from_matrix(T[:3, :3]) * Rotation.from_quat(qn[:, [1, 2, 3, 0]])
    xyzw = rot.as_quat()
    q2 = torch.as_tensor(xyzw[:, [3, 0, 1, 2]])
    np.testing.assert_allclose(s1.numpy(), R.covariance3d(ls, q2).numpy(), atol=1e-15)
    np.testing.assert_allclose(np.linalg.eigvalsh(s1.numpy()), np.linalg.eigvalsh(R.covariance3d(ls, q).numpy()),
                               rtol=1e-10)


def test_rendering_is_invariant_under_the_correction():
    """Moving the submap by T_c and its keyframe camera by T_c (Eq. 8)
    leaves the rendered colour, depth and alpha unchanged."""
    sc = synth.scene_tiny(7, 300, 48, 36, 45.0)
    cam = R.Camera(**sc["cam"])
    g = R.to_f64(sc["gauss"])
    c2w = np.eye(4)
    c2w[:3, 3] = [0.05, -0.02, 0.1]
    T = _rigid(8, deg=30.0, metres=0.5)
    m1, _ = A.adjust_gaussians(g["mean"], g["log_scale"], g["quat"], T)
    qn = g["quat"].numpy() / np.linalg.norm(g["quat"].numpy(), axis=1, keepdims=True)
    q1 = (Rotation.from_matrix(T[:3, :3]) * Rotation.from_quat(qn[:, [1, 2, 3, 0]])).as_quat()[:, [3, 0, 1, 2]]
    g1 = dict(g, mean=m1, quat=torch.as_tensor(q1))
    c2w1 = A.adjust_poses(c2w[None], T)[0]
    o0 = R.render(g, cam, torch.as_tensor(np.linalg.inv(c2w)[:3]), with_margins=False)
    o1 = R.render(g1, cam, torch.as_tensor(np.linalg.inv(c2w1)[:3]), with_margins=False)
    for k in ("rgb", "depth", "alpha"):
        np.testing.assert_allclose(o1[k].numpy(), o0[k].numpy(), atol=1e-9)
    assert float(o0["alpha"].max()) > 0.5
