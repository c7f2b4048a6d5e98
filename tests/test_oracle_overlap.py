"""Pins of the overlap-ratio oracle (supplement, Eq. 9; readings R31-R32):
a hand-worked example, pure-Python brute force, an FP64 k-d tree, and the
invariants of identical and rigidly moved point sets.  CPU only."""

import numpy as np
from scipy.spatial import cKDTree
from scipy.spatial.transform import Rotation

from oracle import overlap as O


def test_hand_worked_example():
    """P = {0, 1, 2} on the x axis, Q = {0.05, 0.9, 3}: nn_Q = (0, 1, 2)
    (2 is 1.0 from 3 and 1.1 from 0.9), nn_P = (0, 1, 2); three reciprocal
    pairs at 0.05, 0.1 and 1.0, so tau = 0.08 keeps one and tau = 0.2 two."""
    P = np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0]], np.float32)
    Q = np.array([[0.05, 0, 0], [0.9, 0, 0], [3, 0, 0]], np.float32)
    r, pairs, inl, nn_pq, nn_qp = O.overlap_ratio(P, Q, np.eye(4), 0.08)
    assert list(nn_pq) == [0, 1, 2] and list(nn_qp) == [0, 1, 2]
    assert (pairs, inl) == (3, 1) and abs(r - 1 / 3) < 1e-15
    r, pairs, inl, _, _ = O.overlap_ratio(P, Q, np.eye(4), 0.2)
    assert (pairs, inl) == (3, 2)
    # moved by +1 in x, P is {1, 2, 3}: nn_Q = (1, 2, 2), nn_P = (0, 0, 2);
    # reciprocal pairs (0, 1) at 0.1 and (2, 2) at 0; (1, 2) is one-sided
    T = np.eye(4)
    T[0, 3] = 1.0
    r, pairs, inl, nn_pq, nn_qp = O.overlap_ratio(P, Q, T, 0.15)
    assert list(nn_pq) == [1, 2, 2] and list(nn_qp) == [0, 0, 2]
    assert (pairs, inl, r) == (2, 2, 1.0)
    r, pairs, inl, _, _ = O.overlap_ratio(P, Q, T, 0.05)
    assert (pairs, inl, r) == (2, 1, 0.5)
    # a point within tau of its match that is not matched back does not count:
    # P = {0, 0.02}, Q = {0.05}: both P points pick Q's, Q picks 0.02
    P2 = np.array([[0, 0, 0], [0.02, 0, 0]], np.float32)
    Q2 = np.array([[0.05, 0, 0]], np.float32)
    r, pairs, inl, nn_pq, nn_qp = O.overlap_ratio(P2, Q2, np.eye(4), 0.1)
    assert list(nn_pq) == [0, 0] and list(nn_qp) == [1] and (pairs, inl, r) == (1, 1, 1.0)


def test_ties_go_to_the_lower_index_and_empty_sets():
    P = np.array([[0, 0, 0]], np.float32)
    Q = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0]], np.float32)  # three equidistant points
    _, _, _, nn_pq, _ = O.overlap_ratio(P, Q, np.eye(4), 0.5)
    assert nn_pq[0] == 0
    r, pairs, inl, nn_pq, nn_qp = O.overlap_ratio(P, np.zeros((0, 3), np.float32), np.eye(4), 0.5)
    assert (r, pairs, inl) == (0.0, 0, 0) and list(nn_pq) == [-1] and len(nn_qp) == 0


def test_matches_pure_python_brute_force():
    rng = np.random.default_rng(0)
    P = rng.uniform(-1, 1, (60, 3)).astype(np.float32)
    Q = rng.uniform(-1, 1, (45, 3)).astype(np.float32)
    idx, d2 = O.nearest(P, Q)
    for i in range(60):
        best, bj = None, -1
        for j in range(45):
            dx = np.float32(P[i, 0] - Q[j, 0])
            dy = np.float32(P[i, 1] - Q[j, 1])
            dz = np.float32(P[i, 2] - Q[j, 2])
            d = np.float32(np.float32(np.float32(dx * dx) + np.float32(dy * dy)) + np.float32(dz * dz))
            if best is None or d < best:
                best, bj = d, j
        assert idx[i] == bj and d2[i] == best


def test_agrees_with_an_fp64_kd_tree_up_to_rounding():
    rng = np.random.default_rng(1)
    P = rng.normal(size=(3000, 3)).astype(np.float32)
    Q = rng.normal(size=(2500, 3)).astype(np.float32)
    T = np.eye(4)
    T[:3, :3] = Rotation.from_rotvec([0.1, -0.2, 0.3]).as_matrix()
    T[:3, 3] = [0.05, 0.0, -0.1]
    T32 = T.astype(np.float32).astype(np.float64)
    pt = O.transform_points_f32(P, T32)
    np.testing.assert_allclose(pt, P.astype(np.float64) @ T32[:3, :3].T + T32[:3, 3], atol=1e-6)
    idx, d2 = O.nearest(pt, Q)
    dk, ik = cKDTree(Q.astype(np.float64)).query(pt.astype(np.float64))
    same = idx == ik
    # where they differ, both candidates are equally near up to FP32 rounding
    d_ours = np.linalg.norm(pt.astype(np.float64) - Q[idx].astype(np.float64), axis=1)
    assert np.all(np.abs(d_ours[~same] - dk[~same]) <= 1e-6 * np.maximum(dk[~same], 1e-3))
    assert same.mean() > 0.999
    np.testing.assert_allclose(np.sqrt(d2.astype(np.float64)), dk, rtol=1e-5, atol=1e-6)


def test_identical_sets_and_rigid_invariance():
    rng = np.random.default_rng(2)
    P = rng.uniform(-2, 2, (500, 3)).astype(np.float32)
    r, pairs, inl, nn_pq, nn_qp = O.overlap_ratio(P, P, np.eye(4), 0.01)
    assert (r, pairs, inl) == (1.0, 500, 500)
    assert np.array_equal(nn_pq, np.arange(500)) and np.array_equal(nn_qp, np.arange(500))
    # Q is P moved by T (in FP32): the estimate T brings every point home
    T = np.eye(4)
    T[:3, :3] = Rotation.from_rotvec([0.3, 0.1, -0.2]).as_matrix()
    T[:3, 3] = [1.0, -2.0, 0.5]
    T = T.astype(np.float32).astype(np.float64)
    Q = O.transform_points_f32(P, T)
    r, pairs, inl, nn_pq, _ = O.overlap_ratio(P, Q, T, 1e-4)
    assert (r, pairs, inl) == (1.0, 500, 500) and np.array_equal(nn_pq, np.arange(500))
    # the identity instead of T: most points are far from their partner
    r, _, _, _, _ = O.overlap_ratio(P, Q, np.eye(4), 0.1)
    assert r < 0.1
