"""GPU overlap ratio (ls_overlap_ratio; supplement, Eq. 9) against the
oracle.  Matches are integer decisions on FP32 values taken with one
rounding sequence on both sides, so the bar is bit-exact: every nearest
neighbour index and both counts."""

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

from oracle import overlap as O
from paper_2408_10154_amd import synth

pytestmark = pytest.mark.gpu


def _dev(pts):
    return torch.as_tensor(np.ascontiguousarray(np.asarray(pts, np.float32).T), device="cuda").contiguous()


def _gpu(P, Q, T, tau):
    from paper_2408_10154_amd.render import overlap_ratio

    r, pairs, inl, nn_pq, nn_qp = overlap_ratio(_dev(P), _dev(Q), T, tau)
    return r, pairs, inl, nn_pq.cpu().numpy(), nn_qp.cpu().numpy()


def _rigid(rng, deg, metres):
    T = np.eye(4)
    T[:3, :3] = Rotation.from_rotvec(rng.normal(size=3) / np.sqrt(3) * np.deg2rad(deg)).as_matrix()
    T[:3, 3] = rng.uniform(-metres, metres, 3)
    return T.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("case", ["uniform", "clustered", "duplicates", "far", "tiny", "empty"])
def test_overlap_matches_oracle_bit_exact(gpu, case):
    """Point sets that exercise the search: uniform clouds of ragged sizes,
    tight clusters on surfaces, exact duplicates (ties to the lower index),
    two clouds 5 m apart (every match far away, little pruning), one point
    against a few, and an empty set."""
    seeds = {"uniform": 1, "clustered": 2, "duplicates": 3, "far": 4, "tiny": 5, "empty": 6}
    rng = np.random.default_rng(seeds[case])
    T = _rigid(rng, 8.0, 0.2)
    if case == "uniform":
        P, Q = rng.uniform(-2, 2, (5003, 3)), rng.uniform(-2, 2, (4099, 3))
    elif case == "clustered":
        c = rng.uniform(-3, 3, (40, 3))
        P = c[rng.integers(0, 40, 6000)] + rng.normal(scale=0.02, size=(6000, 3))
        Q = c[rng.integers(0, 40, 5000)] + rng.normal(scale=0.02, size=(5000, 3))
    elif case == "duplicates":
        base = rng.uniform(-1, 1, (300, 3))
        P = base[rng.integers(0, 300, 2000)]
        Q = base[rng.integers(0, 300, 1500)]
        T = np.eye(4)
    elif case == "far":
        P = rng.uniform(-1, 1, (3000, 3))
        Q = rng.uniform(-1, 1, (2500, 3)) + [5.0, 0.0, 0.0]
    elif case == "tiny":
        P, Q = rng.uniform(-1, 1, (1, 3)), rng.uniform(-1, 1, (5, 3))
    else:
        P, Q = rng.uniform(-1, 1, (100, 3)), np.zeros((0, 3))
    P, Q = P.astype(np.float32), Q.astype(np.float32)
    for tau in (0.05, 0.2):
        got = _gpu(P, Q, T, tau)
        ref = O.overlap_ratio(P, Q, T, tau)
        assert got[1:3] == ref[1:3], (case, tau, got[1:3], ref[1:3])
        np.testing.assert_array_equal(got[3], ref[3])
        np.testing.assert_array_equal(got[4], ref[4])
        assert got[0] == ref[0]


def test_overlap_of_the_registration_pair(gpu):
    """The single-pair registration workload (150k + 120k Gaussians, 60 %
    shared, ground truth up to 10 deg / 0.3 m) at full size: nearest
    neighbours of 2,000 sampled points of each set against the oracle's
    brute force over the whole other set, both counts recomputed from the
    GPU's full match arrays, and the ratio under the ground truth far above
    the ratio under the identity."""
    d = synth.registration_pair(2, 150000, 120000, views_p=1, views_q=1)
    P = np.asarray(d["P"]["mean"], np.float32).T
    Q = np.asarray(d["Q"]["mean"], np.float32).T
    T = d["T_gt"].astype(np.float32).astype(np.float64)
    tau = 0.2
    r, pairs, inl, nn_pq, nn_qp = _gpu(P, Q, T, tau)
    rng = np.random.default_rng(4)
    pt = O.transform_points_f32(P, T)
    sp = rng.choice(len(P), 2000, replace=False)
    sq = rng.choice(len(Q), 2000, replace=False)
    np.testing.assert_array_equal(nn_pq[sp], O.nearest(pt[sp], Q)[0])
    np.testing.assert_array_equal(nn_qp[sq], O.nearest(Q[sq], pt)[0])
    recip = nn_qp[nn_pq] == np.arange(len(P))
    dx = pt[recip] - Q[nn_pq[recip]]
    d2 = (dx[:, 0] * dx[:, 0] + dx[:, 1] * dx[:, 1]) + dx[:, 2] * dx[:, 2]
    tau2 = np.float32(np.float32(tau) * np.float32(tau))
    assert pairs == int(recip.sum()) and inl == int((d2 < tau2).sum())
    assert r > 0.5
    r_id = _gpu(P, Q, np.eye(4), tau)[0]
    assert r_id < r
