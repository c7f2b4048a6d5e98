"""The library's host-side Eq. 7 fusion against the oracle's SVD form.
No GPU: ls_fuse_estimates is pure host code."""

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import register as G
from paper_2408_10154_amd import register as REG


def _random_rigid(rng, deg, metres):
    out = np.eye(4)
    out[:3, :3] = Rotation.from_rotvec(rng.normal(size=3) / np.sqrt(3) * np.radians(deg)).as_matrix()
    out[:3, 3] = rng.normal(size=3) * metres
    return out


@pytest.mark.parametrize("seed", range(6))
def test_fusion_matches_oracle(seed):
    rng = np.random.default_rng(seed)
    base = _random_rigid(rng, 40.0, 0.5)
    n = int(rng.integers(2, 12))
    ests, res, rev = [], [], []
    for i in range(n):
        noise = _random_rigid(rng, 3.0, 0.02)
        e = noise @ base
        r = bool(rng.integers(0, 2))
        ests.append(G.inv_rigid(e) if r else e)
        res.append(float(rng.uniform(0.01, 1.0)))
        rev.append(r)
    ours = REG.fuse_estimates(ests, res, rev)
    ref = G.fuse(ests, res, rev)
    np.testing.assert_allclose(ours, ref, atol=1e-9)


def test_fusion_large_spread_and_single_estimate():
    rng = np.random.default_rng(9)
    e = _random_rigid(rng, 170.0, 2.0)
    np.testing.assert_allclose(REG.fuse_estimates([e], [0.3], [False]), e, atol=1e-12)
    ests = [_random_rigid(rng, 90.0, 1.0) for _ in range(5)]
    np.testing.assert_allclose(REG.fuse_estimates(ests, [1, 2, 3, 4, 5], [0] * 5), G.fuse(ests, [1, 2, 3, 4, 5], [0] * 5),
                               atol=1e-9)
