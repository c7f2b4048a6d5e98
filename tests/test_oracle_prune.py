"""Pins of the opacity-pruning oracle (supplement, submap update): hand
cases, the FP64 sigmoid definition, order and content of the kept set.
CPU only."""

import math

import numpy as np
import pytest

from oracle import prune as PR


def _sig(w):
    return 1.0 / (1.0 + np.exp(-np.asarray(w, np.float64)))


def test_hand_cases():
    """Opacities 0.05, 0.1, 0.3, 0.5, 0.9 (as logits): o_thre 0.1 keeps all
    but the first, 0.5 keeps the last two; equality keeps."""
    o = np.array([0.05, 0.1, 0.3, 0.5, 0.9])
    w = np.log(o / (1 - o)).astype(np.float32)
    w[3] = 0.0  # exactly 0.5
    assert PR.keep_mask(w, 0.5).tolist() == [False, False, False, True, True]
    k = PR.keep_mask(w, 0.1)
    assert k[0] == False and k[2:].all()  # noqa: E712
    # the 0.1 entry sits on the threshold up to rounding: it is kept iff its FP32 logit is not below fl32(ln(1/9))
    assert k[1] == (np.float32(w[1]) >= np.float32(math.log(1 / 9)))
    assert PR.logit_threshold(0.5) == 0.0
    assert PR.logit_threshold(0.1) == np.float32(-2.1972245773362196)


def test_nan_and_infinities():
    w = np.array([np.nan, np.inf, -np.inf, 3.0], np.float32)
    assert PR.keep_mask(w, 0.5).tolist() == [False, True, False, True]


@pytest.mark.parametrize("o_thre", [0.1, 0.5, 0.9])
def test_matches_fp64_sigmoid_away_from_the_threshold(o_thre):
    """Brute force against the definition opacity = sigmoid(logit) < o_thre
    in FP64: identical decisions for every logit farther than 1e-6 from the
    threshold, and the kept count equals the definition's up to those."""
    rng = np.random.default_rng(4)
    w = rng.normal(0.0, 2.0, 200_000).astype(np.float32)
    ref = _sig(w) >= o_thre
    got = PR.keep_mask(w, o_thre)
    far = np.abs(w.astype(np.float64) - math.log(o_thre / (1 - o_thre))) > 1e-6
    assert far.mean() > 0.999
    np.testing.assert_array_equal(got[far], ref[far])


def test_prune_keeps_order_and_rows():
    """Kept indices ascend, every SoA array is gathered along its last axis,
    and a planted mistake (keeping the low-opacity ones) fails the pin."""
    rng = np.random.default_rng(5)
    n = 1001
    g = dict(mean=rng.normal(size=(3, n)).astype(np.float32), log_scale=rng.normal(size=(3, n)).astype(np.float32),
             quat=rng.normal(size=(4, n)).astype(np.float32), opacity_logit=rng.normal(size=n).astype(np.float32),
             rgb=rng.random((3, n)).astype(np.float32))
    idx, out = PR.prune(g, 0.5)
    assert np.all(np.diff(idx) > 0)
    assert len(idx) == int((g["opacity_logit"] >= 0).sum())
    for name, a in g.items():
        np.testing.assert_array_equal(out[name], a[..., idx])
    assert np.all(_sig(out["opacity_logit"]) >= 0.5)
    wrong = np.nonzero(g["opacity_logit"] < 0)[0]
    assert not np.array_equal(wrong, idx)


def test_empty_and_all():
    assert PR.prune(dict(opacity_logit=np.zeros(0, np.float32)), 0.1)[0].size == 0
    w = np.full(7, 5.0, np.float32)
    assert PR.prune(dict(opacity_logit=w), 0.5)[0].tolist() == list(range(7))
    assert PR.prune(dict(opacity_logit=-w), 0.5)[0].size == 0
