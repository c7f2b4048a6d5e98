"""Oracle of opacity pruning after mapping (supplement, Implementation
Details, "Submap Update").

TEST INFRASTRUCTURE ONLY (see the package docstring): never imported by the
product path.

Once the mapping optimisation of a new keyframe has finished, every Gaussian
of the submap whose opacity is below a threshold o_thre (0.1 on the synthetic
dataset, 0.5 on the real ones) is removed; the others are kept, in their
order, with all their parameters.

  R34 decision precision: the opacity is sigmoid(opacity_logit) (R1) and
      sigmoid is increasing, so o < o_thre <=> logit < ln(o_thre / (1 -
      o_thre)).  The keep test is taken on the stored FP32 logit against the
      FP32 rounding of that threshold, logit >= fl32(ln(o / (1 - o))), so
      that both sides decide in the same precision (o_thre is taken as an
      FP32 value, the logarithm in FP64); a Gaussian whose opacity
      equals the threshold is kept ("lower than" prunes).  A NaN logit is
      pruned.  The oracle's decisions equal the FP64 definition sigmoid(w) <
      o_thre everywhere except within FP32 rounding of the threshold (pinned
      in tests/test_oracle_prune.py).
"""

from __future__ import annotations

import math

import numpy as np


def logit_threshold(o_thre: float) -> np.float32:
    """The keep threshold on the FP32 logit: fl32(ln(o / (1 - o))) with o the
    FP32 value of o_thre, the logarithm taken in FP64 (R34)."""
    o = float(np.float32(o_thre))
    if not 0.0 < o < 1.0:
        raise ValueError("o_thre must lie in (0, 1)")
    return np.float32(math.log(o / (1.0 - o)))


def keep_mask(opacity_logit, o_thre: float) -> np.ndarray:
    """Boolean mask of the Gaussians kept (opacity >= o_thre), R34."""
    w = np.asarray(opacity_logit, np.float32)
    with np.errstate(invalid="ignore"):
        return w >= logit_threshold(o_thre)


def prune(gauss: dict, o_thre: float):
    """Gaussians of a submap after pruning: returns (kept indices [k] int64
    in ascending order, dict of the kept parameters with the same layouts as
    the input, SoA [c][n] -> [c][k])."""
    keep = keep_mask(gauss["opacity_logit"], o_thre)
    idx = np.nonzero(keep)[0]
    out = {name: np.asarray(a)[..., idx] for name, a in gauss.items()}
    return idx, out
