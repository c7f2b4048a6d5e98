"""Oracle of the geometric overlap ratio of two submaps (supplement, loop
detection, Eq. 9).

TEST INFRASTRUCTURE ONLY (see the package docstring): never imported by the
product path.

The overlap ratio counts, among the putative correspondences K found by
reciprocal nearest-neighbour matching between the Gaussians of P (moved by
the current estimate of T_{P->Q}) and those of Q, the fraction whose
distance is below tau_1.  The paper keeps loops with a ratio above a
threshold (0.2; the supplement's table lists 0.1 / 0.2 per dataset) and
uses tau_1 = 0.1 m (synthetic data) or 0.2 m (real data).

  R31 the points are the Gaussian means; q = nn_Q(p) is the point of Q with
      the smallest squared distance to T(p), ties going to the lower index;
      (p, q) is in K when also nn_P(q) = p.  OR = 0 when K is empty.
  R32 these are integer decisions taken on floating-point values, so both the
      oracle and the GPU take them in FP32 with one fixed rounding sequence:
      T(p)_r = ((R_r0 x + R_r1 y) + R_r2 z) + t_r and
      d^2 = (dx^2 + dy^2) + dz^2 with dx = T(p)_x - q_x, every operation
      rounded to FP32 (no fused multiply-add); the threshold test is
      d^2 < fl32(tau^2).  The FP64 distances of a k-d tree pin the matches
      up to that rounding.
"""

from __future__ import annotations

import numpy as np

F32 = np.float32


def transform_points_f32(pts: np.ndarray, T: np.ndarray) -> np.ndarray:
    """T(p) for p in pts [N, 3] (float32), with the rounding sequence of R32."""
    p = np.asarray(pts, F32)
    T = np.asarray(T, np.float64)[:3, :4].astype(F32)
    out = np.empty_like(p)
    for r in range(3):
        out[:, r] = ((T[r, 0] * p[:, 0] + T[r, 1] * p[:, 1]) + T[r, 2] * p[:, 2]) + T[r, 3]
    return out


def sq_dist_f32(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """FP32 squared distances of R32 between rows of a [n, 3] and b [m, 3]: [n, m]."""
    dx = a[:, None, 0] - b[None, :, 0]
    dy = a[:, None, 1] - b[None, :, 1]
    dz = a[:, None, 2] - b[None, :, 2]
    return (dx * dx + dy * dy) + dz * dz


def nearest(a: np.ndarray, b: np.ndarray, chunk: int = 1024):
    """For every row of a: (index of its nearest row of b, that squared
    distance), by brute force over all of b; -1 and inf when b is empty."""
    a = np.asarray(a, F32)
    b = np.asarray(b, F32)
    n = a.shape[0]
    idx = np.full(n, -1, np.int64)
    d2 = np.full(n, np.inf, F32)
    if b.shape[0] == 0:
        return idx, d2
    for s in range(0, n, chunk):
        d = sq_dist_f32(a[s:s + chunk], b)
        k = np.argmin(d, axis=1)  # first (lowest) index among equal minima
        idx[s:s + chunk] = k
        d2[s:s + chunk] = d[np.arange(d.shape[0]), k]
    return idx, d2


def overlap_ratio(p: np.ndarray, q: np.ndarray, T: np.ndarray, tau: float):
    """Eq. 9 for Gaussian means p [Np, 3] of P and q [Nq, 3] of Q under the
    estimate T of T_{P->Q}.  Returns (ratio, reciprocal pairs, pairs closer
    than tau, nn_pq, nn_qp)."""
    pt = transform_points_f32(p, T)
    q = np.asarray(q, F32)
    nn_pq, d_pq = nearest(pt, q)
    nn_qp, _ = nearest(q, pt)
    recip = np.zeros(pt.shape[0], bool)
    has = nn_pq >= 0
    recip[has] = nn_qp[nn_pq[has]] == np.arange(pt.shape[0])[has]
    tau2 = F32(F32(tau) * F32(tau))
    pairs = int(recip.sum())
    inliers = int((recip & (d_pq < tau2)).sum())
    return (inliers / pairs if pairs else 0.0), pairs, inliers, nn_pq, nn_qp
