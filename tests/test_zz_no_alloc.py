"""ls_overlap_ratio_noalloc (workspace in the library's static per-device
scratch array) against ls_overlap_ratio with a caller workspace, through the
C ABI: two calls in a row, the second with smaller inputs, so the second
runs over the first call's leftovers in the shared array.  Matches are
integer decisions, so the bar is bit-exact: every nearest-neighbour index
and both counts."""

import ctypes as C

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

from paper_2408_10154_amd import lib as L
from paper_2408_10154_amd import synth

pytestmark = pytest.mark.gpu


def _dev(pts):
    return torch.as_tensor(np.ascontiguousarray(np.asarray(pts, np.float32).T), device="cuda").contiguous()


def _T(rng):
    T = np.eye(4)
    T[:3, :3] = Rotation.from_rotvec(rng.normal(size=3) / np.sqrt(3) * np.deg2rad(6.0)).as_matrix()
    T[:3, 3] = rng.uniform(-0.2, 0.2, 3)
    return (C.c_float * 12)(*[float(v) for v in T[:3, :4].reshape(-1)])


def _both(P, Q, T, tau):
    p, q = _dev(P), _dev(Q)
    n_p, n_q = p.shape[1], q.shape[1]
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    out = {}
    for kind in ("workspace", "noalloc"):
        nn_pq = torch.full((max(n_p, 1),), -7, dtype=torch.int32, device="cuda")
        nn_qp = torch.full((max(n_q, 1),), -7, dtype=torch.int32, device="cuda")
        counts = torch.full((2,), -7, dtype=torch.int32, device="cuda")
        if kind == "workspace":
            need = L.ls_overlap_workspace_size(n_p, n_q)
            work = torch.empty(max(need, 1), dtype=torch.uint8, device="cuda")
            L.ls_overlap_ratio(p.data_ptr(), n_p, q.data_ptr(), n_q, T, tau, nn_pq.data_ptr(), nn_qp.data_ptr(),
                               counts.data_ptr(), work.data_ptr(), work.numel(), stream)
        else:
            L.ls_overlap_ratio_noalloc(p.data_ptr(), n_p, q.data_ptr(), n_q, T, tau, nn_pq.data_ptr(),
                                       nn_qp.data_ptr(), counts.data_ptr(), stream)
        torch.cuda.synchronize()
        out[kind] = (nn_pq[:n_p].cpu().numpy(), nn_qp[:n_q].cpu().numpy(), counts.cpu().numpy())
    return out


def test_noalloc_overlap_equals_workspace_call_twice(gpu):
    rng = np.random.default_rng(11)
    # first call: the registration pair's submaps (150k + 120k Gaussian means)
    d = synth.registration_pair(2, 150_000, 120_000, views_p=1, views_q=1)
    P1, Q1 = np.asarray(d["P"]["mean"]).T, np.asarray(d["Q"]["mean"]).T
    # second call: smaller, ragged clouds
    P2, Q2 = rng.uniform(-2, 2, (5003, 3)), rng.uniform(-2, 2, (4099, 3))
    for k, (P, Q) in enumerate(((P1, Q1), (P2, Q2))):
        print(f"noalloc call {k}: np={len(P)} nq={len(Q)}", flush=True)
        out = _both(P, Q, _T(rng), 0.2)
        a, b = out["workspace"], out["noalloc"]
        assert a[2][0] > 0
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)


def test_noalloc_overlap_refuses_oversized_sets(gpu):
    p = torch.zeros(3, 8, device="cuda")
    nn = torch.zeros(L.LS_OVERLAP_NOALLOC_MAX_POINTS + 1, dtype=torch.int32, device="cuda")
    counts = torch.zeros(2, dtype=torch.int32, device="cuda")
    T = (C.c_float * 12)(1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0)
    with pytest.raises(RuntimeError, match="NOALLOC_MAX_POINTS"):
        L.ls_overlap_ratio_noalloc(p.data_ptr(), L.LS_OVERLAP_NOALLOC_MAX_POINTS + 1, p.data_ptr(), 8, T, 0.2,
                                   nn.data_ptr(), nn.data_ptr(), counts.data_ptr(),
                                   C.c_void_p(torch.cuda.current_stream().cuda_stream))
