"""Serving loop: batch invariance, continuous admission, budget, overflow
recovery, non-finite inputs, graph replay vs eager launches."""

import math
import time

import numpy as np
import pytest
import torch

from paper_2408_10154_amd import synth

pytestmark = pytest.mark.gpu

ITERS = 60


def _pair(seed, n_p, n_q, views, w=256, h=192, f=200.0):
    from paper_2408_10154_amd import register as REG
    from paper_2408_10154_amd.render import GaussianSet

    d = synth.registration_pair(seed, n_p, n_q, views_p=views, views_q=views, width=w, height=h, f=f,
                                rot_deg_max=4.0, trans_max=0.1)
    P, Q = GaussianSet.from_numpy(d["P"]), GaussianSet.from_numpy(d["Q"])
    rgbP, depP = REG.keyframe_targets(P, d["cam"], d["kf_p"])
    rgbQ, depQ = REG.keyframe_targets(Q, d["cam"], d["kf_q"])
    return dict(d=d, args=(P, Q, d["cam"], d["kf_p"], d["kf_q"], rgbP, depP, rgbQ, depQ))


def _plain(p):
    from paper_2408_10154_amd import register as REG

    return REG.register_pair(*p["args"], params=REG.default_params(ITERS))


def _same(a, b):
    """Pose-only registration is deterministic and batch-invariant: compare bits."""
    return np.array_equal(a["T"], b["T"]) and np.array_equal(a["per_view"], b["per_view"]) and \
        np.array_equal(a["residual"], b["residual"])


@pytest.fixture(scope="module")
def pairs(gpu):
    return [_pair(11, 20000, 15000, 2), _pair(12, 9000, 12000, 3), _pair(13, 30000, 25000, 2)]


@pytest.mark.parametrize("graphs", [True, False])
def test_result_is_the_same_alone_and_in_the_mix(pairs, graphs):
    from paper_2408_10154_amd import register as REG
    from paper_2408_10154_amd.serve import Server

    alone = [_plain(p) for p in pairs]
    with Server(chunk_iters=7, use_graphs=graphs) as sv:
        tickets = [sv.submit(*p["args"], params=REG.default_params(ITERS)) for p in pairs]
        mixed = [sv.wait(t) for t in tickets]
        st = sv.stats()
    for a, m in zip(alone, mixed):
        assert m["status"] == 0 and m["iters"] == ITERS
        # pose-only gradients are reduced without atomics and never mix renders: bit-identical
        np.testing.assert_array_equal(m["per_view"], a["per_view"])
        np.testing.assert_array_equal(m["residual"], a["residual"])
        np.testing.assert_array_equal(m["T"], a["T"])
    assert st["completed"] == len(pairs) and st["failed"] == 0
    assert (st["graph_replays"] > 0) == graphs


def test_requests_join_while_others_run(pairs):
    """A request submitted while another is mid-run is admitted at the next
    chunk boundary (the active set is rebuilt, the running pair's optimiser
    state is carried over) and both results equal the plain path's bits."""
    from paper_2408_10154_amd import register as REG
    from paper_2408_10154_amd.serve import Server

    long_iters = 4 * ITERS
    with Server(chunk_iters=5) as sv:
        t0 = sv.submit(*pairs[2]["args"], params=REG.default_params(long_iters))
        t_start = time.time()
        while sv.stats()["iterations"] < 10 and time.time() - t_start < 60:
            time.sleep(0.001)
        t1 = sv.submit(*pairs[1]["args"], params=REG.default_params(ITERS))
        r0, r1 = sv.wait(t0), sv.wait(t1)
        st = sv.stats()
    assert st["epochs"] >= 2
    assert st["iterations"] < long_iters + ITERS  # the two overlapped in batched iterations
    assert r0["status"] == 0 and r1["status"] == 0
    assert _same(r0, REG.register_pair(*pairs[2]["args"], params=REG.default_params(long_iters)))
    assert _same(r1, _plain(pairs[1]))


def test_budget_admits_one_at_a_time_and_rejects_oversized(pairs):
    from paper_2408_10154_amd import lib as L
    from paper_2408_10154_amd import register as REG
    from paper_2408_10154_amd.serve import Server

    with Server(budget_bytes=40 << 20, max_slots=8) as sv:
        with pytest.raises(L.LsError) as e:
            sv.submit(*pairs[2]["args"], params=REG.default_params(ITERS))
        assert e.value.status == L.LS_ERR_BUDGET
    with Server(budget_bytes=450 << 20, max_slots=8) as sv:
        ts = [sv.submit(*p["args"], params=REG.default_params(ITERS)) for p in pairs[:2]]
        rs = [sv.wait(t) for t in ts]
        st = sv.stats()
    assert all(r["status"] == 0 for r in rs)
    assert st["peak_bytes"] <= 450 << 20
    assert rs[1]["times"]["queue"] > 0.0


@pytest.mark.parametrize("cap,peak", [(300_000, 1), (500_000, 2)])
def test_active_pixel_cap_limits_concurrency(pairs, cap, peak):
    """Pairs render 196,608 / 294,912 / 196,608 pixels per iteration.  A cap of
    300k admits one pair at a time (the head always enters an empty active
    set); 500k lets the first two share.  Results stay bit-identical."""
    from paper_2408_10154_amd import register as REG
    from paper_2408_10154_amd.serve import Server

    with Server(chunk_iters=8, max_active_pixels=cap) as sv:
        ts = [sv.submit(*p["args"], params=REG.default_params(ITERS)) for p in pairs]
        rs = [sv.wait(t) for t in ts]
        st = sv.stats()
    assert st["peak_active"] == peak, st
    for r, p in zip(rs, pairs):
        assert r["status"] == 0 and _same(r, _plain(p))


def test_capacity_overflow_is_recovered(pairs):
    """headroom 0.5 sizes the instance buffers to half the count measured at
    each rebuild: the first chunk overflows, is rolled back and re-run with
    more room, and every result still equals the plain path's bits."""
    from paper_2408_10154_amd import register as REG
    from paper_2408_10154_amd.serve import Server

    with Server(chunk_iters=4, instance_headroom=0.5) as sv:
        ts = [sv.submit(*p["args"], params=REG.default_params(ITERS)) for p in pairs]
        rs = [sv.wait(t) for t in ts]
        st = sv.stats()
    assert st["overflow_retries"] >= 1
    for r, p in zip(rs, pairs):
        assert r["status"] == 0 and _same(r, _plain(p))


def test_non_finite_pair_is_rejected_others_continue(pairs):
    from paper_2408_10154_amd import lib as L
    from paper_2408_10154_amd import register as REG
    from paper_2408_10154_amd.render import GaussianSet
    from paper_2408_10154_amd.serve import Server

    args = list(pairs[1]["args"])
    bad = GaussianSet(*[t.clone() for t in args[0].tensors()])
    bad.mean[1, 17] = float("nan")
    args[0] = bad
    with Server() as sv:
        good = sv.submit(*pairs[0]["args"], params=REG.default_params(ITERS))
        with pytest.raises(L.LsError) as e:
            sv.submit(*args, params=REG.default_params(ITERS))
        assert e.value.status == L.LS_ERR_NONFINITE
        r = sv.wait(good)
    assert r["status"] == 0


def test_reused_server_state_matches_plain(pairs):
    """One slot: the three pairs run in three successive active sets on reused
    buffers; each result still equals the plain path's bits (the per-view
    gradient accumulator is cleared when a view is admitted)."""
    from paper_2408_10154_amd import register as REG
    from paper_2408_10154_amd.serve import Server

    with Server(max_slots=1, chunk_iters=9) as sv:
        ts = [sv.submit(*p["args"], params=REG.default_params(ITERS)) for p in reversed(pairs)]
        rs = [sv.wait(t) for t in ts]
        st = sv.stats()
    assert st["epochs"] >= 3
    for r, p in zip(rs, reversed(pairs)):
        assert r["status"] == 0 and _same(r, _plain(p))


def test_server_step_exit_matches_plain(pairs):
    """Early exit by the step rule in the serving loop: the pairs' views
    freeze at the same iterations as in ls_register_pair (the rule runs in
    the same kernel on per-view state), so the results are the same bits;
    a request with the loss rule is refused by a server that runs the step
    rule."""
    from paper_2408_10154_amd import lib as L
    from paper_2408_10154_amd import register as REG
    from paper_2408_10154_amd.serve import Server

    prm = REG.default_params(ITERS, exit_rel_tol=0.2, exit_patience=5, exit_mode="step")
    plain = [REG.register_pair(*p["args"], params=prm) for p in pairs]
    with Server(max_slots=8, chunk_iters=8) as sv:
        ts = [sv.submit(*p["args"], params=prm) for p in pairs]
        with pytest.raises(L.LsError):
            sv.submit(*pairs[0]["args"], params=REG.default_params(ITERS, exit_rel_tol=0.2, exit_patience=5))
        rs = [sv.wait(t) for t in ts]
    for r, b in zip(rs, plain):
        assert r["status"] == 0 and b["status"] == 0 and _same(r, b)
    print("plain iterations", [b["iters"] for b in plain])


def test_server_fused_l1_matches_the_loss_kernel_path(pairs, monkeypatch):
    """A server whose iterations form the L1 gradient inside the backward
    (the default for plain L1) and one that runs the loss kernel every
    iteration give the same results bit for bit."""
    from paper_2408_10154_amd import register as REG
    from paper_2408_10154_amd.serve import Server

    out = {}
    for mode in ("1", "0"):
        monkeypatch.setenv("LS_FUSED_L1", mode)
        with Server(max_slots=8, chunk_iters=8) as sv:
            ts = [sv.submit(*p["args"], params=REG.default_params(ITERS)) for p in pairs]
            out[mode] = [sv.wait(t) for t in ts]
    for a, b in zip(out["1"], out["0"]):
        assert a["status"] == 0 and b["status"] == 0 and _same(a, b)


def test_submit_orders_reads_after_the_producer_stream(pairs):
    """A request whose Gaussians are written on a side stream just before
    submitting (behind a chain of long kernels): the server's finiteness
    check and its iterations read them only after the producer's work, so
    the request is accepted (the buffers start as NaN) and its result equals
    the plain path's bit for bit."""
    from paper_2408_10154_amd import register as REG
    from paper_2408_10154_amd.render import GaussianSet
    from paper_2408_10154_amd.serve import Server

    args = list(pairs[0]["args"])
    src_p, src_q = args[0], args[1]
    Pn = GaussianSet(*[torch.full_like(t, float("nan")) for t in src_p.tensors()])
    Qn = GaussianSet(*[torch.full_like(t, float("nan")) for t in src_q.tensors()])
    big = torch.randn(4096, 4096, device="cuda")
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    with Server() as sv:
        with torch.cuda.stream(side):
            for _ in range(16):
                big = big @ big
                big = big / big.norm()
            for dst, src in zip(Pn.tensors() + Qn.tensors(), src_p.tensors() + src_q.tensors()):
                dst.copy_(src)
            ticket = sv.submit(Pn, Qn, *args[2:], params=REG.default_params(ITERS))
        r = sv.wait(ticket)
    assert r["status"] == 0
    assert _same(r, _plain(pairs[0]))
