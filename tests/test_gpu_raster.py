"""GPU parity of the rasterizer C ABI against the FP64 oracle.

Every stage is checked twice: in isolation, with both sides fed identical
FP32 inputs (projected records written from the oracle), and end to end from
the Gaussian parameters.  Tolerances: images 1e-4 relative (1 m unit for
depth), gradients 1e-3 relative; pixels whose alpha/clamp/stop decision sits
within a rounding margin of its threshold (the oracle reports it) are left out
of the element-wise image check and counted."""

import math

import numpy as np
import pytest
import torch

from oracle import raster as R
from paper_2408_10154_amd import synth
from tests import _util as U

pytestmark = pytest.mark.gpu

F64 = torch.float64


def _batch(jobs_np, capacity=None):
    from paper_2408_10154_amd.render import GaussianSet, RenderBatch

    jobs = [(GaussianSet.from_numpy(g), cam, w2c) for g, cam, w2c in jobs_np]
    return RenderBatch(jobs, capacity=capacity)


def _three_scenes():
    """Three renders of different sizes (one ragged in both directions)."""
    a = synth.scene_small(0, n=1500)
    b = synth.scene_tiny(5, 700, 100, 70, 90.0)
    c = synth.scene_tiny(6, 300, 33, 17, 30.0)
    return [(s["gauss"], s["cam"], s["w2c"]) for s in (a, b, c)], [a["target_pose"], b["target_pose"], c["target_pose"]]


def _load_records(batch, per_render):
    rec = np.zeros((batch.M, 12), np.float32)
    rad = np.zeros(batch.M, np.int32)
    til = np.zeros(batch.M, np.int32)
    for r, (rc, rd, tl) in enumerate(per_render):
        o = int(batch.item_off[r])
        rec[o:o + len(rd)] = rc
        rad[o:o + len(rd)] = rd
        til[o:o + len(rd)] = tl
    batch.rec.copy_(torch.as_tensor(rec))
    batch.radius.copy_(torch.as_tensor(rad))
    batch.tiles.copy_(torch.as_tensor(til))


def test_project_matches_oracle(gpu):
    jobs, poses = _three_scenes()
    b = _batch(jobs)
    pose = torch.as_tensor(np.stack(poses), device="cuda")
    b.project(pose)
    rec = b.rec.cpu().numpy()
    rad = b.radius.cpu().numpy()
    til = b.tiles.cpu().numpy()
    for r, (g, cam, w2c) in enumerate(jobs):
        o, e = int(b.item_off[r]), int(b.item_off[r + 1])
        gt = R.to_f64(g)
        pr = R.project(gt["mean"], gt["log_scale"], gt["quat"], U.oracle_camera(cam), torch.as_tensor(w2c, dtype=F64),
                       torch.as_tensor(poses[r], dtype=F64))
        near = pr["margin_px"] < 1e-3
        same = (rad[o:e] == pr["radius"]) & (til[o:e] == pr["tiles"])
        assert np.all(same | near), (r, np.nonzero(~(same | near))[0][:10])
        assert near.mean() < 0.01
        vis = (pr["radius"] > 0) & same
        ref = U.records_from_oracle(pr, g)[0]
        conic = pr["conic"].detach().numpy()
        for col, refv in ((0, pr["u"].detach().numpy()), (1, pr["v"].detach().numpy()), (6, pr["depth"].detach().numpy())):
            np.testing.assert_allclose(rec[o:e, col][vis], refv[vis], rtol=2e-6, atol=2e-5)
        for k in range(3):
            np.testing.assert_allclose(rec[o:e, 2 + k][vis], conic[vis, k], rtol=1e-4,
                                       atol=1e-4 * np.abs(conic[vis]).max())
        np.testing.assert_allclose(rec[o:e, 5][vis], ref[vis, 5], rtol=1e-6)
        np.testing.assert_array_equal(rec[o:e, 8:11][vis], ref[vis, 8:11])


@pytest.mark.parametrize("compact", ["0", "1"])
def test_bin_sort_bit_exact_with_ties(gpu, monkeypatch, compact):
    """Equal-depth runs across many Gaussians, three renders, a small capacity;
    with and without the compaction of kept items before the depth sort."""
    monkeypatch.setenv("LS_COMPACT", compact)
    jobs, poses = _three_scenes()
    b = _batch(jobs, capacity=4096)  # deliberately small: exercises the regrow path
    per, expect_tiles, expect_items = [], [], []
    for r, (g, cam, w2c) in enumerate(jobs):
        gt = R.to_f64(g)
        pr = R.project(gt["mean"], gt["log_scale"], gt["quat"], U.oracle_camera(cam), torch.as_tensor(w2c, dtype=F64),
                       torch.as_tensor(poses[r], dtype=F64))
        rc, rd, tl = U.records_from_oracle(pr, g)
        # equal-depth ties: runs of identical depth bits across many Gaussians
        rc[20:80, 6] = rc[20, 6]
        rc[100:400:7, 6] = np.float32(2.5)
        per.append((rc, rd, tl))
        tile_of, gid, _ = R.bin_sort(rc[:, 0], rc[:, 1], rc[:, 6], rd.astype(np.int64), U.oracle_camera(cam))
        expect_tiles.append(tile_of + int(b.tile_off[r]))
        expect_items.append(gid + int(b.item_off[r]))
    _load_records(b, per)
    b.bin_sort()
    n = b.instances()
    exp_t = np.concatenate(expect_tiles)
    exp_i = np.concatenate(expect_items)
    assert n == len(exp_t)
    assert int(b.count[1].item()) == 0
    np.testing.assert_array_equal(b.tile_of[:n].cpu().numpy().astype(np.int64), exp_t)
    np.testing.assert_array_equal(b.item[:n].cpu().numpy().astype(np.int64), exp_i)
    rng = b.range.cpu().numpy()
    for t in range(b.T):
        s, e = rng[t]
        sel = np.nonzero(exp_t == t)[0]
        if len(sel):
            assert (s, e) == (sel[0], sel[-1] + 1)
        else:
            assert (s, e) == (0, 0)


@pytest.mark.parametrize("compact", ["0", "1"])
@pytest.mark.parametrize("n_items,seed", [(1500, 11), (9000, 12)])
def test_bin_sort_bit_exact_long_tile_lists(gpu, monkeypatch, n_items, seed, compact):
    """Tile lists from a few hundred to ~9,000 entries (items covering up to
    the whole 5 x 3 tile grid), with equal-depth runs, culled items and a
    ragged grid; the order must equal the oracle's (tile, depth bits, item),
    with and without the compaction of kept items before the depth sort."""
    monkeypatch.setenv("LS_COMPACT", compact)
    rng = np.random.default_rng(seed)
    s = synth.scene_tiny(seed, n_items, 70, 45, 60.0)  # 5 x 3 tiles, the last column and row partial
    jobs = [(s["gauss"], s["cam"], s["w2c"])]
    b = _batch(jobs, capacity=4 * n_items * 15)
    camo = U.oracle_camera(s["cam"])
    u = rng.uniform(-10.0, 80.0, n_items).astype(np.float32)
    v = rng.uniform(-10.0, 55.0, n_items).astype(np.float32)
    rad = rng.integers(1, 40, n_items).astype(np.int64)
    rad[rng.random(n_items) < 0.05] = 0  # culled
    z = rng.uniform(0.5, 9.0, n_items).astype(np.float32)
    z[100:700] = np.float32(2.0)          # a long run of equal depths
    z[1000::37] = z[1000]                 # scattered ties
    x0, x1, y0, y1 = R.tile_rect_f32(u, v, rad, camo)
    tl = np.where(rad > 0, np.maximum(x1 - x0, 0) * np.maximum(y1 - y0, 0), 0)
    rad = np.where(tl > 0, rad, 0)
    rc = np.zeros((n_items, 12), np.float32)
    rc[:, 0], rc[:, 1], rc[:, 6] = u, v, z
    rc[:, 2], rc[:, 4], rc[:, 5] = 0.01, 0.01, 0.5
    _load_records(b, [(rc, rad.astype(np.int32), tl.astype(np.int32))])
    exp_t, exp_i, ranges = R.bin_sort(u, v, z, rad, camo)
    lens = np.diff(np.asarray(ranges), axis=1).ravel()
    b.bin_sort()
    n = b.instances()
    assert n == len(exp_t) and int(b.count[1].item()) == 0
    if n_items > 5000:
        assert lens.max() > 4096  # lists longer than a radix-sort block takes
    np.testing.assert_array_equal(b.tile_of[:n].cpu().numpy().astype(np.int64), exp_t)
    np.testing.assert_array_equal(b.item[:n].cpu().numpy().astype(np.int64), exp_i)
    np.testing.assert_array_equal(b.range.cpu().numpy().reshape(-1, 2), np.asarray(ranges).reshape(-1, 2))


@pytest.mark.parametrize("views,digit_bits", [(2, 6), (4, 7), (16, 8)])
def test_bin_sort_bit_exact_across_tile_digit_widths(gpu, views, digit_bits):
    """Batches of 640x480 renders (1,200 tiles each) whose tile keys take 12,
    13 and 15 bits, so the tile passes run on 6-, 7- and 8-bit digits: the
    lists, ranges and counts equal the oracle's per-render bin sort (tile
    keys offset by each render's first tile), with equal-depth runs, culled
    items and items on the image border."""
    rng = np.random.default_rng(40 + views)
    per, exp_t, exp_i = [], [], []
    jobs = []
    for r in range(views):
        s = synth.scene_tiny(70 + r, 600, 640, 480, 500.0)
        jobs.append((s["gauss"], s["cam"], s["w2c"]))
    b = _batch(jobs, capacity=600 * views * 60)
    bits = int(np.ceil(np.log2(b.T)))
    assert {12: 6, 13: 7, 14: 7, 15: 8, 16: 8}[bits] == digit_bits
    for r, (g, cam, w2c) in enumerate(jobs):
        camo = U.oracle_camera(cam)
        n = 600
        u = rng.uniform(-30.0, 670.0, n).astype(np.float32)
        v = rng.uniform(-30.0, 510.0, n).astype(np.float32)
        rad = rng.integers(1, 48, n).astype(np.int64)
        rad[rng.random(n) < 0.05] = 0
        z = rng.uniform(0.5, 9.0, n).astype(np.float32)
        z[50:150] = np.float32(3.0)
        x0, x1, y0, y1 = R.tile_rect_f32(u, v, rad, camo)
        tl = np.where(rad > 0, np.maximum(x1 - x0, 0) * np.maximum(y1 - y0, 0), 0)
        rad = np.where(tl > 0, rad, 0)
        rc = np.zeros((n, 12), np.float32)
        rc[:, 0], rc[:, 1], rc[:, 6] = u, v, z
        rc[:, 2], rc[:, 4], rc[:, 5] = 0.01, 0.01, 0.5
        per.append((rc, rad.astype(np.int32), tl.astype(np.int32)))
        t, i, _ = R.bin_sort(u, v, z, rad, camo)
        exp_t.append(np.asarray(t) + int(b.tile_off[r]))
        exp_i.append(np.asarray(i) + int(b.item_off[r]))
    _load_records(b, per)
    b.bin_sort()
    exp_t, exp_i = np.concatenate(exp_t), np.concatenate(exp_i)
    n = b.instances()
    assert n == len(exp_t) and int(b.count[1].item()) == 0
    np.testing.assert_array_equal(b.tile_of[:n].cpu().numpy().astype(np.int64), exp_t)
    np.testing.assert_array_equal(b.item[:n].cpu().numpy().astype(np.int64), exp_i)
    rng_ = b.range.cpu().numpy().reshape(-1, 2)
    starts = np.searchsorted(exp_t, np.arange(b.T), side="left")
    ends = np.searchsorted(exp_t, np.arange(b.T), side="right")
    expect = np.where((ends > starts)[:, None], np.stack([starts, ends], 1), 0)
    np.testing.assert_array_equal(rng_, expect)


def test_render_fwd_same_inputs(gpu):
    jobs, poses = _three_scenes()
    b = _batch(jobs)
    per = []
    oracle_imgs = []
    bg = [0.1, 0.2, 0.3]
    for r, (g, cam, w2c) in enumerate(jobs):
        gt = R.to_f64(g)
        camo = U.oracle_camera(cam)
        pr = R.project(gt["mean"], gt["log_scale"], gt["quat"], camo, torch.as_tensor(w2c, dtype=F64),
                       torch.as_tensor(poses[r], dtype=F64))
        rc, rd, tl = U.records_from_oracle(pr, g)
        per.append((rc, rd, tl))
        _, gid, ranges = R.bin_sort(rc[:, 0], rc[:, 1], rc[:, 6], rd.astype(np.int64), camo)
        t64 = lambda x: torch.as_tensor(np.asarray(x, np.float64))  # noqa: E731
        out = R.composite(t64(rc[:, 0]), t64(rc[:, 1]), t64(rc[:, 2:5]), t64(rc[:, 5]), t64(rc[:, 8:11]), t64(rc[:, 6]),
                          gid, ranges, camo, bg=torch.tensor(bg, dtype=F64))
        oracle_imgs.append(out)
    _load_records(b, per)
    b.bin_sort()
    b.render_fwd(bg)
    total_px = flagged = 0
    for r in range(len(jobs)):
        v = b.image_views(r)
        o = oracle_imgs[r]
        ok = o["margin"] >= 1e-5
        total_px += ok.size
        flagged += int((~ok).sum())
        assert U.image_close(v["rgb"].cpu().numpy(), o["rgb"].numpy(), ok[None]) == 0
        assert U.image_close(v["depth"].cpu().numpy(), o["depth"].numpy(), ok) == 0
        assert U.image_close(v["alpha"].cpu().numpy(), o["alpha"].numpy(), ok) == 0
        assert U.image_close(v["T_final"].cpu().numpy(), o["T_final"].numpy(), ok) == 0
        np.testing.assert_array_equal(v["n_last"].cpu().numpy()[ok], o["n_last"][ok])
    assert flagged <= 0.001 * total_px


def test_end_to_end_forward(gpu):
    jobs, poses = _three_scenes()
    b = _batch(jobs)
    pose = torch.as_tensor(np.stack(poses), device="cuda")
    b.project(pose)
    b.bin_sort()
    b.render_fwd()
    total = flagged = 0
    for r, (g, cam, w2c) in enumerate(jobs):
        _, _, o = U.oracle_render(g, cam, w2c, poses[r])
        v = b.image_views(r)
        ok = o["margin"] >= 2e-4
        total += ok.size
        flagged += int((~ok).sum())
        for key in ("rgb", "depth", "alpha"):
            mask = ok[None] if key == "rgb" else ok
            assert U.image_close(v[key].cpu().numpy(), o[key].detach().numpy(), mask) == 0, key
    assert flagged <= 0.01 * total


def _backward_case(jobs, poses, want_pose=True, seed=0):
    b = _batch(jobs)
    rng = np.random.default_rng(seed)
    up = synth.random_image_grads(rng, b.P)
    pose = torch.as_tensor(np.stack(poses), device="cuda")
    b.project(pose)
    b.bin_sort()
    b.render_fwd()
    from paper_2408_10154_amd.render import GaussianSet  # noqa: F401

    grads = [gs.zeros_like() for gs in b.gsets]
    pose_grad = torch.zeros_like(pose)
    dev = lambda x: torch.as_tensor(x, device="cuda")  # noqa: E731
    b.render_bwd(up_rgb=dev(up["rgb"].reshape(-1)), up_depth=dev(up["depth"]), up_alpha=dev(up["alpha"]),
                 grads=grads, pose=pose, pose_grad=pose_grad if want_pose else None)
    return b, up, grads, pose_grad


def test_backward_matches_oracle(gpu):
    """Gradients of a random linear function of the three renders' images
    (colour, depth, alpha) to every Gaussian parameter and the pose, against
    the oracle: the norm clause over all Gaussians and the element clause
    over those not touched by a flipped decision."""
    jobs, poses = _three_scenes()
    b, up, grads, pose_grad = _backward_case(jobs, poses)
    for r, (g, cam, w2c) in enumerate(jobs):
        gt, pt, o = U.oracle_render(g, cam, w2c, poses[r], requires_grad=True)
        H, W = cam["height"], cam["width"]
        p0 = int(b.pix_off[r])
        ur = torch.as_tensor(up["rgb"].reshape(-1)[3 * p0:3 * p0 + 3 * H * W].reshape(3, H, W), dtype=F64)
        ud = torch.as_tensor(up["depth"][p0:p0 + H * W].reshape(H, W), dtype=F64)
        ua = torch.as_tensor(up["alpha"][p0:p0 + H * W].reshape(H, W), dtype=F64)
        ((o["rgb"] * ur).sum() + (o["depth"] * ud).sum() + (o["alpha"] * ua).sum()).backward()
        gg = grads[r]
        n = len(g["opacity_logit"])
        excl = U.render_flips(b, r, o, n)
        pairs = []
        for name in ("mean", "log_scale", "quat", "opacity_logit", "rgb"):
            got = getattr(gg, name).cpu().numpy()
            pairs.append((name, got.T if got.ndim == 2 else got, gt[name].grad.numpy()))
        print(U.check_gradients(pairs, excl, f"render {r} (excluded {int(excl.sum())} of {n})"))
        print(U.check_gradients([("pose", pose_grad[r].cpu().numpy()[None], pt.grad.numpy()[None])], None,
                                f"render {r}"))


def test_loss_l1_matches_oracle(gpu):
    jobs, _ = _three_scenes()
    b = _batch(jobs)
    rng = np.random.default_rng(3)
    pr = rng.random(3 * b.P).astype(np.float32)
    pdp = (rng.random(b.P) * 3).astype(np.float32)
    tr = rng.random(3 * b.P).astype(np.float32)
    td = np.where(rng.random(b.P) < 0.2, 0.0, rng.random(b.P) * 3).astype(np.float32)
    td[int(b.pix_off[2]):int(b.pix_off[3])] = 0.0  # a render with no valid pixel
    pr[:7] = tr[:7]  # exact ties: sign(0) = 0
    b.rgb.copy_(torch.as_tensor(pr))
    b.depth.copy_(torch.as_tensor(pdp))
    loss, g_rgb, g_depth, scale = b.loss_l1(torch.as_tensor(tr, device="cuda"), torch.as_tensor(td, device="cuda"))
    for r, (_, cam, _) in enumerate(jobs):
        H, W = cam["height"], cam["width"]
        p0 = int(b.pix_off[r])
        prr = torch.as_tensor(pr[3 * p0:3 * p0 + 3 * H * W].reshape(3, H, W), dtype=F64).requires_grad_(True)
        pdd = torch.as_tensor(pdp[p0:p0 + H * W].reshape(H, W), dtype=F64).requires_grad_(True)
        ref = R.loss_l1(prr, pdd, torch.as_tensor(tr[3 * p0:3 * p0 + 3 * H * W].reshape(3, H, W), dtype=F64),
                        torch.as_tensor(td[p0:p0 + H * W].reshape(H, W), dtype=F64))
        np.testing.assert_allclose(loss[r].item(), ref.item(), rtol=1e-5)
        if ref.requires_grad:
            ref.backward()
            sc = scale[r].item()
            np.testing.assert_allclose(g_rgb[3 * p0:3 * p0 + 3 * H * W].cpu().numpy() * sc,
                                       prr.grad.numpy().reshape(-1), rtol=1e-6, atol=1e-9)
            np.testing.assert_allclose(g_depth[p0:p0 + H * W].cpu().numpy() * sc, pdd.grad.numpy().reshape(-1),
                                       rtol=1e-6, atol=1e-9)
        else:
            assert scale[r].item() == 0.0


def test_adam_matches_oracle(gpu):
    from oracle import register as G
    from paper_2408_10154_amd.render import adam

    rng = np.random.default_rng(1)
    sizes = [7, 1000, 4097]
    lrs = [0.01, 0.003, 0.1]
    ps = [rng.normal(size=n) for n in sizes]
    dev = [[torch.as_tensor(p, dtype=torch.float32, device="cuda"), torch.zeros(n, device="cuda"),
            torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda"), lr] for p, n, lr in zip(ps, sizes, lrs)]
    ref = [[torch.as_tensor(p), torch.zeros(n, dtype=F64), torch.zeros(n, dtype=F64)] for p, n in zip(ps, sizes)]
    for step in range(1, 21):
        for i, n in enumerate(sizes):
            gr = rng.normal(size=n)
            dev[i][1].copy_(torch.as_tensor(gr))
            G.adam_step(ref[i][0], torch.as_tensor(gr), ref[i][1], ref[i][2], step, lrs[i])
        adam([tuple(d) for d in dev], step)
        for d in dev:
            assert float(d[1].abs().max()) == 0.0  # gradients consumed
    for d, rf in zip(dev, ref):
        np.testing.assert_allclose(d[0].cpu().numpy(), rf[0].numpy(), rtol=1e-5, atol=1e-5)


def test_fused_backward_adam_matches_separate_steps(gpu):
    """Three renders of their own Gaussian sets (some Gaussians behind the
    camera, so culled), four mapping iterations against fixed targets:
    ls_render_bwd_project_adam updates the parameters and moments bit for bit
    as ls_render_bwd_project into gradient arrays followed by ls_adam does,
    and accumulates the same pose gradients; culled Gaussians step like the
    others; renders sharing a Gaussian set are refused.  The tile backward
    sums a Gaussian's per-tile contributions with float atomics in no fixed
    order, so each iteration the fused side takes over the other side's
    workspace (its accumulated tile gradients) before its projection
    backward: both then chain the same accumulators."""
    from paper_2408_10154_amd import lib as L
    from paper_2408_10154_amd.render import adam

    jobs, poses = _three_scenes()
    for g, _, _ in jobs:
        g["mean"][2, ::9] = -np.abs(g["mean"][2, ::9])  # every ninth Gaussian behind the camera
    pose = torch.as_tensor(np.stack(poses), device="cuda").contiguous()
    names = ("mean", "log_scale", "quat", "opacity_logit", "rgb")
    lrs = dict(mean=1e-3, log_scale=5e-3, quat=1e-3, opacity_logit=5e-2, rgb=2.5e-3)
    sides = []
    for _ in range(2):
        b = _batch(jobs)
        b.project(pose)
        b.bin_sort()
        b.render_fwd()
        sides.append(b)
    tgt = [(sides[0].rgb.clone() * 0.9 + 0.05, sides[0].depth.clone() * 1.02)]
    a, f = sides
    grads = [g.zeros_like() for g in a.gsets]
    mom_a = [[(torch.zeros_like(t), torch.zeros_like(t)) for t in g.tensors()] for g in a.gsets]
    mom_f = [{n: (torch.zeros_like(t), torch.zeros_like(t), lrs[n]) for n, t in zip(names, g.tensors())}
             for g in f.gsets]
    pg = [torch.zeros_like(pose), torch.zeros_like(pose)]
    for step in range(1, 5):
        for i, b in enumerate(sides):
            b.project(pose)
            b.bin_sort()
            b.render_fwd()
            loss = torch.zeros(b.R, device="cuda")
            g_rgb, g_depth, scale = torch.zeros_like(b.rgb), torch.zeros_like(b.depth), torch.zeros(b.R, device="cuda")
            b.loss_l1(tgt[0][0], tgt[0][1], loss, g_rgb, g_depth, scale)
            b.render_bwd_tiles(up_rgb=g_rgb, up_depth=g_depth, scale=scale)
            if i == 0:
                snap = b.work.clone()  # the tile accumulators this side chains
                b.render_bwd_project(grads=grads, pose=pose, pose_grad=pg[0])
                groups = []
                for g, gr, mm in zip(b.gsets, grads, mom_a):
                    for n, t, tg, (m, v) in zip(names, g.tensors(), gr.tensors(), mm):
                        groups.append((t, tg, m, v, lrs[n]))
                adam(groups, step)
            else:
                b.work.copy_(snap)
                b.render_bwd_project_adam(mom_f, step, pose=pose, pose_grad=pg[1])
    torch.cuda.synchronize()
    for ga, gf, ma, mf in zip(a.gsets, f.gsets, mom_a, mom_f):
        for n, ta, tf, (m1, v1) in zip(names, ga.tensors(), gf.tensors(), ma):
            np.testing.assert_array_equal(tf.cpu().numpy(), ta.cpu().numpy(), err_msg=n)
            np.testing.assert_array_equal(mf[n][0].cpu().numpy(), m1.cpu().numpy(), err_msg=n)
            np.testing.assert_array_equal(mf[n][1].cpu().numpy(), v1.cpu().numpy(), err_msg=n)
    np.testing.assert_array_equal(pg[1].cpu().numpy(), pg[0].cpu().numpy())
    moved = [float((t - torch.as_tensor(jobs[0][0][n], device="cuda")).abs().max()) for n, t in
             zip(names, f.gsets[0].tensors())]
    assert min(moved) > 0  # every array took steps
    # one more iteration in which the poses step too: fused into the pose
    # reduction on one side, ls_adam over the accumulated gradient on the other
    poses2 = [pose.clone(), pose.clone()]
    pmv = [(torch.zeros_like(pose), torch.zeros_like(pose)) for _ in range(2)]
    for i, b in enumerate(sides):
        b.project(poses2[i])
        b.bin_sort()
        b.render_fwd()
        loss = torch.zeros(b.R, device="cuda")
        g_rgb, g_depth, scale = torch.zeros_like(b.rgb), torch.zeros_like(b.depth), torch.zeros(b.R, device="cuda")
        b.loss_l1(tgt[0][0], tgt[0][1], loss, g_rgb, g_depth, scale)
        b.render_bwd_tiles(up_rgb=g_rgb, up_depth=g_depth, scale=scale)
        pg[i].zero_()
        if i == 0:
            snap = b.work.clone()
            b.render_bwd_project(grads=grads, pose=poses2[0], pose_grad=pg[0])
            for r in range(b.R):  # per render: quaternion and translation groups, as the bench steps a pose
                adam([(poses2[0][r, :4], pg[0][r, :4], pmv[0][0][r, :4], pmv[0][1][r, :4], 2e-3),
                      (poses2[0][r, 4:], pg[0][r, 4:], pmv[0][0][r, 4:], pmv[0][1][r, 4:], 1e-2)], 5)
        else:
            b.work.copy_(snap)
            b.render_bwd_project_adam(mom_f, 5, pose=poses2[1], pose_grad=pg[1],
                                      pose_adam=(pmv[1][0], pmv[1][1], 2e-3, 1e-2))
    torch.cuda.synchronize()
    assert float(pg[1].abs().max()) == 0.0  # consumed by the fused step
    # against ls_adam steps of the same gradient
    np.testing.assert_array_equal(poses2[1].cpu().numpy(), poses2[0].cpu().numpy())
    assert float((poses2[1] - pose).abs().max()) > 0  # the poses moved
    # a batch whose renders share one Gaussian set is refused
    from paper_2408_10154_amd.render import GaussianSet, RenderBatch

    gs = GaussianSet.from_numpy(jobs[0][0])
    shared = RenderBatch([(gs, jobs[0][1], jobs[0][2]), (gs, jobs[0][1], jobs[0][2])])
    shared.project()
    shared.bin_sort()
    st = {n: (torch.zeros_like(t), torch.zeros_like(t), 1e-3) for n, t in zip(names, gs.tensors())}
    with pytest.raises(L.LsError):
        shared.render_bwd_project_adam([st, st], 1)


@pytest.mark.parametrize("compact", ["0", "1"])
@pytest.mark.parametrize("frac", [0.0, 0.37, 1.0])
def test_bin_sort_overflow_stays_within_capacity(gpu, monkeypatch, frac, compact):
    """Capacity below the instance count I (and 0, and exactly I): count is
    {min(I, capacity), I > capacity, I, 0}, nothing is written past the
    capacity in the instance arrays or past the workspace, and a re-run at
    capacity count[2] gives the lists of an ample capacity bit for bit."""
    from paper_2408_10154_amd import lib as L

    monkeypatch.setenv("LS_COMPACT", compact)
    jobs, poses = _three_scenes()
    pose = torch.as_tensor(np.stack(poses), device="cuda")
    ref = _batch(jobs)
    ref.project(pose)
    ref.bin_sort()
    n = ref.instances()
    assert n > 1000 and int(ref.count[1].item()) == 0
    b = _batch(jobs, capacity=max(n, 1))
    b.auto_grow = False
    b.project(pose)
    cap, guard = int(n * frac), 4096
    tile_of = torch.full((cap + guard,), -7, dtype=torch.int32, device="cuda")
    item = torch.full((cap + guard,), -7, dtype=torch.int32, device="cuda")
    wbytes = int(L.ls_batch_query(b.h, cap).workspace_bytes)
    work = torch.zeros(wbytes + 256 + guard, dtype=torch.uint8, device="cuda")
    wp = (work.data_ptr() + 255) // 256 * 256
    tail = wp - work.data_ptr() + wbytes
    work[tail:] = 0xA5
    bins = L.ls_bins(cap, tile_of.data_ptr(), item.data_ptr(), b.range.data_ptr(), b.count.data_ptr(), wp)
    L.ls_bin_sort(b.h, b.proj, bins, L.C.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert b.count.cpu().tolist() == [min(n, cap), int(n > cap), n, 0]
    assert bool((tile_of[cap:] == -7).all()) and bool((item[cap:] == -7).all())
    assert bool((work[tail:] == 0xA5).all())
    if cap == n:
        np.testing.assert_array_equal(tile_of[:n].cpu().numpy(), ref.tile_of[:n].cpu().numpy())
        np.testing.assert_array_equal(item[:n].cpu().numpy(), ref.item[:n].cpu().numpy())
        return
    b._alloc_bins(int(b.count[2].item()))
    b.bin_sort()
    assert int(b.count[1].item()) == 0 and b.instances() == n
    np.testing.assert_array_equal(b.tile_of[:n].cpu().numpy(), ref.tile_of[:n].cpu().numpy())
    np.testing.assert_array_equal(b.item[:n].cpu().numpy(), ref.item[:n].cpu().numpy())
    np.testing.assert_array_equal(b.range.cpu().numpy(), ref.range.cpu().numpy())


@pytest.mark.parametrize("compact", ["0", "1"])
def test_empty_and_fully_culled_renders(gpu, monkeypatch, compact):
    monkeypatch.setenv("LS_COMPACT", compact)
    s = synth.scene_small(0, n=500)
    behind = {k: v.copy() for k, v in s["gauss"].items()}
    behind["mean"][2] = -np.abs(behind["mean"][2])  # every Gaussian behind the camera
    empty = {k: v[..., :0].copy() for k, v in s["gauss"].items()}
    jobs = [(s["gauss"], s["cam"], s["w2c"]), (behind, s["cam"], s["w2c"]), (empty, synth.camera(50, 50, 8, 8, 17, 9),
                                                                          s["w2c"])]
    b = _batch(jobs)
    b.project()
    b.bin_sort()
    b.render_fwd([0.5, 0.25, 0.125])
    for r in (1, 2):
        v = b.image_views(r)
        assert float(v["alpha"].abs().max()) == 0.0
        assert float(v["T_final"].min()) == 1.0
        np.testing.assert_array_equal(v["rgb"].cpu().numpy()[:, 0, 0], np.float32([0.5, 0.25, 0.125]))
    assert int(b.tiles[int(b.item_off[1]):int(b.item_off[2])].sum()) == 0
    _, _, o = U.oracle_render(s["gauss"], s["cam"], s["w2c"], bg=[0.5, 0.25, 0.125])
    ok = o["margin"] >= 2e-4
    assert U.image_close(b.image_views(0)["rgb"].cpu().numpy(), o["rgb"].detach().numpy(), ok[None]) == 0


def test_autograd_function_matches_direct_calls(gpu):
    from paper_2408_10154_amd.render import render

    s = synth.scene_small(0, n=1200)
    jobs = [(s["gauss"], s["cam"], s["w2c"])]
    b = _batch(jobs)
    pose = torch.as_tensor(s["target_pose"][None], device="cuda").clone().requires_grad_(True)
    for t in b.gsets[0].tensors():
        t.requires_grad_(True)
    rgb, depth, alpha = render(b, pose)
    rng = np.random.default_rng(2)
    w = [torch.as_tensor(rng.normal(size=x.shape).astype(np.float32), device="cuda") for x in (rgb, depth, alpha)]
    ((rgb * w[0]).sum() + (depth * w[1]).sum() + (alpha * w[2]).sum()).backward()
    g_auto = [t.grad.clone() for t in b.gsets[0].tensors()] + [pose.grad.clone()]
    b2, _, grads, pose_grad = None, None, None, None
    b2 = _batch(jobs)
    pose2 = torch.as_tensor(s["target_pose"][None], device="cuda")
    b2.project(pose2)
    b2.bin_sort()
    b2.render_fwd()
    grads = [b2.gsets[0].zeros_like()]
    pose_grad = torch.zeros_like(pose2)
    b2.render_bwd(up_rgb=w[0], up_depth=w[1], up_alpha=w[2], grads=grads, pose=pose2, pose_grad=pose_grad)
    g_direct = grads[0].tensors() + [pose_grad]
    for a, c in zip(g_auto, g_direct):
        assert U.rel_err(a.cpu().numpy(), c.cpu().numpy()) < 1e-5
    assert math.isfinite(float(rgb.sum()))


def test_small_workload_full_step_matches_oracle(gpu):
    """The plain single-view workload exactly as configured (4,096 Gaussians,
    160x120, f = 150): render at the identity pose, L1 loss against the render
    at the 2 deg / 3 cm perturbed pose (the same FP32 target on both sides),
    backward through the loss to every Gaussian parameter and the pose; all
    80 tiles against the FP64 oracle."""
    sc = synth.scene_small(0)
    cam, w2c = sc["cam"], sc["w2c"]
    b = _batch([(sc["gauss"], cam, w2c)])
    b.project(torch.as_tensor(sc["target_pose"][None], device="cuda"))
    b.bin_sort()
    b.render_fwd()
    tgt_rgb, tgt_depth = b.rgb.clone(), b.depth.clone()
    pose_np = synth.identity_pose()
    pose = torch.as_tensor(pose_np[None], device="cuda").contiguous()
    b.project(pose)
    b.bin_sort()
    b.render_fwd()
    loss, g_rgb, g_depth, g_scale = b.loss_l1(tgt_rgb, tgt_depth)
    grads = [b.gsets[0].zeros_like()]
    pose_grad = torch.zeros_like(pose)
    b.render_bwd(up_rgb=g_rgb, up_depth=g_depth, scale=g_scale, grads=grads, pose=pose, pose_grad=pose_grad)
    torch.cuda.synchronize()
    g, pt, o = U.oracle_render(sc["gauss"], cam, w2c, pose_np, requires_grad=True)
    H, W = cam["height"], cam["width"]
    ok = o["margin"] >= 2e-4
    assert ok.mean() > 0.99
    v = b.image_views(0)
    for key in ("rgb", "depth", "alpha"):
        mask = ok[None] if key == "rgb" else ok
        assert U.image_close(v[key].cpu().numpy(), o[key].detach().numpy(), mask) == 0, key
    t_rgb = torch.as_tensor(tgt_rgb.cpu().numpy().reshape(3, H, W), dtype=F64)
    t_dep = torch.as_tensor(tgt_depth.cpu().numpy().reshape(H, W), dtype=F64)
    ref = R.loss_l1(o["rgb"], o["depth"], t_rgb, t_dep)
    np.testing.assert_allclose(loss[0].item(), ref.item(), rtol=1e-4)
    ref.backward()
    valid = (t_dep.numpy() > 0).astype(np.float64)
    signs = [(g_rgb.cpu().numpy().reshape(3, H, W), (o["rgb"].detach().numpy() - t_rgb.numpy()) * valid[None]),
             (g_depth.cpu().numpy().reshape(H, W), (o["depth"].detach().numpy() - t_dep.numpy()) * valid)]
    excl = U.render_flips(b, 0, o, len(sc["gauss"]["opacity_logit"]), sign_pairs=signs)
    pairs = []
    for name in ("mean", "log_scale", "quat", "opacity_logit", "rgb"):
        got = getattr(grads[0], name).cpu().numpy()
        pairs.append((name, got.T if got.ndim == 2 else got, g[name].grad.numpy()))
    print(U.check_gradients(pairs, excl, f"4096-Gaussian step (excluded {int(excl.sum())})"))
    print(U.check_gradients([("pose", pose_grad[0].cpu().numpy()[None], pt.grad.numpy()[None])], None, "step"))


def test_render_loop_workload_sampled_tiles_match_oracle(gpu):
    """The render-loop workload at its full size (200k Gaussians, 1200x680,
    1.6 M tile instances), run through the same calls and kernels the bench
    times, checked on 96 tiles spread over the image: the forward images and
    n_last there, and the Gaussian and pose gradients of a loss whose
    upstream gradients are zero outside those tiles (so both sides see the
    same pixels), against the FP64 oracle restricted to the same tiles."""
    sc = synth.scene_room_volume(seed=1, n=200000)
    cam, w2c, pose_np = sc["cam"], sc["w2c"], sc["target_pose"]
    jobs = [(sc["gauss"], cam, w2c)]
    b = _batch(jobs)
    W, H = cam["width"], cam["height"]
    tx, ty = (W + 15) // 16, (H + 15) // 16
    sub = np.linspace(0, tx * ty - 1, 96).round().astype(int)
    sel = np.zeros((H, W), bool)
    for t in sub:
        y0, x0 = (t // tx) * 16, (t % tx) * 16
        sel[y0:y0 + 16, x0:x0 + 16] = True
    rng = np.random.default_rng(21)
    up = synth.random_image_grads(rng, b.P)
    up_rgb = (up["rgb"].reshape(3, H, W) * sel).astype(np.float32)
    up_d = (up["depth"].reshape(H, W) * sel).astype(np.float32)
    up_a = (up["alpha"].reshape(H, W) * sel).astype(np.float32)
    dev = lambda x: torch.as_tensor(np.ascontiguousarray(x).reshape(-1), device="cuda")  # noqa: E731
    pose = torch.as_tensor(pose_np[None], device="cuda").contiguous()
    b.project(pose)
    b.bin_sort()
    assert b.instances() > 1_000_000 and int(b.count[1].item()) == 0
    b.render_fwd()
    grads = [b.gsets[0].zeros_like()]
    pose_grad = torch.zeros_like(pose)
    b.render_bwd(up_rgb=dev(up_rgb), up_depth=dev(up_d), up_alpha=dev(up_a), grads=grads, pose=pose,
                 pose_grad=pose_grad)
    torch.cuda.synchronize()
    g, pt, o = U.oracle_render(sc["gauss"], cam, w2c, pose_np, requires_grad=True, tiles_subset=sub)
    v = b.image_views(0)
    ok = sel & (o["margin"] >= 1e-5)
    assert ok.sum() > 0.95 * sel.sum()
    for key in ("rgb", "depth", "alpha"):
        mask = ok[None] if key == "rgb" else ok
        assert U.image_close(v[key].cpu().numpy(), o[key].detach().numpy(), mask) == 0, key
    np.testing.assert_array_equal(v["n_last"].cpu().numpy()[ok], o["n_last"][ok])
    f64 = lambda a: torch.as_tensor(a, dtype=F64)  # noqa: E731
    ((o["rgb"] * f64(up_rgb)).sum() + (o["depth"] * f64(up_d)).sum() + (o["alpha"] * f64(up_a)).sum()).backward()
    # decision flips only count inside the sampled tiles (the oracle left the rest at background)
    vv = {k: t.cpu().numpy() for k, t in v.items()}
    for k in ("rgb", "depth", "alpha", "n_last"):
        ora = o[k] if k == "n_last" else o[k].detach().numpy()
        vv[k] = np.where(sel[None] if k == "rgb" else sel, vv[k], ora)
    excl, flip = U.decision_flips(o, vv, 200000, b.radius.cpu().numpy())
    flip &= sel
    assert flip.sum() <= 1e-3 * sel.sum() and np.all(np.asarray(o["margin"])[flip] < 1e-3)
    pairs = []
    for name in ("mean", "log_scale", "quat", "opacity_logit", "rgb"):
        got = getattr(grads[0], name).cpu().numpy()
        pairs.append((name, got.T if got.ndim == 2 else got, g[name].grad.numpy()))
    print(U.check_gradients(pairs, excl, f"render loop, 96 tiles (flipped px {int(flip.sum())}, "
                                         f"excluded {int(excl.sum())})"))
    print(U.check_gradients([("pose", pose_grad[0].cpu().numpy()[None], pt.grad.numpy()[None])], None, "loop"))


def test_pose_only_backward_matches_full_and_is_bitwise_repeatable(gpu):
    """The pose-only backward (pose Jacobian applied per tile, fixed-order
    reduction, no atomics) gives the full backward's pose gradient and the
    same bits on every run."""
    jobs, poses = _three_scenes()
    b = _batch(jobs)
    rng = np.random.default_rng(4)
    up = synth.random_image_grads(rng, b.P)
    dev = lambda x: torch.as_tensor(x, device="cuda")  # noqa: E731
    pose = torch.as_tensor(np.stack(poses), device="cuda")
    b.project(pose)
    b.bin_sort()
    b.render_fwd()
    kw = dict(up_rgb=dev(up["rgb"].reshape(-1)), up_depth=dev(up["depth"]), up_alpha=dev(up["alpha"]), pose=pose)
    full = torch.zeros_like(pose)
    b.render_bwd(grads=[gs.zeros_like() for gs in b.gsets], pose_grad=full, **kw)
    runs = []
    for _ in range(2):
        pg = torch.zeros_like(pose)
        b.render_bwd(grads=None, pose_grad=pg, **kw)
        runs.append(pg.cpu().numpy())
    np.testing.assert_array_equal(runs[0], runs[1])
    for r in range(len(jobs)):
        assert U.rel_err(runs[0][r], full[r].cpu().numpy()) < 1e-4


@pytest.mark.parametrize("pose_only", [False, True])
def test_persistent_backward_matches_plain(gpu, monkeypatch, pose_only):
    """The persistent backward kernels (tiles claimed from device queues; the
    library picks them for launches with many tiles per resident block) give
    what the one-block-per-tile kernels give: the pose-only gradient bit for
    bit (per-tile partials, fixed-order reduction), the full-mode Gaussian
    gradients to float-atomic ordering.  Each form runs twice, so the second
    persistent launch also checks that the queues were left at zero."""
    jobs, poses = _three_scenes()
    b = _batch(jobs)
    rng = np.random.default_rng(9)
    up = synth.random_image_grads(rng, b.P)
    dev = lambda x: torch.as_tensor(x, device="cuda")  # noqa: E731
    pose = torch.as_tensor(np.stack(poses), device="cuda")
    b.project(pose)
    b.bin_sort()
    b.render_fwd()
    kw = dict(up_rgb=dev(up["rgb"].reshape(-1)), up_depth=dev(up["depth"]), up_alpha=dev(up["alpha"]), pose=pose)
    out = {}
    for mode in ("0", "1", "1", "0"):
        monkeypatch.setenv("LS_PERSISTENT", mode)
        pg = torch.zeros_like(pose)
        grads = None if pose_only else [gs.zeros_like() for gs in b.gsets]
        b.render_bwd(grads=grads, pose_grad=pg, **kw)
        torch.cuda.synchronize()
        res = [pg.cpu().numpy()] + ([] if pose_only else [t.cpu().numpy() for g in grads for t in g.tensors()])
        out.setdefault(mode, []).append(res)
    plain, pers = out["0"][0], out["1"][0]
    if pose_only:
        for mode in ("0", "1"):  # each form repeats itself bit for bit
            np.testing.assert_array_equal(out[mode][0][0], out[mode][1][0])
        np.testing.assert_array_equal(plain[0], pers[0])
    else:
        for mode in ("0", "1"):
            for x, y in zip(out[mode][0], out[mode][1]):
                assert U.rel_err(x, y) < 1e-5
        for x, y in zip(pers, plain):
            assert U.rel_err(x, y) < 1e-5


@pytest.mark.parametrize("lambda_c,inlier_k,alpha_power", [(0.6, 50.0, 3), (0.3, 0.0, 0), (1.0, 2.0, 1)])
def test_loss_tracking_matches_oracle(gpu, lambda_c, inlier_k, alpha_power):
    """Masked tracking loss on identical FP32 inputs: the median depth error of
    every render bit-exact (exact selection, ties included), the loss within
    1e-5 and the image gradients within 1e-5 of the FP64 oracle.  Renders:
    640x480 (many blocks), 100x70, 33x17 (ragged), 5x3 with one valid pixel
    and 33x17 with none."""
    sizes = [(640, 480), (100, 70), (33, 17), (5, 3), (33, 17)]
    jobs = []
    for k, (w, h) in enumerate(sizes):
        sc = synth.scene_tiny(40 + k, 50, w, h, 0.8 * w)
        jobs.append((sc["gauss"], sc["cam"], sc["w2c"]))
    b = _batch(jobs)
    rng = np.random.default_rng(11)
    pr = rng.random(3 * b.P).astype(np.float32)
    tr = rng.random(3 * b.P).astype(np.float32)
    td = np.where(rng.random(b.P) < 0.2, 0.0, rng.random(b.P) * 3 + 0.5).astype(np.float32)
    # depth errors on a coarse grid (many exact ties), a few gross outliers
    off = (np.round(rng.normal(0.0, 4.0, b.P)) * 0.01).astype(np.float32)
    off[rng.random(b.P) < 0.02] = 5.0
    pdp = (td + off).astype(np.float32)
    al = rng.random(b.P).astype(np.float32)
    o3, o4, o5 = (int(b.pix_off[i]) for i in (3, 4, 5))
    td[o3:o4] = 0.0
    td[o3 + 7] = 1.25                                     # one valid pixel
    td[o4:o5] = 0.0                                       # none
    pr[:5] = tr[:5]                                       # sign(0) = 0
    dev = lambda a: torch.as_tensor(a, device="cuda")     # noqa: E731
    loss, med, g_rgb, g_depth, scale = b.loss_tracking(dev(tr), dev(td), lambda_c, inlier_k, alpha_power,
                                                       pred=(dev(pr), dev(pdp), dev(al)))
    torch.cuda.synchronize()
    for r, (_, cam, _) in enumerate(jobs):
        H, W = cam["height"], cam["width"]
        p0 = int(b.pix_off[r])
        sl, sl3 = slice(p0, p0 + H * W), slice(3 * p0, 3 * p0 + 3 * H * W)
        prr = torch.as_tensor(pr[sl3].reshape(3, H, W), dtype=F64).requires_grad_(True)
        pdd = torch.as_tensor(pdp[sl].reshape(H, W), dtype=F64).requires_grad_(True)
        ref, ref_med = R.loss_tracking(prr, pdd, torch.as_tensor(al[sl].reshape(H, W), dtype=F64),
                                       torch.as_tensor(tr[sl3].reshape(3, H, W), dtype=F64),
                                       torch.as_tensor(td[sl].reshape(H, W), dtype=F64),
                                       lambda_c=lambda_c, alpha_power=alpha_power, inlier_k=inlier_k)
        if inlier_k > 0:
            assert np.float32(med[r].item()) == np.float32(ref_med), (r, med[r].item(), ref_med)
        np.testing.assert_allclose(loss[r].item(), ref.item(), rtol=1e-5, atol=1e-12)
        n = int((td[sl] > 0).sum())
        if n == 0:
            assert scale[r].item() == 0.0 and loss[r].item() == 0.0
            continue
        np.testing.assert_allclose(scale[r].item(), 1.0 / n, rtol=1e-6)
        ref.backward()
        sc = scale[r].item()
        np.testing.assert_allclose(g_rgb[sl3].cpu().numpy() * sc, prr.grad.numpy().reshape(-1), rtol=1e-5, atol=1e-12)
        np.testing.assert_allclose(g_depth[sl].cpu().numpy() * sc, pdd.grad.numpy().reshape(-1), rtol=1e-5,
                                   atol=1e-12)
    # a second call on the same batch (workspace left zeroed) gives the same result
    loss2, med2, *_ = b.loss_tracking(dev(tr), dev(td), lambda_c, inlier_k, alpha_power,
                                      pred=(dev(pr), dev(pdp), dev(al)))
    assert torch.equal(loss, loss2) and (inlier_k <= 0 or torch.equal(med, med2))


def test_gpu_gradients_match_gpu_finite_differences(gpu):
    """FP32 check of the backward against the forward alone (no oracle): for
    L = sum w . image with smooth weights, single components of every
    parameter group (Gaussian mean, log-scale, quaternion, opacity logit,
    colour; the pose) are moved by +-h and the central difference of the
    GPU's own FP32 forward (L summed in FP64, the step taken as the FP32
    difference of the two parameter values) must equal the GPU gradient
    within 1e-2.  Samples are components whose gradient is at least 0.1 of
    the group's largest, and a sample is rejected when any discrete decision
    differs between the base point and either side of the step: radius or
    tile count of any Gaussian, the stop position of any pixel, or the number
    of composited entries (an alpha-skip decision), or when the differences
    at h and h/2 disagree by more than 0.5 % (a flip that leaves the counts
    unchanged).  A pose step moves every Gaussian and flips some decision of
    a dense scene at any step that FP32 can resolve, so the pose (and the
    means and scales of that scene) is checked on three broad Gaussians that
    take no decision anywhere in the image, at h = 1e-3."""
    for n, groups in ((800, dict(mean=[1e-4], log_scale=[1e-4], quat=[1e-4], opacity_logit=[1e-4], rgb=[1e-3])),
                      (3, dict(pose=[1e-3], mean=[1e-3], log_scale=[1e-3]))):
        sc = synth.scene_small(0, n=n)
        if n == 3:
            # three broad Gaussians (sigma ~ 0.8 m at 2-3 m, opacity 0.5) whose alpha stays between 1/255
            # and 0.99 over the whole image and whose transmittance never reaches 1e-4: no decision exists
            # for a step to flip, so the pose is checked at the survey's h = 1e-3
            g = sc["gauss"]
            g["mean"] = np.array([[0.05, -0.1, 0.08], [0.02, 0.06, -0.05], [2.0, 2.5, 3.0]], np.float32)
            g["log_scale"] = np.log(np.array([[0.8, 0.9, 1.0], [0.7, 0.85, 0.95], [0.75, 0.8, 1.1]], np.float32))
            g["opacity_logit"] = np.zeros(3, np.float32)
        cam, w2c = sc["cam"], sc["w2c"]
        b = _batch([(sc["gauss"], cam, w2c)])
        H, W = cam["height"], cam["width"]
        yy, xx = np.mgrid[0:H, 0:W]
        field = 1.0 + 0.5 * np.sin(xx / 23.0) * np.cos(yy / 17.0)
        w_rgb = torch.as_tensor(np.stack([field, 0.8 * field, 1.2 * field]).reshape(-1), device="cuda")
        w_dep = torch.as_tensor((0.3 * field).reshape(-1), device="cuda")
        gs = b.gsets[0]
        pose = torch.as_tensor(sc["target_pose"][None], device="cuda").contiguous()

        def forward():
            b.project(pose)
            b.bin_sort()
            b.render_fwd()
            val = float((b.rgb.double() * w_rgb).sum() + (b.depth.double() * w_dep).sum())
            dec = (b.radius.cpu().numpy().tobytes(), b.tiles.cpu().numpy().tobytes(),
                   b.n_last.cpu().numpy().tobytes(), b.render_stats())
            return val, dec

        _, dec0 = forward()
        grads = [gs.zeros_like()]
        pose_grad = torch.zeros_like(pose)
        b.render_bwd(up_rgb=w_rgb.float(), up_depth=w_dep.float(), grads=grads, pose=pose, pose_grad=pose_grad)
        torch.cuda.synchronize()
        rng = np.random.default_rng(5)
        accepted = {}
        for name, hs in groups.items():
            param = pose[0] if name == "pose" else getattr(gs, name)
            grad = (pose_grad[0] if name == "pose" else getattr(grads[0], name)).cpu().numpy().astype(np.float64)
            flat = grad.reshape(-1)
            cand = np.nonzero(np.abs(flat) >= 0.1 * np.abs(flat).max())[0]
            accepted[name] = 0
            for idx in rng.choice(cand, size=min(len(cand), 8), replace=False):
                pv = param.view(-1)
                x0 = pv[idx].item()

                def central(h):
                    vals, xs, ok = [], [], True
                    for sgn in (1, -1):
                        pv[idx] = float(np.float32(x0 + sgn * h))
                        xs.append(pv[idx].item())
                        v, dec = forward()
                        vals.append(v)
                        ok &= dec == dec0
                    pv[idx] = x0
                    return (vals[0] - vals[1]) / (xs[0] - xs[1]), ok

                fd = None
                for h in hs:
                    f1, ok1 = central(h)
                    f2, ok2 = central(0.5 * h)
                    # two step sizes must agree: a decision that flips inside the step without changing
                    # the counted decisions (two contours crossing in opposite directions) gives a jump
                    # whose slope scales with 1/h
                    if ok1 and ok2 and abs(f1 - f2) <= 5e-3 * max(abs(f1), abs(f2)):
                        fd = f1
                        break
                if fd is None:
                    continue
                assert abs(fd - flat[idx]) <= 1e-2 * abs(flat[idx]), (name, int(idx), h, fd, flat[idx])
                accepted[name] += 1
        print(f"{n} Gaussians: accepted finite-difference samples per group:", accepted)
        assert all(v >= 3 for v in accepted.values()), accepted


@pytest.mark.parametrize("pose_only", [False, True])
@pytest.mark.parametrize("empty_render", [False, True])
def test_fused_l1_backward_matches_loss_then_backward(gpu, pose_only, empty_render):
    """ls_render_bwd_tiles_l1 (the Sec. 3.2 L1 gradient formed inside the
    compositing backward) against ls_loss_l1 + ls_render_bwd_tiles on three
    ragged renders whose targets lack depth on every seventh pixel (outside
    Omega): the same per-pixel gradients, so pose-only partials and pose
    gradients are bit-identical and full-mode Gaussian gradients agree to the
    float-atomic order; the tile-summed loss equals ls_loss_l1's to FP32
    rounding.  With empty_render the second render's targets have no depth
    at all (an empty Omega): its loss is exactly 0 on both paths and its pose
    gets no gradient."""
    jobs, poses = _three_scenes()
    pose = torch.as_tensor(np.stack(poses), device="cuda").contiguous()
    b = _batch(jobs)
    b.project(pose)
    b.bin_sort()
    b.render_fwd()
    tgt_rgb = (b.rgb * 0.9 + 0.05).contiguous()
    tgt_depth = (b.depth * 1.02).contiguous()
    tgt_depth[::7] = 0.0
    if empty_render:
        tgt_depth[int(b.pix_off[1]):int(b.pix_off[2])] = 0.0
    loss, g_rgb, g_depth, scale = b.loss_l1(tgt_rgb, tgt_depth)
    out = []
    for fused in (False, True):
        grads = None if pose_only else [g.zeros_like() for g in b.gsets]
        pg = torch.zeros_like(pose)
        if fused:
            b.render_bwd_tiles_l1(tgt_rgb, tgt_depth, scale, pose=pose, pose_only=pose_only)
            lt = b.loss_l1_tiles()
        else:
            b.render_bwd_tiles(up_rgb=g_rgb, up_depth=g_depth, scale=scale, pose=pose, pose_only=pose_only)
            lt = loss
        b.render_bwd_project(grads=grads, pose=pose, pose_grad=pg, pose_only=pose_only)
        torch.cuda.synchronize()
        out.append((grads, pg.cpu().numpy(), lt.cpu().numpy()))
    (ga, pa, la), (gf, pf, lf) = out
    np.testing.assert_allclose(lf, la, rtol=2e-6)
    if empty_render:
        assert la[1] == 0.0 and lf[1] == 0.0 and float(scale[1].item()) == 0.0
        assert (pf[1] == 0.0).all() and (pa[1] == 0.0).all()
        assert la[0] > 0 and la[2] > 0
    else:
        assert (la > 0).all()
    if pose_only:
        np.testing.assert_array_equal(pf, pa)
        return
    np.testing.assert_allclose(pf, pa, rtol=1e-4, atol=1e-5 * np.abs(pa).max())
    for x, y in zip(ga, gf):
        for n, ta, tf in zip(("mean", "log_scale", "quat", "opacity_logit", "rgb"), x.tensors(), y.tensors()):
            a_, f_ = ta.cpu().numpy(), tf.cpu().numpy()
            np.testing.assert_allclose(f_, a_, rtol=1e-4, atol=1e-5 * max(np.abs(a_).max(), 1e-30), err_msg=n)


@pytest.mark.parametrize("which", ["three_renders", "room_200k"])
def test_forward_cover_skip_is_bitwise_neutral(gpu, monkeypatch, which):
    """The forward stages an entry for a band by the pixels its alpha >= 1/255
    support reaches (per-row intervals) and skips it once all of those pixels
    have stopped.  Against LS_COVER=0 (the band rectangle test, every staged
    entry walked) the images, T_final and n_last are bit-identical, and so
    are the pose-only backward's gradients (deterministic, and it walks only
    the entries the forward marked as composited), on three ragged renders
    and on the 200k-Gaussian 1200x680 render-loop scene."""
    from paper_2408_10154_amd.render import GaussianSet, RenderBatch

    if which == "three_renders":
        jobs, poses = _three_scenes()
        b = _batch(jobs)
    else:
        s = synth.scene_room_volume(seed=1, n=200_000)
        b = RenderBatch([(GaussianSet.from_numpy(s["gauss"]), s["cam"], s["w2c"])], auto_grow=True)
        poses = [s["target_pose"]]
    pose = torch.as_tensor(np.stack(poses), device="cuda").contiguous()
    out = {}
    for mode in ("0", "1"):
        monkeypatch.setenv("LS_COVER", mode)
        b.project(pose)
        b.bin_sort()
        b.render_fwd()
        g = torch.Generator(device="cpu").manual_seed(3)
        up_rgb = torch.randn(b.rgb.numel(), generator=g).to("cuda")
        up_depth = torch.randn(b.depth.numel(), generator=g).to("cuda")
        pg = torch.zeros_like(pose)
        b.render_bwd(up_rgb=up_rgb, up_depth=up_depth, grads=None, pose=pose, pose_grad=pg)
        torch.cuda.synchronize()
        out[mode] = [t.cpu().numpy().copy() for t in (b.rgb, b.depth, b.alpha, b.T_final, b.n_last, pg)]
    for name, x0, x1 in zip(("rgb", "depth", "alpha", "T_final", "n_last", "pose_grad"), out["0"], out["1"]):
        np.testing.assert_array_equal(x1, x0, err_msg=name)
