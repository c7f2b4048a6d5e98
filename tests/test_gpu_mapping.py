"""GPU parity of the mapping loss (ls_loss_mapping, ls_loss_isotropic;
Sec. 3.1 Eq. 3-5) against the FP64 oracle.  Bars: loss values within 1e-5
relative (1e-6 absolute); image gradients within 1e-3 of the reference, both
as the L2 relative error and as the largest deviation over the largest
reference entry; the depth gradient (a weighted sign) exactly; Gaussian
gradients through the rasterizer within 1e-3 (L2 relative per parameter
group, and element-wise away from flipped decisions)."""

import numpy as np
import pytest
import torch

from oracle import mapping as M
from oracle import raster as R
from paper_2408_10154_amd import synth
from tests import _util as U

pytestmark = pytest.mark.gpu

F64 = torch.float64


def _batch(jobs_np):
    from paper_2408_10154_amd.render import GaussianSet, RenderBatch

    b = RenderBatch([(GaussianSet.from_numpy(g), cam, w2c) for g, cam, w2c in jobs_np])
    b.sizes = [(cam["height"], cam["width"]) for _, cam, _ in jobs_np]  # (H, W) per render, for the checks
    return b


def _grad_close(got, ref, tol=1e-3):
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    assert U.rel_err(got, ref) < tol
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()


def _images(b, rng):
    """Per render: 0 uniform noise; 1 a smooth low-contrast image against a
    shifted copy (the cancellation-prone case of the variance terms); 2 a
    shaded pattern with noise and no pixel with a target depth."""
    pr = np.zeros(3 * b.P, np.float32)
    tr = np.zeros(3 * b.P, np.float32)
    pdp = (rng.random(b.P) * 3 + 0.5).astype(np.float32)
    td = np.where(rng.random(b.P) < 0.2, 0.0, rng.random(b.P) * 3 + 0.5).astype(np.float32)
    for r in range(b.R):
        H, W = b.sizes[r]
        p0, n = int(b.pix_off[r]), H * W
        if r % 3 == 0:
            x = rng.random((3, H, W))
            y = rng.random((3, H, W))
        elif r % 3 == 1:
            x = 0.5 + 0.01 * rng.normal(size=(3, H, W))
            y = x + 0.02 + 0.005 * rng.normal(size=(3, H, W))
        else:
            yy, xx = np.mgrid[0:H, 0:W]
            base = 0.5 + 0.3 * np.sin(xx / 13.0)[None] * np.cos(yy / 7.0)[None]
            x = np.clip(base + 0.03 * rng.normal(size=(3, H, W)), 0, 1)
            y = np.clip(base + 0.05 + 0.03 * rng.normal(size=(3, H, W)), 0, 1)
            td[p0:p0 + n] = 0.0
        pr[3 * p0:3 * p0 + 3 * n] = x.reshape(-1)
        tr[3 * p0:3 * p0 + 3 * n] = y.reshape(-1)
    pr[:5] = tr[:5]  # exact ties: sign(0) = 0
    return pr, pdp, tr, td


def _oracle_render_loss(b, r, pr, pdp, tr, td, lam):
    H, W = b.sizes[r]
    p0, n = int(b.pix_off[r]), H * W
    x = torch.as_tensor(pr[3 * p0:3 * p0 + 3 * n].reshape(3, H, W), dtype=F64).requires_grad_(True)
    d = torch.as_tensor(pdp[p0:p0 + n].reshape(H, W), dtype=F64).requires_grad_(True)
    loss = M.loss_mapping(x, d, tr[3 * p0:3 * p0 + 3 * n].reshape(3, H, W).astype(np.float64),
                          td[p0:p0 + n].reshape(H, W).astype(np.float64), *lam)
    gx, gd = torch.autograd.grad(loss, [x, d], allow_unused=True)
    gd = torch.zeros_like(d) if gd is None else gd
    return loss.item(), gx.numpy().reshape(-1), gd.numpy().reshape(-1)


@pytest.mark.parametrize("lam", [(0.2, 1.0, 1.0), (0.6, 0.8, 0.3)])
def test_mapping_loss_matches_oracle(gpu, lam):
    """Three renders of different sizes in one batch (160x120, 100x70 and a
    33x17 one smaller than a tile, both ragged against the 32x32 tiling);
    the last render has no target depth, so only its SSIM term is left."""
    a = synth.scene_small(0, n=200)
    bb = synth.scene_tiny(5, 100, 100, 70, 90.0)
    c = synth.scene_tiny(6, 50, 33, 17, 30.0)
    b = _batch([(s["gauss"], s["cam"], s["w2c"]) for s in (a, bb, c)])
    pr, pdp, tr, td = _images(b, np.random.default_rng(11))
    b.rgb.copy_(torch.as_tensor(pr))
    b.depth.copy_(torch.as_tensor(pdp))
    loss, g_rgb, g_depth, g_scale = b.loss_mapping(torch.as_tensor(tr, device="cuda"),
                                                   torch.as_tensor(td, device="cuda"), *lam)
    torch.cuda.synchronize()
    assert torch.all(g_scale == 1.0)
    for r in range(b.R):
        H, W = b.sizes[r]
        p0, n = int(b.pix_off[r]), H * W
        ref, gx, gd = _oracle_render_loss(b, r, pr, pdp, tr, td, lam)
        np.testing.assert_allclose(loss[r].item(), ref, rtol=1e-5, atol=1e-6)
        _grad_close(g_rgb[3 * p0:3 * p0 + 3 * n].cpu().numpy(), gx)
        np.testing.assert_allclose(g_depth[p0:p0 + n].cpu().numpy(), gd, rtol=1e-6, atol=0)


def test_mapping_loss_without_ssim_is_the_l1_loss_bitwise(gpu):
    """lambda_ssim = 0, unit weights: the colour and depth gradients equal the
    L1 loss's sign gradients times its scale, bit for bit (same count, same
    reciprocal)."""
    a = synth.scene_small(0, n=200)
    c = synth.scene_tiny(6, 50, 33, 17, 30.0)
    b = _batch([(s["gauss"], s["cam"], s["w2c"]) for s in (a, c)])
    pr, pdp, tr, td = _images(b, np.random.default_rng(12))
    b.rgb.copy_(torch.as_tensor(pr))
    b.depth.copy_(torch.as_tensor(pdp))
    trd, tdd = torch.as_tensor(tr, device="cuda"), torch.as_tensor(td, device="cuda")
    l_m, gr_m, gd_m, _ = b.loss_mapping(trd, tdd, 0.0, 1.0, 1.0)
    l_1, gr_1, gd_1, sc = b.loss_l1(trd, tdd)
    torch.cuda.synchronize()
    for r in range(b.R):
        H, W = b.sizes[r]
        p0, n = int(b.pix_off[r]), H * W
        s = sc[r]
        assert torch.equal(gr_m[3 * p0:3 * p0 + 3 * n], gr_1[3 * p0:3 * p0 + 3 * n] * s)
        assert torch.equal(gd_m[p0:p0 + n], gd_1[p0:p0 + n] * s)
        np.testing.assert_allclose(l_m[r].item(), l_1[r].item(), rtol=1e-6)


def test_mapping_loss_render_loop_size_matches_oracle(gpu):
    """The render-loop workload's images at full size (200k Gaussians,
    1200x680): the render at the identity pose against the render at the
    perturbed pose, every pixel and channel against the FP64 oracle."""
    sc = synth.scene_room_volume(seed=1, n=200000)
    cam, w2c = sc["cam"], sc["w2c"]
    b = _batch([(sc["gauss"], cam, w2c)])
    b.project(torch.as_tensor(sc["target_pose"][None], device="cuda"))
    b.bin_sort()
    b.render_fwd()
    tgt_rgb, tgt_depth = b.rgb.clone(), b.depth.clone()
    b.project(torch.as_tensor(synth.identity_pose()[None], device="cuda"))
    b.bin_sort()
    b.render_fwd()
    loss, g_rgb, g_depth, _ = b.loss_mapping(tgt_rgb, tgt_depth)
    torch.cuda.synchronize()
    pr, pdp = b.rgb.cpu().numpy(), b.depth.cpu().numpy()
    tr, td = tgt_rgb.cpu().numpy(), tgt_depth.cpu().numpy()
    assert (td > 0).mean() > 0.5
    ref, gx, gd = _oracle_render_loss(b, 0, pr, pdp, tr, td, (0.2, 1.0, 1.0))
    np.testing.assert_allclose(loss[0].item(), ref, rtol=1e-5, atol=1e-6)
    _grad_close(g_rgb.cpu().numpy(), gx)
    np.testing.assert_allclose(g_depth.cpu().numpy(), gd, rtol=1e-6, atol=0)


def test_small_workload_mapping_step_matches_oracle(gpu):
    """One mapping iteration of the 4,096-Gaussian 160x120 workload: render,
    mapping loss (L1 + SSIM colour, depth) plus the isotropic regulariser,
    backward to every Gaussian parameter, against the FP64 oracle."""
    from paper_2408_10154_amd.render import loss_isotropic

    sc = synth.scene_small(0)
    cam, w2c = sc["cam"], sc["w2c"]
    b = _batch([(sc["gauss"], cam, w2c)])
    b.project(torch.as_tensor(sc["target_pose"][None], device="cuda"))
    b.bin_sort()
    b.render_fwd()
    tgt_rgb, tgt_depth = b.rgb.clone(), b.depth.clone()
    b.project(None)
    b.bin_sort()
    b.render_fwd()
    loss, g_rgb, g_depth, g_scale = b.loss_mapping(tgt_rgb, tgt_depth)
    grads = [b.gsets[0].zeros_like()]
    b.render_bwd(up_rgb=g_rgb, up_depth=g_depth, scale=g_scale, grads=grads)
    reg = loss_isotropic(b.gsets[0].log_scale, 1.0, grad=grads[0].log_scale)
    torch.cuda.synchronize()
    g, _, o = U.oracle_render(sc["gauss"], cam, w2c, None, requires_grad=True)
    H, W = cam["height"], cam["width"]
    ref = M.loss_mapping(o["rgb"], o["depth"], tgt_rgb.cpu().numpy().reshape(3, H, W).astype(np.float64),
                         tgt_depth.cpu().numpy().reshape(H, W).astype(np.float64))
    ref_reg = M.loss_isotropic(g["log_scale"])
    np.testing.assert_allclose(loss[0].item(), ref.item(), rtol=1e-4)
    np.testing.assert_allclose(reg.item(), ref_reg.item(), rtol=1e-5)
    (ref + ref_reg).backward()
    # excluded from the element clause: Gaussians at flipped compositing
    # decisions, at pixels whose L1 residual is within FP32 reach of zero
    # (sign decided by rounding), and Gaussians whose scale sits within 1e-6
    # of its mean (the regulariser's sign decided by rounding)
    t_rgb = tgt_rgb.cpu().numpy().reshape(3, H, W).astype(np.float64)
    t_dep = tgt_depth.cpu().numpy().reshape(H, W).astype(np.float64)
    close = [(o["rgb"].detach().numpy() - t_rgb, 1e-5 * np.maximum(np.abs(t_rgb), 1.0)),
             (o["depth"].detach().numpy() - t_dep, 1e-5 * np.maximum(np.abs(t_dep), 1.0))]
    n = len(sc["gauss"]["opacity_logit"])
    excl = U.render_flips(b, 0, o, n, close_pairs=close)
    sc_ = np.exp(np.asarray(sc["gauss"]["log_scale"], np.float64).T)
    excl |= (np.abs(sc_ - sc_.mean(1, keepdims=True)).min(1) / sc_.mean(1)) < 1e-6
    pairs = []
    for name in ("mean", "log_scale", "quat", "opacity_logit", "rgb"):
        got = getattr(grads[0], name).cpu().numpy()
        pairs.append((name, got.T if got.ndim == 2 else got, g[name].grad.numpy()))
    print(U.check_gradients(pairs, excl, f"mapping step (excluded {int(excl.sum())} of {n})"))


@pytest.mark.parametrize("n", [0, 1, 5003, 200_003])
def test_isotropic_regulariser_matches_oracle(gpu, n):
    """Loss and accumulated gradient for n Gaussians (log-normal scales, some
    exactly isotropic); entries whose scale sits within 1e-6 of its mean,
    where FP32 rounding decides the sign, are left out of the element-wise
    check and counted."""
    from paper_2408_10154_amd.render import loss_isotropic

    rng = np.random.default_rng(n + 7)
    ls = rng.normal(np.log(0.02), 0.3, size=(3, n)).astype(np.float32)
    ls[:, : n // 50] = ls[0, : n // 50]  # isotropic: no loss, no gradient
    dev = torch.as_tensor(ls, device="cuda").contiguous()
    init = (rng.random((3, n)) * 1e-6).astype(np.float32)  # accumulated onto (same magnitude as the increments)
    grad = torch.as_tensor(init, device="cuda").contiguous()
    loss = loss_isotropic(dev, 0.7, grad=grad)
    torch.cuda.synchronize()
    x = torch.as_tensor(ls.T.astype(np.float64)).requires_grad_(True)
    ref = M.loss_isotropic(x, 0.7)
    if n == 0:
        assert loss.item() == 0.0
        return
    np.testing.assert_allclose(loss.item(), ref.item(), rtol=1e-5, atol=1e-9)
    (gref,) = torch.autograd.grad(ref, [x])
    s = np.exp(ls.T.astype(np.float64))
    d = np.abs(s - s.mean(1, keepdims=True)).min(1) / s.mean(1)
    keep = (d > 1e-6) | (d < 1e-12)  # the isotropic ones: equal scales, equal signs, no gradient
    assert (~keep).mean() < 1e-3
    got = (grad.cpu().numpy().astype(np.float64) - init.astype(np.float64)).T
    np.testing.assert_allclose(got[keep], gref.numpy()[keep], rtol=1e-4, atol=1e-6 * np.abs(gref.numpy()).max())
