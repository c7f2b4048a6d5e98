"""Pins of the FP64 mapping-loss oracle (Eq. 3-5, readings R26-R29) against
closed forms, brute-force window sums, special cases and finite differences.
CPU only."""

import math

import numpy as np
import pytest
import torch

from oracle import mapping as M
from oracle import raster as R

F64 = torch.float64


def _window_variance():
    """Sum_k g_k k^2 of the 11-tap window, from its definition."""
    g = [math.exp(-k * k / (2 * 1.5 ** 2)) for k in range(-5, 6)]
    return sum(w * k * k for w, k in zip(g, range(-5, 6))) / sum(g)


def test_window_is_the_normalised_gaussian():
    g = M.ssim_window().numpy()
    assert g.shape == (11,)
    assert abs(g.sum() - 1.0) < 1e-15
    np.testing.assert_allclose(g, g[::-1], rtol=0, atol=0)
    np.testing.assert_allclose(g[5] / g[4], math.exp(1 / (2 * 1.5 ** 2)), rtol=1e-14)
    np.testing.assert_allclose(g[5] / g[0], math.exp(25 / (2 * 1.5 ** 2)), rtol=1e-13)


def test_identical_images_give_one():
    rng = np.random.default_rng(0)
    x = torch.as_tensor(rng.uniform(size=(3, 19, 23)))
    np.testing.assert_allclose(M.ssim_map(x, x).numpy(), 1.0, atol=1e-12)


def test_constant_images_closed_form_interior_and_corner():
    """x = a, y = b everywhere.  At a pixel whose window keeps mass m inside
    the image, the zero-padded moments are mu = a m, var = a^2 (m - m^2),
    cov = a b (m - m^2); interior pixels have m = 1."""
    a, b = 0.7, 0.3
    x = torch.full((1, 24, 30), a, dtype=F64)
    y = torch.full((1, 24, 30), b, dtype=F64)
    s = M.ssim_map(x, y).numpy()[0]
    c1, c2 = 0.01 ** 2, 0.03 ** 2
    np.testing.assert_allclose(s[12, 15], (2 * a * b + c1) / (a * a + b * b + c1), rtol=1e-12)
    g = [math.exp(-k * k / (2 * 1.5 ** 2)) for k in range(-5, 6)]
    m = (sum(g[5:]) / sum(g)) ** 2  # corner: half the window along each axis
    v = m - m * m
    expect = ((2 * a * b * m * m + c1) * (2 * a * b * v + c2)) / (((a * a + b * b) * m * m + c1) *
                                                                ((a * a + b * b) * v + c2))
    np.testing.assert_allclose(s[0, 0], expect, rtol=1e-12)


@pytest.mark.parametrize("alpha,beta,c", [(0.02, 0.03, 0.1), (0.02, -0.01, 0.6), (0.01, 0.05, 0.0)])
def test_linear_ramps_closed_form(alpha, beta, c):
    """x = alpha j, y = beta j + c (j = column): at an interior pixel the
    symmetric window gives mu_x = alpha j, mu_y = beta j + c, var_x =
    alpha^2 v, var_y = beta^2 v, cov = alpha beta v with v = sum g_k k^2;
    this fixes both the luminance and the structure term, factors of 2
    included."""
    h, w = 20, 40
    j = np.arange(w, dtype=np.float64)
    x = torch.as_tensor(np.broadcast_to(alpha * j, (1, h, w)).copy())
    y = torch.as_tensor(np.broadcast_to(beta * j + c, (1, h, w)).copy())
    s = M.ssim_map(x, y).numpy()[0]
    v = _window_variance()
    c1, c2 = 0.01 ** 2, 0.03 ** 2
    for jj in (7, 20, 31):
        mx, my = alpha * jj, beta * jj + c
        expect = ((2 * mx * my + c1) * (2 * alpha * beta * v + c2)) / ((mx * mx + my * my + c1) *
                                                                      ((alpha ** 2 + beta ** 2) * v + c2))
        np.testing.assert_allclose(s[10, jj], expect, rtol=1e-10)


def test_brute_force_window_sums_including_borders():
    rng = np.random.default_rng(1)
    x = rng.uniform(size=(3, 9, 13))
    y = np.clip(x + rng.normal(scale=0.2, size=x.shape), 0, 1)
    s = M.ssim_map(torch.as_tensor(x), torch.as_tensor(y)).numpy()
    for ch, i, j in [(0, 0, 0), (1, 4, 6), (2, 8, 12), (0, 2, 11), (2, 7, 1)]:
        np.testing.assert_allclose(s[ch, i, j], M.ssim_brute_force(x, y, ch, i, j), rtol=1e-12)


def test_symmetric_and_bounded():
    rng = np.random.default_rng(2)
    x = torch.as_tensor(rng.uniform(size=(3, 17, 21)))
    y = torch.as_tensor(rng.uniform(size=(3, 17, 21)))
    a, b = M.ssim_map(x, y), M.ssim_map(y, x)
    np.testing.assert_allclose(a.numpy(), b.numpy(), rtol=1e-13)
    assert a.max() <= 1.0 and a.min() >= -1.0


def test_mapping_loss_without_ssim_is_the_l1_loss():
    rng = np.random.default_rng(3)
    rgb = torch.as_tensor(rng.uniform(size=(3, 12, 16)))
    dep = torch.as_tensor(rng.uniform(1, 3, size=(12, 16)))
    trgb = rng.uniform(size=(3, 12, 16))
    tdep = rng.uniform(1, 3, size=(12, 16))
    tdep[rng.uniform(size=tdep.shape) < 0.2] = 0.0
    a = M.loss_mapping(rgb, dep, trgb, tdep, lambda_ssim=0.0)
    b = R.loss_l1(rgb, dep, torch.as_tensor(trgb), torch.as_tensor(tdep))
    np.testing.assert_allclose(float(a), float(b), rtol=1e-14)
    # SSIM alone: lc = 1, ls = 1, ld = 0 -> 1 - mean SSIM
    c = M.loss_mapping(rgb, dep, trgb, tdep, lambda_ssim=1.0, lambda_depth=0.0)
    np.testing.assert_allclose(float(c), 1.0 - float(M.ssim_map(rgb, torch.as_tensor(trgb)).mean()), rtol=1e-14)


def test_mapping_loss_gradient_matches_finite_differences():
    rng = np.random.default_rng(4)
    h, w = 8, 10
    trgb = rng.uniform(0.2, 0.8, size=(3, h, w))
    tdep = rng.uniform(1, 3, size=(h, w))
    tdep[0, :3] = 0.0
    # keep every residual away from the L1 kink
    off = rng.choice([-1.0, 1.0], size=(3, h, w)) * rng.uniform(0.05, 0.15, size=(3, h, w))
    rgb = torch.as_tensor(trgb + off, dtype=F64).requires_grad_(True)
    dep = torch.as_tensor(tdep + rng.choice([-1.0, 1.0], size=(h, w)) * 0.1, dtype=F64).requires_grad_(True)
    loss = M.loss_mapping(rgb, dep, trgb, tdep, lambda_ssim=0.2, lambda_color=1.0, lambda_depth=0.7)
    g_rgb, g_dep = torch.autograd.grad(loss, [rgb, dep])
    eps = 1e-6
    base = rgb.detach().clone()
    for idx in [(0, 0, 0), (1, 3, 4), (2, 7, 9), (0, 5, 1), (2, 0, 9)]:
        p, m = base.clone(), base.clone()
        p[idx] += eps
        m[idx] -= eps
        fd = (float(M.loss_mapping(p, dep.detach(), trgb, tdep, 0.2, 1.0, 0.7)) -
              float(M.loss_mapping(m, dep.detach(), trgb, tdep, 0.2, 1.0, 0.7))) / (2 * eps)
        np.testing.assert_allclose(float(g_rgb[idx]), fd, rtol=1e-6, atol=1e-9)
    # depth: valid pixels get ld sign / |Omega|, the unmeasured ones nothing
    n = int((tdep > 0).sum())
    expect = 0.7 * np.sign(dep.detach().numpy() - tdep) * (tdep > 0) / n
    np.testing.assert_allclose(g_dep.numpy(), expect, rtol=1e-14, atol=0)


def test_isotropic_regulariser_closed_form_and_gradient():
    # scales (1, 2, 3): mean 2, |.|_1 = 2; an isotropic Gaussian adds 0
    ls = torch.as_tensor(np.log([[1.0, 2.0, 3.0], [0.5, 0.5, 0.5]]))
    np.testing.assert_allclose(float(M.loss_isotropic(ls)), 2.0 / 2, rtol=1e-14)
    np.testing.assert_allclose(float(M.loss_isotropic(ls, lambda_reg=3.0)), 3.0, rtol=1e-14)
    assert float(M.loss_isotropic(ls[1:])) == 0.0
    # d/d log s_j of sum_i |s_i - mean(s)| = s_j (sign(s_j - m) - mean_i sign(s_i - m))
    rng = np.random.default_rng(5)
    x = torch.as_tensor(rng.normal(np.log(0.02), 0.3, size=(6, 3))).requires_grad_(True)
    (g,) = torch.autograd.grad(M.loss_isotropic(x, 0.5), [x])
    s = np.exp(x.detach().numpy())
    sg = np.sign(s - s.mean(1, keepdims=True))
    expect = 0.5 / 6 * s * (sg - sg.mean(1, keepdims=True))
    np.testing.assert_allclose(g.numpy(), expect, rtol=1e-12, atol=1e-18)
    eps = 1e-7
    for idx in [(0, 0), (3, 2), (5, 1)]:
        p, m = x.detach().clone(), x.detach().clone()
        p[idx] += eps
        m[idx] -= eps
        fd = (float(M.loss_isotropic(p, 0.5)) - float(M.loss_isotropic(m, 0.5))) / (2 * eps)
        np.testing.assert_allclose(float(g[idx]), fd, rtol=1e-6)
