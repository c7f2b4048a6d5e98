"""GPU opacity pruning (ls_prune_gaussians; supplement, submap update)
against the oracle.  Selection and compaction are integer decisions and
copies, so the bar is bit-exact: the kept index list, the count and every
compacted array."""

import numpy as np
import pytest
import torch

from oracle import prune as PR
from paper_2408_10154_amd import synth

pytestmark = pytest.mark.gpu


def _gauss(rng, n, tau=None):
    g = synth.gaussians_in_box(rng, n, (-1, -1, 1), (1, 1, 3))
    g["opacity_logit"] = rng.normal(0.0, 2.0, n).astype(np.float32)
    if tau is not None and n >= 8:
        w = g["opacity_logit"]
        w[: n // 50 + 1] = tau                                   # exactly at the threshold: kept
        w[n // 50 + 1: n // 25 + 2] = np.nextafter(tau, np.float32(-np.inf))  # one ulp below: pruned
        w[-3:] = [np.nan, np.inf, -np.inf]
        rng.shuffle(w)
    return g


@pytest.mark.parametrize("n", [0, 1, 1023, 1024, 1025, 200_003, 1_100_003])
@pytest.mark.parametrize("o_thre", [0.1, 0.5])
def test_prune_matches_oracle_bit_exact(gpu, n, o_thre):
    from paper_2408_10154_amd.render import GaussianSet, prune_gaussians

    rng = np.random.default_rng(n + int(o_thre * 10))
    g = _gauss(rng, n, PR.logit_threshold(o_thre))
    gs = GaussianSet.from_numpy(g)
    m = torch.as_tensor(rng.normal(size=(3, n)).astype(np.float32), device="cuda").contiguous()
    v = torch.as_tensor(rng.random(n).astype(np.float32), device="cuda").contiguous()
    out, kept, (m2, v2) = prune_gaussians(gs, o_thre, extra=(m, v))
    idx, ref = PR.prune(g, o_thre)
    np.testing.assert_array_equal(kept.cpu().numpy(), idx)
    for name in GaussianSet.FIELDS:
        np.testing.assert_array_equal(getattr(out, name).cpu().numpy(), ref[name])
    np.testing.assert_array_equal(m2.cpu().numpy(), m.cpu().numpy()[:, idx])
    np.testing.assert_array_equal(v2.cpu().numpy(), v.cpu().numpy()[idx])


@pytest.mark.parametrize("case", ["all_kept", "all_pruned"])
def test_prune_degenerate(gpu, case):
    from paper_2408_10154_amd.render import GaussianSet, prune_gaussians

    rng = np.random.default_rng(3)
    g = _gauss(rng, 5000)
    g["opacity_logit"][:] = 4.0 if case == "all_kept" else -4.0
    out, kept, _ = prune_gaussians(GaussianSet.from_numpy(g), 0.5)
    assert out.n == (5000 if case == "all_kept" else 0)
    if case == "all_kept":
        np.testing.assert_array_equal(kept.cpu().numpy(), np.arange(5000))
        np.testing.assert_array_equal(out.quat.cpu().numpy(), g["quat"])


def test_pruned_submap_renders_like_the_oracle_submap(gpu):
    """After pruning, the kept set is an ordinary Gaussian set: rendering it
    on the GPU equals rendering the oracle's pruned arrays on the GPU bit for
    bit (the same inputs reach the rasterizer)."""
    from paper_2408_10154_amd.render import GaussianSet, RenderBatch, prune_gaussians

    sc = synth.scene_small(0, n=4096)
    gs = GaussianSet.from_numpy(sc["gauss"])
    out, _, _ = prune_gaussians(gs, 0.5)
    _, ref = PR.prune(sc["gauss"], 0.5)
    imgs = []
    for g in (out, GaussianSet.from_numpy(ref)):
        b = RenderBatch([(g, sc["cam"], sc["w2c"])])
        b.project()
        b.bin_sort()
        b.render_fwd()
        imgs.append(b.rgb.cpu().numpy())
    np.testing.assert_array_equal(imgs[0], imgs[1])
