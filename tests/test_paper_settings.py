"""The library's default settings against the values the paper prints
(tests/golden/supplement_hyperparameters.json, cited there).  CPU only."""

import json
import os

import pytest

from paper_2408_10154_amd import lib as L

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "supplement_hyperparameters.json")))
REAL = 1  # the real-data (TUM-RGBD) column, shared by ScanNet


def test_registration_defaults_are_the_real_data_loop_closure_column():
    from paper_2408_10154_amd.register import default_params

    lc, pd = GOLDEN["loop_closure"], GOLDEN["per_dataset"]
    p = default_params()
    assert p.lr_rot == pytest.approx(lc["lr_rotation"][REAL]) and p.lr_trans == pytest.approx(lc["lr_translation"][REAL])
    assert p.iters == pd["iters_tracking"][REAL]
    assert p.track.lambda_c == pytest.approx(pd["lambda_c"][REAL])
    assert p.track.inlier_k == GOLDEN["tracking_inlier_factor"] and p.track.alpha_power == 3
    assert p.exposure == 0 and p.lr_exposure == pytest.approx(lc["lr_exposure"][REAL])


def test_mapping_loss_weights_are_the_supplements():
    import inspect

    from oracle import mapping as M
    from paper_2408_10154_amd.render import RenderBatch

    w = GOLDEN["mapping_loss_weights"]
    sig = inspect.signature(RenderBatch.loss_mapping).parameters
    assert sig["lambda_color"].default == w["lambda_color"] and sig["lambda_depth"].default == w["lambda_depth"]
    osig = inspect.signature(M.loss_mapping).parameters
    assert osig["lambda_color"].default == w["lambda_color"] and osig["lambda_depth"].default == w["lambda_depth"]
    assert inspect.signature(M.loss_isotropic).parameters["lambda_reg"].default == w["lambda_reg"]


def test_bench_uses_the_real_data_settings():
    """The render loop's pose learning rates are the tracking column's, the
    overlap threshold the real-data tau_1, the exposure run the supplement's
    rate (through default_params)."""
    src = open(os.path.join(os.path.dirname(os.path.dirname(__file__)), "bench.py")).read()
    pd = GOLDEN["per_dataset"]
    assert f"{pd['lr_rotation_tracking'][REAL]:.0e}".replace("e-0", "e-") in src  # 2e-3
    assert "1e-2" in src and pd["lr_translation_tracking"][REAL] == 0.01
    assert f"overlap_ratio(p, q, T, {GOLDEN['overlap_tau_m']['real']}" in src


def test_golden_file_is_well_formed():
    for table in ("per_dataset", "loop_closure"):
        t = GOLDEN[table]
        assert all(len(v) == len(t["columns"]) for k, v in t.items() if k != "columns")
    assert L.ls_reg_params  # the binding exposes the struct the defaults fill
