"""Argument checks of the Python binding's helpers, which run before any
device call (CPU only)."""

import types

import numpy as np
import pytest
import torch

from paper_2408_10154_amd.render import adjust_submaps, loss_isotropic, overlap_ratio


def test_isotropic_needs_a_contiguous_3_by_n_device_tensor():
    with pytest.raises(ValueError):
        loss_isotropic(torch.zeros(3, 10))  # host tensor
    with pytest.raises(ValueError):
        loss_isotropic(torch.zeros(10, 3))


def test_overlap_needs_3_by_n_device_means():
    with pytest.raises(ValueError):
        overlap_ratio(torch.zeros(3, 5), torch.zeros(3, 4), np.eye(4), 0.1)
    with pytest.raises(ValueError):
        overlap_ratio(torch.zeros(5, 3), torch.zeros(3, 4), np.eye(4), 0.1)


def test_adjust_needs_device_pose_rows_of_twelve():
    g = types.SimpleNamespace(n=0, mean=torch.zeros(3, 0), quat=torch.zeros(4, 0))
    with pytest.raises(ValueError):
        adjust_submaps([(g, torch.zeros(2, 12), np.eye(4))])  # host poses
