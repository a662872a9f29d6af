"""Input generators: the torch phantom generator reproduces the numpy one."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from workloads import ellipse_phantom_params, phantom_cell_averages, phantom_cell_averages_torch


def test_torch_phantoms_equal_numpy():
    ps = [ellipse_phantom_params(s) for s in (50000, 50001, 70000)]
    a = np.stack([phantom_cell_averages(p, 6) for p in ps])
    b = phantom_cell_averages_torch(ps, 6, "cpu").numpy()
    assert np.max(np.abs(a - b)) <= 1e-15 * np.max(np.abs(a))
