"""The seeded input recipes (CPU): shapes, determinism, value ranges and
load totals of the workloads that the parity tests and bench.py use."""

import numpy as np
import pytest

from workloads import batched_designs, load_top_traction, make_problem
from workloads.square_wall import density_gaussian_sum, four_load_cases


def test_recipes_are_deterministic():
    a, b = make_problem("wall64"), make_problem("wall64")
    np.testing.assert_array_equal(a.x, b.x)
    np.testing.assert_array_equal(density_gaussian_sum(48, 32, 7), density_gaussian_sum(48, 32, 7))
    assert not np.array_equal(density_gaussian_sum(48, 32, 7), density_gaussian_sum(48, 32, 8))


def test_wall64_shape_and_ranges():
    p = make_problem("wall64")
    assert p.x.shape == (64, 64, 3) and p.levels == 3 and not p.mixed
    s = p.x.sum(axis=2)
    assert np.all(p.x >= 0) and np.all(s <= 1 + 1e-12)
    assert 0.70 < s.mean() < 0.80


def test_wall1024_recipe_at_a_small_size():
    p = make_problem("wall1024", n=128, levels=4)
    assert p.x.shape == (128, 128, 3) and p.mixed
    assert np.all(p.x >= 0) and np.all(p.x.sum(axis=2) <= 1 + 1e-12)
    E = 1e-9 + np.sum(p.x ** 3 * (np.array([1.0, 0.6, 0.2]) - 1e-9), axis=2)
    assert 0.005 < E.min() and E.max() < 0.6


@pytest.mark.parametrize("nx,ny", [(8, 8), (12, 6)])
def test_loads_total_one(nx, ny):
    F = load_top_traction(nx, ny)
    assert F[..., 0].sum() == 0.0
    assert F[..., 1].sum() == pytest.approx(-1.0)
    assert np.all(F[:-1] == 0)
    for k, case in enumerate(four_load_cases(nx, ny)):
        assert case[..., 1].sum() == pytest.approx(-1.0)
        # nothing on the clamped row, except the left traction's share at
        # the clamped corner (carried by the support)
        row0 = case[0].copy()
        if k == 2:
            assert row0[0, 1] == pytest.approx(-0.5 / ny)
            row0[0, 1] = 0.0
        assert np.all(row0 == 0)


def test_batched_workload_layout():
    probs = batched_designs(per_size=1)
    assert [(p.nelx, p.levels) for p in probs] == [(128, 4), (384, 5), (768, 6)]
    assert all(p.F.shape == (4, p.nely + 1, p.nelx + 1, 2) for p in probs)
    assert all(p.nelx % 2 ** (p.levels - 1) == 0 and p.nelx >> (p.levels - 1) <= 32 for p in probs)


def test_binary_contrast_recipe():
    p = make_problem("wall256", n=64, levels=3)
    x = p.x
    assert x.shape == (64, 64, 3)
    assert set(np.unique(x)) <= {0.0, 1.0}
    s = x.sum(axis=2)
    assert np.all(s[0] == 1) and np.all(s[-1] == 1)         # loaded and clamped rows solid
    assert 0.4 < s[1:-1].mean() < 0.6                        # half of the rest
    assert p.fd_elements.shape == (64, 2) and p.fd_zero_pairs.shape == (8, 2)
    # FD pairs sit on solid elements, on their own phase
    e, k = p.fd_elements[:, 0], p.fd_elements[:, 1]
    assert np.all(x.reshape(-1, 3)[e, k] == 1.0)


def test_near_binary_recipe_spans_top_to_bottom():
    from scipy import ndimage
    p = make_problem("wall2048", n=128, levels=4)
    x = p.x
    assert x.shape == (128, 128, 4)
    assert set(np.round(np.unique(x), 6)) <= {1e-3, round(1 - 3e-3, 6)}
    solid = x.max(axis=2) > 0.5
    lab, _ = ndimage.label(solid)
    assert np.intersect1d(lab[0][lab[0] > 0], lab[-1][lab[-1] > 0]).size > 0
