"""Pins for the oracle's cone filters (Section 4, radius rf of Table 2).

Each check rests on something other than the filter's own formula:
hand-computed weights, preserved constants, the adjoint identity of the
chain rule, the identity at radius <= 1, and scipy.ndimage's correlation
as an independent implementation of the same weighted sums.
"""

import math

import numpy as np
import pytest
from scipy import ndimage

from oracle import cone_filter as cf

SHAPES = [(7, 5), (13, 9), (20, 3)]


def test_weights_by_hand():
    H = cf.cone_matrix(5, 5, 1.5)
    c = 2 * 5 + 2                      # element (2, 2)
    assert H[c, c] == 1.5
    assert H[c, c + 1] == pytest.approx(0.5, abs=1e-15)          # right neighbour, distance 1
    assert H[c, c + 5] == pytest.approx(0.5, abs=1e-15)          # upper neighbour
    assert H[c, c + 6] == pytest.approx(1.5 - math.sqrt(2.0), abs=1e-15)   # diagonal
    assert H[c, c + 2] == 0.0                                     # distance 2 > rf
    assert H[c].nnz == 9
    # a corner element keeps only its in-grid neighbours
    assert H[0].nnz == 4
    assert (H != H.T).nnz == 0


@pytest.mark.parametrize("nx,ny", SHAPES)
@pytest.mark.parametrize("rf", [1.5, 2.0, 3.7])
def test_density_preserves_constants(nx, ny, rf):
    y = np.full((ny, nx, 2), 0.37)
    np.testing.assert_allclose(cf.density(y, rf), 0.37, rtol=1e-15)


@pytest.mark.parametrize("nx,ny", SHAPES)
@pytest.mark.parametrize("rf", [1.2, 2.5, 4.0])
def test_adjoint_identity(nx, ny, rf):
    rng = np.random.default_rng(nx * ny)
    a = rng.standard_normal((ny, nx, 3))
    b = rng.standard_normal((ny, nx, 3))
    lhs = np.sum(cf.density(a, rf) * b)
    rhs = np.sum(a * cf.density_adjoint(b, rf))
    assert lhs == pytest.approx(rhs, rel=1e-13)


@pytest.mark.parametrize("nx,ny", SHAPES)
@pytest.mark.parametrize("rf", [1.5, 2.3, 3.0, 5.5])
def test_density_matches_scipy_correlation(nx, ny, rf):
    """The same normalised cone average from scipy.ndimage (zero outside the grid)."""
    R = cf.radius_cells(rf)
    dj, di = np.meshgrid(np.arange(-R, R + 1), np.arange(-R, R + 1), indexing="ij")
    kern = np.maximum(0.0, rf - np.sqrt(di ** 2 + dj ** 2))
    rng = np.random.default_rng(7)
    y = rng.random((ny, nx, 2))
    num = np.stack([ndimage.correlate(y[..., k], kern, mode="constant", cval=0.0) for k in range(2)], -1)
    den = ndimage.correlate(np.ones((ny, nx)), kern, mode="constant", cval=0.0)
    np.testing.assert_allclose(cf.density(y, rf), num / den[..., None], rtol=1e-13)


@pytest.mark.parametrize("rf", [0.3, 1.0])
def test_radius_at_most_one_is_the_identity(rf):
    rng = np.random.default_rng(3)
    y = rng.random((6, 9, 2))
    x = rng.random((6, 9, 2))
    np.testing.assert_allclose(cf.density(y, rf), y, rtol=1e-15)
    np.testing.assert_allclose(cf.sensitivity(x, y, rf, 1e-3), x * y / np.maximum(1e-3, x), rtol=1e-15)


def test_sensitivity_of_full_density_is_the_density_filter():
    rng = np.random.default_rng(4)
    g = rng.standard_normal((8, 11, 3))
    np.testing.assert_allclose(cf.sensitivity(np.ones_like(g), g, 2.5), cf.density(g, 2.5), rtol=1e-14)


def test_sensitivity_floor_keeps_void_finite():
    g = np.ones((5, 5, 1))
    x = np.zeros((5, 5, 1))
    x[2, 2] = 1.0
    s = cf.sensitivity(x, g, 1.5, 1e-3)
    assert np.all(np.isfinite(s))
    # the centre of an isolated solid element: its own term over its own weight sum
    H = cf.cone_matrix(5, 5, 1.5)
    assert s[2, 2, 0] == pytest.approx(1.5 / H[12].sum(), rel=1e-15)


@pytest.mark.parametrize("kind", ["density", "adjoint", "sensitivity"])
def test_filter_at_agrees_with_the_matrix(kind):
    rng = np.random.default_rng(5)
    y = rng.standard_normal((9, 12, 2))
    x = rng.random((9, 12, 2))
    rf = 2.6
    full = {"density": lambda: cf.density(y, rf), "adjoint": lambda: cf.density_adjoint(y, rf),
            "sensitivity": lambda: cf.sensitivity(x, y, rf)}[kind]()
    for i, j in [(0, 0), (11, 8), (5, 4), (1, 7)]:
        np.testing.assert_allclose(cf.filter_at(y, i, j, rf, kind, x), full[j, i], rtol=1e-13)
