"""Cone filter of element fields (Section 4, radius rf of Table 2) — TEST INFRASTRUCTURE ONLY.

The paper filters the sensitivities after the adjoint gradient and lists a
filter radius rf, but does not write the filter out.  This is the usual
cone (linear hat) filter on element centres, applied to each phase:

* weights H_ef = max(0, rf - |c_e - c_f|), with distances measured in
  element widths between the centres of elements e and f; the sum runs
  over the elements of the grid only (truncated at its edges);
* ``density(y)``       = (H y) / (H 1), a normalised weighted average;
* ``density_adjoint(g)`` = H^T (g / (H 1)), the chain rule through
  ``density`` (H is symmetric, so this is H (g / (H 1)));
* ``sensitivity(x, g)`` = H (x g) / (max(gmin, x) (H 1)), the
  mesh-independency sensitivity filter (x: densities of the same phase,
  gmin a floor that keeps void elements finite).

Fields are [nely][nelx][m] arrays (element (i, j) in row j, column i, m
phases), as the design variables.  ``cone_matrix`` builds H as a sparse
matrix, the plain definition; ``filter_at`` evaluates one output element by
a double loop, for sampled checks on grids too large for the matrix.
Every function is pinned by tests/test_oracle_cone_filter.py (hand-computed
weights, constants preserved, the adjoint identity, scipy.ndimage's
correlation as an independent implementation).
"""

from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp


def radius_cells(rf: float) -> int:
    """Largest offset |di| or |dj| with a positive weight: centres closer
    than rf, so offsets up to ceil(rf) - 1."""
    return max(0, int(math.ceil(rf)) - 1)


def cone_matrix(nelx: int, nely: int, rf: float) -> sp.csr_matrix:
    """H with H[e, f] = max(0, rf - dist(e, f)), e = j * nelx + i."""
    R = radius_cells(rf)
    jj, ii = np.meshgrid(np.arange(nely), np.arange(nelx), indexing="ij")
    rows, cols, vals = [], [], []
    for dj in range(-R, R + 1):
        for di in range(-R, R + 1):
            w = rf - math.sqrt(di * di + dj * dj)
            if w <= 0.0:
                continue
            ok = (ii + di >= 0) & (ii + di < nelx) & (jj + dj >= 0) & (jj + dj < nely)
            e = (jj * nelx + ii)[ok]
            f = ((jj + dj) * nelx + (ii + di))[ok]
            rows.append(e)
            cols.append(f)
            vals.append(np.full(e.size, w))
    n = nelx * nely
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))


def _per_phase(field: np.ndarray):
    ny, nx = field.shape[:2]
    return field.reshape(ny * nx, -1), (ny, nx)


def density(y: np.ndarray, rf: float) -> np.ndarray:
    """(H y) / (H 1) for each phase of y [nely][nelx][m]."""
    Y, (ny, nx) = _per_phase(y)
    H = cone_matrix(nx, ny, rf)
    s = H @ np.ones(nx * ny)
    return ((H @ Y) / s[:, None]).reshape(y.shape)


def density_adjoint(g: np.ndarray, rf: float) -> np.ndarray:
    """H^T (g / (H 1)): the gradient with respect to y of a function of density(y)."""
    G, (ny, nx) = _per_phase(g)
    H = cone_matrix(nx, ny, rf)
    s = H @ np.ones(nx * ny)
    return (H.T @ (G / s[:, None])).reshape(g.shape)


def sensitivity(x: np.ndarray, g: np.ndarray, rf: float, gmin: float = 1e-3) -> np.ndarray:
    """H (x g) / (max(gmin, x) (H 1)) per phase."""
    X, (ny, nx) = _per_phase(x)
    G, _ = _per_phase(g)
    H = cone_matrix(nx, ny, rf)
    s = H @ np.ones(nx * ny)
    return ((H @ (X * G)) / (np.maximum(gmin, X) * s[:, None])).reshape(g.shape)


def filter_at(y: np.ndarray, i: int, j: int, rf: float, kind: str = "density",
              x: np.ndarray | None = None, gmin: float = 1e-3) -> np.ndarray:
    """One output element (all phases) by a direct loop over its neighbours.

    kind: "density", "adjoint" (needs the normalisation of every neighbour,
    formed by its own loop) or "sensitivity" (needs x)."""
    ny, nx = y.shape[:2]
    R = radius_cells(rf)

    def wsum(a, b):
        s = 0.0
        for dj in range(-R, R + 1):
            for di in range(-R, R + 1):
                w = rf - math.sqrt(di * di + dj * dj)
                if w > 0.0 and 0 <= a + di < nx and 0 <= b + dj < ny:
                    s += w
        return s

    acc = np.zeros(y.shape[2])
    for dj in range(-R, R + 1):
        for di in range(-R, R + 1):
            w = rf - math.sqrt(di * di + dj * dj)
            a, b = i + di, j + dj
            if w <= 0.0 or not (0 <= a < nx and 0 <= b < ny):
                continue
            if kind == "density":
                acc += w * y[b, a]
            elif kind == "adjoint":
                acc += w * y[b, a] / wsum(a, b)
            elif kind == "sensitivity":
                acc += w * x[b, a] * y[b, a]
            else:
                raise ValueError(kind)
    if kind == "adjoint":
        return acc
    if kind == "sensitivity":
        return acc / (np.maximum(gmin, x[j, i]) * wsum(i, j))
    return acc / wsum(i, j)
