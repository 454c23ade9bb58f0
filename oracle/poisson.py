"""Poisson model problem of Section 5.1 — TEST INFRASTRUCTURE ONLY.

-Laplace(u) = f on the unit square, u = 0 on the whole boundary, bilinear
(Q4) elements on an n x n grid of square elements of side h = 1/n.  The
paper runs pCGMG on this problem with the coarsest grid 2 x 2 (one
unknown) and meshes 16^2 .. 256^2 (levels 3 .. 7).  Written out plainly:

* ``element_matrix``: the Q4 Laplace matrix, the integral of grad N_a .
  grad N_b over one element by 2x2 Gauss quadrature (exact here); it does
  not depend on h in 2D;
* ``assemble``: K over all (n+1)^2 nodes, then restricted to the interior
  nodes (i, j in 1 .. n-1, row-major, i fastest);
* ``load``: consistent nodal loads of a source f given at the nodes and
  interpolated bilinearly, F = M f with the Q4 mass matrix;
* ``hierarchy``: Galerkin coarse operators P^T K P with P the bilinear
  interpolation between interior nodes (boundary values are 0), in the
  form ``multigrid.cycle`` consumes, so the multigrid cycle and PCG are the
  oracle's own (Algorithms 1 and 2).
Node values are [n+1][n+1] arrays (row j, column i) where a full field is
meant, interior vectors elsewhere.  Every function is pinned by
tests/test_oracle_poisson.py: hand-computed element matrices, the 9-point
stencil, second-order convergence to a closed-form solution, Galerkin
operators equal to the coarse discretisation, a symmetric positive definite
cycle and mesh-independent iteration counts.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fe, linalg, multigrid

GAUSS = (0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0))


def element_matrix() -> np.ndarray:
    """4 x 4 Q4 Laplace matrix; local nodes (0,0), (1,0), (1,1), (0,1)."""
    K = np.zeros((4, 4))
    for xi in GAUSS:
        for eta in GAUSS:
            dxi, deta = fe.shape_gradients(xi, eta)
            G = np.vstack([dxi, deta])          # 2 x 4, unit square element
            K += 0.25 * G.T @ G                 # weight 1/4 per point
    return K


def element_mass() -> np.ndarray:
    """4 x 4 Q4 mass matrix of the unit square (times h^2 on the grid)."""
    M = np.zeros((4, 4))
    for xi in GAUSS:
        for eta in GAUSS:
            N = np.array([(1 - xi) * (1 - eta), xi * (1 - eta), xi * eta, (1 - xi) * eta])
            M += 0.25 * np.outer(N, N)
    return M


def _element_nodes(n: int) -> np.ndarray:
    j, i = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    base = (j * (n + 1) + i).ravel()
    return np.stack([base, base + 1, base + n + 2, base + n + 1], axis=1)


def _assemble(n: int, Ke: np.ndarray) -> sp.csr_matrix:
    en = _element_nodes(n)
    rows = np.repeat(en, 4, axis=1).ravel()
    cols = np.tile(en, (1, 4)).ravel()
    vals = np.tile(Ke.ravel(), n * n)
    N = (n + 1) ** 2
    return sp.csr_matrix((vals, (rows, cols)), shape=(N, N))


def interior(n: int) -> np.ndarray:
    """Indices of the interior nodes, row-major."""
    j, i = np.meshgrid(np.arange(1, n), np.arange(1, n), indexing="ij")
    return (j * (n + 1) + i).ravel()


def assemble(n: int) -> sp.csr_matrix:
    """K restricted to the interior nodes."""
    K = _assemble(n, element_matrix())
    f = interior(n)
    return K[f][:, f].tocsr()


def load(n: int, f_nodes: np.ndarray) -> np.ndarray:
    """Interior part of M f for nodal source values f_nodes [n+1][n+1]."""
    M = _assemble(n, element_mass()) / float(n * n)
    return (M @ np.ravel(f_nodes))[interior(n)]


def prolongation(nc: int) -> sp.csr_matrix:
    """Bilinear interpolation from the interior nodes of an nc x nc grid to
    those of the 2nc x 2nc grid."""
    P1 = multigrid.prolongation_1d(nc)[1:-1, 1:-1]
    return sp.kron(P1, P1).tocsr()


class _Level:
    def __init__(self, n: int, K: sp.csr_matrix):
        self.nelx = self.nely = n
        self.K = K
        self.diag = K.diagonal().copy()
        self.P = None
        self.chol = None


class Hierarchy:
    """levels[0] is the coarsest grid; n must be divisible by 2^(levels-1)
    and the coarsest grid must have an interior node."""

    def __init__(self, n: int, n_levels: int):
        s = 2 ** (n_levels - 1)
        if n % s or n // s < 2:
            raise ValueError("n must be a multiple of 2^(levels-1) with a coarsest grid of at least 2 x 2")
        levels = [_Level(n, assemble(n))]
        for _ in range(n_levels - 1):
            f = levels[-1]
            P = prolongation(f.nelx // 2)
            f.P = P
            levels.append(_Level(f.nelx // 2, (P.T @ (f.K @ P)).tocsr()))
        levels.reverse()
        levels[0].chol = linalg.cholesky(levels[0].K.toarray())
        self.levels = levels

    @property
    def n_levels(self) -> int:
        return len(self.levels)


def solve_mgpcg(n: int, levels: int, F: np.ndarray, omega: float = 0.6, n_pre: int = 2, n_post: int = 2,
                rel_tol: float = 1e-8, max_iter: int = 1000, gamma: int = 1):
    """PCG (Algorithm 2) on the interior system with one multigrid cycle
    (Algorithm 1) as preconditioner; returns linalg.pcg's result."""
    H = Hierarchy(n, levels)
    M = multigrid.preconditioner(H, omega, n_pre, n_post, gamma)
    K = H.levels[-1].K
    return linalg.pcg(lambda v: K @ v, F, M, rel_tol=rel_tol, max_iter=max_iter)


def solve_direct(n: int, F: np.ndarray) -> np.ndarray:
    """u = K^{-1} F on the interior nodes (sparse direct solve)."""
    from scipy.sparse.linalg import spsolve
    return spsolve(assemble(n).tocsc(), F)


def to_grid(n: int, u_int: np.ndarray) -> np.ndarray:
    """Interior vector -> [n+1][n+1] nodal field with zero boundary."""
    U = np.zeros((n + 1) * (n + 1))
    U[interior(n)] = u_int
    return U.reshape(n + 1, n + 1)
