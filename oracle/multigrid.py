"""Multigrid gamma-cycle preconditioner (Section 2.1, Algorithm 1; Section 2.2).

Grids are nested by halving the element count in both directions; a
hierarchy with L levels has grids l = 0 (coarsest) .. L-1 (the finest,
the problem grid), so nelx and nely must be divisible by 2^(L-1).

* Prolongation P_l maps level l-1 nodal values to level l by bilinear
  interpolation of each displacement component (weights 1, 1/2, 1/4);
  restriction is its transpose, R_l = P_l^T.
* Coarse operators are Galerkin products K_{l-1} = P_l^T K_l P_l.  (The
  paper forms each K_n by discretising on mesh Omega_n; for a uniform
  modulus the two agree exactly, which a test checks.)
* Clamped nodes are removed at every level; P maps coarse free DOFs to fine
  free DOFs exactly because coarse and fine share the clamped edge.
* ``cycle`` is Algorithm 1: at l = 0 solve K_0 U = F directly (Cholesky,
  Algorithm 3); otherwise pre-smooth theta_1 times, restrict the residual,
  start the coarse iterate at zero, recurse gamma times, prolongate and
  correct, post-smooth theta_2 times.  The smoother is damped Jacobi
  (Section 2.3).  As a PCG preconditioner the cycle starts from U = 0, so it
  is a fixed linear map, symmetric because pre- and post-smoothing use the
  same Jacobi sweep (Section 2.2).
"""

from __future__ import annotations

from typing import List, Optional

import numpy as np
import scipy.sparse as sp

from . import fe, linalg


def prolongation_1d(nc: int) -> sp.csr_matrix:
    """(2nc+1) x (nc+1) linear interpolation from nc coarse to 2nc fine intervals."""
    rows, cols, vals = [], [], []
    for i in range(2 * nc + 1):
        if i % 2 == 0:
            rows.append(i); cols.append(i // 2); vals.append(1.0)
        else:
            rows += [i, i]; cols += [i // 2, i // 2 + 1]; vals += [0.5, 0.5]
    return sp.csr_matrix((vals, (rows, cols)), shape=(2 * nc + 1, nc + 1))


def prolongation(nelx_c: int, nely_c: int) -> sp.csr_matrix:
    """Bilinear P from a nelx_c x nely_c grid to the 2x refined grid, all DOFs.

    Node ordering is row-major (x fastest) with two interleaved DOFs; the
    weight of coarse node (I, J) at fine node (i, j) is w_x(i, I) w_y(j, J).
    """
    Px = prolongation_1d(nelx_c)
    Py = prolongation_1d(nely_c)
    Pn = sp.kron(Py, Px).tocsr()               # nodes: (j, i) row-major
    return sp.kron(Pn, sp.identity(2)).tocsr()  # two interleaved components


class Level:
    def __init__(self, nelx: int, nely: int, K: sp.csr_matrix):
        self.nelx = nelx
        self.nely = nely
        self.K = K                      # free-DOF operator of this grid
        self.diag = K.diagonal().copy()
        self.P: Optional[sp.csr_matrix] = None  # from level l-1 to this level (free DOFs)
        self.chol: Optional[np.ndarray] = None  # coarsest level only


class Hierarchy:
    """Galerkin hierarchy for the clamped-bottom wall; levels[0] is coarsest."""

    def __init__(self, nelx: int, nely: int, K_ff: sp.csr_matrix, n_levels: int):
        if n_levels < 1:
            raise ValueError("need at least one level")
        s = 2 ** (n_levels - 1)
        if nelx % s or nely % s:
            raise ValueError("grid not divisible by 2^(levels-1)")
        fine = Level(nelx, nely, K_ff.tocsr())
        levels = [fine]
        for _ in range(n_levels - 1):
            f = levels[-1]
            cx, cy = f.nelx // 2, f.nely // 2
            Pall = prolongation(cx, cy)
            ff = fe.free_dofs(f.nelx, f.nely)
            cf = fe.free_dofs(cx, cy)
            P = Pall[ff][:, cf].tocsr()
            f.P = P
            Kc = (P.T @ (f.K @ P)).tocsr()
            levels.append(Level(cx, cy, Kc))
        levels.reverse()
        levels[0].chol = linalg.cholesky(levels[0].K.toarray())
        self.levels: List[Level] = levels

    @property
    def n_levels(self) -> int:
        return len(self.levels)


def cycle(H: Hierarchy, l: int, F: np.ndarray, U: Optional[np.ndarray] = None,
          omega: float = 0.6, n_pre: int = 2, n_post: int = 2, gamma: int = 1) -> np.ndarray:
    """Algorithm 1, MG_gamma^l(U_l, F_l); U = None means a zero initial iterate."""
    lev = H.levels[l]
    if l == 0:
        return linalg.cholesky_solve(lev.chol, F)
    U = np.zeros_like(F) if U is None else U
    U = linalg.damped_jacobi(lev.K, F, U, omega, n_pre, lev.diag)
    Fc = lev.P.T @ (F - lev.K @ U)
    Uc = np.zeros_like(Fc)
    for _ in range(gamma):
        Uc = cycle(H, l - 1, Fc, Uc, omega, n_pre, n_post, gamma)
    U = U + lev.P @ Uc
    U = linalg.damped_jacobi(lev.K, F, U, omega, n_post, lev.diag)
    return U


def preconditioner(H: Hierarchy, omega: float = 0.6, n_pre: int = 2, n_post: int = 2,
                   gamma: int = 1):
    """r -> M^{-1} r: one cycle on the finest grid from a zero iterate."""
    top = H.n_levels - 1
    return lambda r: cycle(H, top, r, None, omega, n_pre, n_post, gamma)
