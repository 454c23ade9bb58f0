"""The compliance problem solved two ways (Sections 3-4).

* ``solve_direct``: the plain definition u_f = K_ff^{-1} f_f (u = 0 on the
  clamped edge), using a sparse direct factorisation as a library step, or
  the dense Cholesky of Algorithm 3 on tiny grids.  Because K_ff is
  symmetric positive definite the solution is unique; pCGMG, Jacobi-PCG and
  Cholesky differ only in rounding.
* ``solve_mgpcg``: PCG (Algorithm 2) preconditioned by the V-cycle
  (Algorithm 1) over a Galerkin hierarchy — the oracle's own pCGMG, used
  where a direct solve is too slow, and timed as the CPU baseline.

Both return the full displacement field [n_cases, nely+1, nelx+1, 2],
the compliance per load case and the compliance gradient per load case.
"""

from __future__ import annotations

import dataclasses
import time
from typing import Optional

import numpy as np
import scipy.sparse.linalg as spla

from . import fe, linalg, multigrid


@dataclasses.dataclass
class Solution:
    U: np.ndarray          # [n_cases, nely+1, nelx+1, 2]
    c: np.ndarray          # [n_cases]
    dcdx: Optional[np.ndarray]  # [n_cases, nely, nelx, m]
    iters: list
    relres: list           # true ||f - K u|| / ||f|| per case
    t_setup: float = 0.0
    t_solve: float = 0.0


def system(nelx, nely, x, E_phase, E_min, penal, nu):
    """Element moduli (Eq. 5), the free-DOF stiffness K_ff and the free DOF list."""
    E = fe.interpolate_modulus(x, E_phase, E_min, penal)
    K = fe.assemble_stiffness(nelx, nely, E, nu)
    free = fe.free_dofs(nelx, nely)
    return E, K, fe.restrict_to_free(K, free), free


def _finish(nelx, nely, x, E_phase, E_min, penal, nu, F, Uf_list, K, free, iters, grad):
    n_cases = F.shape[0]
    U = np.zeros((n_cases, (nely + 1) * (nelx + 1) * 2))
    c = np.zeros(n_cases)
    rel = []
    dc = [] if grad else None
    for k in range(n_cases):
        U[k, free] = Uf_list[k]
        f = F[k].ravel()
        c[k] = fe.compliance(f, U[k])
        rf = f[free] - K[free][:, free] @ U[k, free]
        nf = np.linalg.norm(f[free])
        rel.append(float(np.linalg.norm(rf) / nf) if nf > 0 else 0.0)
        if grad:
            dc.append(fe.compliance_gradient(x, U[k], E_phase, E_min, penal, nu))
    U = U.reshape(n_cases, nely + 1, nelx + 1, 2)
    return Solution(U, c, np.stack(dc) if grad else None, iters, rel)


def solve_direct(nelx, nely, x, E_phase, E_min, penal, nu, F, grad=True,
                 dense_cholesky=False) -> Solution:
    """u_f = K_ff^{-1} f_f for every load case (sparse LU, or Algorithm 3 when asked)."""
    F = np.asarray(F, dtype=np.float64).reshape(-1, nely + 1, nelx + 1, 2)
    t0 = time.perf_counter()
    _, K, Kff, free = system(nelx, nely, x, E_phase, E_min, penal, nu)
    if dense_cholesky:
        L = linalg.cholesky(Kff.toarray())
        t1 = time.perf_counter()
        Uf = [linalg.cholesky_solve(L, F[k].ravel()[free]) for k in range(F.shape[0])]
    else:
        lu = spla.splu(Kff.tocsc(), permc_spec="MMD_AT_PLUS_A")
        t1 = time.perf_counter()
        Uf = [lu.solve(F[k].ravel()[free]) for k in range(F.shape[0])]
    t2 = time.perf_counter()
    sol = _finish(nelx, nely, x, E_phase, E_min, penal, nu, F, Uf, K, free,
                  [0] * F.shape[0], grad)
    sol.t_setup, sol.t_solve = t1 - t0, t2 - t1
    return sol


def solve_mgpcg(nelx, nely, x, E_phase, E_min, penal, nu, F, levels, omega=0.6, n_pre=2,
                n_post=2, rel_tol=1e-8, max_iter=1000, grad=True, gamma=1,
                max_iter_override=None, dtype=np.float64) -> Solution:
    """PCG preconditioned by one multigrid cycle per iteration (pCGMG).

    ``dtype=np.longdouble`` runs every step in extended precision (64-bit
    mantissa on x86) from the same FP64 data, to separate what rounding does
    to the iteration count from what the method does."""
    F = np.asarray(F, dtype=dtype).reshape(-1, nely + 1, nelx + 1, 2)
    t0 = time.perf_counter()
    _, K, Kff, free = system(nelx, nely, np.asarray(x, dtype=dtype), E_phase, E_min, penal, nu)
    H = multigrid.Hierarchy(nelx, nely, Kff, levels)
    M = multigrid.preconditioner(H, omega, n_pre, n_post, gamma)
    t1 = time.perf_counter()
    Uf, iters = [], []
    for k in range(F.shape[0]):
        res = linalg.pcg(lambda v: Kff @ v, F[k].ravel()[free], M, rel_tol=rel_tol,
                         max_iter=max_iter if max_iter_override is None else max_iter_override)
        Uf.append(res.x)
        iters.append(res.iters)
    t2 = time.perf_counter()
    sol = _finish(nelx, nely, x, E_phase, E_min, penal, nu, F, Uf, K, free, iters, grad)
    sol.t_setup, sol.t_solve = t1 - t0, t2 - t1
    return sol
