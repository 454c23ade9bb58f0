"""Linear-algebra steps of Section 2, written out plainly in FP64 (or in the
extended precision of their inputs, when those are np.longdouble).

* ``cholesky`` follows Algorithm 3: for each column k take the square root
  of the pivot, scale the column below it, then subtract the outer product
  of that column from the trailing lower triangle.  The printed loop and
  Eq. (4) carry typesetting slips (an index i for t in the update, a stray
  square root in Eq. 4); the reading used here is the textbook one:
  L_jj = sqrt(A_jj - sum_{k<j} L_jk^2), L_ij = (A_ij - sum_{k<j} L_ik L_jk) / L_jj.
* forward / back substitution solve L y = b and L^T x = y (Section 2.3).
* ``damped_jacobi`` is x <- x + omega D^{-1} (b - A x), i.e.
  x_{k+1} = (I - omega D^{-1} A) x_k + omega D^{-1} b (Section 2.3).
* ``pcg`` is Algorithm 2: z = M^{-1} r, beta = z_i^T r_i / z_{i-1}^T r_{i-1},
  p = z + beta p, alpha = z^T r / p^T A p, x += alpha p, r -= alpha A p.  The
  stop test "r_i = 0" is read as ||r_i||_2 <= rel_tol ||b||_2.
"""

from __future__ import annotations

from typing import Callable, Optional

import numpy as np


def cholesky(A: np.ndarray) -> np.ndarray:
    """Lower-triangular L with A = L L^T (Algorithm 3, right-looking)."""
    A = np.array(A, dtype=np.result_type(A, np.float64), copy=True)
    n = A.shape[0]
    L = np.zeros_like(A)
    for k in range(n):
        piv = A[k, k]
        if not piv > 0.0:
            raise np.linalg.LinAlgError(f"matrix not positive definite at column {k}")
        L[k, k] = np.sqrt(piv)
        L[k + 1:, k] = A[k + 1:, k] / L[k, k]
        col = L[k + 1:, k]
        # trailing update of the lower triangle (the upper part is never read)
        A[k + 1:, k + 1:] -= np.outer(col, col)
    return L


def forward_substitution(L: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Solve L y = b for lower-triangular L."""
    n = L.shape[0]
    y = np.zeros(n, dtype=np.result_type(L, b))
    for i in range(n):
        y[i] = (b[i] - np.dot(L[i, :i], y[:i])) / L[i, i]
    return y


def back_substitution(L: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Solve L^T x = y for lower-triangular L."""
    n = L.shape[0]
    x = np.zeros(n, dtype=np.result_type(L, y))
    for i in range(n - 1, -1, -1):
        x[i] = (y[i] - np.dot(L[i + 1:, i], x[i + 1:])) / L[i, i]
    return x


def cholesky_solve(L: np.ndarray, b: np.ndarray) -> np.ndarray:
    """x = A^{-1} b from the factor L of A (forward then back substitution)."""
    return back_substitution(L, forward_substitution(L, b))


def damped_jacobi(A, b: np.ndarray, x: np.ndarray, omega: float, sweeps: int,
                  diag: Optional[np.ndarray] = None) -> np.ndarray:
    """`sweeps` damped-Jacobi iterations x <- x + omega D^{-1} (b - A x)."""
    d = A.diagonal() if diag is None else diag
    x = np.array(x, dtype=np.result_type(x, b, np.float64), copy=True)
    for _ in range(sweeps):
        x = x + omega * (b - A @ x) / d
    return x


class PCGResult:
    def __init__(self, x, iters, relres, converged, history):
        self.x = x
        self.iters = iters
        self.relres = relres
        self.converged = converged
        self.history = history


def pcg(apply_A: Callable[[np.ndarray], np.ndarray], b: np.ndarray,
        apply_Minv: Callable[[np.ndarray], np.ndarray], x0: Optional[np.ndarray] = None,
        rel_tol: float = 1e-8, max_iter: int = 1000) -> PCGResult:
    """Preconditioned conjugate gradients, Algorithm 2.

    Returns x with ||b - A x||_2 <= rel_tol ||b||_2 (recursive residual) or
    after max_iter iterations.  ``iters`` counts updates of x.
    """
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.result_type(b, np.float64), copy=True)
    r = b - apply_A(x)
    bnorm = np.linalg.norm(b)
    hist = [np.linalg.norm(r) / bnorm if bnorm > 0 else 0.0]
    if bnorm == 0.0 or np.linalg.norm(r) <= rel_tol * bnorm:
        return PCGResult(x, 0, hist[-1], True, hist)
    p = None
    rz_old = None
    for i in range(max_iter):
        z = apply_Minv(r)
        rz = np.dot(z, r)
        if p is None:
            p = z.copy()
        else:
            beta = rz / rz_old
            p = z + beta * p
        q = apply_A(p)
        alpha = rz / np.dot(p, q)
        x = x + alpha * p
        r = r - alpha * q
        rz_old = rz
        hist.append(np.linalg.norm(r) / bnorm)
        if hist[-1] <= rel_tol:
            return PCGResult(x, i + 1, hist[-1], True, hist)
    return PCGResult(x, max_iter, hist[-1], False, hist)
