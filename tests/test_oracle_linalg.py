"""Pins for the oracle's Cholesky, substitution, damped Jacobi and PCG (Section 2)."""

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import fe, linalg, multigrid, solve
from workloads import load_top_traction


def _spd(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    return A @ A.T + n * np.eye(n)


@pytest.mark.parametrize("n", [1, 2, 7, 40])
def test_cholesky_matches_lapack(n):
    A = _spd(n, n)
    L = linalg.cholesky(A)
    np.testing.assert_allclose(L, np.linalg.cholesky(A), rtol=1e-12, atol=1e-12)
    assert np.all(np.triu(L, 1) == 0)


def test_cholesky_rejects_indefinite():
    A = np.array([[1.0, 2.0], [2.0, 1.0]])
    with pytest.raises(np.linalg.LinAlgError):
        linalg.cholesky(A)


def test_substitutions_and_solve_match_lapack():
    A = _spd(30, 1)
    b = np.random.default_rng(2).standard_normal(30)
    L = linalg.cholesky(A)
    y = linalg.forward_substitution(L, b)
    np.testing.assert_allclose(y, sla.solve_triangular(L, b, lower=True), rtol=1e-12)
    x = linalg.cholesky_solve(L, b)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-11)


def test_stiffness_cholesky_matches_lapack():
    rng = np.random.default_rng(7)
    n = 6
    E = rng.uniform(0.01, 1.0, (n, n))
    K = fe.assemble_stiffness(n, n, E, 0.3)
    Kff = fe.restrict_to_free(K, fe.free_dofs(n, n)).toarray()
    np.testing.assert_allclose(linalg.cholesky(Kff), np.linalg.cholesky(Kff), rtol=1e-11, atol=1e-13)


def test_damped_jacobi_contraction_factor():
    # the error of x <- x + w D^-1 (b - A x) is multiplied by I - w D^-1 A;
    # for SPD A the spectral radius is max |1 - w lambda(D^-1 A)|
    rng = np.random.default_rng(8)
    n = 6
    E = rng.uniform(0.1, 1.0, (n, n))
    Kff = fe.restrict_to_free(fe.assemble_stiffness(n, n, E, 0.3), fe.free_dofs(n, n))
    A = Kff.toarray()
    d = np.diag(A)
    lam = sla.eigh(A, np.diag(d), eigvals_only=True)
    w = 0.6
    rho = np.max(np.abs(1 - w * lam))
    xs = rng.standard_normal(A.shape[0])
    b = A @ xs
    x0 = np.zeros_like(b)
    # exact solution is a fixed point
    np.testing.assert_allclose(linalg.damped_jacobi(Kff, b, xs, w, 3), xs, rtol=1e-12)
    e = [np.linalg.norm(linalg.damped_jacobi(Kff, b, x0, w, k) - xs) for k in (200, 400)]
    assert e[1] / e[0] == pytest.approx(rho ** 200, rel=0.2)


def test_pcg_cg_bound_and_exactness():
    A = _spd(25, 9)
    b = np.ones(25)
    xs = np.linalg.solve(A, b)
    ev = np.linalg.eigvalsh(A)
    kappa = ev[-1] / ev[0]
    q = (np.sqrt(kappa) - 1) / (np.sqrt(kappa) + 1)
    enorm = lambda v: np.sqrt((v - xs) @ A @ (v - xs))
    e0 = enorm(np.zeros(25))
    for k in (1, 3, 6):
        r = linalg.pcg(lambda v: A @ v, b, lambda v: v, rel_tol=0.0, max_iter=k)
        # Eq. (2) with the textbook factor 2
        assert enorm(r.x) <= 2 * e0 * q ** k * (1 + 1e-12)
    r = linalg.pcg(lambda v: A @ v, b, lambda v: v, rel_tol=1e-13, max_iter=200)
    np.testing.assert_allclose(r.x, xs, rtol=1e-11)


@pytest.mark.parametrize("n,levels", [(16, 3), (32, 4)])
def test_mg_and_jacobi_pcg_match_dense_cholesky(n, levels):
    rng = np.random.default_rng(n)
    x = rng.uniform(0.0, 1.0, (n, n, 3)) / 3
    Eph, Emin, p, nu = [1.0, 0.6, 0.2], 1e-9, 3.0, 0.3
    F = load_top_traction(n, n)[None]
    ref = solve.solve_direct(n, n, x, Eph, Emin, p, nu, F, dense_cholesky=True)
    mg = solve.solve_mgpcg(n, n, x, Eph, Emin, p, nu, F, levels, rel_tol=1e-13)
    np.testing.assert_allclose(mg.U, ref.U, rtol=0, atol=1e-12 * np.abs(ref.U).max())
    _, K, Kff, free = solve.system(n, n, x, Eph, Emin, p, nu)
    jr = linalg.pcg(lambda v: Kff @ v, F[0].ravel()[free], lambda v: v / Kff.diagonal(),
                    rel_tol=1e-13, max_iter=20000)
    np.testing.assert_allclose(jr.x, ref.U[0].ravel()[free], rtol=0,
                               atol=1e-11 * np.abs(ref.U).max())
    assert mg.iters[0] < jr.iters


def test_extended_precision_cholesky_against_exact_rationals():
    """The oracle's steps keep np.longdouble inputs in long double: on the
    8 x 8 Hilbert matrix (kappa 1.5e10, FP64 data) the solve's error
    against the exact rational solution of the same data shrinks by about
    the ratio of the two machine epsilons (2^11 on x86)."""
    from fractions import Fraction
    n = 8
    H = np.array([[1.0 / (i + j + 1) for j in range(n)] for i in range(n)])
    b = H.sum(1)
    M = [[Fraction(H[i, j]) for j in range(n)] + [Fraction(b[i])] for i in range(n)]
    for k in range(n):
        for i in range(k + 1, n):
            f = M[i][k] / M[k][k]
            M[i] = [a - f * c for a, c in zip(M[i], M[k])]
    xe = [Fraction(0)] * n
    for i in range(n - 1, -1, -1):
        xe[i] = (M[i][n] - sum(M[i][j] * xe[j] for j in range(i + 1, n))) / M[i][i]
    xe = np.array([float(v) for v in xe])
    err = {}
    for dt in (np.float64, np.longdouble):
        x = linalg.cholesky_solve(linalg.cholesky(H.astype(dt)), b.astype(dt))
        assert x.dtype == dt
        err[dt] = float(np.max(np.abs(x - xe)) / np.max(np.abs(xe)))
    if np.finfo(np.longdouble).eps < np.finfo(np.float64).eps:
        assert err[np.longdouble] <= err[np.float64] / 100, err
    assert err[np.float64] <= 1.5e10 * np.finfo(np.float64).eps * 10


def test_mgpcg_in_extended_precision_matches_fp64():
    """The extended-precision pCGMG solves the same system: on a smooth
    design it takes the FP64 run's iteration count and lands on its answer."""
    n, levels = 16, 3
    rng = np.random.default_rng(3)
    x = rng.uniform(0.0, 1.0, (n, n, 3)) / 3
    args = (n, n, x, [1.0, 0.6, 0.2], 1e-9, 3.0, 0.3, load_top_traction(n, n)[None], levels)
    a = solve.solve_mgpcg(*args, rel_tol=1e-10, grad=False)
    b = solve.solve_mgpcg(*args, rel_tol=1e-10, grad=False, dtype=np.longdouble)
    assert a.iters == b.iters
    np.testing.assert_allclose(b.U, a.U, rtol=0, atol=1e-9 * np.abs(a.U).max())
