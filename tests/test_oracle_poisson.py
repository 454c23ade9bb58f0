"""Pins for the oracle's Poisson model problem (Section 5.1).

Checked against what the mathematics fixes: the textbook Q4 Laplace and
mass matrices, the 9-point stencil (8 u_c - sum of the 8 neighbours) / 3,
second-order convergence to the exact solution u = sin(pi x) sin(pi y) of
-Laplace(u) = 2 pi^2 u, Galerkin coarse operators equal to the coarse
discretisation (the variational property in 2D), and pCGMG iteration
counts that do not grow with the mesh (the paper's observation).
"""

import numpy as np
import pytest

from oracle import multigrid, poisson


def test_element_matrices_by_hand():
    K = poisson.element_matrix()
    want = np.array([[4, -1, -2, -1], [-1, 4, -1, -2], [-2, -1, 4, -1], [-1, -2, -1, 4]]) / 6.0
    np.testing.assert_allclose(K, want, atol=1e-15)
    M = poisson.element_mass()
    want = np.array([[4, 2, 1, 2], [2, 4, 2, 1], [1, 2, 4, 2], [2, 1, 2, 4]]) / 36.0
    np.testing.assert_allclose(M, want, atol=1e-15)


def test_interior_stencil():
    n = 6
    K = poisson.assemble(n)
    u = np.zeros((n + 1, n + 1))
    u[3, 3] = 1.0
    q = poisson.to_grid(n, K @ u[1:-1, 1:-1].ravel())
    np.testing.assert_allclose(q[3, 3], 8.0 / 3.0)
    for dj in (-1, 0, 1):
        for di in (-1, 0, 1):
            if dj or di:
                np.testing.assert_allclose(q[3 + dj, 3 + di], -1.0 / 3.0)
    assert abs(q).sum() == pytest.approx(8.0 / 3.0 + 8.0 / 3.0)


def test_second_order_convergence():
    errs = []
    for n in (8, 16, 32):
        x = np.linspace(0.0, 1.0, n + 1)
        X, Y = np.meshgrid(x, x)
        exact = np.sin(np.pi * X) * np.sin(np.pi * Y)
        F = poisson.load(n, 2 * np.pi ** 2 * exact)
        u = poisson.to_grid(n, poisson.solve_direct(n, F))
        errs.append(np.abs(u - exact).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.9), (errs, rates)


@pytest.mark.parametrize("n,L", [(16, 3), (32, 4)])
def test_galerkin_equals_rediscretisation(n, L):
    H = poisson.Hierarchy(n, L)
    for lev in H.levels:
        diff = abs(lev.K - poisson.assemble(lev.nelx)).max()
        assert diff < 1e-13


def test_mgpcg_iterations_do_not_grow_with_the_mesh():
    its = []
    for n, L in ((16, 3), (32, 4), (64, 5), (128, 6)):
        F = poisson.load(n, np.ones((n + 1, n + 1)))
        res = poisson.solve_mgpcg(n, L, F, rel_tol=1e-8)
        assert res.converged
        u = poisson.solve_direct(n, F)
        assert np.linalg.norm(res.x - u) <= 1e-6 * np.linalg.norm(u)
        its.append(res.iters)
    assert max(its) - min(its) <= 2, its


def test_cycle_is_symmetric_positive_definite():
    H = poisson.Hierarchy(16, 3)
    N = H.levels[-1].K.shape[0]
    M = np.column_stack([multigrid.cycle(H, 2, e, None, 0.6, 2, 2) for e in np.eye(N)])
    np.testing.assert_allclose(M, M.T, atol=1e-13)
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0
