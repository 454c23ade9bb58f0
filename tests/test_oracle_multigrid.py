"""Pins for the oracle's transfers, Galerkin coarse operators and cycle (Sections 2.1-2.2)."""

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import fe, multigrid, solve
from workloads import load_top_traction, make_problem


def test_prolongation_reproduces_bilinear_fields():
    cx, cy = 3, 2
    P = multigrid.prolongation(cx, cy)
    def field(nx, ny, h):
        j, i = np.meshgrid(np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
        X, Y = i * h, j * h
        u = np.stack([1 + 2 * X - 3 * Y + 0.5 * X * Y, -2 + X + 4 * Y - X * Y], axis=-1)
        return u.ravel()
    np.testing.assert_allclose(P @ field(cx, cy, 1.0), field(2 * cx, 2 * cy, 0.5), atol=1e-14)
    # partition of unity and nonnegative weights
    np.testing.assert_allclose(np.asarray(P.sum(axis=1)).ravel() / 1.0, 1.0)
    assert P.min() >= 0


def test_galerkin_equals_rediscretisation_for_uniform_modulus():
    nx, ny = 8, 4
    Kf = fe.restrict_to_free(fe.assemble_stiffness(nx, ny, np.ones((ny, nx)), 0.3),
                             fe.free_dofs(nx, ny))
    H = multigrid.Hierarchy(nx, ny, Kf, 3)
    for lev in H.levels:
        Kr = fe.restrict_to_free(fe.assemble_stiffness(lev.nelx, lev.nely,
                                                       np.ones((lev.nely, lev.nelx)), 0.3),
                                 fe.free_dofs(lev.nelx, lev.nely))
        assert abs(lev.K - Kr).max() < 1e-14


def test_unconstrained_galerkin_keeps_rigid_modes():
    rng = np.random.default_rng(11)
    nx, ny = 8, 8
    K = fe.assemble_stiffness(nx, ny, rng.uniform(1e-3, 1, (ny, nx)), 0.3)
    P = multigrid.prolongation(nx // 2, ny // 2)
    Kc = P.T @ K @ P
    R = fe.rigid_body_modes(nx // 2, ny // 2, 2.0 / nx)
    assert np.abs(Kc @ R.T).max() < 1e-13
    assert abs(Kc - Kc.T).max() < 1e-14


def test_fine_jacobi_spectral_bound():
    # lambda_max(D^-1 K) <= lambda_max(K0) / K0_11 = 6 (1 + nu) / (3 - nu) for any moduli
    rng = np.random.default_rng(12)
    n = 8
    E = np.exp(rng.uniform(np.log(1e-9), 0, (n, n)))
    Kff = fe.restrict_to_free(fe.assemble_stiffness(n, n, E, 0.3), fe.free_dofs(n, n)).toarray()
    lam = sla.eigh(Kff, np.diag(np.diag(Kff)), eigvals_only=True)
    assert lam.max() <= 6 * 1.3 / 2.7 + 1e-9


def _hier(n, levels, seed, log_contrast=False):
    rng = np.random.default_rng(seed)
    E = (np.exp(rng.uniform(np.log(1e-6), 0, (n, n))) if log_contrast
         else rng.uniform(0.05, 1, (n, n)))
    Kff = fe.restrict_to_free(fe.assemble_stiffness(n, n, E, 0.3), fe.free_dofs(n, n))
    return multigrid.Hierarchy(n, n, Kff, levels), Kff


@pytest.mark.parametrize("log_contrast", [False, True])
def test_vcycle_preconditioner_is_symmetric_positive_definite(log_contrast):
    H, Kff = _hier(8, 3, 13, log_contrast)
    M = multigrid.preconditioner(H)
    N = Kff.shape[0]
    Mi = np.stack([M(e) for e in np.eye(N)], axis=1)
    assert np.abs(Mi - Mi.T).max() <= 1e-12 * np.abs(Mi).max()
    assert np.linalg.eigvalsh(0.5 * (Mi + Mi.T)).min() > 0


def test_two_grid_without_smoothing_is_k_orthogonal_projection():
    # Eq. (1) with no smoothing: M^-1 = P K_c^-1 P^T, so M^-1 K is a projector
    H, Kff = _hier(8, 2, 14)
    M = multigrid.preconditioner(H, n_pre=0, n_post=0)
    N = Kff.shape[0]
    Mi = np.stack([M(e) for e in np.eye(N)], axis=1)
    T = Mi @ Kff.toarray()
    np.testing.assert_allclose(T @ T, T, atol=1e-10)
    KT = Kff.toarray() @ T
    np.testing.assert_allclose(KT, KT.T, atol=1e-10)


def test_single_level_cycle_is_exact_solve():
    H, Kff = _hier(4, 1, 15)
    b = np.random.default_rng(1).standard_normal(Kff.shape[0])
    np.testing.assert_allclose(Kff @ multigrid.preconditioner(H)(b), b, atol=1e-12)


def test_wcycle_matches_direct():
    n = 16
    H, Kff = _hier(n, 3, 16)
    F = load_top_traction(n, n)[None]
    f = F[0].ravel()[fe.free_dofs(n, n)]
    from oracle import linalg
    u = linalg.pcg(lambda v: Kff @ v, f, multigrid.preconditioner(H, gamma=2), rel_tol=1e-13).x
    np.testing.assert_allclose(Kff @ u, f, atol=1e-12 * np.abs(f).max())


def test_mgpcg_on_random_cone_wall():
    p = make_problem("wall64")
    ref = solve.solve_direct(p.nelx, p.nely, p.x, p.E_phase, p.E_min, p.penal, p.nu, p.F)
    mg = solve.solve_mgpcg(p.nelx, p.nely, p.x, p.E_phase, p.E_min, p.penal, p.nu, p.F,
                           p.levels, rel_tol=1e-8)
    assert mg.relres[0] <= 1e-8
    err = np.linalg.norm(mg.U - ref.U) / np.linalg.norm(ref.U)
    assert err <= 1e-6
    assert mg.c[0] == pytest.approx(ref.c[0], rel=1e-7)
    np.testing.assert_allclose(mg.dcdx, ref.dcdx, rtol=1e-5, atol=1e-9 * np.abs(ref.dcdx).max())


def _cycle_matrix(H, l, gamma):
    N = H.levels[l].K.shape[0]
    return np.column_stack([multigrid.cycle(H, l, e, None, 0.6, 2, 2, gamma) for e in np.eye(N)])


def test_wcycle_coarse_correction_is_two_visits():
    """gamma = 2: the coarse problem is visited twice, the second visit from
    the first one's result.  A cycle from a start U is the affine map
    U + M (F - K U), so two visits give (2 M - M K M) Fc with M the coarse
    level's own W-cycle matrix; the level above is that coarse correction
    between two damped Jacobi sweeps before and after (written here with
    plain matrices)."""
    H, _ = _hier(8, 3, 21)
    top = H.levels[2]
    Kc = H.levels[1].K.toarray()
    Mc = _cycle_matrix(H, 1, 2)
    C = 2 * Mc - Mc @ Kc @ Mc                     # two visits from zero
    K = top.K.toarray()
    P = top.P.toarray()
    S = np.eye(K.shape[0]) - 0.6 * (K / top.diag[:, None])   # one sweep's error map
    I = np.eye(K.shape[0])
    pre = (I - S @ S) @ np.linalg.inv(K)          # two sweeps from zero
    # U = pre F; U += P C P^T (F - K U); two post-sweeps: U <- S U + (I - S) K^-1 F
    Kinv = np.linalg.inv(K)
    M_coarse = pre + P @ C @ P.T @ (I - K @ pre)
    M = S @ S @ M_coarse + (I - S @ S) @ Kinv
    np.testing.assert_allclose(_cycle_matrix(H, 2, 2), M, atol=1e-10 * np.abs(M).max())
    # and the V-cycle differs (one visit: C would be Mc alone)
    assert np.abs(_cycle_matrix(H, 2, 1) - M).max() > 1e-3 * np.abs(M).max()
