"""Pins for the oracle's finite-element model (Section 3, Eqs. 5-10).

Each check compares the oracle with something it does not compute itself:
closed forms derived by hand from Eqs. (7)-(9), printed mesh facts,
spectral facts, exact invariants and an independent brute-force table.
"""

import json
import os

import numpy as np
import pytest

from oracle import fe, solve
from workloads import load_top_traction

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def ke_closed_form(nu):
    """Hand-integrated unit-modulus Q4 plane-stress stiffness (square element)."""
    a = 0.5 - nu / 6
    b = 0.125 + nu / 8
    c = -0.25 - nu / 12
    d = -0.125 + 3 * nu / 8
    e = -0.25 + nu / 12
    f = -0.125 - nu / 8
    g = nu / 6
    k = 0.125 - 3 * nu / 8
    M = np.array([
        [a, b, c, d, e, f, g, k],
        [b, a, k, g, f, e, d, c],
        [c, k, a, f, g, d, e, b],
        [d, g, f, a, k, c, b, e],
        [e, f, g, k, a, b, c, d],
        [f, e, d, c, b, a, k, g],
        [g, d, e, b, c, k, a, f],
        [k, c, b, e, d, g, f, a],
    ])
    return M / (1 - nu * nu)


@pytest.mark.parametrize("nu", [0.0, 0.3, 0.45])
def test_element_stiffness_matches_closed_form(nu):
    np.testing.assert_allclose(fe.element_stiffness(nu), ke_closed_form(nu), rtol=0, atol=1e-14)


def test_element_stiffness_row0_values():
    row0 = [0.494505494505, 0.178571428571, -0.302197802198, -0.013736263736,
            -0.247252747253, -0.178571428571, 0.054945054945, 0.013736263736]
    np.testing.assert_allclose(fe.element_stiffness(0.3)[0], row0, atol=1e-12)


@pytest.mark.parametrize("nu", [0.0, 0.3, 0.45])
def test_element_stiffness_spectrum(nu):
    ev = np.sort(np.linalg.eigvalsh(fe.element_stiffness(nu)))
    want = np.sort([0, 0, 0, 1 / (1 + nu), 1 / (1 + nu), (3 - nu) / (6 * (1 - nu ** 2)),
                    (3 - nu) / (6 * (1 - nu ** 2)), 1 / (1 - nu)])
    np.testing.assert_allclose(ev, want, atol=1e-13)


def test_element_stiffness_h_independent_and_rigid_modes():
    for h in (1.0, 0.125, 1.0 / 1024):
        np.testing.assert_allclose(fe.element_stiffness(0.3, h), fe.element_stiffness(0.3), atol=1e-13)
    R = fe.rigid_body_modes(1, 1, 1.0)[:, fe.element_dof_map(1, 1)[0]]
    assert np.abs(fe.element_stiffness(0.3) @ R.T).max() < 1e-15


def test_node_count_printed_in_paper():
    g = json.load(open(os.path.join(GOLD, "paper_node_counts.json")))
    for m in g["meshes"]:
        dofs = fe.element_dof_map(m["nelx"], m["nely"])
        assert dofs.max() // 2 + 1 == m["nodes"]
        assert len(fe.free_dofs(m["nelx"], m["nely"])) == 2 * (m["nodes"] - (m["nelx"] + 1))


def test_interpolation_special_cases():
    E_ph = np.array([1.0, 0.6, 0.2])
    x = np.zeros((2, 2, 3))
    assert np.all(fe.interpolate_modulus(x, E_ph, 1e-9, 3.0) == 1e-9)
    for i in range(3):
        x1 = np.zeros((1, 1, 3))
        x1[0, 0, i] = 1.0
        assert fe.interpolate_modulus(x1, E_ph, 1e-9, 3.0)[0, 0] == pytest.approx(E_ph[i], abs=1e-16)
    # SIMP penalty: half density of phase 0 gives 1/8 of its modulus gap
    x1 = np.zeros((1, 1, 3)); x1[0, 0, 0] = 0.5
    assert fe.interpolate_modulus(x1, E_ph, 1e-9, 3.0)[0, 0] == pytest.approx(1e-9 + (1 - 1e-9) / 8, rel=1e-15)


def test_assembled_stiffness_symmetric_rigid_and_spd():
    rng = np.random.default_rng(3)
    nx, ny = 6, 4
    E = rng.uniform(0.01, 1, (ny, nx))
    K = fe.assemble_stiffness(nx, ny, E, 0.3)
    assert abs(K - K.T).max() < 1e-15
    R = fe.rigid_body_modes(nx, ny, 1.0 / nx)
    assert np.abs(K @ R.T).max() < 1e-13
    free = fe.free_dofs(nx, ny)
    Kff = fe.restrict_to_free(K, free).toarray()
    assert np.linalg.eigvalsh(Kff).min() > 0


@pytest.mark.parametrize("nu,E", [(0.3, 1.0), (0.0, 1.0), (0.25, 3.5)])
def test_single_element_closed_form_compliance(nu, E):
    # one element, bottom clamped, unit total traction on top:
    # c = (9 - nu)(1 - nu^2) / (E (9 - nu - 6 nu^2))
    x = np.ones((1, 1, 1))
    F = load_top_traction(1, 1)[None]
    s = solve.solve_direct(1, 1, x, [E], 1e-9, 3.0, nu, F, grad=False, dense_cholesky=True)
    want = (9 - nu) * (1 - nu ** 2) / (E * (9 - nu - 6 * nu ** 2))
    assert s.c[0] == pytest.approx(want, rel=1e-13)


def test_uniform_wall_refinement_table():
    g = json.load(open(os.path.join(GOLD, "uniform_wall_compliance.json")))
    prev = 0.0
    for ns, want in sorted(g["compliance"].items(), key=lambda kv: int(kv[0])):
        n = int(ns)
        x = np.ones((n, n, 1))
        F = load_top_traction(n, n)[None]
        s = solve.solve_direct(n, n, x, [1.0], 1e-9, 3.0, g["nu"], F, grad=False)
        assert s.c[0] == pytest.approx(want, rel=1e-11)
        # conforming FE: compliance grows under nested refinement
        assert s.c[0] > prev
        prev = s.c[0]


def _random_problem(n, seed, m=3):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.05, 1.0, (n, n, m)) / m
    return x, np.array([1.0, 0.6, 0.2][:m]), 1e-9, 3.0, 0.3, load_top_traction(n, n)[None]


def test_compliance_identities_and_scaling():
    n = 8
    x, Eph, Emin, p, nu, F = _random_problem(n, 4)
    s = solve.solve_direct(n, n, x, Eph, Emin, p, nu, F)
    U = s.U[0].ravel()
    E = fe.interpolate_modulus(x, Eph, Emin, p)
    K = fe.assemble_stiffness(n, n, E, nu)
    assert s.c[0] == pytest.approx(U @ (K @ U), rel=1e-12)
    energy = np.sum(E * fe.element_energies(U, n, n, nu))
    assert s.c[0] == pytest.approx(energy, rel=1e-12)
    # scaling every modulus by 7 scales u and c by 1/7
    s7 = solve.solve_direct(n, n, x, 7 * Eph, 7 * Emin, p, nu, F)
    np.testing.assert_allclose(s7.U, s.U / 7, rtol=1e-10, atol=1e-14)


def test_gradient_finite_difference_and_euler_identity():
    n = 8
    x, Eph, Emin, p, nu, F = _random_problem(n, 5)
    s = solve.solve_direct(n, n, x, Eph, Emin, p, nu, F)
    g = s.dcdx[0]
    assert np.all(g <= 0)
    rng = np.random.default_rng(6)
    for _ in range(12):
        j, i, ph = rng.integers(0, n), rng.integers(0, n), rng.integers(0, 3)
        hstep = 1e-6
        xp = x.copy(); xp[j, i, ph] += hstep
        xm = x.copy(); xm[j, i, ph] -= hstep
        cp = solve.solve_direct(n, n, xp, Eph, Emin, p, nu, F, grad=False).c[0]
        cm = solve.solve_direct(n, n, xm, Eph, Emin, p, nu, F, grad=False).c[0]
        fd = (cp - cm) / (2 * hstep)
        assert fd == pytest.approx(g[j, i, ph], rel=1e-5)
    # Euler identity for the degree-p homogeneous part of E(x)
    U = s.U[0].ravel()
    w = fe.element_energies(U, n, n, nu)
    lhs = np.sum(x * g)
    rhs = -p * (s.c[0] - Emin * np.sum(w))
    assert lhs == pytest.approx(rhs, rel=1e-12)
