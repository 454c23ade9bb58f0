"""Pins of the oracle's alternating active-phase OC loop (Section 4, Table 2).

The paper does not print the update, so the pins are what any correct
reading of an OC pair update must satisfy: conservation (the pair's sum per
element, the first phase's volume), the bounds, closed forms where the
bisection has an exact answer, an independent root finder for the
multiplier, the KKT sign conditions of the binary sub-problem at a fixed
point of the update, and a falling compliance over a few outer iterations
on a small wall.  A wrong sign of the pair sensitivity, a swapped phase or
a wrong exponent fails at least one of them.
"""

import numpy as np
import pytest
import scipy.optimize

from oracle import oc, solve
from workloads import Problem, load_top_traction


def random_state(rng, n=300, m=3, eps=1e-3):
    """Valid densities: every solid phase and the void in [eps, 1]."""
    w = rng.random((n, m + 1)) + 0.05
    w /= w.sum(axis=1, keepdims=True)
    w = eps + (1 - (m + 1) * eps) * w
    return w[:, :m].reshape(1, n, m)


@pytest.mark.parametrize("a,b", [(0, 1), (0, 3), (1, 2), (2, 3)])
def test_pair_update_conserves_sums_and_bounds(a, b):
    rng = np.random.default_rng(10 * a + b)
    x = random_state(rng)
    g = -rng.random(x.shape) * np.array([3.0, 2.0, 1.0])
    xa = x[..., a]
    vol = float(xa.mean()) * 1.05
    y, lam, active = oc.pair_update(x, a, b, g, vol, move=0.2, eta=0.5, eps=1e-3)
    assert lam > 0
    # the first phase's volume meets its target
    assert abs(y[..., a].sum() - vol * xa.size) <= 1e-10 * vol * xa.size
    # the pair's sum per element is unchanged; the other phases untouched
    void0, void1 = 1 - x.sum(-1), 1 - y.sum(-1)
    sb0 = x[..., b] if b < 3 else void0
    sb1 = y[..., b] if b < 3 else void1
    np.testing.assert_allclose(y[..., a] + sb1, x[..., a] + sb0, rtol=0, atol=1e-15)
    for k in range(3):
        if k not in (a, b):
            assert np.array_equal(y[..., k], x[..., k])
    # every phase, void included, in [eps, 1]; the move limit holds
    assert np.all(y >= 1e-3 - 1e-15) and np.all(void1 >= 1e-3 - 1e-15) and np.all(y <= 1)
    assert np.all(np.abs(y[..., a] - x[..., a]) <= 0.2 + 1e-15)
    assert set(np.unique(active)) <= {-1, 0, 1}


@pytest.mark.parametrize("eta", [1.0, 0.5])
def test_multiplier_closed_form_without_active_bounds(eta):
    """No active bound: y = ya (-d / lambda)^eta, so sum y = target gives
    lambda = (sum(ya (-d)^eta) / target)^(1/eta) exactly; with the target
    of lambda = 1, y = ya (-d)^eta."""
    rng = np.random.default_rng(1)
    n = 500
    ya = rng.uniform(0.3, 0.6, n)
    d = -rng.uniform(1.0, 1.5, n)
    s = np.full(n, 0.95)
    lo, hi = oc.pair_bounds(ya, s, 1e-3, 10.0)
    target = float(np.sum(ya * (-d) ** eta))   # lambda = 1 puts every y inside (0.3, 0.9)
    lam = oc.pair_multiplier(ya, d, lo, hi, target, eta=eta)
    assert lam == pytest.approx(1.0, rel=1e-12)
    y = oc.pair_candidate(ya, d, lo, hi, lam, eta)
    np.testing.assert_allclose(y, ya * (-d) ** eta, rtol=1e-12)
    # another target: the multiplier scales as (target ratio)^(-1/eta)
    lam2 = oc.pair_multiplier(ya, d, lo, hi, 0.9 * target, eta=eta)
    assert lam2 == pytest.approx(0.9 ** (-1.0 / eta), rel=1e-12)


def test_uniform_pair_sensitivity_scales_uniformly():
    """The same pair sensitivity everywhere: the update is a uniform scaling
    y = ya * target / sum(ya), whatever eta."""
    rng = np.random.default_rng(2)
    n = 400
    ya = rng.uniform(0.2, 0.4, n)
    d = np.full(n, -0.7)
    s = np.full(n, 0.9)
    lo, hi = oc.pair_bounds(ya, s, 1e-3, 0.5)
    target = 1.1 * ya.sum()
    for eta in (0.3, 0.5, 1.0):
        lam = oc.pair_multiplier(ya, d, lo, hi, target, eta)
        y = oc.pair_candidate(ya, d, lo, hi, lam, eta)
        np.testing.assert_allclose(y, ya * 1.1, rtol=1e-11)


@pytest.mark.parametrize("seed", range(4))
def test_multiplier_matches_brentq(seed):
    """Active bounds on both sides: lambda from the bisection equals the root
    of sum(y(lambda)) - target from scipy's brentq."""
    rng = np.random.default_rng(seed)
    n = 1000
    ya = rng.uniform(0.01, 0.9, n)
    s = np.minimum(1.0, ya + rng.uniform(0.01, 0.5, n))
    d = -np.exp(rng.normal(0, 2, n))
    d[rng.random(n) < 0.1] *= -1          # some elements prefer the other phase
    lo, hi = oc.pair_bounds(ya, s, 1e-3, 0.2)
    target = float(ya.sum()) * rng.uniform(0.9, 1.1)
    lam = oc.pair_multiplier(ya, d, lo, hi, target, 0.5)
    f = lambda t: float(np.sum(oc.pair_candidate(ya, d, lo, hi, t, 0.5))) - target
    lam_hi = float(np.max(np.maximum(0, -d) * (ya / lo) ** 2))
    ref = scipy.optimize.brentq(f, 1e-300, lam_hi, xtol=1e-300, rtol=1e-14, maxiter=2000)
    y = oc.pair_candidate(ya, d, lo, hi, lam, 0.5)
    yr = oc.pair_candidate(ya, d, lo, hi, ref, 0.5)
    assert lam == pytest.approx(ref, rel=1e-10)
    np.testing.assert_allclose(y, yr, rtol=0, atol=1e-10)
    assert abs(y.sum() - target) <= 1e-9 * target


def test_fixed_point_satisfies_kkt():
    """With a fixed (linear) objective the repeated update converges to the
    solution of min sum d_e y_e s.t. sum y = V, lo <= y <= hi: elements at
    the upper bound have -d >= lambda, those at the lower bound -d <=
    lambda, and those between (they carry the fraction) have -d = lambda."""
    rng = np.random.default_rng(5)
    n = 200
    m = 1
    x = np.full((1, n, m), 0.4)
    # pair sensitivities 1.5 % apart, so the iteration settles in a few hundred steps
    g = -np.exp(rng.permutation(np.linspace(0.0, 3.0, n))).reshape(1, n, m)
    for _ in range(5000):
        y, lam, active = oc.pair_update(x, 0, 1, g, 0.4, move=0.2, eta=0.5, eps=1e-3)
        if np.max(np.abs(y - x)) <= 1e-12:
            break
        x = y
    assert np.max(np.abs(y - x)) <= 1e-12        # a fixed point
    mg = -g.ravel()
    at_hi = y.ravel() >= 1 - 1e-3 - 1e-12
    at_lo = y.ravel() <= 1e-3 + 1e-12
    assert np.all(mg[at_hi] >= lam * (1 - 1e-9))
    assert np.all(mg[at_lo] <= lam * (1 + 1e-9))
    # an element between its bounds is stationary only where -d equals lambda
    inner = ~(at_hi | at_lo)
    assert np.all(np.abs(mg[inner] / lam - 1) <= 1e-8)
    # so the material sits on the elements of largest -d: a threshold split
    assert mg[at_hi].min() >= mg[at_lo].max()
    assert 75 <= at_hi.sum() <= 80


def table2_wall(n=16):
    """A small square wall with the moduli of Table 2 (three materials and
    void) and a unit top traction."""
    m = 3
    x = np.zeros((n, n, m))
    return Problem("oc", n, n, x, np.array([9.0, 3.0, 1.0]), 1e-9, 3.0, 0.3, load_top_traction(n, n)[None], 3)


def test_aap_loop_lowers_compliance_and_meets_volumes():
    """Three outer iterations from the uniform start at the Table 2 volume
    fractions: every phase ends each iteration at its volume target, every
    density (void included) in [eps, 1], and the compliance falls."""
    p = table2_wall(16)
    vols = [0.16, 0.08, 0.08, 0.68]
    x = oc.initial_design(p.nelx, p.nely, vols)
    c_first = None
    c_last = None
    for it in range(3):
        x, cs, change = oc.aap_iteration(p, x, vols, rf=2.0)
        c_first = cs[0] if c_first is None else c_first
        c_last = cs[-1]
        assert change > 0
        for k in range(3):
            assert x[..., k].mean() == pytest.approx(vols[k], rel=1e-9)
        void = 1 - x.sum(-1)
        assert void.mean() == pytest.approx(vols[3], rel=1e-9)
        assert x.min() >= 1e-3 - 1e-12 and void.min() >= 1e-3 - 1e-12 and x.max() <= 1.0
    c_end, _ = oc.analysis(p, x)
    assert c_end < 0.8 * c_first, (c_first, c_last, c_end)
    # the analysis is the plain definition: the direct solve's compliance
    sol = solve.solve_direct(p.nelx, p.nely, x, p.E_phase, p.E_min, p.penal, p.nu, p.F, grad=False)
    assert c_end == pytest.approx(float(sol.c.sum()), rel=1e-14)
