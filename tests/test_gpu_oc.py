"""The alternating active-phase OC update on the GPU against the oracle (Section 4).

* mtomg_oc_update (one binary sub-problem) against oracle.oc.pair_update on
  random valid densities: every pair of m = 3 solid phases and the void,
  targets above, below and at the current volume and beyond reach, grids
  from one workgroup to more than the 1,024 workgroups of a pass (grid-
  stride loops), ragged sizes.  The bar: the new densities to 1e-9
  absolute (the multiplier is found to ~1e-14 of the volume on either side,
  which moves the few elements between their bounds by at most that much
  in total), the volume to 1e-12 relative, lambda to 1e-8 relative where
  some element lies between its bounds, and bit-exact equality wherever the
  oracle's element sits on a bound with a margin (the bounds are the same
  IEEE expressions on both sides).
* mtomg_aap_step (one outer iteration: solve, gradient, filter, update for
  every pair) against oracle.oc.aap_iteration on a small wall with the
  moduli and volume fractions of Table 2: compliance before each pair, the
  densities and the largest change after each of two iterations.
"""

import numpy as np
import pytest
import torch

from oracle import oc
from workloads import Problem, load_top_traction

pytestmark = pytest.mark.gpu


def random_state(rng, ny, nx, m=3, eps=1e-3):
    w = rng.random((ny * nx, m + 1)) ** 2 + 0.02
    w /= w.sum(axis=1, keepdims=True)
    w = eps + (1 - (m + 1) * eps) * w
    return w[:, :m].reshape(ny, nx, m).copy()


def random_gradient(rng, x):
    g = -np.exp(rng.normal(0, 1.5, x.shape)) * np.array([3.0, 2.0, 1.0])
    g[rng.random(x.shape) < 0.05] *= -0.1      # a few entries of the other sign
    return g


SHAPES = [(1, 1), (7, 5), (70, 37), (300, 200), (600, 512)]


@pytest.mark.parametrize("ny,nx", SHAPES, ids=lambda v: str(v))
@pytest.mark.parametrize("a,b", [(0, 1), (0, 3), (1, 2), (2, 3)])
@pytest.mark.parametrize("scale", [0.9, 1.0, 1.07])
def test_pair_update_matches_oracle(ny, nx, a, b, scale):
    from paper_2301_07457_amd import PCGMGSolver
    rng = np.random.default_rng(ny * 1000 + nx + 10 * a + b)
    x = random_state(rng, ny, nx)
    g = random_gradient(rng, x)
    vol = float(x[..., a].mean()) * scale
    want, lam, active = oc.pair_update(x, a, b, g, vol, move=0.2, eta=0.5, eps=1e-3)
    s = PCGMGSolver(max_designs=1)
    xt = torch.from_numpy(x).cuda()
    info = s.oc_update(xt, torch.from_numpy(g), a, b, vol, move=0.2, eta=0.5, eps=1e-3)
    got = xt.cpu().numpy()
    print(f"[oc {ny}x{nx} ({a},{b}) x{scale}] lambda={info[0]:.9e} (oracle {lam:.9e}) passes={info[3]}")
    assert np.max(np.abs(got - want)) <= 1e-9
    n = ny * nx
    ya = x[..., a].ravel()
    d = g[..., a].ravel() - (g[..., b].ravel() if b < 3 else 0.0)
    lo, hi = oc.pair_bounds(ya, ya + (x[..., b].ravel() if b < 3 else 1 - x.sum(-1).ravel()), 1e-3, 0.2)
    # the volume meets its target wherever the target is reachable
    if lo.sum() < vol * n < np.where(d < 0, hi, lo).sum():
        assert abs(got[..., a].sum() - vol * n) <= 1e-12 * vol * n
    # elements on a bound with a margin: the same bits
    cand = oc.pair_candidate(ya, d, -np.inf, np.inf, lam, 0.5) if 0 < lam < np.inf else np.zeros_like(ya)
    firm = ((active.ravel() == -1) & (cand < lo * (1 - 1e-7))) | ((active.ravel() == 1) & (cand > hi * (1 + 1e-7)))
    assert np.array_equal(got[..., a].ravel()[firm], want[..., a].ravel()[firm])
    if np.any(active == 0):
        assert info[0] == pytest.approx(lam, rel=1e-8)
    assert info[3] == int(info[3]) and info[3] < 24, info   # converged within the pass limit


@pytest.mark.parametrize("vol", [0.0, 1.0])
def test_pair_update_unreachable_target(vol):
    """A target below (above) every reachable volume: every element at its
    lower bound (every element preferring phase a at its upper one)."""
    from paper_2301_07457_amd import PCGMGSolver
    rng = np.random.default_rng(3)
    x = random_state(rng, 40, 30)
    g = random_gradient(rng, x)
    want, _, _ = oc.pair_update(x, 0, 3, g, vol, move=0.2, eta=0.5, eps=1e-3)
    s = PCGMGSolver(max_designs=1)
    xt = torch.from_numpy(x).cuda()
    s.oc_update(xt, torch.from_numpy(g), 0, 3, vol)
    assert np.array_equal(xt.cpu().numpy(), want)


def test_pair_update_rejects_bad_arguments():
    from paper_2301_07457_amd import PCGMGSolver, _lib
    s = PCGMGSolver(max_designs=1)
    x = torch.full((4, 4, 3), 0.2, dtype=torch.float64, device="cuda")
    g = torch.zeros_like(x)
    for kw in (dict(a=1, b=1), dict(a=0, b=4), dict(a=-1, b=2)):
        with pytest.raises(_lib.MtomgError):
            s.oc_update(x, g, kw["a"], kw["b"], 0.2)
    with pytest.raises(_lib.MtomgError):
        s.oc_update(x, g, 0, 1, 1.5)
    with pytest.raises(_lib.MtomgError):
        s.oc_update(x, g, 0, 1, 0.2, eps=0.2)


def table2_wall(n):
    return Problem("oc", n, n, np.zeros((n, n, 3)), np.array([9.0, 3.0, 1.0]), 1e-9, 3.0, 0.3,
                   load_top_traction(n, n)[None], 3)


@pytest.mark.parametrize("n,rf", [(32, 2.0), (48, 8.0)])
def test_aap_step_matches_oracle(n, rf):
    """Two outer iterations from the uniform start, Table 2 moduli and volume
    fractions: the GPU step (pCGMG to 1e-11, FP64) against the oracle's
    (direct solves)."""
    from paper_2301_07457_amd import PCGMGSolver
    p = table2_wall(n)
    vols = [0.16, 0.08, 0.08, 0.68]
    x_or = oc.initial_design(n, n, vols)
    s = PCGMGSolver(max_designs=1)
    s.add_design(0, n, n, torch.from_numpy(p.F), list(p.E_phase), p.E_min, p.penal, p.nu, p.levels, 2, 2, 0.6, "fp64")
    xt = torch.from_numpy(x_or.copy()).cuda()
    for it in range(2):
        x_or, cs_or, ch_or = oc.aap_iteration(p, x_or, vols, rf=rf)
        cs, ch, iters = s.aap_step(0, xt, vols, rf=rf, rel_tol=1e-11, max_iter=2000)
        got = xt.cpu().numpy()
        print(f"[aap {n} rf={rf} it {it}] c={cs} (oracle {cs_or}) change={ch:.6f} (oracle {ch_or:.6f}) "
              f"iters={iters} max|dx|={np.max(np.abs(got - x_or)):.2e}")
        np.testing.assert_allclose(cs, cs_or, rtol=1e-8)
        assert np.max(np.abs(got - x_or)) <= 1e-6
        assert ch == pytest.approx(ch_or, abs=1e-6)
        for k in range(3):
            assert got[..., k].mean() == pytest.approx(vols[k], rel=1e-10)


def test_aap_step_sums_load_cases_like_the_oracle():
    """Four load cases (top traction, corner and midpoint point loads, left
    shear): the step's objective and gradient are the sums over the cases,
    as in the oracle's loop."""
    from paper_2301_07457_amd import PCGMGSolver
    from workloads import four_load_cases
    n = 32
    p = table2_wall(n)
    p.F = four_load_cases(n, n)
    vols = [0.16, 0.08, 0.08, 0.68]
    x_or = oc.initial_design(n, n, vols)
    s = PCGMGSolver(max_designs=1)
    s.add_design(0, n, n, torch.from_numpy(p.F), list(p.E_phase), p.E_min, p.penal, p.nu, p.levels, 2, 2, 0.6, "fp64")
    xt = torch.from_numpy(x_or.copy()).cuda()
    x_or, cs_or, ch_or = oc.aap_iteration(p, x_or, vols, rf=2.0)
    cs, ch, iters = s.aap_step(0, xt, vols, rf=2.0, rel_tol=1e-11, max_iter=2000)
    np.testing.assert_allclose(cs, cs_or, rtol=1e-8)
    assert np.max(np.abs(xt.cpu().numpy() - x_or)) <= 1e-6
    assert ch == pytest.approx(ch_or, abs=1e-6)
