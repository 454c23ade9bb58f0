"""Alternating active-phase optimality-criteria loop (Section 4) — TEST INFRASTRUCTURE ONLY.

The paper's optimiser is an optimality-criteria (OC) method that alternates
over pairs of active phases, in a Gauss-Seidel order, and treats each pair
as a binary sub-problem (Section 4 and its flowchart; parameters in Table
2).  It does not write the update out, so this module takes the following
reading (every choice is a parameter):

* Phases.  m solid phases plus void.  The void share is implicit,
  alpha_void = 1 - sum of the solid densities, and has no sensitivity (the
  modulus law of Eq. 5 is read with an implicit void phase, E = E_min +
  sum x_i^p (E_i - E_min)).  Every phase, void included, stays in
  [eps, 1] (the bounds of Eq. 6).
* Volumes.  Target fractions V_0 .. V_m (void last) with sum 1, as the
  volume fractions of Table 2; a pair update holds the volume of its first
  phase at its target, sum_e alpha_{e,a} = V_a N_e.
* One outer iteration visits every pair (a, b), a < b, in the order
  (0,1), (0,2), ..., (0,m), (1,2), ..., (m-1,m).  For each pair, with the
  densities left by the previous pair: solve the state equation, form the
  compliance gradient (summed over load cases), apply the sensitivity
  filter to each solid phase's gradient, then update the pair.
* Pair update.  With s_e = alpha_{e,a} + alpha_{e,b} held fixed per element
  (so alpha_b follows alpha_a), the pair sensitivity is
  d_e = g_{e,a} - g_{e,b} (g of the void is 0).  Bounds
  lo_e = max(eps, alpha_{e,a} - move), hi_e = min(1, s_e - eps, alpha_{e,a} + move)
  keep both phases in [eps, 1] and apply a move limit.  The OC step is
  y_e(lambda) = clamp(alpha_{e,a} (max(0, -d_e) / lambda)^eta, lo_e, hi_e),
  with lambda > 0 the multiplier of the volume constraint, chosen by
  bisection so that sum_e y_e(lambda) = V_a N_e.  Then alpha_a = y and
  alpha_b = s - y.
* Stop when the largest change of any density over an outer iteration is
  at most tol (Table 2: tol = 1e-3), or after a set number of iterations.

Densities are [nely][nelx][m] arrays of the solid phases, as everywhere.
Pinned by tests/test_oracle_oc.py: volume and per-element sums conserved,
bounds held, closed forms (eta = 1 without active bounds; a uniform pair
sensitivity), lambda against scipy's brentq root finder, the KKT sign
conditions at a fixed point of the update, and compliance falling over the
loop on a small wall.
"""

from __future__ import annotations

import numpy as np

from . import cone_filter, solve


def pair_bounds(ya: np.ndarray, s: np.ndarray, eps: float, move: float):
    """lo, hi of the pair update: both phases in [eps, 1], |change| <= move."""
    lo = np.maximum(eps, ya - move)
    hi = np.minimum(np.minimum(1.0, s - eps), ya + move)
    return lo, hi


def pair_candidate(ya, d, lo, hi, lam: float, eta: float) -> np.ndarray:
    """y(lambda) = clamp(ya (max(0, -d) / lambda)^eta, lo, hi); lambda = inf
    gives lo."""
    if lam <= 0.0:
        return np.where(-d > 0.0, hi, lo)
    return np.clip(ya * (np.maximum(0.0, -d) / lam) ** eta, lo, hi)


def pair_multiplier(ya, d, lo, hi, target: float, eta: float, rtol: float = 1e-13,
                    max_steps: int = 400) -> float:
    """lambda with sum_e y_e(lambda) = target, by bisection on [0, lambda_hi],
    lambda_hi the smallest multiplier that puts every element at lo.  The
    sum is non-increasing in lambda; a target above sum(y(0+)) drives
    lambda to 0 (every element with d < 0 at hi), a target at or below
    sum(lo) gives lambda = inf (every element at lo, exactly)."""
    g = np.maximum(0.0, -d)
    lam_hi = float(np.max(g * (ya / lo) ** (1.0 / eta))) if g.size else 0.0
    if lam_hi <= 0.0:
        return 0.0
    if target <= np.sum(lo):
        return np.inf          # every element exactly at lo
    l1, l2 = 0.0, lam_hi
    for _ in range(max_steps):
        mid = 0.5 * (l1 + l2)
        if np.sum(pair_candidate(ya, d, lo, hi, mid, eta)) > target:
            l1 = mid
        else:
            l2 = mid
        if l2 - l1 <= rtol * l2:
            break
    return 0.5 * (l1 + l2)


def pair_update(x: np.ndarray, a: int, b: int, g: np.ndarray, vol_a: float, move: float = 0.2,
                eta: float = 0.5, eps: float = 1e-3):
    """One binary sub-problem on phases a < b of the densities x
    [nely][nelx][m] (b = m is the void).  g: filtered compliance gradient
    [nely][nelx][m].  vol_a: target volume fraction of phase a.  Returns
    (new x, lambda, active) with active[e] = -1 at lo, +1 at hi, 0 between."""
    m = x.shape[-1]
    xa = x[..., a].ravel()
    xb = x[..., b].ravel() if b < m else 1.0 - x.sum(axis=-1).ravel()
    gb = g[..., b].ravel() if b < m else np.zeros_like(xa)
    d = g[..., a].ravel() - gb
    s = xa + xb
    lo, hi = pair_bounds(xa, s, eps, move)
    target = vol_a * xa.size
    lam = pair_multiplier(xa, d, lo, hi, target, eta)
    y = pair_candidate(xa, d, lo, hi, lam, eta)
    out = x.copy()
    out[..., a] = y.reshape(x.shape[:-1])
    if b < m:
        out[..., b] = (s - y).reshape(x.shape[:-1])
    active = np.where(y <= lo, -1, np.where(y >= hi, 1, 0))
    return out, lam, active


def pairs(m: int):
    """The Gauss-Seidel order of the pairs over m solid phases and the void (index m)."""
    return [(a, b) for a in range(m) for b in range(a + 1, m + 1)]


def analysis(p, x):
    """Compliance summed over load cases and its gradient (plain definition:
    direct solve), for densities x."""
    sol = solve.solve_direct(p.nelx, p.nely, x, p.E_phase, p.E_min, p.penal, p.nu, p.F, grad=True)
    return float(np.sum(sol.c)), sol.dcdx.sum(axis=0)


def aap_iteration(p, x, vols, rf: float = 8.0, move: float = 0.2, eta: float = 0.5, eps: float = 1e-3,
                  gmin: float = 1e-3):
    """One outer iteration over every pair, each with a fresh analysis.
    Returns (new x, [compliance before each pair update], largest density change)."""
    x0 = x.copy()
    cs = []
    for a, b in pairs(x.shape[-1]):
        c, g = analysis(p, x)
        cs.append(c)
        g = cone_filter.sensitivity(x, g, rf, gmin)
        x, _, _ = pair_update(x, a, b, g, vols[a], move, eta, eps)
    void0 = 1.0 - x0.sum(axis=-1)
    void1 = 1.0 - x.sum(axis=-1)
    change = max(float(np.max(np.abs(x - x0))), float(np.max(np.abs(void1 - void0))))
    return x, cs, change


def initial_design(nelx: int, nely: int, vols) -> np.ndarray:
    """Uniform start at the target fractions of the solid phases."""
    m = len(vols) - 1
    return np.broadcast_to(np.asarray(vols[:m], dtype=np.float64), (nely, nelx, m)).copy()
