"""The cone filter on the GPU (mtomg_filter) against the oracle's filters.

Bar: FP64 with a different summation order than the oracle, so 1e-12
relative per element and 1e-13 in norm.  Grids cover one tile, ragged
tiles, a radius larger than the grid, radius <= 1 (no neighbours) and the
paper's rf = 8 (Table 2) at the 1024^2 workload size (sampled outputs from
the oracle's one-element loop).  The chain rule through the density filter
is checked end to end by finite differences of the GPU compliance.
"""

import numpy as np
import pytest
import torch

from oracle import cone_filter as cf
from tests.gpu_util import rel, relerr

pytestmark = pytest.mark.gpu

MODES = ["DENSITY", "DENSITY_ADJOINT", "SENSITIVITY"]
CASES = [(64, 32, 1, 1.5), (70, 37, 3, 2.5), (130, 70, 2, 8.0), (20, 9, 4, 16.0), (33, 65, 3, 0.7),
         (128, 96, 3, 3.0)]


@pytest.fixture(scope="module")
def solver():
    from paper_2301_07457_amd import PCGMGSolver
    return PCGMGSolver(max_designs=1)


def oracle(mode, x, g, rf):
    if mode == "DENSITY":
        return cf.density(g, rf)
    if mode == "DENSITY_ADJOINT":
        return cf.density_adjoint(g, rf)
    return cf.sensitivity(x, g, rf, 1e-3)


@pytest.mark.parametrize("nx,ny,m,rf", CASES, ids=lambda v: str(v))
@pytest.mark.parametrize("mode", MODES)
def test_filter_matches_oracle(solver, nx, ny, m, rf, mode):
    rng = np.random.default_rng(nx * 100 + ny + m)
    x = rng.random((ny, nx, m))
    x[rng.random((ny, nx)) < 0.2] = 0.0          # void elements hit the gmin floor
    g = rng.standard_normal((ny, nx, m))
    want = oracle(mode, x, g, rf)
    got = solver.filter(torch.from_numpy(g), rf, mode, torch.from_numpy(x)).cpu().numpy()
    assert relerr(got, want) < 1e-13, (mode, rel(got, want))
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())


def test_full_size_rf8_sampled(solver):
    """1024^2, three phases, rf = 8: sampled outputs (corners, edges, interior)
    against the oracle's one-element loop; constants pass the density filter."""
    n, m, rf = 1024, 3, 8.0
    rng = np.random.default_rng(42)
    x = rng.random((n, n, m))
    g = rng.standard_normal((n, n, m))
    xt, gt = torch.from_numpy(x).cuda(), torch.from_numpy(g).cuda()
    out = {mode: solver.filter(gt, rf, mode, xt).cpu().numpy() for mode in MODES}
    pts = [(0, 0), (n - 1, n - 1), (0, n - 1), (n - 1, 0), (3, 500), (700, 6), (511, 512), (1020, 333),
           (64, 32), (63, 31), (127, 96)]
    kinds = {"DENSITY": "density", "DENSITY_ADJOINT": "adjoint", "SENSITIVITY": "sensitivity"}
    for mode in MODES:
        for i, j in pts:
            want = cf.filter_at(g, i, j, rf, kinds[mode], x)
            np.testing.assert_allclose(out[mode][j, i], want, rtol=1e-12, atol=1e-13, err_msg=f"{mode} ({i},{j})")
    ones = solver.filter(torch.full((n, n, m), 0.25, dtype=torch.float64, device="cuda"), rf).cpu().numpy()
    np.testing.assert_allclose(ones, 0.25, rtol=1e-14)


def test_adjoint_identity_on_device(solver):
    rng = np.random.default_rng(9)
    a = torch.from_numpy(rng.standard_normal((384, 512, 2))).cuda()
    b = torch.from_numpy(rng.standard_normal((384, 512, 2))).cuda()
    lhs = torch.sum(solver.filter(a, 5.0, "DENSITY") * b).item()
    rhs = torch.sum(a * solver.filter(b, 5.0, "DENSITY_ADJOINT")).item()
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_filter_rejects_bad_arguments(solver):
    from paper_2301_07457_amd import _lib
    g = torch.zeros((8, 8, 1), dtype=torch.float64, device="cuda")
    for kw in (dict(rf=0.0), dict(rf=16.5), dict(rf=float("nan"))):
        with pytest.raises(RuntimeError):
            solver.filter(g, kw["rf"])
    with pytest.raises(RuntimeError):
        solver.filter(g, 2.0, "SENSITIVITY")          # no densities
    with pytest.raises(RuntimeError):                # out aliases in
        _lib.mtomg_filter(solver.ctx, 8, 8, 1, 2.0, "DENSITY", 1e-3, 0, g.data_ptr(), g.data_ptr())
    with pytest.raises(RuntimeError):                # more phases than designs allow
        big = torch.zeros((4, 4, 9), dtype=torch.float64, device="cuda")
        solver.filter(big, 2.0)


def test_density_filter_chain_rule_by_finite_differences():
    """c(x) = compliance of the design whose densities are the density-filtered x:
    the adjoint filter of the GPU gradient matches central differences of the
    GPU compliance (FP64 cycle, solves to 1e-12)."""
    from paper_2301_07457_amd import PCGMGSolver
    from workloads import make_problem
    p = make_problem("wall64")
    rf = 2.5
    s = PCGMGSolver(max_designs=1)
    s.add_design(0, p.nelx, p.nely, torch.from_numpy(p.F), list(p.E_phase), p.E_min, p.penal, p.nu,
                 p.levels, 2, 2, p.omega, "fp64")
    x0 = torch.from_numpy(p.x).cuda()

    def compliance(x):
        s.set_densities(0, s.filter(x, rf, "DENSITY"))
        st = s.solve(1e-12, 1000)[0]
        assert st["status"] == 0
        c, dc = s.compliance_and_grad(0)
        return c[0].item(), dc[0]

    c0, dc_t = compliance(x0)
    grad = s.filter(dc_t, rf, "DENSITY_ADJOINT").cpu().numpy()
    h = 1e-6
    for (j, i, k) in [(63, 10, 0), (40, 40, 1), (5, 60, 2), (62, 32, 0)]:
        xp = x0.clone()
        xp[j, i, k] += h
        xm = x0.clone()
        xm[j, i, k] -= h
        fd = (compliance(xp)[0] - compliance(xm)[0]) / (2 * h)
        assert fd == pytest.approx(grad[j, i, k], rel=1e-5, abs=1e-6 * np.abs(grad).max()), (j, i, k)
