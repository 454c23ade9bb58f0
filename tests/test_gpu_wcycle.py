"""The W-cycle (cycle index gamma = 2 of Algorithm 1, Section 2.1) on the GPU.

One preconditioner application from every level is compared element by
element with the oracle's gamma-cycle (same bars as the V-cycle: 2e-11
relative in FP64, 1e-5 in FP32), for several sweep counts, including
n_pre = 0 (the second visit of a level then starts by copying the first
visit's result) and n_post = 0.  PCG with the W-cycle matches the oracle's
pCGMG with gamma = 2 in iteration count (within 1) and the direct solution
to 1e-6; graph replay, batching of two designs and switching the option on
a live solver give the same bits as eager, solo and fresh runs.
"""

import numpy as np
import pytest
import torch

from oracle import multigrid, solve
from tests.gpu_util import OracleLevels, free_of, gpu_solver, rel, relerr
from workloads import Problem, load_top_traction

pytestmark = pytest.mark.gpu


def rand_prob(nx, ny, L, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.05, 1.0, (ny, nx, 3)) / 3
    return Problem("rand", nx, ny, x, np.array([1.0, 0.6, 0.2]), 1e-9, 3.0, 0.3,
                   load_top_traction(nx, ny)[None], L)


def rnd_nodal(rng, nx, ny):
    v = rng.standard_normal((ny + 1, nx + 1, 2))
    v[0] = 0.0
    return v


def cycle_gpu(s, prec, level, b):
    dt = torch.float64 if prec == "fp64" else torch.float32
    t = torch.from_numpy(np.ravel(b)).to("cuda", dt)
    out = s.debug_apply(0, level, "VCYCLE", t, b.shape, dt)
    torch.cuda.synchronize()
    return out.double().cpu().numpy()


@pytest.mark.parametrize("sweeps", [(2, 2), (0, 2), (3, 1), (1, 0)], ids=lambda p: f"pre{p[0]}-post{p[1]}")
@pytest.mark.parametrize("prec", ["fp64", "fp32mg"])
def test_w_cycle_every_level_matches_oracle(sweeps, prec):
    n_pre, n_post = sweeps
    nx0, ny0, L = 124, 60, 3
    prob = rand_prob(nx0, ny0, L, 11)
    o = OracleLevels(nx0, ny0, prob.x, prob.E_phase, prob.E_min, prob.penal, prob.nu, L)
    s = gpu_solver(prob, prec, n_pre=n_pre, n_post=n_post)
    s.set_option("GAMMA", 2)
    rng = np.random.default_rng(n_pre * 10 + n_post)
    bar = 2e-11 if prec == "fp64" else 1e-5
    for l in range(1, L):
        nx, ny = o.dims(l)
        b = rnd_nodal(rng, nx, ny)
        want = multigrid.cycle(o.H, l, free_of(b, nx), None, prob.omega, n_pre, n_post, gamma=2)
        got = cycle_gpu(s, prec, l, b)
        assert relerr(free_of(got, nx), want) < bar, (prec, sweeps, l)
        # the V-cycle differs from it (the option is really in effect)
        v = multigrid.cycle(o.H, l, free_of(b, nx), None, prob.omega, n_pre, n_post, gamma=1)
        if l >= 2:
            assert rel(want, v) > 100 * bar


@pytest.mark.parametrize("prec", ["fp64", "fp32mg"])
def test_w_cycle_deep_hierarchy(prec):
    """Five levels down to a 4 x 2 coarsest grid: level 1 is visited eight
    times per application, each with its own exact coarse solve."""
    nx0, ny0, L = 64, 32, 5
    prob = rand_prob(nx0, ny0, L, 12)
    o = OracleLevels(nx0, ny0, prob.x, prob.E_phase, prob.E_min, prob.penal, prob.nu, L)
    s = gpu_solver(prob, prec)
    s.set_option("GAMMA", 2)
    rng = np.random.default_rng(5)
    nx, ny = o.dims(L - 1)
    b = rnd_nodal(rng, nx, ny)
    want = multigrid.cycle(o.H, L - 1, free_of(b, nx), None, prob.omega, 2, 2, gamma=2)
    got = cycle_gpu(s, prec, L - 1, b)
    assert relerr(free_of(got, nx), want) < (2e-11 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("prec", ["fp64", "fp32mg"])
def test_w_cycle_pcg_matches_oracle(prec):
    p = rand_prob(128, 64, 4, 13)
    print(f"[w-cycle pcg] {prec}", flush=True)
    ref = solve.solve_direct(p.nelx, p.nely, p.x, p.E_phase, p.E_min, p.penal, p.nu, p.F)
    o = solve.solve_mgpcg(p.nelx, p.nely, p.x, p.E_phase, p.E_min, p.penal, p.nu, p.F, p.levels,
                          rel_tol=1e-8, grad=False, gamma=2)
    s = gpu_solver(p, prec)
    st_v = s.solve(1e-8, 1000)[0]
    U_v = s.U(0).clone()
    s.set_option("GAMMA", 2)
    st = s.solve(1e-8, 1000)[0]
    assert st["status"] == 0 and st["relres_true"] <= 1.05e-8, st
    assert abs(st["iters"] - o.iters[0]) <= 1, (st["iters"], o.iters)
    assert st["iters"] <= st_v["iters"], (st["iters"], st_v["iters"])
    U = s.U(0).clone()
    assert relerr(U.cpu().numpy(), ref.U) <= 1e-6
    assert not torch.equal(U, U_v)
    # eager launches give the same bits as the captured graphs
    s.set_option("GRAPHS", 0)
    st2 = s.solve(1e-8, 1000)[0]
    assert st2["iters"] == st["iters"] and torch.equal(s.U(0), U)
    # a fresh solver with the W-cycle from the start gives the same bits
    f = gpu_solver(p, prec)
    f.set_option("GAMMA", 2)
    st3 = f.solve(1e-8, 1000)[0]
    assert st3["iters"] == st["iters"] and torch.equal(f.U(0), U)
    # and back to the V-cycle
    s.set_option("GRAPHS", 1)
    s.set_option("GAMMA", 1)
    st4 = s.solve(1e-8, 1000)[0]
    assert st4["iters"] == st_v["iters"] and torch.equal(s.U(0), U_v)


def test_w_cycle_two_designs_in_one_group_equal_solo():
    from paper_2301_07457_amd import PCGMGSolver
    probs = [rand_prob(64, 64, 3, 21), rand_prob(64, 64, 3, 22)]

    def add(s, k, p):
        s.add_design(k, p.nelx, p.nely, torch.from_numpy(p.F), list(p.E_phase), p.E_min, p.penal, p.nu,
                     p.levels, 2, 2, p.omega, "fp32mg")

    s = PCGMGSolver(max_designs=2)
    for k, p in enumerate(probs):
        add(s, k, p)
    s.set_option("GAMMA", 2)
    for k, p in enumerate(probs):
        s.set_densities(k, torch.from_numpy(p.x))
    st = s.solve(1e-8, 1000)
    assert len(st) == 2 and all(a["status"] == 0 for a in st)
    for k, p in enumerate(probs):
        solo = PCGMGSolver(max_designs=1)
        add(solo, 0, p)
        solo.set_option("GAMMA", 2)
        solo.set_densities(0, torch.from_numpy(p.x))
        st1 = solo.solve(1e-8, 1000)
        assert st1[0]["iters"] == st[k]["iters"]
        assert torch.equal(solo.U(0), s.U(k)), k


def test_gamma_option_rejects_other_values():
    from paper_2301_07457_amd import PCGMGSolver
    s = PCGMGSolver(max_designs=1)
    for bad in (0, 3, -1):
        with pytest.raises(RuntimeError):
            s.set_option("GAMMA", bad)


@pytest.mark.parametrize("levels", [4, 5, 6, 7, 8])
@pytest.mark.parametrize("gamma", [1, 2])
def test_level_and_cycle_sweep_iterations_match_oracle(levels, gamma):
    """The sweep of bench.py --cycle-sweep at 128^2 (coarsest 16^2 down to
    1 element): FP64 cycle, iterations within 1 of the oracle's pCGMG with
    the same levels and cycle index."""
    from workloads import make_problem
    p = make_problem("wall1024", n=128, levels=levels, mixed=False)
    o = solve.solve_mgpcg(p.nelx, p.nely, p.x, p.E_phase, p.E_min, p.penal, p.nu, p.F, levels,
                          rel_tol=1e-8, grad=False, gamma=gamma)
    s = gpu_solver(p, "fp64")
    s.set_option("GAMMA", gamma)
    st = s.solve(1e-8, 1000)[0]
    assert st["status"] == 0 and st["relres_true"] <= 1.05e-8, st
    assert abs(st["iters"] - o.iters[0]) <= 1, (levels, gamma, st["iters"], o.iters)


# The paper's meshes (Tables 3-5: 32 x 32, 32 x 64, 64 x 64 and, below, the
# larger ones in bench.py) with every level count from the two-grid method up
PAPER_MESHES = [(32, 32, l) for l in range(2, 7)] + [(32, 64, l) for l in range(2, 7)] + \
               [(64, 64, l) for l in range(2, 8)]


@pytest.mark.parametrize("nx,ny,levels", PAPER_MESHES, ids=lambda v: str(v))
def test_paper_meshes_every_level_count_match_oracle(nx, ny, levels):
    """Levels l = 2 (two grids, coarsest 16 x 16 to 32 x 32) up to a 1-element
    coarsest side on the paper's smaller meshes, smooth 3-phase densities:
    FP64 cycle, iterations within 1 of the oracle's pCGMG with the same
    levels, u against the oracle's direct solve."""
    from workloads import Problem, density_gaussian_sum, load_top_traction
    x = density_gaussian_sum(nx, ny, 2)
    p = Problem("paper", nx, ny, x, np.array([1.0, 0.6, 0.2]), 1e-9, 3.0, 0.3, load_top_traction(nx, ny)[None],
                levels)
    o = solve.solve_mgpcg(p.nelx, p.nely, p.x, p.E_phase, p.E_min, p.penal, p.nu, p.F, levels,
                          rel_tol=1e-8, grad=False)
    s = gpu_solver(p, "fp64")
    st = s.solve(1e-8, 1000)[0]
    assert st["status"] == 0 and st["relres_true"] <= 1.05e-8, st
    assert abs(st["iters"] - o.iters[0]) <= 1, (st["iters"], o.iters)
    assert relerr(s.U(0).cpu().numpy(), o.U) <= 1e-6
