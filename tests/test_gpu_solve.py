"""End-to-end parity of the HIP pCGMG solve with the oracle (Algorithm 2 + Algorithm 1).

The bar (FP64 CG in both precisions): true relative residual <= 1e-8 and
||u - u_oracle|| / ||u_oracle|| <= 1e-6; compliance to 1e-7 relative and
the gradient to 1e-5 relative against the oracle's direct solve.
"""

import numpy as np
import pytest
import torch

from oracle import fe, solve
from tests.gpu_util import gpu_solver, rel, relerr
from workloads import Problem, load_top_traction, make_problem

pytestmark = pytest.mark.gpu


def oracle_direct(p):
    return solve.solve_direct(p.nelx, p.nely, p.x, p.E_phase, p.E_min, p.penal, p.nu, p.F)


def rand_prob(nx, ny, L, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.05, 1.0, (ny, nx, 3)) / 3
    return Problem("rand", nx, ny, x, np.array([1.0, 0.6, 0.2]), 1e-9, 3.0, 0.3,
                   load_top_traction(nx, ny)[None], L)


CASES = [("wall64", "fp64"), ("wall64", "fp32mg"), ("rand124x60", "fp64"), ("rand124x60", "fp32mg"),
         ("rand256x128", "fp32mg")]


def get_prob(name):
    if name == "wall64":
        return make_problem("wall64")
    if name == "rand124x60":
        return rand_prob(124, 60, 3, 7)
    if name == "rand256x128":
        return rand_prob(256, 128, 4, 8)
    raise KeyError(name)


@pytest.mark.parametrize("name,prec", CASES)
def test_solve_matches_oracle(name, prec):
    p = get_prob(name)
    print(f"[solve] {name} {prec}", flush=True)
    ref = oracle_direct(p)
    s = gpu_solver(p, prec)
    st = s.solve(1e-8, 1000)[0]
    assert st["status"] == 0, st
    assert st["relres_true"] <= 1e-8 * 1.05, st
    U = s.U(0).cpu().numpy()
    assert relerr(U, ref.U) <= 1e-6
    c, dc = s.compliance_and_grad(0)
    c = c.cpu().numpy()
    dc = dc.cpu().numpy()
    np.testing.assert_allclose(c, ref.c, rtol=1e-7)
    assert relerr(dc, ref.dcdx) <= 1e-5
    # the oracle's own energy identity on the GPU displacements
    E = fe.interpolate_modulus(p.x, p.E_phase, p.E_min, p.penal)
    energy = np.sum(E * fe.element_energies(U[0], p.nelx, p.nely, p.nu))
    assert c[0] == pytest.approx(energy, rel=1e-7)


def test_iteration_count_matches_oracle_pcgmg():
    p = make_problem("wall64")
    o = solve.solve_mgpcg(p.nelx, p.nely, p.x, p.E_phase, p.E_min, p.penal, p.nu, p.F, p.levels,
                          rel_tol=1e-8, grad=False)
    s = gpu_solver(p, "fp64")
    st = s.solve(1e-8, 1000)[0]
    assert abs(st["iters"] - o.iters[0]) <= 1, (st, o.iters)


@pytest.mark.parametrize("prec", ["fp64", "fp32mg"])
def test_deterministic(prec):
    p = rand_prob(124, 60, 3, 9)
    s = gpu_solver(p, prec)
    s.solve(1e-8, 1000)
    a = s.U(0).clone()
    s.solve(1e-8, 1000)
    assert torch.equal(a, s.U(0))


def test_warm_start_and_status_paths():
    p = rand_prob(64, 64, 3, 10)
    s = gpu_solver(p, "fp64")
    st = s.solve(1e-8, 1000)[0]
    assert st["status"] == 0
    st2 = s.solve(1e-8, 1000, warm_start=True)[0]
    assert st2["status"] == 0 and st2["iters"] <= 1
    st3 = s.solve(1e-8, 1)[0]
    assert st3["status"] == -2 and st3["iters"] == 1
    assert st3["relres_true"] > 1e-8
    st4 = s.solve(1e-8, 0)[0]
    assert st4["status"] == -2 and st4["iters"] == 0
    assert torch.count_nonzero(s.U(0)) == 0


def test_zero_load_gives_zero_displacement():
    p = rand_prob(32, 32, 2, 11)
    p.F[:] = 0.0
    s = gpu_solver(p, "fp64")
    st = s.solve(1e-8, 100)[0]
    assert st["status"] == 0 and st["iters"] == 0
    assert torch.count_nonzero(s.U(0)) == 0


def test_multiple_load_cases():
    from workloads.square_wall import four_load_cases
    p = rand_prob(64, 32, 3, 12)
    p.F = four_load_cases(64, 32)
    ref = oracle_direct(p)
    s = gpu_solver(p, "fp32mg")
    stats = s.solve(1e-8, 1000)
    assert all(st["status"] == 0 and st["relres_true"] <= 1.05e-8 for st in stats)
    assert relerr(s.U(0).cpu().numpy(), ref.U) <= 1e-6
    c, dc = s.compliance_and_grad(0)
    np.testing.assert_allclose(c.cpu().numpy(), ref.c, rtol=1e-7)
    assert relerr(dc.cpu().numpy(), ref.dcdx) <= 1e-5


def test_bad_inputs_are_rejected():
    from paper_2301_07457_amd import PCGMGSolver
    from paper_2301_07457_amd._lib import MtomgError
    s = PCGMGSolver()
    F = torch.zeros((1, 33, 33, 2), dtype=torch.float64)
    with pytest.raises(MtomgError):
        s.add_design(0, 32, 32, F, [1.0], levels=7)       # 32 not divisible by 64
    with pytest.raises(MtomgError):
        s.add_design(0, 32, 32, F, [1.0], E_min=0.0)      # E_min must be > 0
    with pytest.raises(MtomgError):
        s.add_design(0, 256, 256, torch.zeros((1, 257, 257, 2)), [1.0], levels=2)  # coarsest too big


@pytest.mark.parametrize("prec", ["fp64", "fp32mg"])
@pytest.mark.parametrize("nx,ny", [(96, 48), (128, 64)])
def test_two_grids_with_large_coarsest_match_oracle(nx, ny, prec):
    """Two grids (the paper's l = 2) with a coarsest grid beyond 32 x 32
    elements, factorised by the dense block sequence: 48 x 24 (2,352 DOFs;
    the coarse solve stages its right-hand side in LDS) and 64 x 32 (4,160
    DOFs; read through L2).  u against the oracle's direct solve; at 96 x 48
    also the iteration count against the oracle's two-grid pCGMG."""
    p = rand_prob(nx, ny, 2, nx + ny)
    ref = oracle_direct(p)
    s = gpu_solver(p, prec)
    st = s.solve(1e-8, 1000)[0]
    assert st["status"] == 0 and st["relres_true"] <= 1.05e-8, st
    assert relerr(s.U(0).cpu().numpy(), ref.U) <= 1e-6
    if nx == 96 and prec == "fp64":
        o = solve.solve_mgpcg(p.nelx, p.nely, p.x, p.E_phase, p.E_min, p.penal, p.nu, p.F, 2, rel_tol=1e-8,
                              grad=False)
        assert abs(st["iters"] - o.iters[0]) <= 1, (st["iters"], o.iters)
    print(f"[two grids {nx}x{ny}] {prec} iters={st['iters']} setup_ms={st['t_setup_ms']:.2f} "
          f"solve_ms={st['t_solve_ms']:.2f}")


def test_autograd_function_matches_oracle_gradient():
    from paper_2301_07457_amd import ComplianceFn
    p = rand_prob(64, 64, 3, 13)
    ref = oracle_direct(p)
    s = gpu_solver(p, "fp64")
    x = torch.from_numpy(p.x).cuda().requires_grad_(True)
    c = ComplianceFn.apply(x, s, 0, 1e-10, 1000)
    c.sum().backward()
    assert c.item() == pytest.approx(ref.c[0], rel=1e-9)
    assert relerr(x.grad.cpu().numpy(), ref.dcdx[0]) <= 1e-6


@pytest.mark.parametrize("m", range(1, 9))
def test_gradient_every_phase_count_matches_oracle(m):
    """The gradient kernel (Eq. 6 and Section 4) for every phase count the
    library accepts: each count has its own rows per wave and register
    layout.  130 x 70 elements give a ragged third strip (4 of 63 element
    columns) and ragged row chunks for every row count.  The oracle's
    formula is applied to the GPU's own displacements, so the comparison is
    of the kernel alone, element by element."""
    nx, ny = 130, 70
    rng = np.random.default_rng(100 + m)
    x = rng.uniform(0.05, 1.0, (ny, nx, m)) / m
    E_phase = np.linspace(1.0, 0.2, m)
    prob = Problem(f"rand{m}", nx, ny, x, E_phase, 1e-9, 3.0, 0.3, load_top_traction(nx, ny)[None], 2)
    print(f"[grad] m={m}", flush=True)
    s = gpu_solver(prob, "fp64")
    st = s.solve(1e-10, 1000)[0]
    assert st["status"] == 0, st
    U = s.U(0).cpu().numpy()
    _, dc = s.compliance_and_grad(0)
    dc = dc.cpu().numpy()[0]
    ref = fe.compliance_gradient(x, U[0], E_phase, 1e-9, 3.0, 0.3)
    assert dc.shape == ref.shape
    assert relerr(dc, ref) <= 1e-12


@pytest.mark.parametrize("sweeps", [1, 3, 4])
@pytest.mark.parametrize("prec", ["fp64", "fp32mg"])
def test_other_sweep_counts(sweeps, prec):
    """n_pre = n_post in {1, 3, 4}: single, paired and paired + single
    post-smoothing launches.  The solution matches the direct solve and the
    iteration count the oracle's pCGMG with the same cycle (within 1)."""
    from paper_2301_07457_amd import PCGMGSolver
    p = rand_prob(124, 60, 3, 30 + sweeps)
    ref = oracle_direct(p)
    o = solve.solve_mgpcg(p.nelx, p.nely, p.x, p.E_phase, p.E_min, p.penal, p.nu, p.F, p.levels,
                          n_pre=sweeps, n_post=sweeps, rel_tol=1e-8, grad=False)
    s = PCGMGSolver()
    s.add_design(0, p.nelx, p.nely, torch.from_numpy(p.F), list(p.E_phase), p.E_min, p.penal, p.nu,
                 p.levels, sweeps, sweeps, p.omega, prec)
    s.set_densities(0, torch.from_numpy(p.x))
    st = s.solve(1e-8, 1000)[0]
    assert st["status"] == 0 and st["relres_true"] <= 1.05e-8, st
    assert abs(st["iters"] - o.iters[0]) <= 1, (st["iters"], o.iters)
    assert relerr(s.U(0).cpu().numpy(), ref.U) <= 1e-6


@pytest.mark.parametrize("nx,ny,L", [(2, 2, 2), (4, 4, 2), (8, 6, 2), (8, 8, 3), (6, 20, 2)])
@pytest.mark.parametrize("prec", ["fp64", "fp32mg"])
def test_tiny_grids(nx, ny, L, prec):
    """Degenerate sizes: a single coarsest element, one- and two-block coarse
    factorisations, one strip narrower than a wave."""
    p = rand_prob(nx, ny, L, 40 + nx + ny)
    ref = oracle_direct(p)
    s = gpu_solver(p, prec)
    st = s.solve(1e-8, 1000)[0]
    assert st["status"] == 0 and st["relres_true"] <= 1.05e-8, st
    assert relerr(s.U(0).cpu().numpy(), ref.U) <= 1e-6
    c, dc = s.compliance_and_grad(0)
    np.testing.assert_allclose(c.cpu().numpy(), ref.c, rtol=1e-7)
    assert relerr(dc.cpu().numpy(), ref.dcdx) <= 1e-5


def test_autotune_picks_a_candidate_and_keeps_parity():
    p = rand_prob(124, 60, 3, 50)
    ref = oracle_direct(p)
    s = gpu_solver(p, "fp32mg")
    cands = ((0, 0), (1, 1), (2, 2), (4, 1))
    best, timings = s.autotune(1e-8, 1000, candidates=cands, repeats=1)
    assert best in cands and set(cands) <= set(timings)
    # then the outer-CG apply and the two grids below the finest, one knob at a time
    assert {"ROWS_CG=4", "ROWS_CG=8", "ROWS_LEVEL1=1", "ROWS_LEVEL2=4"} <= set(timings)
    assert s.tuned["ROWS_FINE"] == best[0] and s.tuned["ROWS_COARSE"] == best[1]
    assert s.tuned["ROWS_CG"] in (0, 4, 8) and s.tuned["ROWS_LEVEL1"] in (0, 1, 2, 4)
    assert all(t > 0 for t in timings.values())
    st = s.solve(1e-8, 1000)[0]
    assert st["status"] == 0 and st["relres_true"] <= 1e-8
    assert relerr(s.U(0).cpu().numpy(), ref.U) <= 1e-6


@pytest.fixture(scope="module")
def wall576():
    """The 1024^2 workload's recipe at 576^2, 6 grids (coarsest 18^2): its
    second-finest level (288^2, 83,521 nodes) is above both fusion
    thresholds (single post-smoother there, fused restriction +
    pre-smoothing and paired post-smoothers further down).  The grid two
    below the finest (144^2) is small enough for the restriction-presmoothing
    fusion, so the finest grid runs its pre-smoothing and restriction as
    separate launches (the fused path of 1024^2 is tested at 768^2)."""
    p = make_problem("wall1024", n=576, levels=6)
    print("[wall576] oracle direct solve", flush=True)
    return p, oracle_direct(p)


@pytest.mark.parametrize("prec", ["fp64", "fp32mg"])
@pytest.mark.parametrize("pair", __import__("paper_2301_07457_amd").PCGMGSolver.AUTOTUNE_CANDIDATES,
                         ids=lambda t: f"rows{t[0]}-{t[1]}")
def test_every_autotune_tile_pair_matches_oracle(wall576, pair, prec):
    """Each (fine, coarse) rows-per-wave pair the autotuner may pick gives the
    oracle's solution, compliance and gradient."""
    p, ref = wall576
    s = gpu_solver(p, prec)
    s.set_option("ROWS_FINE", pair[0])
    s.set_option("ROWS_COARSE", pair[1])
    st = s.solve(1e-8, 1000)[0]
    assert st["status"] == 0 and st["relres_true"] <= 1.05e-8, st
    assert relerr(s.U(0).cpu().numpy(), ref.U) <= 1e-6
    c, dc = s.compliance_and_grad(0)
    np.testing.assert_allclose(c.cpu().numpy(), ref.c, rtol=1e-7)
    assert relerr(dc.cpu().numpy(), ref.dcdx) <= 1e-5
    print(f"[tiles {pair}] {prec} iters={st['iters']} solve_ms={st['t_solve_ms']:.2f}")


@pytest.mark.parametrize("bad,want", [(float("nan"), -4), (float("inf"), -4), (1.5, -1), (-1.0, -1),
                                      (1.0 + 2.0 ** -52, -1)],
                         ids=["nan", "inf", "1.5", "-1", "1+ulp"])
@pytest.mark.parametrize("prec", ["fp64", "fp32mg"])
def test_invalid_density_is_reported_by_the_solve(bad, want, prec):
    """One density outside [0, 1] (BAD_INPUT) or not finite (NAN): the
    device-side check of set_densities is reported by the next solve for the
    design's load case, a second solve on the same densities reports it
    again, and valid densities clear it."""
    from paper_2301_07457_amd import _lib
    p = make_problem("wall64")
    x = p.x.copy()
    x[5, 7, 1] = bad
    s = gpu_solver(p, prec)
    s.set_densities(0, torch.from_numpy(x))
    for _ in range(2):
        st = s.solve(1e-8, 200)[0]
        assert st["status"] == want, st
    assert _lib.mtomg_last_error(s.ctx) == _lib.mtomg_status_string(want)
    s.set_densities(0, torch.from_numpy(p.x))
    st = s.solve(1e-8, 1000)[0]
    assert st["status"] == 0 and st["relres_true"] <= 1.05e-8, st
    x[5, 7, 1] = 1.0   # the bounds themselves are valid
    x[0, 0, 0] = 0.0
    s.set_densities(0, torch.from_numpy(x))
    assert s.solve(1e-8, 1000)[0]["status"] == 0


@pytest.mark.parametrize("prec,cg,l1,l2", [("fp32mg", 1, 1, 1), ("fp32mg", 2, 2, 2), ("fp32mg", 4, 4, 4),
                                           ("fp32mg", 8, 8, 8), ("fp64", 8, 4, 2)],
                         ids=lambda v: str(v))
def test_per_kernel_and_per_level_rows_match_oracle(wall576, prec, cg, l1, l2):
    """The autotuner's per-kernel knobs: rows per wave of the outer-CG apply
    (ROWS_CG) and of the two grids below the finest (ROWS_LEVEL1/2), every
    value each may take, give the oracle's solution."""
    p, ref = wall576
    s = gpu_solver(p, prec)
    s.set_option("ROWS_CG", cg)
    s.set_option("ROWS_LEVEL1", l1)
    s.set_option("ROWS_LEVEL2", l2)
    st = s.solve(1e-8, 1000)[0]
    assert st["status"] == 0 and st["relres_true"] <= 1.05e-8, st
    assert relerr(s.U(0).cpu().numpy(), ref.U) <= 1e-6
    c, dc = s.compliance_and_grad(0)
    np.testing.assert_allclose(c.cpu().numpy(), ref.c, rtol=1e-7)
    assert relerr(dc.cpu().numpy(), ref.dcdx) <= 1e-5


@pytest.mark.parametrize("prec", ["fp64", "fp32mg"])
def test_fused_presmoothing_matches_separate_launches_and_oracle(prec):
    """MTOMG_OPT_FUSE_PRE on design 32 of the batched workload (768^2, 6
    grids, four load cases): the grid two below the finest has 37,249 nodes,
    so, as at 1024^2, the finest grid's CG update, pre-smoothing and
    restriction run in one launch, the convergence test opens the 384^2
    grid with its own fused launch, and the 192^2 grid keeps the
    restriction-presmoothing fusion.  Against the separate launches (which
    round differently only through the compiler's multiply-add contraction):
    the same iteration counts and displacements within the oracle bar;
    against the oracle: its stored direct-solve samples
    (tests/golden/batch32_samples.json)."""
    import json
    import os
    from tests.test_gpu_fullsize import check_against_samples
    from workloads import batched_design
    p = batched_design(32)
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "batch32_samples.json")))
    out = {}
    for fuse in (1, 0):
        s = gpu_solver(p, prec)
        s.set_option("FUSE_PRE", fuse)
        stats = s.solve(1e-8, 1000)
        assert all(st["status"] == 0 and st["relres_true"] <= 1.05e-8 for st in stats), stats
        out[fuse] = ([st["iters"] for st in stats], s.U(0).clone(), s)
        print(f"[fuse_pre={fuse}] {prec} iters={out[fuse][0]} solve_ms={stats[0]['t_solve_ms']:.2f}")
    assert out[1][0] == out[0][0]
    d = relerr(out[1][1].cpu().numpy(), out[0][1].cpu().numpy())
    print(f"[fuse_pre] {prec} fused vs separate: relerr(u) {d:.2e}")
    assert d <= 1e-6
    s = out[1][2]
    U = out[1][1].cpu().numpy()
    c, dc = s.compliance_and_grad(0)
    for case in range(4):
        check_against_samples(gold, p, s, case, U[case], c[case].item(), dc[case].cpu().numpy())


@pytest.mark.parametrize("pair", [tuple(t) + (0,) for t in
                                  __import__("paper_2301_07457_amd").PCGMGSolver.AUTOTUNE_CANDIDATES] +
                         [(0, 0, 1), (0, 0, 2), (0, 0, 4)],
                         ids=lambda t: f"rows{t[0]}-{t[1]}-level1-{t[2]}")
def test_fused_presmoothing_every_tile_pair_matches_oracle(pair):
    """The fused path at 768^2 (design 32 of the batched workload, FP32
    cycle) with each (fine, coarse) rows-per-wave pair the autotuner may
    pick, and each rows-per-wave value of the grid below the finest: the
    fused launches take 1, 2 or 4 rows per wave (at most 4), so every
    instantiation the bench can run meets the oracle's stored direct-solve
    samples."""
    import json
    import os
    from tests.test_gpu_fullsize import check_against_samples
    from workloads import batched_design
    p = batched_design(32)
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "batch32_samples.json")))
    s = gpu_solver(p, "fp32mg")
    s.set_option("ROWS_FINE", pair[0])
    s.set_option("ROWS_COARSE", pair[1])
    s.set_option("ROWS_LEVEL1", pair[2])   # the fused launch with the convergence test
    s.set_densities(0, torch.from_numpy(p.x))
    stats = s.solve(1e-8, 1000)
    assert all(st["status"] == 0 and st["relres_true"] <= 1.05e-8 for st in stats), stats
    U = s.U(0).cpu().numpy()
    c, dc = s.compliance_and_grad(0)
    for case in range(4):
        check_against_samples(gold, p, s, case, U[case], c[case].item(), dc[case].cpu().numpy())


def test_option_values_are_checked():
    from paper_2301_07457_amd import PCGMGSolver, _lib
    s = PCGMGSolver()
    for name, v in (("RESTARTS", -1), ("RESTARTS", 65), ("ROWS_CG", 3), ("ROWS_LEVEL1", 16), ("ROWS_LEVEL14", 2)):
        with pytest.raises(_lib.MtomgError):
            _lib.mtomg_set_option(s.ctx, name, v)
    _lib.mtomg_set_option(s.ctx, "RESTARTS", 10)
