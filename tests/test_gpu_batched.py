"""Batched solve: many designs of uneven sizes, each with four load cases,
in one mtomg_solve call (every launch serves all systems of a same-shape
group; all groups iterate in lockstep inside one captured graph).

Checks, per system: the oracle's direct solve (relative error 1e-6,
compliance 1e-7, gradient 1e-5) and bit-for-bit equality with the same
design solved on its own, which shows that systems sharing a launch do not
interact.  A design without densities keeps its displacements and is not
reported.
"""

import numpy as np
import pytest
import torch

from oracle import solve
from tests.gpu_util import rel, relerr
from workloads import Problem
from workloads.square_wall import density_gaussian_sum, four_load_cases

pytestmark = pytest.mark.gpu

# (nelx, nely, levels, precision, seed)
DESIGNS = [
    (64, 64, 3, "fp32mg", 2001),
    (96, 48, 4, "fp64", 2002),
    (64, 64, 3, "fp32mg", 2003),
    (64, 64, 3, "fp64", 2004),
    (96, 48, 4, "fp64", 2005),
    (64, 64, 3, "fp32mg", 2006),
]


def make(nx, ny, levels, seed):
    x = density_gaussian_sum(nx, ny, seed)
    return Problem(f"b{seed}", nx, ny, x, np.array([1.0, 0.6, 0.2]), 1e-9, 3.0, 0.3,
                   four_load_cases(nx, ny), levels)


def add(s, k, p, prec):
    s.add_design(k, p.nelx, p.nely, torch.from_numpy(p.F), list(p.E_phase), p.E_min, p.penal, p.nu,
                 p.levels, 2, 2, 0.6, prec)


@pytest.fixture(scope="module")
def batch():
    from paper_2301_07457_amd import PCGMGSolver
    probs = [make(nx, ny, L, seed) for nx, ny, L, _, seed in DESIGNS]
    s = PCGMGSolver(max_designs=len(probs))
    for k, (p, d) in enumerate(zip(probs, DESIGNS)):
        add(s, k, p, d[3])
    for k, p in enumerate(probs):
        s.set_densities(k, torch.from_numpy(p.x))
    print(f"[batched] {len(probs)} designs x 4 cases", flush=True)
    stats = s.solve(1e-8, 1000)
    return probs, s, stats


def test_batched_systems_match_oracle(batch):
    probs, s, stats = batch
    assert len(stats) == 4 * len(probs)
    for k, p in enumerate(probs):
        ref = solve.solve_direct(p.nelx, p.nely, p.x, p.E_phase, p.E_min, p.penal, p.nu, p.F)
        for q in range(4):
            st = stats[4 * k + q]
            assert st["status"] == 0 and st["relres_true"] <= 1.05e-8, (k, q, st)
        U = s.U(k).cpu().numpy()
        for q in range(4):
            assert relerr(U[q], ref.U[q]) <= 1e-6, (k, q)
        c, dc = s.compliance_and_grad(k)
        np.testing.assert_allclose(c.cpu().numpy(), ref.c, rtol=1e-7)
        assert relerr(dc.cpu().numpy(), ref.dcdx) <= 1e-5
        print(f"[batched] design {k} {p.nelx}x{p.nely} iters={[st['iters'] for st in stats[4*k:4*k+4]]}")


def test_batched_equals_solo_bitwise(batch):
    from paper_2301_07457_amd import PCGMGSolver
    probs, s, stats = batch
    for k in (0, 1, 3):
        p, prec = probs[k], DESIGNS[k][3]
        solo = PCGMGSolver(max_designs=1)
        add(solo, 0, p, prec)
        solo.set_densities(0, torch.from_numpy(p.x))
        st = solo.solve(1e-8, 1000)
        assert [a["iters"] for a in st] == [b["iters"] for b in stats[4 * k:4 * k + 4]]
        assert torch.equal(solo.U(0), s.U(k)), k


def test_design_without_densities_is_untouched():
    from paper_2301_07457_amd import PCGMGSolver
    a = make(64, 64, 3, 2101)
    b = make(64, 64, 3, 2102)
    s = PCGMGSolver(max_designs=2)
    add(s, 0, a, "fp32mg")
    add(s, 1, b, "fp32mg")          # same group, no densities
    s.U(1).fill_(7.0)
    s.set_densities(0, torch.from_numpy(a.x))
    stats = s.solve(1e-8, 1000)
    assert len(stats) == 4 and all(st["status"] == 0 for st in stats)
    assert torch.all(s.U(1) == 7.0)
    # solving again after densities arrive for design 1 covers both
    s.set_densities(1, torch.from_numpy(b.x))
    stats = s.solve(1e-8, 1000)
    assert len(stats) == 8 and all(st["status"] == 0 for st in stats)
    ref = solve.solve_direct(b.nelx, b.nely, b.x, b.E_phase, b.E_min, b.penal, b.nu, b.F)
    assert relerr(s.U(1).cpu().numpy(), ref.U) <= 1e-6


def test_graphs_on_and_off_agree(batch):
    probs, s, stats = batch
    U0 = [s.U(k).clone() for k in range(len(probs))]
    s.set_option("GRAPHS", 0)
    try:
        st2 = s.solve(1e-8, 1000)
    finally:
        s.set_option("GRAPHS", 1)
    assert [a["iters"] for a in st2] == [b["iters"] for b in stats]
    for k in range(len(probs)):
        assert torch.equal(U0[k], s.U(k))


SLICE = (0, 1, 2, 16, 17, 18, 32, 33, 34)   # designs of the 48-design workload: 3 per size


@pytest.fixture(scope="module")
def config4_slice():
    """Nine designs of the batched workload itself (three each at 128^2,
    384^2 and 768^2, four load cases each) and their oracle references: the
    direct solve for designs 0-2 and 16, the stored direct-solve samples of
    design 32 (tests/golden/make_golden.py batch32)."""
    import json
    import os
    from workloads import batched_design
    probs = [batched_design(d) for d in SLICE]
    refs = {}
    for k in (0, 1, 2, 3):
        p = probs[k]
        print(f"[config4 slice] oracle direct solve {p.name} ({p.nelx}^2)", flush=True)
        refs[k] = solve.solve_direct(p.nelx, p.nely, p.x, p.E_phase, p.E_min, p.penal, p.nu, p.F)
    path = os.path.join(os.path.dirname(__file__), "golden", "batch32_samples.json")
    gold = json.load(open(path))
    return probs, refs, gold


@pytest.mark.parametrize("pair", __import__("paper_2301_07457_amd").PCGMGSolver.AUTOTUNE_CANDIDATES,
                         ids=lambda t: f"rows{t[0]}-{t[1]}")
def test_config4_slice_matches_oracle(config4_slice, pair):
    """The batched workload's shapes in one solve, with each tile pair the
    autotuner may pick: every system reaches the residual bar; the 128^2
    designs and a 384^2 design match the oracle's direct solve (u element
    by element, compliance, gradient) in all four load cases, and a 768^2
    design its stored direct-solve samples."""
    from paper_2301_07457_amd import PCGMGSolver
    from tests.test_gpu_fullsize import check_against_samples
    probs, refs, gold = config4_slice
    s = PCGMGSolver(max_designs=len(probs))
    for k, p in enumerate(probs):
        add(s, k, p, "fp32mg")
    s.set_option("ROWS_FINE", pair[0])
    s.set_option("ROWS_COARSE", pair[1])
    for k, p in enumerate(probs):
        s.set_densities(k, torch.from_numpy(p.x))
    stats = s.solve(1e-8, 1000)
    assert len(stats) == 4 * len(probs)
    assert all(st["status"] == 0 and st["relres_true"] <= 1.05e-8 for st in stats), stats
    for k, ref in refs.items():
        c, dc = s.compliance_and_grad(k)
        assert relerr(s.U(k).cpu().numpy(), ref.U) <= 1e-6, k
        np.testing.assert_allclose(c.cpu().numpy(), ref.c, rtol=1e-7)
        assert relerr(dc.cpu().numpy(), ref.dcdx) <= 1e-5, k
    k32 = SLICE.index(32)
    p = probs[k32]
    U = s.U(k32).cpu().numpy()
    c, dc = s.compliance_and_grad(k32)
    for case in range(4):
        check_against_samples(gold, p, s, case, U[case], c[case].item(), dc[case].cpu().numpy())
    print(f"[config4 slice {pair}] solve {stats[0]['t_solve_ms']:.2f} ms, iters "
          f"{sorted(set(st['iters'] for st in stats))}")


def test_invalid_design_reports_bad_input_and_spares_the_group():
    """x = -1 lies outside [0, 1] (and gives negative moduli, so the coarsest
    matrix is not positive definite either): the device-side input check
    reports BAD_INPUT for each load case of that design, while a valid
    design of the same group solves."""
    from paper_2301_07457_amd import PCGMGSolver
    a = make(64, 64, 3, 2201)
    s = PCGMGSolver(max_designs=2)
    add(s, 0, a, "fp32mg")
    add(s, 1, a, "fp32mg")
    s.set_densities(0, torch.from_numpy(-np.ones_like(a.x)))
    s.set_densities(1, torch.from_numpy(a.x))
    stats = s.solve(1e-8, 200)
    assert [st["status"] for st in stats[:4]] == [-1] * 4
    assert all(st["status"] == 0 and st["relres_true"] <= 1e-8 for st in stats[4:])
    ref = solve.solve_direct(a.nelx, a.nely, a.x, a.E_phase, a.E_min, a.penal, a.nu, a.F)
    assert relerr(s.U(1).cpu().numpy(), ref.U) <= 1e-6
    # new valid densities clear the failure
    s.set_densities(0, torch.from_numpy(a.x))
    stats = s.solve(1e-8, 1000)
    assert all(st["status"] == 0 for st in stats)


def test_invalid_single_design_reports_bad_input():
    """A design alone in its group starts its factorisation inside
    set_densities; invalid densities are still reported (BAD_INPUT for each
    load case), and valid densities clear it."""
    from paper_2301_07457_amd import PCGMGSolver
    a = make(64, 64, 3, 2301)
    s = PCGMGSolver(max_designs=1)
    add(s, 0, a, "fp32mg")
    s.set_densities(0, torch.from_numpy(-np.ones_like(a.x)))
    stats = s.solve(1e-8, 200)
    assert [st["status"] for st in stats] == [-1] * 4
    s.set_densities(0, torch.from_numpy(a.x))
    stats = s.solve(1e-8, 1000)
    assert all(st["status"] == 0 and st["relres_true"] <= 1e-8 for st in stats)
    ref = solve.solve_direct(a.nelx, a.nely, a.x, a.E_phase, a.E_min, a.penal, a.nu, a.F)
    assert relerr(s.U(0).cpu().numpy(), ref.U) <= 1e-6


def test_densities_set_twice_before_a_solve():
    """Densities replaced before the solve (the first factorisation may still
    be queued): the solve uses the second set."""
    from paper_2301_07457_amd import PCGMGSolver
    a = make(64, 64, 3, 2401)
    b = make(64, 64, 3, 2402)
    s = PCGMGSolver(max_designs=1)
    add(s, 0, a, "fp64")
    s.set_densities(0, torch.from_numpy(a.x))
    s.set_densities(0, torch.from_numpy(b.x))
    stats = s.solve(1e-8, 1000)
    assert all(st["status"] == 0 for st in stats)
    ref = solve.solve_direct(b.nelx, b.nely, b.x, b.E_phase, b.E_min, b.penal, b.nu, b.F)
    assert relerr(s.U(0).cpu().numpy(), ref.U) <= 1e-6
