"""Parity at the full workload sizes, in the configuration bench.py times.

* 256 x 256, binary 1e9 contrast (5 levels, FP64): against the oracle's
  direct solve element by element, and the adjoint gradient against central
  finite differences on 64 solid (element, phase) pairs plus 8 pairs whose
  gradient is ~0 (relative 1e-5 for gradients of at least 1e-6 max|g|,
  absolute 1e-11 max|g| below), each difference from two solves to 1e-12.  At this contrast the residual 1e-8 leaves an error of
  ~6e-6 in u (condition number ~1e9), so the u comparison solves to 1e-10.
* 1024 x 1024 smooth field (7 levels, FP32 cycle): against oracle samples
  written by tests/golden/make_golden.py (compliance, u at 512 nodes,
  gradient at 64 pairs), and properties that hold at any size: the
  oracle's energy identity c = sum_e E_e u_e^T K0 u_e on the GPU field, the
  oracle's nodal residual at sampled nodes, FP32-cycle and FP64-cycle
  solutions agreeing.
* 2048 x 2048 near-binary 4-phase field (8 levels, contrast 3e8): pCGMG
  needs ~1e4 iterations here (the oracle's own pCGMG does not finish in
  hours), so the full size is checked through the properties above in both
  precisions, and the same recipe at 128 x 128 against the oracle's direct
  solve.  At 2048^2 the recursive and true residuals drift apart, which the
  true-residual confirmation and restart of the solver must absorb.
"""

import dataclasses
import json
import os

import numpy as np
import pytest
import torch

from oracle import fe, solve
from tests.gpu_util import gpu_solver, rel, relerr
from workloads import make_problem

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# 256 x 256 high contrast
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def wall256():
    p = make_problem("wall256")
    print("[wall256] oracle direct solve", flush=True)
    ref = solve.solve_direct(p.nelx, p.nely, p.x, p.E_phase, p.E_min, p.penal, p.nu, p.F)
    return p, ref


def test_wall256_fp64_matches_direct_solve(wall256):
    p, ref = wall256
    s = gpu_solver(p, "fp64")
    st = s.solve(1e-8, 20000)[0]
    assert st["status"] == 0 and st["relres_true"] <= 1.05e-8, st
    st = s.solve(1e-10, 20000)[0]
    assert st["status"] == 0, st
    U = s.U(0).cpu().numpy()
    assert relerr(U, ref.U) <= 1e-6
    c, dc = s.compliance_and_grad(0)
    assert c.item() == pytest.approx(ref.c[0], rel=1e-7)
    assert relerr(dc.cpu().numpy(), ref.dcdx) <= 1e-5
    print(f"[wall256] iters={st['iters']} relres={st['relres_true']:.2e} err={rel(U, ref.U):.2e}")


def test_wall256_fp32_cycle_converges(wall256):
    p, ref = wall256
    s = gpu_solver(p, "fp32mg")
    st = s.solve(1e-8, 20000)[0]
    assert st["status"] == 0 and st["relres_true"] <= 1.05e-8, st
    c, _ = s.compliance_and_grad(0, grad=False)
    assert c.item() == pytest.approx(ref.c[0], rel=1e-6)


def _fd_solve(s, tol=3e-11, warm=False):
    """Solve to the FP64 floor of this design: 1e-12 is asked for, and the
    ± solves stop at a true relative residual of 1.8-2.0e-11, so the
    tolerance is 3e-11 (a tighter one only adds restarts that end at the
    same floor).  warm: start from the current U (the stopping test is
    relative to f either way, so the bar is the same)."""
    st = s.solve(tol, 40000, warm_start=warm)[0]
    assert st["status"] in (0, -2) and st["relres_true"] <= 50 * tol, st
    return st


@pytest.mark.parametrize("chunk", range(9))
def test_wall256_gradient_central_differences(wall256, chunk):
    """Central differences, h = 1e-6, every solve to a relative residual of
    1e-12 (or the FP64 floor just above it): |fd - g| <= 1e-5 max(|g|, 1e-6
    max|g|) on 64 solid (element, phase) pairs and 8 pairs whose gradient
    is ~0, each centred at x0 = clip(x, h, 1 - h) and compared with the
    GPU gradient of the design with that element at x0.  fd is the
    cancellation-free exact difference c+ - c- = -(E+ - E-) u-_e^T K0 u+_e
    (exact for a symmetric K changed in one element).  The naive
    (c+ - c-) / 2h is printed beside it and asserted to the same bar only
    where its error bound, (eps |c| + the solves' error in c = f.u) / (2h |g|),
    stays below 1e-6: at this contrast c ~ 1e2 and 2h|g| ~ 1e-8, so the
    differences of two compliances cancel ~10 digits and the bound is not met
    (the naive values agree with g to ~1e-4 only), which is why the exact
    difference is the gate."""
    p, ref = wall256
    pairs = np.concatenate([p.fd_elements, p.fd_zero_pairs])[chunk * 8:(chunk + 1) * 8]
    h = 1e-6
    s = gpu_solver(p, "fp64")
    _fd_solve(s)
    c0, g = s.compliance_and_grad(0)
    c0 = c0.item()
    gmax = np.abs(g[0].cpu().numpy()).max()
    g_or = ref.dcdx[0].reshape(-1, p.m)
    fnorm, unorm = np.linalg.norm(p.F[0]), float(torch.linalg.norm(s.U(0)))
    KE = fe.element_stiffness(p.nu)
    dofs = fe.element_dof_map(p.nelx, p.nely)
    eps = np.finfo(np.float64).eps
    for e, ph in pairs:
        # the library takes densities in [0, 1] only, so the difference is
        # centred at x0 = clip(x, h, 1 - h) (solid pairs sit at 1, the
        # zero pairs at 0) and compared with the gradient at x0
        xb = p.x.copy()
        xb.reshape(-1, p.m)[e, ph] = min(max(xb.reshape(-1, p.m)[e, ph], h), 1 - h)
        s.set_densities(0, torch.from_numpy(xb))
        _fd_solve(s, warm=True)
        _, gb = s.compliance_and_grad(0)
        g = gb[0].cpu().numpy().reshape(-1, p.m)
        out = []
        for sign in (+1, -1):
            x = xb.copy()
            x.reshape(-1, p.m)[e, ph] += sign * h
            s.set_densities(0, torch.from_numpy(x))
            st = _fd_solve(s, warm=True)
            c, _ = s.compliance_and_grad(0, grad=False)
            E = fe.interpolate_modulus(x.reshape(-1, p.m)[e], p.E_phase, p.E_min, p.penal)
            out.append((c.item(), E, s.U(0).cpu().numpy().ravel()[dofs[e]], st["relres_true"]))
        (cp, Ep, up, rp), (cm, Em, um, rm) = out
        fd = -(Ep - Em) * (um @ KE @ up) / (2 * h)
        naive = (cp - cm) / (2 * h)
        tol = 1e-5 * max(abs(g[e, ph]), 1e-6 * gmax)
        # error bound of the naive difference relative to g: rounding of c
        # (eps |c|) plus the solves' own error in c = f.u, |r.u*| <= ||r|| ||u||
        # per solve, over 2h|g|
        dc_err = eps * abs(c0) + 2 * max(rp, rm) * fnorm * unorm
        bound = dc_err / (2 * h * abs(g[e, ph])) if g[e, ph] != 0 else np.inf
        print(f"[fd] e={e} ph={ph} grad={g[e, ph]:.9e} fd={fd:.9e} naive={naive:.9e} "
              f"oracle={g_or[e, ph]:.9e} relres={max(rp, rm):.1e} naive_bound={bound:.1e}", flush=True)
        assert abs(fd - g[e, ph]) <= tol, (e, ph, fd, g[e, ph], naive, g_or[e, ph])
        if bound <= 1e-6:
            assert abs(naive - g[e, ph]) <= tol, (e, ph, naive, g[e, ph])


# ---------------------------------------------------------------------------
# 1024 x 1024 and 2048 x 2048 against stored oracle samples
# ---------------------------------------------------------------------------
def _samples(name):
    path = os.path.join(GOLD, f"{name}_samples.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated (tests/golden/make_golden.py)")
    return json.load(open(path))


def _nodal_residual(p, U, nodes):
    """Oracle f - K u at the given nodes, element by element (free DOFs)."""
    KE = fe.element_stiffness(p.nu)
    E = fe.interpolate_modulus(p.x, p.E_phase, p.E_min, p.penal)
    nx = p.nelx
    Uf = U.ravel()
    res = []
    for n in nodes:
        i, j = n % (nx + 1), n // (nx + 1)
        if j == 0:
            continue
        r = p.F[0].reshape(-1, 2)[n].copy()
        for ej in (j - 1, j):
            for ei in (i - 1, i):
                if 0 <= ei < nx and 0 <= ej < p.nely:
                    n0 = ej * (nx + 1) + ei
                    gn = [n0, n0 + 1, n0 + nx + 2, n0 + nx + 1]
                    ue = np.concatenate([Uf[2 * q:2 * q + 2] for q in gn])
                    loc = gn.index(n)
                    r -= E[ej, ei] * (KE[2 * loc:2 * loc + 2] @ ue)
        res.append(r)
    return np.array(res)


def check_against_samples(gold, p, s, k, U, c, dc):
    """Load case k of a GPU solve against the oracle samples (u at 512
    nodes element by element, ||u||, compliance, gradient at 64 pairs)."""
    case = gold["cases"][k]
    Uf = U.reshape(-1, 2)
    assert relerr(Uf[gold["nodes"]], np.array(case["u_nodes"])) <= 1e-6
    assert np.linalg.norm(U) == pytest.approx(case["u_norm"], rel=1e-6)
    assert c == pytest.approx(gold["compliance"][k], rel=1e-7)
    g = dc.reshape(-1, p.m)[gold["grad_elems"], gold["grad_phases"]]
    assert relerr(g, case["grad"]) <= 1e-5


@pytest.mark.parametrize("name", ["wall1024"])
def test_fullsize_fp32_cycle_against_oracle_samples(name):
    gold = _samples(name)
    p = make_problem(name)
    print(f"[{name}] gpu solve (FP32 cycle)", flush=True)
    s = gpu_solver(p, "fp32mg")
    st = s.solve(1e-8, 1000)[0]
    assert st["status"] == 0 and st["relres_true"] <= 1.05e-8, st
    U = s.U(0).cpu().numpy()
    c, dc = s.compliance_and_grad(0)
    check_against_samples(gold, p, s, 0, U[0], c.item(), dc[0].cpu().numpy())
    # oracle energy identity on the GPU displacements
    E = fe.interpolate_modulus(p.x, p.E_phase, p.E_min, p.penal)
    energy = np.sum(E * fe.element_energies(U[0], p.nelx, p.nely, p.nu))
    assert c.item() == pytest.approx(energy, rel=1e-7)
    # oracle nodal residual at 2000 sampled nodes is within the global bound
    nodes = np.random.default_rng(7).choice((p.nelx + 1) * (p.nely + 1), 2000, replace=False)
    r = _nodal_residual(p, U[0], nodes)
    assert np.linalg.norm(r) <= 1e-8 * np.linalg.norm(p.F[0])
    print(f"[{name}] iters={st['iters']} solve_ms={st['t_solve_ms']:.2f} relres={st['relres_true']:.2e} "
          f"c={c.item():.12g} (oracle {gold['compliance'][0]:.12g})")


def test_wall1024_fp32_cycle_agrees_with_fp64_cycle():
    p = make_problem("wall1024")
    s32 = gpu_solver(p, "fp32mg")
    s64 = gpu_solver(p, "fp64")
    st32 = s32.solve(1e-8, 1000)[0]
    st64 = s64.solve(1e-8, 1000)[0]
    assert st32["status"] == 0 and st64["status"] == 0
    d = float(torch.linalg.norm(s32.U(0) - s64.U(0)) / torch.linalg.norm(s64.U(0)))
    assert d <= 1e-6
    print(f"[wall1024] fp32 cycle {st32['iters']} it {st32['t_solve_ms']:.2f} ms; "
          f"fp64 cycle {st64['iters']} it {st64['t_solve_ms']:.2f} ms; rel diff {d:.2e}")


# ---------------------------------------------------------------------------
# near-binary 4-phase stress field (2048 x 2048 and a small copy)
# ---------------------------------------------------------------------------
def test_nearbinary_small_matches_direct_solve():
    p = make_problem("wall2048", n=128, levels=4)
    ref = solve.solve_direct(p.nelx, p.nely, p.x, p.E_phase, p.E_min, p.penal, p.nu, p.F)
    for prec in ("fp64", "fp32mg"):
        s = gpu_solver(p, prec)
        st = s.solve(1e-8, 20000)[0]
        assert st["status"] == 0 and st["relres_true"] <= 1e-8, (prec, st)
        st = s.solve(1e-10, 20000)[0]
        assert st["status"] == 0 and st["relres_true"] <= 1e-10, (prec, st)
        assert relerr(s.U(0).cpu().numpy(), ref.U) <= 1e-6
        c, dc = s.compliance_and_grad(0)
        assert c.item() == pytest.approx(ref.c[0], rel=1e-7)
        assert relerr(dc.cpu().numpy(), ref.dcdx) <= 1e-5
        print(f"[near-binary 128] {prec} iters={st['iters']}")


HIST_KS = (1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 60)


@pytest.mark.parametrize("prec", ["fp64", "fp32mg"])
def test_nearbinary_residual_history_matches_oracle(prec):
    """||r_k|| / ||f|| after k = 1 .. 60 pCGMG iterations on the near-binary
    recipe (contrast 3e8) at 128^2 and 256^2 against the oracle's history
    (tests/golden/nearbinary_history.json).  Every step of Algorithms 1-2
    enters r_k, so a missing or extra sweep, a wrong transfer or a wrong CG
    coefficient moves it by far more than rounding does.  Bars: FP64 cycle
    5e-9 relative (the two sides' operators differ by rounding, amplified by
    this operator's conditioning: 1e-11 at 128^2 and 5e-10 at 256^2 after 60
    iterations, measured), FP32 cycle 1e-5 (its cycle rounds at 6e-8)."""
    bar = 5e-9 if prec == "fp64" else 1e-5
    gold = json.load(open(os.path.join(GOLD, "nearbinary_history.json")))
    for case in gold["cases"]:
        p = make_problem("wall2048", n=case["n"], levels=case["levels"])
        s = gpu_solver(p, prec)
        s.set_option("RESTARTS", 0)
        worst = 0.0
        for k in HIST_KS:
            st = s.solve(1e-30, k)[0]
            h = case["history"][k]
            assert st["iters"] == k and st["status"] == -2, st
            worst = max(worst, abs(st["relres_rec"] - h) / h)
            assert abs(st["relres_rec"] - h) <= bar * h, (case["n"], k, st["relres_rec"], h)
        print(f"[near-binary {case['n']}] {prec} history k<=60: max rel diff {worst:.2e}")


def test_nearbinary_iteration_counts_match_oracle():
    """pCGMG iteration counts on the near-binary recipe (FP64 cycle) at 128^2
    and 256^2 to relative residual 1e-8, against the oracle's
    (tests/golden/nearbinary_iters.json).  At contrast 3e8 the count of a
    run of 1e3-4e3 iterations is decided by rounding as much as by the
    method (the early residual history above is not): the oracle's FP64
    count moves by up to 9% when the loads are scaled by 1 +- 2^-50 or 3,
    its long-double run differs again, and the GPU's own counts move the
    same way.  So the counts are compared as samples: the median of the
    GPU's four counts (same load scales) must lie within 25% of the median
    of the oracle's four FP64 counts."""
    gold = json.load(open(os.path.join(GOLD, "nearbinary_iters.json")))
    for case in gold["cases"]:
        ref = [case["iters"]] + case["iters_perturbed"]
        p = make_problem("wall2048", n=case["n"], levels=case["levels"])
        counts = []
        for scale in [1.0] + case["load_scales"]:
            s = gpu_solver(dataclasses.replace(p, F=p.F * scale), "fp64")
            s.set_option("RESTARTS", 0)   # Algorithm 2's count, without the true-residual restarts
            st = s.solve(1e-8, 20000)[0]
            assert st["relres_rec"] <= 1e-8 and st["relres_true"] <= 2e-8, st
            counts.append(st["iters"])
            del s
        print(f"[near-binary {case['n']}] gpu iters={counts} oracle fp64={ref} "
              f"oracle long double={case['iters_extended']}")
        assert abs(np.median(counts) / np.median(ref) - 1.0) <= 0.25, (counts, ref)


def test_nearbinary512_matches_direct_solve():
    """512^2 near-binary (6 grids): u, compliance and gradient against the
    oracle's direct solve (whose own residual is 1.2e-9), both cycle
    precisions, at the standard 1e-8 (measured: u 1.6e-7 in norm, 1.9e-7
    element-wise; tighter tolerances leave the difference at ~1.5e-7, the
    direct solve's own error)."""
    p = make_problem("wall2048", n=512, levels=6)
    print("[near-binary 512] oracle direct solve", flush=True)
    ref = solve.solve_direct(p.nelx, p.nely, p.x, p.E_phase, p.E_min, p.penal, p.nu, p.F)
    for prec in ("fp64", "fp32mg"):
        s = gpu_solver(p, prec)
        st = s.solve(1e-8, 60000)[0]
        assert st["status"] == 0 and st["relres_true"] <= 1e-8, (prec, st)
        assert relerr(s.U(0).cpu().numpy(), ref.U) <= 1e-6, prec
        c, dc = s.compliance_and_grad(0)
        assert c.item() == pytest.approx(ref.c[0], rel=1e-7)
        assert relerr(dc.cpu().numpy(), ref.dcdx) <= 1e-5
        print(f"[near-binary 512] {prec} iters={st['iters']} relres_true={st['relres_true']:.2e} "
              f"err={relerr(s.U(0).cpu().numpy(), ref.U):.2e}")


def test_true_residual_confirmation_restarts():
    """512^2 near-binary, FP64 cycle: the recursive residual reaches 1e-8
    while the true one is ~2e-8; the confirmation restarts PCG from u."""
    p = make_problem("wall2048", n=512, levels=6)
    s = gpu_solver(p, "fp64")
    st = s.solve(1e-8, 60000)[0]
    assert st["status"] == 0 and st["relres_true"] <= 1e-8, st
    assert st["vcycles"] >= st["iters"] + 1
    print(f"[near-binary 512] iters={st['iters']} vcycles={st['vcycles']} relres_true={st['relres_true']:.2e}")


@pytest.fixture(scope="module")
def nearbinary2048():
    p = make_problem("wall2048")
    out = {}
    for prec in ("fp64", "fp32mg"):
        print(f"[near-binary 2048] {prec} solve", flush=True)
        s = gpu_solver(p, prec)
        st = s.solve(1e-8, 60000)[0]
        c, dc = s.compliance_and_grad(0)
        out[prec] = (st, s.U(0).cpu().numpy(), c.item(), dc[0].cpu().numpy())
        print(f"[near-binary 2048] {prec} iters={st['iters']} vcycles={st['vcycles']} "
              f"solve_ms={st['t_solve_ms']:.0f} relres_true={st['relres_true']:.2e}", flush=True)
        del s
        torch.cuda.empty_cache()
    return p, out


def _residual_floor(p, U):
    """eps ||(|K| |u|)_free|| / ||f||: the rounding floor of an FP64
    evaluation of f - K u (oracle element matrices, absolute values)."""
    KEa = np.abs(fe.element_stiffness(p.nu))
    E = fe.interpolate_modulus(p.x, p.E_phase, p.E_min, p.penal).ravel()
    dofs = fe.element_dof_map(p.nelx, p.nely)
    au = np.abs(U.ravel())
    acc = np.zeros(U.size)
    for a in range(8):
        acc += np.bincount(dofs[:, a], weights=E * (au[dofs] @ KEa[a]), minlength=U.size)
    free = fe.free_dofs(p.nelx, p.nely)
    return np.finfo(np.float64).eps * np.linalg.norm(acc[free]) / np.linalg.norm(p.F[0].ravel()[free])


# Residual floor of an FP64 displacement field for the 2048^2 near-binary
# design: rounding each entry of its solution to FP64 (half an ulp, random
# signs) changes f - K u by 1.06e-7 ||f||, measured in extended precision
# (64-bit mantissa) on the GPU's solution, whose own residual evaluated there
# equals the GPU's FP64 evaluation (6.16e-8).  The near-rigid parts of this
# compliant design carry displacements up to 2e5 while ||f|| = 0.022, so no
# FP64 u meets 1e-8.
NEARBINARY2048_FP64_FLOOR = 1.1e-7


@pytest.mark.parametrize("prec", ["fp64", "fp32mg"])
def test_nearbinary2048_converges_with_oracle_properties(nearbinary2048, prec):
    """The recursive residual reaches 1e-8; the true residual reaches the
    FP64 floor of this design (above 1e-8, see NEARBINARY2048_FP64_FLOOR),
    and the solver reports NOT_CONVERGED rather than claiming 1e-8."""
    p, out = nearbinary2048
    st, U, c, dc = out[prec]
    floor = _residual_floor(p, U[0])
    print(f"[near-binary 2048] {prec} relres_true={st['relres_true']:.2e} (FP64 floor {NEARBINARY2048_FP64_FLOOR:.1e})")
    assert st["relres_rec"] <= 1e-8, st
    assert st["relres_true"] <= NEARBINARY2048_FP64_FLOOR, st
    assert st["status"] == (0 if st["relres_true"] <= 1e-8 else -2), st
    # c = f.u and u^T K u differ by r.u, |r.u| <= ||r|| ||u|| with ||r|| = relres ||f||
    E = fe.interpolate_modulus(p.x, p.E_phase, p.E_min, p.penal)
    energy = np.sum(E * fe.element_energies(U[0], p.nelx, p.nely, p.nu))
    gap = st["relres_true"] * np.linalg.norm(p.F[0]) * np.linalg.norm(U[0]) / c
    assert c == pytest.approx(energy, rel=max(1e-7, 2 * gap))
    # the oracle's residual at sampled nodes is part of the reported true residual
    nodes = np.random.default_rng(8).choice((p.nelx + 1) * (p.nely + 1), 2000, replace=False)
    r = _nodal_residual(p, U[0], nodes)
    assert np.linalg.norm(r) <= max(1e-8, st["relres_true"] + 2 * floor) * np.linalg.norm(p.F[0])
    # oracle sensitivity formula at sampled elements on the GPU displacements
    KE = fe.element_stiffness(p.nu)
    rng = np.random.default_rng(9)
    els = rng.choice(p.nelx * p.nely, 64, replace=False)
    ph = rng.integers(0, p.m, 64)
    ue = U[0].ravel()[fe.element_dof_map(p.nelx, p.nely)[els]]
    w = np.einsum("ea,ab,eb->e", ue, KE, ue)
    xs = p.x.reshape(-1, p.m)[els, ph]
    want = -p.penal * xs ** (p.penal - 1) * (p.E_phase[ph] - p.E_min) * w
    # u_e^T K0 u_e cancels for near-rigid elements (large u, tiny strain):
    # the kernel's strain/stress form and the oracle's 8x8 product round
    # differently there, by ~1e-11 relative
    assert relerr(dc.reshape(-1, p.m)[els, ph], want) <= 1e-9


def test_nearbinary2048_precisions_agree(nearbinary2048):
    _, out = nearbinary2048
    c64, c32 = out["fp64"][2], out["fp32mg"][2]
    assert c32 == pytest.approx(c64, rel=1e-7)
