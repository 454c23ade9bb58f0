"""Write sampled oracle values for the full-size square-wall workloads.

Calls only the CPU oracle (oracle/) and the seeded input generators
(workloads/); nothing here touches the HIP library.  For each workload the
oracle solves with its own MG-preconditioned CG to a relative residual of
1e-11 and stores: the compliance, ||u||_2, u at 512 seeded nodes, and the
compliance gradient at 64 seeded (element, phase) pairs.  The GPU parity
tests compare the HIP solve with these samples.

For "batch32", a 768 x 768 design of the 48-design batched workload with its
four load cases, the oracle's direct solve (the plain definition u_f =
K_ff^{-1} f_f by a sparse factorisation) supplies the values instead, per
load case.

"nearbinary_iters" stores the oracle's pCGMG iteration counts on the
near-binary recipe at 128^2 and 256^2 instead, in FP64 (also with the loads
scaled by rounding-level factors) and in extended precision.

"nearbinary_history" stores the oracle's recursive relative residual after
each of the first 60 pCGMG iterations on the same recipe: where the counts
above depend on rounding, the early history does not.

Usage: python tests/golden/make_golden.py [wall1024] [batch32] [nearbinary_iters] [nearbinary_history]
(about 3 minutes each on one host core).  The 2048 x 2048 near-binary field is
not sampled this way: pCGMG needs ~1e4 iterations there and the oracle's
scipy cycle does not finish in hours, so that workload is checked through
properties that hold at any size instead.
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import fe, linalg, multigrid, solve  # noqa: E402
from workloads import batched_design, make_problem  # noqa: E402


def sample_indices(n_nodes: int, n_elem: int, m: int, seed: int):
    rng = np.random.default_rng(seed)
    nodes = np.sort(rng.choice(n_nodes, 512, replace=False))
    elems = rng.choice(n_elem, 64, replace=False)
    phases = rng.integers(0, m, 64)
    return nodes, elems, phases


def _case_samples(p, U, nodes, elems, phases):
    Uf = U.reshape(-1, 2)
    # the oracle's gradient (Eq. 6 and the sensitivity step of Section 4), sampled
    g = fe.compliance_gradient(p.x, U, p.E_phase, p.E_min, p.penal, p.nu).reshape(-1, p.m)[elems, phases]
    return {"u_norm": float(np.linalg.norm(U)), "u_nodes": Uf[nodes].tolist(), "grad": g.tolist()}


def make_nearbinary_iters():
    """pCGMG iteration counts of the oracle (FP64 cycle, 2 + 2 damped Jacobi,
    omega 0.6, relative residual 1e-8) on the near-binary 4-phase recipe at
    128^2 (4 grids) and 256^2 (5 grids)."""
    out = {"source": "oracle/solve.py solve_mgpcg (scipy, pCGMG; FP64 and long double) to relative residual 1e-8",
           "recipe": "workloads make_problem('wall2048', n, levels)", "cases": []}
    # the count of this ill-conditioned recipe moves by several percent under
    # rounding-level changes of the data, so each case is also solved with
    # the loads scaled by 1 + 2^-50, 1 - 2^-50 and 3 (every rounding changes,
    # the solution only by that factor)
    for n, lv in ((128, 4), (256, 5)):
        t0 = time.time()
        p = make_problem("wall2048", n=n, levels=lv)
        iters = []
        for scale in (1.0, 1.0 + 2.0 ** -50, 1.0 - 2.0 ** -50, 3.0):
            sol = solve.solve_mgpcg(p.nelx, p.nely, p.x, p.E_phase, p.E_min, p.penal, p.nu, p.F * scale, p.levels,
                                    rel_tol=1e-8, max_iter=20000, grad=False)
            iters.append(int(sol.iters[0]))
            relres = float(sol.relres[0]) if scale == 1.0 else relres
        # the same run with every step in long double: the count with much
        # less rounding in it
        ext = solve.solve_mgpcg(p.nelx, p.nely, p.x, p.E_phase, p.E_min, p.penal, p.nu, p.F, p.levels,
                                rel_tol=1e-8, max_iter=20000, grad=False, dtype=np.longdouble)
        out["cases"].append({"n": n, "levels": lv, "iters": iters[0], "iters_perturbed": iters[1:],
                             "load_scales": [1.0 + 2.0 ** -50, 1.0 - 2.0 ** -50, 3.0],
                             "iters_extended": int(ext.iters[0]),
                             "extended_mantissa_bits": int(np.finfo(np.longdouble).nmant) + 1,
                             "relres_true": relres, "seconds": time.time() - t0})
        print(out["cases"][-1], flush=True)
    path = os.path.join(HERE, "nearbinary_iters.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)


def make_nearbinary_history(n_iter: int = 60):
    """||r_k|| / ||f|| for k = 0 .. n_iter of the oracle's pCGMG (FP64, Algorithm 2
    with one V-cycle of Algorithm 1 per iteration) on the near-binary recipe."""
    out = {"source": "oracle linalg.pcg with multigrid.preconditioner (FP64), recursive residual",
           "recipe": "workloads make_problem('wall2048', n, levels)", "cases": []}
    for n, lv in ((128, 4), (256, 5)):
        p = make_problem("wall2048", n=n, levels=lv)
        _, K, Kff, free = solve.system(p.nelx, p.nely, p.x, p.E_phase, p.E_min, p.penal, p.nu)
        M = multigrid.preconditioner(multigrid.Hierarchy(p.nelx, p.nely, Kff, p.levels))
        res = linalg.pcg(lambda v: Kff @ v, p.F[0].ravel()[free], M, rel_tol=0.0, max_iter=n_iter)
        out["cases"].append({"n": n, "levels": lv, "history": [float(h) for h in res.history]})
        print(n, out["cases"][-1]["history"][:6], flush=True)
    with open(os.path.join(HERE, "nearbinary_history.json"), "w") as fh:
        json.dump(out, fh, indent=1)


def make(name: str):
    t0 = time.time()
    if name.startswith("batch"):
        p = batched_design(int(name[5:]))
        sol = solve.solve_direct(p.nelx, p.nely, p.x, p.E_phase, p.E_min, p.penal, p.nu, p.F, grad=False)
        source = "oracle/solve.py solve_direct (FP64 sparse LU of K_ff), every load case"
    else:
        p = make_problem(name)
        sol = solve.solve_mgpcg(p.nelx, p.nely, p.x, p.E_phase, p.E_min, p.penal, p.nu, p.F, p.levels,
                                rel_tol=1e-11, max_iter=2000, grad=False)
        source = "oracle/solve.py solve_mgpcg (FP64 scipy, pCGMG) to relative residual 1e-11"
    n_nodes = (p.nelx + 1) * (p.nely + 1)
    nodes, elems, phases = sample_indices(n_nodes, p.nelx * p.nely, p.m, 12345)
    cases = [_case_samples(p, sol.U[k], nodes, elems, phases) for k in range(sol.U.shape[0])]
    out = {
        "workload": name,
        "source": source,
        "nelx": p.nelx, "nely": p.nely, "levels": p.levels,
        "oracle_iters": [int(i) for i in sol.iters],
        "oracle_relres_true": [float(r) for r in sol.relres],
        "nodes": nodes.tolist(),
        "grad_elems": elems.tolist(),
        "grad_phases": phases.tolist(),
        "compliance": [float(c) for c in sol.c],
        "cases": cases,
        "seconds": time.time() - t0,
    }
    path = os.path.join(HERE, f"{name}_samples.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print(f"{name}: c={out['compliance']} iters={out['oracle_iters']} relres={out['oracle_relres_true']} "
          f"({out['seconds']:.0f} s) -> {path}")


if __name__ == "__main__":
    for name in (sys.argv[1:] or ["wall1024"]):
        if name == "nearbinary_iters":
            make_nearbinary_iters()
        elif name == "nearbinary_history":
            make_nearbinary_history()
        else:
            make(name)
