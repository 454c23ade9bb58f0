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

Usage: python tests/golden/make_golden.py [wall1024] [batch32]
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

from oracle import fe, solve  # noqa: E402
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
        make(name)
