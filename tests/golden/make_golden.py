"""Write sampled oracle values for the full-size square-wall workloads.

Calls only the CPU oracle (oracle/) and the seeded input generators
(workloads/); nothing here touches the HIP library.  For each workload the
oracle solves with its own MG-preconditioned CG to a relative residual of
1e-11 and stores: the compliance, ||u||_2, u at 512 seeded nodes, and the
compliance gradient at 64 seeded (element, phase) pairs.  The GPU parity
tests compare the HIP solve with these samples.

Usage: python tests/golden/make_golden.py [wall1024]
(about 3 minutes on one host core).  The 2048 x 2048 near-binary field is
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
from workloads import make_problem  # noqa: E402


def sample_indices(n_nodes: int, n_elem: int, m: int, seed: int):
    rng = np.random.default_rng(seed)
    nodes = np.sort(rng.choice(n_nodes, 512, replace=False))
    elems = rng.choice(n_elem, 64, replace=False)
    phases = rng.integers(0, m, 64)
    return nodes, elems, phases


def make(name: str):
    p = make_problem(name)
    t0 = time.time()
    sol = solve.solve_mgpcg(p.nelx, p.nely, p.x, p.E_phase, p.E_min, p.penal, p.nu, p.F, p.levels,
                            rel_tol=1e-11, max_iter=2000, grad=False)
    U = sol.U[0]
    n_nodes = (p.nelx + 1) * (p.nely + 1)
    nodes, elems, phases = sample_indices(n_nodes, p.nelx * p.nely, p.m, 12345)
    Uf = U.reshape(-1, 2)
    # the oracle's gradient (Eq. 6 and the sensitivity step of Section 4), sampled
    g = fe.compliance_gradient(p.x, U, p.E_phase, p.E_min, p.penal, p.nu).reshape(-1, p.m)[elems, phases]
    out = {
        "workload": name,
        "source": "oracle/solve.py solve_mgpcg (FP64 scipy, pCGMG) to relative residual 1e-11",
        "nelx": p.nelx, "nely": p.nely, "levels": p.levels,
        "oracle_iters": int(sol.iters[0]),
        "oracle_relres_true": float(sol.relres[0]),
        "compliance": float(sol.c[0]),
        "u_norm": float(np.linalg.norm(U)),
        "nodes": nodes.tolist(),
        "u_nodes": Uf[nodes].tolist(),
        "grad_elems": elems.tolist(),
        "grad_phases": phases.tolist(),
        "grad": g.tolist(),
        "seconds": time.time() - t0,
    }
    path = os.path.join(HERE, f"{name}_samples.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print(f"{name}: c={out['compliance']:.12g} iters={out['oracle_iters']} relres={out['oracle_relres_true']:.2e} "
          f"({out['seconds']:.0f} s) -> {path}")


if __name__ == "__main__":
    for name in (sys.argv[1:] or ["wall1024"]):
        make(name)
