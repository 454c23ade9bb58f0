"""Graph-replayed PCG iterations give exactly the eager result.

The iteration body (two PCG iterations) is captured once and replayed many
times per solve; between replays the host reads the convergence state, and
between solves eager kernels (setup, residuals, gradient) run on the same
stream.  Every replayed solve is compared bitwise with the same solve
launched kernel by kernel.
"""

import numpy as np
import pytest
import torch

from paper_2301_07457_amd import _lib
from tests.gpu_util import gpu_solver
from workloads import Problem, load_top_traction

pytestmark = pytest.mark.gpu


def rand_prob(nx, ny, L, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.05, 1.0, (ny, nx, 3)) / 3
    return Problem("rand", nx, ny, x, np.array([1.0, 0.6, 0.2]), 1e-9, 3.0, 0.3,
                   load_top_traction(nx, ny)[None], L)


@pytest.mark.parametrize("prec", ["fp64", "fp32mg"])
def test_graph_replays_match_eager(prec):
    p = rand_prob(128, 96, 4, 21)
    se = gpu_solver(p, prec)
    _lib.mtomg_set_option(se.ctx, "GRAPHS", 0)
    sg = gpu_solver(p, prec)
    _lib.mtomg_set_option(sg.ctx, "BATCH", 2)     # many host checks between replays
    rng = np.random.default_rng(0)
    x = p.x.copy()
    for rep in range(4):
        for tol in (1e-8, 1e-10):
            ste = se.solve(tol, 1000)[0]
            Ue = se.U(0).clone()
            stg = sg.solve(tol, 1000)[0]
            Ug = sg.U(0).clone()
            assert ste["status"] == 0 and stg["status"] == 0
            assert ste["iters"] == stg["iters"]
            assert torch.equal(Ue, Ug), (rep, tol)
            ce, _ = se.compliance_and_grad(0)
            cg, _ = sg.compliance_and_grad(0)
            assert torch.equal(ce, cg)
        # eager work between replays: new densities for both
        x = np.clip(x * (1 + 0.05 * rng.standard_normal(x.shape)), 0.0, 1.0)
        se.set_densities(0, torch.from_numpy(x))
        sg.set_densities(0, torch.from_numpy(x))
