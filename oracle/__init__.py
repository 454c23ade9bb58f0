"""CPU oracle for the pCGMG compliance solve — TEST INFRASTRUCTURE ONLY.

A plain, slow, FP64 reimplementation of what the HIP solver computes,
written from the paper (Luu & Banh, "A novel preconditioned conjugate
gradient multigrid method for multi-material topology optimization"):

* ``fe``        — multi-phase SIMP modulus (Eq. 5), Q4 plane-stress element
                  stiffness (Eqs. 7-9), assembly, clamped/traction boundary
                  conditions (Eq. 10), compliance (Eq. 6) and its gradient.
* ``linalg``    — dense Cholesky (Algorithm 3 with Eqs. 3-4), triangular
                  substitution, damped Jacobi (Section 2.3) and
                  preconditioned CG (Algorithm 2).
* ``multigrid`` — bilinear prolongation, restriction as its transpose,
                  Galerkin coarse operators and the gamma-cycle
                  (Algorithm 1) used as a PCG preconditioner (Section 2.2).
* ``cone_filter`` — the cone density and sensitivity filters of the
                  optimisation loop (Section 4, radius rf of Table 2).
* ``poisson``   — the Poisson model problem of Section 5.1 (scalar Q4,
                  zero boundary values) with its Galerkin hierarchy.
* ``oc``        — the alternating active-phase optimality-criteria loop of
                  Section 4 (pairs of phases in Gauss-Seidel order, each a
                  binary sub-problem with a bisection on the multiplier).
* ``solve``     — the plain definition u = K_ff^{-1} f_f by a direct solve,
                  and the oracle's own MG-preconditioned CG.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP path
and never imports it.
"""

from . import cone_filter, fe, linalg, multigrid, oc, poisson, solve  # noqa: F401
