// Poisson model problem of Section 5.1: -Laplace(u) = f on the unit square
// with u = 0 on the boundary, Q4 elements on an n x n grid.  On every grid
// the operator is the Q4 Laplace stencil (the Galerkin product of the finer
// one, which is scale-free in 2D): (K u)_c = (8 u_c - sum of the 8
// neighbours) / 3 at interior nodes.  Nodal arrays are [n+1][n+1] FP64,
// row-major, boundary entries held at 0.
#pragma once

#include <hip/hip_runtime.h>

namespace mtomg {

// r = f - K u at interior nodes, 0 on the boundary (u == nullptr: u = 0).
void launch_pois_residual(hipStream_t st, int n, const double* f, const double* u, double* r);
// q = K u at interior nodes, 0 on the boundary.
void launch_pois_apply(hipStream_t st, int n, const double* u, double* q);
// u_out = u_in + omega (3/8) (b - K u_in) at interior nodes (u_in == nullptr: 0).
void launch_pois_jacobi(hipStream_t st, int n, double omega, const double* b, const double* u_in, double* u_out);
// b_c = P^T r_f, full weighting (weights 1, 1/2, 1/4), from the 2n_c grid to the n_c grid.
void launch_pois_restrict(hipStream_t st, int nc, const double* rf, double* bc);
// u_f += P e_c (bilinear), interior fine nodes.
void launch_pois_prolong_add(hipStream_t st, int nc, const double* ec, double* uf);
// 2 x 2 coarsest grid: its one unknown e = b / (8/3); boundary entries 0.
void launch_pois_coarse(hipStream_t st, const double* b, double* e);
// y += sa (num / den) x (num, den device scalars), every node; nothing when
// *state != 0 (state may be null).
void launch_pois_axpy(hipStream_t st, int n, const double* num, const double* den, double sa, const double* x,
                      double* y, const int* state);
// p = z + (num / den) p (num, den device scalars; den == nullptr: p = z);
// nothing when *state != 0 (state may be null).
void launch_pois_xpby(hipStream_t st, int n, const double* z, const double* num, const double* den, double* p,
                      const int* state);
// The PCG tests on the device: sc = {f.f, r.z, r.z, p.q, r.r}; state[0]
// (0 running, 1 converged, 3 breakdown, 4 not finite), state[1] iterations.
void launch_pois_check(hipStream_t st, const double* sc, double tol2, int* state);
void launch_pois_check_rz(hipStream_t st, const double* rz, int* state);

}  // namespace mtomg
