// Kernels of the Poisson model problem (Section 5.1): one thread per node of
// an [n+1][n+1] grid, the 9-point Q4 Laplace stencil read straight from
// HBM/L2 (neighbouring threads share rows, so every value is fetched once
// from HBM).  The work is a few bytes per node and the grids of Section 5.1
// are small, so these kernels are launch- and latency-bound; they keep the
// multigrid and PCG steps of Algorithms 1 and 2 on the device.
#include "poisson_kernels.h"

namespace mtomg {

namespace {

constexpr int PT = 256;

__device__ __forceinline__ bool pois_interior(int i, int j, int n) { return i >= 1 && i < n && j >= 1 && j < n; }

// (K u) at interior node (i, j); u may be nullptr (zero).
__device__ __forceinline__ double pois_apply(const double* __restrict__ u, int i, int j, int n) {
    if (!u) return 0.0;
    const int w = n + 1;
    const double* c = u + (size_t)j * w + i;
    const double nb = (c[-w - 1] + c[-w] + c[-w + 1]) + (c[-1] + c[1]) + (c[w - 1] + c[w] + c[w + 1]);
    return (8.0 * c[0] - nb) / 3.0;
}

__global__ void k_pois_residual(int n, const double* __restrict__ f, const double* __restrict__ u,
                                double* __restrict__ r) {
    const int id = blockIdx.x * PT + threadIdx.x;
    const int w = n + 1;
    if (id >= w * w) return;
    const int i = id % w, j = id / w;
    r[id] = pois_interior(i, j, n) ? f[id] - pois_apply(u, i, j, n) : 0.0;
}

__global__ void k_pois_apply(int n, const double* __restrict__ u, double* __restrict__ q) {
    const int id = blockIdx.x * PT + threadIdx.x;
    const int w = n + 1;
    if (id >= w * w) return;
    const int i = id % w, j = id / w;
    q[id] = pois_interior(i, j, n) ? pois_apply(u, i, j, n) : 0.0;
}

__global__ void k_pois_jacobi(int n, double omega, const double* __restrict__ b, const double* __restrict__ u_in,
                              double* __restrict__ u_out) {
    const int id = blockIdx.x * PT + threadIdx.x;
    const int w = n + 1;
    if (id >= w * w) return;
    const int i = id % w, j = id / w;
    double v = 0.0;
    if (pois_interior(i, j, n)) {
        const double u0 = u_in ? u_in[id] : 0.0;
        v = u0 + omega * (b[id] - pois_apply(u_in, i, j, n)) / (8.0 / 3.0);
    }
    u_out[id] = v;
}

__global__ void k_pois_restrict(int nc, const double* __restrict__ rf, double* __restrict__ bc) {
    const int id = blockIdx.x * PT + threadIdx.x;
    const int wc = nc + 1, wf = 2 * nc + 1;
    if (id >= wc * wc) return;
    const int I = id % wc, J = id / wc;
    double v = 0.0;
    if (pois_interior(I, J, nc)) {
        const double* c = rf + (size_t)(2 * J) * wf + 2 * I;
        const double row_m = 0.5 * c[-wf - 1] + c[-wf] + 0.5 * c[-wf + 1];
        const double row_0 = 0.5 * c[-1] + c[0] + 0.5 * c[1];
        const double row_p = 0.5 * c[wf - 1] + c[wf] + 0.5 * c[wf + 1];
        v = 0.5 * row_m + row_0 + 0.5 * row_p;
    }
    bc[id] = v;
}

__global__ void k_pois_prolong_add(int nc, const double* __restrict__ ec, double* __restrict__ uf) {
    const int id = blockIdx.x * PT + threadIdx.x;
    const int nf = 2 * nc, wf = nf + 1, wc = nc + 1;
    if (id >= wf * wf) return;
    const int i = id % wf, j = id / wf;
    if (!pois_interior(i, j, nf)) return;
    const int I0 = i >> 1, J0 = j >> 1;
    const int I1 = I0 + (i & 1), J1 = J0 + (j & 1);
    const double wx = (i & 1) ? 0.5 : 1.0, wy = (j & 1) ? 0.5 : 1.0;
    double v = ec[(size_t)J0 * wc + I0];
    if (i & 1) v += ec[(size_t)J0 * wc + I1];
    if (j & 1) {
        v += ec[(size_t)J1 * wc + I0];
        if (i & 1) v += ec[(size_t)J1 * wc + I1];
    }
    uf[id] += wx * wy * v;
}

__global__ void k_pois_coarse(const double* __restrict__ b, double* __restrict__ e) {
    const int id = threadIdx.x;
    if (id < 9) e[id] = id == 4 ? b[4] / (8.0 / 3.0) : 0.0;
}

__global__ void k_pois_axpy(int n, const double* __restrict__ num, const double* __restrict__ den, double sa,
                            const double* __restrict__ x, double* __restrict__ y, const int* state) {
    if (state && *state != 0) return;
    const int id = blockIdx.x * PT + threadIdx.x;
    const int w = n + 1;
    if (id >= w * w) return;
    y[id] += (sa * (*num / *den)) * x[id];
}

__global__ void k_pois_xpby(int n, const double* __restrict__ z, const double* __restrict__ num,
                            const double* __restrict__ den, double* __restrict__ p, const int* state) {
    if (state && *state != 0) return;
    const int id = blockIdx.x * PT + threadIdx.x;
    const int w = n + 1;
    if (id >= w * w) return;
    p[id] = den ? z[id] + (*num / *den) * p[id] : z[id];
}

// Convergence and breakdown tests of one PCG iteration on the device
// (state[0]: 0 running, 1 converged, 3 breakdown, 4 not finite; state[1]:
// iterations whose update of u ran).  After the update: count it, then stop
// on a non-finite p.q or r.r, on p.q <= 0, or on r.r <= tol2 f.f.
__global__ void k_pois_check(const double* __restrict__ sc, double tol2, int* __restrict__ state) {
    if (threadIdx.x != 0 || state[0] != 0) return;
    const double ff = sc[0], pq = sc[3], rr = sc[4];
    state[1] += 1;
    if (!isfinite(rr) || !isfinite(pq)) state[0] = 4;
    else if (!(pq > 0.0)) state[0] = 3;
    else if (rr <= tol2 * ff) state[0] = 1;
}

// After the next preconditioner application: breakdown on r.z <= 0.
__global__ void k_pois_check_rz(const double* __restrict__ rz, int* __restrict__ state) {
    if (threadIdx.x != 0 || state[0] != 0) return;
    if (!(*rz > 0.0)) state[0] = isfinite(*rz) ? 3 : 4;
}

inline dim3 grid_of(int n) { return dim3((unsigned)(((size_t)(n + 1) * (n + 1) + PT - 1) / PT)); }

}  // namespace

void launch_pois_residual(hipStream_t st, int n, const double* f, const double* u, double* r) {
    hipLaunchKernelGGL(k_pois_residual, grid_of(n), dim3(PT), 0, st, n, f, u, r);
}
void launch_pois_apply(hipStream_t st, int n, const double* u, double* q) {
    hipLaunchKernelGGL(k_pois_apply, grid_of(n), dim3(PT), 0, st, n, u, q);
}
void launch_pois_jacobi(hipStream_t st, int n, double omega, const double* b, const double* u_in, double* u_out) {
    hipLaunchKernelGGL(k_pois_jacobi, grid_of(n), dim3(PT), 0, st, n, omega, b, u_in, u_out);
}
void launch_pois_restrict(hipStream_t st, int nc, const double* rf, double* bc) {
    hipLaunchKernelGGL(k_pois_restrict, grid_of(nc), dim3(PT), 0, st, nc, rf, bc);
}
void launch_pois_prolong_add(hipStream_t st, int nc, const double* ec, double* uf) {
    hipLaunchKernelGGL(k_pois_prolong_add, grid_of(2 * nc), dim3(PT), 0, st, nc, ec, uf);
}
void launch_pois_coarse(hipStream_t st, const double* b, double* e) {
    hipLaunchKernelGGL(k_pois_coarse, dim3(1), dim3(64), 0, st, b, e);
}
void launch_pois_axpy(hipStream_t st, int n, const double* num, const double* den, double sa, const double* x,
                      double* y, const int* state) {
    hipLaunchKernelGGL(k_pois_axpy, grid_of(n), dim3(PT), 0, st, n, num, den, sa, x, y, state);
}
void launch_pois_xpby(hipStream_t st, int n, const double* z, const double* num, const double* den, double* p,
                      const int* state) {
    hipLaunchKernelGGL(k_pois_xpby, grid_of(n), dim3(PT), 0, st, n, z, num, den, p, state);
}
void launch_pois_check(hipStream_t st, const double* sc, double tol2, int* state) {
    hipLaunchKernelGGL(k_pois_check, dim3(1), dim3(64), 0, st, sc, tol2, state);
}
void launch_pois_check_rz(hipStream_t st, const double* rz, int* state) {
    hipLaunchKernelGGL(k_pois_check_rz, dim3(1), dim3(64), 0, st, rz, state);
}

}  // namespace mtomg
