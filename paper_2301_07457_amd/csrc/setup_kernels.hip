// Per-design setup of the preconditioner and post-solve kernels:
//  * element moduli from phase densities (Eq. 5, implicit void phase);
//  * Galerkin coarse operators as six moments per coarse element, computed
//    exactly by a 2x2 -> 1 recursion (FP64 accumulation);
//  * dense coarsest matrix, its Cholesky factor (Algorithm 3, right-looking)
//    and the explicit inverse K_0^{-1} = L^-T L^-1 used by the coarse solve;
//  * compliance gradient dc/dx = -p x^(p-1) (E_i - E_min) u_e^T K^0 u_e and
//    fixed-order reductions.
#include "device_common.h"
#include "kernels.h"

namespace mtomg {

__global__ void k_interp(const double* __restrict__ x, Phases ph, int n_e, double* __restrict__ E64,
                         float* __restrict__ E32) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_e) return;
    double E = ph.E_min;
    for (int k = 0; k < ph.m; ++k) E += pow(x[(size_t)e * ph.m + k], ph.penal) * ph.dE[k];
    E64[e] = E;
    if (E32) E32[e] = (float)E;
}

__global__ void k_moments_from_fine(const double* __restrict__ E, int nxf, int nyf, double* __restrict__ m64,
                                    float* __restrict__ m32) {
    const int nxc = nxf / 2, nyc = nyf / 2;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nxc * nyc) return;
    const int I = e % nxc, J = e / nxc;
    Mom<double> P = mom_zero<double>();
    for (int t = 0; t < 2; ++t)
        for (int s = 0; s < 2; ++s)
            mom_accumulate_child(P, mom_const<double>(E[(size_t)(2 * J + t) * nxf + 2 * I + s]), s, t);
    const size_t ps = (size_t)nxc * nyc;
    const double v[6] = {P.m00, P.m10, P.m01, P.m20, P.m11, P.m02};
    for (int k = 0; k < 6; ++k) {
        m64[k * ps + e] = v[k];
        if (m32) m32[k * ps + e] = (float)v[k];
    }
}

__global__ void k_moments_coarsen(const double* __restrict__ mf, int nxf, int nyf, double* __restrict__ m64,
                                  float* __restrict__ m32) {
    const int nxc = nxf / 2, nyc = nyf / 2;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nxc * nyc) return;
    const int I = e % nxc, J = e / nxc;
    const size_t pf = (size_t)nxf * nyf;
    Mom<double> P = mom_zero<double>();
    for (int t = 0; t < 2; ++t)
        for (int s = 0; s < 2; ++s) {
            const size_t c = (size_t)(2 * J + t) * nxf + 2 * I + s;
            const Mom<double> ch{mf[c], mf[pf + c], mf[2 * pf + c], mf[3 * pf + c], mf[4 * pf + c],
                                 mf[5 * pf + c]};
            mom_accumulate_child(P, ch, s, t);
        }
    const size_t ps = (size_t)nxc * nyc;
    const double v[6] = {P.m00, P.m10, P.m01, P.m20, P.m11, P.m02};
    for (int k = 0; k < 6; ++k) {
        m64[k * ps + e] = v[k];
        if (m32) m32[k * ps + e] = (float)v[k];
    }
}

// Dense free-DOF matrix of the coarsest grid: thread per (free node, one of
// its 9 neighbours); each computes the 2x2 block as the sum over the shared
// elements of element responses to unit displacements.
template <bool FINE>
__global__ void k_assemble_dense(LevelOp<double> op, Mat<double> mat, double* __restrict__ A) {
    const int nx = op.nx, ny = op.ny;
    const int n0 = 2 * (nx + 1) * ny;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int node = t / 9, o = t % 9;
    if (node >= (nx + 1) * ny) return;
    const int i = node % (nx + 1), j = node / (nx + 1) + 1;
    const int mi = i + (o % 3) - 1, mj = j + (o / 3) - 1;
    if (mi < 0 || mi > nx || mj < 1 || mj > ny) return;
    double blk[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    for (int ej = j - 1; ej <= j; ++ej)
        for (int ei = i - 1; ei <= i; ++ei) {
            if (ei < 0 || ei >= nx || ej < 0 || ej >= ny) continue;
            const int ln_x = i - ei, ln_y = j - ej, lm_x = mi - ei, lm_y = mj - ej;
            if (lm_x < 0 || lm_x > 1 || lm_y < 0 || lm_y > 1) continue;
            const int ln = ln_y ? (ln_x ? 2 : 3) : (ln_x ? 1 : 0);
            const int lm = lm_y ? (lm_x ? 2 : 3) : (lm_x ? 1 : 0);
            const Mom<double> m = load_elem<double, FINE>(op, ei, ej);
            for (int b = 0; b < 2; ++b) {
                V2<double> u[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
                if (b == 0) u[lm].x = 1.0; else u[lm].y = 1.0;
                V2<double> f[4];
                elem_force(m, mat, u[0], u[1], u[2], u[3], f[0], f[1], f[2], f[3]);
                blk[0][b] += f[ln].x;
                blk[1][b] += f[ln].y;
            }
        }
    const int rn = 2 * ((j - 1) * (nx + 1) + i), cm = 2 * ((mj - 1) * (nx + 1) + mi);
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) A[(size_t)(rn + a) * n0 + cm + b] = blk[a][b];
}

// In-place Cholesky A = L L^T of the lower triangle (Algorithm 3: pivot
// square root, column scaling, trailing outer-product update), one
// workgroup.  status = 1 if a pivot is not positive.
__global__ __launch_bounds__(1024) void k_cholesky(double* __restrict__ A, int n, int* __restrict__ status) {
    extern __shared__ double col[];
    __shared__ double piv;
    const int tid = threadIdx.x, nth = blockDim.x;
    const int lane = tid & 63, wv = tid >> 6, nw = nth >> 6;
    for (int k = 0; k < n; ++k) {
        if (tid == 0) {
            const double a = A[(size_t)k * n + k];
            if (a > 0.0) {
                piv = sqrt(a);
                A[(size_t)k * n + k] = piv;
            } else {
                piv = -1.0;
                *status = 1;
            }
        }
        __syncthreads();
        if (!(piv > 0.0)) return;
        const double inv = 1.0 / piv;
        for (int r = k + 1 + tid; r < n; r += nth) {
            const double v = A[(size_t)r * n + k] * inv;
            A[(size_t)r * n + k] = v;
            col[r] = v;
        }
        __syncthreads();
        for (int r = k + 1 + wv; r < n; r += nw) {
            const double lr = col[r];
            double* row = A + (size_t)r * n;
            for (int c = k + 1 + lane; c <= r; c += 64) row[c] -= lr * col[c];
        }
        __syncthreads();
    }
}

// W = L^{-1} by forward substitution, one wave per column c (two waves per
// block); the running column lives in LDS.  W row-major, lower triangular.
__global__ __launch_bounds__(128) void k_trinv(const double* __restrict__ L, double* __restrict__ W, int n) {
    extern __shared__ double wl[];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int c = blockIdx.x * 2 + wv;
    if (c >= n) return;
    double* w = wl + (size_t)wv * n;
    for (int r = lane; r < n; r += 64) w[r] = 0.0;
    __syncthreads();
    for (int r = c; r < n; ++r) {
        const double* Lr = L + (size_t)r * n;
        double s = 0.0;
        for (int t = c + lane; t < r; t += 64) s += Lr[t] * w[t];
        s = wave_sum(s);
        s = __shfl(s, 0, 64);
        const double v = ((r == c ? 1.0 : 0.0) - s) / Lr[r];
        if (lane == 0) w[r] = v;
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_wave_barrier();
    }
    for (int r = lane; r < n; r += 64) W[(size_t)r * n + c] = w[r];
}

// K_0^{-1} = W^T W, W = L^{-1}: one wave per output row a, lanes over
// columns; the sum runs over t ascending, so the result is bitwise symmetric.
__global__ __launch_bounds__(256) void k_gram(const double* __restrict__ W, double* __restrict__ Ainv, int n) {
    const int a = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (a >= n) return;
    for (int b0 = 0; b0 < n; b0 += 64) {
        const int b = b0 + lane;
        double s = 0.0;
        const int t0 = a;
        for (int t = t0; t < n; ++t) {
            const double wa = W[(size_t)t * n + a];
            if (b < n) s += wa * W[(size_t)t * n + b];
        }
        if (b < n) Ainv[(size_t)a * n + b] = s;
    }
}

template <typename T>
__global__ void k_fill(T* __restrict__ p, size_t n, T v) {
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) p[k] = v;
}

__global__ void k_cast_f32(const double* __restrict__ a, float* __restrict__ b, size_t n) {
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
        b[k] = (float)a[k];
}

// dc/dx_{e,i} = -p x^(p-1) (E_i - E_min) u_e^T K^0 u_e, one thread per element.
__global__ void k_grad(const double* __restrict__ U, const double* __restrict__ x, Phases ph, Mat<double> mat,
                       int nx, int ny, double* __restrict__ dcdx) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nx * ny) return;
    const int i = e % nx, j = e / nx;
    const V2<double> u0 = load_node(U, nx, ny, i, j), u1 = load_node(U, nx, ny, i + 1, j);
    const V2<double> u2 = load_node(U, nx, ny, i + 1, j + 1), u3 = load_node(U, nx, ny, i, j + 1);
    V2<double> f0, f1, f2, f3;
    elem_force(mom_const<double>(1.0), mat, u0, u1, u2, u3, f0, f1, f2, f3);
    const double w = (u0.x * f0.x + u0.y * f0.y) + (u1.x * f1.x + u1.y * f1.y) +
                     (u2.x * f2.x + u2.y * f2.y) + (u3.x * f3.x + u3.y * f3.y);
    for (int k = 0; k < ph.m; ++k) {
        const double xv = x[(size_t)e * ph.m + k];
        dcdx[(size_t)e * ph.m + k] = -ph.penal * pow(xv, ph.penal - 1.0) * ph.dE[k] * w;
    }
}

// partials[b] = sum over block b's contiguous slice of a . b (fixed order)
__global__ __launch_bounds__(WG_THREADS) void k_dot_partials(const double* __restrict__ a, const double* __restrict__ b,
                                                             size_t n, double* __restrict__ partials) {
    const size_t per = (n + gridDim.x - 1) / gridDim.x;
    const size_t s0 = blockIdx.x * per, s1 = min(n, s0 + per);
    double s = 0.0;
    for (size_t k = s0 + threadIdx.x; k < s1; k += WG_THREADS) s += a[k] * b[k];
    s = block_sum(s);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(WG_THREADS) void k_sums(SumJob job, double* __restrict__ out) {
    for (int k = 0; k < job.count; ++k) {
        const double s = sum_partials(job.p[k], job.n[k]);
        if (threadIdx.x == 0) out[k] = s;
    }
}

// ---------------------------------------------------------------------------
static inline unsigned blocks_for(size_t n, unsigned bs) { return (unsigned)((n + bs - 1) / bs); }

void launch_interp(hipStream_t st, const double* x, Phases ph, int n_e, double* E64, float* E32) {
    hipLaunchKernelGGL(k_interp, dim3(blocks_for(n_e, 256)), dim3(256), 0, st, x, ph, n_e, E64, E32);
}
void launch_moments_from_fine(hipStream_t st, const double* E64, int nxf, int nyf, double* m64, float* m32) {
    const int n = (nxf / 2) * (nyf / 2);
    hipLaunchKernelGGL(k_moments_from_fine, dim3(blocks_for(n, 256)), dim3(256), 0, st, E64, nxf, nyf, m64, m32);
}
void launch_moments_coarsen(hipStream_t st, const double* mf, int nxf, int nyf, double* m64, float* m32) {
    const int n = (nxf / 2) * (nyf / 2);
    hipLaunchKernelGGL(k_moments_coarsen, dim3(blocks_for(n, 256)), dim3(256), 0, st, mf, nxf, nyf, m64, m32);
}
void launch_assemble_dense(hipStream_t st, bool fine, LevelOp<double> op, Mat<double> mat, double* A) {
    const int n = 9 * (op.nx + 1) * op.ny;
    if (fine) hipLaunchKernelGGL(k_assemble_dense<true>, dim3(blocks_for(n, 256)), dim3(256), 0, st, op, mat, A);
    else hipLaunchKernelGGL(k_assemble_dense<false>, dim3(blocks_for(n, 256)), dim3(256), 0, st, op, mat, A);
}
void launch_cholesky(hipStream_t st, double* A, int n, int* status) {
    hipLaunchKernelGGL(k_cholesky, dim3(1), dim3(1024), n * sizeof(double), st, A, n, status);
}
void launch_trinv(hipStream_t st, const double* L, double* W, int n) {
    hipLaunchKernelGGL(k_trinv, dim3((n + 1) / 2), dim3(128), 2 * n * sizeof(double), st, L, W, n);
}
void launch_gram(hipStream_t st, const double* W, double* Ainv, int n) {
    hipLaunchKernelGGL(k_gram, dim3((n + 3) / 4), dim3(256), 0, st, W, Ainv, n);
}
template <typename T>
void launch_fill(hipStream_t st, T* p, size_t n, T v) {
    if (n == 0) return;
    const unsigned nb = (unsigned)std::min<size_t>(blocks_for(n, 256), 4096);
    hipLaunchKernelGGL(k_fill<T>, dim3(nb), dim3(256), 0, st, p, n, v);
}
template void launch_fill<double>(hipStream_t, double*, size_t, double);
template void launch_fill<float>(hipStream_t, float*, size_t, float);
template void launch_fill<int>(hipStream_t, int*, size_t, int);
void launch_cast_f32(hipStream_t st, const double* a, float* b, size_t n) {
    const unsigned nb = (unsigned)std::min<size_t>(blocks_for(n, 256), 4096);
    hipLaunchKernelGGL(k_cast_f32, dim3(nb), dim3(256), 0, st, a, b, n);
}
void launch_grad(hipStream_t st, const double* U, const double* x, Phases ph, Mat<double> mat, int nx, int ny,
                 double* dcdx) {
    hipLaunchKernelGGL(k_grad, dim3(blocks_for((size_t)nx * ny, 256)), dim3(256), 0, st, U, x, ph, mat, nx, ny, dcdx);
}
void launch_dot_partials(hipStream_t st, const double* a, const double* b, size_t n, double* partials, int n_part) {
    hipLaunchKernelGGL(k_dot_partials, dim3(n_part), dim3(WG_THREADS), 0, st, a, b, n, partials);
}
void launch_sums(hipStream_t st, SumJob job, double* out) {
    hipLaunchKernelGGL(k_sums, dim3(1), dim3(WG_THREADS), 0, st, job, out);
}
void launch_sum_to(hipStream_t st, const double* partials, int n, double* out) {
    SumJob j{};
    j.p[0] = partials;
    j.n[0] = n;
    j.count = 1;
    launch_sums(st, j, out);
}

}  // namespace mtomg
