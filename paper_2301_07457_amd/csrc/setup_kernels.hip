// Per-design setup of the preconditioner and post-solve kernels:
//  * element moduli from phase densities (Eq. 5, implicit void phase);
//  * Galerkin coarse operators as six moments per coarse element, computed
//    exactly by a 2x2 -> 1 recursion (FP64 accumulation);
//  * dense coarsest matrix, its blocked Cholesky factor (Algorithm 3) and the
//    explicit inverse K_0^{-1} = L^-T L^-1 used by the coarse solve;
//  * compliance gradient dc/dx = -p x^(p-1) (E_i - E_min) u_e^T K^0 u_e and
//    fixed-order reductions.
#include "device_common.h"
#include "kernels.h"

namespace mtomg {

// x^p; repeated multiplication when p is a small whole number (the usual
// SIMP exponents), pow otherwise.
__device__ __forceinline__ double powp(double x, double p) {
    const int n = (int)p;
    if ((double)n == p && n >= 0 && n <= 8) {
        double r = 1.0;
        for (int k = 0; k < n; ++k) r *= x;
        return r;
    }
    return pow(x, p);
}

// Element moduli (Eq. 5).  Densities outside [0, 1] (code 1) or not finite
// (code 2) are reported in *flag as (seq << 2) | code by an atomic maximum,
// so a later reader can tell this call's report from an older one and a
// non-finite entry outranks an out-of-range one; valid inputs write nothing.
__global__ void k_interp(const double* __restrict__ x, Phases ph, int n_e, double* __restrict__ E64,
                         float* __restrict__ E32, int* __restrict__ flag, int seq) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_e) return;
    double E = ph.E_min;
    int code = 0;
    for (int k = 0; k < ph.m; ++k) {
        const double v = x[(size_t)e * ph.m + k];
        if (!(v >= 0.0 && v <= 1.0)) code = max(code, isfinite(v) ? 1 : 2);
        E += powp(v, ph.penal) * ph.dE[k];
    }
    E64[e] = E;
    if (E32) E32[e] = (float)E;
    if (code && flag) atomicMax(flag, (seq << 2) | code);
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

// Galerkin moments of up to five consecutive coarse levels in one launch.
// Each workgroup owns a T x T tile of the first output level (level of
// src, halved) and coarsens it in LDS down to the last one (tile T >> (n-1)),
// each parent from its four children in the order of k_moments_coarsen.
// src: fine moduli (FROM_E) or the six moment planes of the level above.
template <bool FROM_E>
__global__ __launch_bounds__(256) void k_moments_tree(const double* __restrict__ src, int nxs, int nys, int T,
                                                      int nlev, MomLevels out) {
    __shared__ double buf[2][6][256];
    const int nx0 = nxs / 2, ny0 = nys / 2;
    const int t = threadIdx.x;
    auto put = [&](int lv, int I, int J, const Mom<double>& P) {
        const int nxl = nx0 >> lv, nyl = ny0 >> lv;
        const size_t ps = (size_t)nxl * nyl, e = (size_t)J * nxl + I;
        const double v[6] = {P.m00, P.m10, P.m01, P.m20, P.m11, P.m02};
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            out.m64[lv][k * ps + e] = v[k];
            if (out.m32[lv]) out.m32[lv][k * ps + e] = (float)v[k];
            buf[lv & 1][k][t] = v[k];
        }
    };
    if (t < T * T) {
        const int I = blockIdx.x * T + t % T, J = blockIdx.y * T + t / T;
        Mom<double> P = mom_zero<double>();
        const size_t pf = (size_t)nxs * nys;
        for (int tt = 0; tt < 2; ++tt)
            for (int ss = 0; ss < 2; ++ss) {
                const size_t c = (size_t)(2 * J + tt) * nxs + 2 * I + ss;
                if constexpr (FROM_E) {
                    mom_accumulate_child(P, mom_const<double>(src[c]), ss, tt);
                } else {
                    const Mom<double> ch{src[c], src[pf + c], src[2 * pf + c], src[3 * pf + c], src[4 * pf + c],
                                         src[5 * pf + c]};
                    mom_accumulate_child(P, ch, ss, tt);
                }
            }
        put(0, I, J, P);
    }
    for (int lv = 1; lv < nlev; ++lv) {
        __syncthreads();
        const int Tl = T >> lv, Tp = T >> (lv - 1);
        if (t < Tl * Tl) {
            const int il = t % Tl, jl = t / Tl;
            Mom<double> P = mom_zero<double>();
            for (int tt = 0; tt < 2; ++tt)
                for (int ss = 0; ss < 2; ++ss) {
                    const int c = (2 * jl + tt) * Tp + 2 * il + ss;
                    const double(*b)[256] = buf[(lv - 1) & 1];
                    const Mom<double> ch{b[0][c], b[1][c], b[2][c], b[3][c], b[4][c], b[5][c]};
                    mom_accumulate_child(P, ch, ss, tt);
                }
            put(lv, blockIdx.x * Tl + il, blockIdx.y * Tl + jl, P);
        }
    }
}

// Dense free-DOF matrix of the coarsest grid: thread per (free node, one of
// its 9 neighbours); each computes the 2x2 block as the sum over the shared
// elements of element responses to unit displacements.
template <bool FINE>
__global__ void k_assemble_dense(LevelOp<double> op, Mat<double> mat, double* __restrict__ A, int ld,
                                 int* __restrict__ status) {
    const int nx = op.nx, ny = op.ny;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (status && t == 0) {
        // positive definite so far; factor this design at the next opportunity
        status[0] = 0;
        status[1] = 1;
    }
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
        for (int b = 0; b < 2; ++b) A[(size_t)(rn + a) * ld + cm + b] = blk[a][b];
}

// ---------------------------------------------------------------------------
// Coarsest solve setup: blocked Cholesky (Algorithm 3 carried out on 32 x 32
// blocks) and the explicit inverse K_0^{-1} = W^T W with W = L^{-1}.
// The matrix is padded to a multiple of the block size with an identity
// tail, so every block is full; row-major, leading dimension np.
// ---------------------------------------------------------------------------
constexpr int NB = 32;

// Each of the 256 threads owns one row r and four columns c4..c4+3 of a block.
__device__ __forceinline__ void blk_coords(int& r, int& c4) {
    r = threadIdx.x >> 3;
    c4 = (threadIdx.x & 7) * 4;
}

__device__ __forceinline__ void blk_load(double (*S)[NB + 1], const double* __restrict__ A, int np, int bi, int bj) {
    for (int k = threadIdx.x; k < NB * NB; k += 256) {
        const int r = k / NB, c = k % NB;
        S[r][c] = A[(size_t)(bi * NB + r) * np + bj * NB + c];
    }
}

// ---------------------------------------------------------------------------
// Factor and inverse of one SPD 32x32 block by a single wave, in registers.
// Lanes 0..31 hold the rows r of the block, lanes 32..63 the columns c of
// X (initially I).  Step k of the right-looking factorisation scales column
// k into L and, as the same elementary row operation applied to X, row k of
// X; then every row below eliminates: S[r][c] -= L[r][k] L[c][k] and
// X[r][:] -= L[r][k] X[k][:].  After 32 steps X = L^{-1} (Gauss-Jordan on
// the factor).  With X held by columns, both updates read as
// v[j] -= own * L[j][k] for j > k (own = L[r][k] on a row lane, X[k][c] on
// a column lane), so one instruction stream serves both halves.  Steps go
// in pairs: every lane forms the 2 x 2 corner of steps k, k+1 from three
// broadcast entries, applies both steps to its own columns k and k+1, and
// the two new columns of L travel through LDS together; each element still
// receives the updates of step k and then of step k+1, as a step at a time
// would apply them.  The lanes of one wave access LDS in order, so only the
// compiler is fenced between the write and the reads.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// 1/sqrt(d): hardware estimate, then two Newton steps y <- y (3 - d y^2) / 2
__device__ __forceinline__ double rsqrt_nr(double d) {
    double y = __builtin_amdgcn_rsq(d);
    const double hd = 0.5 * d;
    y = y * fma(-hd, y * y, 1.5);
    y = y * fma(-hd, y * y, 1.5);
    return y;
}

// S: input block (LDS, lower triangle read); Li: receives L^{-1} (full
// block, zero above the diagonal); buf: 64 doubles of LDS, 16-byte
// aligned.  Call from one whole wave.  Returns false (uniformly) if a pivot
// is not positive; Li is then not meaningful.
template <int LD>
__device__ __forceinline__ bool wave_potrf_inv(const double (*S)[LD], double (*Li)[LD], double* buf) {
    static_assert(NB % 2 == 0, "pivots go in pairs");
    const int lane = threadIdx.x & 63;
    const bool xl = lane >= 32;   // column lane of X
    const int q = lane & 31;      // row of S / column of X
    double v[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const double sv = S[q][j];
        v[j] = xl ? (j == q ? 1.0 : 0.0) : sv;
    }
    bool ok = true;
#pragma unroll
    for (int k = 0; k < NB; k += 2) {
        const double d0 = readlane_d(v[k], k);
        const double e = readlane_d(v[k], k + 1);
        const double d1 = readlane_d(v[k + 1], k + 1);
        const double inv0 = rsqrt_nr(d0);
        const double l10 = e * inv0;                  // L[k+1][k]
        const double d1p = fma(-l10, l10, d1);        // A[k+1][k+1] after step k
        ok = ok && (d0 > 0.0) && (d1p > 0.0);
        const double inv1 = rsqrt_nr(d1p);
        // step k on this lane's columns k (scale) and k+1 (eliminate): L[q][k]
        // on a row lane (zero above the diagonal; on lane k, v[k] is d0 itself,
        // so the product is sqrt(d0)), X[k][c] on a column lane
        const double own0 = (xl || q >= k) ? v[k] * inv0 : 0.0;
        v[k] = own0;
        v[k + 1] = fma(-own0, l10, v[k + 1]);
        // step k + 1 on column k+1 (on lane k+1, v[k+1] is now d1p)
        const double own1 = (xl || q >= k + 1) ? v[k + 1] * inv1 : 0.0;
        v[k + 1] = own1;
        if (!xl) *reinterpret_cast<double2*>(&buf[2 * q]) = make_double2(own0, own1);
        wave_fence();
        double2 bk[NB];
#pragma unroll
        for (int j = k + 2; j < NB; ++j) bk[j] = *reinterpret_cast<const double2*>(&buf[2 * j]);
#pragma unroll
        for (int j = k + 2; j < NB; ++j) {
            v[j] = fma(-own0, bk[j].x, v[j]);
            v[j] = fma(-own1, bk[j].y, v[j]);
            // materialise the update in this step (deferring it would keep
            // every step's columns live and spill)
            asm volatile("" : "+v"(v[j]));
        }
        wave_fence();
    }
    if (xl) {
#pragma unroll
        for (int r = 0; r < NB; ++r) Li[r][q] = v[r];
    }
    return ok;
}

// C (LDS) = X Y^T for 32x32 blocks in LDS; thread (r, c4..c4+3).
__device__ __forceinline__ void blk_gemm_nt(double (*C)[NB + 1], double (*X)[NB + 1], double (*Y)[NB + 1]) {
    int r, c4;
    blk_coords(r, c4);
    double acc[4] = {0, 0, 0, 0};
    for (int s = 0; s < NB; ++s) {
        const double xr = X[r][s];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] += xr * Y[c4 + q][s];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) C[r][c4 + q] = acc[q];
}

// One launch of the coarsest factorisation, k = 0 .. nblk (np = 32 nblk):
//  * Cholesky part (k < nblk): workgroup (ib, jb), ib >= jb >= k, forms
//    L[ib,k-1] = A[ib,k-1] Linv_{k-1}^T and L[jb,k-1], applies
//    A[ib,jb] -= L[ib,k-1] L[jb,k-1]^T; workgroups with jb == k store
//    L[ib,k-1]; the one with ib == jb == k then factors the finished
//    diagonal block k: Dinv[k] = L_kk^{-1}, also written as W's diagonal
//    block.  For k = 0 a single workgroup factors block 0.
//  * W = L^{-1} part, step t = k - 2 (0 <= t <= nblk-2): workgroup (i, j),
//    i > t >= j: S[i,j] (+)= L[i,t] W[t,j] (W[t,t] = Dinv[t]); for i == t+1
//    the sum is complete and W[t+1,j] = -Dinv[t+1] S[t+1,j].
//  * K_0^{-1} = W^T W part, block row t = k - 2 of W (complete since the
//    previous launch), 0 <= t <= nblk-1: workgroup (i, j), t >= i >= j:
//    Ainv[i,j] (+)= W[t,i]^T W[t,j], summed over t in increasing order; the
//    last row (t = nblk-1) also writes the mirrored block Ainv[j,i], so the
//    inverse is exactly symmetric.
// Every block a launch reads was written by an earlier launch; launches
// run for k = 0 .. nblk+1.
__global__ __launch_bounds__(256) void k_factor_step(double* __restrict__ A, int np, int k, double* __restrict__ Dinv,
                                                     double* __restrict__ Lbuf, double* __restrict__ W,
                                                     double* __restrict__ Sacc, double* __restrict__ Ainv,
                                                     int* __restrict__ status, long long ds) {
    __shared__ double B0[NB][NB + 1], B1[NB][NB + 1], B2[NB][NB + 1], B4[NB][NB + 1];
    __shared__ __align__(16) double B3[NB][NB + 1];
    // design blockIdx.y; skipped unless flagged for factorisation and still positive definite
    const long long off = (long long)blockIdx.y * ds;
    status = at(status, off);
    if (status[1] == 0 || status[0] != 0) return;
    A = at(A, off);
    Dinv = at(Dinv, off);
    Lbuf = at(Lbuf, off);
    W = at(W, off);
    Sacc = at(Sacc, off);
    Ainv = at(Ainv, off);
    const int nblk = np / NB;
    int r, c4;
    blk_coords(r, c4);
    const int n_chol = (k >= nblk) ? 0 : (k == 0 ? 1 : (nblk - k) * (nblk - k + 1) / 2);
    const int t_inv = k - 2;
    const int n_inv = (t_inv >= 0 && t_inv <= nblk - 2) ? (nblk - 1 - t_inv) * (t_inv + 1) : 0;
    if ((int)blockIdx.x >= n_chol + n_inv) {
        // ---- Ainv = W^T W, block row t of W
        const int t = k - 2;
        int i = 0, j = blockIdx.x - n_chol - n_inv;
        while (j > i) { j -= i + 1; ++i; }
        blk_load(B0, W, np, t, i);
        blk_load(B1, W, np, t, j);
        __syncthreads();
        double* blk = Ainv + (size_t)(i * NB + r) * np + j * NB + c4;
        double acc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = (t == i) ? 0.0 : blk[q];
        for (int s = 0; s < NB; ++s) {
            const double wr = B0[s][r];
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] += wr * B1[s][c4 + q];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) blk[q] = acc[q];
        if (t == nblk - 1 && i != j) {
#pragma unroll
            for (int q = 0; q < 4; ++q) Ainv[(size_t)(j * NB + c4 + q) * np + i * NB + r] = acc[q];
        }
        return;
    }
    if ((int)blockIdx.x >= n_chol) {
        // ---- W = L^{-1}, step t
        const int t = k - 2;
        const int b = blockIdx.x - n_chol;
        const int j = b % (t + 1);
        const int i = t + 1 + b / (t + 1);
        blk_load(B0, Lbuf, np, i, t);
        if (j == t) {
            for (int x = threadIdx.x; x < NB * NB; x += 256) B1[x / NB][x % NB] = Dinv[(size_t)t * NB * NB + x];
        } else {
            blk_load(B1, W, np, t, j);
        }
        __syncthreads();
        double acc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = (j == t) ? 0.0 : Sacc[(size_t)(i * NB + r) * np + j * NB + c4 + q];
        for (int s = 0; s < NB; ++s) {
            const double lr = B0[r][s];
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] += lr * B1[s][c4 + q];
        }
        if (i != t + 1) {
#pragma unroll
            for (int q = 0; q < 4; ++q) Sacc[(size_t)(i * NB + r) * np + j * NB + c4 + q] = acc[q];
            return;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) B2[r][c4 + q] = acc[q];
        for (int x = threadIdx.x; x < NB * NB; x += 256) B3[x / NB][x % NB] = Dinv[(size_t)i * NB * NB + x];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = c4 + q;
            double s = 0.0;
            for (int u = 0; u <= r; ++u) s += B3[r][u] * B2[u][c];
            W[(size_t)(i * NB + r) * np + j * NB + c] = -s;
        }
        return;
    }
    // ---- Cholesky
    __shared__ int not_spd;
    auto finish_diag = [&](int kk) {
        // B0 holds the finished diagonal block kk; wave 0 factors it into B2 = L_kk^{-1}
        __syncthreads();
        if (threadIdx.x < WAVE) {
            const bool ok = wave_potrf_inv<NB + 1>(B0, B2, &B3[0][0]);
            if (threadIdx.x == 0) not_spd = ok ? 0 : 1;
        }
        __syncthreads();
        if (not_spd) {
            if (threadIdx.x == 0) *status = 1;
            return;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double v = B2[r][c4 + q];
            Dinv[(size_t)kk * NB * NB + r * NB + c4 + q] = v;
            W[(size_t)(kk * NB + r) * np + kk * NB + c4 + q] = v;
        }
    };
    if (k == 0) {
        blk_load(B0, A, np, 0, 0);
        finish_diag(0);
        return;
    }
    int a = 0, rem = blockIdx.x;
    while (rem > a) { rem -= a + 1; ++a; }
    const int ib = k + a, jb = k + rem;
    blk_load(B0, A, np, ib, k - 1);
    if (jb != ib) blk_load(B1, A, np, jb, k - 1);
    for (int x = threadIdx.x; x < NB * NB; x += 256) B2[x / NB][x % NB] = Dinv[(size_t)(k - 1) * NB * NB + x];
    __syncthreads();
    blk_gemm_nt(B3, B0, B2);
    if (jb != ib) blk_gemm_nt(B4, B1, B2);
    __syncthreads();
    double (*Lj)[NB + 1] = (jb != ib) ? B4 : B3;
    if (jb == k) {
#pragma unroll
        for (int q = 0; q < 4; ++q) Lbuf[(size_t)(ib * NB + r) * np + (k - 1) * NB + c4 + q] = B3[r][c4 + q];
    }
    double upd[4] = {0, 0, 0, 0};
    for (int s = 0; s < NB; ++s) {
        const double lr = B3[r][s];
#pragma unroll
        for (int q = 0; q < 4; ++q) upd[q] += lr * Lj[c4 + q][s];
    }
    double* blk = A + (size_t)(ib * NB + r) * np + jb * NB + c4;
    double nv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        nv[q] = blk[q] - upd[q];
        blk[q] = nv[q];
    }
    if (ib == k && jb == k) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) B0[r][c4 + q] = nv[q];
        finish_diag(k);
    }
}

// ---------------------------------------------------------------------------
// Banded form of the same factorisation.  The coarsest matrix couples DOFs
// at most 2 nx0 + 5 apart (neighbouring nodes, two DOFs each, rows of
// nx0 + 1 nodes), so with 32 x 32 blocks only the NBW = ceil(bw / 32)
// blocks below the diagonal are nonzero, and Cholesky creates no fill
// outside that band.  Every operation of the dense launch sequence that
// involves a block outside the band adds exact zeros; the kernels below
// skip those, so they compute the same L^{-1} blocks, W and K_0^{-1} (up to
// the rounding order of the matrix-core products).
// ---------------------------------------------------------------------------

// Blocks of the banded kernels sit in LDS with a row stride of BL doubles.
// Their 32 x 32 x 32 block products run on the FP64 matrix cores
// (v_mfma_f64_16x16x4: A[i][k] from lane i + 16 k, B[k][j] from lane
// j + 16 k, result element (4 v + lane / 16, lane % 16) in register v);
// wave w of a 256-thread workgroup owns the 16 x 16 quadrant
// (w >> 1, w & 1) of every block product.
constexpr int BL = NB + 2;
typedef double dbl4 __attribute__((ext_vector_type(4)));

struct Quad {
    int i0, j0, li, lk;
};
__device__ __forceinline__ Quad quad_of_wave() {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    return Quad{16 * (w >> 1), 16 * (w & 1), l & 15, l >> 4};
}

// acc += X[i0.., :] Y[j0.., :]^T  (sum over s of X[i][s] Y[j][s])
__device__ __forceinline__ dbl4 mfma_nt(const double (*X)[BL], const double (*Y)[BL], const Quad& q, dbl4 acc) {
#pragma unroll
    for (int kk = 0; kk < NB; kk += 4) {
        const double a = X[q.i0 + q.li][kk + q.lk];
        const double b = Y[q.j0 + q.li][kk + q.lk];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    return acc;
}
// acc += X[i0.., :] Y[:, j0..]  (sum over s of X[i][s] Y[s][j])
__device__ __forceinline__ dbl4 mfma_nn(const double (*X)[BL], const double (*Y)[BL], const Quad& q, dbl4 acc) {
#pragma unroll
    for (int kk = 0; kk < NB; kk += 4) {
        const double a = X[q.i0 + q.li][kk + q.lk];
        const double b = Y[kk + q.lk][q.j0 + q.li];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    return acc;
}
// acc += X[:, i0..]^T Y[:, j0..]  (sum over s of X[s][i] Y[s][j])
__device__ __forceinline__ dbl4 mfma_tn(const double (*X)[BL], const double (*Y)[BL], const Quad& q, dbl4 acc) {
#pragma unroll
    for (int kk = 0; kk < NB; kk += 4) {
        const double a = X[kk + q.lk][q.i0 + q.li];
        const double b = Y[kk + q.lk][q.j0 + q.li];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    return acc;
}
// the quadrant's elements: (i0 + 4 v + lk, j0 + li), v = 0..3
__device__ __forceinline__ void quad_store(double (*C)[BL], const Quad& q, dbl4 d) {
#pragma unroll
    for (int v = 0; v < 4; ++v) C[q.i0 + 4 * v + q.lk][q.j0 + q.li] = d[v];
}
__device__ __forceinline__ void quad_store_g(double* __restrict__ G, size_t ld, const Quad& q, dbl4 d) {
#pragma unroll
    for (int v = 0; v < 4; ++v) G[(size_t)(q.i0 + 4 * v + q.lk) * ld + q.j0 + q.li] = d[v];
}
__device__ __forceinline__ dbl4 quad_load(const double (*C)[BL], const Quad& q) {
    dbl4 d;
#pragma unroll
    for (int v = 0; v < 4; ++v) d[v] = C[q.i0 + 4 * v + q.lk][q.j0 + q.li];
    return d;
}

__device__ __forceinline__ void ld4(double* v, const double* __restrict__ p) {
    const double2 a = *reinterpret_cast<const double2*>(p);
    const double2 b = *reinterpret_cast<const double2*>(p + 2);
    v[0] = a.x;
    v[1] = a.y;
    v[2] = b.x;
    v[3] = b.y;
}
__device__ __forceinline__ void st4(double* p, const double* v) {
    *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
    *reinterpret_cast<double2*>(p + 2) = make_double2(v[2], v[3]);
}

// Cholesky of the band by one workgroup per design.  Block step k factors
// the diagonal block (Dinv_k = L_kk^{-1}, also W's diagonal block), forms
// the panel L[k+d][k] = A[k+d][k] Dinv_k^T (d = 1..NBW; stored to Lbuf) and
// applies A[i][j] -= L[i][k] L[j][k]^T, k < j <= i <= k + NBW.  Only the
// chain Dinv_k -> L[k+1][k] -> A[k+1][k+1] -> Dinv_{k+1} is serial; the
// rest of step k (with NBW = 2: L[k+2][k] and the updates of A[k+2][k+1],
// A[k+2][k+2]) runs on waves 1..3 during step k+1, while wave 0 factors
// the next diagonal block.  Per step:
//   A  wave 0: factor A[k][k]; waves 1..3: fetch block row k+2 from A and
//      finish step k-1 (each forms L[k+1][k-1] whole in its own scratch
//      block, then a share of the two updates of block row k+1);
//   B  all waves: L[k+1][k] (one 16 x 16 quadrant each);
//   C  all waves: A[k+1][k+1] -= L[k+1][k] L[k+1][k]^T.
// Block rows k..k+2 live in LDS (block (i, i-d) in slot [i % 3][d]);
// Dinv_k and L[k+1][k] alternate between two buffers by the parity of k.
template <int NBW>
__global__ __launch_bounds__(256) void k_band_chol(const double* __restrict__ A, int np, double* __restrict__ Dinv,
                                                   double* __restrict__ Lbuf, double* __restrict__ W,
                                                   int* __restrict__ status, long long ds) {
    static_assert(NBW == 1 || NBW == 2, "band of one or two blocks");
    constexpr int NR = 3;
    __shared__ __align__(16) double win[NR][NBW + 1][NB][BL];
    __shared__ __align__(16) double Dk[2][NB][BL];
    __shared__ __align__(16) double Lc[2][NB][BL];
    __shared__ __align__(16) double scr[NBW == 2 ? 3 : 1][NB][BL];
    __shared__ __align__(16) double gbuf[2 * NB];
    __shared__ int not_spd;
    const long long off = (long long)blockIdx.y * ds;
    status = at(status, off);
    if (status[1] == 0 || status[0] != 0) return;
    A = at(A, off);
    Dinv = at(Dinv, off);
    Lbuf = at(Lbuf, off);
    W = at(W, off);
    const int nblk = np / NB;
    int r, c4;
    blk_coords(r, c4);
    const Quad qd = quad_of_wave();
    const int wave = threadIdx.x >> 6;
    auto gblk = [&](int bi, int bj) { return (size_t)(bi * NB + r) * np + bj * NB + c4; };
    auto gbase = [&](int bi, int bj) { return (size_t)(bi * NB) * np + bj * NB; };
    for (int i = 0; i <= 1 && i < nblk; ++i)
        for (int d = 0; d <= NBW && d <= i; ++d) ld4(&win[i % NR][d][r][c4], A + gblk(i, i - d));
    for (int k = 0; k < nblk; ++k) {
        __syncthreads();
        // ---- A
        if (wave == 0) {
            const bool ok = wave_potrf_inv<BL>(win[k % NR][0], Dk[k & 1], gbuf);
            if (threadIdx.x == 0) not_spd = ok ? 0 : 1;
        } else {
            const int rn = k + 2;   // its slot held block row k - 1, finished
            if (rn < nblk) {
                constexpr int TOT = (NBW + 1) * NB * NB / 2;   // double2 elements
                constexpr int NT = 256 - WAVE;
                constexpr int PER = (TOT + NT - 1) / NT;
                const int t0 = threadIdx.x - WAVE;
                double2 v[PER];
#pragma unroll
                for (int u = 0; u < PER; ++u) {
                    const int e = min(t0 + u * NT, TOT - 1);
                    const int d = e / (NB * NB / 2), rem = e % (NB * NB / 2);
                    v[u] = *reinterpret_cast<const double2*>(A + (size_t)(rn * NB + rem / (NB / 2)) * np +
                                                             (rn - d) * NB + (rem % (NB / 2)) * 2);
                }
#pragma unroll
                for (int u = 0; u < PER; ++u) {
                    const int e = t0 + u * NT;
                    if (e < TOT) {
                        const int d = e / (NB * NB / 2), rem = e % (NB * NB / 2);
                        *reinterpret_cast<double2*>(&win[rn % NR][d][rem / (NB / 2)][(rem % (NB / 2)) * 2]) = v[u];
                    }
                }
            }
            if constexpr (NBW == 2) {
                if (k >= 1 && k + 1 < nblk) {
                    // rest of step k-1: L[k+1][k-1] = A[k+1][k-1] Dinv_{k-1}^T (whole block per wave)
                    double(*Lx)[BL] = scr[wave - 1];
                    const double(*Ain)[BL] = win[(k + 1) % NR][2];
                    const double(*Dp)[BL] = Dk[(k - 1) & 1];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const Quad qq{16 * (q >> 1), 16 * (q & 1), qd.li, qd.lk};
                        const dbl4 lx = mfma_nt(Ain, Dp, qq, dbl4{0, 0, 0, 0});
                        quad_store(Lx, qq, lx);
                        if (wave == 1) quad_store_g(Lbuf + gbase(k + 1, k - 1), np, qq, lx);
                    }
                    wave_fence();
                    // A[k+1][k] -= L[k+1][k-1] L[k][k-1]^T, A[k+1][k+1] -= L[k+1][k-1] L[k+1][k-1]^T:
                    // eight quadrant products shared 3 / 3 / 2 by waves 1..3
#pragma unroll
                    for (int u = 0; u < 3; ++u) {
                        const int job = (wave - 1) * 3 + u;
                        if (job < 8) {
                            const int q = job & 3;
                            const Quad qq{16 * (q >> 1), 16 * (q & 1), qd.li, qd.lk};
                            const bool diag = job >= 4;
                            const double(*Lj)[BL] = diag ? Lx : Lc[(k - 1) & 1];
                            double(*T)[BL] = win[(k + 1) % NR][diag ? 0 : 1];
                            const dbl4 upd = mfma_nt(Lx, Lj, qq, dbl4{0, 0, 0, 0});
                            quad_store(T, qq, quad_load(T, qq) - upd);
                        }
                    }
                }
            }
        }
        __syncthreads();
        if (not_spd) {
            if (threadIdx.x == 0) *status = 1;
            return;
        }
        // ---- B
        st4(Dinv + (size_t)k * NB * NB + r * NB + c4, &Dk[k & 1][r][c4]);
        st4(W + gblk(k, k), &Dk[k & 1][r][c4]);
        if (k + 1 >= nblk) break;
        {
            const dbl4 l1 = mfma_nt(win[(k + 1) % NR][1], Dk[k & 1], qd, dbl4{0, 0, 0, 0});
            quad_store(Lc[k & 1], qd, l1);
            quad_store_g(Lbuf + gbase(k + 1, k), np, qd, l1);
        }
        __syncthreads();
        // ---- C
        {
            double(*T)[BL] = win[(k + 1) % NR][0];
            const dbl4 upd = mfma_nt(Lc[k & 1], Lc[k & 1], qd, dbl4{0, 0, 0, 0});
            quad_store(T, qd, quad_load(T, qd) - upd);
        }
    }
}

// W = L^{-1}, block column j per workgroup: W[j][j] = Dinv_j and, for
// i > j, W[i][j] = -Dinv_i S with S = sum over t = max(j, i-NBW) .. i-1 of
// L[i][t] W[t][j].  The L blocks and Dinv_i of the next block row are
// fetched while the current one is formed.
template <int NBW>
__global__ __launch_bounds__(256) void k_band_winv(const double* __restrict__ Dinv, const double* __restrict__ Lbuf,
                                                   double* __restrict__ W, int np, const int* __restrict__ status,
                                                   long long ds) {
    constexpr int NQ = NBW + 1;
    __shared__ __align__(16) double Wq[NQ][NB][BL];   // W[t][j] at slot t % NQ
    __shared__ __align__(16) double Lq[NBW][NB][BL];  // L[i][i-d] at slot d-1
    __shared__ __align__(16) double Dq[NB][BL];       // Dinv_i
    __shared__ __align__(16) double Sq[NB][BL];
    const long long off = (long long)blockIdx.y * ds;
    status = at(status, off);
    if (status[1] == 0 || status[0] != 0) return;
    Dinv = at(Dinv, off);
    Lbuf = at(Lbuf, off);
    W = at(W, off);
    const int nblk = np / NB;
    const int j = blockIdx.x;
    int r, c4;
    blk_coords(r, c4);
    const Quad qd = quad_of_wave();
    auto gblk = [&](int bi, int bj) { return (size_t)(bi * NB + r) * np + bj * NB + c4; };
    double pl[NBW][4], pd[4];
    auto fetch = [&](int i) {
#pragma unroll
        for (int d = 1; d <= NBW; ++d)
            if (d <= i - j) ld4(pl[d - 1], Lbuf + gblk(i, i - d));
        ld4(pd, Dinv + (size_t)i * NB * NB + r * NB + c4);
    };
    {
        double w0[4];
        ld4(w0, Dinv + (size_t)j * NB * NB + r * NB + c4);
        st4(&Wq[j % NQ][r][c4], w0);
    }
    if (j + 1 < nblk) fetch(j + 1);
    for (int i = j + 1; i < nblk; ++i) {
        const int dmax = min(NBW, i - j);
#pragma unroll
        for (int d = 1; d <= NBW; ++d)
            if (d <= dmax) st4(&Lq[d - 1][r][c4], pl[d - 1]);
        st4(&Dq[r][c4], pd);
        if (i + 1 < nblk) fetch(i + 1);
        __syncthreads();
        dbl4 acc = {0, 0, 0, 0};
#pragma unroll
        for (int d = NBW; d >= 1; --d)
            if (d <= dmax) acc = mfma_nn(Lq[d - 1], Wq[(i - d) % NQ], qd, acc);
        quad_store(Sq, qd, acc);
        __syncthreads();
        const dbl4 w = -mfma_nn(Dq, Sq, qd, dbl4{0, 0, 0, 0});
        quad_store(Wq[i % NQ], qd, w);
        quad_store_g(W + (size_t)(i * NB) * np + j * NB, np, qd, w);
        __syncthreads();
    }
}

// K_0^{-1} = W^T W: workgroup (i, j), i >= j, sums W[t][i]^T W[t][j] over
// t = i .. nblk-1 and writes block (i, j) and its mirror (j, i).  The blocks
// of the next t are fetched during the product.
__global__ __launch_bounds__(256) void k_band_gram(const double* __restrict__ W, double* __restrict__ Ainv, int np,
                                                   const int* __restrict__ status, long long ds) {
    __shared__ __align__(16) double B[2][2][NB][BL];
    const long long off = (long long)blockIdx.y * ds;
    status = at(status, off);
    if (status[1] == 0 || status[0] != 0) return;
    W = at(W, off);
    Ainv = at(Ainv, off);
    const int nblk = np / NB;
    int i = 0, j = blockIdx.x;
    while (j > i) { j -= i + 1; ++i; }
    int r, c4;
    blk_coords(r, c4);
    const Quad qd = quad_of_wave();
    auto gblk = [&](int bi, int bj) { return (size_t)(bi * NB + r) * np + bj * NB + c4; };
    double pa[4], pb[4];
    ld4(pa, W + gblk(i, i));
    ld4(pb, W + gblk(i, j));
    dbl4 acc = {0, 0, 0, 0};
    for (int t = i; t < nblk; ++t) {
        const int cur = (t - i) & 1;
        st4(&B[cur][0][r][c4], pa);
        st4(&B[cur][1][r][c4], pb);
        if (t + 1 < nblk) {
            ld4(pa, W + gblk(t + 1, i));
            ld4(pb, W + gblk(t + 1, j));
        }
        __syncthreads();
        acc = mfma_tn(B[cur][0], B[cur][1], qd, acc);
    }
    quad_store_g(Ainv + (size_t)(i * NB) * np + j * NB, np, qd, acc);
    if (i != j) {
        // mirror: element (a, b) of block (i, j) goes to (b, a) of block (j, i)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            Ainv[(size_t)(j * NB + qd.j0 + qd.li) * np + i * NB + qd.i0 + 4 * v + qd.lk] = acc[v];
    }
}

__global__ void k_pad_identity(double* __restrict__ A, int n0, int np, const int* __restrict__ status,
                               long long ds) {
    const long long off = (long long)blockIdx.y * ds;
    if (at(status, off)[1] == 0) return;
    A = at(A, off);
    const int k = n0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (k < np) A[(size_t)k * np + k] = 1.0;
}

template <typename T>
__global__ void k_fill(T* __restrict__ p, size_t n, T v) {
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) p[k] = v;
}

__global__ void k_cast_f32(const double* __restrict__ a, float* __restrict__ b, size_t n) {
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
        b[k] = (float)a[k];
}

// dc/dx_{e,i} = -p x^(p-1) (E_i - E_min) u_e^T K^0 u_e.
// A wave owns 63 element columns (64 node columns, lane l at node column
// i0 + l) and GRAD_ROWS element rows.  It issues every load first: its
// GRAD_ROWS + 1 node rows of U and the densities of its element rows (the
// M phases of a row's 63 elements are contiguous in x, so lane l takes
// entries l, l + 64, ... of the row: M per lane).  Then it marches up:
// element (i, j) takes nodes (i, j) and (i, j+1) from its own lane and
// (i+1, .) from the next lane (DPP).  The densities and the outputs of a
// row go through LDS, so both are read and written as whole coalesced
// rows.  Consecutive tiles share an XCD (xcd_tile), so the one halo row
// between row chunks hits L2.  Two rows per wave: at 1024^2 with three
// phases the launch took 12.7 us, against 13.9 with four rows and 16.8
// with eight, whose fewer workgroups hide less latency.
constexpr int GRAD_COLS = 63, GRAD_ROWS = 2;
template <int M>
__global__ __launch_bounds__(WG_THREADS) void k_grad(const double* __restrict__ U, const double* __restrict__ x,
                                                    Phases ph, Mat<double> mat, int nx, int ny, int n_strips,
                                                    int n_tiles, double* __restrict__ dcdx) {
    constexpr int ROWS = GRAD_ROWS;
    // 64 M per wave: every lane writes its M slots of a row, also past the
    // strip's n_e M entries (values nobody stores), so no write is under a
    // branch that the compiler could sink a load into
    __shared__ double stage[WAVES_PER_WG][WAVE * M];
    const int tile = xcd_tile(n_tiles);
    if (tile >= n_tiles) return;
    const int lane = lane_id(), w = wave_id();
    const int strip = tile % n_strips;
    const int j0 = ((tile / n_strips) * WAVES_PER_WG + w) * ROWS;
    if (j0 >= ny) return;                            // a wave past the grid, before any load
    const int i0 = strip * GRAD_COLS, i = i0 + lane;
    const int ne = min(GRAD_COLS, nx - i0);          // elements of this strip
    const int nm = ne * M;
    double* buf = stage[w];
    V2<double> un[ROWS + 1];
#pragma unroll
    for (int s = 0; s <= ROWS; ++s) un[s] = load_node(U, nx, ny, i, j0 + s);
    // densities of rows j0 .. j0+ROWS-1 (rows past the grid read the last
    // row; nothing of them is stored), slot q of a row = its entry lane + 64 q
    double xr[ROWS][M];
#pragma unroll
    for (int s = 0; s < ROWS; ++s) {
        const size_t base = ((size_t)min(j0 + s, ny - 1) * nx + i0) * M;
#pragma unroll
        for (int q = 0; q < M; ++q) xr[s][q] = x[base + min(lane + q * WAVE, nm - 1)];
    }
    V2<double> right_lo = from_right(un[0]);
#pragma unroll
    for (int s = 0; s < ROWS; ++s) {
        const int j = j0 + s;
        const V2<double> right_hi = from_right(un[s + 1]);
        V2<double> f0, f1, f2, f3;
        elem_force(mom_const<double>(1.0), mat, un[s], right_lo, right_hi, un[s + 1], f0, f1, f2, f3);
        const double we = (un[s].x * f0.x + un[s].y * f0.y) + (right_lo.x * f1.x + right_lo.y * f1.y) +
                          (right_hi.x * f2.x + right_hi.y * f2.y) + (un[s + 1].x * f3.x + un[s + 1].y * f3.y);
        right_lo = right_hi;
        // the row's densities into LDS; each lane takes its element's
#pragma unroll
        for (int q = 0; q < M; ++q) buf[lane + q * WAVE] = xr[s][q];
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const double xv = buf[lane * M + k];
            buf[lane * M + k] = -ph.penal * powp(xv, ph.penal - 1.0) * ph.dE[k] * we;
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        if (j < ny) {                                  // uniform over the wave
            const size_t base = ((size_t)j * nx + i0) * M;
#pragma unroll
            for (int q = 0; q < M; ++q) {
                const int k = lane + q * WAVE;
                if (k < nm) dcdx[base + k] = buf[k];
            }
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    }
}

// partials[b] = sum over block b's contiguous slice of a . b (fixed order)
__global__ __launch_bounds__(WG_THREADS) void k_dot_partials(const double* __restrict__ a, const double* __restrict__ b,
                                                             size_t n, double* __restrict__ partials) {
    const size_t per = (n + gridDim.x - 1) / gridDim.x;
    const size_t s0 = blockIdx.x * per, s1 = min(n, s0 + per);
    // thread t adds a[k] b[k] for k = s0 + t, s0 + t + 256, ... in order;
    // the loads of U consecutive terms are issued before any is added
    constexpr int U = 8;
    double s = 0.0;
    if (s1 > s0) {
        for (size_t base = s0; base < s1; base += (size_t)U * WG_THREADS) {
            double va[U], vb[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const size_t k = min(base + threadIdx.x + (size_t)u * WG_THREADS, s1 - 1);
                va[u] = a[k];
                vb[u] = b[k];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const size_t k = base + threadIdx.x + (size_t)u * WG_THREADS;
                s = (k < s1) ? s + va[u] * vb[u] : s;
            }
        }
    }
    s = block_sum(s);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void k_fill_strided(int* __restrict__ p, long long stride, int n, int v) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) *at(p, (long long)k * stride) = v;
}

// solve statistics of system blockIdx.y (see launch_solve_sums)
__global__ __launch_bounds__(WG_THREADS) void k_solve_sums(const double* __restrict__ ff, int n_ff,
                                                           const double* __restrict__ rr0,
                                                           const double* __restrict__ rr1, int n_rr0, int n_rr,
                                                           const double* __restrict__ trr,
                                                           int* __restrict__ state, double* __restrict__ out,
                                                           Batch bt) {
    const SysOff so = sys_off(bt);
    state = at(state, so.c);
    const int st0 = state[0];
    const int iters = state[1];
    const double* rr = at(iters & 1 ? rr1 : rr0, so.c);
    const double* ps[3] = {at(ff, so.c), rr, at(trr, so.c)};
    const int ns[3] = {n_ff, iters == 0 ? n_rr0 : n_rr, n_ff};
    double sv[3];
    sum_partials_k<3>(ps, ns, sv);
    const double a = sv[0], b = sv[1], c = sv[2];
    if (threadIdx.x == 0) {
        double* o = at(out, so.c);
        o[0] = a;
        o[1] = b;
        o[2] = c;
        // converged with its last x update applied (mode 4 or 3 ran before): done
        if (st0 == 1) state[0] = 2;
    }
}

__global__ __launch_bounds__(WG_THREADS) void k_sums(SumJob job, double* __restrict__ out) {
    for (int k = 0; k < job.count; ++k) {
        const double s = sum_partials(job.p[k], job.n[k]);
        if (threadIdx.x == 0) out[k] = s;
    }
}

// ---------------------------------------------------------------------------
static inline unsigned blocks_for(size_t n, unsigned bs) { return (unsigned)((n + bs - 1) / bs); }

void launch_interp(hipStream_t st, const double* x, Phases ph, int n_e, double* E64, float* E32, int* flag,
                   int seq) {
    hipLaunchKernelGGL(k_interp, dim3(blocks_for(n_e, 256)), dim3(256), 0, st, x, ph, n_e, E64, E32, flag, seq);
}
void launch_moments_from_fine(hipStream_t st, const double* E64, int nxf, int nyf, double* m64, float* m32) {
    const int n = (nxf / 2) * (nyf / 2);
    hipLaunchKernelGGL(k_moments_from_fine, dim3(blocks_for(n, 256)), dim3(256), 0, st, E64, nxf, nyf, m64, m32);
}
void launch_moments_coarsen(hipStream_t st, const double* mf, int nxf, int nyf, double* m64, float* m32) {
    const int n = (nxf / 2) * (nyf / 2);
    hipLaunchKernelGGL(k_moments_coarsen, dim3(blocks_for(n, 256)), dim3(256), 0, st, mf, nxf, nyf, m64, m32);
}
void launch_assemble_dense(hipStream_t st, bool fine, LevelOp<double> op, Mat<double> mat, double* A, int ld,
                           int* status) {
    const int n = 9 * (op.nx + 1) * op.ny;
    if (fine)
        hipLaunchKernelGGL(k_assemble_dense<true>, dim3(blocks_for(n, 256)), dim3(256), 0, st, op, mat, A, ld, status);
    else
        hipLaunchKernelGGL(k_assemble_dense<false>, dim3(blocks_for(n, 256)), dim3(256), 0, st, op, mat, A, ld,
                           status);
}
void launch_moments_tree(hipStream_t st, bool from_e, const double* src, int nxs, int nys, int T, int nlev,
                         const MomLevels& out) {
    const dim3 grid((nxs / 2) / T, (nys / 2) / T);
    if (from_e) hipLaunchKernelGGL(k_moments_tree<true>, grid, dim3(256), 0, st, src, nxs, nys, T, nlev, out);
    else hipLaunchKernelGGL(k_moments_tree<false>, grid, dim3(256), 0, st, src, nxs, nys, T, nlev, out);
}
void launch_coarse_factor(hipStream_t st, double* A, int n0, int np, double* Dinv, double* W, double* Ainv,
                          int* status, double* Lbuf, double* Sacc, int n_designs, long long ds, int half_bw) {
    if (np > n0)
        hipLaunchKernelGGL(k_pad_identity, dim3(blocks_for(np - n0, 256), n_designs), dim3(256), 0, st, A, n0, np,
                           status, ds);
    const int nblk = np / NB;
    const int nbw = half_bw > 0 ? (half_bw + NB - 1) / NB : nblk;
    if (nbw <= 2) {
        if (nbw <= 1) {
            hipLaunchKernelGGL(k_band_chol<1>, dim3(1, n_designs), dim3(256), 0, st, A, np, Dinv, Lbuf, W, status, ds);
            hipLaunchKernelGGL(k_band_winv<1>, dim3(nblk, n_designs), dim3(256), 0, st, Dinv, Lbuf, W, np, status, ds);
        } else {
            hipLaunchKernelGGL(k_band_chol<2>, dim3(1, n_designs), dim3(256), 0, st, A, np, Dinv, Lbuf, W, status, ds);
            hipLaunchKernelGGL(k_band_winv<2>, dim3(nblk, n_designs), dim3(256), 0, st, Dinv, Lbuf, W, np, status, ds);
        }
        hipLaunchKernelGGL(k_band_gram, dim3(nblk * (nblk + 1) / 2, n_designs), dim3(256), 0, st, W, Ainv, np, status,
                           ds);
        return;
    }
    for (int k = 0; k <= nblk + 1; ++k) {
        const int m = nblk - k;
        const int n_chol = (k >= nblk) ? 0 : (k == 0 ? 1 : m * (m + 1) / 2);
        const int t = k - 2;
        const int n_inv = (t >= 0 && t <= nblk - 2) ? (nblk - 1 - t) * (t + 1) : 0;
        const int n_gram = (t >= 0 && t <= nblk - 1) ? (t + 1) * (t + 2) / 2 : 0;
        if (n_chol + n_inv + n_gram == 0) continue;
        hipLaunchKernelGGL(k_factor_step, dim3(n_chol + n_inv + n_gram, n_designs), dim3(256), 0, st, A, np, k,
                           Dinv, Lbuf, W, Sacc, Ainv, status, ds);
    }
}

void launch_fill_strided(hipStream_t st, int* p, long long stride_bytes, int n, int v) {
    if (n > 0)
        hipLaunchKernelGGL(k_fill_strided, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, stride_bytes, n, v);
}

void launch_solve_sums(hipStream_t st, const double* ff, int n_ff, const double* rr0, const double* rr1,
                       int n_rr0, int n_rr, const double* trr, int* state, double* out, const Batch& bt) {
    hipLaunchKernelGGL(k_solve_sums, dim3(1, bt.n), dim3(WG_THREADS), 0, st, ff, n_ff, rr0, rr1, n_rr0, n_rr, trr,
                       state, out, bt);
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
template <int M>
void launch_grad_m(hipStream_t st, const double* U, const double* x, const Phases& ph, const Mat<double>& mat,
                   int nx, int ny, double* dcdx) {
    constexpr int ROWS = GRAD_ROWS;
    const int n_strips = (nx + GRAD_COLS - 1) / GRAD_COLS;
    const int chunks = (ny + ROWS - 1) / ROWS;
    const int n_tiles = n_strips * ((chunks + WAVES_PER_WG - 1) / WAVES_PER_WG);
    const int grid = (n_tiles + 7) / 8 * 8;   // whole rounds over the 8 XCDs (xcd_tile)
    hipLaunchKernelGGL(k_grad<M>, dim3(grid), dim3(WG_THREADS), 0, st, U, x, ph, mat, nx, ny, n_strips, n_tiles,
                       dcdx);
}
// ph.m is 1 .. 8 (checked by set_grid)
void launch_grad(hipStream_t st, const double* U, const double* x, Phases ph, Mat<double> mat, int nx, int ny,
                 double* dcdx) {
    switch (ph.m) {
        case 1: launch_grad_m<1>(st, U, x, ph, mat, nx, ny, dcdx); break;
        case 2: launch_grad_m<2>(st, U, x, ph, mat, nx, ny, dcdx); break;
        case 3: launch_grad_m<3>(st, U, x, ph, mat, nx, ny, dcdx); break;
        case 4: launch_grad_m<4>(st, U, x, ph, mat, nx, ny, dcdx); break;
        case 5: launch_grad_m<5>(st, U, x, ph, mat, nx, ny, dcdx); break;
        case 6: launch_grad_m<6>(st, U, x, ph, mat, nx, ny, dcdx); break;
        case 7: launch_grad_m<7>(st, U, x, ph, mat, nx, ny, dcdx); break;
        default: launch_grad_m<8>(st, U, x, ph, mat, nx, ny, dcdx); break;
    }
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
