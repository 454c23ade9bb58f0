// Internal launcher interface between the host library and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "device_common.h"

namespace mtomg {

// Launch geometry of a marching sweep: tiles are (strip, block of
// WAVES_PER_WG row chunks); `rows` node rows (coarse rows for restriction)
// per wave.
struct Sweep {
    int n_strips, n_tiles, rows;
};

// Finest-grid right-hand side of the pre-smoother inside PCG.
struct CgRhs {
    const double* r_old;
    const double* q;
    double* r_new;
    float* r32;
    const double* zr;
    int n_zr;
    const double* pq;
    int n_pq;
    double* rr_out;
    int update;
    int* conv_rw;
    int* iters;
};

// Convergence test ||r||^2 <= tol2 ||f||^2 from partial sums.
struct ConvCheck {
    const double* rr;
    int n_rr;
    const double* ff;
    int n_ff;
    double tol2;
    int* conv_rw;
};

template <typename TZ>
void launch_cg_apply(hipStream_t st, LevelOp<double> op, Mat<double> mat, Sweep sw, const TZ* z,
                     const double* p_old, double* p_new, double* x, double* q, const double* zr_cur,
                     const double* zr_prev, int n_zr, const double* pq_prev, int n_pq,
                     double* pq_out, const int* conv, int mode);
void launch_residual(hipStream_t st, LevelOp<double> op, Mat<double> mat, Sweep sw, const double* f,
                     double* x, int use_x, double* r, double* rr_out, double* ff_out);
template <typename T>
void launch_presmooth(hipStream_t st, bool fine, bool cgmode, LevelOp<T> op, Mat<T> mat, Sweep sw,
                      const T* b, T* u_out, int sweeps, const CgRhs& cg, const int* conv);
template <typename T>
void launch_restrict(hipStream_t st, bool fine, bool check, LevelOp<T> op, Mat<T> mat, Sweep sw,
                     const T* b, const T* u, T* rc, const ConvCheck& chk, const int* conv);
template <typename T>
void launch_post(hipStream_t st, bool fine, bool prolong, bool dot, LevelOp<T> op, Mat<T> mat, Sweep sw,
                 const T* u_in, const T* ec, const T* b, T* u_out, const double* r64, double* zr_out,
                 const int* conv);
template <typename T>
void launch_apply(hipStream_t st, bool fine, bool diag, LevelOp<T> op, Mat<T> mat, Sweep sw, const T* u,
                  T* q);
template <typename T>
void launch_coarse_solve(hipStream_t st, const double* Ainv, int n0, int ld, int nx0, const T* b, T* e,
                         const int* conv);

// setup
struct Phases {
    double dE[8];   // E_i - E_min
    int m;
    double E_min, penal;
};
void launch_interp(hipStream_t st, const double* x, Phases ph, int n_e, double* E64, float* E32);
void launch_moments_from_fine(hipStream_t st, const double* E64, int nxf, int nyf, double* mom64,
                              float* mom32);
void launch_moments_coarsen(hipStream_t st, const double* momf, int nxf, int nyf, double* mom64,
                            float* mom32);
constexpr int COARSE_NB = 32;   // block size of the coarse factorisation
void launch_assemble_dense(hipStream_t st, bool fine, LevelOp<double> op, Mat<double> mat, double* A, int ld);
// A (np x np, n0 used, identity padding written here; overwritten) ->
// Dinv = inverses of the diagonal blocks of L, W = L^{-1}, Ainv = A^{-1}.
void launch_coarse_factor(hipStream_t st, double* A, int n0, int np, double* Dinv, double* W, double* Ainv,
                          int* status, double* Lbuf /* np x np */, double* Sacc /* np x np */);
template <typename T>
void launch_fill(hipStream_t st, T* p, size_t n, T v);
void launch_cast_f32(hipStream_t st, const double* a, float* b, size_t n);

// after the solve
void launch_grad(hipStream_t st, const double* U, const double* x, Phases ph, Mat<double> mat, int nx,
                 int ny, double* dcdx);
void launch_dot_partials(hipStream_t st, const double* a, const double* b, size_t n, double* partials,
                         int n_part);
void launch_sum_to(hipStream_t st, const double* partials, int n, double* out);
// out[0..] = sums of several partial arrays (one block)
struct SumJob {
    const double* p[4];
    int n[4];
    int count;
};
void launch_sums(hipStream_t st, SumJob job, double* out);

}  // namespace mtomg
