// Internal launcher interface between the host library and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "device_common.h"

namespace mtomg {

// The independent systems of one launch, system s = blockIdx.y.  Buffers
// owned by a load case lie `cs` bytes apart, buffers owned by a design `ds`
// bytes apart, and design g owns systems g * cpd .. g * cpd + cpd - 1.  The
// caller's loads F and displacements U are looked up per system when the
// tables are given.  The default describes one system.
struct Batch {
    long long cs = 0, ds = 0;
    int cpd = 1, n = 1;
    const double* const* F = nullptr;
    double* const* U = nullptr;
};

struct SysOff {
    long long c, d;
    int s;
};
__device__ __forceinline__ SysOff sys_off(const Batch& b) {
    const int s = blockIdx.y;
    return SysOff{(long long)s * b.cs, (long long)(s / b.cpd) * b.ds, s};
}
// p shifted by `off` bytes (a null pointer stays null)
template <typename P> __device__ __forceinline__ P* at(P* p, long long off) {
    return p ? reinterpret_cast<P*>(reinterpret_cast<char*>(const_cast<void*>(static_cast<const void*>(p))) + off) : p;
}

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
    double* pq;   // partials of p.q; the kernel stores their total after them
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

// The next sweep or coarse-solve launch records `start` and `stop` from its
// own dispatch (profiling); both events must exist.
void time_next_launch(hipEvent_t start, hipEvent_t stop);

// p[n] = the sum of the partials p[0 .. n-1] (fixed order), per system.
void launch_partial_total(hipStream_t st, double* p, int n, const int* conv, const Batch& bt = Batch{});
template <typename TZ>
void launch_cg_apply(hipStream_t st, LevelOp<double> op, Mat<double> mat, Sweep sw, const TZ* z,
                     const double* p_old, double* p_new, double* x, double* q, const double* zr_cur,
                     const double* zr_prev, int n_zr, const double* pq_prev, int n_pq,
                     double* pq_out, const int* conv, int mode, const Batch& bt = Batch{});
void launch_residual(hipStream_t st, LevelOp<double> op, Mat<double> mat, Sweep sw, const double* f,
                     double* x, int use_x, double* r, double* rr_out, double* ff_out, const int* conv = nullptr,
                     const Batch& bt = Batch{});
template <typename T>
void launch_presmooth(hipStream_t st, bool fine, bool cgmode, LevelOp<T> op, Mat<T> mat, Sweep sw,
                      const T* b, T* u_out, int sweeps, const CgRhs& cg, const int* conv,
                      const Batch& bt = Batch{});
template <typename T>
void launch_restrict(hipStream_t st, bool fine, bool check, LevelOp<T> op, Mat<T> mat, Sweep sw,
                     const T* b, const T* u, T* rc, const ConvCheck& chk, const int* conv,
                     const Batch& bt = Batch{});
// two pre-smoothing sweeps from zero on level l and the restriction of the
// residual they leave: u_out = S(S(0)), rc = P^T (b - K u_out); with cgmode
// b is the outer residual updated from cg (finest grid), with check the
// outer PCG's convergence test (chk) runs first; geometry: 28 coarse
// columns per strip, at most 4 rows per wave
template <typename T>
void launch_pre_restrict(hipStream_t st, bool fine, bool cgmode, bool check, LevelOp<T> op, Mat<T> mat, Sweep sw,
                         const T* b, T* u_out, T* rc, const CgRhs& cg, const ConvCheck& chk, const int* conv,
                         const Batch& bt = Batch{});
// restriction to level l-1 fused with its first (up to two) pre-smoothing
// sweeps; op / opc: levels l and l-1; geometry: 28 coarse columns per strip
template <typename T>
void launch_restrict_pre(hipStream_t st, bool fine, bool check, LevelOp<T> op, LevelOp<T> opc, Mat<T> mat,
                         Sweep sw, const T* b, const T* u, T* rc, T* uc, int sweeps, const ConvCheck& chk,
                         const int* conv, const Batch& bt = Batch{});
template <typename T>
void launch_post(hipStream_t st, bool fine, bool prolong, bool dot, LevelOp<T> op, Mat<T> mat, Sweep sw,
                 const T* u_in, const T* ec, const T* b, T* u_out, const double* r64, double* zr_out,
                 const int* conv, const Batch& bt = Batch{});
// two post-smoothing sweeps in one launch (geometry: 60 output columns per strip)
template <typename T>
void launch_post2(hipStream_t st, bool fine, bool prolong, bool dot, LevelOp<T> op, Mat<T> mat, Sweep sw,
                  const T* u_in, const T* ec, const T* b, T* u_out, const double* r64, double* zr_out,
                  const int* conv, const Batch& bt = Batch{});
// the paired post-smoother of coarse levels l (opc) and l+1 (opf) in one
// launch: u_out = S^2(uf_in + P S^2(uc_in + P ee)) (S: one damped-Jacobi
// sweep of the level; null iterates read zero); geometry: sw of k_post2 on
// level l+1
template <typename T>
void launch_post2_pair(hipStream_t st, LevelOp<T> opc, LevelOp<T> opf, Mat<T> mat, Sweep sw, const T* uc_in,
                       const T* ee, const T* bc, const T* uf_in, const T* bf, T* u_out, const int* conv,
                       const Batch& bt = Batch{});
template <typename T>
void launch_apply(hipStream_t st, bool fine, bool diag, LevelOp<T> op, Mat<T> mat, Sweep sw, const T* u,
                  T* q);
template <typename T>
void launch_coarse_solve(hipStream_t st, const double* Ainv, int n0, int ld, int nx0, const T* b, T* e,
                         const int* conv, const Batch& bt = Batch{});

// setup
struct Phases {
    double dE[8];   // E_i - E_min
    int m;
    double E_min, penal;
};
// flag: the design's input-check word (see k_interp); seq: this call's number (0 .. 2^29 - 1)
void launch_interp(hipStream_t st, const double* x, Phases ph, int n_e, double* E64, float* E32, int* flag,
                   int seq);
void launch_moments_from_fine(hipStream_t st, const double* E64, int nxf, int nyf, double* mom64,
                              float* mom32);
void launch_moments_coarsen(hipStream_t st, const double* momf, int nxf, int nyf, double* mom64,
                            float* mom32);
// moments of nlev (<= 5) consecutive levels below src (moduli when from_e,
// else moment planes) in one launch; T (<= 16, a power of two dividing both
// dimensions of the first output level, T >> (nlev-1) >= 1) is the tile of
// the first output level per workgroup; out.m32[l] may be null
struct MomLevels {
    double* m64[5];
    float* m32[5];
};
void launch_moments_tree(hipStream_t st, bool from_e, const double* src, int nxs, int nys, int T, int nlev,
                         const MomLevels& out);
constexpr int COARSE_NB = 32;   // block size of the coarse factorisation
constexpr int COARSE_LDS_MAX = 4096;   // coarsest DOFs whose right-hand side the coarse solve stages in LDS
// Largest coarsest grid (elements): its dense FP64 factorisation and explicit
// inverse take 5 n0^2 doubles of workspace (11 GB at 64 x 128 elements).
constexpr long MAX_COARSE_ELEMS = 8192;
// also sets status = {0, 1, 0, 0} when given (factor this design)
void launch_assemble_dense(hipStream_t st, bool fine, LevelOp<double> op, Mat<double> mat, double* A, int ld,
                           int* status = nullptr);
// A (np x np, n0 used, identity padding written here; overwritten) ->
// Dinv = inverses of the diagonal blocks of L, W = L^{-1}, Ainv = A^{-1}.
// status[0]: 0 or 1 (not positive definite); status[1]: factor this design
// (the launch skips designs with 0).  `n_designs` designs, `ds` bytes apart.
// half_bw > 0: A[i][j] = 0 for |i - j| > half_bw; up to 64 this selects the
// banded kernels (one workgroup per design for the Cholesky chain, block
// products on the FP64 matrix cores); half_bw <= 0 (or wider bands) runs
// the dense block sequence.  Both give the same factors to rounding.
void launch_coarse_factor(hipStream_t st, double* A, int n0, int np, double* Dinv, double* W, double* Ainv,
                          int* status, double* Lbuf /* np x np */, double* Sacc /* np x np */,
                          int n_designs = 1, long long ds = 0, int half_bw = 0);
// p[k * stride_bytes] = v for k < n
void launch_fill_strided(hipStream_t st, int* p, long long stride_bytes, int n, int v);
template <typename T>
void launch_fill(hipStream_t st, T* p, size_t n, T v);
void launch_cast_f32(hipStream_t st, const double* a, float* b, size_t n);

// after the solve
void launch_grad(hipStream_t st, const double* U, const double* x, Phases ph, Mat<double> mat, int nx,
                 int ny, double* dcdx);
void launch_dot_partials(hipStream_t st, const double* a, const double* b, size_t n, double* partials,
                         int n_part);
// Partial count of a dot product of n terms: one workgroup per 2048 terms
// (one batch of loads per thread), so a large vector gets enough workgroups
// to keep the loads in flight, at most DOT_PARTS_MAX.
constexpr int DOT_PARTS_MAX = 4096;
inline int dot_parts(size_t n) {
    const size_t k = (n + 2047) / 2048;
    return (int)(k < 1 ? 1 : k > (size_t)DOT_PARTS_MAX ? (size_t)DOT_PARTS_MAX : k);
}
void launch_sum_to(hipStream_t st, const double* partials, int n, double* out);
// out[0..] = sums of several partial arrays (one block)
struct SumJob {
    const double* p[4];
    int n[4];
    int count;
};
void launch_sums(hipStream_t st, SumJob job, double* out);
// Per system after a solve: out[0] = ||f||^2, out[1] = recursive ||r||^2
// (from rr[iters & 1], iters = state[1]), out[2] = true ||r||^2; a state
// word 1 (converged, its final x update applied before this launch)
// becomes 2 (done).
void launch_solve_sums(hipStream_t st, const double* ff, int n_ff, const double* rr0, const double* rr1,
                       int n_rr0, int n_rr, const double* trr, int* state, double* out, const Batch& bt);

}  // namespace mtomg
