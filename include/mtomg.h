/*
 * mtomg — pCGMG solver for the multi-material SIMP compliance problem on
 * MI355X (gfx950).
 *
 * The library solves K(x) u = f for a 2D plane-stress wall meshed with
 * nelx x nely square bilinear (Q4) elements, then returns the compliance
 * c = f^T u and its gradient with respect to the phase densities x.  The
 * method is the preconditioned conjugate gradient of Algorithm 2 with one
 * multigrid cycle (Algorithm 1: the V-cycle, gamma = 1, or the W-cycle,
 * gamma = 2, see MTOMG_OPT_GAMMA) as the preconditioner, damped Jacobi
 * smoothing (Section 2.3) and a direct Cholesky solve (Algorithm 3) on the
 * coarsest grid; the stiffness follows Eqs. (5)-(10).  mtomg_filter adds
 * the cone filter that an optimisation loop applies to the densities and
 * sensitivities (Section 4), and mtomg_poisson_solve the Poisson model
 * problem of Section 5.1.
 *
 * Conventions shared by every entry point:
 *   - Node (i, j), i = 0..nelx, j = 0..nely, stores its two displacement
 *     components contiguously; nodal arrays are [nely+1][nelx+1][2]
 *     row-major (x fastest).  Nodes with j = 0 are clamped (u = 0).
 *   - Element (i, j) has phase densities x[j][i][0..m-1] (row-major).
 *   - Pointers marked "device" are HIP device pointers owned by the
 *     caller; the library keeps them (set_grid) or reads them during the
 *     call, and never frees them.  Pointers marked "host" are read during
 *     the call only.
 *   - All device work is ordered on the HIP stream given to mtomg_create.
 *     mtomg_solve blocks until the solve is finished; the other calls are
 *     asynchronous with respect to the host.
 *   - Every call returns MTOMG_OK (0) or a negative status; on failure
 *     mtomg_last_error() describes the cause.  No C++ exception crosses
 *     this interface.  A context is not thread-safe.
 */
#ifndef MTOMG_H
#define MTOMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mtomg_ctx mtomg_ctx;

enum {
    MTOMG_OK = 0,
    MTOMG_BAD_INPUT = -1,     /* invalid argument or size                        */
    MTOMG_NOT_CONVERGED = -2, /* max_iter reached, or the true residual stays    */
                              /* above rel_tol; U holds the last iterate         */
    MTOMG_BREAKDOWN = -3,     /* p^T K p <= 0 or z^T r <= 0 inside PCG, or the   */
                              /* coarsest matrix is not positive definite        */
    MTOMG_NAN = -4,           /* non-finite residual or non-finite densities     */
    MTOMG_WORKSPACE = -5,     /* workspace missing or too small                  */
    MTOMG_HIP_ERROR = -6,     /* a HIP runtime call failed                       */
    MTOMG_STATE = -7          /* call out of order (e.g. solve before set_grid)  */
};

/* Arithmetic of the multigrid preconditioner.  The outer CG recurrences
 * (residual and iterate updates, dot products), the coarsest Cholesky
 * factor and the compliance are FP64 in both modes. */
enum { MTOMG_FP64 = 0, MTOMG_FP32MG = 1 };

/* Per (design, load case) solve statistics. */
typedef struct {
    int32_t status;      /* MTOMG_OK / NOT_CONVERGED / BREAKDOWN / NAN, or    */
                         /* BAD_INPUT for densities outside [0, 1]            */
    int32_t iters;       /* PCG iterations (updates of u), all runs            */
    int32_t vcycles;     /* preconditioner applications                        */
    int32_t n_dof;       /* 2 (nelx+1)(nely+1), clamped DOFs included          */
    double relres_rec;   /* recursive ||r|| / ||f|| at exit                    */
    double relres_true;  /* ||f - K u|| / ||f|| recomputed in FP64 at exit     */
    double t_setup_ms;   /* device time of the last set_densities plus the     */
                         /* coarsest factorisation (shared by its group)       */
    double t_solve_ms;   /* device time of the whole solve call (all systems), */
                         /* including waits for coarsest factorisations that   */
                         /* run beside its first V-cycle                       */
    double model_bytes;  /* algorithmic HBM bytes of one PCG iteration         */
} mtomg_stats;

/* Create a context for up to max_designs independent designs.
 * hip_stream: a hipStream_t (NULL = the null stream) on which all work is
 * ordered.  Returns BAD_INPUT if max_designs < 1, HIP_ERROR if no device. */
int mtomg_create(mtomg_ctx **ctx, int max_designs, void *hip_stream);

/* Release every device resource the library allocated.  Caller-owned
 * buffers are untouched.  NULL is accepted. */
int mtomg_destroy(mtomg_ctx *ctx);

/* Describe design `design` (0 <= design < max_designs).
 * The wall is the rectangle [0, nelx h] x [0, nely h] of square elements of
 * side h and thickness 1.  There is no h argument: the plane-stress element
 * stiffness of Eqs. (7)-(9) does not depend on the element size in 2D, so h
 * enters only through the loads, which the caller gives as nodal forces F.
 *   nelx, nely   element counts; both divisible by 2^(levels-1), and the
 *                coarsest grid at most 8192 elements (e.g. 64 x 128): its
 *                FP64 factorisation and explicit inverse are kept in
 *                device memory, about 5 n0^2 doubles of workspace for its
 *                n0 = 2 (nx0 + 1) ny0 free DOFs (11 GB at 64 x 128; up to
 *                24 x 24 elements a banded factorisation needs less work).
 *   nu           Poisson ratio of the plane-stress law, Eq. (8), in [0, 0.5).
 *   m, E_phase   number of solid phases and their moduli (host [m]), Eq. (5).
 *   E_min        modulus of the void phase, > 0.
 *   penal        SIMP exponent p >= 1 of Eq. (5).
 *   levels       number of grids of the hierarchy (Algorithm 1), 2..14.
 *                One grid is not accepted: its "cycle" would be the exact
 *                coarsest solve of the whole system, a direct method
 *                rather than the multigrid preconditioner.
 *   n_pre/n_post damped-Jacobi sweeps before/after the coarse correction
 *                (theta_1, theta_2 of Algorithm 1), 0..8; equal values
 *                keep the preconditioner symmetric (Section 2.2).
 *   omega        damping of the Jacobi smoother (Section 2.3), in (0, 1].
 *   precision    MTOMG_FP64 or MTOMG_FP32MG.
 *   n_cases      number of load cases sharing this stiffness, 1..64.
 *   F            device [n_cases][nely+1][nelx+1][2] FP64 nodal loads; read
 *                at each solve.  Values on the clamped row are ignored.
 *   U            device, same shape, FP64; receives the displacements (and
 *                is the initial guess when solve is called with warm_start).
 * Invalidates the workspace: call mtomg_workspace_bytes/set_workspace (or
 * let the library allocate) before the next set_densities. */
int mtomg_set_grid(mtomg_ctx *ctx, int design, int nelx, int nely, double nu, int m,
                   const double *E_phase, double E_min, double penal, int levels,
                   int n_pre, int n_post, double omega, int precision, int n_cases,
                   const double *F, double *U);

/* Bytes of device workspace needed by all designs described so far. */
size_t mtomg_workspace_bytes(const mtomg_ctx *ctx);

/* Hand the library a caller-owned device buffer of at least
 * mtomg_workspace_bytes() bytes (256-byte aligned).  The caller keeps it
 * alive until the next set_grid or destroy.  Without this call the library
 * allocates its own workspace with hipMalloc at the first set_densities. */
int mtomg_set_workspace(mtomg_ctx *ctx, void *dev, size_t bytes);

/* Load phase densities for a design and build its preconditioner:
 * element moduli by Eq. (5), Galerkin coarse operators for every level and
 * the assembled coarsest matrix.  Its Cholesky factor (Algorithm 3), turned
 * into an explicit inverse, is computed on a private stream of the context:
 * for a design alone in its group (the designs sharing its shape, see
 * mtomg_solve) it starts at once, after the assembly; otherwise the next
 * solve starts it, together with those of the other designs of the group
 * whose densities changed (one launch sequence for all of them).  Either way
 * the first coarse solve of the next solve waits for it.
 * x: device [nely][nelx][m] FP64 in [0, 1], read in stream order (keep it
 * alive until the work is done).  Asynchronous, so x is checked on the
 * device, and the next solve reports the result for every load case of the
 * design without extra synchronisation: BAD_INPUT if some density lies
 * outside [0, 1], NAN if some density is not finite, BREAKDOWN if the
 * coarsest matrix is not positive definite.  Such a design takes no further
 * PCG runs after the first, and its U then holds no solution. */
int mtomg_set_densities(mtomg_ctx *ctx, int design, const double *x);

/* Solve every load case of every design that has densities: PCG
 * (Algorithm 2) from u = 0 (or from U when warm_start != 0), stopping when
 * ||r||_2 <= rel_tol ||f||_2 over the free DOFs, or after max_iter
 * iterations.  The test runs on the recursively updated residual and is
 * confirmed on the true FP64 residual f - K u; a system that fails the
 * confirmation (the two drift apart over thousands of iterations at high
 * modulus contrast) restarts PCG from its current u, at most 4 times, with
 * max_iter counting the iterations of all runs.  Designs that share nelx, nely, levels, precision, n_pre,
 * n_post, nu, omega and n_cases form a group: each kernel launch serves
 * every (design, load case) system of a group, all groups iterate together
 * and two iterations of all of them replay as one HIP graph; a system that
 * has converged skips the remaining launches.  Designs without densities
 * are left untouched.  stats: host array with one entry per load case of
 * every design that has densities, in design then case order.  Blocks
 * until done.  Returns the worst status. */
int mtomg_solve(mtomg_ctx *ctx, double rel_tol, int max_iter, int warm_start,
                mtomg_stats *stats);

/* Compliance c_k = f_k^T u_k (Eq. 6) of every load case, and optionally
 * its gradient dc_k/dx_{e,i} = -p x_{e,i}^(p-1) (E_i - E_min) u_e^T K^0 u_e
 * (the sensitivity step of Section 4; compliance is self-adjoint).
 *   c     device [n_cases] FP64.
 *   dcdx  device [n_cases][nely][nelx][m] FP64, or NULL to skip.
 * Uses the displacements of the last solve. */
int mtomg_compliance_and_grad(mtomg_ctx *ctx, int design, double *c, double *dcdx);

/* Cone filter of an element field, one pass per phase: the sensitivity
 * filtering of the optimisation loop (Section 4) with the filter radius rf
 * of Table 2.  The paper does not write the filter out; this is the usual
 * cone filter on element centres,
 *   H_ef = max(0, rf - |c_e - c_f|)   (distance in element widths),
 *   S_e  = sum_f H_ef                 (over the elements of the grid),
 * with, per phase,
 *   MTOMG_FILTER_DENSITY:          out_e = sum_f H_ef in_f / S_e
 *   MTOMG_FILTER_DENSITY_ADJOINT:  out_e = sum_f H_ef in_f / S_f, the chain
 *                                  rule through the density filter (H is
 *                                  symmetric): in = dJ/d(filtered x),
 *                                  out = dJ/dx;
 *   MTOMG_FILTER_SENSITIVITY:      out_e = sum_f H_ef x_f in_f
 *                                          / (max(gmin, x_e) S_e).
 * x, in, out: device [nely][nelx][m] FP64; x is read by the sensitivity
 * filter only (densities of the same phases), gmin > 0 keeps void elements
 * finite there (1e-3 is usual).  0 < rf <= 16; rf <= 1 leaves only the
 * element itself.  At most 2^22 columns, 2^20 rows and 2^30 elements.
 * out must not alias in or x.  Asynchronous on the
 * context's stream; needs no design.  Returns BAD_INPUT for invalid
 * arguments. */
enum { MTOMG_FILTER_DENSITY = 0, MTOMG_FILTER_DENSITY_ADJOINT = 1, MTOMG_FILTER_SENSITIVITY = 2 };
int mtomg_filter(mtomg_ctx *ctx, int nelx, int nely, int m, double rf, int mode, double gmin, const double *x,
                 const double *in, double *out);

/* mtomg_filter for callers that cannot allocate device or host memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same filter and the same kernels, with the weight table
 * held in a statically allocated device array of 1,985 doubles (15.9 KB,
 * the table of the largest radius, rf = 16) instead of a per-context
 * buffer.  Needs no context: work is ordered on hip_stream (a hipStream_t,
 * NULL = the null stream) of the current device.  Each call rebuilds the
 * table for its rf on the device and then filters, allocating nothing.
 * Every call on one GPU shares that GPU's table: calls that overlap in time
 * on one GPU (different streams, or several host threads) race and must be
 * serialised by the caller; calls ordered on one stream are safe.  Each GPU
 * keeps its copy until the process ends.  Arguments, layouts and limits as
 * mtomg_filter (rf beyond 16 is rejected).  Returns MTOMG_OK, BAD_INPUT for
 * invalid arguments (there is no context to hold a message), or HIP_ERROR
 * if the launch fails.  Asynchronous. */
int mtomg_filter_noalloc(void *hip_stream, int nelx, int nely, int m, double rf, int mode, double gmin,
                         const double *x, const double *in, double *out);

/* One binary sub-problem of the alternating active-phase optimality-criteria
 * update (Section 4: pairs of active phases, Gauss-Seidel order; parameters
 * of Table 2).  The paper does not write the update out; this is the
 * reading implemented.  x holds the m solid phases, the void share
 * 1 - sum_i x_i is implicit (phase index m) and has no sensitivity.  For
 * phases a < b (b = m: the void), with s_e = x_{e,a} + x_{e,b} held fixed per
 * element and the pair sensitivity d_e = g_{e,a} - g_{e,b}:
 *   lo_e = max(eps, x_{e,a} - move),  hi_e = min(1, s_e - eps, x_{e,a} + move),
 *   y_e(lambda) = clamp(x_{e,a} (max(0, -d_e) / lambda)^eta, lo_e, hi_e),
 * with lambda > 0 chosen so that sum_e y_e = vol_a nelx nely (the volume of
 * phase a); then x_{e,a} = y_e and x_{e,b} = s_e - y_e.  lambda is found on
 * the device (Newton steps on the piecewise-linear volume sum, kept in a
 * bracket); a target outside the reachable range puts every element at
 * its lower (or every element with d_e < 0 at its upper) bound.
 *   g:     device [nely][nelx][m] FP64, the (filtered) compliance gradient.
 *   x:     device [nely][nelx][m] FP64, updated in place; every phase, void
 *          included, must lie in [eps, 1] on entry and stays there.
 *   vol_a: target volume fraction of phase a, in [0, 1].
 *   move > 0, eta in (0, 2] (1/2 is usual), eps in (0, 1/(2(m+1))).
 *   info:  host [4] or NULL: lambda, the largest |change| of x_{e,a},
 *          sum y - target, and the number of passes (+ 0.5 if the pass
 *          limit ended it before convergence); with info the call
 *          synchronises, otherwise it is asynchronous.
 * Uses a workspace the context allocates on first use.  Returns BAD_INPUT
 * for invalid arguments. */
int mtomg_oc_update(mtomg_ctx *ctx, int nelx, int nely, int m, int a, int b, const double *g, double vol_a,
                    double move, double eta, double eps, double *x, double *info);

/* One outer iteration of the alternating active-phase loop (Section 4) on
 * design `design`, which must be the only design of its context with
 * densities: for every pair (a, b), a < b, in the order (0,1), (0,2), ...,
 * (0,m), (1,2), ..., (m-1,m), with the densities left by the previous pair,
 * set_densities(x), a warm-started solve (from U) to rel_tol, compliance and
 * gradient of every load case, the gradient summed over the load cases, the
 * sensitivity filter of radius rf (floor gmin, mtomg_filter) on each solid
 * phase, then mtomg_oc_update with the target vols[a].
 *   vols:    host [m+1] target volume fractions, void last, summing to 1.
 *   x:       device [nely][nelx][m], the densities, updated in place (every
 *            phase, void included, in [eps, 1]).
 *   c_pairs: host [m(m+1)/2], the compliance summed over load cases before
 *            each pair's update.
 *   change:  host, the largest change of any density (void included) over
 *            the iteration; the loop stops when it is at most tol
 *            (Table 2: 1e-3).
 *   iters:   host [m(m+1)/2] or NULL: PCG iterations of each pair's solve
 *            (the most over the load cases).
 * A solve that does not reach rel_tol ends the step with its status.
 * Blocks until done. */
int mtomg_aap_step(mtomg_ctx *ctx, int design, const double *vols, double rf, double move, double eta, double eps,
                   double gmin, double rel_tol, int max_iter, double *x, double *c_pairs, double *change,
                   int *iters);

/* The Poisson model problem of Section 5.1: -Laplace(u) = f on the unit
 * square with u = 0 on the whole boundary, bilinear (Q4) elements on an
 * n x n grid of square elements, solved by PCG (Algorithm 2) with one
 * multigrid V-cycle (Algorithm 1: n_pre + n_post damped Jacobi sweeps with
 * weight omega, full-weighting restriction, bilinear prolongation) down to
 * the 2 x 2 grid, where the one unknown is solved exactly, as in the
 * paper's runs (16^2 .. 256^2 with 3 .. 7 levels).  All arithmetic is
 * FP64; the operator on every grid is the Q4 Laplace stencil, which equals
 * the Galerkin product of the finer one.
 *   n:      power of two in [4, 8192]; levels = log2(n).
 *   f:      device [n+1][n+1] FP64, the nodal load vector (the Q4 mass
 *           matrix applied to the source); boundary entries are ignored.
 *   u:      device [n+1][n+1] FP64 output (boundary entries 0); must not
 *           alias f.
 *   stats:  host, one entry (n_dof = (n-1)^2 interior unknowns,
 *           t_solve_ms the device time of the call, t_setup_ms 0).
 * Stops when ||f - K u|| <= rel_tol ||f|| on the recursive residual, or
 * after max_iter iterations.  Uses the context's stream and a workspace the
 * context allocates on first use (kept until mtomg_destroy); the host reads
 * the residual once per iteration.  Blocks until done.  Returns the status
 * (also in stats). */
int mtomg_poisson_solve(mtomg_ctx *ctx, int n, int n_pre, int n_post, double omega, double rel_tol, int max_iter,
                        const double *f, double *u, mtomg_stats *stats);

/* Static description of a status code. */
const char *mtomg_status_string(int status);

/* Message of the last failure on this context ("" if none). */
const char *mtomg_last_error(const mtomg_ctx *ctx);

/* Options of a context.
 *   MTOMG_OPT_GRAPHS (default 1): replay the PCG iteration body from a
 *     captured HIP graph (two iterations per replay) instead of launching
 *     its kernels one by one; results are identical either way.
 *   MTOMG_OPT_BATCH (default 8, 1..1000): iterations launched before the
 *     host first reads the convergence state; later solves start from the
 *     previous iteration count instead.  Setting it clears that history.
 *   MTOMG_OPT_ROWS_FINE / MTOMG_OPT_ROWS_COARSE (default 0 = automatic;
 *     1, 2, 4 or 8): node rows each wave marches through in the sweeps of
 *     the finest grid / of the coarse grids (a tuning knob).  Changing it
 *     re-plans every design: a workspace given with set_workspace must be
 *     given again (the size may change) and densities set again.
 *   MTOMG_OPT_DENSE_FACTOR (default 0): 1 factors the coarsest matrix by the
 *     dense 32 x 32 block sequence (one launch per block step, vector FP64
 *     products) instead of the banded kernels (one workgroup per design for
 *     the Cholesky chain, products on the FP64 matrix cores); both give
 *     K_0^{-1} to rounding (a test and comparison knob).  Applies to
 *     factorisations run after the call.
 *   MTOMG_OPT_GAMMA (default 1; 1 or 2): the cycle index gamma of
 *     Algorithm 1 (Section 2.1), used by every design of the context.
 *     1 is the V-cycle; 2 the W-cycle, in which each level below the
 *     finest is visited twice per visit of the level above, the second
 *     visit starting from the first one's result.  The coarsest level is
 *     the exact solve, so a repeated visit there gives the same result and
 *     runs once.  A W-cycle visits level l 2^(L-1-l) times per
 *     preconditioner application (L levels), so it pays only where the
 *     V-cycle needs many more iterations.  Changing it drops the captured
 *     graphs and the iteration-count history (MTOMG_OPT_BATCH).
 *   MTOMG_OPT_RESTARTS (default 4; 0..64): how many times a system whose
 *     true residual fails the confirmation restarts PCG from its current u
 *     (within max_iter in total).
 *   MTOMG_OPT_ROWS_CG (default 0 = automatic, as for the sweeps; 1, 2, 4
 *     or 8): node rows per wave of the outer-CG stiffness apply,
 *     independent of MTOMG_OPT_ROWS_FINE.
 *   MTOMG_OPT_ROWS_LEVEL + k, k = 1..13 (default 0 = MTOMG_OPT_ROWS_COARSE;
 *     1, 2, 4 or 8): rows per wave on the grid k levels below the finest.
 *   The ROWS options re-plan every design, as MTOMG_OPT_ROWS_FINE does.
 *   MTOMG_OPT_FUSE_PRE (default 1): run the two pre-smoothing sweeps of a
 *     level and the restriction of the residual they leave in one launch
 *     (Section 2.3 steps fused; on the finest grid together with the CG
 *     update of r, the convergence test then opening the level below)
 *     where no other fusion of that level is used: n_pre = 2, the V-cycle,
 *     and for the finest grid 3 levels or a grid two below the finest of
 *     more than 32768 nodes.  0 launches the steps one by one.  Both take
 *     the same operations per node in the same order; they differ by
 *     rounding only (the compiler forms fused multiply-adds differently
 *     in the two kernels, and the partial sums of ||r||^2 are grouped by
 *     different tiles). */
enum { MTOMG_OPT_GRAPHS = 0, MTOMG_OPT_BATCH = 1, MTOMG_OPT_ROWS_FINE = 2, MTOMG_OPT_ROWS_COARSE = 3,
       MTOMG_OPT_DENSE_FACTOR = 4, MTOMG_OPT_GAMMA = 5, MTOMG_OPT_RESTARTS = 6, MTOMG_OPT_ROWS_CG = 7,
       MTOMG_OPT_FUSE_PRE = 8, MTOMG_OPT_ROWS_LEVEL = 16 };
int mtomg_set_option(mtomg_ctx *ctx, int option, int value);

/* Profiling: time every launch of one solver kernel during the following
 * solves with a pair of HIP events stamped by that launch's own dispatch
 * (hipExtLaunchKernel), so a duration is the kernel's execution alone;
 * graphs are not replayed meanwhile (kernel = MTOMG_KERNEL_NONE switches
 * it off).  At most 4096 launches are timed between reads.
 * mtomg_profile_read synchronises the stream, writes the duration in ms of
 * each timed launch since the last read, in launch order, to ms[0..cap-1]
 * (host) and their count to *launches (host), then starts a new record.
 * Launches that found the solve already converged exit at once and show as
 * near-zero durations. */
enum {
    MTOMG_KERNEL_NONE = 0,
    MTOMG_KERNEL_CG_APPLY = 1,        /* FP64 p update + K p + p.q (outer CG)      */
    MTOMG_KERNEL_FINE_PRESMOOTH = 2,  /* r update + two Jacobi sweeps, finest grid
                                         (+ residual restriction when fused)      */
    MTOMG_KERNEL_FINE_RESTRICT = 3,   /* residual + restriction, finest grid
                                         (no launch when fused, see FUSE_PRE)     */
    MTOMG_KERNEL_FINE_POST = 4,       /* prolongation + Jacobi sweep, finest grid  */
    MTOMG_KERNEL_FINE_POST_DOT = 5,   /* last Jacobi sweep + z.r, finest grid      */
    MTOMG_KERNEL_COARSE_SOLVE = 6     /* explicit-inverse coarsest solve           */
};
int mtomg_profile_kernel(mtomg_ctx *ctx, int kernel);
int mtomg_profile_read(mtomg_ctx *ctx, double *ms, int cap, int *launches);

/* Practical HBM ceiling for the roofline of the bandwidth-bound kernels:
 * time `reps` back-to-back passes of a hand-written streaming kernel over n
 * doubles (16-byte loads and stores, 8 workgroups per compute unit) with
 * HIP events on the context's stream, after one untimed pass.
 *   MTOMG_PROBE_READ:  reads a (8 n bytes); writes one double per workgroup
 *                      into b.
 *   MTOMG_PROBE_COPY:  b = a (16 n bytes).
 *   MTOMG_PROBE_TRIAD: a = b + 3 c (24 n bytes).
 * a, b, c: device arrays of n doubles, 16-byte aligned (c used by TRIAD
 * only); n even and at least 2^20.  *ms (host): device time per pass.
 * Blocks until done. */
enum { MTOMG_PROBE_READ = 0, MTOMG_PROBE_COPY = 1, MTOMG_PROBE_TRIAD = 2 };
int mtomg_stream_probe(mtomg_ctx *ctx, int kind, double *a, double *b, double *c, size_t n, int reps, double *ms);

/* Test hook: run one internal operator of level `level` (0 = coarsest,
 * levels-1 = finest) of a design whose densities are set.  Vectors are
 * nodal arrays of that level ([ny_l+1][nx_l+1][2]) in the multigrid
 * precision (float for MTOMG_FP32MG, double otherwise) except
 * MTOMG_OP_APPLY64, which is FP64.  `in` holds the listed inputs back to
 * back; `out` receives one vector.  Both are device pointers.
 *   APPLY     in: u           out: K_l u
 *   APPLY64   in: u (FP64)    out: K u on the finest grid in FP64
 *   DIAG      in: -           out: diag(K_l)
 *   PRESMOOTH in: b           out: n_pre damped-Jacobi sweeps from u = 0
 *   RESIDUAL_RESTRICT
 *             in: b, u        out (level l-1): P_l^T (b - K_l u)
 *   PROLONG_POSTSMOOTH
 *             in: b, u, e_c   out: n_post sweeps from u + P_l e_c
 *                               (e_c is a level l-1 vector)
 *   SMOOTH    in: b, u        out: one damped-Jacobi sweep from u
 *   COARSE_SOLVE (level 0)
 *             in: b           out: K_0^{-1} b
 *   VCYCLE    in: b           out: MG_1^l(0, b) (Algorithm 1)
 *   PRESMOOTH_RESTRICT (n_pre = 2)
 *             in: b           out: P_l^T (b - K_l u) (a level l-1 vector)
 *                               followed by u, two damped-Jacobi sweeps
 *                               from 0 (the fused launch of FUSE_PRE)
 */
enum {
    MTOMG_OP_APPLY = 0,
    MTOMG_OP_APPLY64 = 1,
    MTOMG_OP_DIAG = 2,
    MTOMG_OP_PRESMOOTH = 3,
    MTOMG_OP_RESIDUAL_RESTRICT = 4,
    MTOMG_OP_PROLONG_POSTSMOOTH = 5,
    MTOMG_OP_SMOOTH = 6,
    MTOMG_OP_COARSE_SOLVE = 7,
    MTOMG_OP_VCYCLE = 8,
    MTOMG_OP_PRESMOOTH_RESTRICT = 9
};
int mtomg_debug_apply(mtomg_ctx *ctx, int design, int level, int op, const void *in, void *out);

#ifdef __cplusplus
}
#endif

#endif /* MTOMG_H */
