// Level sweeps of the pCGMG solver: the FP64 stiffness apply of the outer
// CG (Algorithm 2), and the damped-Jacobi smoothing, residual restriction
// and prolongation steps of the multigrid cycle (Algorithm 1, Section 2.3).
//
// Execution model (every kernel below): a wave owns a vertical strip of 64
// node columns and a chunk of `rows` node rows; lane l holds node column
// i = strip * W_OUT - H_L + l and the element column i to its right.  The
// wave marches upward one element row per step, keeping the two node rows
// an element touches in registers.  Each step computes the element's nodal
// forces (and diagonal) once; node (i, j) collects its four elements as
//   own element row j (local node 0) + left lane's (local node 1)
//   + carry from element row j-1: own (local node 3) + left lane's (node 2),
// with left/right neighbours exchanged by lane shuffles.  Loads are
// therefore one coalesced node value and one element record per lane and
// row.  Lanes at the strip edges only feed their neighbours; strips overlap
// by H_L + H_R columns and chunks re-read one or two halo rows.
// Four waves form a workgroup (four stacked chunks of one strip).
#include <hip/hip_ext.h>

#include "device_common.h"
#include "kernels.h"

namespace mtomg {

struct TileInfo {
    int tile, strip, j0, j1;
    bool block_ok;
};

template <int R>
__device__ __forceinline__ TileInfo tile_info(const Sweep& s, int n_rows) {
    TileInfo t;
    t.tile = xcd_tile(s.n_tiles);
    t.block_ok = t.tile < s.n_tiles;
    t.strip = t.tile % s.n_strips;
    const int chunk = (t.tile / s.n_strips) * WAVES_PER_WG + wave_id();
    t.j0 = chunk * R;
    t.j1 = min(t.j0 + R, n_rows);
    return t;
}

// ===========================================================================
// Total of a sweep's n partial sums, stored after them (p[n]) for the
// kernels that need it at their start: one workgroup per system, the fixed
// order of sum_partials.  Systems whose state word is not 0 are skipped
// (their producer did not run).
// ===========================================================================
__global__ __launch_bounds__(WG_THREADS) void k_partial_total(double* __restrict__ p, int n, const int* conv,
                                                              Batch bt) {
    const SysOff so = sys_off(bt);
    if (load_state(at(conv, so.c)) != 0) return;
    p = at(p, so.c);
    const double s = sum_partials(p, n);
    if (threadIdx.x == 0) p[n] = s;
}

// ===========================================================================
// Outer CG: p = z + beta p_old, x += alpha_prev p_old, q = K p, partial p.q
// mode 0: iteration i >= 1; mode 1: first iteration (beta = 0, no x update);
// mode 2: only the pending x update (after the last iteration); mode 3: the
// same for the systems whose state is 0 (iteration limit) or 1 (converged,
// update pending), nothing for the others; mode 4: the same for state 1
// only (systems still running are left to continue).
// Geometry: H_L = 1, H_R = 1, 62 output columns per strip.
// Every kernel first issues all loads of its rows (masked, branch-free),
// then marches through the rows from registers.
// ===========================================================================
template <typename TZ, int R>
__global__ __launch_bounds__(WG_THREADS) void k_cg_apply(
    LevelOp<double> op, Mat<double> mat, Sweep sw, const TZ* __restrict__ z,
    const double* __restrict__ p_old, double* __restrict__ p_new, double* __restrict__ x,
    double* __restrict__ q, const double* __restrict__ zr_cur, const double* __restrict__ zr_prev,
    int n_zr, const double* __restrict__ pq_prev, int n_pq, double* __restrict__ pq_out,
    const int* conv, int mode, Batch bt) {
    const SysOff so = sys_off(bt);
    conv = at(conv, so.c);
    op.data = at(op.data, so.d);
    z = at(z, so.c);
    p_old = at(p_old, so.c);
    p_new = at(p_new, so.c);
    x = bt.U ? bt.U[so.s] : x;
    q = at(q, so.c);
    zr_cur = at(zr_cur, so.c);
    zr_prev = at(zr_prev, so.c);
    pq_prev = at(pq_prev, so.c);
    pq_out = at(pq_out, so.c);
    const int cst = *conv;
    const bool final_only = (mode >= 2) || (mode == 0 && cst == 1);
    if (mode == 1 && cst != 0) return;
    if ((mode == 0 || mode == 3) && cst != 0 && cst != 1) return;
    if (mode == 4 && cst != 1) return;
    const int nx = op.nx, ny = op.ny;
    const TileInfo t = tile_info<R>(sw, ny + 1);
    if (!t.block_ok) return;
    constexpr int HL = 1, WOUT = 62;
    const int lane = lane_id();
    const int i = t.strip * WOUT - HL + lane;
    const bool out_lane = lane >= HL && lane < HL + WOUT && i <= nx;

    double alpha_prev = 0.0, beta = 0.0, rho_prev = 1.0, rho_cur = 0.0;
    if (mode != 1) {
        // rho_{i-1}, p_{i-1}.q_{i-1} and rho_i: totals stored after the
        // partials by their producers (rho_i is unused by the final-only
        // modes; its slot is valid memory there)
        rho_prev = zr_prev[n_zr];
        alpha_prev = rho_prev / pq_prev[n_pq];
        rho_cur = zr_cur[n_zr];
    }
    if (final_only) {
        if (out_lane) {
            for (int j = max(t.j0, 1); j < t.j1; ++j) {
                V2<double> xv = load_node(x, nx, ny, i, j);
                const V2<double> pv = load_node(p_old, nx, ny, i, j);
                xv.x += alpha_prev * pv.x;
                xv.y += alpha_prev * pv.y;
                store_node(x, nx, i, j, xv);
            }
        }
        return;
    }
    if (mode == 0) beta = rho_cur / rho_prev;

    double dot = 0.0;
    if (t.j0 < t.j1) {
        // rows j0-1 .. j0+R of z and p_old, element rows j0-1 .. j0+R-1, x of rows j0 .. j0+R-1
        V2<TZ> zr[R + 2];
        V2<double> po[R + 2], xr[R];
        Mom<double> me[R + 1];
#pragma unroll
        for (int s = 0; s < R + 2; ++s) zr[s] = load_node(z, nx, ny, i, t.j0 - 1 + s);
        if (mode == 0) {
#pragma unroll
            for (int s = 0; s < R + 2; ++s) po[s] = load_node(p_old, nx, ny, i, t.j0 - 1 + s);
#pragma unroll
            for (int s = 0; s < R; ++s) xr[s] = load_node(x, nx, ny, i, t.j0 + s);
        } else {
#pragma unroll
            for (int s = 0; s < R + 2; ++s) po[s] = V2<double>{0.0, 0.0};
        }
#pragma unroll
        for (int s = 0; s < R + 1; ++s) me[s] = load_elem<double, true>(op, i, t.j0 - 1 + s);

        V2<double> p[R + 2];
#pragma unroll
        for (int s = 0; s < R + 2; ++s) {
            p[s] = V2<double>{(double)zr[s].x + beta * po[s].x, (double)zr[s].y + beta * po[s].y};
            const int jj = t.j0 - 1 + s;
            if (s >= 1 && s <= R && out_lane && jj < t.j1) {
                if (jj >= 1) {
                    store_node(p_new, nx, i, jj, p[s]);
                    if (mode == 0) {
                        const V2<double> xv{xr[s - 1].x + alpha_prev * po[s].x, xr[s - 1].y + alpha_prev * po[s].y};
                        store_node(x, nx, i, jj, xv);
                    }
                } else {
                    store_node(p_new, nx, i, jj, V2<double>{0.0, 0.0});
                }
            }
        }
        V2<double> f0, f1, f2, f3;
        V2<double> pr_lo = from_right(p[0]), pr_hi = from_right(p[1]);
        elem_force<true>(me[0], mat, p[0], pr_lo, pr_hi, p[1], f0, f1, f2, f3);
        V2<double> carry = f3 + from_left(f2);
#pragma unroll
        for (int s = 0; s < R; ++s) {
            const int j = t.j0 + s;
            pr_lo = pr_hi;
            pr_hi = from_right(p[s + 2]);
            elem_force<true>(me[s + 1], mat, p[s + 1], pr_lo, pr_hi, p[s + 2], f0, f1, f2, f3);
            const V2<double> qv = carry + f0 + from_left(f1);
            carry = f3 + from_left(f2);
            if (out_lane && j < t.j1) {
                if (j >= 1) {
                    store_node(q, nx, i, j, qv);
                    dot += p[s + 1].x * qv.x + p[s + 1].y * qv.y;
                } else {
                    store_node(q, nx, i, j, V2<double>{0.0, 0.0});
                }
            }
        }
    }
    const double s = block_sum(dot);
    if (threadIdx.x == 0) pq_out[t.tile] = s;
}

// ===========================================================================
// Residual r = f - K x (FP64) at the start of a solve; x = 0 unless warm.
// Writes r (clamped row zeroed) and x (clamped row zeroed), partial sums of
// ||r||^2 and ||f||^2 over free DOFs.  Also used for the true residual
// (then r may be null).  Systems whose state is 5 (not part of this solve)
// are left alone.  Geometry as k_cg_apply.
// ===========================================================================
template <int R>
__global__ __launch_bounds__(WG_THREADS) void k_residual(
    LevelOp<double> op, Mat<double> mat, Sweep sw, const double* __restrict__ f,
    double* __restrict__ x, int use_x, double* __restrict__ r, double* __restrict__ rr_out,
    double* __restrict__ ff_out, const int* conv, Batch bt) {
    const SysOff so = sys_off(bt);
    conv = at(conv, so.c);
    if (conv && *conv == 5) return;
    op.data = at(op.data, so.d);
    f = bt.F ? bt.F[so.s] : f;
    x = bt.U ? bt.U[so.s] : x;
    r = at(r, so.c);
    rr_out = at(rr_out, so.c);
    ff_out = at(ff_out, so.c);
    const int nx = op.nx, ny = op.ny;
    const TileInfo t = tile_info<R>(sw, ny + 1);
    if (!t.block_ok) return;
    constexpr int HL = 1, WOUT = 62;
    const int lane = lane_id();
    const int i = t.strip * WOUT - HL + lane;
    const bool out_lane = lane >= HL && lane < HL + WOUT && i <= nx;
    double rr = 0.0, ff = 0.0;
    // every wave issues its loads, none under a branch (rows past the grid
    // are masked); a cold start (use_x = 0) reads f, which is finite, in
    // place of x under a zero mask, so U's old contents never enter
    const double* xs = use_x ? x : f;
    V2<double> xr[R + 2], fr[R];
    Mom<double> me[R + 1];
#pragma unroll
    for (int s = 0; s < R + 2; ++s) xr[s] = load_node(xs, nx, ny, i, t.j0 - 1 + s, use_x != 0);
#pragma unroll
    for (int s = 0; s < R; ++s) fr[s] = load_node(f, nx, ny, i, t.j0 + s);
#pragma unroll
    for (int s = 0; s < R + 1; ++s) me[s] = load_elem<double, true>(op, i, t.j0 - 1 + s);
    __builtin_amdgcn_sched_barrier(0);   // one batch of loads ahead of the arithmetic
    // the arithmetic runs on every wave and its values are used without a
    // branch (only the stores are conditional), so no load is sunk into one
    V2<double> f0, f1, f2, f3;
    V2<double> xr_lo = from_right(xr[0]), xr_hi = from_right(xr[1]);
    elem_force<true>(me[0], mat, xr[0], xr_lo, xr_hi, xr[1], f0, f1, f2, f3);
    V2<double> carry = f3 + from_left(f2);
#pragma unroll
    for (int s = 0; s < R; ++s) {
        const int j = t.j0 + s;
        xr_lo = xr_hi;
        xr_hi = from_right(xr[s + 2]);
        elem_force<true>(me[s + 1], mat, xr[s + 1], xr_lo, xr_hi, xr[s + 2], f0, f1, f2, f3);
        const V2<double> kx = carry + f0 + from_left(f1);
        carry = f3 + from_left(f2);
        const bool own = out_lane && j < t.j1;
        const bool fre = own && j >= 1;
        const V2<double> rv = fr[s] - kx;
        rr += fre ? rv.x * rv.x + rv.y * rv.y : 0.0;
        ff += fre ? fr[s].x * fr[s].x + fr[s].y * fr[s].y : 0.0;
        if (own) {
            if (j >= 1) {
                if (r) store_node(r, nx, i, j, rv);
                if (!use_x) store_node(x, nx, i, j, V2<double>{0.0, 0.0});
            } else {
                if (r) store_node(r, nx, i, j, V2<double>{0.0, 0.0});
                store_node(x, nx, i, j, V2<double>{0.0, 0.0});
            }
        }
    }
    block_sum2(rr, ff);
    if (threadIdx.x == 0) {
        rr_out[t.tile] = rr;
        if (ff_out) ff_out[t.tile] = ff;
    }
}

// ===========================================================================
// Pre-smoothing from a zero iterate: u1 = w D^-1 b, then (if two sweeps)
// u2 = u1 + w D^-1 (b - K u1).  On the finest grid inside PCG (CG = true)
// the right-hand side is the residual, updated on the fly as
// r_new = r_old - alpha q (alpha = rho / p.q from the partials), stored in
// FP64 (and as an FP32 copy for an FP32 cycle), with partial ||r_new||^2.
// Geometry: H_L = 2, H_R = 1, 61 output columns per strip.  The diagonal
// stage runs one element row ahead of the force stage.
// ===========================================================================
template <typename T, bool FINE, bool CG, int R>
__global__ __launch_bounds__(WG_THREADS) void k_presmooth(
    LevelOp<T> op, Mat<T> mat, Sweep sw, const T* __restrict__ b, T* __restrict__ u_out,
    int sweeps, CgRhs cg, const int* conv, Batch bt) {
    const SysOff so = sys_off(bt);
    conv = at(conv, so.c);
    op.data = at(op.data, so.d);
    b = at(b, so.c);
    u_out = at(u_out, so.c);
    if constexpr (CG) {
        cg.r_old = at(cg.r_old, so.c);
        cg.q = at(cg.q, so.c);
        cg.r_new = at(cg.r_new, so.c);
        cg.r32 = at(cg.r32, so.c);
        cg.zr = at(cg.zr, so.c);
        cg.pq = at(cg.pq, so.c);
        cg.rr_out = at(cg.rr_out, so.c);
        cg.conv_rw = at(cg.conv_rw, so.c);
        cg.iters = at(cg.iters, so.c);
    }
    // a running system has state 0; latency-bound coarse sweeps test it
    // after issuing their loads
    const int cst = load_state(conv);
    if constexpr (CG) {
        if (cst == 1 && blockIdx.x == 0 && threadIdx.x == 0) *cg.conv_rw = 2;
    }
    if constexpr (FINE || CG) {
        if (cst != 0) return;
    }
    const int nx = op.nx, ny = op.ny;
    const TileInfo t = tile_info<R>(sw, ny + 1);
    if (!t.block_ok) return;
    constexpr int HL = 2, WOUT = 61;
    const int lane = lane_id();
    const int i = t.strip * WOUT - HL + lane;
    const bool out_lane = lane >= HL && lane < HL + WOUT && i <= nx;
    const bool node_col = i >= 0 && i <= nx;

    double rr = 0.0;
    // right-hand side rows j0-1 .. j0+R, element rows j0-2 .. j0+R
    V2<T> br[R + 2];
    Mom<T> me[R + 3];
    if constexpr (CG) {
        // the loads of the CG apply's p.q partials go out first, then the
        // tile's (every wave, rows clamped), then the block sums p.q:
        // alpha = rho / p.q, rho from its producer's total; the p.q total
        // is stored for the next CG apply
        PartialSums<1> pqs;
        if (cg.update) {
            const double* ps[1] = {cg.pq};
            const int ns[1] = {cg.n_pq};
            pqs.issue(ps, ns);
        }
        __builtin_amdgcn_sched_barrier(0);   // the partials' loads ahead of the tile's
        // q is loaded whether or not it is used (the initial cycle leaves r
        // alone): a load under a branch would be waited for at the join
        V2<double> ro[R + 2], qr[R + 2];
#pragma unroll
        for (int s = 0; s < R + 2; ++s) ro[s] = load_node(cg.r_old, nx, ny, i, t.j0 - 1 + s);
#pragma unroll
        for (int s = 0; s < R + 2; ++s) qr[s] = load_node(cg.q, nx, ny, i, t.j0 - 1 + s);
#pragma unroll
        for (int s = 0; s < R + 3; ++s) me[s] = load_elem<T, FINE>(op, i, t.j0 - 2 + s);
        __builtin_amdgcn_sched_barrier(0);
        double alpha = 0.0;
        if (cg.update) {
            const double rho = cg.zr[cg.n_zr];
            double pqv[1];
            pqs.finish(pqv);
            const double pq = pqv[0];
            if (blockIdx.x == 0 && threadIdx.x == 0) cg.pq[cg.n_pq] = pq;
            alpha = rho / pq;
            if (!(pq > 0.0) || !(rho > 0.0) || !isfinite(alpha)) {
                if (blockIdx.x == 0 && threadIdx.x == 0) *cg.conv_rw = isfinite(alpha) ? 3 : 4;
                return;
            }
            if (blockIdx.x == 0 && threadIdx.x == 0) *cg.iters += 1;
        }
        if (t.j0 < t.j1) {
#pragma unroll
            for (int s = 0; s < R + 2; ++s) {
                V2<double> rv = ro[s];
                if (cg.update) {
                    rv.x -= alpha * qr[s].x;
                    rv.y -= alpha * qr[s].y;
                }
                const int jj = t.j0 - 1 + s;
                if (out_lane && jj >= t.j0 && jj < t.j1) {
                    if (jj >= 1) {
                        if (cg.update) {
                            store_node(cg.r_new, nx, i, jj, rv);
                            rr += rv.x * rv.x + rv.y * rv.y;
                        }
                        if constexpr (sizeof(T) == 4) store_node(cg.r32, nx, i, jj, V2<float>{(float)rv.x, (float)rv.y});
                    } else {
                        if (cg.update) store_node(cg.r_new, nx, i, jj, V2<double>{0.0, 0.0});
                        if constexpr (sizeof(T) == 4) store_node(cg.r32, nx, i, jj, V2<float>{0.f, 0.f});
                    }
                }
                br[s] = V2<T>{(T)rv.x, (T)rv.y};
            }
        }
    } else {
        if (t.j0 < t.j1) {
#pragma unroll
            for (int s = 0; s < R + 2; ++s) br[s] = load_node(b, nx, ny, i, t.j0 - 1 + s);
#pragma unroll
            for (int s = 0; s < R + 3; ++s) me[s] = load_elem<T, FINE>(op, i, t.j0 - 2 + s);
            if constexpr (!FINE) {
                __builtin_amdgcn_sched_barrier(0);
                if (cst != 0) return;
            }
        }
    }
    if (t.j0 < t.j1) {
        if (t.j0 == 0 && out_lane) store_node(u_out, nx, i, 0, V2<T>{T(0), T(0)});

        V2<T> d0, d1, d2, d3;
        elem_diag<FINE>(me[0], mat, d0, d1, d2, d3);
        V2<T> dcarry = d3 + from_left(d2);
        V2<T> fcarry{T(0), T(0)};
        V2<T> u1_prev{T(0), T(0)}, u1r_prev{T(0), T(0)}, b_prev{T(0), T(0)}, wD_prev{T(0), T(0)};
#pragma unroll
        for (int s = 0; s < R + 2; ++s) {
            const int k = t.j0 - 1 + s;   // node row completed by the diagonal stage
            elem_diag<FINE>(me[s + 1], mat, d0, d1, d2, d3);
            const V2<T> D = dcarry + d0 + from_left(d1);
            dcarry = d3 + from_left(d2);
            const V2<T> bk = br[s];
            const bool kok = node_col && k >= 1 && k <= ny;
            const V2<T> wD{w_over(mat.omega, D.x), w_over(mat.omega, D.y)};   // w D^-1, reused by the second sweep
            const V2<T> u1{kok ? bk.x * wD.x : T(0), kok ? bk.y * wD.y : T(0)};
            const V2<T> u1r = from_right(u1);
            if (s >= 1) {
                // force stage for element row k-1 -> node row k-1 complete
                V2<T> f0, f1, f2, f3;
                elem_force<FINE>(me[s], mat, u1_prev, u1r_prev, u1r, u1, f0, f1, f2, f3);
                const V2<T> fs = fcarry + f0 + from_left(f1);
                fcarry = f3 + from_left(f2);
                const int jr = k - 1;
                if (jr >= t.j0 && jr < t.j1 && jr >= 1 && out_lane) {
                    V2<T> uo = sweeps == 0 ? V2<T>{T(0), T(0)} : u1_prev;
                    if (sweeps >= 2) {
                        uo.x = u1_prev.x + (b_prev.x - fs.x) * wD_prev.x;
                        uo.y = u1_prev.y + (b_prev.y - fs.y) * wD_prev.y;
                    }
                    store_node(u_out, nx, i, jr, uo);
                }
            }
            u1_prev = u1;
            u1r_prev = u1r;
            b_prev = bk;
            wD_prev = wD;
        }
    }
    if constexpr (CG) {
        if (cg.update) {
            const double s = block_sum(rr);
            if (threadIdx.x == 0) cg.rr_out[t.tile] = s;
        }
    }
}

// The outer PCG's convergence test of Algorithm 2 on the device, from the
// partials of ||r||^2 and ||f||^2 (fixed order, the same bits in every
// block): issue_check sends the partials' loads (before the caller's tile
// loads), converged_or_bad sums them; block 0 records 1 (converged) or 4
// (not finite) in the state word and every block returns whether to stop.
// All threads of the block call both.
__device__ __forceinline__ void issue_check(const ConvCheck& chk, PartialSums<2>& ps) {
    const double* p[2] = {chk.rr, chk.ff};
    const int n[2] = {chk.n_rr, chk.n_ff};
    ps.issue(p, n);
}
__device__ __forceinline__ bool converged_or_bad(const ConvCheck& chk, PartialSums<2>& ps) {
    double sv[2];
    ps.finish(sv);
    const double rr = sv[0], ff = sv[1];
    const int code = !(rr == rr) ? 4 : rr <= chk.tol2 * ff ? 1 : 0;
    if (code != 0 && blockIdx.x == 0 && threadIdx.x == 0) *chk.conv_rw = code;
    return code != 0;
}

// ===========================================================================
// Residual and restriction: rc = P^T (b - K u) onto the next coarser grid
// (full weighting: weights 1, 1/2, 1/4 from the 3x3 fine neighbourhood of
// each coarse node).  u may be null (zero iterate).  On the finest grid
// inside PCG this kernel also takes the convergence decision from the
// partial ||r||^2 and ||f||^2 (CHECK = true).
// Geometry: H_L = 2, 60 fine columns (30 coarse) per strip; the chunk is in
// coarse rows.
// ===========================================================================
// Residual restriction rc = P^T (b - K u) of one wave's tile: coarse rows
// j0 .. j1-1 (j0 < j1) of strip `strip` (60 fine columns; even lanes own
// the coarse columns).  store(I, J, v) receives every coarse node of the
// tile (J = 0, the clamped row, with v = 0); a wave with j0 >= j1 loads
// (clamped rows) and stores nothing.  pre() runs before the loads and
// abort() once they are issued, by every wave of the block: the wave
// returns if abort() says so (the caller overlaps the state read or the
// convergence test with the loads).
template <typename T, bool FINE, int R, typename Pre, typename Abort, typename Store>
__device__ __forceinline__ void restrict_tile(const LevelOp<T>& op, const Mat<T>& mat, int strip, int j0, int j1,
                                              const T* __restrict__ b, const T* __restrict__ u, Pre pre,
                                              Abort abort, Store store) {
    const int nx = op.nx, ny = op.ny;
    const int ncx = nx / 2;
    constexpr int HL = 2, WOUT = 60;
    const int lane = lane_id();
    const int i = strip * WOUT - HL + lane;   // even lanes <-> even fine columns
    const int I = i >> 1;
    const bool out_lane = lane >= HL && lane < HL + WOUT && !(lane & 1) && I <= ncx;
    const bool node_col = i >= 0 && i <= nx;
    constexpr int NF = 2 * R + 1;              // fine rows jf0 .. jf0 + 2R
    const int jf0 = 2 * j0 - 1;
    V2<T> ur[NF + 2], br[NF];
    Mom<T> me[NF + 1];
    const T* uu = u ? u : b;   // u == null reads zeros, without a branch
    pre();
    __builtin_amdgcn_sched_barrier(0);   // pre()'s loads ahead of the tile's
#pragma unroll
    for (int s = 0; s < NF + 2; ++s) ur[s] = load_node(uu, nx, ny, i, jf0 - 1 + s, u != nullptr);
#pragma unroll
    for (int s = 0; s < NF; ++s) br[s] = load_node(b, nx, ny, i, jf0 + s);
#pragma unroll
    for (int s = 0; s < NF + 1; ++s) me[s] = load_elem<T, FINE>(op, i, jf0 - 1 + s);
    __builtin_amdgcn_sched_barrier(0);   // one batch of loads ahead of abort()
    if (abort()) return;
    V2<T> f0, f1, f2, f3;
    V2<T> ur_lo = from_right(ur[0]), ur_hi = from_right(ur[1]);
    elem_force<FINE>(me[0], mat, ur[0], ur_lo, ur_hi, ur[1], f0, f1, f2, f3);
    V2<T> carry = f3 + from_left(f2);
    V2<T> h_m2{T(0), T(0)}, h_m1{T(0), T(0)};
#pragma unroll
    for (int s = 0; s < NF; ++s) {
        const int j = jf0 + s;
        ur_lo = ur_hi;
        ur_hi = from_right(ur[s + 2]);
        elem_force<FINE>(me[s + 1], mat, ur[s + 1], ur_lo, ur_hi, ur[s + 2], f0, f1, f2, f3);
        const V2<T> ku = carry + f0 + from_left(f1);
        carry = f3 + from_left(f2);
        const bool jok = node_col && j >= 1 && j <= ny;
        const V2<T> rr{jok ? br[s].x - ku.x : T(0), jok ? br[s].y - ku.y : T(0)};
        const V2<T> rl = from_left(rr), rrt = from_right(rr);
        const V2<T> h{rr.x + T(0.5) * (rl.x + rrt.x), rr.y + T(0.5) * (rl.y + rrt.y)};
        if ((s & 1) == 0 && s >= 2) {
            const int J = (j - 1) >> 1;
            if (out_lane && J < j1) {
                V2<T> v{h_m1.x + T(0.5) * (h_m2.x + h.x), h_m1.y + T(0.5) * (h_m2.y + h.y)};
                if (J == 0) v = V2<T>{T(0), T(0)};
                store(I, J, v);
            }
        }
        h_m2 = h_m1;
        h_m1 = h;
    }
}

template <typename T, bool FINE, bool CHECK, int R>
__global__ __launch_bounds__(WG_THREADS) void k_restrict(
    LevelOp<T> op, Mat<T> mat, Sweep sw, const T* __restrict__ b, const T* __restrict__ u,
    T* __restrict__ rc, ConvCheck chk, const int* conv, Batch bt) {
    const SysOff so = sys_off(bt);
    conv = at(conv, so.c);
    op.data = at(op.data, so.d);
    b = at(b, so.c);
    u = at(u, so.c);
    rc = at(rc, so.c);
    if constexpr (CHECK) {
        chk.rr = at(chk.rr, so.c);
        chk.ff = at(chk.ff, so.c);
        chk.conv_rw = at(chk.conv_rw, so.c);
    }
    const int cst = load_state(conv);   // coarse levels test it after issuing their loads
    if constexpr (FINE || CHECK) {
        if (cst != 0) return;
    }
    const int nx = op.nx, ny = op.ny;
    const int ncx = nx / 2, ncy = ny / 2;
    const TileInfo t = tile_info<R>(sw, ncy + 1);
    if (!t.block_ok) return;
    // with CHECK every wave runs the tile's loads and the block-wide test
    if constexpr (!CHECK) {
        if (t.j0 >= t.j1) return;
    }
    PartialSums<2> cps;
    restrict_tile<T, FINE, R>(op, mat, t.strip, t.j0, t.j1, b, u,
                              [&]() {
                                  if constexpr (CHECK) issue_check(chk, cps);
                              },
                              [&]() {
                                  if constexpr (CHECK) return converged_or_bad(chk, cps);
                                  else return !FINE && cst != 0;
                              },
                              [&](int I, int J, const V2<T>& v) { store_node(rc, ncx, I, J, v); });
}

// ===========================================================================
// Restriction to level l-1 fused with the pre-smoothing there.  Phase A
// (lanes = fine columns) forms rc = P^T (b - K u) for the chunk's coarse
// rows J0-1 .. J0+R, exactly as k_restrict; phase B (lanes 0..31 = coarse
// columns) takes them through LDS and runs the first `sweeps` (1 or 2)
// damped-Jacobi sweeps from zero on level l-1, as k_presmooth.  rc is
// stored as well (the post-smoother of level l-1 reads it).  With CHECK the
// convergence test of k_restrict comes first.
// Geometry: a wave covers 64 fine = 32 coarse columns; phase A's rc is
// valid on coarse lanes 1..30, so the smoothed values are valid and owned
// on coarse lanes 2..29 (28 coarse columns per strip).
// ===========================================================================
template <typename T, bool FINE, bool CHECK, int R>
__global__ __launch_bounds__(WG_THREADS) void k_restrict_pre(
    LevelOp<T> op, LevelOp<T> opc, Mat<T> mat, Sweep sw, const T* __restrict__ b, const T* __restrict__ u,
    T* __restrict__ rc, T* __restrict__ uc, int sweeps, ConvCheck chk, const int* conv, Batch bt) {
    constexpr int RA = R + 2;                  // coarse rows formed in phase A
    __shared__ V2<T> cbuf[WAVES_PER_WG][RA][32];
    const SysOff so = sys_off(bt);
    conv = at(conv, so.c);
    op.data = at(op.data, so.d);
    opc.data = at(opc.data, so.d);
    b = at(b, so.c);
    u = at(u, so.c);
    rc = at(rc, so.c);
    uc = at(uc, so.c);
    if constexpr (CHECK) {
        chk.rr = at(chk.rr, so.c);
        chk.ff = at(chk.ff, so.c);
        chk.conv_rw = at(chk.conv_rw, so.c);
    }
    const int cst = load_state(conv);   // coarse levels test it after issuing their loads
    if constexpr (FINE || CHECK) {
        if (cst != 0) return;
    }
    const int nx = op.nx, ny = op.ny;
    const int ncx = opc.nx, ncy = opc.ny;
    const TileInfo t = tile_info<R>(sw, ncy + 1);
    if (!t.block_ok) return;
    // with CHECK every wave runs phase A's loads and the block-wide test (a
    // wave without rows stores nothing)
    if constexpr (!CHECK) {
        if (t.j0 >= t.j1) return;
    }
    constexpr int CHL = 2, CWOUT = 28;
    const int lane = lane_id();
    const int Ib = t.strip * CWOUT - CHL;      // coarse column of coarse lane 0
    V2<T>(*cb)[32] = cbuf[wave_id()];
    // coarse lane c = lane & 31 <-> coarse column Ib + c (phase B)
    const int cl = lane & 31;
    const int ic = Ib + cl;
    // phase B's coarse element rows j0-2 .. j0+R, loaded with phase A's data
    Mom<T> mc[R + 3];
    PartialSums<2> cps;   // the convergence test's partials (CHECK)

    // ---- phase A: fine lane l <-> fine column 2 Ib + l
    {
        const int i = 2 * Ib + lane;
        const bool node_col = i >= 0 && i <= nx;
        constexpr int NF = 2 * RA + 1;         // fine rows jf0 .. jf0 + 2 RA
        const int jf0 = 2 * (t.j0 - 1) - 1;
        V2<T> ur[NF + 2], br[NF];
        Mom<T> me[NF + 1];
        const T* uu = u ? u : b;   // u == null reads zeros, without a branch
        if constexpr (CHECK) issue_check(chk, cps);
        __builtin_amdgcn_sched_barrier(0);   // the partials' loads ahead of the tile's
#pragma unroll
        for (int s = 0; s < NF + 2; ++s) ur[s] = load_node(uu, nx, ny, i, jf0 - 1 + s, u != nullptr);
#pragma unroll
        for (int s = 0; s < NF; ++s) br[s] = load_node(b, nx, ny, i, jf0 + s);
#pragma unroll
        for (int s = 0; s < NF + 1; ++s) me[s] = load_elem<T, FINE>(op, i, jf0 - 1 + s);
#pragma unroll
        for (int s = 0; s < R + 3; ++s) mc[s] = load_elem<T, false>(opc, ic, t.j0 - 2 + s);
        __builtin_amdgcn_sched_barrier(0);   // one batch of loads ahead of the tests
        if constexpr (CHECK) {
            if (converged_or_bad(chk, cps)) return;
        } else if constexpr (!FINE) {
            if (cst != 0) return;
        }
        V2<T> f0, f1, f2, f3;
        V2<T> ur_lo = from_right(ur[0]), ur_hi = from_right(ur[1]);
        elem_force<FINE>(me[0], mat, ur[0], ur_lo, ur_hi, ur[1], f0, f1, f2, f3);
        V2<T> carry = f3 + from_left(f2);
        V2<T> h_m2{T(0), T(0)}, h_m1{T(0), T(0)};
#pragma unroll
        for (int s = 0; s < NF; ++s) {
            const int j = jf0 + s;
            ur_lo = ur_hi;
            ur_hi = from_right(ur[s + 2]);
            elem_force<FINE>(me[s + 1], mat, ur[s + 1], ur_lo, ur_hi, ur[s + 2], f0, f1, f2, f3);
            const V2<T> ku = carry + f0 + from_left(f1);
            carry = f3 + from_left(f2);
            const bool jok = node_col && j >= 1 && j <= ny;
            const V2<T> rr{jok ? br[s].x - ku.x : T(0), jok ? br[s].y - ku.y : T(0)};
            const V2<T> rl = from_left(rr), rrt = from_right(rr);
            const V2<T> h{rr.x + T(0.5) * (rl.x + rrt.x), rr.y + T(0.5) * (rl.y + rrt.y)};
            if ((s & 1) == 0 && s >= 2) {
                // coarse row J = J0 - 1 + (s - 2) / 2
                const int J = (j - 1) >> 1;
                V2<T> v{h_m1.x + T(0.5) * (h_m2.x + h.x), h_m1.y + T(0.5) * (h_m2.y + h.y)};
                if (J <= 0) v = V2<T>{T(0), T(0)};
                if (!(lane & 1)) cb[(s - 2) >> 1][lane >> 1] = v;
            }
            h_m2 = h_m1;
            h_m1 = h;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    // ---- phase B: lane c < 32 <-> coarse column Ib + c (lanes 32..63 mirror them, unused)
    const int i = ic;
    const bool node_col = lane < 32 && i >= 0 && i <= ncx;
    const bool out_lane = lane >= CHL && lane < CHL + CWOUT && i <= ncx;
    V2<T> br[R + 2];
    const Mom<T>* me = mc;
#pragma unroll
    for (int s = 0; s < R + 2; ++s) br[s] = cb[s][cl];   // coarse rows j0-1 .. j0+R
#pragma unroll
    for (int s = 1; s <= R; ++s) {
        const int jj = t.j0 - 1 + s;
        if (out_lane && jj < t.j1) store_node(rc, ncx, i, jj, br[s]);
    }
    if (t.j0 == 0 && out_lane) store_node(uc, ncx, i, 0, V2<T>{T(0), T(0)});
    V2<T> d0, d1, d2, d3;
    elem_diag(me[0], mat, d0, d1, d2, d3);
    V2<T> dcarry = d3 + from_left(d2);
    V2<T> fcarry{T(0), T(0)};
    V2<T> u1_prev{T(0), T(0)}, u1r_prev{T(0), T(0)}, b_prev{T(0), T(0)}, wD_prev{T(0), T(0)};
#pragma unroll
    for (int s = 0; s < R + 2; ++s) {
        const int k = t.j0 - 1 + s;   // coarse node row completed by the diagonal stage
        elem_diag(me[s + 1], mat, d0, d1, d2, d3);
        const V2<T> D = dcarry + d0 + from_left(d1);
        dcarry = d3 + from_left(d2);
        const V2<T> bk = br[s];
        const bool kok = node_col && k >= 1 && k <= ncy;
        const V2<T> wD{w_over(mat.omega, D.x), w_over(mat.omega, D.y)};   // w D^-1, reused by the second sweep
        const V2<T> u1{kok ? bk.x * wD.x : T(0), kok ? bk.y * wD.y : T(0)};
        const V2<T> u1r = from_right(u1);
        if (s >= 1) {
            V2<T> f0, f1, f2, f3;
            elem_force(me[s], mat, u1_prev, u1r_prev, u1r, u1, f0, f1, f2, f3);
            const V2<T> fs = fcarry + f0 + from_left(f1);
            fcarry = f3 + from_left(f2);
            const int jr = k - 1;
            if (jr >= t.j0 && jr < t.j1 && jr >= 1 && out_lane) {
                V2<T> uo = u1_prev;
                if (sweeps >= 2) {
                    uo.x = u1_prev.x + (b_prev.x - fs.x) * wD_prev.x;
                    uo.y = u1_prev.y + (b_prev.y - fs.y) * wD_prev.y;
                }
                store_node(uc, ncx, i, jr, uo);
            }
        }
        u1_prev = u1;
        u1r_prev = u1r;
        b_prev = bk;
        wD_prev = wD;
    }
}

// Coarse-correction rows for the prolongation onto fine rows j0-1 .. j0+R:
// coarse rows (j0 >> 1) - 1 .. + NC - 1 at coarse columns I0 and I1 (the
// same rows for either parity of j0).
template <typename T, int R>
__device__ __forceinline__ void load_prolongation(V2<T>* c0, V2<T>* c1, const T* __restrict__ ec, int ncx,
                                                  int ncy, int I0, int I1, int j0) {
    constexpr int NC = R / 2 + 3;
    const int Jb = (j0 >> 1) - 1;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        c0[k] = load_node(ec, ncx, ncy, I0, Jb + k);
        c1[k] = load_node(ec, ncx, ncy, I1, Jb + k);
    }
}

// v(i, jj) += (P e_c)(i, jj) for the fine rows jj = j0-1 .. j0+R of one
// lane (bilinear weights; nodes off the grid or on the clamped row get 0),
// from the coarse rows of load_prolongation.  With PAR = parity of j0 the
// coarse row below/above fine row j0-1+s is at offset ((PAR-1+s)>>1)+1 /
// ((PAR+s)>>1)+1, both compile-time constants.
template <typename T, int R, int PAR>
__device__ __forceinline__ void add_prolongation(V2<T>* vr, const V2<T>* c0, const V2<T>* c1, int j0,
                                                 bool node_col, int ny) {
#pragma unroll
    for (int s = 0; s < R + 2; ++s) {
        const int k0 = ((PAR - 1 + s) >> 1) + 1, k1 = ((PAR + s) >> 1) + 1;
        const int jj = j0 - 1 + s;
        const bool ok = node_col && jj >= 1 && jj <= ny;
        const T w = ok ? T(0.25) : T(0);
        vr[s].x += w * ((c0[k0].x + c1[k0].x) + (c0[k1].x + c1[k1].x));
        vr[s].y += w * ((c0[k0].y + c1[k0].y) + (c0[k1].y + c1[k1].y));
    }
}

// ===========================================================================
// Post-smoothing sweep: u_out = v + w D^-1 (b - K v), where
// v = u_in + P e_c when PROLONG (bilinear prolongation of the coarse
// correction, then the correction step of Algorithm 1), else v = u_in.
// With DOT (finest grid inside PCG) also partial sums of u_out . r over the
// free DOFs, r being the FP64 residual.
// Geometry: H_L = 1, H_R = 1, 62 output columns per strip.
// ===========================================================================
template <typename T, bool FINE, bool PROLONG, bool DOT, int R>
__global__ __launch_bounds__(WG_THREADS) void k_post(
    LevelOp<T> op, Mat<T> mat, Sweep sw, const T* __restrict__ u_in, const T* __restrict__ ec,
    const T* __restrict__ b, T* __restrict__ u_out, const double* __restrict__ r64,
    double* __restrict__ zr_out, const int* conv, Batch bt) {
    const SysOff so = sys_off(bt);
    conv = at(conv, so.c);
    op.data = at(op.data, so.d);
    u_in = at(u_in, so.c);
    ec = at(ec, so.c);
    b = at(b, so.c);
    u_out = at(u_out, so.c);
    r64 = at(r64, so.c);
    zr_out = at(zr_out, so.c);
    if (load_state(conv) != 0) return;
    const int nx = op.nx, ny = op.ny;
    const int ncx = nx / 2, ncy = ny / 2;
    const TileInfo t = tile_info<R>(sw, ny + 1);
    if (!t.block_ok) return;
    constexpr int HL = 1, WOUT = 62;
    const int lane = lane_id();
    const int i = t.strip * WOUT - HL + lane;
    const bool out_lane = lane >= HL && lane < HL + WOUT && i <= nx;
    const bool node_col = i >= 0 && i <= nx;
    const int I0 = i >> 1, I1 = (i + 1) >> 1;
    double dot = 0.0;
    if (t.j0 < t.j1) {
        // v rows j0-1 .. j0+R, element rows j0-1 .. j0+R-1, b (and r) rows j0 .. j0+R-1
        V2<T> vr[R + 2], br[R];
        Mom<T> me[R + 1];
        V2<double> rr64[DOT ? R : 1];
        constexpr int NC = PROLONG ? R / 2 + 3 : 1;
        V2<T> c0[NC], c1[NC];
        // all loads first, none inside a branch (u_in == null reads zeros)
        const T* uin = u_in ? u_in : b;
#pragma unroll
        for (int s = 0; s < R + 2; ++s) vr[s] = load_node(uin, nx, ny, i, t.j0 - 1 + s, u_in != nullptr);
        if constexpr (PROLONG) load_prolongation<T, R>(c0, c1, ec, ncx, ncy, I0, I1, t.j0);
#pragma unroll
        for (int s = 0; s < R; ++s) br[s] = load_node(b, nx, ny, i, t.j0 + s);
        if constexpr (DOT) {
#pragma unroll
            for (int s = 0; s < R; ++s) rr64[s] = load_node(r64, nx, ny, i, t.j0 + s);
        }
#pragma unroll
        for (int s = 0; s < R + 1; ++s) me[s] = load_elem<T, FINE>(op, i, t.j0 - 1 + s);
        if constexpr (!FINE) __builtin_amdgcn_sched_barrier(0);   // latency-bound: one batch of loads
        if constexpr (PROLONG) {
            // the parity of j0 is uniform over the wave: one branch, then
            // compile-time indices into the coarse rows held in registers
            if (t.j0 & 1) add_prolongation<T, R, 1>(vr, c0, c1, t.j0, node_col, ny);
            else add_prolongation<T, R, 0>(vr, c0, c1, t.j0, node_col, ny);
        }

        V2<T> f0, f1, f2, f3, d0, d1, d2, d3;
        V2<T> vr_lo = from_right(vr[0]), vr_hi = from_right(vr[1]);
        elem_force<FINE>(me[0], mat, vr[0], vr_lo, vr_hi, vr[1], f0, f1, f2, f3);
        elem_diag<FINE>(me[0], mat, d0, d1, d2, d3);
        V2<T> fcarry = f3 + from_left(f2);
        V2<T> dcarry = d3 + from_left(d2);
#pragma unroll
        for (int s = 0; s < R; ++s) {
            const int j = t.j0 + s;
            vr_lo = vr_hi;
            vr_hi = from_right(vr[s + 2]);
            elem_force<FINE>(me[s + 1], mat, vr[s + 1], vr_lo, vr_hi, vr[s + 2], f0, f1, f2, f3);
            elem_diag<FINE>(me[s + 1], mat, d0, d1, d2, d3);
            const V2<T> fs = fcarry + f0 + from_left(f1);
            const V2<T> D = dcarry + d0 + from_left(d1);
            fcarry = f3 + from_left(f2);
            dcarry = d3 + from_left(d2);
            if (out_lane && j < t.j1) {
                if (j >= 1) {
                    V2<T> uo;
                    uo.x = vr[s + 1].x + (br[s].x - fs.x) * w_over(mat.omega, D.x);
                    uo.y = vr[s + 1].y + (br[s].y - fs.y) * w_over(mat.omega, D.y);
                    store_node(u_out, nx, i, j, uo);
                    if constexpr (DOT) dot += (double)uo.x * rr64[s].x + (double)uo.y * rr64[s].y;
                } else {
                    store_node(u_out, nx, i, j, V2<T>{T(0), T(0)});
                }
            }
        }
    }
    if constexpr (DOT) {
        const double s = block_sum(dot);
        if (threadIdx.x == 0) zr_out[t.tile] = s;
    }
}

// ===========================================================================
// Two pre-smoothing sweeps from zero and the restriction of the residual
// they leave, in one pass: u1 = w D^-1 b, u2 = u1 + w D^-1 (b - K u1),
// rc = P^T (b - K u2).  u2 is stored (the post-smoother starts from it);
// u1 and the residual stay in registers.  With CG (finest grid inside PCG)
// b is the outer residual updated on the fly, r_new = r_old - alpha q, as
// in k_presmooth (r_new, its FP32 copy and partial ||r_new||^2 stored).
// With CHECK the outer PCG's convergence test on the partials of
// ||r||^2 (from the finest grid's launch) comes first, overlapped with the
// tile's loads.  Per node the operations and their order are those of
// k_presmooth followed by k_restrict (the two agree to rounding: the
// compiler contracts multiply-adds differently in each kernel).
// Geometry: lane l <-> node column i = 56 strip - 4 + l.  A wave owns the
// coarse rows j0 .. j1-1 and the coarse columns 28 strip .. 28 strip + 27,
// i.e. the fine columns 56 strip .. 56 strip + 55 (lanes 4..59) and fine
// rows 2 j0 .. 2 j1 - 1, and marches over the node rows 2 j0 - 3 ..
// 2 j0 + 2R + 1 (NS = 2R + 5): the diagonal, hence u1, is valid on lanes
// 1..63 (lane 0 lacks its left element), u2 on 2..62, the residual on
// 3..61 and its horizontal full weighting on 4..60.  Step s forms u1 on
// node row k = 2 j0 - 3 + s, u2 on row k-1 and the residual on row k-2;
// the coarse row (k-3)/2 is complete when k-2 is odd.
// ===========================================================================
template <typename T, bool FINE, bool CG, bool CHECK, int R>
__global__ __launch_bounds__(WG_THREADS) void k_pre_restrict(
    LevelOp<T> op, Mat<T> mat, Sweep sw, const T* __restrict__ b, T* __restrict__ u_out, T* __restrict__ rc,
    CgRhs cg, ConvCheck chk, const int* conv, Batch bt) {
    constexpr int NS = 2 * R + 5;
    const SysOff so = sys_off(bt);
    conv = at(conv, so.c);
    op.data = at(op.data, so.d);
    b = at(b, so.c);
    u_out = at(u_out, so.c);
    rc = at(rc, so.c);
    if constexpr (CG) {
        cg.r_old = at(cg.r_old, so.c);
        cg.q = at(cg.q, so.c);
        cg.r_new = at(cg.r_new, so.c);
        cg.r32 = at(cg.r32, so.c);
        cg.zr = at(cg.zr, so.c);
        cg.pq = at(cg.pq, so.c);
        cg.rr_out = at(cg.rr_out, so.c);
        cg.conv_rw = at(cg.conv_rw, so.c);
        cg.iters = at(cg.iters, so.c);
    }
    if constexpr (CHECK) {
        chk.rr = at(chk.rr, so.c);
        chk.ff = at(chk.ff, so.c);
        chk.conv_rw = at(chk.conv_rw, so.c);
    }
    const int cst = load_state(conv);
    if constexpr (CG) {
        if (cst == 1 && blockIdx.x == 0 && threadIdx.x == 0) *cg.conv_rw = 2;
    }
    if constexpr (FINE || CG || CHECK) {
        if (cst != 0) return;
    }
    const int nx = op.nx, ny = op.ny;
    const int ncx = nx / 2, ncy = ny / 2;
    const TileInfo t = tile_info<R>(sw, ncy + 1);
    if (!t.block_ok) return;
    // a wave without rows (t.j0 >= t.j1) runs along and stores nothing: the
    // block-wide sums need every wave
    constexpr int HL = 4, WOUT = 56;
    const int lane = lane_id();
    const int i = t.strip * WOUT - HL + lane;
    const bool node_col = i >= 0 && i <= nx;
    const bool own_col = lane >= HL && lane < HL + WOUT && i <= nx;
    const bool out_lane = own_col && !(i & 1);   // even fine column 2I <-> coarse column I
    const int I = i >> 1;
    const int base = 2 * t.j0 - 3;               // node row of step 0
    const int fr0 = 2 * t.j0, fr1 = min(2 * t.j1 - 1, ny);   // owned fine rows

    PartialSums<1> pqs;
    PartialSums<2> cps;
    if constexpr (CG) {
        if (cg.update) {
            const double* ps[1] = {cg.pq};
            const int ns[1] = {cg.n_pq};
            pqs.issue(ps, ns);
        }
    }
    if constexpr (CHECK) issue_check(chk, cps);
    __builtin_amdgcn_sched_barrier(0);   // the partials' loads ahead of the tile's
    // right-hand side rows base .. base+NS-1, element rows base-1 .. base+NS-1
    // loads in the order the march uses them (row s: its right-hand side and
    // the element row above it), so the first steps can start while the
    // later rows are still arriving (loads complete in order)
    V2<T> br[NS];
    Mom<T> me[NS + 1];
    V2<double> ro[CG ? NS : 1], qr[CG ? NS : 1];
    // (right-hand-side values off the grid are never used unselected: u1,
    // u2 and the residual are selected by their node's validity, r_new is
    // stored on owned grid nodes only; so they load unmasked)
    me[0] = load_elem<T, FINE>(op, i, base - 1);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        if constexpr (CG) {
            // q is loaded whether or not it is used, as in k_presmooth
            ro[s] = load_node_clamped(cg.r_old, nx, ny, i, base + s);
            qr[s] = load_node_clamped(cg.q, nx, ny, i, base + s);
        } else {
            br[s] = load_node_clamped(b, nx, ny, i, base + s);
        }
        me[s + 1] = load_elem<T, FINE>(op, i, base + s);
    }
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (CHECK) {
        if (converged_or_bad(chk, cps)) return;
    } else if constexpr (!FINE && !CG) {
        if (cst != 0) return;
    }

    double rr = 0.0;
    double alpha = 0.0;
    if constexpr (CG) {
        if (cg.update) {
            const double rho = cg.zr[cg.n_zr];
            double pqv[1];
            pqs.finish(pqv);
            const double pq = pqv[0];
            if (blockIdx.x == 0 && threadIdx.x == 0) cg.pq[cg.n_pq] = pq;
            alpha = rho / pq;
            if (!(pq > 0.0) || !(rho > 0.0) || !isfinite(alpha)) {
                if (blockIdx.x == 0 && threadIdx.x == 0) *cg.conv_rw = isfinite(alpha) ? 3 : 4;
                return;
            }
            if (blockIdx.x == 0 && threadIdx.x == 0) *cg.iters += 1;
        }
    }
    // CG: r_new = r_old - alpha q on row s (stored on owned rows), b = its FP32 value
    auto cg_row = [&](int s) {
        if constexpr (CG) {
            V2<double> rv = ro[s];
            if (cg.update) {
                rv.x -= alpha * qr[s].x;
                rv.y -= alpha * qr[s].y;
            }
            const int jj = base + s;
            if (own_col && jj >= fr0 && jj <= fr1) {
                if (jj >= 1) {
                    if (cg.update) {
                        store_node(cg.r_new, nx, i, jj, rv);
                        rr += rv.x * rv.x + rv.y * rv.y;
                    }
                    if constexpr (sizeof(T) == 4) store_node(cg.r32, nx, i, jj, V2<float>{(float)rv.x, (float)rv.y});
                } else {
                    if (cg.update) store_node(cg.r_new, nx, i, jj, V2<double>{0.0, 0.0});
                    if constexpr (sizeof(T) == 4) store_node(cg.r32, nx, i, jj, V2<float>{0.f, 0.f});
                }
            }
            br[s] = V2<T>{(T)rv.x, (T)rv.y};
        }
    };

    // The march.  Step s forms u1 on node row base+s (stage A), u2 on row
    // base+s-2 from u1 of earlier steps (stage B) and the residual on row
    // base+s-4 from u2 of earlier steps (stage C): the three stages of a
    // step do not depend on each other, so their instruction chains
    // interleave.  Per-row values live in arrays indexed by the unrolled s.
    V2<T> d0, d1, d2, d3;
    elem_diag<FINE>(me[0], mat, d0, d1, d2, d3);
    V2<T> dcarry = d3 + from_left(d2);
    V2<T> fcarry{T(0), T(0)}, gcarry{T(0), T(0)};
    V2<T> u1[NS], u1r[NS], wD[NS], u2[NS], u2r[NS];
    bool kok[NS];
    V2<T> h_m1{T(0), T(0)}, h_m2{T(0), T(0)};
#pragma unroll
    for (int s = 0; s < NS + 2; ++s) {
        if (s < NS) {
            // stage A: the diagonal of node row base+s (element rows base+s-1,
            // base+s) and u1 there
            cg_row(s);
            const int k = base + s;
            elem_diag<FINE>(me[s + 1], mat, d0, d1, d2, d3);
            const V2<T> D = dcarry + d0 + from_left(d1);
            dcarry = d3 + from_left(d2);
            kok[s] = node_col && k >= 1 && k <= ny;
            wD[s] = V2<T>{w_over(mat.omega, D.x), w_over(mat.omega, D.y)};   // w D^-1, reused by the second sweep
            u1[s] = V2<T>{kok[s] ? br[s].x * wD[s].x : T(0), kok[s] ? br[s].y * wD[s].y : T(0)};
            u1r[s] = from_right(u1[s]);
        }
        if (s >= 2 && s <= NS) {
            // stage B: element row base+q (q = s-2) on u1 rows q, q+1 completes
            // K u1 at node row base+q -> u2 there
            const int q = s - 2;
            V2<T> f0, f1, f2, f3;
            elem_force<FINE>(me[q + 1], mat, u1[q], u1r[q], u1r[q + 1], u1[q + 1], f0, f1, f2, f3);
            const V2<T> fs = fcarry + f0 + from_left(f1);
            fcarry = f3 + from_left(f2);
            const int jr = base + q;
            u2[q] = V2<T>{kok[q] ? u1[q].x + (br[q].x - fs.x) * wD[q].x : T(0),
                          kok[q] ? u1[q].y + (br[q].y - fs.y) * wD[q].y : T(0)};
            if (own_col && jr >= fr0 && jr <= fr1) store_node(u_out, nx, i, jr, u2[q]);
            u2r[q] = from_right(u2[q]);
        }
        if (s >= 4) {
            // stage C: element row base+p (p = s-4) on u2 rows p, p+1 completes
            // K u2 at node row j = base+p -> residual
            const int p = s - 4;
            V2<T> g0, g1, g2, g3;
            elem_force<FINE>(me[p + 1], mat, u2[p], u2r[p], u2r[p + 1], u2[p + 1], g0, g1, g2, g3);
            const V2<T> ku = gcarry + g0 + from_left(g1);
            gcarry = g3 + from_left(g2);
            const int j = base + p;
            const bool jok = node_col && j >= 1 && j <= ny;
            const V2<T> res{jok ? br[p].x - ku.x : T(0), jok ? br[p].y - ku.y : T(0)};
            const V2<T> rl = from_left(res), rrt = from_right(res);
            const V2<T> h{res.x + T(0.5) * (rl.x + rrt.x), res.y + T(0.5) * (rl.y + rrt.y)};
            // stage D: j = 2J + 1 (p even) completes coarse row J from fine rows 2J-1 .. 2J+1
            if ((p & 1) == 0 && p >= 4) {
                const int J = t.j0 - 2 + p / 2;
                if (out_lane && J < t.j1) {
                    V2<T> v{h_m1.x + T(0.5) * (h_m2.x + h.x), h_m1.y + T(0.5) * (h_m2.y + h.y)};
                    if (J == 0) v = V2<T>{T(0), T(0)};
                    store_node(rc, ncx, I, J, v);
                }
            }
            h_m2 = h_m1;
            h_m1 = h;
        }
    }
    if constexpr (CG) {
        if (cg.update) {
            const double s = block_sum(rr);
            if (threadIdx.x == 0) cg.rr_out[t.tile] = s;
        }
    }
}

// The two stages of the paired post-smoother on one wave's rows j0 ..
// j0+RR-1 (lanes = node columns of the level): v rows j0-2 .. j0+RR+1 (the
// prolonged iterate), b rows j0-1 .. j0+RR, element rows j0-2 .. j0+RR.
// out(jr, u) receives row jr = j0 .. j0+RR-1 of u = S(S(v)) (S: one damped
// Jacobi sweep); it is meaningful on lanes with both neighbours in the
// wave, for grid nodes off the clamped row.
template <typename T, bool FINE, int RR, typename Out>
__device__ __forceinline__ void post2_stages(const Mat<T>& mat, const V2<T>* vr, const V2<T>* br, const Mom<T>* me,
                                             int j0, bool node_col, int ny, Out out) {
    V2<T> f0, f1, f2, f3, d0, d1, d2, d3;
    V2<T> vlo = from_right(vr[0]), vhi = from_right(vr[1]);
    elem_force<FINE>(me[0], mat, vr[0], vlo, vhi, vr[1], f0, f1, f2, f3);
    elem_diag<FINE>(me[0], mat, d0, d1, d2, d3);
    V2<T> fc1 = f3 + from_left(f2), dc1 = d3 + from_left(d2);
    V2<T> fc2{T(0), T(0)};
    V2<T> u1_prev{T(0), T(0)}, u1r_prev{T(0), T(0)}, wD_prev{T(0), T(0)};
#pragma unroll
    for (int s = 1; s < RR + 3; ++s) {
        // stage 1: element row j0-2+s completes node row k = j0-2+s
        const int k = j0 - 2 + s;
        vlo = vhi;
        vhi = from_right(vr[s + 1]);
        elem_force<FINE>(me[s], mat, vr[s], vlo, vhi, vr[s + 1], f0, f1, f2, f3);
        elem_diag<FINE>(me[s], mat, d0, d1, d2, d3);
        const V2<T> F = fc1 + f0 + from_left(f1);
        const V2<T> D = dc1 + d0 + from_left(d1);
        fc1 = f3 + from_left(f2);
        dc1 = d3 + from_left(d2);
        const bool kok = node_col && k >= 1 && k <= ny;
        const V2<T> bk = br[s - 1];
        const V2<T> wD{w_over(mat.omega, D.x), w_over(mat.omega, D.y)};   // w D^-1, reused by the second stage
        const V2<T> u1{kok ? vr[s].x + (bk.x - F.x) * wD.x : T(0),
                       kok ? vr[s].y + (bk.y - F.y) * wD.y : T(0)};
        const V2<T> u1r = from_right(u1);
        if (s >= 2) {
            // stage 2: element row k-1 from u1 rows k-1, k completes node row k-1
            V2<T> g0, g1, g2, g3;
            elem_force<FINE>(me[s - 1], mat, u1_prev, u1r_prev, u1r, u1, g0, g1, g2, g3);
            const V2<T> G = fc2 + g0 + from_left(g1);
            fc2 = g3 + from_left(g2);
            if (s >= 3) {
                const V2<T> bj = br[s - 2];
                V2<T> uo;
                uo.x = u1_prev.x + (bj.x - G.x) * wD_prev.x;
                uo.y = u1_prev.y + (bj.y - G.y) * wD_prev.y;
                out(k - 1, s - 3, uo);
            }
        }
        u1_prev = u1;
        u1r_prev = u1r;
        wD_prev = wD;
    }
}

// ===========================================================================
// Two post-smoothing sweeps in one pass: u1 = v + w D^-1 (b - K v) and
// u_out = u1 + w D^-1 (b - K u1), with v = u_in + P e_c when PROLONG.
// The second stage marches one element row behind the first, so u1 never
// leaves registers.  With DOT, partial sums of u_out . r over the free DOFs.
// Geometry: H_L = 2, H_R = 2, 60 output columns per strip.
// ===========================================================================
template <typename T, bool FINE, bool PROLONG, bool DOT, int R>
__global__ __launch_bounds__(WG_THREADS) void k_post2(
    LevelOp<T> op, Mat<T> mat, Sweep sw, const T* __restrict__ u_in, const T* __restrict__ ec,
    const T* __restrict__ b, T* __restrict__ u_out, const double* __restrict__ r64,
    double* __restrict__ zr_out, const int* conv, Batch bt) {
    const SysOff so = sys_off(bt);
    conv = at(conv, so.c);
    op.data = at(op.data, so.d);
    u_in = at(u_in, so.c);
    ec = at(ec, so.c);
    b = at(b, so.c);
    u_out = at(u_out, so.c);
    r64 = at(r64, so.c);
    zr_out = at(zr_out, so.c);
    if (load_state(conv) != 0) return;
    const int nx = op.nx, ny = op.ny;
    const int ncx = nx / 2, ncy = ny / 2;
    const TileInfo t = tile_info<R>(sw, ny + 1);
    if (!t.block_ok) return;
    constexpr int HL = 2, WOUT = 60;
    const int lane = lane_id();
    const int i = t.strip * WOUT - HL + lane;
    const bool out_lane = lane >= HL && lane < HL + WOUT && i <= nx;
    const bool node_col = i >= 0 && i <= nx;
    const int I0 = i >> 1, I1 = (i + 1) >> 1;
    double dot = 0.0;
    if (t.j0 < t.j1) {
        // v rows j0-2 .. j0+R+1, element rows j0-2 .. j0+R, b rows j0-1 .. j0+R
        V2<T> vr[R + 4], br[R + 2];
        Mom<T> me[R + 3];
        V2<double> rr64[DOT ? R : 1];
        constexpr int NC = PROLONG ? (R + 2) / 2 + 3 : 1;
        V2<T> c0[NC], c1[NC];
        // all loads first, none inside a branch (u_in == null reads zeros)
        const T* uin = u_in ? u_in : b;
#pragma unroll
        for (int s = 0; s < R + 4; ++s) vr[s] = load_node(uin, nx, ny, i, t.j0 - 2 + s, u_in != nullptr);
        // fine rows j0-2 .. j0+R+1 = rows (j0-1)-1 .. (j0-1)+(R+2)
        if constexpr (PROLONG) load_prolongation<T, R + 2>(c0, c1, ec, ncx, ncy, I0, I1, t.j0 - 1);
        // b and r are used only through u1 and the output, both selected by
        // the node's validity: unmasked loads
#pragma unroll
        for (int s = 0; s < R + 2; ++s) br[s] = load_node_clamped(b, nx, ny, i, t.j0 - 1 + s);
        if constexpr (DOT) {
#pragma unroll
            for (int s = 0; s < R; ++s) rr64[s] = load_node_clamped(r64, nx, ny, i, t.j0 + s);
        }
#pragma unroll
        for (int s = 0; s < R + 3; ++s) me[s] = load_elem<T, FINE>(op, i, t.j0 - 2 + s);
        if constexpr (!FINE) __builtin_amdgcn_sched_barrier(0);   // latency-bound: one batch of loads
        if constexpr (PROLONG) {
            if (t.j0 & 1) add_prolongation<T, R + 2, 0>(vr, c0, c1, t.j0 - 1, node_col, ny);
            else add_prolongation<T, R + 2, 1>(vr, c0, c1, t.j0 - 1, node_col, ny);
        }

        post2_stages<T, FINE, R>(mat, vr, br, me, t.j0, node_col, ny, [&](int jr, int q, const V2<T>& uo) {
            if (out_lane && jr < t.j1) {
                if (jr >= 1) {
                    store_node(u_out, nx, i, jr, uo);
                    if constexpr (DOT) dot += (double)uo.x * rr64[q].x + (double)uo.y * rr64[q].y;
                } else {
                    store_node(u_out, nx, i, jr, V2<T>{T(0), T(0)});
                }
            }
        });
    }
    if constexpr (DOT) {
        const double s = block_sum(dot);
        if (threadIdx.x == 0) zr_out[t.tile] = s;
    }
}

// ===========================================================================
// The paired post-smoother of two consecutive coarse levels in one launch:
// level l gets u_l + P e_{l-1} followed by two sweeps (= e_l), and level
// l+1 then u_{l+1} + P e_l followed by two sweeps, written to u_out.
// Phase A (lanes = level-l columns): the four waves of a workgroup share
// the NU level-l rows that the prolongation of their 4R level-(l+1) rows
// reads, RA rows each; e_l passes through LDS and never reaches memory.
// Phase B (lanes = level-(l+1) columns) is k_post2.  Both phases issue
// their loads before the first wait.  A level-l node may be formed by
// several workgroups, each in the operation order of k_post2, so the
// result equals two k_post2 launches.
// Geometry: that of k_post2 on level l+1 (60 output columns per strip).
// ===========================================================================
template <typename T, int R>
__global__ __launch_bounds__(WG_THREADS) void k_post2_pair(
    LevelOp<T> opc, LevelOp<T> opf, Mat<T> mat, Sweep sw, const T* __restrict__ uc_in, const T* __restrict__ ee,
    const T* __restrict__ bc, const T* __restrict__ uf_in, const T* __restrict__ bf, T* __restrict__ u_out,
    const int* conv, Batch bt) {
    constexpr int NC = (R + 2) / 2 + 3;                     // level-l rows one wave's prolongation reads
    constexpr int NU = ((3 * R - 1) >> 1) + NC + 1;         // their union over the workgroup
    constexpr int RA = (NU + WAVES_PER_WG - 1) / WAVES_PER_WG;
    __shared__ V2<T> ebuf[RA * WAVES_PER_WG][WAVE];
    const SysOff so = sys_off(bt);
    conv = at(conv, so.c);
    opc.data = at(opc.data, so.d);
    opf.data = at(opf.data, so.d);
    uc_in = at(uc_in, so.c);
    ee = at(ee, so.c);
    bc = at(bc, so.c);
    uf_in = at(uf_in, so.c);
    bf = at(bf, so.c);
    u_out = at(u_out, so.c);
    if (load_state(conv) != 0) return;   // uniform over the workgroup (one system)
    const int nxf = opf.nx, nyf = opf.ny, nxc = opc.nx, nyc = opc.ny;
    const TileInfo t = tile_info<R>(sw, nyf + 1);
    if (!t.block_ok) return;
    constexpr int HL = 2, WOUT = 60;
    const int lane = lane_id();
    // phase B: level-(l+1) column i; phase A: level-l column ic (64 columns
    // from the one left of this strip's, so phase B's I0, I1 = i >> 1,
    // (i+1) >> 1 sit on lanes 2 .. 34 of phase A, all with both neighbours)
    const int i = t.strip * WOUT - HL + lane;
    const bool out_lane = lane >= HL && lane < HL + WOUT && i <= nxf;
    const bool node_col = i >= 0 && i <= nxf;
    const int icb = t.strip * (WOUT / 2) - 3;
    const int ic = icb + lane;
    const bool node_colc = ic >= 0 && ic <= nxc;
    // the workgroup's first level-(l+1) row is even, so its level-l rows
    // start at JU0 = j/2 - 2; this wave forms rows JA .. JA + RA - 1
    const int jw0 = t.j0 - wave_id() * R;
    const int JU0 = (jw0 >> 1) - 2;
    const int JA = JU0 + wave_id() * RA;

    // ---- all loads
    V2<T> va[RA + 4], ba[RA + 2];
    Mom<T> ma[RA + 3];
    constexpr int NE = (RA + 2) / 2 + 3;
    V2<T> e0[NE], e1[NE];
    const T* ucin = uc_in ? uc_in : bc;
#pragma unroll
    for (int s = 0; s < RA + 4; ++s) va[s] = load_node(ucin, nxc, nyc, ic, JA - 2 + s, uc_in != nullptr);
    load_prolongation<T, RA + 2>(e0, e1, ee, nxc / 2, nyc / 2, ic >> 1, (ic + 1) >> 1, JA - 1);
#pragma unroll
    for (int s = 0; s < RA + 2; ++s) ba[s] = load_node(bc, nxc, nyc, ic, JA - 1 + s);
#pragma unroll
    for (int s = 0; s < RA + 3; ++s) ma[s] = load_elem<T, false>(opc, ic, JA - 2 + s);
    V2<T> vr[R + 4], br[R + 2];
    Mom<T> me[R + 3];
    const T* ufin = uf_in ? uf_in : bf;
#pragma unroll
    for (int s = 0; s < R + 4; ++s) vr[s] = load_node(ufin, nxf, nyf, i, t.j0 - 2 + s, uf_in != nullptr);
#pragma unroll
    for (int s = 0; s < R + 2; ++s) br[s] = load_node(bf, nxf, nyf, i, t.j0 - 1 + s);
#pragma unroll
    for (int s = 0; s < R + 3; ++s) me[s] = load_elem<T, false>(opf, i, t.j0 - 2 + s);
    __builtin_amdgcn_sched_barrier(0);

    // ---- phase A: e_l on rows JA .. JA + RA - 1, zero off the grid and on the clamped row
    if ((JA - 1) & 1) add_prolongation<T, RA + 2, 1>(va, e0, e1, JA - 1, node_colc, nyc);
    else add_prolongation<T, RA + 2, 0>(va, e0, e1, JA - 1, node_colc, nyc);
    post2_stages<T, false, RA>(mat, va, ba, ma, JA, node_colc, nyc, [&](int jr, int q, const V2<T>& uo) {
        const bool ok = node_colc && jr >= 1 && jr <= nyc;
        ebuf[wave_id() * RA + q][lane] = ok ? uo : V2<T>{T(0), T(0)};
    });
    __syncthreads();
    if (t.j0 >= t.j1) return;

    // ---- phase B: k_post2 on level l+1 with e_l from LDS (rows Jb .. Jb + NC - 1)
    const int Jb = ((t.j0 - 1) >> 1) - 1;
    V2<T> c0[NC], c1[NC];
    const int l0 = (i >> 1) - icb, l1 = ((i + 1) >> 1) - icb;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        c0[k] = ebuf[Jb - JU0 + k][l0];
        c1[k] = ebuf[Jb - JU0 + k][l1];
    }
    if (t.j0 & 1) add_prolongation<T, R + 2, 0>(vr, c0, c1, t.j0 - 1, node_col, nyf);
    else add_prolongation<T, R + 2, 1>(vr, c0, c1, t.j0 - 1, node_col, nyf);
    post2_stages<T, false, R>(mat, vr, br, me, t.j0, node_col, nyf, [&](int jr, int q, const V2<T>& uo) {
        if (out_lane && jr < t.j1) store_node(u_out, nxf, i, jr, jr >= 1 ? uo : V2<T>{T(0), T(0)});
    });
}

// ===========================================================================
// Plain stiffness apply q = K_l u (or its diagonal) in the level precision
// (test hook and building block).  Geometry as k_cg_apply.
// ===========================================================================
template <typename T, bool FINE, bool DIAG, int R>
__global__ __launch_bounds__(WG_THREADS) void k_apply(LevelOp<T> op, Mat<T> mat, Sweep sw,
                                                      const T* __restrict__ u, T* __restrict__ q) {
    const int nx = op.nx, ny = op.ny;
    const TileInfo t = tile_info<R>(sw, ny + 1);
    if (!t.block_ok) return;
    constexpr int HL = 1, WOUT = 62;
    const int lane = lane_id();
    const int i = t.strip * WOUT - HL + lane;
    const bool out_lane = lane >= HL && lane < HL + WOUT && i <= nx;
    if (t.j0 >= t.j1) return;
    V2<T> ur[R + 2];
    Mom<T> me[R + 1];
#pragma unroll
    for (int s = 0; s < R + 2; ++s) ur[s] = DIAG ? V2<T>{T(0), T(0)} : load_node(u, nx, ny, i, t.j0 - 1 + s);
#pragma unroll
    for (int s = 0; s < R + 1; ++s) me[s] = load_elem<T, FINE>(op, i, t.j0 - 1 + s);
    V2<T> f0, f1, f2, f3;
    V2<T> ur_lo = from_right(ur[0]), ur_hi = from_right(ur[1]);
    if (DIAG) elem_diag<FINE>(me[0], mat, f0, f1, f2, f3);
    else elem_force<FINE>(me[0], mat, ur[0], ur_lo, ur_hi, ur[1], f0, f1, f2, f3);
    V2<T> carry = f3 + from_left(f2);
#pragma unroll
    for (int s = 0; s < R; ++s) {
        const int j = t.j0 + s;
        ur_lo = ur_hi;
        ur_hi = from_right(ur[s + 2]);
        if (DIAG) elem_diag<FINE>(me[s + 1], mat, f0, f1, f2, f3);
        else elem_force<FINE>(me[s + 1], mat, ur[s + 1], ur_lo, ur_hi, ur[s + 2], f0, f1, f2, f3);
        V2<T> qv = carry + f0 + from_left(f1);
        carry = f3 + from_left(f2);
        if (out_lane && j < t.j1) {
            if (j < 1) qv = V2<T>{T(0), T(0)};
            store_node(q, nx, i, j, qv);
        }
    }
}

// ===========================================================================
// Coarsest direct solve e = K_0^{-1} b with the explicit FP64 inverse of
// the Cholesky factorisation (row-major n0 x n0 over the free DOFs, which
// are the nodal DOFs of rows j >= 1 in order).  One wave per matrix row.
// With LDS the workgroup stages b in LDS first (n0 doubles); without, for
// large coarsest grids, every wave reads b from memory (through L2).
// ===========================================================================
template <typename T, bool LDS>
__global__ __launch_bounds__(WG_THREADS) void k_coarse_solve(const double* __restrict__ Ainv, int n0,
                                                             int ld, int nx0, const T* __restrict__ b,
                                                             T* __restrict__ e, const int* conv, Batch bt) {
    const SysOff so = sys_off(bt);
    // the state word, b and the first U * 64 entries of this wave's row of
    // K0^-1 are all requested before the first wait
    const int cst = load_state(at(conv, so.c));
    Ainv = at(Ainv, so.d);
    b = at(b, so.c);
    e = at(e, so.c);
    extern __shared__ double sb[];
    const int off = 2 * (nx0 + 1);
    // loads are issued in batches of U per thread before they are used, so a
    // wave waits for one memory round trip per batch, not one per element
    constexpr int U = 16;
    const int row = blockIdx.x * WAVES_PER_WG + wave_id();
    const double* a = Ainv + (size_t)min(row, n0 - 1) * ld;
    double va[U];
#pragma unroll
    for (int u = 0; u < U; ++u) va[u] = a[min(lane_id() + u * WAVE, n0 - 1)];
    if constexpr (LDS) {
        for (int base = 0; base < n0; base += U * WG_THREADS) {
            T v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = b[off + min(base + (int)threadIdx.x + u * WG_THREADS, n0 - 1)];
            if (base == 0 && cst != 0) return;   // uniform over the block (one system)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = base + threadIdx.x + u * WG_THREADS;
                if (k < n0) sb[k] = (double)v[u];
            }
        }
    } else {
        if (cst != 0) return;
    }
    if (blockIdx.x == 0) {
        for (int k = threadIdx.x; k < off; k += WG_THREADS) e[k] = T(0);
    }
    if constexpr (LDS) __syncthreads();
    if (row >= n0) return;
    // s = sum over k = lane, lane + 64, ... of a[k] b[k], in that order
    double s = 0.0;
    for (int base = 0; base < n0; base += U * WAVE) {
        double v[U];
        if (base == 0) {
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = va[u];
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = a[min(base + lane_id() + u * WAVE, n0 - 1)];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = base + lane_id() + u * WAVE;
            const double bk = LDS ? sb[min(k, n0 - 1)] : (double)b[off + min(k, n0 - 1)];
            s = (k < n0) ? s + v[u] * bk : s;
        }
    }
    s = wave_sum(s);
    if (lane_id() == 0) e[off + row] = (T)s;
}

// ===========================================================================
// launchers: the rows per wave (a compile-time loop length, so all loads of
// a wave can be issued together) is chosen per level on the host.
// ===========================================================================
// Profiling: a start/stop event pair for the next launch, stamped by the
// kernel's own dispatch (hipExtLaunchKernel), so the interval is the
// kernel's execution without the launch gaps around it.
static hipEvent_t g_ev_start = nullptr, g_ev_stop = nullptr;
void time_next_launch(hipEvent_t start, hipEvent_t stop) {
    g_ev_start = start;
    g_ev_stop = stop;
}
#define MTOMG_LAUNCH(K, GRID, BLOCK, SHM, ST, ...)                                                   \
    do {                                                                                         \
        if (g_ev_start) {                                                                        \
            hipExtLaunchKernelGGL(K, GRID, BLOCK, SHM, ST, g_ev_start, g_ev_stop, 0, __VA_ARGS__); \
            g_ev_start = g_ev_stop = nullptr;                                                    \
        } else {                                                                                 \
            hipLaunchKernelGGL(K, GRID, BLOCK, SHM, ST, __VA_ARGS__);                            \
        }                                                                                        \
    } while (0)

// x: tiles (a multiple of 8, for the XCD-aware tile order), y: systems
static inline dim3 grid_of(const Sweep& s, const Batch& bt = Batch{}) {
    return dim3(8 * ((s.n_tiles + 7) / 8), bt.n);
}

// rows per wave of k_pre_restrict: at most 4 (it holds 2R + 5 node rows)
#define MTOMG_ROWS4_SWITCH(R_, CALL)              \
    switch (R_) {                                 \
        case 1: { constexpr int RR = 1; CALL; } break; \
        case 2: { constexpr int RR = 2; CALL; } break; \
        default: { constexpr int RR = 4; CALL; } break; \
    }

#define MTOMG_ROWS_SWITCH(R_, CALL)               \
    switch (R_) {                                 \
        case 1: { constexpr int RR = 1; CALL; } break; \
        case 2: { constexpr int RR = 2; CALL; } break; \
        case 4: { constexpr int RR = 4; CALL; } break; \
        default: { constexpr int RR = 8; CALL; } break; \
    }

void launch_partial_total(hipStream_t st, double* p, int n, const int* conv, const Batch& bt) {
    MTOMG_LAUNCH(k_partial_total, dim3(1, bt.n), dim3(WG_THREADS), 0, st, p, n, conv, bt);
}

template <typename TZ>
void launch_cg_apply(hipStream_t st, LevelOp<double> op, Mat<double> mat, Sweep sw, const TZ* z,
                     const double* p_old, double* p_new, double* x, double* q, const double* zr_cur,
                     const double* zr_prev, int n_zr, const double* pq_prev, int n_pq,
                     double* pq_out, const int* conv, int mode, const Batch& bt) {
    MTOMG_ROWS_SWITCH(sw.rows, MTOMG_LAUNCH((k_cg_apply<TZ, RR>), grid_of(sw, bt), dim3(WG_THREADS), 0, st,
                                                   op, mat, sw, z, p_old, p_new, x, q, zr_cur, zr_prev, n_zr,
                                                   pq_prev, n_pq, pq_out, conv, mode, bt))
}
template void launch_cg_apply<float>(hipStream_t, LevelOp<double>, Mat<double>, Sweep, const float*,
                                     const double*, double*, double*, double*, const double*,
                                     const double*, int, const double*, int, double*, const int*, int,
                                     const Batch&);
template void launch_cg_apply<double>(hipStream_t, LevelOp<double>, Mat<double>, Sweep, const double*,
                                      const double*, double*, double*, double*, const double*,
                                      const double*, int, const double*, int, double*, const int*, int,
                                      const Batch&);

void launch_residual(hipStream_t st, LevelOp<double> op, Mat<double> mat, Sweep sw, const double* f,
                     double* x, int use_x, double* r, double* rr_out, double* ff_out, const int* conv,
                     const Batch& bt) {
    MTOMG_ROWS_SWITCH(sw.rows, MTOMG_LAUNCH((k_residual<RR>), grid_of(sw, bt), dim3(WG_THREADS), 0, st, op,
                                                   mat, sw, f, x, use_x, r, rr_out, ff_out, conv, bt))
}

template <typename T>
void launch_presmooth(hipStream_t st, bool fine, bool cgmode, LevelOp<T> op, Mat<T> mat, Sweep sw,
                      const T* b, T* u_out, int sweeps, const CgRhs& cg, const int* conv, const Batch& bt) {
#define MTOMG_PRE(F, C)                                                                              \
    MTOMG_ROWS_SWITCH(sw.rows, MTOMG_LAUNCH((k_presmooth<T, F, C, RR>), grid_of(sw, bt), dim3(WG_THREADS), \
                                                   0, st, op, mat, sw, b, u_out, sweeps, cg, conv, bt))
    if (cgmode) MTOMG_PRE(true, true)
    else if (fine) MTOMG_PRE(true, false)
    else MTOMG_PRE(false, false)
#undef MTOMG_PRE
}

template <typename T>
void launch_restrict(hipStream_t st, bool fine, bool check, LevelOp<T> op, Mat<T> mat, Sweep sw,
                     const T* b, const T* u, T* rc, const ConvCheck& chk, const int* conv, const Batch& bt) {
#define MTOMG_RES(F, C)                                                                              \
    MTOMG_ROWS_SWITCH(sw.rows, MTOMG_LAUNCH((k_restrict<T, F, C, RR>), grid_of(sw, bt), dim3(WG_THREADS), \
                                                   0, st, op, mat, sw, b, u, rc, chk, conv, bt))
    if (check) MTOMG_RES(true, true)
    else if (fine) MTOMG_RES(true, false)
    else MTOMG_RES(false, false)
#undef MTOMG_RES
}

template <typename T>
void launch_pre_restrict(hipStream_t st, bool fine, bool cgmode, bool check, LevelOp<T> op, Mat<T> mat, Sweep sw,
                         const T* b, T* u_out, T* rc, const CgRhs& cg, const ConvCheck& chk, const int* conv,
                         const Batch& bt) {
#define MTOMG_PR(F, C, K)                                                                             \
    MTOMG_ROWS4_SWITCH(sw.rows, MTOMG_LAUNCH((k_pre_restrict<T, F, C, K, RR>), grid_of(sw, bt),          \
                                             dim3(WG_THREADS), 0, st, op, mat, sw, b, u_out, rc, cg, chk, \
                                             conv, bt))
    if (cgmode) MTOMG_PR(true, true, false)
    else if (fine) MTOMG_PR(true, false, false)
    else if (check) MTOMG_PR(false, false, true)
    else MTOMG_PR(false, false, false)
#undef MTOMG_PR
}

template <typename T>
void launch_restrict_pre(hipStream_t st, bool fine, bool check, LevelOp<T> op, LevelOp<T> opc, Mat<T> mat,
                         Sweep sw, const T* b, const T* u, T* rc, T* uc, int sweeps, const ConvCheck& chk,
                         const int* conv, const Batch& bt) {
#define MTOMG_RP(F, C)                                                                               \
    MTOMG_ROWS_SWITCH(sw.rows, MTOMG_LAUNCH((k_restrict_pre<T, F, C, RR>), grid_of(sw, bt), dim3(WG_THREADS), \
                                             0, st, op, opc, mat, sw, b, u, rc, uc, sweeps, chk, conv, bt))
    if (check) MTOMG_RP(true, true)
    else if (fine) MTOMG_RP(true, false)
    else MTOMG_RP(false, false)
#undef MTOMG_RP
}

template <typename T>
void launch_post(hipStream_t st, bool fine, bool prolong, bool dot, LevelOp<T> op, Mat<T> mat, Sweep sw,
                 const T* u_in, const T* ec, const T* b, T* u_out, const double* r64, double* zr_out,
                 const int* conv, const Batch& bt) {
#define MTOMG_POST(F, P, D)                                                                          \
    MTOMG_ROWS_SWITCH(sw.rows, MTOMG_LAUNCH((k_post<T, F, P, D, RR>), grid_of(sw, bt), dim3(WG_THREADS), \
                                                   0, st, op, mat, sw, u_in, ec, b, u_out, r64, zr_out, conv, bt))
    if (fine) {
        if (prolong) { if (dot) MTOMG_POST(true, true, true) else MTOMG_POST(true, true, false) }
        else { if (dot) MTOMG_POST(true, false, true) else MTOMG_POST(true, false, false) }
    } else {
        if (prolong) MTOMG_POST(false, true, false)
        else MTOMG_POST(false, false, false)
    }
#undef MTOMG_POST
}

template <typename T>
void launch_post2(hipStream_t st, bool fine, bool prolong, bool dot, LevelOp<T> op, Mat<T> mat, Sweep sw,
                  const T* u_in, const T* ec, const T* b, T* u_out, const double* r64, double* zr_out,
                  const int* conv, const Batch& bt) {
#define MTOMG_POST2(F, P, D)                                                                         \
    MTOMG_ROWS_SWITCH(sw.rows, MTOMG_LAUNCH((k_post2<T, F, P, D, RR>), grid_of(sw, bt), dim3(WG_THREADS), \
                                                   0, st, op, mat, sw, u_in, ec, b, u_out, r64, zr_out, conv, bt))
    if (fine) {
        if (prolong) { if (dot) MTOMG_POST2(true, true, true) else MTOMG_POST2(true, true, false) }
        else { if (dot) MTOMG_POST2(true, false, true) else MTOMG_POST2(true, false, false) }
    } else {
        if (prolong) MTOMG_POST2(false, true, false)
        else MTOMG_POST2(false, false, false)
    }
#undef MTOMG_POST2
}

template <typename T>
void launch_post2_pair(hipStream_t st, LevelOp<T> opc, LevelOp<T> opf, Mat<T> mat, Sweep sw, const T* uc_in,
                       const T* ee, const T* bc, const T* uf_in, const T* bf, T* u_out, const int* conv,
                       const Batch& bt) {
    MTOMG_ROWS_SWITCH(sw.rows, MTOMG_LAUNCH((k_post2_pair<T, RR>), grid_of(sw, bt), dim3(WG_THREADS), 0, st, opc, opf,
                                            mat, sw, uc_in, ee, bc, uf_in, bf, u_out, conv, bt));
}

template <typename T>
void launch_apply(hipStream_t st, bool fine, bool diag, LevelOp<T> op, Mat<T> mat, Sweep sw, const T* u,
                  T* q) {
#define MTOMG_APP(F, D)                                                                              \
    MTOMG_ROWS_SWITCH(sw.rows, MTOMG_LAUNCH((k_apply<T, F, D, RR>), grid_of(sw), dim3(WG_THREADS), 0, st, \
                                                   op, mat, sw, u, q))
    if (fine) { if (diag) MTOMG_APP(true, true) else MTOMG_APP(true, false) }
    else { if (diag) MTOMG_APP(false, true) else MTOMG_APP(false, false) }
#undef MTOMG_APP
}

template <typename T>
void launch_coarse_solve(hipStream_t st, const double* Ainv, int n0, int ld, int nx0, const T* b, T* e,
                         const int* conv, const Batch& bt) {
    const int nblk = (n0 + WAVES_PER_WG - 1) / WAVES_PER_WG;
    // b staged in LDS up to 32 KB; larger coarsest grids read it through L2
    if (n0 <= COARSE_LDS_MAX)
        MTOMG_LAUNCH((k_coarse_solve<T, true>), dim3(nblk, bt.n), dim3(WG_THREADS), n0 * sizeof(double), st, Ainv,
                     n0, ld, nx0, b, e, conv, bt);
    else
        MTOMG_LAUNCH((k_coarse_solve<T, false>), dim3(nblk, bt.n), dim3(WG_THREADS), 0, st, Ainv, n0, ld, nx0, b,
                     e, conv, bt);
}

#define MTOMG_INST(T)                                                                              \
    template void launch_presmooth<T>(hipStream_t, bool, bool, LevelOp<T>, Mat<T>, Sweep, const T*, T*, \
                                      int, const CgRhs&, const int*, const Batch&);                \
    template void launch_restrict<T>(hipStream_t, bool, bool, LevelOp<T>, Mat<T>, Sweep, const T*,    \
                                     const T*, T*, const ConvCheck&, const int*, const Batch&);    \
    template void launch_pre_restrict<T>(hipStream_t, bool, bool, bool, LevelOp<T>, Mat<T>, Sweep, const T*, \
                                         T*, T*, const CgRhs&, const ConvCheck&, const int*, const Batch&); \
    template void launch_restrict_pre<T>(hipStream_t, bool, bool, LevelOp<T>, LevelOp<T>, Mat<T>, Sweep,  \
                                         const T*, const T*, T*, T*, int, const ConvCheck&, const int*, \
                                         const Batch&);                                            \
    template void launch_post<T>(hipStream_t, bool, bool, bool, LevelOp<T>, Mat<T>, Sweep, const T*,  \
                                 const T*, const T*, T*, const double*, double*, const int*,       \
                                 const Batch&);                                                    \
    template void launch_post2<T>(hipStream_t, bool, bool, bool, LevelOp<T>, Mat<T>, Sweep, const T*, \
                                  const T*, const T*, T*, const double*, double*, const int*,      \
                                  const Batch&);                                                   \
    template void launch_apply<T>(hipStream_t, bool, bool, LevelOp<T>, Mat<T>, Sweep, const T*, T*);  \
    template void launch_coarse_solve<T>(hipStream_t, const double*, int, int, int, const T*, T*, const int*, \
                                         const Batch&);                                            \
    template void launch_post2_pair<T>(hipStream_t, LevelOp<T>, LevelOp<T>, Mat<T>, Sweep, const T*, const T*, \
                                       const T*, const T*, const T*, T*, const int*, const Batch&);
MTOMG_INST(float)
MTOMG_INST(double)
#undef MTOMG_INST

}  // namespace mtomg
