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
// Outer CG: p = z + beta p_old, x += alpha_prev p_old, q = K p, partial p.q
// mode 0: iteration i >= 1; mode 1: first iteration (beta = 0, no x update);
// mode 2: only the pending x update (after the last iteration).
// Geometry: H_L = 1, H_R = 1, 62 output columns per strip.
// ===========================================================================
template <typename TZ, int R>
__global__ __launch_bounds__(WG_THREADS) void k_cg_apply(
    LevelOp<double> op, Mat<double> mat, Sweep sw, const TZ* __restrict__ z,
    const double* __restrict__ p_old, double* __restrict__ p_new, double* __restrict__ x,
    double* __restrict__ q, const double* __restrict__ zr_cur, const double* __restrict__ zr_prev,
    int n_zr, const double* __restrict__ pq_prev, int n_pq, double* __restrict__ pq_out,
    const int* conv, int mode) {
    const int cst = *conv;
    const bool final_only = (mode == 2) || (mode == 0 && cst == 1);
    if (mode == 1 && cst != 0) return;
    if (mode == 0 && cst != 0 && cst != 1) return;
    const int nx = op.nx, ny = op.ny;
    const TileInfo t = tile_info<R>(sw, ny + 1);
    if (!t.block_ok) return;
    constexpr int HL = 1, WOUT = 62;
    const int lane = lane_id();
    const int i = t.strip * WOUT - HL + lane;
    const bool out_lane = lane >= HL && lane < HL + WOUT && i <= nx;

    double alpha_prev = 0.0, beta = 0.0, rho_prev = 1.0;
    if (mode != 1) {
        rho_prev = sum_partials(zr_prev, n_zr);
        alpha_prev = rho_prev / sum_partials(pq_prev, n_pq);
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
    if (mode == 0) beta = sum_partials(zr_cur, n_zr) / rho_prev;

    auto getp = [&](int jj) -> V2<double> {
        if (i < 0 || i > nx || jj < 1 || jj > ny) return V2<double>{0.0, 0.0};
        const V2<TZ> zv = load_node(z, nx, ny, i, jj);
        V2<double> pv{(double)zv.x, (double)zv.y};
        V2<double> po{0.0, 0.0};
        if (mode == 0) {
            po = load_node(p_old, nx, ny, i, jj);
            pv.x += beta * po.x;
            pv.y += beta * po.y;
        }
        if (out_lane && jj >= t.j0 && jj < t.j1) {
            store_node(p_new, nx, i, jj, pv);
            if (mode == 0) {
                V2<double> xv = load_node(x, nx, ny, i, jj);
                xv.x += alpha_prev * po.x;
                xv.y += alpha_prev * po.y;
                store_node(x, nx, i, jj, xv);
            }
        }
        return pv;
    };

    double dot = 0.0;
    if (t.j0 < t.j1) {
        V2<double> pa = getp(t.j0 - 1), pa_r = from_right(pa);
        V2<double> pb = getp(t.j0), pb_r = from_right(pb);
        V2<double> f0, f1, f2, f3;
        elem_force(load_elem<double, true>(op, i, t.j0 - 1), mat, pa, pa_r, pb_r, pb, f0, f1, f2, f3);
        V2<double> carry = f3 + from_left(f2);
#pragma unroll
        for (int s = 0; s < R; ++s) {
            const int j = t.j0 + s;
            pa = pb; pa_r = pb_r;
            pb = getp(j + 1); pb_r = from_right(pb);
            elem_force(load_elem<double, true>(op, i, j), mat, pa, pa_r, pb_r, pb, f0, f1, f2, f3);
            const V2<double> qv = carry + f0 + from_left(f1);
            carry = f3 + from_left(f2);
            if (out_lane && j < t.j1) {
                if (j >= 1) {
                    store_node(q, nx, i, j, qv);
                    dot += pa.x * qv.x + pa.y * qv.y;
                } else {
                    store_node(q, nx, i, j, V2<double>{0.0, 0.0});
                    store_node(p_new, nx, i, j, V2<double>{0.0, 0.0});
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
// (then r may be null).  Geometry as k_cg_apply.
// ===========================================================================
template <int R>
__global__ __launch_bounds__(WG_THREADS) void k_residual(
    LevelOp<double> op, Mat<double> mat, Sweep sw, const double* __restrict__ f,
    double* __restrict__ x, int use_x, double* __restrict__ r, double* __restrict__ rr_out,
    double* __restrict__ ff_out) {
    const int nx = op.nx, ny = op.ny;
    const TileInfo t = tile_info<R>(sw, ny + 1);
    if (!t.block_ok) return;
    constexpr int HL = 1, WOUT = 62;
    const int lane = lane_id();
    const int i = t.strip * WOUT - HL + lane;
    const bool out_lane = lane >= HL && lane < HL + WOUT && i <= nx;
    auto getx = [&](int jj) -> V2<double> {
        if (!use_x) return V2<double>{0.0, 0.0};
        return load_node(x, nx, ny, i, jj);
    };
    double rr = 0.0, ff = 0.0;
    if (t.j0 < t.j1) {
        V2<double> xa = getx(t.j0 - 1), xa_r = from_right(xa);
        V2<double> xb = getx(t.j0), xb_r = from_right(xb);
        V2<double> f0, f1, f2, f3;
        elem_force(load_elem<double, true>(op, i, t.j0 - 1), mat, xa, xa_r, xb_r, xb, f0, f1, f2, f3);
        V2<double> carry = f3 + from_left(f2);
#pragma unroll
        for (int s = 0; s < R; ++s) {
            const int j = t.j0 + s;
            xa = xb; xa_r = xb_r;
            xb = getx(j + 1); xb_r = from_right(xb);
            elem_force(load_elem<double, true>(op, i, j), mat, xa, xa_r, xb_r, xb, f0, f1, f2, f3);
            const V2<double> kx = carry + f0 + from_left(f1);
            carry = f3 + from_left(f2);
            if (out_lane && j < t.j1) {
                if (j >= 1) {
                    const V2<double> fv = load_node(f, nx, ny, i, j);
                    const V2<double> rv = fv - kx;
                    if (r) store_node(r, nx, i, j, rv);
                    if (!use_x) store_node(x, nx, i, j, V2<double>{0.0, 0.0});
                    rr += rv.x * rv.x + rv.y * rv.y;
                    ff += fv.x * fv.x + fv.y * fv.y;
                } else {
                    if (r) store_node(r, nx, i, j, V2<double>{0.0, 0.0});
                    store_node(x, nx, i, j, V2<double>{0.0, 0.0});
                }
            }
        }
    }
    const double srr = block_sum(rr);
    const double sff = block_sum(ff);
    if (threadIdx.x == 0) {
        rr_out[t.tile] = srr;
        if (ff_out) ff_out[t.tile] = sff;
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
    int sweeps, CgRhs cg, const int* conv) {
    int cst = 0;
    if (conv) cst = *conv;
    if constexpr (CG) {
        if (cst == 1 && blockIdx.x == 0 && threadIdx.x == 0) *cg.conv_rw = 2;
    }
    if (cst != 0) return;
    const int nx = op.nx, ny = op.ny;
    const TileInfo t = tile_info<R>(sw, ny + 1);
    if (!t.block_ok) return;
    constexpr int HL = 2, WOUT = 61;
    const int lane = lane_id();
    const int i = t.strip * WOUT - HL + lane;
    const bool out_lane = lane >= HL && lane < HL + WOUT && i <= nx;
    const bool node_col = i >= 0 && i <= nx;

    double alpha = 0.0;
    if constexpr (CG) {
        if (cg.update) {
            const double rho = sum_partials(cg.zr, cg.n_zr);
            const double pq = sum_partials(cg.pq, cg.n_pq);
            alpha = rho / pq;
            if (!(pq > 0.0) || !(rho > 0.0) || !isfinite(alpha)) {
                if (blockIdx.x == 0 && threadIdx.x == 0) *cg.conv_rw = isfinite(alpha) ? 3 : 4;
                return;
            }
            if (blockIdx.x == 0 && threadIdx.x == 0) *cg.iters += 1;
        }
    }
    double rr = 0.0;
    auto getb = [&](int jj) -> V2<T> {
        if (!node_col || jj < 1 || jj > ny) return V2<T>{T(0), T(0)};
        if constexpr (CG) {
            V2<double> rv = load_node(cg.r_old, nx, ny, i, jj);
            if (cg.update) {
                const V2<double> qv = load_node(cg.q, nx, ny, i, jj);
                rv.x -= alpha * qv.x;
                rv.y -= alpha * qv.y;
            }
            if (out_lane && jj >= t.j0 && jj < t.j1) {
                if (cg.update) {
                    store_node(cg.r_new, nx, i, jj, rv);
                    rr += rv.x * rv.x + rv.y * rv.y;
                }
                if constexpr (sizeof(T) == 4) store_node(cg.r32, nx, i, jj, V2<float>{(float)rv.x, (float)rv.y});
            }
            return V2<T>{(T)rv.x, (T)rv.y};
        } else {
            return load_node(b, nx, ny, i, jj);
        }
    };

    if (t.j0 < t.j1) {
        // zero the clamped row of the outputs
        if (t.j0 == 0 && out_lane) {
            store_node(u_out, nx, i, 0, V2<T>{T(0), T(0)});
            if constexpr (CG) {
                if (cg.update) store_node(cg.r_new, nx, i, 0, V2<double>{0.0, 0.0});
                if constexpr (sizeof(T) == 4) store_node(cg.r32, nx, i, 0, V2<float>{0.f, 0.f});
            }
        }
        V2<T> d0, d1, d2, d3;
        // diagonal carry from element row j0-2
        elem_diag(load_elem<T, FINE>(op, i, t.j0 - 2), mat, d0, d1, d2, d3);
        V2<T> dcarry = d3 + from_left(d2);
        V2<T> fcarry{T(0), T(0)};
        Mom<T> m_prev = mom_zero<T>();
        V2<T> u1_prev{T(0), T(0)}, u1r_prev{T(0), T(0)}, b_prev{T(0), T(0)}, D_prev{T(1), T(1)};
#pragma unroll
        for (int s = 0; s < R + 2; ++s) {
            const int k = t.j0 - 1 + s;
            const Mom<T> mk = load_elem<T, FINE>(op, i, k);
            elem_diag(mk, mat, d0, d1, d2, d3);
            const V2<T> D = dcarry + d0 + from_left(d1);
            dcarry = d3 + from_left(d2);
            const V2<T> bk = getb(k);
            V2<T> u1{T(0), T(0)};
            if (node_col && k >= 1 && k <= ny) {
                u1.x = mat.omega * bk.x / D.x;
                u1.y = mat.omega * bk.y / D.y;
            }
            const V2<T> u1r = from_right(u1);
            if (s >= 1) {
                // force stage for element row k-1 -> node row k-1 complete
                V2<T> f0, f1, f2, f3;
                elem_force(m_prev, mat, u1_prev, u1r_prev, u1r, u1, f0, f1, f2, f3);
                const V2<T> fs = fcarry + f0 + from_left(f1);
                fcarry = f3 + from_left(f2);
                const int jr = k - 1;
                if (jr >= t.j0 && jr < t.j1 && jr >= 1 && out_lane) {
                    V2<T> uo = sweeps == 0 ? V2<T>{T(0), T(0)} : u1_prev;
                    if (sweeps >= 2) {
                        uo.x = u1_prev.x + mat.omega * (b_prev.x - fs.x) / D_prev.x;
                        uo.y = u1_prev.y + mat.omega * (b_prev.y - fs.y) / D_prev.y;
                    }
                    store_node(u_out, nx, i, jr, uo);
                }
            }
            m_prev = mk;
            u1_prev = u1;
            u1r_prev = u1r;
            b_prev = bk;
            D_prev = D;
        }
    }
    if constexpr (CG) {
        if (cg.update) {
            const double s = block_sum(rr);
            if (threadIdx.x == 0) cg.rr_out[t.tile] = s;
        }
    }
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
template <typename T, bool FINE, bool CHECK, int R>
__global__ __launch_bounds__(WG_THREADS) void k_restrict(
    LevelOp<T> op, Mat<T> mat, Sweep sw, const T* __restrict__ b, const T* __restrict__ u,
    T* __restrict__ rc, ConvCheck chk, const int* conv) {
    int cst = 0;
    if (conv) cst = *conv;
    if (cst != 0) return;
    const int nx = op.nx, ny = op.ny;
    const int ncx = nx / 2, ncy = ny / 2;
    const TileInfo t = tile_info<R>(sw, ncy + 1);
    if (!t.block_ok) return;
    if constexpr (CHECK) {
        const double rr = sum_partials(chk.rr, chk.n_rr);
        const double ff = sum_partials(chk.ff, chk.n_ff);
        const bool done = rr <= chk.tol2 * ff;
        if (!(rr == rr)) {
            if (blockIdx.x == 0 && threadIdx.x == 0) *chk.conv_rw = 4;
            return;
        }
        if (done) {
            if (blockIdx.x == 0 && threadIdx.x == 0) *chk.conv_rw = 1;
            return;
        }
    }
    constexpr int HL = 2, WOUT = 60;
    const int lane = lane_id();
    const int i = t.strip * WOUT - HL + lane;   // even lanes <-> even fine columns
    const int I = i >> 1;
    const bool out_lane = lane >= HL && lane < HL + WOUT && !(lane & 1) && I <= ncx;
    const bool node_col = i >= 0 && i <= nx;
    if (t.j0 >= t.j1) return;
    auto getu = [&](int jj) -> V2<T> {
        if (!u) return V2<T>{T(0), T(0)};
        return load_node(u, nx, ny, i, jj);
    };
    const int jf0 = 2 * t.j0 - 1;   // fine rows computed: jf0 .. jf0 + 2R
    V2<T> ua = getu(jf0 - 1), ua_r = from_right(ua);
    V2<T> ub = getu(jf0), ub_r = from_right(ub);
    V2<T> f0, f1, f2, f3;
    elem_force(load_elem<T, FINE>(op, i, jf0 - 1), mat, ua, ua_r, ub_r, ub, f0, f1, f2, f3);
    V2<T> carry = f3 + from_left(f2);
    V2<T> h_m2{T(0), T(0)}, h_m1{T(0), T(0)};
#pragma unroll
    for (int s = 0; s <= 2 * R; ++s) {
        const int j = jf0 + s;
        ua = ub; ua_r = ub_r;
        ub = getu(j + 1); ub_r = from_right(ub);
        elem_force(load_elem<T, FINE>(op, i, j), mat, ua, ua_r, ub_r, ub, f0, f1, f2, f3);
        const V2<T> ku = carry + f0 + from_left(f1);
        carry = f3 + from_left(f2);
        V2<T> rr{T(0), T(0)};
        if (node_col && j >= 1 && j <= ny) rr = load_node(b, nx, ny, i, j) - ku;
        const V2<T> rl = from_left(rr), rrt = from_right(rr);
        const V2<T> h{rr.x + T(0.5) * (rl.x + rrt.x), rr.y + T(0.5) * (rl.y + rrt.y)};
        if ((s & 1) == 0 && s >= 2) {
            const int J = (j - 1) >> 1;
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
    double* __restrict__ zr_out, const int* conv) {
    int cst = 0;
    if (conv) cst = *conv;
    if (cst != 0) return;
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
    auto getv = [&](int jj) -> V2<T> {
        if (!node_col || jj < 1 || jj > ny) return V2<T>{T(0), T(0)};
        V2<T> v = u_in ? load_node(u_in, nx, ny, i, jj) : V2<T>{T(0), T(0)};
        if constexpr (PROLONG) {
            const int J0 = jj >> 1, J1 = (jj + 1) >> 1;
            const V2<T> a = load_node(ec, ncx, ncy, I0, J0);
            const V2<T> bb = load_node(ec, ncx, ncy, I1, J0);
            const V2<T> c = load_node(ec, ncx, ncy, I0, J1);
            const V2<T> d = load_node(ec, ncx, ncy, I1, J1);
            v.x += T(0.25) * ((a.x + bb.x) + (c.x + d.x));
            v.y += T(0.25) * ((a.y + bb.y) + (c.y + d.y));
        }
        return v;
    };
    double dot = 0.0;
    if (t.j0 < t.j1) {
        V2<T> va = getv(t.j0 - 1), va_r = from_right(va);
        V2<T> vb = getv(t.j0), vb_r = from_right(vb);
        V2<T> f0, f1, f2, f3, d0, d1, d2, d3;
        {
            const Mom<T> m = load_elem<T, FINE>(op, i, t.j0 - 1);
            elem_force(m, mat, va, va_r, vb_r, vb, f0, f1, f2, f3);
            elem_diag(m, mat, d0, d1, d2, d3);
        }
        V2<T> fcarry = f3 + from_left(f2);
        V2<T> dcarry = d3 + from_left(d2);
#pragma unroll
        for (int s = 0; s < R; ++s) {
            const int j = t.j0 + s;
            va = vb; va_r = vb_r;
            vb = getv(j + 1); vb_r = from_right(vb);
            const Mom<T> m = load_elem<T, FINE>(op, i, j);
            elem_force(m, mat, va, va_r, vb_r, vb, f0, f1, f2, f3);
            elem_diag(m, mat, d0, d1, d2, d3);
            const V2<T> fs = fcarry + f0 + from_left(f1);
            const V2<T> D = dcarry + d0 + from_left(d1);
            fcarry = f3 + from_left(f2);
            dcarry = d3 + from_left(d2);
            if (out_lane && j < t.j1) {
                if (j >= 1) {
                    const V2<T> bv = load_node(b, nx, ny, i, j);
                    V2<T> uo;
                    uo.x = va.x + mat.omega * (bv.x - fs.x) / D.x;
                    uo.y = va.y + mat.omega * (bv.y - fs.y) / D.y;
                    store_node(u_out, nx, i, j, uo);
                    if constexpr (DOT) {
                        const V2<double> rv = load_node(r64, nx, ny, i, j);
                        dot += (double)uo.x * rv.x + (double)uo.y * rv.y;
                    }
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
// Plain stiffness apply q = K_l u in the level precision (test hook and
// building block): Geometry as k_cg_apply.
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
    auto getu = [&](int jj) -> V2<T> { return DIAG ? V2<T>{T(0), T(0)} : load_node(u, nx, ny, i, jj); };
    V2<T> ua = getu(t.j0 - 1), ua_r = from_right(ua);
    V2<T> ub = getu(t.j0), ub_r = from_right(ub);
    V2<T> f0, f1, f2, f3;
    {
        const Mom<T> m = load_elem<T, FINE>(op, i, t.j0 - 1);
        if (DIAG) elem_diag(m, mat, f0, f1, f2, f3);
        else elem_force(m, mat, ua, ua_r, ub_r, ub, f0, f1, f2, f3);
    }
    V2<T> carry = f3 + from_left(f2);
#pragma unroll
    for (int s = 0; s < R; ++s) {
        const int j = t.j0 + s;
        ua = ub; ua_r = ub_r;
        ub = getu(j + 1); ub_r = from_right(ub);
        const Mom<T> m = load_elem<T, FINE>(op, i, j);
        if (DIAG) elem_diag(m, mat, f0, f1, f2, f3);
        else elem_force(m, mat, ua, ua_r, ub_r, ub, f0, f1, f2, f3);
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
// ===========================================================================
template <typename T>
__global__ __launch_bounds__(WG_THREADS) void k_coarse_solve(const double* __restrict__ Ainv, int n0,
                                                             int ld, int nx0, const T* __restrict__ b,
                                                             T* __restrict__ e, const int* conv) {
    if (conv && *conv != 0) return;
    extern __shared__ double sb[];
    const int off = 2 * (nx0 + 1);
    for (int k = threadIdx.x; k < n0; k += WG_THREADS) sb[k] = (double)b[off + k];
    if (blockIdx.x == 0) {
        for (int k = threadIdx.x; k < off; k += WG_THREADS) e[k] = T(0);
    }
    __syncthreads();
    const int row = blockIdx.x * WAVES_PER_WG + wave_id();
    if (row >= n0) return;
    const double* a = Ainv + (size_t)row * ld;
    double s = 0.0;
    for (int k = lane_id(); k < n0; k += WAVE) s += a[k] * sb[k];
    s = wave_sum(s);
    if (lane_id() == 0) e[off + row] = (T)s;
}

// ===========================================================================
// launchers: the rows per wave (a compile-time loop length, so all loads of
// a wave can be issued together) is chosen per level on the host.
// ===========================================================================
static inline dim3 grid_of(const Sweep& s) { return dim3(8 * ((s.n_tiles + 7) / 8)); }

#define MTOMG_ROWS_SWITCH(R_, CALL)               \
    switch (R_) {                                 \
        case 1: { constexpr int RR = 1; CALL; } break; \
        case 2: { constexpr int RR = 2; CALL; } break; \
        case 4: { constexpr int RR = 4; CALL; } break; \
        default: { constexpr int RR = 8; CALL; } break; \
    }

template <typename TZ>
void launch_cg_apply(hipStream_t st, LevelOp<double> op, Mat<double> mat, Sweep sw, const TZ* z,
                     const double* p_old, double* p_new, double* x, double* q, const double* zr_cur,
                     const double* zr_prev, int n_zr, const double* pq_prev, int n_pq,
                     double* pq_out, const int* conv, int mode) {
    MTOMG_ROWS_SWITCH(sw.rows, hipLaunchKernelGGL((k_cg_apply<TZ, RR>), grid_of(sw), dim3(WG_THREADS), 0, st, op,
                                                   mat, sw, z, p_old, p_new, x, q, zr_cur, zr_prev, n_zr, pq_prev,
                                                   n_pq, pq_out, conv, mode))
}
template void launch_cg_apply<float>(hipStream_t, LevelOp<double>, Mat<double>, Sweep, const float*,
                                     const double*, double*, double*, double*, const double*,
                                     const double*, int, const double*, int, double*, const int*, int);
template void launch_cg_apply<double>(hipStream_t, LevelOp<double>, Mat<double>, Sweep, const double*,
                                      const double*, double*, double*, double*, const double*,
                                      const double*, int, const double*, int, double*, const int*, int);

void launch_residual(hipStream_t st, LevelOp<double> op, Mat<double> mat, Sweep sw, const double* f,
                     double* x, int use_x, double* r, double* rr_out, double* ff_out) {
    MTOMG_ROWS_SWITCH(sw.rows, hipLaunchKernelGGL((k_residual<RR>), grid_of(sw), dim3(WG_THREADS), 0, st, op, mat,
                                                   sw, f, x, use_x, r, rr_out, ff_out))
}

template <typename T>
void launch_presmooth(hipStream_t st, bool fine, bool cgmode, LevelOp<T> op, Mat<T> mat, Sweep sw,
                      const T* b, T* u_out, int sweeps, const CgRhs& cg, const int* conv) {
#define MTOMG_PRE(F, C)                                                                              \
    MTOMG_ROWS_SWITCH(sw.rows, hipLaunchKernelGGL((k_presmooth<T, F, C, RR>), grid_of(sw), dim3(WG_THREADS), 0, \
                                                   st, op, mat, sw, b, u_out, sweeps, cg, conv))
    if (cgmode) MTOMG_PRE(true, true)
    else if (fine) MTOMG_PRE(true, false)
    else MTOMG_PRE(false, false)
#undef MTOMG_PRE
}

template <typename T>
void launch_restrict(hipStream_t st, bool fine, bool check, LevelOp<T> op, Mat<T> mat, Sweep sw,
                     const T* b, const T* u, T* rc, const ConvCheck& chk, const int* conv) {
#define MTOMG_RES(F, C)                                                                              \
    MTOMG_ROWS_SWITCH(sw.rows, hipLaunchKernelGGL((k_restrict<T, F, C, RR>), grid_of(sw), dim3(WG_THREADS), 0, \
                                                   st, op, mat, sw, b, u, rc, chk, conv))
    if (check) MTOMG_RES(true, true)
    else if (fine) MTOMG_RES(true, false)
    else MTOMG_RES(false, false)
#undef MTOMG_RES
}

template <typename T>
void launch_post(hipStream_t st, bool fine, bool prolong, bool dot, LevelOp<T> op, Mat<T> mat, Sweep sw,
                 const T* u_in, const T* ec, const T* b, T* u_out, const double* r64, double* zr_out,
                 const int* conv) {
#define MTOMG_POST(F, P, D)                                                                          \
    MTOMG_ROWS_SWITCH(sw.rows, hipLaunchKernelGGL((k_post<T, F, P, D, RR>), grid_of(sw), dim3(WG_THREADS), 0, \
                                                   st, op, mat, sw, u_in, ec, b, u_out, r64, zr_out, conv))
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
void launch_apply(hipStream_t st, bool fine, bool diag, LevelOp<T> op, Mat<T> mat, Sweep sw, const T* u,
                  T* q) {
#define MTOMG_APP(F, D)                                                                              \
    MTOMG_ROWS_SWITCH(sw.rows, hipLaunchKernelGGL((k_apply<T, F, D, RR>), grid_of(sw), dim3(WG_THREADS), 0, st, \
                                                   op, mat, sw, u, q))
    if (fine) { if (diag) MTOMG_APP(true, true) else MTOMG_APP(true, false) }
    else { if (diag) MTOMG_APP(false, true) else MTOMG_APP(false, false) }
#undef MTOMG_APP
}

template <typename T>
void launch_coarse_solve(hipStream_t st, const double* Ainv, int n0, int ld, int nx0, const T* b, T* e,
                         const int* conv) {
    const int nblk = (n0 + WAVES_PER_WG - 1) / WAVES_PER_WG;
    hipLaunchKernelGGL((k_coarse_solve<T>), dim3(nblk), dim3(WG_THREADS), n0 * sizeof(double), st, Ainv,
                       n0, ld, nx0, b, e, conv);
}

#define MTOMG_INST(T)                                                                              \
    template void launch_presmooth<T>(hipStream_t, bool, bool, LevelOp<T>, Mat<T>, Sweep, const T*, T*, \
                                      int, const CgRhs&, const int*);                              \
    template void launch_restrict<T>(hipStream_t, bool, bool, LevelOp<T>, Mat<T>, Sweep, const T*,    \
                                     const T*, T*, const ConvCheck&, const int*);                  \
    template void launch_post<T>(hipStream_t, bool, bool, bool, LevelOp<T>, Mat<T>, Sweep, const T*,  \
                                 const T*, const T*, T*, const double*, double*, const int*);      \
    template void launch_apply<T>(hipStream_t, bool, bool, LevelOp<T>, Mat<T>, Sweep, const T*, T*);  \
    template void launch_coarse_solve<T>(hipStream_t, const double*, int, int, int, const T*, T*, const int*);
MTOMG_INST(float)
MTOMG_INST(double)
#undef MTOMG_INST

}  // namespace mtomg
