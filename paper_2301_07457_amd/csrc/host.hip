// Host side of the C ABI declared in include/mtomg.h: contexts, workspace
// layout, preconditioner setup and the PCG driver (Algorithm 2 with the
// multigrid cycle of Algorithm 1 as preconditioner).
//
// Batching.  Designs with the same grid, hierarchy, smoother, material law
// and number of load cases form a group; every (design, load case) pair of
// a group is one system.  Each system's vectors live in a case slab and
// each design's operators in a design slab, all slabs of a group the same
// size, so one launch serves every system of the group (blockIdx.y picks
// the system and the kernels shift their pointers by whole slabs).  All
// groups iterate in lockstep in one solve, and two PCG iterations of every
// group are captured in one HIP graph.  The coarsest factorisation of a
// design whose densities changed runs on a side stream: started by
// set_densities when the design is alone in its group, else at the start of
// the next solve with the other changed designs of its group (one launch
// sequence per group); the first coarse solve waits for it.
//
// Solve loop.  All PCG scalars stay on the device: every kernel that needs
// alpha = rho / p^T q or beta = rho_i / rho_{i-1} re-sums the per-workgroup
// partial dot products of the kernel that produced them, in a fixed order,
// so the run is deterministic and needs no host round trip.  Partial
// buffers and the r / p vectors alternate by iteration parity.  A small
// per-system state word carries convergence: 0 running, 1 converged (the
// last x update is pending), 2 finished, 3 breakdown, 4 NaN, 5 not part of
// this solve; every kernel exits at once when it is set, so the host can
// launch iterations in batches and read the states only between batches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mtomg.h"
#include "filter_kernels.h"
#include "kernels.h"
#include "oc_kernels.h"
#include "poisson_kernels.h"
#include "probe_kernels.h"

using namespace mtomg;

namespace {

constexpr int MAX_PHASES = 8;
constexpr int ST_INACTIVE = 5;

struct LevelBufs {
    int nx = 0, ny = 0;
    double* op64 = nullptr;   // E (finest) or 6 moment planes
    float* op32 = nullptr;    // FP32 copy for the FP32 cycle
    Sweep sw_apply{}, sw_pre{}, sw_res{}, sw_post{};
    Sweep sw_cg{};      // outer-CG apply (finest level)
    Sweep sw_post2{};   // two fused post-smoothing sweeps
    Sweep sw_rp{};      // restriction fused with the next level's pre-smoothing (coarse geometry)
    Sweep sw_pr{};      // two pre-smoothing sweeps fused with the restriction (coarse geometry, <= 4 rows)
    size_t nodes() const { return (size_t)(nx + 1) * (ny + 1); }
};

struct CaseBufs {
    const double* F = nullptr;   // caller-owned load of this case
    double* U = nullptr;         // caller-owned displacement of this case
    double *r[2] = {nullptr, nullptr}, *p[2] = {nullptr, nullptr}, *q = nullptr;
    void* z = nullptr;
    float* r32 = nullptr;
    std::vector<void*> b, u2, u4, e;   // per level, precision of the cycle
    double *zr[2] = {nullptr, nullptr}, *pq[2] = {nullptr, nullptr}, *rr[2] = {nullptr, nullptr};
    double *ff = nullptr, *trr = nullptr, *sums = nullptr, *cpart = nullptr;
    int* state = nullptr;   // [0] state word, [1] iterations
};

struct Design {
    bool has_grid = false, has_dens = false;
    bool needs_factor = false;   // densities set since the last factorisation
    bool fac_launched = false;   // its factorisation is queued on the side stream, not yet finalised
    bool fac_failed = false;     // coarsest matrix not positive definite
    int dens_seq = 0;            // number of the last set_densities call (1 .. 2^29 - 1)
    int x_code = 0;              // densities of that call: 0 valid, 1 outside [0, 1], 2 not finite
    int nelx = 0, nely = 0, m = 0, levels = 0, n_pre = 2, n_post = 2, precision = 0, n_cases = 1;
    double nu = 0.3, E_min = 1e-9, penal = 3.0, omega = 0.6;
    double E_phase[MAX_PHASES] = {};
    const double* F = nullptr;
    double* U = nullptr;
    std::vector<LevelBufs> lev;   // 0 = coarsest
    int n0 = 0, np0 = 0;   // coarsest free DOFs, padded to the block size
    double *A0 = nullptr, *W0 = nullptr, *Ainv = nullptr, *Dinv = nullptr, *Lbuf = nullptr, *Sacc = nullptr;
    int* chol_status = nullptr;   // [0] not positive definite, [1] factor pending, [2] input check (k_interp)
    std::vector<CaseBufs> cases;
    const double* x_dev = nullptr;
    int group = -1, gidx = 0;     // group and position in it
    float t_setup_ms = 0.f;
    hipEvent_t ev[2] = {nullptr, nullptr};   // around the last set_densities
    hipEvent_t fev[2] = {nullptr, nullptr};  // around the last factorisation of its group (group lead)
    int fine() const { return levels - 1; }
    bool mixed() const { return precision == MTOMG_FP32MG; }
    // partial sums of z.r come from the last post-smoothing launch: a fused
    // pair when n_post is even and positive, a single sweep otherwise
    int zr_tiles() const {
        const LevelBufs& L = lev[fine()];
        return (n_post >= 2 && n_post % 2 == 0) ? L.sw_post2.n_tiles : L.sw_post.n_tiles;
    }
};

// Designs solved together (same shape); see the file comment.
struct Group {
    std::vector<int> designs;
    int cpd = 1, n_sys = 0;
    long long cs = 0, ds = 0;   // case / design slab bytes
    const double** Ftab = nullptr;   // device [n_sys]
    double** Utab = nullptr;         // device [n_sys]
    Batch batch() const {
        Batch b;
        b.cs = cs;
        b.ds = ds;
        b.cpd = cpd;
        b.n = n_sys;
        b.F = Ftab;
        b.U = Utab;
        return b;
    }
};

// Event brackets around the launches of one kernel (profiling hook).
struct Prof {
    int kernel = 0;
    std::vector<hipEvent_t> ev;
    int used = 0;
    // exactly one kernel launch happens between begin and end; it stamps
    // the two events from its own dispatch
    void begin(int id, hipStream_t) {
        if (id != kernel || used + 2 > (int)ev.size()) return;
        time_next_launch(ev[used], ev[used + 1]);
    }
    void end(int id, hipStream_t) {
        if (id != kernel || used + 2 > (int)ev.size()) return;
        used += 2;
    }
};

}  // namespace

struct mtomg_ctx {
    Prof prof;
    hipStream_t stream = nullptr;
    int device = 0;
    std::vector<Design> d;
    std::vector<Group> groups;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    bool ws_owned = false;
    bool laid_out = false;
    std::string err;
    int* host_state = nullptr;    // pinned [cap][4]
    double* host_sums = nullptr;  // pinned [cap][4]
    int host_cap = 0;
    int batch = 8;                // iterations between host checks (first solve)
    int last_iters = 0;           // most iterations of the previous solve (batch hint)
    bool use_graphs = true;
    bool dense_factor = false;   // coarsest factorisation by the dense block sequence
    int rows_fine = 0, rows_coarse = 0;   // rows per wave overrides (0 = automatic)
    int rows_cg = 0;                      // rows per wave of the outer-CG apply (0 = automatic)
    int rows_depth[16] = {};              // per grid k levels below the finest (0 = rows_coarse)
    int max_restarts = 4;                 // PCG restarts after a failed true-residual check
    int gamma = 1;                        // cycle index of Algorithm 1: 1 V-cycle, 2 W-cycle
    bool fuse_pre = true;                 // MTOMG_OPT_FUSE_PRE
    double* filt_tab = nullptr;           // device weight table of mtomg_filter (FILTER_TAB_MAX doubles)
    double* filt_host = nullptr;          // pinned staging copy of it
    double filt_rf = -1.0;                // radius the table holds
    double* pois_buf = nullptr;           // mtomg_poisson_solve workspace
    size_t pois_bytes = 0;
    double* pois_host = nullptr;          // pinned copies of its scalars
    hipGraphExec_t pois_exec = nullptr;   // two Poisson PCG iterations (parities 1, 2)
    std::vector<double> pois_key;         // what pois_exec was captured for
    int pois_last_n = 0, pois_last_iters = 0;   // the previous Poisson solve (first batch hint)
    double* oc_buf = nullptr;             // OC update and optimisation-step workspace (grown on demand)
    size_t oc_bytes = 0;
    double* oc_host = nullptr;            // pinned: compliance per pair and load case, change, state
    size_t oc_host_bytes = 0;
    hipStream_t cap_stream = nullptr;     // capture stream (default priority)
    hipStream_t side_stream = nullptr;    // coarsest factorisations during a solve (default priority)
    hipStream_t br_st[4] = {};            // concurrent branches of the shape groups (default priority; [0] unused)
    hipEvent_t br_fork = nullptr, br_join[4] = {};
    hipEvent_t ev_fac[2] = {nullptr, nullptr};   // [0] main -> side, [1] side -> main
    bool fac_inflight = false;   // ev_fac[1] marks factorisations queued by set_densities
    int* host_chol = nullptr;             // pinned [cap][4]: coarsest-factor flags
    hipGraphExec_t pair_exec = nullptr;   // two PCG iterations (parities 1, 0) of the groups below
    double pair_tol2 = -1.0;
    std::vector<int> pair_groups;
    hipEvent_t ev_solve[2] = {nullptr, nullptr};
};

namespace {

int fail(mtomg_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

void drop_graphs(mtomg_ctx* c) {
    if (c->pair_exec) {
        hipGraphExecDestroy(c->pair_exec);
        c->pair_exec = nullptr;
    }
    c->pair_tol2 = -1.0;
    c->pair_groups.clear();
}

#define HIPCHK(ctx, call)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(ctx, MTOMG_HIP_ERROR, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define LAUNCHCHK(ctx)                                                                      \
    do {                                                                                    \
        hipError_t e_ = hipGetLastError();                                                  \
        if (e_ != hipSuccess)                                                               \
            return fail(ctx, MTOMG_HIP_ERROR, std::string("kernel launch: ") + hipGetErrorString(e_)); \
    } while (0)

// ----------------------------------------------------------------------------
// launch geometry
// ----------------------------------------------------------------------------
int pick_rows(int strips, int rows_total) {
    // rows per wave in {1, 2, 4}: the largest that still gives enough waves
    // to fill 256 CUs a few times over (8 only on request: its register
    // footprint lowers occupancy)
    int R = 4;
    while (R > 1 && (long)strips * ((rows_total + R - 1) / R) < 4096) R >>= 1;
    return R;
}

Sweep make_sweep(int cols, int wout, int rows_total, int R = 0) {
    Sweep s;
    s.n_strips = (cols + wout - 1) / wout;
    s.rows = R > 0 ? R : pick_rows(s.n_strips, rows_total);
    const int chunks = (rows_total + s.rows - 1) / s.rows;
    s.n_tiles = s.n_strips * ((chunks + WAVES_PER_WG - 1) / WAVES_PER_WG);
    return s;
}

void plan_level(LevelBufs& L, int R = 0, int Rcg = 0) {
    // The outer-CG apply has its own knob (Rcg), not R.  Automatic choice as
    // for the sweeps: at 1024^2, 4 rows per wave measured 19.8 us per launch
    // against 21.4 us with 8 (fewer waves in flight).
    L.sw_cg = make_sweep(L.nx + 1, 62, L.ny + 1, Rcg);
    L.sw_apply = make_sweep(L.nx + 1, 62, L.ny + 1, R);
    L.sw_post = L.sw_apply;
    L.sw_post2 = make_sweep(L.nx + 1, 60, L.ny + 1, R);
    L.sw_pre = make_sweep(L.nx + 1, 61, L.ny + 1, R);
    if (L.nx % 2 == 0 && L.ny % 2 == 0) {
        L.sw_res = make_sweep(L.nx / 2 + 1, 30, L.ny / 2 + 1, R);
        L.sw_rp = make_sweep(L.nx / 2 + 1, 28, L.ny / 2 + 1, R);
        L.sw_pr = make_sweep(L.nx / 2 + 1, 28, L.ny / 2 + 1, R);
        if (L.sw_pr.rows > 4) L.sw_pr = make_sweep(L.nx / 2 + 1, 28, L.ny / 2 + 1, 4);
    }
}



// Rows per wave of every level of a design from the context's knobs.
void plan_design(const int rows_fine, const int rows_coarse, const int rows_cg, const int* rows_depth, Design& d) {
    for (int l = 0; l < d.levels; ++l) {
        const int k = d.levels - 1 - l;   // levels below the finest
        const int R = k == 0 ? rows_fine : (rows_depth[k] ? rows_depth[k] : rows_coarse);
        plan_level(d.lev[l], R, k == 0 ? rows_cg : 0);
    }
}

// ----------------------------------------------------------------------------
// workspace layout (bump allocation; a null base only measures)
// ----------------------------------------------------------------------------
struct Bump {
    char* base;
    size_t off = 0;
    template <typename T> T* take(size_t n) {
        off = (off + 255) & ~(size_t)255;
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += n * sizeof(T);
        return p;
    }
};

// operators and the coarsest factorisation of one design
void layout_design_slab(Design& d, Bump& B) {
    const bool mx = d.mixed();
    for (int l = 0; l < d.levels; ++l) {
        LevelBufs& L = d.lev[l];
        const size_t ne = (size_t)L.nx * L.ny;
        const bool fine = l == d.fine();
        L.op64 = B.take<double>(fine ? ne : 6 * ne);
        L.op32 = mx ? B.take<float>(fine ? ne : 6 * ne) : nullptr;
    }
    d.A0 = B.take<double>((size_t)d.np0 * d.np0);
    d.W0 = B.take<double>((size_t)d.np0 * d.np0);
    d.Ainv = B.take<double>((size_t)d.np0 * d.np0);
    d.Dinv = B.take<double>((size_t)d.np0 * COARSE_NB);
    d.Lbuf = B.take<double>((size_t)d.np0 * d.np0);
    d.Sacc = B.take<double>((size_t)d.np0 * d.np0);
    d.chol_status = B.take<int>(4);
}

// vectors, partial sums and state of one load case
void layout_case_slab(const Design& d, CaseBufs& c, Bump& B) {
    const bool mx = d.mixed();
    const size_t tsz = mx ? sizeof(float) : sizeof(double);
    const LevelBufs& Lf = d.lev[d.fine()];
    const size_t nf = Lf.nodes() * 2;
    const int np = std::max({Lf.sw_apply.n_tiles, Lf.sw_cg.n_tiles, Lf.sw_pre.n_tiles, Lf.sw_post.n_tiles,
                             Lf.sw_post2.n_tiles, Lf.sw_pr.n_tiles, 1});
    // partial-sum arrays: n partials and, for z.r and p.q, their total after them
    for (int k = 0; k < 2; ++k) {
        c.r[k] = B.take<double>(nf);
        c.p[k] = B.take<double>(nf);
        c.zr[k] = B.take<double>(np + 1);
        c.pq[k] = B.take<double>(np + 1);
        c.rr[k] = B.take<double>(np);
    }
    c.q = B.take<double>(nf);
    c.z = B.take<char>(nf * tsz);
    c.r32 = mx ? B.take<float>(nf) : nullptr;
    c.ff = B.take<double>(np);
    c.trr = B.take<double>(np);
    c.cpart = B.take<double>(DOT_PARTS_MAX);
    c.sums = B.take<double>(8);
    c.state = B.take<int>(4);
    c.b.assign(d.levels, nullptr);
    c.u2.assign(d.levels, nullptr);
    c.u4.assign(d.levels, nullptr);
    c.e.assign(d.levels, nullptr);
    for (int l = 0; l < d.levels; ++l) {
        const size_t n = d.lev[l].nodes() * 2 * tsz;
        if (l != d.fine()) {
            c.b[l] = B.take<char>(n);
            c.e[l] = B.take<char>(n);
        }
        if (l != 0) {
            c.u2[l] = B.take<char>(n);
            c.u4[l] = B.take<char>(n);
        }
    }
}

bool same_shape(const Design& a, const Design& b) {
    return a.nelx == b.nelx && a.nely == b.nely && a.levels == b.levels && a.precision == b.precision &&
           a.n_pre == b.n_pre && a.n_post == b.n_post && a.nu == b.nu && a.omega == b.omega &&
           a.n_cases == b.n_cases;
}

void form_groups(std::vector<Design>& D, std::vector<Group>& G) {
    G.clear();
    for (int i = 0; i < (int)D.size(); ++i) {
        if (!D[i].has_grid) continue;
        int gi = -1;
        for (int k = 0; k < (int)G.size(); ++k)
            if (same_shape(D[G[k].designs[0]], D[i])) {
                gi = k;
                break;
            }
        if (gi < 0) {
            G.emplace_back();
            gi = (int)G.size() - 1;
            G[gi].cpd = D[i].n_cases;
        }
        D[i].group = gi;
        D[i].gidx = (int)G[gi].designs.size();
        G[gi].designs.push_back(i);
        G[gi].n_sys += D[i].n_cases;
    }
}

// Groups, then per group: F/U tables, design slabs, case slabs.  Returns
// the bytes used; with a null base only sizes are computed (on copies).
size_t layout_into(std::vector<Design>& D, std::vector<Group>& G, char* base) {
    form_groups(D, G);
    Bump B{base};
    for (Group& g : G) {
        {
            Design tmp = D[g.designs[0]];
            Bump m{nullptr};
            layout_design_slab(tmp, m);
            g.ds = (long long)((m.off + 255) & ~(size_t)255);
            CaseBufs cb;
            Bump mc{nullptr};
            layout_case_slab(tmp, cb, mc);
            g.cs = (long long)((mc.off + 255) & ~(size_t)255);
        }
        g.Ftab = B.take<const double*>(g.n_sys);
        g.Utab = B.take<double*>(g.n_sys);
        char* dbase = B.take<char>((size_t)g.ds * g.designs.size());
        char* cbase = B.take<char>((size_t)g.cs * g.n_sys);
        for (size_t gi = 0; gi < g.designs.size(); ++gi) {
            Design& d = D[g.designs[gi]];
            Bump bd{base ? dbase + gi * g.ds : nullptr};
            layout_design_slab(d, bd);
            const size_t nf = 2 * d.lev[d.fine()].nodes();
            for (int k = 0; k < d.n_cases; ++k) {
                CaseBufs& cb = d.cases[k];
                Bump bc{base ? cbase + (gi * g.cpd + k) * g.cs : nullptr};
                layout_case_slab(d, cb, bc);
                cb.F = d.F + k * nf;
                cb.U = d.U + k * nf;
            }
        }
    }
    return B.off + 256;
}

size_t measure_workspace(const mtomg_ctx* c) {
    std::vector<Design> D = c->d;
    std::vector<Group> G;
    return layout_into(D, G, nullptr);
}

int ensure_workspace(mtomg_ctx* c) {
    if (c->laid_out) return MTOMG_OK;
    const size_t need = measure_workspace(c);
    if (c->ws && c->ws_bytes < need)
        return fail(c, MTOMG_WORKSPACE, "workspace smaller than mtomg_workspace_bytes()");
    if (!c->ws) {
        HIPCHK(c, hipMalloc(&c->ws, need));
        c->ws_bytes = need;
        c->ws_owned = true;
    }
    drop_graphs(c);
    layout_into(c->d, c->groups, reinterpret_cast<char*>(c->ws));
    int total = 0;
    for (Group& g : c->groups) {
        // input-check words start at zero (k_interp only raises them)
        launch_fill_strided(c->stream, c->d[g.designs[0]].chol_status + 2, g.ds, (int)g.designs.size(), 0);
        std::vector<const double*> F;
        std::vector<double*> U;
        for (int di : g.designs)
            for (const CaseBufs& cb : c->d[di].cases) {
                F.push_back(cb.F);
                U.push_back(cb.U);
            }
        HIPCHK(c, hipMemcpyAsync(g.Ftab, F.data(), F.size() * sizeof(F[0]), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(g.Utab, U.data(), U.size() * sizeof(U[0]), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        total += g.n_sys;
    }
    if (total > c->host_cap) {
        if (c->host_state) hipHostFree(c->host_state);
        if (c->host_sums) hipHostFree(c->host_sums);
        if (c->host_chol) hipHostFree(c->host_chol);
        c->host_state = nullptr;
        c->host_sums = nullptr;
        c->host_chol = nullptr;
        c->host_cap = 0;
        HIPCHK(c, hipHostMalloc((void**)&c->host_state, (size_t)total * 4 * sizeof(int), hipHostMallocDefault));
        HIPCHK(c, hipHostMalloc((void**)&c->host_sums, (size_t)total * 4 * sizeof(double), hipHostMallocDefault));
        HIPCHK(c, hipHostMalloc((void**)&c->host_chol, (size_t)total * 4 * sizeof(int), hipHostMallocDefault));
        c->host_cap = total;
    }
    c->laid_out = true;
    return MTOMG_OK;
}

template <typename T> Mat<T> make_mat(const Design& d, double omega) {
    const double cc = 1.0 / (1.0 - d.nu * d.nu);
    return Mat<T>{(T)cc, (T)(cc * d.nu), (T)(cc * (1.0 - d.nu) / 2.0), (T)omega};
}

template <typename T> LevelOp<T> level_op(const Design& d, int l) {
    const LevelBufs& L = d.lev[l];
    if constexpr (sizeof(T) == 4) return LevelOp<T>{L.nx, L.ny, L.op32};
    else return LevelOp<T>{L.nx, L.ny, L.op64};
}

Phases phases_of(const Design& d) {
    Phases ph{};
    for (int k = 0; k < d.m; ++k) ph.dE[k] = d.E_phase[k] - d.E_min;
    ph.m = d.m;
    ph.E_min = d.E_min;
    ph.penal = d.penal;
    return ph;
}

// ----------------------------------------------------------------------------
// multigrid cycle on one case
// ----------------------------------------------------------------------------
template <typename T> struct CycleCtx {
    Design* d;
    CaseBufs* c;
    hipStream_t st;
    const int* conv;   // nullable (debug use)
    Prof* prof = nullptr;
    Batch bt{};        // systems of every launch (pointers above are system 0's)
    hipEvent_t wait_coarse = nullptr;   // the coarse solve waits for it (coarsest factors ready)
    int gamma = 1;                      // coarse-grid visits per level (Algorithm 1)
    bool fuse = true;                   // pre-smoothing fused with the restriction where it pays
    void begin(int id) { if (prof) prof->begin(id, st); }
    void end(int id) { if (prof) prof->end(id, st); }
};

// n sweeps of the post-smoother chain; returns the buffer holding the result
template <typename T>
void post_chain(CycleCtx<T>& cx, int l, const T* u_cur, const T* ec, const T* b, T* out, T* t0, T* t1,
                bool dot, const double* r64, double* zr_out) {
    Design& d = *cx.d;
    const bool fine = l == d.fine();
    const LevelOp<T> op = level_op<T>(d, l);
    const LevelBufs& L = d.lev[l];
    const int n = d.n_post;
    if (n == 0) {
        launch_post<T>(cx.st, fine, true, dot, op, make_mat<T>(d, 0.0), L.sw_post, u_cur, ec, b, out, r64, zr_out, cx.conv,
                       cx.bt);
        return;
    }
    // pairs of sweeps in one launch, a single sweep for an odd remainder
    const T* in = u_cur;
    for (int k = 0; k < n;) {
        const int step = (n - k >= 2) ? 2 : 1;
        const bool first = k == 0, last = k + step == n;
        T* dst = last ? out : ((in == t0) ? t1 : t0);
        const int pid = !fine ? 0 : (last ? MTOMG_KERNEL_FINE_POST_DOT : MTOMG_KERNEL_FINE_POST);
        cx.begin(pid);
        if (step == 2)
            launch_post2<T>(cx.st, fine, first, dot && last, op, make_mat<T>(d, d.omega), L.sw_post2, in,
                            first ? ec : nullptr, b, dst, r64, zr_out, cx.conv, cx.bt);
        else
            launch_post<T>(cx.st, fine, first, dot && last, op, make_mat<T>(d, d.omega), L.sw_post, in,
                           first ? ec : nullptr, b, dst, r64, zr_out, cx.conv, cx.bt);
        cx.end(pid);
        in = dst;
        k += step;
    }
}

// Extra pre-smoothing sweeps after the fused first two; returns current buffer.
template <typename T>
T* pre_chain_extra(CycleCtx<T>& cx, int l, T* cur, const T* b, T* t0, T* t1) {
    Design& d = *cx.d;
    const bool fine = l == d.fine();
    for (int k = 3; k <= d.n_pre; ++k) {
        T* dst = (cur == t0) ? t1 : t0;
        launch_post<T>(cx.st, fine, false, false, level_op<T>(d, l), make_mat<T>(d, d.omega), d.lev[l].sw_post,
                       cur, nullptr, b, dst, nullptr, nullptr, cx.conv, cx.bt);
        cur = dst;
    }
    return cur;
}

// Residual restriction from level l to l-1.  When level l-1 has a smoother
// (l - 1 >= 1) and is small, the same launch also runs its first
// pre-smoothing sweeps from zero into u2[l-1]; returns whether it did.
// The fused kernel re-forms two halo rows of the restriction per wave, so
// it only pays where launches, not bytes, dominate: up to 32768 coarse
// nodes summed over the systems of the launch.
constexpr long FUSE_MAX_COARSE_NODES = 32768;
// Pairs of post-smoothers in one launch (k_post2_pair) re-form the rows of
// level l that each wave's prolongation needs, so they pay up to a level
// l+1 of this many nodes summed over the systems of the launch.
constexpr long PAIR_MAX_NODES = 70000;

// Two pre-smoothing sweeps fused with the restriction (k_pre_restrict) on
// level l of a V-cycle, where the restriction is not already fused with the
// pre-smoothing of level l-1 (which removes more launches).
template <typename T>
bool use_pre_restrict(const CycleCtx<T>& cx, int l) {
    const Design& d = *cx.d;
    const bool rp = l - 1 >= 1 && (long)d.lev[l - 1].nodes() * cx.bt.n <= FUSE_MAX_COARSE_NODES;
    return cx.fuse && cx.gamma == 1 && d.n_pre == 2 && l >= 1 && !rp;
}
// The finest grid's pre-smoothing, restriction and CG update in one launch.
// The convergence test then moves to the first launch on the level below,
// which must be a k_pre_restrict too: level f-2 is the coarsest or too big
// for the restriction-presmoothing fusion for any number of systems.
bool fine_fused(bool fuse, int gamma, const Design& d) {
    if (!fuse || gamma != 1 || d.levels < 3 || d.n_pre != 2) return false;
    return d.levels == 3 || (long)d.lev[d.fine() - 2].nodes() > FUSE_MAX_COARSE_NODES;
}
// partial sums of ||r||^2 of a PCG iteration: from the fused launch or k_presmooth
int rr_tiles(bool fuse, int gamma, const Design& d) {
    const LevelBufs& L = d.lev[d.fine()];
    return fine_fused(fuse, gamma, d) ? L.sw_pr.n_tiles : L.sw_pre.n_tiles;
}
template <typename T>
bool restrict_down(CycleCtx<T>& cx, int l, const T* b, const T* u, bool check, const ConvCheck& chk) {
    Design& d = *cx.d;
    CaseBufs& c = *cx.c;
    const bool fine = l == d.fine();
    const bool fuse = l - 1 >= 1 && d.n_pre > 0 &&
                      (long)d.lev[l - 1].nodes() * cx.bt.n <= FUSE_MAX_COARSE_NODES;
    if (fuse)
        launch_restrict_pre<T>(cx.st, fine, check, level_op<T>(d, l), level_op<T>(d, l - 1), make_mat<T>(d, d.omega),
                               d.lev[l].sw_rp, b, u, (T*)c.b[l - 1], (T*)c.u2[l - 1], std::min(d.n_pre, 2), chk,
                               cx.conv, cx.bt);
    else
        launch_restrict<T>(cx.st, fine, check, level_op<T>(d, l), make_mat<T>(d, d.omega), d.lev[l].sw_res, b, u,
                           (T*)c.b[l - 1], chk, cx.conv, cx.bt);
    return fuse;
}

// Levels top .. 0 of Algorithm 1 given the restricted right-hand side in
// c.b[top] (and, when top_pre, its first pre-smoothing sweeps already in
// u2[top]); leaves the coarse correction in c.e[top].  The pre-smoothed
// iterate of each level stays in u2 or u4 (which one depends on the number
// of sweeps only), so a captured launch sequence is the same every time.
template <typename T>
void coarse_cycle(CycleCtx<T>& cx, int top, bool top_pre, const ConvCheck* chk) {
    Design& d = *cx.d;
    CaseBufs& c = *cx.c;
    ConvCheck nochk{};
    CgRhs nocg{};
    T* pre[16] = {};
    bool pre_done = top_pre;
    for (int l = top; l >= 1; --l) {
        T* b = (T*)c.b[l];
        T* t0 = (T*)c.u2[l];
        T* t1 = (T*)c.u4[l];
        T* cur = t0;
        if (!pre_done && use_pre_restrict(cx, l)) {
            // with chk (top level below a fused finest grid) the convergence test runs here
            const bool check = chk && l == top;
            launch_pre_restrict<T>(cx.st, false, false, check, level_op<T>(d, l), make_mat<T>(d, d.omega),
                                   d.lev[l].sw_pr, b, t0, (T*)c.b[l - 1], nocg, check ? *chk : nochk, cx.conv,
                                   cx.bt);
            pre[l] = t0;
            continue;
        }
        if (d.n_pre > 0) {
            if (!pre_done)
                launch_presmooth<T>(cx.st, false, false, level_op<T>(d, l), make_mat<T>(d, d.omega), d.lev[l].sw_pre,
                                    b, t0, std::min(d.n_pre, 2), nocg, cx.conv, cx.bt);
            cur = pre_chain_extra<T>(cx, l, cur, b, t0, t1);
        }
        pre_done = restrict_down<T>(cx, l, b, d.n_pre > 0 ? cur : nullptr, false, nochk);
        pre[l] = cur;
    }
    if (cx.wait_coarse) hipStreamWaitEvent(cx.st, cx.wait_coarse, 0);
    cx.begin(MTOMG_KERNEL_COARSE_SOLVE);
    launch_coarse_solve<T>(cx.st, d.Ainv, d.n0, d.np0, d.lev[0].nx, (const T*)c.b[0], (T*)c.e[0], cx.conv, cx.bt);
    cx.end(MTOMG_KERNEL_COARSE_SOLVE);
    for (int l = 1; l <= top;) {
        // two sweeps per level and a small level l+1: one launch for levels l and l+1
        if (d.n_post == 2 && l + 1 <= top && (long)d.lev[l + 1].nodes() * cx.bt.n <= PAIR_MAX_NODES) {
            launch_post2_pair<T>(cx.st, level_op<T>(d, l), level_op<T>(d, l + 1), make_mat<T>(d, d.omega),
                                 d.lev[l + 1].sw_post2, d.n_pre > 0 ? pre[l] : nullptr, (const T*)c.e[l - 1],
                                 (const T*)c.b[l], d.n_pre > 0 ? pre[l + 1] : nullptr, (const T*)c.b[l + 1],
                                 (T*)c.e[l + 1], cx.conv, cx.bt);
            l += 2;
            continue;
        }
        T* other = pre[l] == (T*)c.u2[l] ? (T*)c.u4[l] : (T*)c.u2[l];
        post_chain<T>(cx, l, d.n_pre > 0 ? pre[l] : nullptr, (const T*)c.e[l - 1], (const T*)c.b[l], (T*)c.e[l],
                      other, pre[l], false, nullptr, nullptr);
        ++l;
    }
}

// n_pre damped Jacobi sweeps on level l from a nonzero iterate `in`
// (never written), ping-ponging between t0 and t1; returns the buffer
// holding the result.  With n_pre = 0 the iterate is copied into t0 (a
// sweep with omega = 0), so the caller may overwrite `in`.
template <typename T>
T* smooth_from(CycleCtx<T>& cx, int l, const T* in, const T* b, T* t0, T* t1) {
    Design& d = *cx.d;
    const LevelBufs& L = d.lev[l];
    const LevelOp<T> op = level_op<T>(d, l);
    if (d.n_pre == 0) {
        launch_post<T>(cx.st, false, false, false, op, make_mat<T>(d, 0.0), L.sw_post, in, nullptr, b, t0, nullptr,
                       nullptr, cx.conv, cx.bt);
        return t0;
    }
    const T* cur = in;
    T* dst = t0;
    for (int k = 0; k < d.n_pre;) {
        const int step = (d.n_pre - k >= 2) ? 2 : 1;
        if (step == 2)
            launch_post2<T>(cx.st, false, false, false, op, make_mat<T>(d, d.omega), L.sw_post2, cur, nullptr, b, dst,
                            nullptr, nullptr, cx.conv, cx.bt);
        else
            launch_post<T>(cx.st, false, false, false, op, make_mat<T>(d, d.omega), L.sw_post, cur, nullptr, b, dst,
                           nullptr, nullptr, cx.conv, cx.bt);
        cur = dst;
        dst = dst == t0 ? t1 : t0;
        k += step;
    }
    return const_cast<T*>(cur);
}

// One visit of coarse level l in a W-cycle (gamma = 2), Algorithm 1:
// pre-smooth on c.b[l] from zero (from_e = false; pre_done: the fused
// restriction above already did the first sweeps into u2[l]) or from the
// previous visit's result in c.e[l] (from_e = true), restrict the residual,
// visit level l-1 twice (its second visit starts from the first one's
// result), prolongate, correct and post-smooth into c.e[l].  Level 0 is the
// exact solve, which a second visit would repeat bit for bit, so it runs
// once per visit of level 1.
template <typename T>
void w_visit(CycleCtx<T>& cx, int l, bool from_e, bool pre_done) {
    Design& d = *cx.d;
    CaseBufs& c = *cx.c;
    if (l == 0) {
        if (cx.wait_coarse) {
            hipStreamWaitEvent(cx.st, cx.wait_coarse, 0);
            cx.wait_coarse = nullptr;   // one wait covers every later coarse solve on the stream
        }
        cx.begin(MTOMG_KERNEL_COARSE_SOLVE);
        launch_coarse_solve<T>(cx.st, d.Ainv, d.n0, d.np0, d.lev[0].nx, (const T*)c.b[0], (T*)c.e[0], cx.conv, cx.bt);
        cx.end(MTOMG_KERNEL_COARSE_SOLVE);
        return;
    }
    ConvCheck nochk{};
    CgRhs nocg{};
    T* b = (T*)c.b[l];
    T* t0 = (T*)c.u2[l];
    T* t1 = (T*)c.u4[l];
    T* cur = nullptr;
    if (from_e) {
        cur = smooth_from<T>(cx, l, (const T*)c.e[l], b, t0, t1);
    } else if (d.n_pre > 0) {
        if (!pre_done)
            launch_presmooth<T>(cx.st, false, false, level_op<T>(d, l), make_mat<T>(d, d.omega), d.lev[l].sw_pre, b,
                                t0, std::min(d.n_pre, 2), nocg, cx.conv, cx.bt);
        cur = pre_chain_extra<T>(cx, l, t0, b, t0, t1);
    }
    const bool sub_pre = restrict_down<T>(cx, l, b, cur, false, nochk);
    w_visit<T>(cx, l - 1, false, sub_pre);
    if (l - 1 >= 1) w_visit<T>(cx, l - 1, true, false);
    T* other = cur == t0 ? t1 : t0;
    post_chain<T>(cx, l, cur, (const T*)c.e[l - 1], b, (T*)c.e[l], other, cur ? cur : t1, false, nullptr, nullptr);
}

// Coarse-grid correction of the level above `top` into c.e[top]: levels
// top .. 0 of Algorithm 1 with cycle index cx.gamma (the V-cycle visits
// each level once, the W-cycle visits level top twice and recurses).
template <typename T>
void coarse_correction(CycleCtx<T>& cx, int top, bool top_pre, const ConvCheck* chk = nullptr) {
    if (cx.gamma == 1) {
        coarse_cycle<T>(cx, top, top_pre, chk);
        return;
    }
    w_visit<T>(cx, top, false, top_pre);
    if (top >= 1) w_visit<T>(cx, top, true, false);
}

// One preconditioner application on the finest grid inside PCG.
//   it < 0: initial cycle on r_0 (no residual update, writes rho_0)
//   it >= 0: iteration it: r_{it+1} = r_it - alpha q, then z_{it+1} = M^-1 r_{it+1}
template <typename T>
void fine_cycle(CycleCtx<T>& cx, int it, double tol2) {
    Design& d = *cx.d;
    CaseBufs& c = *cx.c;
    const int f = d.fine();
    const int par = it < 0 ? 0 : (it & 1);
    const int nxt = it < 0 ? 0 : 1 - par;
    const LevelBufs& L = d.lev[f];
    CgRhs cg{};
    cg.r_old = c.r[par];
    cg.q = c.q;
    cg.r_new = c.r[nxt];
    cg.r32 = c.r32;
    cg.zr = c.zr[par];
    cg.n_zr = d.zr_tiles();
    cg.pq = c.pq[par];
    cg.n_pq = L.sw_cg.n_tiles;
    cg.rr_out = c.rr[nxt];
    cg.update = it >= 0;
    cg.conv_rw = c.state;
    cg.iters = c.state + 1;
    T* t0 = (T*)c.u2[f];
    T* t1 = (T*)c.u4[f];
    const T* bfine = d.mixed() ? (const T*)(void*)c.r32 : (const T*)(void*)c.r[nxt];
    if (fine_fused(cx.fuse, cx.gamma, d)) {
        // pre-smoothing, restriction and the CG update of r in one launch;
        // the convergence test on its ||r||^2 partials opens level f-1
        cx.begin(MTOMG_KERNEL_FINE_PRESMOOTH);
        launch_pre_restrict<T>(cx.st, true, true, false, level_op<T>(d, f), make_mat<T>(d, d.omega), L.sw_pr,
                               nullptr, t0, (T*)c.b[f - 1], cg, ConvCheck{}, cx.conv, cx.bt);
        cx.end(MTOMG_KERNEL_FINE_PRESMOOTH);
        ConvCheck chk{};
        chk.rr = c.rr[nxt];
        chk.n_rr = it < 0 ? L.sw_apply.n_tiles : L.sw_pr.n_tiles;
        chk.ff = c.ff;
        chk.n_ff = L.sw_apply.n_tiles;
        chk.tol2 = tol2;
        chk.conv_rw = c.state;
        coarse_correction<T>(cx, f - 1, false, &chk);
        post_chain<T>(cx, f, t0, (const T*)c.e[f - 1], bfine, (T*)c.z, t1, t0, true, c.r[nxt],
                      c.zr[it < 0 ? 0 : nxt]);
        launch_partial_total(cx.st, c.zr[it < 0 ? 0 : nxt], d.zr_tiles(), cx.conv, cx.bt);
        return;
    }
    cx.begin(MTOMG_KERNEL_FINE_PRESMOOTH);
    launch_presmooth<T>(cx.st, true, true, level_op<T>(d, f), make_mat<T>(d, d.omega), L.sw_pre, nullptr, t0,
                        std::min(d.n_pre, 2), cg, cx.conv, cx.bt);
    cx.end(MTOMG_KERNEL_FINE_PRESMOOTH);
    T* cur = pre_chain_extra<T>(cx, f, t0, bfine, t0, t1);
    ConvCheck chk{};
    chk.rr = c.rr[nxt];
    chk.n_rr = it < 0 ? L.sw_apply.n_tiles : L.sw_pre.n_tiles;
    chk.ff = c.ff;
    chk.n_ff = L.sw_apply.n_tiles;
    chk.tol2 = tol2;
    chk.conv_rw = c.state;
    cx.begin(MTOMG_KERNEL_FINE_RESTRICT);
    const bool pre_done = restrict_down<T>(cx, f, bfine, d.n_pre > 0 ? cur : nullptr, true, chk);
    cx.end(MTOMG_KERNEL_FINE_RESTRICT);
    coarse_correction<T>(cx, f - 1, pre_done);
    post_chain<T>(cx, f, d.n_pre > 0 ? cur : nullptr, (const T*)c.e[f - 1], bfine, (T*)c.z, cur == t0 ? t1 : t0,
                  cur, true, c.r[nxt], c.zr[it < 0 ? 0 : nxt]);
    // z.r once, for the next CG apply (which would otherwise re-sum the
    // partials in every workgroup) and pre-smoother
    launch_partial_total(cx.st, c.zr[it < 0 ? 0 : nxt], d.zr_tiles(), cx.conv, cx.bt);
}

template <typename T>
void cg_step(CycleCtx<T>& cx, int it, int mode) {
    Design& d = *cx.d;
    CaseBufs& c = *cx.c;
    const LevelBufs& L = d.lev[d.fine()];
    const int par = it & 1, prv = 1 - par;
    cx.begin(MTOMG_KERNEL_CG_APPLY);
    launch_cg_apply<T>(cx.st, level_op<double>(d, d.fine()), make_mat<double>(d, d.omega), L.sw_cg,
                       (const T*)c.z, c.p[prv], c.p[par], c.U, c.q, c.zr[par], c.zr[prv], d.zr_tiles(),
                       c.pq[prv], L.sw_cg.n_tiles, c.pq[par], c.state, mode, cx.bt);
    cx.end(MTOMG_KERNEL_CG_APPLY);
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
namespace {

// One V-cycle M^-1 b from a zero iterate on `level` (test hook).
template <typename T>
int debug_vcycle(mtomg_ctx* ctx, Design& d, CaseBufs& cb, hipStream_t st, int level, const T* vin, T* vout) {
    const bool fine = level == d.fine();
    const size_t n = 2 * d.lev[level].nodes();
    T* bl = fine ? (T*)(d.mixed() ? (void*)cb.r32 : (void*)cb.r[0]) : (T*)cb.b[level];
    HIPCHK(ctx, hipMemcpyAsync(bl, vin, n * sizeof(T), hipMemcpyDeviceToDevice, st));
    const LevelOp<T> opT = level_op<T>(d, level);
    const Mat<T> mat = make_mat<T>(d, d.omega);
    CgRhs nocg{};
    ConvCheck nochk{};
    CycleCtx<T> cx{&d, &cb, st, nullptr};
    cx.gamma = ctx->gamma;
    cx.fuse = ctx->fuse_pre;
    T* t0 = (T*)cb.u2[level];
    T* t1 = (T*)cb.u4[level];
    T* cur = t0;
    if (d.n_pre > 0) {
        launch_presmooth<T>(st, fine, false, opT, mat, d.lev[level].sw_pre, bl, t0, std::min(d.n_pre, 2), nocg, nullptr);
        cur = pre_chain_extra<T>(cx, level, cur, bl, t0, t1);
    }
    const bool pre_done = restrict_down<T>(cx, level, bl, d.n_pre > 0 ? cur : nullptr, false, nochk);
    coarse_correction<T>(cx, level - 1, pre_done);
    post_chain<T>(cx, level, d.n_pre > 0 ? cur : nullptr, (const T*)cb.e[level - 1], bl, vout, cur == t0 ? t1 : t0,
                  cur, false, nullptr, nullptr);
    return MTOMG_OK;
}

int check_design(mtomg_ctx* c, int design, bool need_dens) {
    if (!c) return MTOMG_BAD_INPUT;
    if (design < 0 || design >= (int)c->d.size()) return fail(c, MTOMG_BAD_INPUT, "design index out of range");
    if (!c->d[design].has_grid) return fail(c, MTOMG_STATE, "set_grid not called for this design");
    if (need_dens && !c->d[design].has_dens) return fail(c, MTOMG_STATE, "set_densities not called for this design");
    return MTOMG_OK;
}

// algorithmic bytes of one PCG iteration of one system (each array touched once per kernel)
double model_bytes(const Design& d) {
    double bytes = 0.0;
    const double t = d.mixed() ? 4.0 : 8.0;
    for (int l = 0; l < d.levels; ++l) {
        const double n = (double)d.lev[l].nodes(), ne = (double)d.lev[l].nx * d.lev[l].ny;
        if (l == d.fine()) {
            bytes += n * 16 * 6 + ne * 8;                      // cg_apply: z,p_old,x in; p,q,x out; E
            bytes += n * 16 * 3 + (d.mixed() ? n * 8 : 0);     // r, q in; r out (+ r32)
            bytes += n * 2 * t * 5 + ne * t * 4 + n * 16;      // smoothing/transfer sweeps + r for dot
        } else if (l > 0) {
            bytes += n * 2 * t * 7 + ne * 6 * t * 4;
        } else {
            bytes += 8.0 * d.n0 * d.n0 + n * 2 * t * 2;
        }
    }
    return bytes;
}

// The dense coarsest matrix K_0 of a design from its level-0 moments, and
// its factorisation flags reset to {0, 1, 0, 0} (positive definite so far,
// factor this design).  The dense block factorisation overwrites K_0 with
// its trailing updates, so a factorisation that runs again needs this first.
void assemble_coarsest(hipStream_t st, Design& d) {
    launch_fill<double>(st, d.A0, (size_t)d.np0 * d.np0, 0.0);
    launch_assemble_dense(st, false, level_op<double>(d, 0), make_mat<double>(d, d.omega), d.A0, d.np0,
                          d.chol_status);
}

// Coarsest factorisation (Algorithm 3 and the explicit inverse) of every
// design whose densities changed since its last factorisation, on stream
// st: one launch sequence per group, designs not flagged skip it.  The
// positive-definiteness flags are copied to host_chol (row = design slot of
// the group's systems) and read by factor_finalize after a synchronisation.
// Returns whether anything was launched in *ran_any.
int factor_launch(mtomg_ctx* c, hipStream_t st, bool* ran_any, int only_group = -1) {
    *ran_any = false;
    int sys0 = 0;
    for (size_t gi = 0; gi < c->groups.size(); ++gi) {
        Group& g = c->groups[gi];
        bool ran = false;
        for (int di : g.designs) {
            const Design& d = c->d[di];
            ran = ran || (d.has_dens && d.needs_factor && !d.fac_launched);
        }
        if (ran && (only_group < 0 || only_group == (int)gi)) {
            for (int di : g.designs) {
                Design& d = c->d[di];
                if (d.has_dens && d.needs_factor) d.fac_launched = true;
            }
            *ran_any = true;
            Design& d0 = c->d[g.designs[0]];
            const int nd = (int)g.designs.size();
            HIPCHK(c, hipEventRecord(d0.fev[0], st));
            // DOFs 2 ((j-1)(nx+1) + i) + c: neighbouring nodes lie at most 2 nx + 5 apart
            const int half_bw = c->dense_factor ? 0 : 2 * d0.lev[0].nx + 5;
            launch_coarse_factor(st, d0.A0, d0.n0, d0.np0, d0.Dinv, d0.W0, d0.Ainv, d0.chol_status, d0.Lbuf,
                                 d0.Sacc, nd, g.ds, half_bw);
            launch_fill_strided(st, d0.chol_status + 1, g.ds, nd, 0);
            HIPCHK(c, hipEventRecord(d0.fev[1], st));
            LAUNCHCHK(c);
            HIPCHK(c, hipMemcpy2DAsync(c->host_chol + 4 * sys0, 4 * sizeof(int), d0.chol_status, (size_t)g.ds,
                                       4 * sizeof(int), nd, hipMemcpyDeviceToHost, st));
        }
        sys0 += g.n_sys;
    }
    return MTOMG_OK;
}

// After the factorisation has completed: flags and setup times per design.
int factor_finalize(mtomg_ctx* c) {
    int sys0 = 0;
    for (size_t gi = 0; gi < c->groups.size(); ++gi) {
        Group& g = c->groups[gi];
        bool ran = false;
        for (int di : g.designs) ran = ran || (c->d[di].has_dens && c->d[di].needs_factor && c->d[di].fac_launched);
        if (ran) {
            float fac_ms = 0.f;
            Design& d0 = c->d[g.designs[0]];
            HIPCHK(c, hipEventElapsedTime(&fac_ms, d0.fev[0], d0.fev[1]));
            for (size_t k = 0; k < g.designs.size(); ++k) {
                Design& d = c->d[g.designs[k]];
                if (!(d.has_dens && d.needs_factor && d.fac_launched)) continue;
                float ms = 0.f;
                HIPCHK(c, hipEventElapsedTime(&ms, d.ev[0], d.ev[1]));
                d.t_setup_ms = ms + fac_ms;
                d.fac_failed = c->host_chol[4 * (sys0 + k)] != 0;
                const int xv = c->host_chol[4 * (sys0 + k) + 2];
                d.x_code = (xv >> 2) == d.dens_seq ? (xv & 3) : 0;
                d.needs_factor = false;
                d.fac_launched = false;
            }
        }
        sys0 += g.n_sys;
    }
    return MTOMG_OK;
}

// Factorise now and wait (used outside the solve, e.g. by the test hook).
int factor_pending(mtomg_ctx* c) {
    bool ran = false;
    int rc = factor_launch(c, c->stream, &ran);
    if (rc) return rc;
    if (!ran && !c->fac_inflight) return MTOMG_OK;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipStreamSynchronize(c->side_stream));
    c->fac_inflight = false;
    return factor_finalize(c);
}

// Queued factorisations are dropped (the layout or the densities change).
void forget_factorisations(mtomg_ctx* c) {
    c->fac_inflight = false;
    for (Design& d : c->d) d.fac_launched = false;
}

template <typename T>
CycleCtx<T> group_cycle(mtomg_ctx* c, Group& g, hipStream_t st, Prof* prof) {
    Design& d0 = c->d[g.designs[0]];
    CycleCtx<T> cx{&d0, &d0.cases[0], st, d0.cases[0].state, prof};
    cx.bt = g.batch();
    cx.gamma = c->gamma;
    cx.fuse = c->fuse_pre;
    return cx;
}

// Shape groups of one solve run as up to MAX_BRANCHES concurrent branches:
// forked from the solve stream by an event, joined back by one event per
// branch (captured, they become parallel branches of the graph, which the
// runtime executes concurrently).  Their latency-bound coarse levels then
// overlap instead of queueing behind each other; a group's launches stay in
// order on its branch, so every result is the same as in one stream.
constexpr int MAX_BRANCHES = 4;
int ensure_branches(mtomg_ctx* c) {
    if (c->br_fork) return MTOMG_OK;
    for (int b = 1; b < MAX_BRANCHES; ++b) {
        HIPCHK(c, hipStreamCreateWithFlags(&c->br_st[b], hipStreamNonBlocking));
        HIPCHK(c, hipEventCreateWithFlags(&c->br_join[b], hipEventDisableTiming));
    }
    HIPCHK(c, hipEventCreateWithFlags(&c->br_fork, hipEventDisableTiming));
    return MTOMG_OK;
}

// PCG iteration `it` of every group in `act` (mode as k_cg_apply); one
// stream while a kernel is being profiled (its events are in launch order)
int run_iteration(mtomg_ctx* c, const std::vector<int>& act, hipStream_t st, int it, int mode, double tol2,
                  Prof* prof) {
    const int nb = (c->br_fork && c->prof.kernel == MTOMG_KERNEL_NONE)
                       ? std::min<int>((int)act.size(), MAX_BRANCHES) : 1;
    if (nb > 1) {
        HIPCHK(c, hipEventRecord(c->br_fork, st));
        for (int b = 1; b < nb; ++b) HIPCHK(c, hipStreamWaitEvent(c->br_st[b], c->br_fork, 0));
    }
    for (size_t k = 0; k < act.size(); ++k) {
        Group& g = c->groups[act[k]];
        hipStream_t gs = (nb > 1 && k % nb) ? c->br_st[k % nb] : st;
        if (c->d[g.designs[0]].mixed()) {
            CycleCtx<float> cx = group_cycle<float>(c, g, gs, prof);
            cg_step<float>(cx, it, mode);
            if (mode < 2) fine_cycle<float>(cx, it, tol2);
        } else {
            CycleCtx<double> cx = group_cycle<double>(c, g, gs, prof);
            cg_step<double>(cx, it, mode);
            if (mode < 2) fine_cycle<double>(cx, it, tol2);
        }
    }
    if (nb > 1) {
        for (int b = 1; b < nb; ++b) {
            HIPCHK(c, hipEventRecord(c->br_join[b], c->br_st[b]));
            HIPCHK(c, hipStreamWaitEvent(st, c->br_join[b], 0));
        }
    }
    return MTOMG_OK;
}

// Capture iterations 1 and 2 (parities 1, 0) of every group in `act` into
// one graph; replaying it runs any later pair of iterations.
int capture_pair(mtomg_ctx* c, const std::vector<int>& act, double tol2) {
    drop_graphs(c);
    hipStream_t cs = c->cap_stream;
    HIPCHK(c, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    int rc = MTOMG_OK;
    for (int k = 1; k <= 2 && rc == MTOMG_OK; ++k) rc = run_iteration(c, act, cs, k, 0, tol2, nullptr);
    hipGraph_t g = nullptr;
    HIPCHK(c, hipStreamEndCapture(cs, &g));
    if (rc) {
        if (g) hipGraphDestroy(g);
        return rc;
    }
    const hipError_t e = hipGraphInstantiate(&c->pair_exec, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) {
        c->pair_exec = nullptr;
        return fail(c, MTOMG_HIP_ERROR, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    c->pair_tol2 = tol2;
    c->pair_groups = act;
    return MTOMG_OK;
}

// r_0 = f - K u_0 and the first preconditioner application, every system of a group
template <typename T>
void start_group(mtomg_ctx* c, Group& g, hipStream_t st, int warm, double tol2, hipEvent_t wait_fac) {
    CycleCtx<T> cx = group_cycle<T>(c, g, st, &c->prof);
    cx.wait_coarse = wait_fac;
    Design& d = *cx.d;
    CaseBufs& cb = *cx.c;
    const LevelBufs& L = d.lev[d.fine()];
    launch_residual(st, level_op<double>(d, d.fine()), make_mat<double>(d, d.omega), L.sw_apply, nullptr, nullptr,
                    warm ? 1 : 0, cb.r[0], cb.rr[0], cb.ff, cb.state, cx.bt);
    fine_cycle<T>(cx, -1, tol2);
}

// One run of Algorithm 2 for every system whose host_state word is 0 on
// entry (5 = not part of this run), all groups in lockstep.  On return
// host_state holds each system's final state word and iteration count,
// host_sums its ||f||^2, recursive and true ||r||^2; *ms the device time.
int pcg_round(mtomg_ctx* c, const std::vector<int>& gsys0, double tol2, int max_iter, int warm, float* ms,
              hipEvent_t wait_fac) {
    hipStream_t st = c->stream;
    const bool graphs = c->use_graphs && c->prof.kernel == MTOMG_KERNEL_NONE;
    std::vector<int> act;
    for (size_t gi = 0; gi < c->groups.size(); ++gi) {
        Group& g = c->groups[gi];
        bool any = false;
        for (int q = 0; q < g.n_sys; ++q) any = any || c->host_state[4 * (gsys0[gi] + q)] == 0;
        if (any) {
            act.push_back((int)gi);
            HIPCHK(c, hipMemcpy2DAsync(c->d[g.designs[0]].cases[0].state, (size_t)g.cs, c->host_state + 4 * gsys0[gi],
                                       4 * sizeof(int), 4 * sizeof(int), g.n_sys, hipMemcpyHostToDevice, st));
        }
    }
    if (act.size() > 1) {
        const int r2 = ensure_branches(c);
        if (r2) return r2;
    }
    HIPCHK(c, hipEventRecord(c->ev_solve[0], st));
    auto read_states = [&]() -> int {
        for (int gi : act) {
            Group& g = c->groups[gi];
            HIPCHK(c, hipMemcpy2DAsync(c->host_state + 4 * gsys0[gi], 4 * sizeof(int),
                                       c->d[g.designs[0]].cases[0].state, (size_t)g.cs, 4 * sizeof(int), g.n_sys,
                                       hipMemcpyDeviceToHost, st));
        }
        HIPCHK(c, hipStreamSynchronize(st));
        return MTOMG_OK;
    };
    // after `it` iterations: the pending x update (mode 3 or 4 of k_cg_apply;
    // none for mode < 0), the true residual f - K u and the per-system sums,
    // then one synchronisation for the state words and sums
    auto finish = [&](int it_done, int mode) -> int {
        if (mode >= 0 && it_done > 0) {
            const int r2 = run_iteration(c, act, st, it_done, mode, tol2, &c->prof);
            if (r2) return r2;
        }
        for (int gi : act) {
            Group& g = c->groups[gi];
            Design& d = c->d[g.designs[0]];
            CaseBufs& cb = d.cases[0];
            const LevelBufs& L = d.lev[d.fine()];
            const Batch bt = g.batch();
            launch_residual(st, level_op<double>(d, d.fine()), make_mat<double>(d, d.omega), L.sw_apply, nullptr,
                            nullptr, 1, nullptr, cb.trr, nullptr, cb.state, bt);
            launch_solve_sums(st, cb.ff, L.sw_apply.n_tiles, cb.rr[0], cb.rr[1], L.sw_apply.n_tiles,
                              rr_tiles(c->fuse_pre, c->gamma, d), cb.trr, cb.state, cb.sums, bt);
        }
        LAUNCHCHK(c);
        HIPCHK(c, hipEventRecord(c->ev_solve[1], st));
        for (int gi : act) {
            Group& g = c->groups[gi];
            HIPCHK(c, hipMemcpy2DAsync(c->host_sums + 4 * gsys0[gi], 4 * sizeof(double),
                                       c->d[g.designs[0]].cases[0].sums, (size_t)g.cs, 3 * sizeof(double), g.n_sys,
                                       hipMemcpyDeviceToHost, st));
        }
        return read_states();
    };
    int rc = MTOMG_OK;
    int it = 0;
    if (!act.empty()) {
        for (int gi : act) {
            if (c->d[c->groups[gi].designs[0]].mixed()) start_group<float>(c, c->groups[gi], st, warm, tol2, wait_fac);
            else start_group<double>(c, c->groups[gi], st, warm, tol2, wait_fac);
        }
        LAUNCHCHK(c);
        // iterations [from, from + count): pairs starting at an odd index replay the graph
        auto launch_iters = [&](int from, int count) -> int {
            int k = from;
            const int end = from + count;
            while (k < end) {
                if (graphs && (k & 1) && end - k >= 2) {
                    if (!c->pair_exec || c->pair_tol2 != tol2 || c->pair_groups != act) {
                        const int r2 = capture_pair(c, act, tol2);
                        if (r2) return r2;
                    }
                    HIPCHK(c, hipGraphLaunch(c->pair_exec, st));
                    k += 2;
                } else {
                    const int r2 = run_iteration(c, act, st, k, k == 0 ? 1 : 0, tol2, &c->prof);
                    if (r2) return r2;
                    ++k;
                }
            }
            LAUNCHCHK(c);
            return MTOMG_OK;
        };
        // first batch: the previous solve's count (a design loop changes slowly), then small steps.
        // Iteration it forms r_{it+1} and tests it, so a solve of n iterations
        // stops inside iteration n-1: a batch of exactly n launches nothing after it.
        int batch = c->last_iters > 0 ? c->last_iters : std::max(2, c->batch);
        while (it < max_iter) {
            const int nb = std::min(batch, max_iter - it);
            rc = launch_iters(it, nb);
            if (rc) return rc;
            it += nb;
            // Finish every system that has converged (at the iteration limit
            // every system) before the host looks: its pending x update, true
            // residual and sums, and its state word 1 -> 2.  Systems still
            // running are left alone and continue in the next batch.
            rc = finish(it, it >= max_iter ? 3 : 4);
            if (rc) return rc;
            bool running = false;
            for (int gi : act)
                for (int q = 0; q < c->groups[gi].n_sys; ++q) running = running || c->host_state[4 * (gsys0[gi] + q)] == 0;
            if (!running) break;
            batch = std::max(2, std::min(it / 2, 16));
        }
        LAUNCHCHK(c);
    }
    if (it == 0) {
        // no iteration ran (max_iter = 0 or no active system): sums of the start
        rc = finish(0, -1);
        if (rc) return rc;
    }
    HIPCHK(c, hipEventElapsedTime(ms, c->ev_solve[0], c->ev_solve[1]));
    return MTOMG_OK;
}

// Every system of every design with densities, in lockstep (see the file
// comment).  The stopping test of Algorithm 2 runs on the recursively
// updated residual; at exit the true FP64 residual f - K u is formed, and a
// system whose true residual is still above the tolerance (the two drift
// apart over thousands of iterations at high contrast) restarts PCG from
// its current iterate, up to c->max_restarts times within max_iter in total.
int solve_all(mtomg_ctx* c, double rel_tol, int max_iter, int warm, mtomg_stats* stats) {
    // Coarsest factorisations of designs with new densities run on the side
    // stream, overlapped with the start of the first run (initial residual
    // and the descent of the first V-cycle); only its coarse solve waits.
    // (set_densities may have queued some already: then ev_fac[1] marks them)
    bool fac_ran = c->fac_inflight;
    hipEvent_t wait_fac = fac_ran ? c->ev_fac[1] : nullptr;
    HIPCHK(c, hipEventRecord(c->ev_fac[0], c->stream));
    HIPCHK(c, hipStreamWaitEvent(c->side_stream, c->ev_fac[0], 0));
    bool launched = false;
    int rc = factor_launch(c, c->side_stream, &launched);
    if (rc) return rc;
    if (launched) {
        HIPCHK(c, hipEventRecord(c->ev_fac[1], c->side_stream));
        wait_fac = c->ev_fac[1];
        fac_ran = true;
    }
    const double tol2 = rel_tol * rel_tol;
    std::vector<int> gsys0(c->groups.size(), 0), sys_design;
    int n_sys = 0;
    for (size_t gi = 0; gi < c->groups.size(); ++gi) {
        Group& g = c->groups[gi];
        gsys0[gi] = n_sys;
        for (size_t k = 0; k < g.designs.size(); ++k) {
            const Design& d = c->d[g.designs[k]];
            const int v = (d.has_dens && !d.fac_failed && !d.x_code) ? 0 : ST_INACTIVE;
            for (int q = 0; q < g.cpd; ++q) {
                int* h = c->host_state + 4 * (n_sys + (int)k * g.cpd + q);
                h[0] = v;
                h[1] = h[2] = h[3] = 0;
                sys_design.push_back(g.designs[k]);
            }
        }
        n_sys += g.n_sys;
    }
    // per system: final state, iterations and runs over all rounds, sums of its last run
    std::vector<int> state(n_sys, ST_INACTIVE), iters(n_sys, 0), runs(n_sys, 0);
    std::vector<double> sums(3 * (size_t)n_sys, 0.0);
    float total_ms = 0.f;
    int first_round_most = 0;
    int budget = max_iter, warm_r = warm;
    for (int round = 0; round <= c->max_restarts; ++round) {
        float ms = 0.f;
        rc = pcg_round(c, gsys0, tol2, budget, warm_r, &ms, round == 0 ? wait_fac : nullptr);
        if (rc) return rc;
        total_ms += ms;
        if (round == 0 && fac_ran) {
            HIPCHK(c, hipStreamSynchronize(c->side_stream));
            c->fac_inflight = false;
            rc = factor_finalize(c);
            if (rc) return rc;
        }
        std::vector<int> again;
        int used = 0;
        for (int q = 0; q < n_sys; ++q) {
            if (c->host_state[4 * q] == ST_INACTIVE) continue;   // not in this run
            state[q] = c->host_state[4 * q];
            iters[q] += c->host_state[4 * q + 1];
            runs[q] += 1;
            if (round == 0) first_round_most = std::max(first_round_most, iters[q]);
            for (int k = 0; k < 3; ++k) sums[3 * q + k] = c->host_sums[4 * q + k];
            const double ff = sums[3 * q];
            const Design& dq = c->d[sys_design[q]];
            const bool ok = (state[q] == 1 || state[q] == 2) && !dq.fac_failed && !dq.x_code;
            if (ok && ff > 0.0 && sums[3 * q + 2] > tol2 * ff) {
                again.push_back(q);
                used = std::max(used, iters[q]);
            }
        }
        if (again.empty() || round == c->max_restarts || used >= max_iter) break;
        for (int q = 0; q < n_sys; ++q) {
            int* h = c->host_state + 4 * q;
            h[0] = ST_INACTIVE;
            h[1] = h[2] = h[3] = 0;
        }
        for (int q : again) c->host_state[4 * q] = 0;
        budget = max_iter - used;
        warm_r = 1;
    }
    int k = 0, worst = MTOMG_OK;
    for (Design& d : c->d) {
        if (!d.has_grid || !d.has_dens) continue;
        const Group& g = c->groups[d.group];
        const int s0 = gsys0[d.group] + d.gidx * g.cpd;
        for (int q = 0; q < d.n_cases; ++q) {
            mtomg_stats& o = stats[k++];
            std::memset(&o, 0, sizeof(o));
            o.n_dof = (int)(2 * d.lev[d.fine()].nodes());
            o.t_setup_ms = d.t_setup_ms;
            o.model_bytes = model_bytes(d);
            if (d.x_code) {   // densities outside [0, 1] or not finite (checked by k_interp)
                o.status = d.x_code == 2 ? MTOMG_NAN : MTOMG_BAD_INPUT;
                worst = std::min(worst, o.status);
                continue;
            }
            if (d.fac_failed) {
                o.status = MTOMG_BREAKDOWN;
                worst = std::min(worst, (int)MTOMG_BREAKDOWN);
                continue;
            }
            const int sq = s0 + q;
            const int cv = state[sq];
            const double ff = sums[3 * sq];
            o.relres_rec = ff > 0 ? std::sqrt(sums[3 * sq + 1] / ff) : 0.0;
            o.relres_true = ff > 0 ? std::sqrt(sums[3 * sq + 2] / ff) : 0.0;
            const bool met = ff <= 0.0 || sums[3 * sq + 2] <= tol2 * ff;
            o.status = (cv == 1 || cv == 2) ? (met ? MTOMG_OK : MTOMG_NOT_CONVERGED)
                                           : cv == 3 ? MTOMG_BREAKDOWN : cv == 4 ? MTOMG_NAN : MTOMG_NOT_CONVERGED;
            o.iters = iters[sq];
            o.vcycles = o.iters + runs[sq];
            o.t_solve_ms = total_ms;
            if (o.status < worst) worst = o.status;
        }
    }
    // batch hint for the next solve: the iterations of the first run
    c->last_iters = first_round_most;
    return worst;
}

}  // namespace

extern "C" {

int mtomg_create(mtomg_ctx** ctx, int max_designs, void* hip_stream) {
    if (!ctx || max_designs < 1) return MTOMG_BAD_INPUT;
    *ctx = nullptr;
    mtomg_ctx* c = new (std::nothrow) mtomg_ctx();
    if (!c) return MTOMG_BAD_INPUT;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return MTOMG_HIP_ERROR;
    }
    c->d.resize(max_designs);
    if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return MTOMG_HIP_ERROR;
    }
    if (hipEventCreate(&c->ev_solve[0]) != hipSuccess || hipEventCreate(&c->ev_solve[1]) != hipSuccess ||
        hipStreamCreateWithFlags(&c->side_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_fac[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_fac[1], hipEventDisableTiming) != hipSuccess) {
        mtomg_destroy(c);
        return MTOMG_HIP_ERROR;
    }
    *ctx = c;
    return MTOMG_OK;
}

int mtomg_destroy(mtomg_ctx* c) {
    if (!c) return MTOMG_OK;
    hipStreamSynchronize(c->stream);
    hipStreamSynchronize(c->side_stream);
    drop_graphs(c);
    if (c->side_stream) hipStreamSynchronize(c->side_stream);
    if (c->cap_stream) hipStreamDestroy(c->cap_stream);
    if (c->side_stream) hipStreamDestroy(c->side_stream);
    for (int b = 1; b < MAX_BRANCHES; ++b) {
        if (c->br_st[b]) {
            hipStreamSynchronize(c->br_st[b]);
            hipStreamDestroy(c->br_st[b]);
        }
        if (c->br_join[b]) hipEventDestroy(c->br_join[b]);
    }
    if (c->br_fork) hipEventDestroy(c->br_fork);
    for (hipEvent_t& e : c->ev_fac)
        if (e) hipEventDestroy(e);
    for (Design& d : c->d) {
        for (hipEvent_t& e : d.ev)
            if (e) hipEventDestroy(e);
        for (hipEvent_t& e : d.fev)
            if (e) hipEventDestroy(e);
    }
    for (hipEvent_t& e : c->ev_solve)
        if (e) hipEventDestroy(e);
    if (c->ws_owned && c->ws) hipFree(c->ws);
    if (c->host_state) hipHostFree(c->host_state);
    if (c->host_sums) hipHostFree(c->host_sums);
    if (c->host_chol) hipHostFree(c->host_chol);
    if (c->filt_tab) hipFree(c->filt_tab);
    if (c->filt_host) hipHostFree(c->filt_host);
    if (c->pois_buf) hipFree(c->pois_buf);
    if (c->pois_host) hipHostFree(c->pois_host);
    if (c->pois_exec) hipGraphExecDestroy(c->pois_exec);
    if (c->oc_buf) hipFree(c->oc_buf);
    if (c->oc_host) hipHostFree(c->oc_host);
    for (hipEvent_t& e : c->prof.ev)
        if (e) hipEventDestroy(e);
    delete c;
    return MTOMG_OK;
}

int mtomg_set_grid(mtomg_ctx* c, int design, int nelx, int nely, double nu, int m, const double* E_phase,
                   double E_min, double penal, int levels, int n_pre, int n_post, double omega, int precision,
                   int n_cases, const double* F, double* U) {
    if (!c) return MTOMG_BAD_INPUT;
    if (design < 0 || design >= (int)c->d.size()) return fail(c, MTOMG_BAD_INPUT, "design index out of range");
    if (levels < 2 || levels > 14) return fail(c, MTOMG_BAD_INPUT, "levels must be in [2, 14]");
    const int s = 1 << (levels - 1);
    if (nelx < s || nely < s || nelx % s || nely % s)
        return fail(c, MTOMG_BAD_INPUT, "nelx and nely must be positive multiples of 2^(levels-1)");
    if ((long)(nelx / s) * (nely / s) > MAX_COARSE_ELEMS)
        return fail(c, MTOMG_BAD_INPUT, "coarsest grid larger than 8192 elements; add levels");
    if ((long)(nelx + 1) * (nely + 1) > (1L << 30)) return fail(c, MTOMG_BAD_INPUT, "grid too large");
    if (!(nu >= 0.0 && nu < 0.5)) return fail(c, MTOMG_BAD_INPUT, "nu must be in [0, 0.5)");
    if (m < 1 || m > MAX_PHASES || !E_phase) return fail(c, MTOMG_BAD_INPUT, "m must be in [1, 8] with E_phase given");
    if (!(E_min > 0.0)) return fail(c, MTOMG_BAD_INPUT, "E_min must be > 0");
    for (int k = 0; k < m; ++k)
        if (!(E_phase[k] >= E_min) || !std::isfinite(E_phase[k])) return fail(c, MTOMG_BAD_INPUT, "E_phase must be finite and >= E_min");
    if (!(penal >= 1.0)) return fail(c, MTOMG_BAD_INPUT, "penal must be >= 1");
    if (n_pre < 0 || n_pre > 8 || n_post < 0 || n_post > 8) return fail(c, MTOMG_BAD_INPUT, "n_pre, n_post must be in [0, 8]");
    if (!(omega > 0.0 && omega <= 1.0)) return fail(c, MTOMG_BAD_INPUT, "omega must be in (0, 1]");
    if (precision != MTOMG_FP64 && precision != MTOMG_FP32MG) return fail(c, MTOMG_BAD_INPUT, "unknown precision");
    if (n_cases < 1 || n_cases > 64) return fail(c, MTOMG_BAD_INPUT, "n_cases must be in [1, 64]");
    if (!F || !U) return fail(c, MTOMG_BAD_INPUT, "F and U must be device pointers");
    Design& d = c->d[design];
    hipStreamSynchronize(c->stream);
    hipStreamSynchronize(c->side_stream);
    drop_graphs(c);
    for (hipEvent_t& e : d.ev)
        if (e) hipEventDestroy(e);
    for (hipEvent_t& e : d.fev)
        if (e) hipEventDestroy(e);
    d = Design();
    d.nelx = nelx; d.nely = nely; d.nu = nu; d.m = m; d.E_min = E_min; d.penal = penal; d.levels = levels;
    d.n_pre = n_pre; d.n_post = n_post; d.omega = omega; d.precision = precision; d.n_cases = n_cases;
    d.F = F; d.U = U;
    for (int k = 0; k < m; ++k) d.E_phase[k] = E_phase[k];
    d.lev.resize(levels);
    for (int l = 0; l < levels; ++l) {
        const int sh = levels - 1 - l;
        d.lev[l].nx = nelx >> sh;
        d.lev[l].ny = nely >> sh;
    }
    plan_design(c->rows_fine, c->rows_coarse, c->rows_cg, c->rows_depth, d);
    d.n0 = 2 * (d.lev[0].nx + 1) * d.lev[0].ny;
    d.np0 = (d.n0 + COARSE_NB - 1) / COARSE_NB * COARSE_NB;
    d.cases.assign(n_cases, CaseBufs());
    for (hipEvent_t* e : {&d.ev[0], &d.ev[1], &d.fev[0], &d.fev[1]}) HIPCHK(c, hipEventCreate(e));
    d.has_grid = true;
    // the layout changes: drop an owned workspace, forget a borrowed one
    if (c->ws_owned && c->ws) {
        hipStreamSynchronize(c->stream);
        hipFree(c->ws);
    }
    c->ws = nullptr;
    c->ws_bytes = 0;
    c->ws_owned = false;
    c->laid_out = false;
    for (Design& o : c->d) o.has_dens = false;
    forget_factorisations(c);
    return MTOMG_OK;
}

size_t mtomg_workspace_bytes(const mtomg_ctx* c) {
    if (!c) return 0;
    return measure_workspace(c);
}

int mtomg_set_workspace(mtomg_ctx* c, void* dev, size_t bytes) {
    if (!c) return MTOMG_BAD_INPUT;
    if (!dev || (reinterpret_cast<uintptr_t>(dev) & 255)) return fail(c, MTOMG_BAD_INPUT, "workspace must be a 256-byte aligned device pointer");
    const size_t need = measure_workspace(c);
    if (bytes < need) return fail(c, MTOMG_WORKSPACE, "workspace smaller than mtomg_workspace_bytes()");
    hipStreamSynchronize(c->stream);
    hipStreamSynchronize(c->side_stream);
    drop_graphs(c);
    if (c->ws_owned && c->ws) hipFree(c->ws);
    c->ws = dev;
    c->ws_bytes = bytes;
    c->ws_owned = false;
    c->laid_out = false;
    for (Design& o : c->d) o.has_dens = false;
    forget_factorisations(c);
    return ensure_workspace(c);
}

int mtomg_set_densities(mtomg_ctx* c, int design, const double* x) {
    int rc = check_design(c, design, false);
    if (rc) return rc;
    if (!x) return fail(c, MTOMG_BAD_INPUT, "x must be a device pointer");
    rc = ensure_workspace(c);
    if (rc) return rc;
    Design& d = c->d[design];
    hipStream_t st = c->stream;
    // a factorisation still queued on the side stream reads this design's matrix
    if (c->fac_inflight) HIPCHK(c, hipStreamWaitEvent(st, c->ev_fac[1], 0));
    d.fac_launched = false;   // new densities supersede a queued factorisation
    HIPCHK(c, hipEventRecord(d.ev[0], st));
    const int f = d.fine();
    LevelBufs& Lf = d.lev[f];
    d.dens_seq = d.dens_seq % ((1 << 29) - 1) + 1;
    d.x_code = 0;
    launch_interp(st, x, phases_of(d), Lf.nx * Lf.ny, Lf.op64, d.mixed() ? Lf.op32 : nullptr, d.chol_status + 2,
                  d.dens_seq);
    // coarse moments, up to five levels per launch (tiles of 16 x 16 elements
    // or the largest power of two dividing the level; 1 falls back to one
    // launch per level)
    for (int l = f - 1; l >= 0;) {
        LevelBufs& P = d.lev[l + 1];
        LevelBufs& L = d.lev[l];
        int T = 16;
        while (T > 1 && (L.nx % T || L.ny % T)) T >>= 1;
        if (T == 1) {
            if (l + 1 == f) launch_moments_from_fine(st, P.op64, P.nx, P.ny, L.op64, d.mixed() ? L.op32 : nullptr);
            else launch_moments_coarsen(st, P.op64, P.nx, P.ny, L.op64, d.mixed() ? L.op32 : nullptr);
            --l;
            continue;
        }
        int n = 1;
        while (n < 5 && l - n >= 0 && (T >> n) >= 1) ++n;
        MomLevels out{};
        for (int k = 0; k < n; ++k) {
            out.m64[k] = d.lev[l - k].op64;
            out.m32[k] = d.mixed() ? d.lev[l - k].op32 : nullptr;
        }
        launch_moments_tree(st, l + 1 == f, P.op64, P.nx, P.ny, T, n, out);
        l -= n;
    }
    assemble_coarsest(st, d);
    LAUNCHCHK(c);
    HIPCHK(c, hipEventRecord(d.ev[1], st));
    d.x_dev = x;
    d.has_dens = true;
    d.needs_factor = true;
    d.fac_failed = false;
    // A design alone in its group starts its coarsest factorisation now, on
    // the side stream: it then runs while the host returns and calls the
    // solve.  Designs of larger groups wait for the solve, which factors a
    // whole group per launch.
    if (c->groups[d.group].designs.size() == 1) {
        HIPCHK(c, hipEventRecord(c->ev_fac[0], st));
        HIPCHK(c, hipStreamWaitEvent(c->side_stream, c->ev_fac[0], 0));
        bool ran = false;
        rc = factor_launch(c, c->side_stream, &ran, d.group);
        if (rc) return rc;
        if (ran) {
            HIPCHK(c, hipEventRecord(c->ev_fac[1], c->side_stream));
            c->fac_inflight = true;
        }
    }
    return MTOMG_OK;
}

int mtomg_solve(mtomg_ctx* c, double rel_tol, int max_iter, int warm_start, mtomg_stats* stats) {
    if (!c || !stats) return MTOMG_BAD_INPUT;
    if (!(rel_tol >= 0.0) || max_iter < 0) return fail(c, MTOMG_BAD_INPUT, "rel_tol must be >= 0 and max_iter >= 0");
    bool any = false;
    for (const Design& d : c->d) any = any || (d.has_grid && d.has_dens);
    if (!any) return fail(c, MTOMG_STATE, "no design has densities");
    const int rc = solve_all(c, rel_tol, max_iter, warm_start, stats);
    if (rc == MTOMG_HIP_ERROR) return rc;
    if (rc != MTOMG_OK) c->err = mtomg_status_string(rc);
    return rc;
}

int mtomg_compliance_and_grad(mtomg_ctx* c, int design, double* cout, double* dcdx) {
    int rc = check_design(c, design, true);
    if (rc) return rc;
    if (!cout) return fail(c, MTOMG_BAD_INPUT, "c must be a device pointer");
    Design& d = c->d[design];
    hipStream_t st = c->stream;
    const LevelBufs& L = d.lev[d.fine()];
    const size_t nf = 2 * L.nodes();
    for (int k = 0; k < d.n_cases; ++k) {
        CaseBufs& cb = d.cases[k];
        launch_dot_partials(st, cb.F, cb.U, nf, cb.cpart, dot_parts(nf));
        launch_sum_to(st, cb.cpart, dot_parts(nf), cout + k);
        if (dcdx)
            launch_grad(st, cb.U, d.x_dev, phases_of(d), make_mat<double>(d, d.omega), L.nx, L.ny,
                        dcdx + (size_t)k * L.nx * L.ny * d.m);
    }
    LAUNCHCHK(c);
    return MTOMG_OK;
}

}  // extern "C"

namespace {

// Argument check shared by both filter entry points: nullptr if valid.
const char* filter_args_error(int nelx, int nely, int m, double rf, int mode, double gmin, const double* x,
                              const double* in, const double* out) {
    if (nelx < 1 || nely < 1 || nelx > (1 << 22) || nely > (1 << 20) || (long)nelx * nely > (1L << 30))
        return "filter grid must have 1 .. 2^22 columns, 1 .. 2^20 rows and at most 2^30 elements";
    if (m < 1 || m > MAX_PHASES) return "m must be in [1, 8]";
    if (!(rf > 0.0 && rf <= FILTER_MAX_RF)) return "rf must be in (0, 16]";
    if (mode != MTOMG_FILTER_DENSITY && mode != MTOMG_FILTER_DENSITY_ADJOINT && mode != MTOMG_FILTER_SENSITIVITY)
        return "unknown filter mode";
    if (!in || !out) return "in and out must be device pointers";
    if (in == out) return "out must not alias in";
    if (mode == MTOMG_FILTER_SENSITIVITY) {
        if (!x) return "the sensitivity filter needs the densities x";
        if (x == out) return "out must not alias x";
        if (!(gmin > 0.0 && std::isfinite(gmin))) return "gmin must be finite and > 0";
    }
    return nullptr;
}

}  // namespace

extern "C" {

int mtomg_filter(mtomg_ctx* c, int nelx, int nely, int m, double rf, int mode, double gmin, const double* x,
                 const double* in, double* out) {
    if (!c) return MTOMG_BAD_INPUT;
    if (const char* msg = filter_args_error(nelx, nely, m, rf, mode, gmin, x, in, out))
        return fail(c, MTOMG_BAD_INPUT, msg);
    if (!c->filt_tab) {
        HIPCHK(c, hipMalloc(&c->filt_tab, FILTER_TAB_MAX * sizeof(double)));
        HIPCHK(c, hipHostMalloc(&c->filt_host, FILTER_TAB_MAX * sizeof(double)));
    }
    if (rf != c->filt_rf) {
        // the staging buffer may still feed an earlier copy: let it finish
        HIPCHK(c, hipStreamSynchronize(c->stream));
        filter_table(rf, c->filt_host);
        HIPCHK(c, hipMemcpyAsync(c->filt_tab, c->filt_host, FILTER_TAB_MAX * sizeof(double), hipMemcpyHostToDevice,
                                 c->stream));
        c->filt_rf = rf;
    }
    launch_cone_filter(c->stream, nelx, nely, m, rf, mode, gmin, c->filt_tab, x, in, out);
    LAUNCHCHK(c);
    return MTOMG_OK;
}

int mtomg_filter_noalloc(void* hip_stream, int nelx, int nely, int m, double rf, int mode, double gmin,
                         const double* x, const double* in, double* out) {
    if (filter_args_error(nelx, nely, m, rf, mode, gmin, x, in, out)) return MTOMG_BAD_INPUT;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    double* tab = nullptr;
    if (filter_static_table(&tab) != hipSuccess) return MTOMG_HIP_ERROR;
    launch_filter_table(st, rf, tab);
    launch_cone_filter(st, nelx, nely, m, rf, mode, gmin, tab, x, in, out);
    return hipGetLastError() == hipSuccess ? MTOMG_OK : MTOMG_HIP_ERROR;
}

}  // extern "C"

namespace {

// Buffers of the Poisson solve: per grid level l (n_l = n >> (L-1-l)),
// b (restricted right-hand side), e (correction), t0 / t1 (smoother
// iterates) and res (residual); on the finest grid r, z, p, q.
struct PoisBufs {
    int L = 0;
    int nl[16] = {};
    double* b[16] = {};
    double* e[16] = {};
    double* t0[16] = {};
    double* t1[16] = {};
    double* res[16] = {};
    double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
    double* part = nullptr;   // 64 dot-product partials
    double* sc = nullptr;     // scalars: ff, rz[2], pq, rr
    int* state = nullptr;     // [0] 0 running / 1 converged / 3 breakdown / 4 not finite, [1] iterations
};

size_t pois_layout(int n, int L, PoisBufs* pb, char* base) {
    size_t off = 0;
    auto take = [&](size_t count) -> double* {
        double* ptr = base ? reinterpret_cast<double*>(base + off) : nullptr;
        off += (count * sizeof(double) + 255) / 256 * 256;
        return ptr;
    };
    if (pb) pb->L = L;
    for (int l = 0; l < L; ++l) {
        const int nl = n >> (L - 1 - l);
        const size_t N = (size_t)(nl + 1) * (nl + 1);
        double* b = take(N); double* e = take(N); double* t0 = take(N); double* t1 = take(N); double* res = take(N);
        if (pb) { pb->nl[l] = nl; pb->b[l] = b; pb->e[l] = e; pb->t0[l] = t0; pb->t1[l] = t1; pb->res[l] = res; }
    }
    const size_t N = (size_t)(n + 1) * (n + 1);
    double* r = take(N); double* z = take(N); double* p = take(N); double* q = take(N);
    double* part = take(DOT_PARTS_MAX); double* sc = take(8); double* state = take(1);
    if (pb) {
        pb->r = r; pb->z = z; pb->p = p; pb->q = q; pb->part = part; pb->sc = sc;
        pb->state = reinterpret_cast<int*>(state);
    }
    return off;
}

// One cycle of Algorithm 1 (gamma = 1) on level l: out = M_l^{-1} b.
void pois_cycle(hipStream_t st, const PoisBufs& pb, int l, const double* b, double* out, int n_pre, int n_post,
                double omega) {
    if (l == 0) {
        launch_pois_coarse(st, b, out);
        return;
    }
    const int nl = pb.nl[l], nc = pb.nl[l - 1];
    double* cur = nullptr;
    for (int k = 0; k < n_pre; ++k) {
        double* dst = cur == pb.t0[l] ? pb.t1[l] : pb.t0[l];
        launch_pois_jacobi(st, nl, omega, b, cur, dst);
        cur = dst;
    }
    launch_pois_residual(st, nl, b, cur, pb.res[l]);
    launch_pois_restrict(st, nc, pb.res[l], pb.b[l - 1]);
    pois_cycle(st, pb, l - 1, pb.b[l - 1], pb.e[l - 1], n_pre, n_post, omega);
    if (!cur) {
        launch_fill<double>(st, pb.t0[l], (size_t)(nl + 1) * (nl + 1), 0.0);
        cur = pb.t0[l];
    }
    launch_pois_prolong_add(st, nc, pb.e[l - 1], cur);
    if (n_post == 0) {
        launch_pois_jacobi(st, nl, 0.0, b, cur, out);   // omega = 0: a copy
        return;
    }
    for (int k = 0; k < n_post; ++k) {
        double* dst = k == n_post - 1 ? out : (cur == pb.t0[l] ? pb.t1[l] : pb.t0[l]);
        launch_pois_jacobi(st, nl, omega, b, cur, dst);
        cur = dst;
    }
}

void pois_dot(hipStream_t st, const PoisBufs& pb, int n, const double* a, const double* b, double* out) {
    const size_t N = (size_t)(n + 1) * (n + 1);
    launch_dot_partials(st, a, b, N, pb.part, dot_parts(N));
    launch_sum_to(st, pb.part, dot_parts(N), out);
}

}  // namespace

extern "C" {

int mtomg_poisson_solve(mtomg_ctx* c, int n, int n_pre, int n_post, double omega, double rel_tol, int max_iter,
                        const double* f, double* u, mtomg_stats* stats) {
    if (!c) return MTOMG_BAD_INPUT;
    if (n < 4 || n > 8192 || (n & (n - 1))) return fail(c, MTOMG_BAD_INPUT, "n must be a power of two in [4, 8192]");
    if (n_pre < 0 || n_pre > 8 || n_post < 0 || n_post > 8) return fail(c, MTOMG_BAD_INPUT, "n_pre, n_post must be in [0, 8]");
    if (!(omega > 0.0 && omega <= 1.0)) return fail(c, MTOMG_BAD_INPUT, "omega must be in (0, 1]");
    if (!(rel_tol > 0.0) || max_iter < 0) return fail(c, MTOMG_BAD_INPUT, "rel_tol must be > 0, max_iter >= 0");
    if (!f || !u || !stats) return fail(c, MTOMG_BAD_INPUT, "f, u (device) and stats (host) are required");
    if (f == u) return fail(c, MTOMG_BAD_INPUT, "u must not alias f");
    int L = 0;
    while ((2 << L) <= n) ++L;   // levels down to the 2 x 2 grid: n = 2^L
    hipStream_t st = c->stream;
    const size_t need = pois_layout(n, L, nullptr, nullptr);
    if (need > c->pois_bytes) {
        HIPCHK(c, hipStreamSynchronize(st));
        if (c->pois_buf) HIPCHK(c, hipFree(c->pois_buf));
        c->pois_buf = nullptr;
        c->pois_bytes = 0;
        HIPCHK(c, hipMalloc(&c->pois_buf, need));
        c->pois_bytes = need;
    }
    if (!c->pois_host) HIPCHK(c, hipHostMalloc(&c->pois_host, 8 * sizeof(double)));
    PoisBufs pb;
    pois_layout(n, L, &pb, reinterpret_cast<char*>(c->pois_buf));
    const size_t N = (size_t)(n + 1) * (n + 1);
    double* sc = pb.sc;   // [0] ||f||^2, [1] / [2] r.z of alternate iterations, [3] p.q, [4] ||r||^2
    double* hs = c->pois_host;
    hipEvent_t e0 = c->ev_solve[0], e1 = c->ev_solve[1];
    HIPCHK(c, hipEventRecord(e0, st));
    // u = 0, r = f on the interior (Algorithm 2 from a zero start)
    launch_fill<double>(st, u, N, 0.0);
    launch_pois_residual(st, n, f, nullptr, pb.r);
    pois_dot(st, pb, n, pb.r, pb.r, sc + 0);
    const int fine = L - 1;
    auto read_scalars = [&]() -> int {
        HIPCHK(c, hipMemcpyAsync(hs, sc, 5 * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipMemcpyAsync(hs + 6, pb.state, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        return MTOMG_OK;
    };
    const double tol2 = rel_tol * rel_tol;
    // PCG iteration k (k >= 1): the device tests it, and once its state word
    // is set the updates of u, r and p that follow do nothing, so whole
    // batches of iterations are queued between host reads
    auto iteration = [&](hipStream_t s2, int k) {
        double* rz = sc + 1 + ((k - 1) & 1);   // r_{k-1}.z_{k-1}
        double* rz_next = sc + 1 + (k & 1);
        launch_pois_apply(s2, n, pb.p, pb.q);
        pois_dot(s2, pb, n, pb.p, pb.q, sc + 3);
        launch_pois_axpy(s2, n, rz, sc + 3, 1.0, pb.p, u, pb.state);
        launch_pois_axpy(s2, n, rz, sc + 3, -1.0, pb.q, pb.r, pb.state);
        pois_dot(s2, pb, n, pb.r, pb.r, sc + 4);
        launch_pois_check(s2, sc, tol2, pb.state);
        pois_cycle(s2, pb, fine, pb.r, pb.z, n_pre, n_post, omega);
        pois_dot(s2, pb, n, pb.r, pb.z, rz_next);
        launch_pois_check_rz(s2, rz_next, pb.state);
        launch_pois_xpby(s2, n, pb.z, rz_next, rz, pb.p, pb.state);
    };
    launch_fill_strided(st, pb.state, sizeof(int), 2, 0);
    int rc = read_scalars();
    if (rc) return rc;
    const double ff = hs[0];
    int status = ff > 0.0 ? MTOMG_NOT_CONVERGED : MTOMG_OK, it = 0, cycles = 0;
    double rr = ff;
    if (ff > 0.0 && max_iter > 0) {
        pois_cycle(st, pb, fine, pb.r, pb.z, n_pre, n_post, omega);
        pois_dot(st, pb, n, pb.r, pb.z, sc + 1);
        launch_pois_xpby(st, n, pb.z, nullptr, nullptr, pb.p, nullptr);
        // two iterations (k = 1, 2: both parities) in one graph, replayed
        // for every later pair; captured again when the arguments change
        const std::vector<double> key{(double)n, (double)n_pre, (double)n_post, omega, tol2,
                                      (double)reinterpret_cast<uintptr_t>(u),
                                      (double)reinterpret_cast<uintptr_t>(c->pois_buf)};
        if (!c->pois_exec || c->pois_key != key) {
            if (c->pois_exec) HIPCHK(c, hipGraphExecDestroy(c->pois_exec));
            c->pois_exec = nullptr;
            hipStream_t cs = c->cap_stream;
            HIPCHK(c, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            iteration(cs, 1);
            iteration(cs, 2);
            hipGraph_t g = nullptr;
            HIPCHK(c, hipStreamEndCapture(cs, &g));
            const hipError_t e = hipGraphInstantiate(&c->pois_exec, g, nullptr, nullptr, 0);
            hipGraphDestroy(g);
            if (e != hipSuccess) {
                c->pois_exec = nullptr;
                return fail(c, MTOMG_HIP_ERROR, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
            }
            c->pois_key = key;
        }
        // Batches of iterations between host reads: the first is the
        // previous count at this size (or one pair), the next ones are
        // predicted from the residual's reduction over the last batch, so a
        // converged solve queues few iterations that do nothing.
        int launched = 0;
        int batch = c->pois_last_n == n && c->pois_last_iters > 0 ? c->pois_last_iters : 2;
        double prev_rel = 1.0;   // ||r_0|| / ||f||
        while (launched < max_iter) {
            const int nb = std::min(batch, max_iter - launched);
            int k = 0;
            if (launched & 1) {   // the next iteration has parity 2
                iteration(st, 2);
                ++k;
            }
            for (; nb - k >= 2; k += 2) HIPCHK(c, hipGraphLaunch(c->pois_exec, st));
            if (k < nb) iteration(st, 1);
            launched += nb;
            LAUNCHCHK(c);
            rc = read_scalars();
            if (rc) return rc;
            const int* hst = reinterpret_cast<const int*>(hs + 6);
            if (hst[0] != 0) break;
            const double rel = std::sqrt(std::max(hs[4], 0.0) / ff);
            if (rel > 0.0 && rel < prev_rel) {
                const double rate = std::pow(rel / prev_rel, 1.0 / nb);
                const double need = std::ceil(std::log(rel_tol / rel) / std::log(rate));
                batch = (int)std::min(16.0, std::max(1.0, need));
            } else {
                batch = std::min(2 * nb, 16);
            }
            prev_rel = rel;
        }
        const int* hst = reinterpret_cast<const int*>(hs + 6);
        it = hst[1];
        cycles = it + 1;
        c->pois_last_n = n;
        c->pois_last_iters = it;
        rr = hs[4];
        status = hst[0] == 1 ? MTOMG_OK : hst[0] == 3 ? MTOMG_BREAKDOWN : hst[0] == 4 ? MTOMG_NAN
                                                                                     : MTOMG_NOT_CONVERGED;
    }
    // true residual ||f - K u|| at exit
    launch_pois_residual(st, n, f, u, pb.res[fine]);
    pois_dot(st, pb, n, pb.res[fine], pb.res[fine], sc + 4);
    HIPCHK(c, hipEventRecord(e1, st));
    LAUNCHCHK(c);
    rc = read_scalars();
    if (rc) return rc;
    float ms = 0.0f;
    HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
    mtomg_stats s{};
    s.status = status;
    s.iters = it;
    s.vcycles = cycles;
    s.n_dof = (n - 1) * (n - 1);
    s.relres_rec = ff > 0.0 ? std::sqrt(rr / ff) : 0.0;
    s.relres_true = ff > 0.0 ? std::sqrt(hs[4] / ff) : 0.0;
    s.t_setup_ms = 0.0;
    s.t_solve_ms = ms;
    s.model_bytes = 0.0;
    *stats = s;
    return status;
}

}  // extern "C"

namespace {

// Device workspace of the OC calls, grown on demand (never shrunk).
int oc_reserve(mtomg_ctx* c, size_t bytes, size_t host_bytes) {
    if (bytes > c->oc_bytes) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (c->oc_buf) HIPCHK(c, hipFree(c->oc_buf));
        c->oc_buf = nullptr;
        c->oc_bytes = 0;
        HIPCHK(c, hipMalloc(&c->oc_buf, bytes));
        c->oc_bytes = bytes;
    }
    if (host_bytes > c->oc_host_bytes) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (c->oc_host) HIPCHK(c, hipHostFree(c->oc_host));
        c->oc_host = nullptr;
        c->oc_host_bytes = 0;
        HIPCHK(c, hipHostMalloc((void**)&c->oc_host, host_bytes, hipHostMallocDefault));
        c->oc_host_bytes = host_bytes;
    }
    return MTOMG_OK;
}

const char* oc_args_error(int nelx, int nely, int m, int a, int b, double vol_a, double move, double eta,
                          double eps) {
    if (nelx < 1 || nely < 1 || (long)nelx * nely > (1L << 30)) return "grid must have 1 .. 2^30 elements";
    if (m < 1 || m > MAX_PHASES) return "m must be in [1, 8]";
    if (!(a >= 0 && a < b && b <= m)) return "phases must satisfy 0 <= a < b <= m (b = m: the void)";
    if (!(vol_a >= 0.0 && vol_a <= 1.0)) return "volume fraction must be in [0, 1]";
    if (!(move > 0.0 && std::isfinite(move))) return "move must be finite and > 0";
    if (!(eta > 0.0 && eta <= 2.0)) return "eta must be in (0, 2]";
    if (!(eps > 0.0 && eps < 0.5 / (m + 1))) return "eps must be in (0, 1 / (2 (m + 1)))";
    return nullptr;
}

}  // namespace

extern "C" {

int mtomg_oc_update(mtomg_ctx* c, int nelx, int nely, int m, int a, int b, const double* g, double vol_a,
                    double move, double eta, double eps, double* x, double* info) {
    if (!c) return MTOMG_BAD_INPUT;
    if (const char* msg = oc_args_error(nelx, nely, m, a, b, vol_a, move, eta, eps))
        return fail(c, MTOMG_BAD_INPUT, msg);
    if (!g || !x) return fail(c, MTOMG_BAD_INPUT, "g and x must be device pointers");
    if (g == x) return fail(c, MTOMG_BAD_INPUT, "g must not alias x");
    const int n_e = nelx * nely;
    const size_t nd = oc_scratch_doubles(n_e);
    int rc = oc_reserve(c, nd * sizeof(double) + sizeof(OcState) + 256, sizeof(OcState));
    if (rc) return rc;
    double* scratch = c->oc_buf;
    OcState* state = reinterpret_cast<OcState*>(scratch + nd);
    const OcPair op{n_e, m, a, b, eta, move, eps, vol_a * n_e};
    launch_oc_pair(c->stream, op, g, x, scratch, state);
    LAUNCHCHK(c);
    if (info) {
        HIPCHK(c, hipMemcpyAsync(c->oc_host, state, sizeof(OcState), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        const OcState* hs = reinterpret_cast<const OcState*>(c->oc_host);
        info[0] = hs->lambda;
        info[1] = hs->change;
        info[2] = hs->S - op.target;
        info[3] = hs->passes + (hs->done ? 0.0 : 0.5);
    }
    return MTOMG_OK;
}

int mtomg_aap_step(mtomg_ctx* c, int design, const double* vols, double rf, double move, double eta, double eps,
                   double gmin, double rel_tol, int max_iter, double* x, double* c_pairs, double* change,
                   int* iters) {
    int rc = check_design(c, design, false);
    if (rc) return rc;
    Design& d = c->d[design];
    if (!vols || !x || !c_pairs || !change) return fail(c, MTOMG_BAD_INPUT, "vols, x, c_pairs and change are required");
    for (int k = 0; k < (int)c->d.size(); ++k)
        if (k != design && c->d[k].has_grid && c->d[k].has_dens)
            return fail(c, MTOMG_BAD_INPUT, "the optimised design must be the only design of its context with densities");
    double vsum = 0.0;
    for (int i = 0; i <= d.m; ++i) {
        if (!(vols[i] >= 0.0 && vols[i] <= 1.0)) return fail(c, MTOMG_BAD_INPUT, "volume fractions must be in [0, 1]");
        vsum += vols[i];
    }
    if (std::fabs(vsum - 1.0) > 1e-12) return fail(c, MTOMG_BAD_INPUT, "volume fractions (void last) must sum to 1");
    if (const char* msg = oc_args_error(d.nelx, d.nely, d.m, 0, 1, vols[0], move, eta, eps))
        return fail(c, MTOMG_BAD_INPUT, msg);
    if (!(rf > 0.0 && rf <= FILTER_MAX_RF)) return fail(c, MTOMG_BAD_INPUT, "rf must be in (0, 16]");
    if (!(gmin > 0.0 && std::isfinite(gmin))) return fail(c, MTOMG_BAD_INPUT, "gmin must be finite and > 0");
    const int n_e = d.nelx * d.nely, m = d.m, nc = d.n_cases;
    const size_t ne_m = (size_t)n_e * m;
    const int npairs = m * (m + 1) / 2;
    // device: OC scratch | state | dcdx [nc][n_e][m] | gsum | gfilt | x0 | c [nc] | change partials | change
    const size_t nd = oc_scratch_doubles(n_e);
    const size_t off_state = nd;
    const size_t off_dc = off_state + (sizeof(OcState) + 7) / 8;
    const size_t off_gs = off_dc + (size_t)nc * ne_m;
    const size_t off_gf = off_gs + ne_m;
    const size_t off_x0 = off_gf + ne_m;
    const size_t off_c = off_x0 + ne_m;
    const size_t off_cp = off_c + nc;
    const size_t off_ch = off_cp + OC_BLOCKS;
    const size_t total = off_ch + 1;
    rc = oc_reserve(c, total * sizeof(double), ((size_t)npairs * nc + 1) * sizeof(double));
    if (rc) return rc;
    double* B = c->oc_buf;
    OcState* state = reinterpret_cast<OcState*>(B + off_state);
    double* hc = c->oc_host;
    hipStream_t st = c->stream;
    HIPCHK(c, hipMemcpyAsync(B + off_x0, x, ne_m * sizeof(double), hipMemcpyDeviceToDevice, st));
    std::vector<mtomg_stats> stats(nc);
    int pair = 0;
    for (int a = 0; a < m; ++a) {
        for (int b = a + 1; b <= m; ++b, ++pair) {
            rc = mtomg_set_densities(c, design, x);
            if (rc) return rc;
            rc = solve_all(c, rel_tol, max_iter, 1, stats.data());
            if (rc != MTOMG_OK) return rc == MTOMG_HIP_ERROR ? rc : fail(c, rc, std::string("solve in the OC step: ") + mtomg_status_string(rc));
            if (iters) {
                iters[pair] = 0;
                for (const mtomg_stats& o : stats) iters[pair] = std::max(iters[pair], (int)o.iters);
            }
            rc = mtomg_compliance_and_grad(c, design, B + off_c, B + off_dc);
            if (rc) return rc;
            HIPCHK(c, hipMemcpyAsync(hc + (size_t)pair * nc, B + off_c, nc * sizeof(double), hipMemcpyDeviceToHost, st));
            launch_sum_cases(st, B + off_dc, nc, ne_m, B + off_gs);
            rc = mtomg_filter(c, d.nelx, d.nely, m, rf, MTOMG_FILTER_SENSITIVITY, gmin, x, B + off_gs, B + off_gf);
            if (rc) return rc;
            const OcPair op{n_e, m, a, b, eta, move, eps, vols[a] * n_e};
            launch_oc_pair(st, op, B + off_gf, x, B, state);
            LAUNCHCHK(c);
        }
    }
    launch_oc_change(st, B + off_x0, x, n_e, m, B + off_cp, B + off_ch);
    HIPCHK(c, hipMemcpyAsync(hc + (size_t)npairs * nc, B + off_ch, sizeof(double), hipMemcpyDeviceToHost, st));
    LAUNCHCHK(c);
    HIPCHK(c, hipStreamSynchronize(st));
    for (int k = 0; k < npairs; ++k) {
        double sum = 0.0;
        for (int q = 0; q < nc; ++q) sum += hc[(size_t)k * nc + q];
        c_pairs[k] = sum;
    }
    *change = hc[(size_t)npairs * nc];
    return MTOMG_OK;
}

const char* mtomg_status_string(int s) {
    switch (s) {
        case MTOMG_OK: return "ok";
        case MTOMG_BAD_INPUT: return "bad input (an argument, or densities outside [0, 1])";
        case MTOMG_NOT_CONVERGED: return "not converged (max_iter reached)";
        case MTOMG_BREAKDOWN: return "breakdown (p^T K p <= 0 or z^T r <= 0, or coarsest matrix not SPD)";
        case MTOMG_NAN: return "non-finite residual or densities";
        case MTOMG_WORKSPACE: return "workspace missing or too small";
        case MTOMG_HIP_ERROR: return "HIP runtime error";
        case MTOMG_STATE: return "call out of order";
        default: return "unknown status";
    }
}

const char* mtomg_last_error(const mtomg_ctx* c) { return c ? c->err.c_str() : ""; }

int mtomg_set_option(mtomg_ctx* c, int option, int value) {
    if (!c) return MTOMG_BAD_INPUT;
    switch (option) {
        case MTOMG_OPT_GRAPHS:
            c->use_graphs = value != 0;
            return MTOMG_OK;
        case MTOMG_OPT_FUSE_PRE:
            hipStreamSynchronize(c->stream);
            c->fuse_pre = value != 0;
            drop_graphs(c);   // the captured iteration launches other kernels now
            return MTOMG_OK;
        case MTOMG_OPT_RESTARTS:
            if (value < 0 || value > 64) return fail(c, MTOMG_BAD_INPUT, "restarts must be in [0, 64]");
            c->max_restarts = value;
            return MTOMG_OK;
        case MTOMG_OPT_ROWS_FINE:
        case MTOMG_OPT_ROWS_COARSE:
        case MTOMG_OPT_ROWS_CG:
        default: {
            const bool depth = option >= MTOMG_OPT_ROWS_LEVEL + 1 && option <= MTOMG_OPT_ROWS_LEVEL + 13;
            if (!depth && option != MTOMG_OPT_ROWS_FINE && option != MTOMG_OPT_ROWS_COARSE && option != MTOMG_OPT_ROWS_CG)
                return fail(c, MTOMG_BAD_INPUT, "unknown option");
            if (value != 0 && value != 1 && value != 2 && value != 4 && value != 8)
                return fail(c, MTOMG_BAD_INPUT, "rows per wave must be 0 (automatic), 1, 2, 4 or 8");
            if (depth) c->rows_depth[option - MTOMG_OPT_ROWS_LEVEL] = value;
            else if (option == MTOMG_OPT_ROWS_CG) c->rows_cg = value;
            else (option == MTOMG_OPT_ROWS_FINE ? c->rows_fine : c->rows_coarse) = value;
            hipStreamSynchronize(c->stream);
            hipStreamSynchronize(c->side_stream);
            drop_graphs(c);
            for (Design& d : c->d) plan_design(c->rows_fine, c->rows_coarse, c->rows_cg, c->rows_depth, d);
            // partial-sum buffers are sized by the tile counts: re-lay out the workspace
            c->laid_out = false;
            for (Design& d : c->d) d.has_dens = false;
            forget_factorisations(c);
            if (c->ws_owned && c->ws) { hipFree(c->ws); c->ws = nullptr; c->ws_owned = false; c->ws_bytes = 0; }
            return MTOMG_OK;
        }
        case MTOMG_OPT_DENSE_FACTOR: {
            c->dense_factor = value != 0;
            // factorisations queued by set_densities run again with the new
            // choice, from a freshly assembled K_0 (the dense sequence
            // overwrites the matrix it factors)
            HIPCHK(c, hipStreamSynchronize(c->side_stream));
            c->fac_inflight = false;
            for (Design& d : c->d) {
                if (!(d.has_dens && d.needs_factor && d.fac_launched)) continue;
                d.fac_launched = false;
                assemble_coarsest(c->stream, d);
            }
            LAUNCHCHK(c);
            return MTOMG_OK;
        }
        case MTOMG_OPT_GAMMA:
            if (value != 1 && value != 2) return fail(c, MTOMG_BAD_INPUT, "cycle index must be 1 (V-cycle) or 2 (W-cycle)");
            if (value != c->gamma) {
                HIPCHK(c, hipStreamSynchronize(c->stream));
                drop_graphs(c);
                c->gamma = value;
                c->last_iters = 0;
            }
            return MTOMG_OK;
        case MTOMG_OPT_BATCH:
            if (value < 1 || value > 1000) return fail(c, MTOMG_BAD_INPUT, "batch must be in [1, 1000]");
            c->batch = value;
            c->last_iters = 0;
            return MTOMG_OK;
    }
}

int mtomg_stream_probe(mtomg_ctx* c, int kind, double* a, double* b, double* cc, size_t n, int reps, double* ms) {
    if (!c) return MTOMG_BAD_INPUT;
    if (kind != MTOMG_PROBE_READ && kind != MTOMG_PROBE_COPY && kind != MTOMG_PROBE_TRIAD)
        return fail(c, MTOMG_BAD_INPUT, "unknown probe kind");
    if (n < (1u << 20) || n % 2) return fail(c, MTOMG_BAD_INPUT, "n must be even and at least 2^20");
    if (reps < 1 || reps > 1000 || !ms) return fail(c, MTOMG_BAD_INPUT, "reps must be in [1, 1000] and ms given");
    for (const double* p : {(const double*)a, (const double*)b, (const double*)(kind == MTOMG_PROBE_TRIAD ? cc : a)})
        if (!p || (reinterpret_cast<uintptr_t>(p) & 15)) return fail(c, MTOMG_BAD_INPUT, "arrays must be 16-byte aligned device pointers");
    const int blocks = probe_blocks();
    hipStream_t st = c->stream;
    launch_probe(st, kind, a, b, cc, n, blocks);   // warm-up
    HIPCHK(c, hipEventRecord(c->ev_solve[0], st));
    for (int k = 0; k < reps; ++k) launch_probe(st, kind, a, b, cc, n, blocks);
    HIPCHK(c, hipEventRecord(c->ev_solve[1], st));
    LAUNCHCHK(c);
    HIPCHK(c, hipEventSynchronize(c->ev_solve[1]));
    float t = 0.f;
    HIPCHK(c, hipEventElapsedTime(&t, c->ev_solve[0], c->ev_solve[1]));
    *ms = (double)t / reps;
    return MTOMG_OK;
}

int mtomg_profile_kernel(mtomg_ctx* c, int kernel) {
    if (!c) return MTOMG_BAD_INPUT;
    if (kernel < MTOMG_KERNEL_NONE || kernel > MTOMG_KERNEL_COARSE_SOLVE) return fail(c, MTOMG_BAD_INPUT, "unknown kernel id");
    if (kernel != MTOMG_KERNEL_NONE && c->prof.ev.empty()) {
        c->prof.ev.resize(8192, nullptr);
        for (hipEvent_t& e : c->prof.ev) HIPCHK(c, hipEventCreate(&e));
    }
    c->prof.kernel = kernel;
    c->prof.used = 0;
    return MTOMG_OK;
}

int mtomg_profile_read(mtomg_ctx* c, double* ms_out, int cap, int* launches) {
    if (!c || !launches || (cap > 0 && !ms_out)) return MTOMG_BAD_INPUT;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int k = 0; k + 1 < c->prof.used; k += 2) {
        if (k / 2 >= cap) break;
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->prof.ev[k], c->prof.ev[k + 1]));
        ms_out[k / 2] = ms;
    }
    *launches = c->prof.used / 2;
    c->prof.used = 0;
    return MTOMG_OK;
}

int mtomg_debug_apply(mtomg_ctx* c, int design, int level, int op, const void* in, void* out) {
    int rc = check_design(c, design, true);
    if (rc) return rc;
    rc = factor_pending(c);
    if (rc) return rc;
    Design& d = c->d[design];
    if (d.fac_failed) return fail(c, MTOMG_BREAKDOWN, "coarsest matrix is not positive definite");
    if (level < 0 || level >= d.levels) return fail(c, MTOMG_BAD_INPUT, "level out of range");
    if (!out) return fail(c, MTOMG_BAD_INPUT, "out must be a device pointer");
    hipStream_t st = c->stream;
    const LevelBufs& L = d.lev[level];
    const bool fine = level == d.fine();
    const size_t n = 2 * L.nodes();
    auto run = [&](auto tag) -> int {
        using T = decltype(tag);
        const T* vin = (const T*)in;
        T* vout = (T*)out;
        const LevelOp<T> opT = level_op<T>(d, level);
        const Mat<T> mat = make_mat<T>(d, d.omega);
        CaseBufs& cb = d.cases[0];
        CgRhs nocg{};
        ConvCheck nochk{};
        switch (op) {
            case MTOMG_OP_APPLY: launch_apply<T>(st, fine, false, opT, mat, L.sw_apply, vin, vout); break;
            case MTOMG_OP_DIAG: launch_apply<T>(st, fine, true, opT, mat, L.sw_apply, nullptr, vout); break;
            case MTOMG_OP_PRESMOOTH: {
                if (level == 0) return fail(c, MTOMG_BAD_INPUT, "no smoother on the coarsest level");
                T* t0 = (T*)cb.u2[level];
                T* t1 = (T*)cb.u4[level];
                CycleCtx<T> cx{&d, &cb, st, nullptr};
                if (d.n_pre == 0) { launch_fill<T>(st, vout, n, T(0)); break; }
                launch_presmooth<T>(st, fine, false, opT, mat, L.sw_pre, vin, t0, std::min(d.n_pre, 2), nocg, nullptr);
                T* cur = pre_chain_extra<T>(cx, level, t0, vin, t0, t1);
                HIPCHK(c, hipMemcpyAsync(vout, cur, n * sizeof(T), hipMemcpyDeviceToDevice, st));
                break;
            }
            case MTOMG_OP_PRESMOOTH_RESTRICT: {
                if (level == 0) return fail(c, MTOMG_BAD_INPUT, "no restriction from the coarsest level");
                if (d.n_pre != 2) return fail(c, MTOMG_BAD_INPUT, "the fused pre-smoothing runs two sweeps (n_pre = 2)");
                const size_t nc = 2 * d.lev[level - 1].nodes();
                launch_pre_restrict<T>(st, fine, false, false, opT, mat, L.sw_pr, vin, vout + nc, vout, nocg, nochk,
                                       nullptr);
                break;
            }
            case MTOMG_OP_RESIDUAL_RESTRICT:
                if (level == 0) return fail(c, MTOMG_BAD_INPUT, "no restriction from the coarsest level");
                launch_restrict<T>(st, fine, false, opT, mat, L.sw_res, vin, vin + n, vout, nochk, nullptr);
                break;
            case MTOMG_OP_PROLONG_POSTSMOOTH: {
                if (level == 0) return fail(c, MTOMG_BAD_INPUT, "no prolongation onto the coarsest level");
                CycleCtx<T> cx{&d, &cb, st, nullptr};
                post_chain<T>(cx, level, vin + n, vin + 2 * n, vin, vout, (T*)cb.u2[level], (T*)cb.u4[level], false,
                              nullptr, nullptr);
                break;
            }
            case MTOMG_OP_SMOOTH:
                if (level == 0) return fail(c, MTOMG_BAD_INPUT, "no smoother on the coarsest level");
                launch_post<T>(st, fine, false, false, opT, mat, L.sw_post, vin + n, nullptr, vin, vout, nullptr, nullptr, nullptr);
                break;
            case MTOMG_OP_COARSE_SOLVE:
                if (level != 0) return fail(c, MTOMG_BAD_INPUT, "coarse solve is on level 0");
                launch_coarse_solve<T>(st, d.Ainv, d.n0, d.np0, L.nx, vin, vout, nullptr);
                break;
            case MTOMG_OP_VCYCLE:
                if (level == 0) launch_coarse_solve<T>(st, d.Ainv, d.n0, d.np0, L.nx, vin, vout, nullptr);
                else {
                    const int r2 = debug_vcycle<T>(c, d, cb, st, level, vin, vout);
                    if (r2) return r2;
                }
                break;
            default: return fail(c, MTOMG_BAD_INPUT, "unknown op");
        }
        return MTOMG_OK;
    };
    if (op == MTOMG_OP_APPLY64) {
        if (!fine) return fail(c, MTOMG_BAD_INPUT, "APPLY64 is on the finest level");
        launch_apply<double>(st, true, false, level_op<double>(d, level), make_mat<double>(d, d.omega), L.sw_apply,
                             (const double*)in, (double*)out);
        LAUNCHCHK(c);
        return MTOMG_OK;
    }
    rc = d.mixed() ? run(float()) : run(double());
    if (rc) return rc;
    LAUNCHCHK(c);
    return MTOMG_OK;
}

}  // extern "C"
