#!/usr/bin/env python
"""Benchmark of the pCGMG hot path on one MI355X: 1024 x 1024 Q4 square wall.

One step = the whole path for one design: set_densities (element moduli,
Galerkin hierarchy), solve (coarsest Cholesky and inverse, then PCG with an
FP32 V-cycle inside FP64 CG to relative residual 1e-8) and compliance +
gradient.
Inputs (densities, loads) are resident in device memory before timing.

Prints ONE JSON line: the metric (DOF*iter/s over the timed steps), the
same workload with an all-FP64 cycle for comparison, the roofline of the
stiffness-apply kernel measured with HIP events on the solve stream during
the timed steps, and the oracle timed on the host CPU on a bounded sample.
"""

from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pCGMG DOF-iters/s & solve time, 1024² Q4, FP32-MG vs FP64 at rel.res 1e-8"
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6   # MI355X dense FP64 vector (256 CUs, 2.4 GHz)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_cg_apply_wall1024.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2301_07457_amd", "csrc", f)
                  for f in ("sweep_kernels.hip", "device_common.h", "kernels.h")]


def kernel_source_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the apply kernel from the committed counter
    summary, or None when it is missing or was taken on other kernel sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_digest") != kernel_source_digest():
        return None
    return t.get("hbm_bytes_per_launch")


def copy_calibration(mib: int, reps: int = 3):
    """A plain device-to-device copy of known size (the library's k_copy
    streaming kernel, one untimed pass + `reps`), for scaling the
    FETCH_SIZE / WRITE_SIZE counters to bytes."""
    import torch
    from paper_2301_07457_amd import PCGMGSolver, _lib
    s = PCGMGSolver(max_designs=1)
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    _lib.mtomg_stream_probe(s.ctx, "COPY", a.data_ptr(), b.data_ptr(), 0, n, reps)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_each_way": n * 8, "dispatches": reps + 1}))


def cpu_baseline_worker(n: int, levels: int, warmup: int, runs: int):
    """Oracle pCGMG (FP64, scipy sparse) on the same recipe at n x n: `warmup`
    untimed runs, then `runs` timed runs of setup + solve to 1e-8 + gradient
    (the GPU step's work); prints one JSON line with per-run wall and CPU
    times (CPU time / wall time = host threads actually busy)."""
    from oracle import solve
    from workloads import make_problem
    p = make_problem("wall1024", n=n, levels=levels)
    rows = []
    for k in range(warmup + runs):
        t0, c0 = time.perf_counter(), time.process_time()
        s = solve.solve_mgpcg(p.nelx, p.nely, p.x, p.E_phase, p.E_min, p.penal, p.nu, p.F, p.levels,
                              rel_tol=1e-8, grad=True)
        t1, c1 = time.perf_counter(), time.process_time()
        if k >= warmup:
            rows.append(dict(t_total=t1 - t0, cpu_s=c1 - c0, t_setup=s.t_setup, t_solve=s.t_solve,
                             iters=int(s.iters[0]), relres=float(s.relres[0])))
    print(json.dumps(dict(n_dof=p.n_dof, runs=rows)))


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_cpu_baseline(n: int, levels: int):
    """The oracle timed on the host: all host threads allowed (median of 3
    runs after one warm-up run), and one run restricted to one thread."""
    import numpy as np
    nproc = os.cpu_count() or 1
    out = {}
    for label, threads, warmup, runs in (("all", nproc, 1, 3), ("one", 1, 0, 1)):
        env = dict(os.environ)
        for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
            env[k] = str(threads)
        env["HIP_VISIBLE_DEVICES"] = ""
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-worker",
                            "--cpu-n", str(n), "--cpu-levels", str(levels), "--cpu-warmup", str(warmup),
                            "--cpu-runs", str(runs)],
                           capture_output=True, text=True, env=env, timeout=900)
        if r.returncode != 0:
            return dict(error=r.stderr[-500:])
        d = json.loads(r.stdout.strip().splitlines()[-1])
        t = float(np.median([q["t_total"] for q in d["runs"]]))
        out[label] = dict(n_dof=d["n_dof"], iters=d["runs"][0]["iters"], t_total=t,
                          busy_threads=float(np.mean([q["cpu_s"] / q["t_total"] for q in d["runs"]])),
                          t_setup=float(np.median([q["t_setup"] for q in d["runs"]])),
                          t_solve=float(np.median([q["t_solve"] for q in d["runs"]])),
                          relres=d["runs"][0]["relres"], threads_allowed=threads, runs=len(d["runs"]))
    a, o = out["all"], out["one"]
    return dict(value=a["n_dof"] * a["iters"] / a["t_total"], unit="DOF*iter/s",
                cores=round(a["busy_threads"], 2), kind="oracle",
                sample=(f"oracle pCGMG (scipy CSR, FP64) on the bench workload itself ({n}x{n} Q4, {levels} "
                        f"levels, smooth 3-phase recipe): setup + solve to 1e-8 + gradient per run, median of "
                        f"{a['runs']} runs after 1 warm-up with {nproc} host threads allowed; scipy's sparse "
                        f"kernels are single-threaded, so on average {a['busy_threads']:.2f} threads were busy "
                        f"(CPU time / wall time); {a['iters']} iterations, setup {a['t_setup']:.2f} s, "
                        f"solve {a['t_solve']:.2f} s"),
                host={"cpu_model": host_cpu_model(), "nproc": nproc},
                solve_only_value=a["n_dof"] * a["iters"] / a["t_solve"],
                one_thread={"value": o["n_dof"] * o["iters"] / o["t_total"], "t_total": o["t_total"],
                            "t_setup": o["t_setup"], "t_solve": o["t_solve"], "runs": o["runs"]})


GOLDEN_DIR = os.path.join(ROOT, "tests", "golden")


def oracle_error(name, case, U, c, dc, m):
    """Relative error of one GPU result (load case `case`) against the
    oracle's stored samples of workload `name` (tests/golden, written by
    make_golden.py from the oracle alone): u at 512 nodes, ||u||, the
    compliance and the gradient at 64 (element, phase) pairs; max over
    entries, relative to the largest sample."""
    import numpy as np
    path = os.path.join(GOLDEN_DIR, f"{name}_samples.json")
    if not os.path.exists(path):
        return "parity unpinned (no oracle samples for this workload)"
    g = json.load(open(path))
    k = g["cases"][case]
    Uf = np.asarray(U, dtype=np.float64).reshape(-1, 2)
    un = np.array(k["u_nodes"])
    gd = np.asarray(dc, dtype=np.float64).reshape(-1, m)[g["grad_elems"], g["grad_phases"]]
    gr = np.array(k["grad"])
    return {
        "u_sampled_max_rel": float(np.max(np.abs(Uf[g["nodes"]] - un)) / np.max(np.abs(un))),
        "u_norm_rel": float(abs(np.linalg.norm(U) - k["u_norm"]) / k["u_norm"]),
        "compliance_rel": float(abs(c - g["compliance"][case]) / abs(g["compliance"][case])),
        "grad_sampled_max_rel": float(np.max(np.abs(gd - gr)) / np.max(np.abs(gr))),
        "oracle": g["source"],
    }


def stream_ceiling(mib: int = 1024, reps: int = 20):
    """The practical HBM ceiling: the library's hand-written streaming kernels
    (mtomg_stream_probe: 16-byte loads and stores, 8 workgroups per compute
    unit) over arrays of `mib` MiB each, device time per pass from HIP
    events; GB/s counts bytes read + bytes written."""
    import torch
    from paper_2301_07457_amd import PCGMGSolver, _lib
    s = PCGMGSolver(max_designs=1)
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.ones_like(a)
    c = torch.ones_like(a)
    out = {}
    for kind, nbytes in (("READ", 8 * n), ("COPY", 16 * n), ("TRIAD", 24 * n)):
        ms = _lib.mtomg_stream_probe(s.ctx, kind, a.data_ptr(), b.data_ptr(), c.data_ptr(), n, reps)
        out[kind.lower() + "_gbs"] = nbytes / (ms * 1e-3) / 1e9
    del a, b, c
    return out


def gpu_run(prob, precision, steps, warmup, profile_kernel=None, tiles=None):
    """Time `steps` steps; the tiles (rows per wave: the ROWS_* options) are
    autotuned first unless given as a dict.  Returns the solver, per-step
    stats, elapsed seconds, profiled durations, U and (tiles, timings)."""
    import torch
    from paper_2301_07457_amd import PCGMGSolver
    from paper_2301_07457_amd import _lib
    s = PCGMGSolver(max_designs=1)
    s.add_design(0, prob.nelx, prob.nely, torch.from_numpy(prob.F), list(prob.E_phase), prob.E_min,
                 prob.penal, prob.nu, prob.levels, prob.n_pre, prob.n_post, prob.omega, precision)
    x = torch.from_numpy(prob.x).cuda()
    s.set_densities(0, x)
    tune = None
    if tiles is None:
        _, t = s.autotune(1e-8, 1000)
        tiles = dict(s.tuned)
        tune = {(f"{k[0]},{k[1]}" if isinstance(k, tuple) else k): round(v, 4) for k, v in t.items()}
    else:
        for name, v in tiles.items():
            s.set_option(name, v)

    last = {}

    def step():
        s.set_densities(0, x)
        st = s.solve(1e-8, 1000)[0]
        last["c"], last["dc"] = s.compliance_and_grad(0, grad=True)
        return st

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    if profile_kernel:
        _lib.mtomg_profile_kernel(s.ctx, profile_kernel)
        _lib.mtomg_profile_read(s.ctx)
    durs = []
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        st = step()
        stats.append(st)
        if profile_kernel:
            d = _lib.mtomg_profile_read(s.ctx)
            # launches 1 .. iters-1 are full iterations (0 has no x update,
            # later ones may find the solve converged)
            durs.extend(d[1:st["iters"]])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if profile_kernel:
        _lib.mtomg_profile_kernel(s.ctx, "NONE")
    U = s.U(0).clone()
    s.last_c, s.last_dc = last["c"], last["dc"]
    return s, stats, t1 - t0, durs, U, (tiles, tune)


def batched_run(steps, warmup, per_size=16):
    """The batched workload: 3 x per_size designs (128^2 with 4 levels,
    384^2 with 5, 768^2 with 6; smooth 3-phase fields, seeds 1000 + d), four
    load cases each, FP32 cycle in FP64 CG to 1e-8.  One step = densities
    of every design + one solve of all systems + compliance and gradient of
    every design."""
    import numpy as np
    import torch
    from paper_2301_07457_amd import PCGMGSolver
    from workloads.square_wall import batched_designs
    probs = batched_designs(per_size=per_size)
    s = PCGMGSolver(max_designs=len(probs))
    for k, p in enumerate(probs):
        s.add_design(k, p.nelx, p.nely, torch.from_numpy(p.F), list(p.E_phase), p.E_min, p.penal, p.nu,
                     p.levels, p.n_pre, p.n_post, p.omega, "fp32mg")
    xs = [torch.from_numpy(p.x).cuda() for p in probs]
    for k, x in enumerate(xs):
        s.set_densities(k, x)
    _, tune = s.autotune(1e-8, 1000, repeats=1)
    tiles = dict(s.tuned)

    def step():
        for k, x in enumerate(xs):
            s.set_densities(k, x)
        st = s.solve(1e-8, 1000)
        for k in range(len(probs)):
            s.compliance_and_grad(k, grad=True)
        return st

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    all_stats = [step() for _ in range(steps)]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # design 32 (768^2) against the oracle's direct-solve samples, every load case
    err = "parity unpinned (design 32 not in this run)"
    if len(probs) > 32 and probs[32].nelx == 768:
        c32, dc32 = s.compliance_and_grad(32, grad=True)
        U32 = s.U(32).cpu().numpy()
        err = {f"case{k}": oracle_error("batch32", k, U32[k], c32[k].item(), dc32[k].cpu().numpy(), probs[32].m)
               for k in range(4)}
    dof_iters = sum(st["n_dof"] * st["iters"] for stats in all_stats for st in stats)
    last = all_stats[-1]
    n_sys = len(last)
    return {
        "workload": (f"{len(probs)} designs (128^2 L4, 384^2 L5, 768^2 L6, {per_size} each) x 4 load cases, "
                     f"FP32 cycle in FP64 CG to rel.res 1e-8, one solve call per step"),
        "systems": n_sys,
        "dof_rhs": int(sum(st["n_dof"] for st in last)),
        "value": dof_iters / el,
        "unit": "DOF*iter/s",
        "solves_per_s": n_sys * steps / el,
        "ms_per_step": 1e3 * el / steps,
        "solve_ms": float(np.mean([stats[0]["t_solve_ms"] for stats in all_stats])),
        "iters_max": max(st["iters"] for st in last),
        "iters_min": min(st["iters"] for st in last),
        "relres_true_max": max(st["relres_true"] for st in last),
        "all_ok": all(st["status"] == 0 for st in last),
        "error_vs_oracle_design32": err,
        "tiles": {"rows": tiles, "autotune_solve_ms": {(f"{k[0]},{k[1]}" if isinstance(k, tuple) else k): round(v, 3)
                                                      for k, v in tune.items()}},
    }


def cycle_sweep(n, precision, reps=3):
    """Levels and cycle index at a fixed mesh (Section 2.1: the number of
    levels and gamma of Algorithm 1): for every admissible L (coarsest grid
    from the library's 8192-element limit down to 1 element per side) and
    gamma in (1, 2), the smooth
    3-phase wall at n^2 solved to 1e-8 from new densities.  Per setting:
    iterations, set_densities time, solve time (device time of the solve
    call, the overlapped coarsest factorisation included), time per
    iteration; medians over `reps` steps after one warm-up step, library
    tile choice."""
    import numpy as np
    import torch
    from paper_2301_07457_amd import PCGMGSolver
    from workloads import make_problem
    rows = []
    L_min = 2
    while (n >> (L_min - 1)) ** 2 > 8192:
        L_min += 1
    L_max = int(np.log2(n)) + 1
    for L in range(L_min, L_max + 1):
        prob = make_problem("wall1024", n=n, levels=L, mixed=precision == "fp32mg")
        x = torch.from_numpy(prob.x).cuda()
        for gamma in (1, 2):
            s = PCGMGSolver(max_designs=1)
            s.add_design(0, prob.nelx, prob.nely, torch.from_numpy(prob.F), list(prob.E_phase), prob.E_min,
                         prob.penal, prob.nu, L, prob.n_pre, prob.n_post, prob.omega, precision)
            s.set_option("GAMMA", gamma)
            st_all = []
            for k in range(reps + 1):
                s.set_densities(0, x)
                st = s.solve(1e-8, 1000)[0]
                if k > 0:
                    st_all.append(st)
            torch.cuda.synchronize()
            solve_ms = float(np.median([st["t_solve_ms"] for st in st_all]))
            it = st_all[-1]["iters"]
            rows.append({"levels": L, "coarsest": f"{n >> (L - 1)}^2", "gamma": gamma,
                         "cycle": "V" if gamma == 1 else "W", "iters": it,
                         "setup_ms": round(float(np.median([st["t_setup_ms"] for st in st_all])), 4),
                         "solve_ms": round(solve_ms, 4),
                         "ms_per_iter": round(solve_ms / max(1, it), 4),
                         "status": st_all[-1]["status"], "relres_true": st_all[-1]["relres_true"]})
            print(f"[cycle sweep] n={n} L={L} gamma={gamma}: {rows[-1]}", file=sys.stderr, flush=True)
            del s
    return rows


PAPER_MESHES = ((32, 32), (32, 64), (64, 64), (64, 128), (128, 128), (128, 256))


def paper_mesh_sweep(reps=3):
    """The meshes of the paper's level study (Tables 3-5: 32 x 32 ... 128 x
    256) with every level count from the two-grid method (l = 2) to a
    1-element coarsest side: one solve of the wall with smooth 3-phase
    densities to 1e-8, FP64 V-cycle (the paper's pCGMG), per setting the
    iterations, the set_densities time and the solve time (device time; the
    coarsest factorisation, overlapped with the start of the solve, is in
    it), medians over `reps` steps after one warm-up.  A single solve, not
    the paper's whole optimisation runs."""
    import numpy as np
    import torch
    from paper_2301_07457_amd import PCGMGSolver
    from workloads import Problem, density_gaussian_sum, load_top_traction
    rows = []
    for nx, ny in PAPER_MESHES:
        x = density_gaussian_sum(nx, ny, 2)
        F = torch.from_numpy(load_top_traction(nx, ny)[None])
        xt = torch.from_numpy(x).cuda()
        L = 2
        while (min(nx, ny) >> (L - 1)) >= 1 and min(nx, ny) % (1 << (L - 1)) == 0:
            if (nx >> (L - 1)) * (ny >> (L - 1)) <= 8192:
                s = PCGMGSolver(max_designs=1)
                s.add_design(0, nx, ny, F, [1.0, 0.6, 0.2], 1e-9, 3.0, 0.3, L, 2, 2, 0.6, "fp64")
                sts = []
                for k in range(reps + 1):
                    s.set_densities(0, xt)
                    st = s.solve(1e-8, 2000)[0]
                    if k > 0:
                        sts.append(st)
                torch.cuda.synchronize()
                rows.append({"mesh": f"{nx}x{ny}", "levels": L, "coarsest": f"{nx >> (L - 1)}x{ny >> (L - 1)}",
                             "iters": sts[-1]["iters"],
                             "setup_ms": round(float(np.median([t["t_setup_ms"] for t in sts])), 4),
                             "solve_ms": round(float(np.median([t["t_solve_ms"] for t in sts])), 4),
                             "status": sts[-1]["status"], "relres_true": sts[-1]["relres_true"]})
                print(f"[paper meshes] {rows[-1]}", file=sys.stderr, flush=True)
                del s
            L += 1
    return {"workload": "square wall, smooth 3-phase densities (seed 2), FP64 V-cycle (2+2 damped Jacobi, "
                        "omega 0.6), rel.res 1e-8, the meshes of the paper's Tables 3-5",
            "rows": rows}


def filter_run(n=1024, m=3, rf=8.0, reps=20):
    """The cone filter of the optimisation loop (radius rf = 8 of Table 2) on
    an n^2 three-phase field: device time per call of each mode (HIP events
    around `reps` back-to-back calls after a warm-up), and its roofline as
    FP64 vector arithmetic: one multiply-add per positive weight, phase and
    element."""
    import math
    import numpy as np
    import torch
    from paper_2301_07457_amd import PCGMGSolver
    s = PCGMGSolver(max_designs=1)
    g = torch.randn((n, n, m), dtype=torch.float64, device="cuda")
    x = torch.rand((n, n, m), dtype=torch.float64, device="cuda")
    R = max(0, math.ceil(rf) - 1)
    taps = sum(1 for dj in range(-R, R + 1) for di in range(-R, R + 1) if rf - math.hypot(di, dj) > 0)
    out = {"workload": f"{n}x{n} elements, {m} phases, rf = {rf:g} ({taps} weights per element)"}
    for mode in ("DENSITY", "DENSITY_ADJOINT", "SENSITIVITY"):
        s.filter(g, rf, mode, x)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            s.filter(g, rf, mode, x)
        e1.record()
        torch.cuda.synchronize()
        out[mode.lower() + "_us"] = round(1e3 * e0.elapsed_time(e1) / reps, 2)
    flops = 2.0 * taps * n * n * m
    achieved = flops / (out["density_us"] * 1e-6) / 1e12
    out["roofline"] = {"kernel": "k_cone_filter (density mode)", "bound": "alu", "achieved": achieved,
                       "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                       "flops_per_call": flops}
    return out


def poisson_run(sizes=(16, 32, 64, 128, 256, 1024, 2048), reps=5):
    """The Poisson model problem of Section 5.1 (unit source, zero boundary
    values, V-cycle down to the 2 x 2 grid): iterations to 1e-8 and device
    time of the solve call (median of `reps` after one warm-up) per mesh."""
    import numpy as np
    import torch
    from paper_2301_07457_amd import PCGMGSolver
    s = PCGMGSolver(max_designs=1)
    rows = []
    for n in sizes:
        # consistent loads of f = 1: h^2 at every interior node
        F = torch.full((n + 1, n + 1), 1.0 / (n * n), dtype=torch.float64, device="cuda")
        s.poisson_solve(F, 1e-8, 1000)
        sts = [s.poisson_solve(F, 1e-8, 1000)[1] for _ in range(reps)]
        ms = float(np.median([st["t_solve_ms"] for st in sts]))
        it = sts[-1]["iters"]
        rows.append({"n": n, "levels": int(np.log2(n)), "unknowns": (n - 1) ** 2, "iters": it, "solve_ms": round(ms, 4),
                     "dof_iter_per_s": (n - 1) ** 2 * it / (ms * 1e-3), "relres_true": sts[-1]["relres_true"]})
    return {"workload": "-Laplace(u) = 1 on the unit square, u = 0 on the boundary, Q4, FP64 PCG with a "
                        "V-cycle (2+2 damped Jacobi, omega 0.6) down to the 2x2 grid, rel.res 1e-8",
            "error_vs_oracle": "parity unpinned in this run (true residual per row; the oracle comparison is "
                               "the GPU test suite's, 4^2 to 256^2)",
            "rows": rows}


def oc_run(n=1024, levels=7, steps=2):
    """The alternating active-phase OC loop (Section 4) on the square wall with
    the moduli and volume fractions of Table 2 (E = 9, 3, 1, void 1e-9;
    V = 0.16, 0.08, 0.08, 0.68), rf = 8, FP32 cycle: device-synchronised
    wall time of one outer iteration (six pairs, each set_densities + warm
    solve to 1e-8 + gradient + sensitivity filter + pair update) after one
    warm-up iteration from the uniform start, and the pair update alone
    (HIP events around 10 calls on a resident state)."""
    import numpy as np
    import torch
    from paper_2301_07457_amd import PCGMGSolver
    from workloads import load_top_traction
    vols = [0.16, 0.08, 0.08, 0.68]
    E = [9.0, 3.0, 1.0]
    F = torch.from_numpy(load_top_traction(n, n)[None])
    s = PCGMGSolver(max_designs=1)
    s.add_design(0, n, n, F, E, 1e-9, 3.0, 0.3, levels, 2, 2, 0.6, "fp32mg")
    x = torch.tensor(vols[:3], dtype=torch.float64, device="cuda").expand(n, n, 3).contiguous()
    s.aap_step(0, x, vols, rf=8.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = [s.aap_step(0, x, vols, rf=8.0) for _ in range(steps)]
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    # the pair update alone: phases (0, 3) of the current state, a fixed gradient
    g = -torch.rand((n, n, 3), dtype=torch.float64, device="cuda") - 0.1
    xs = x.clone()
    s.oc_update(xs, g, 0, 3, vols[0])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    info = s.oc_update(xs, g, 0, 3, vols[0])
    e0.record()
    for _ in range(10):
        xs.copy_(x)
        s.oc_update(xs, g, 0, 3, vols[0], info=False)
    e1.record()
    torch.cuda.synchronize()
    # the copy of x is timed too: subtract it
    e2, e3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e2.record()
    for _ in range(10):
        xs.copy_(x)
    e3.record()
    torch.cuda.synchronize()
    upd_ms = (e0.elapsed_time(e1) - e2.elapsed_time(e3)) / 10
    return {
        "workload": (f"square wall {n}x{n}, Table 2 moduli and volume fractions, rf = 8, FP32 cycle in FP64 CG "
                     f"to 1e-8 (warm-started), {levels} levels; one outer iteration = 6 phase pairs"),
        "ms_per_outer_iteration": 1e3 * el,
        "compliance_before_each_pair": hist[-1][0],
        "change": hist[-1][1],
        "pcg_iterations_per_pair": hist[-1][2],
        "pair_update_ms": upd_ms,
        "pair_update_newton_passes": info[3],
    }


def kernel_breakdown(prob, precision):
    """Average device ms per launch of each finest-grid kernel over one solve."""
    import torch
    from paper_2301_07457_amd import PCGMGSolver, _lib
    s = PCGMGSolver(max_designs=1)
    s.add_design(0, prob.nelx, prob.nely, torch.from_numpy(prob.F), list(prob.E_phase), prob.E_min,
                 prob.penal, prob.nu, prob.levels, prob.n_pre, prob.n_post, prob.omega, precision)
    x = torch.from_numpy(prob.x).cuda()
    s.set_densities(0, x)
    s.solve(1e-8, 1000)
    out = {}
    for k in ("CG_APPLY", "FINE_PRESMOOTH", "FINE_RESTRICT", "FINE_POST", "FINE_POST_DOT", "COARSE_SOLVE"):
        _lib.mtomg_profile_kernel(s.ctx, k)
        _lib.mtomg_profile_read(s.ctx)
        st = s.solve(1e-8, 1000)[0]
        d = _lib.mtomg_profile_read(s.ctx)
        real = d[1:st["iters"]]
        out[k] = round(1e3 * sum(real) / max(1, len(real)), 2)
    _lib.mtomg_profile_kernel(s.ctx, "NONE")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1024, help="grid size (elements per side)")
    ap.add_argument("--levels", type=int, default=7)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--breakdown", action="store_true", help="add per-kernel average times")
    ap.add_argument("--no-batched", action="store_true", help="skip the 48-design batched workload")
    ap.add_argument("--no-oc", action="store_true", help="skip the OC loop timing")
    ap.add_argument("--no-cycle-sweep", action="store_true", help="skip the level / cycle-index sweep")
    ap.add_argument("--no-paper-meshes", action="store_true", help="skip the level sweep on the paper's meshes")
    ap.add_argument("--tiles", default=None, metavar="RF,RC[,RCG,R1,R2]",
                    help="rows per wave instead of autotuning (0 = library choice): finest grid, coarse grids, "
                         "and optionally the outer-CG apply and the first two grids below the finest")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain copy of MIB MiB (counter calibration)")
    ap.add_argument("--cycle-sweep", action="store_true",
                    help="instead of the benchmark: iterations and times for every number of levels "
                         "and gamma in (1, 2) at --n (one JSON line)")
    ap.add_argument("--precision", default="fp32mg", choices=("fp32mg", "fp64"),
                    help="precision of the V-cycle for --cycle-sweep")
    ap.add_argument("--cpu-baseline-worker", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--cpu-n", type=int, default=256, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-levels", type=int, default=5, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-warmup", type=int, default=0, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-runs", type=int, default=1, help=argparse.SUPPRESS)
    args = ap.parse_args()

    if args.cpu_baseline_worker:
        cpu_baseline_worker(args.cpu_n, args.cpu_levels, args.cpu_warmup, args.cpu_runs)
        return
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this solver runs on one GPU; multi-GPU runs are not supported "
              "(independent designs would shard over GPUs with no communication)", file=sys.stderr)
        sys.exit(2)

    if args.cycle_sweep:
        rows = cycle_sweep(args.n, args.precision)
        print(json.dumps({"metric": "pCGMG iterations and solve time against levels and cycle index",
                          "workload": (f"square wall {args.n}x{args.n} Q4, smooth 3-phase Gaussian-sum densities "
                                       f"(seed 2), {args.precision}, 2+2 damped Jacobi omega 0.6, rel.res 1e-8"),
                          "unit": "ms", "data": "synthetic", "rows": rows}))
        return

    import numpy as np
    import torch
    from workloads import make_problem

    prob = make_problem("wall1024", n=args.n, levels=args.levels, mixed=True)
    n_dof = prob.n_dof
    n_nodes = (prob.nelx + 1) * (prob.nely + 1)
    n_elem = prob.nelx * prob.nely

    # timed pass: graph-replayed iterations, nothing instrumented
    fixed = None
    if args.tiles:
        vals = [int(v) for v in args.tiles.split(",")]
        fixed = dict(zip(("ROWS_FINE", "ROWS_COARSE", "ROWS_CG", "ROWS_LEVEL1", "ROWS_LEVEL2"), vals))
    s, stats, elapsed, _, U32, (tiles, tune) = gpu_run(prob, "fp32mg", args.steps, args.warmup, tiles=fixed)
    iters_total = sum(st["iters"] for st in stats)
    value = n_dof * iters_total / elapsed
    solve_ms = float(np.mean([st["t_solve_ms"] for st in stats]))
    setup_ms = float(np.mean([st["t_setup_ms"] for st in stats]))
    iters = stats[-1]["iters"]
    golden = "wall1024" if (prob.nelx, prob.nely, prob.levels) == (1024, 1024, 7) else None
    err32 = (oracle_error(golden, 0, U32[0].cpu().numpy(), s.last_c[0].item(), s.last_dc[0].cpu().numpy(), prob.m)
             if golden else "parity unpinned (no oracle samples at this size)")
    del s
    # roofline pass: same steps, kernels launched one by one so every launch of
    # the stiffness apply is bracketed by HIP events on the solve stream
    s, stats_r, elapsed_r, durs, _, _ = gpu_run(prob, "fp32mg", args.steps, 1, "CG_APPLY", tiles=tiles)
    del s

    # roofline of the FP64 stiffness apply of the outer CG: algorithmic bytes per launch
    # (read z (FP32), p_old, x, E; write p, q, x)
    bytes_apply = n_nodes * (8 + 16 + 16 + 16 + 16 + 16) + n_elem * 8
    avg_ms = float(np.mean(durs)) if durs else float("nan")
    achieved = bytes_apply / (avg_ms * 1e-3) / 1e9

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "DOF*iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": (f"square wall {prob.nelx}x{prob.nely} Q4 plane stress, {n_dof} DOFs, "
                         f"{prob.levels}-level V-cycle (2+2 damped Jacobi, omega 0.6, Galerkin coarse "
                         f"operators, FP64 Cholesky on {prob.nelx >> (prob.levels - 1)}^2), FP32 cycle "
                         f"inside FP64 CG to rel.res 1e-8; smooth 3-phase Gaussian-sum densities "
                         f"(seed 2), SIMP p=3, E=(1,0.6,0.2), Emin=1e-9; step = set_densities + "
                         f"solve + compliance/gradient"),
            "n_dof": n_dof,
            "iters": iters,
            "solve_ms": solve_ms,
            "setup_ms": setup_ms,
            "relres_true": stats[-1]["relres_true"],
            "error_vs_oracle": err32,
            "tiles": {"rows": tiles, "autotune_solve_ms": tune},
        },
        "roofline": {
            "kernel": "k_cg_apply (FP64 p-update + stiffness apply + p.q)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(),
            "bytes_per_launch": bytes_apply,
            "avg_launch_us": avg_ms * 1e3,
            "launches_timed": len(durs),
            "timing": "HIP events stamped by each launch's own dispatch (hipExtLaunchKernel) on the solve "
                      "stream, in a second pass of the same steps with eager launches",
            "eager_pass_ms_per_step": 1e3 * elapsed_r / args.steps,
        },
    }
    ceil = stream_ceiling()
    best = max(ceil["copy_gbs"], ceil["triad_gbs"])
    out["roofline"]["stream_ceiling_gbs"] = ceil
    out["roofline"]["frac_of_stream_ceiling"] = achieved / best
    if not args.no_fp64:
        s64, stats64, el64, _, U64, (tiles64, _) = gpu_run(prob, "fp64", max(3, args.steps // 2), 1)
        it64 = sum(st["iters"] for st in stats64)
        out["fp64_cycle"] = {
            "value": n_dof * it64 / el64,
            "ms_per_step": 1e3 * el64 / len(stats64),
            "solve_ms": float(np.mean([st["t_solve_ms"] for st in stats64])),
            "iters": stats64[-1]["iters"],
            "relres_true": stats64[-1]["relres_true"],
            "error_vs_oracle": (oracle_error(golden, 0, U64[0].cpu().numpy(), s64.last_c[0].item(),
                                             s64.last_dc[0].cpu().numpy(), prob.m)
                                if golden else "parity unpinned (no oracle samples at this size)"),
            "tiles": {"rows": tiles64},
        }
        out["fp32mg_vs_fp64_solve_speedup"] = out["fp64_cycle"]["solve_ms"] / solve_ms
        out["fp32mg_vs_fp64_rel_diff_u"] = float(torch.linalg.norm(U32 - U64) / torch.linalg.norm(U64))
        del s64
    if not args.no_batched:
        out["batched"] = batched_run(max(2, args.steps // 5), 1)
    if args.breakdown:
        out["kernel_avg_us_fp32mg"] = kernel_breakdown(prob, "fp32mg")
    out["filter"] = filter_run()
    if not args.no_oc:
        out["oc"] = oc_run()
    out["poisson"] = poisson_run()
    if not args.no_paper_meshes:
        out["paper_meshes"] = paper_mesh_sweep()
    if not args.no_cycle_sweep:
        # levels and cycle index at the bench mesh (Section 2.1), one timed step per setting
        out["cycle_sweep"] = {"workload": (f"square wall {args.n}x{args.n}, smooth 3-phase densities, FP32 cycle, "
                                           f"rel.res 1e-8, new densities per step, library tiles"),
                              "rows": cycle_sweep(args.n, "fp32mg", reps=1)}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = run_cpu_baseline(args.n, args.levels)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
