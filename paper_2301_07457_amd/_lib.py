"""ctypes binding of libmtomg.so: the C ABI of include/mtomg.h, same names.

Argument marshalling only: every computation happens in the HIP library.
Loading fails loudly (ImportError) when the library has not been built.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmtomg.so")

MTOMG_OK = 0
MTOMG_BAD_INPUT = -1
MTOMG_NOT_CONVERGED = -2
MTOMG_BREAKDOWN = -3
MTOMG_NAN = -4
MTOMG_WORKSPACE = -5
MTOMG_HIP_ERROR = -6
MTOMG_STATE = -7

MTOMG_FP64 = 0
MTOMG_FP32MG = 1

OPS = dict(APPLY=0, APPLY64=1, DIAG=2, PRESMOOTH=3, RESIDUAL_RESTRICT=4, PROLONG_POSTSMOOTH=5,
           SMOOTH=6, COARSE_SOLVE=7, VCYCLE=8, PRESMOOTH_RESTRICT=9)

EXPORTS = ["mtomg_create", "mtomg_destroy", "mtomg_set_grid", "mtomg_workspace_bytes",
           "mtomg_set_workspace", "mtomg_set_densities", "mtomg_solve",
           "mtomg_compliance_and_grad", "mtomg_status_string", "mtomg_last_error",
           "mtomg_debug_apply", "mtomg_profile_kernel", "mtomg_profile_read",
           "mtomg_set_option", "mtomg_filter", "mtomg_poisson_solve", "mtomg_filter_noalloc",
           "mtomg_oc_update", "mtomg_aap_step", "mtomg_stream_probe"]

OPTIONS = dict(GRAPHS=0, BATCH=1, ROWS_FINE=2, ROWS_COARSE=3, DENSE_FACTOR=4, GAMMA=5, RESTARTS=6, ROWS_CG=7,
               FUSE_PRE=8, ROWS_LEVEL=16)


def option_code(name: str) -> int:
    """Option number: a name of OPTIONS, or ROWS_LEVEL<k> for MTOMG_OPT_ROWS_LEVEL + k."""
    if name.startswith("ROWS_LEVEL") and name != "ROWS_LEVEL":
        return OPTIONS["ROWS_LEVEL"] + int(name[len("ROWS_LEVEL"):])
    return OPTIONS[name]

FILTERS = dict(DENSITY=0, DENSITY_ADJOINT=1, SENSITIVITY=2)

PROBES = dict(READ=0, COPY=1, TRIAD=2)

KERNELS = dict(NONE=0, CG_APPLY=1, FINE_PRESMOOTH=2, FINE_RESTRICT=3, FINE_POST=4, FINE_POST_DOT=5,
               COARSE_SOLVE=6)


class mtomg_stats(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("iters", ctypes.c_int32),
        ("vcycles", ctypes.c_int32),
        ("n_dof", ctypes.c_int32),
        ("relres_rec", ctypes.c_double),
        ("relres_true", ctypes.c_double),
        ("t_setup_ms", ctypes.c_double),
        ("t_solve_ms", ctypes.c_double),
        ("model_bytes", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class MtomgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"mtomg status {status}: {msg}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libmtomg.so (once).  Raises ImportError if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with `python -m paper_2301_07457_amd.build` "
                          "(the solver has no CPU fallback)")
    lib = ctypes.CDLL(path)
    vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    dp = ctypes.c_void_p
    lib.mtomg_create.argtypes = [ctypes.POINTER(vp), i, vp]
    lib.mtomg_destroy.argtypes = [vp]
    lib.mtomg_set_grid.argtypes = [vp, i, i, i, d, i, ctypes.POINTER(d), d, d, i, i, i, d, i, i, dp, dp]
    lib.mtomg_workspace_bytes.argtypes = [vp]
    lib.mtomg_workspace_bytes.restype = sz
    lib.mtomg_set_workspace.argtypes = [vp, vp, sz]
    lib.mtomg_set_densities.argtypes = [vp, i, dp]
    lib.mtomg_solve.argtypes = [vp, d, i, i, ctypes.POINTER(mtomg_stats)]
    lib.mtomg_compliance_and_grad.argtypes = [vp, i, dp, dp]
    lib.mtomg_status_string.argtypes = [i]
    lib.mtomg_status_string.restype = ctypes.c_char_p
    lib.mtomg_last_error.argtypes = [vp]
    lib.mtomg_last_error.restype = ctypes.c_char_p
    lib.mtomg_debug_apply.argtypes = [vp, i, i, i, dp, dp]
    lib.mtomg_profile_kernel.argtypes = [vp, i]
    lib.mtomg_set_option.argtypes = [vp, i, i]
    lib.mtomg_filter.argtypes = [vp, i, i, i, d, i, d, dp, dp, dp]
    lib.mtomg_filter_noalloc.argtypes = [vp, i, i, i, d, i, d, dp, dp, dp]
    lib.mtomg_stream_probe.argtypes = [vp, i, dp, dp, dp, sz, i, ctypes.POINTER(d)]
    lib.mtomg_oc_update.argtypes = [vp, i, i, i, i, i, dp, d, d, d, d, dp, ctypes.POINTER(d)]
    lib.mtomg_aap_step.argtypes = [vp, i, ctypes.POINTER(d), d, d, d, d, d, d, i, dp, ctypes.POINTER(d),
                                   ctypes.POINTER(d), ctypes.POINTER(i)]
    lib.mtomg_poisson_solve.argtypes = [vp, i, i, i, d, d, i, dp, dp, ctypes.POINTER(mtomg_stats)]
    lib.mtomg_profile_read.argtypes = [vp, ctypes.POINTER(d), i, ctypes.POINTER(i)]
    for name in EXPORTS:
        if name not in ("mtomg_workspace_bytes", "mtomg_status_string", "mtomg_last_error"):
            getattr(lib, name).restype = i
    _lib = lib
    return lib


def check(ctx, status: int, allow=()):
    """Raise MtomgError for a negative status not listed in `allow`."""
    if status == MTOMG_OK or status in allow:
        return status
    lib = load()
    msg = lib.mtomg_last_error(ctx).decode() if ctx else lib.mtomg_status_string(status).decode()
    raise MtomgError(status, msg)


# Thin same-name wrappers -----------------------------------------------------

def mtomg_create(max_designs: int, stream: int = 0):
    lib = load()
    ctx = ctypes.c_void_p()
    check(None, lib.mtomg_create(ctypes.byref(ctx), max_designs, ctypes.c_void_p(stream or None)))
    return ctx


def mtomg_destroy(ctx):
    return load().mtomg_destroy(ctx)


def mtomg_set_grid(ctx, design, nelx, nely, nu, E_phase, E_min, penal, levels, n_pre, n_post, omega,
                   precision, n_cases, F_ptr, U_ptr):
    lib = load()
    m = len(E_phase)
    arr = (ctypes.c_double * m)(*[float(e) for e in E_phase])
    return check(ctx, lib.mtomg_set_grid(ctx, design, nelx, nely, nu, m, arr, E_min, penal, levels,
                                         n_pre, n_post, omega, precision, n_cases,
                                         ctypes.c_void_p(F_ptr), ctypes.c_void_p(U_ptr)))


def mtomg_workspace_bytes(ctx) -> int:
    return int(load().mtomg_workspace_bytes(ctx))


def mtomg_set_workspace(ctx, ptr: int, nbytes: int):
    return check(ctx, load().mtomg_set_workspace(ctx, ctypes.c_void_p(ptr), nbytes))


def mtomg_set_densities(ctx, design, x_ptr):
    return check(ctx, load().mtomg_set_densities(ctx, design, ctypes.c_void_p(x_ptr)))


def mtomg_solve(ctx, rel_tol, max_iter, warm_start, n_systems):
    stats = (mtomg_stats * n_systems)()
    for s in stats:
        s.status = 1   # not a status code: marks entries the call did not write
    st = load().mtomg_solve(ctx, rel_tol, max_iter, int(warm_start), stats)
    # per-system outcomes come back in stats; BAD_INPUT is one of them only
    # when some system reports it (invalid densities), else the call failed
    per_system = (MTOMG_NOT_CONVERGED, MTOMG_BREAKDOWN, MTOMG_NAN)
    if st == MTOMG_BAD_INPUT and any(s.status == MTOMG_BAD_INPUT for s in stats):
        per_system = per_system + (MTOMG_BAD_INPUT,)
    check(ctx, st, allow=per_system)
    return st, [s.as_dict() for s in stats]


def mtomg_compliance_and_grad(ctx, design, c_ptr, dcdx_ptr):
    return check(ctx, load().mtomg_compliance_and_grad(ctx, design, ctypes.c_void_p(c_ptr),
                                                       ctypes.c_void_p(dcdx_ptr or None)))


def mtomg_status_string(status: int) -> str:
    return load().mtomg_status_string(status).decode()


def mtomg_last_error(ctx) -> str:
    return load().mtomg_last_error(ctx).decode()


def mtomg_debug_apply(ctx, design, level, op, in_ptr, out_ptr):
    return check(ctx, load().mtomg_debug_apply(ctx, design, level, op, ctypes.c_void_p(in_ptr or None),
                                               ctypes.c_void_p(out_ptr)))


def mtomg_profile_kernel(ctx, kernel: str):
    return check(ctx, load().mtomg_profile_kernel(ctx, KERNELS[kernel]))


def mtomg_profile_read(ctx, cap: int = 4096):
    """Per-launch durations (ms) of the profiled kernel since the last read."""
    buf = (ctypes.c_double * cap)()
    n = ctypes.c_int(0)
    check(ctx, load().mtomg_profile_read(ctx, buf, cap, ctypes.byref(n)))
    return [buf[k] for k in range(min(n.value, cap))]


def mtomg_set_option(ctx, option: str, value: int):
    return check(ctx, load().mtomg_set_option(ctx, option_code(option), int(value)))


def mtomg_poisson_solve(ctx, n: int, n_pre: int, n_post: int, omega: float, rel_tol: float, max_iter: int,
                        f_ptr: int, u_ptr: int):
    """Returns (status, stats dict); NOT_CONVERGED, BREAKDOWN and NAN come back as a status."""
    st = mtomg_stats()
    status = load().mtomg_poisson_solve(ctx, n, n_pre, n_post, float(omega), float(rel_tol), max_iter,
                                        ctypes.c_void_p(f_ptr or None), ctypes.c_void_p(u_ptr or None),
                                        ctypes.byref(st))
    check(ctx, status, allow=(MTOMG_NOT_CONVERGED, MTOMG_BREAKDOWN, MTOMG_NAN))
    return status, st.as_dict()


def mtomg_filter(ctx, nelx: int, nely: int, m: int, rf: float, mode: str, gmin: float, x_ptr: int, in_ptr: int,
                 out_ptr: int):
    return check(ctx, load().mtomg_filter(ctx, nelx, nely, m, float(rf), FILTERS[mode], float(gmin),
                                          ctypes.c_void_p(x_ptr or None), ctypes.c_void_p(in_ptr or None),
                                          ctypes.c_void_p(out_ptr or None)))


def mtomg_filter_noalloc(stream: int, nelx: int, nely: int, m: int, rf: float, mode: str, gmin: float, x_ptr: int,
                         in_ptr: int, out_ptr: int):
    return check(None, load().mtomg_filter_noalloc(ctypes.c_void_p(stream or None), nelx, nely, m, float(rf),
                                                   FILTERS[mode], float(gmin), ctypes.c_void_p(x_ptr or None),
                                                   ctypes.c_void_p(in_ptr or None), ctypes.c_void_p(out_ptr or None)))


def mtomg_oc_update(ctx, nelx: int, nely: int, m: int, a: int, b: int, g_ptr: int, vol_a: float, move: float,
                    eta: float, eps: float, x_ptr: int, want_info: bool = True):
    """Returns info (lambda, largest change, sum - target, passes), or None
    without want_info (then the call is asynchronous)."""
    info = (ctypes.c_double * 4)() if want_info else None
    check(ctx, load().mtomg_oc_update(ctx, nelx, nely, m, a, b, ctypes.c_void_p(g_ptr), float(vol_a), float(move),
                                      float(eta), float(eps), ctypes.c_void_p(x_ptr), info))
    return tuple(info) if want_info else None


def mtomg_aap_step(ctx, design: int, vols, rf: float, move: float, eta: float, eps: float, gmin: float,
                   rel_tol: float, max_iter: int, x_ptr: int):
    """Returns (compliance before each pair, largest change, PCG iterations per pair)."""
    m = len(vols) - 1
    npairs = m * (m + 1) // 2
    v = (ctypes.c_double * (m + 1))(*[float(t) for t in vols])
    cp = (ctypes.c_double * npairs)()
    ch = ctypes.c_double(0.0)
    it = (ctypes.c_int * npairs)()
    check(ctx, load().mtomg_aap_step(ctx, design, v, float(rf), float(move), float(eta), float(eps), float(gmin),
                                     float(rel_tol), int(max_iter), ctypes.c_void_p(x_ptr), cp, ctypes.byref(ch), it))
    return list(cp), ch.value, list(it)


def mtomg_stream_probe(ctx, kind: str, a_ptr: int, b_ptr: int, c_ptr: int, n: int, reps: int = 20) -> float:
    """Device ms per pass of the READ / COPY / TRIAD streaming kernel over n doubles."""
    ms = ctypes.c_double(0.0)
    check(ctx, load().mtomg_stream_probe(ctx, PROBES[kind], ctypes.c_void_p(a_ptr), ctypes.c_void_p(b_ptr),
                                         ctypes.c_void_p(c_ptr or None), n, reps, ctypes.byref(ms)))
    return ms.value
