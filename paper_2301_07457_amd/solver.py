"""Torch-facing wrapper of the pCGMG library: device memory and stream only.

``PCGMGSolver`` owns the torch tensors the C ABI works on (loads F,
displacements U, the workspace) and forwards every call to libmtomg.so on
the current torch stream.  ``ComplianceFn`` is the differentiable compliance
c(x) of Eq. (6): forward = set_densities + solve + compliance_and_grad,
backward = the adjoint gradient computed by the library (compliance is
self-adjoint, so no second solve is needed).
"""

from __future__ import annotations

from typing import Dict, List, Optional, Sequence

import torch

from . import _lib

PRECISION = {"fp64": _lib.MTOMG_FP64, "fp32mg": _lib.MTOMG_FP32MG}


def _stream_ptr(device) -> int:
    return int(torch.cuda.current_stream(device).cuda_stream)


class PCGMGSolver:
    """One or more square-wall designs solved by the HIP pCGMG library.

    Parameters mirror ``mtomg_set_grid``.  ``F`` is a CUDA float64 tensor
    [n_cases, nely+1, nelx+1, 2].  Several designs are added with
    ``add_design``; the constructor describes design 0.
    """

    def __init__(self, max_designs: int = 1, device="cuda:0"):
        if not torch.cuda.is_available():
            raise RuntimeError("PCGMGSolver needs a ROCm GPU (no CPU fallback)")
        self.device = torch.device(device)
        with torch.cuda.device(self.device):
            self.ctx = _lib.mtomg_create(max_designs, _stream_ptr(self.device))
        self.designs: Dict[int, dict] = {}
        self.workspace: Optional[torch.Tensor] = None

    def __del__(self):
        try:
            if getattr(self, "ctx", None) is not None:
                _lib.mtomg_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    # ------------------------------------------------------------------
    def add_design(self, design: int, nelx: int, nely: int, F: torch.Tensor, E_phase: Sequence[float],
                   E_min: float = 1e-9, penal: float = 3.0, nu: float = 0.3, levels: int = 3,
                   n_pre: int = 2, n_post: int = 2, omega: float = 0.6, precision: str = "fp64"):
        F = F.to(self.device, torch.float64).contiguous()
        if F.dim() == 3:
            F = F.unsqueeze(0)
        if tuple(F.shape[1:]) != (nely + 1, nelx + 1, 2):
            raise ValueError(f"F must be [n_cases, {nely + 1}, {nelx + 1}, 2], got {tuple(F.shape)}")
        U = torch.zeros_like(F)
        _lib.mtomg_set_grid(self.ctx, design, nelx, nely, nu, list(E_phase), E_min, penal, levels,
                            n_pre, n_post, omega, PRECISION[precision], F.shape[0], F.data_ptr(),
                            U.data_ptr())
        self.designs[design] = dict(nelx=nelx, nely=nely, F=F, U=U, m=len(E_phase), x=None,
                                    precision=precision, levels=levels)
        self.workspace = None
        return self

    def set_option(self, name: str, value: int):
        """mtomg_set_option; re-plans the workspace when the launch geometry changes."""
        _lib.mtomg_set_option(self.ctx, name, value)
        if name.startswith("ROWS"):
            self.workspace = None
            self._ensure_workspace()

    def _ensure_workspace(self):
        if self.workspace is None:
            nb = _lib.mtomg_workspace_bytes(self.ctx)
            self.workspace = torch.empty(nb, dtype=torch.uint8, device=self.device)
            _lib.mtomg_set_workspace(self.ctx, self.workspace.data_ptr(), nb)
            # set_workspace drops densities of every design: reload them
            for d, info in self.designs.items():
                if info["x"] is not None:
                    _lib.mtomg_set_densities(self.ctx, d, info["x"].data_ptr())

    AUTOTUNE_CANDIDATES = ((0, 0), (2, 1), (4, 1), (4, 2), (8, 1), (8, 2))
    AUTOTUNE_CG_ROWS = (4, 8)
    AUTOTUNE_LEVEL_ROWS = (1, 2, 4)

    def _time_solve(self, rel_tol, max_iter, repeats):
        self.solve(rel_tol, max_iter)
        return min(self.solve(rel_tol, max_iter)[0]["t_solve_ms"] for _ in range(repeats))

    def autotune(self, rel_tol: float = 1e-8, max_iter: int = 1000, candidates=None, repeats: int = 2,
                 per_kernel: bool = True):
        """Tile autotuner: time the solve of the designs as they are now for
        each (ROWS_FINE, ROWS_COARSE) pair of rows per wave (0 = the
        library's own choice) and keep the fastest; then, with per_kernel,
        the rows of the outer-CG apply (ROWS_CG) and, one grid at a time,
        the rows of the two grids below the finest (ROWS_LEVEL1, ROWS_LEVEL2),
        keeping each choice only if it is faster.  Returns (best pair,
        {setting: ms}); every kept setting is in self.tuned.  Densities must
        be set; they are reloaded for every candidate (the launch geometry
        changes the workspace), and each time is the best of `repeats`
        solves after one warm-up solve."""
        if any(info["x"] is None for info in self.designs.values()):
            raise ValueError("autotune needs densities for every design")
        for name in ("ROWS_CG", "ROWS_LEVEL1", "ROWS_LEVEL2"):
            self.set_option(name, 0)
        timings = {}
        for rf, rc in (candidates or self.AUTOTUNE_CANDIDATES):
            self.set_option("ROWS_FINE", rf)
            self.set_option("ROWS_COARSE", rc)
            timings[(rf, rc)] = self._time_solve(rel_tol, max_iter, repeats)
        best = min(timings, key=timings.get)
        self.set_option("ROWS_FINE", best[0])
        self.set_option("ROWS_COARSE", best[1])
        self.tuned = {"ROWS_FINE": best[0], "ROWS_COARSE": best[1], "ROWS_CG": 0, "ROWS_LEVEL1": 0,
                      "ROWS_LEVEL2": 0}
        if per_kernel:
            best_ms = timings[best]
            for name, values in (("ROWS_CG", self.AUTOTUNE_CG_ROWS), ("ROWS_LEVEL1", self.AUTOTUNE_LEVEL_ROWS),
                                 ("ROWS_LEVEL2", self.AUTOTUNE_LEVEL_ROWS)):
                keep = 0
                for v in values:
                    self.set_option(name, v)
                    ms = self._time_solve(rel_tol, max_iter, repeats)
                    timings[f"{name}={v}"] = ms
                    if ms < best_ms:
                        best_ms, keep = ms, v
                self.set_option(name, keep)
                self.tuned[name] = keep
        return best, timings

    def set_densities(self, design: int, x: torch.Tensor):
        info = self.designs[design]
        x = x.to(self.device, torch.float64).contiguous()
        if tuple(x.shape) != (info["nely"], info["nelx"], info["m"]):
            raise ValueError("x must be [nely, nelx, m]")
        info["x"] = x
        self._ensure_workspace()
        _lib.mtomg_set_densities(self.ctx, design, x.data_ptr())

    def solve(self, rel_tol: float = 1e-8, max_iter: int = 1000, warm_start: bool = False) -> List[dict]:
        n = sum(info["F"].shape[0] for info in self.designs.values() if info["x"] is not None)
        _, stats = _lib.mtomg_solve(self.ctx, rel_tol, max_iter, warm_start, n)
        return stats

    def compliance_and_grad(self, design: int, grad: bool = True):
        info = self.designs[design]
        c = torch.empty(info["F"].shape[0], dtype=torch.float64, device=self.device)
        dc = None
        if grad:
            dc = torch.empty((info["F"].shape[0], info["nely"], info["nelx"], info["m"]),
                             dtype=torch.float64, device=self.device)
        _lib.mtomg_compliance_and_grad(self.ctx, design, c.data_ptr(), dc.data_ptr() if dc is not None else 0)
        return c, dc

    def filter(self, field: torch.Tensor, rf: float, mode: str = "DENSITY", x: Optional[torch.Tensor] = None,
               gmin: float = 1e-3) -> torch.Tensor:
        """mtomg_filter: the cone filter of one element field [nely][nelx][m]
        (or a stack [k][nely][nelx][m], filtered slice by slice) on the device.
        mode: "DENSITY", "DENSITY_ADJOINT" or "SENSITIVITY" (needs x, the
        densities [nely][nelx][m])."""
        f = field.to(self.device, torch.float64).contiguous()
        xs = x.to(self.device, torch.float64).contiguous() if x is not None else None
        out = torch.empty_like(f)
        ny, nx, m = f.shape[-3:]
        for a, o in zip(f.reshape(-1, ny, nx, m), out.view(-1, ny, nx, m)):
            _lib.mtomg_filter(self.ctx, nx, ny, m, rf, mode, gmin, xs.data_ptr() if xs is not None else 0,
                              a.data_ptr(), o.data_ptr())
        return out

    def oc_update(self, x: torch.Tensor, g: torch.Tensor, a: int, b: int, vol_a: float, move: float = 0.2,
                  eta: float = 0.5, eps: float = 1e-3, info: bool = True):
        """mtomg_oc_update: one binary OC sub-problem on phases a < b (b = m:
        the void) of the densities x [nely][nelx][m] (CUDA float64, updated
        in place) with the filtered gradient g.  Returns (lambda, largest
        change, volume sum - target, passes), or None with info=False (then
        nothing synchronises)."""
        ny, nx, m = x.shape
        if not (x.is_cuda and x.dtype == torch.float64 and x.is_contiguous()):
            raise ValueError("x must be a contiguous CUDA float64 tensor (updated in place)")
        gd = g.to(self.device, torch.float64).contiguous()
        return _lib.mtomg_oc_update(self.ctx, nx, ny, m, a, b, gd.data_ptr(), vol_a, move, eta, eps, x.data_ptr(),
                                    info)

    def aap_step(self, design: int, x: torch.Tensor, vols, rf: float = 8.0, move: float = 0.2, eta: float = 0.5,
                 eps: float = 1e-3, gmin: float = 1e-3, rel_tol: float = 1e-8, max_iter: int = 1000):
        """mtomg_aap_step: one outer iteration of the alternating active-phase
        loop on `design` (every pair: solve, gradient, sensitivity filter,
        OC update).  x [nely][nelx][m] is updated in place and stays the
        design's densities.  Returns (compliance before each pair, largest
        change, PCG iterations per pair)."""
        info = self.designs[design]
        if not (x.is_cuda and x.dtype == torch.float64 and x.is_contiguous()):
            raise ValueError("x must be a contiguous CUDA float64 tensor (updated in place)")
        if tuple(x.shape) != (info["nely"], info["nelx"], info["m"]):
            raise ValueError("x must be [nely, nelx, m]")
        info["x"] = x
        self._ensure_workspace()
        return _lib.mtomg_aap_step(self.ctx, design, list(vols), rf, move, eta, eps, gmin, rel_tol, max_iter,
                                   x.data_ptr())

    def optimize(self, design: int, x: torch.Tensor, vols, tol: float = 1e-3, max_outer: int = 100, **kw):
        """Outer iterations of aap_step until the largest density change is
        at most tol (Table 2) or max_outer; returns the per-iteration
        (compliance list, change) history."""
        hist = []
        for _ in range(max_outer):
            cs, ch, _ = self.aap_step(design, x, vols, **kw)
            hist.append((cs, ch))
            if ch <= tol:
                break
        return hist

    def poisson_solve(self, f: torch.Tensor, rel_tol: float = 1e-8, max_iter: int = 1000, n_pre: int = 2,
                      n_post: int = 2, omega: float = 0.6):
        """mtomg_poisson_solve: the Poisson model problem of Section 5.1 on an
        n x n grid (n a power of two).  f: nodal loads [n+1][n+1].  Returns
        (u [n+1][n+1], stats dict); needs no design."""
        fd = f.to(self.device, torch.float64).contiguous()
        n = fd.shape[0] - 1
        if tuple(fd.shape) != (n + 1, n + 1):
            raise ValueError("f must be [n+1, n+1]")
        u = torch.empty_like(fd)
        _, st = _lib.mtomg_poisson_solve(self.ctx, n, n_pre, n_post, omega, rel_tol, max_iter, fd.data_ptr(),
                                         u.data_ptr())
        return u, st

    def U(self, design: int = 0) -> torch.Tensor:
        return self.designs[design]["U"]

    def debug_apply(self, design: int, level: int, op: str, inp: Optional[torch.Tensor],
                    out_shape, dtype) -> torch.Tensor:
        out = torch.empty(out_shape, dtype=dtype, device=self.device)
        ptr = inp.contiguous().data_ptr() if inp is not None else 0
        _lib.mtomg_debug_apply(self.ctx, design, level, _lib.OPS[op], ptr, out.data_ptr())
        return out


class ComplianceFn(torch.autograd.Function):
    """c_k(x) for every load case of one design; gradient from the adjoint kernel."""

    @staticmethod
    def forward(ctx, x: torch.Tensor, solver: PCGMGSolver, design: int = 0, rel_tol: float = 1e-8,
                max_iter: int = 1000):
        solver.set_densities(design, x.detach())
        stats = solver.solve(rel_tol, max_iter)
        bad = [s for s in stats if s["status"] != 0]
        if bad:
            raise _lib.MtomgError(bad[0]["status"], f"solve failed: {bad[0]}")
        c, dc = solver.compliance_and_grad(design, grad=True)
        ctx.save_for_backward(dc)
        ctx.stats = stats
        return c

    @staticmethod
    def backward(ctx, grad_c: torch.Tensor):
        (dc,) = ctx.saved_tensors
        g = torch.einsum("k,kjim->jim", grad_c.to(dc.dtype), dc)
        return g, None, None, None, None
