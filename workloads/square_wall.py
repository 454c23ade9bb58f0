"""Square-wall workloads: seeded phase-density fields and nodal load vectors.

Conventions shared by every consumer of these arrays:

* The wall is the rectangle [0, 1] x [0, nely/nelx], split into nelx x nely
  square elements of side h = 1/nelx, thickness 1.
* Element (i, j) has index j*nelx + i; phase densities are x[j, i, phase].
* Node (i, j), i = 0..nelx, j = 0..nely, has DOFs 2*(j*(nelx+1)+i) (x) and
  +1 (y); load vectors have shape [n_cases, nely+1, nelx+1, 2].
* The bottom edge (j = 0) is clamped; the loads below put their force on the
  other edges.

The paper's own square-wall designs (its optimised topologies) and
optimiser are not available, so these fields stand in for them with the
grid sizes, phase counts and modulus contrast of its square-wall example
(Section 5.2, Table 2); every draw comes from numpy's PCG64 generator with
a fixed seed.
"""

from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np
import scipy.ndimage

# Physics shared by the workloads (plane stress, Poisson ratio 0.3, SIMP
# penalty 3, three solid phases plus a soft void).
PHYSICS = dict(nu=0.3, penal=3.0, E_min=1e-9, E_phase=(1.0, 0.6, 0.2))


@dataclasses.dataclass
class Problem:
    """One design: grid, phase densities, material data, loads, solver setup."""

    name: str
    nelx: int
    nely: int
    x: np.ndarray              # [nely, nelx, m] float64 phase densities
    E_phase: np.ndarray        # [m] float64 solid-phase moduli
    E_min: float
    penal: float
    nu: float
    F: np.ndarray              # [n_cases, nely+1, nelx+1, 2] float64 loads
    levels: int
    n_pre: int = 2
    n_post: int = 2
    omega: float = 0.6
    rel_tol: float = 1e-8
    mixed: bool = False        # FP32 V-cycle inside FP64 CG when True
    fd_elements: Optional[np.ndarray] = None   # [k, 2] (element, phase) for FD checks
    fd_zero_pairs: Optional[np.ndarray] = None  # [k, 2] pairs whose gradient is ~0
    seed: int = 0

    @property
    def m(self) -> int:
        return self.x.shape[2]

    @property
    def n_dof(self) -> int:
        return 2 * (self.nelx + 1) * (self.nely + 1)

    @property
    def n_cases(self) -> int:
        return self.F.shape[0]


# ----------------------------------------------------------------------------
# density fields
# ----------------------------------------------------------------------------

def cone_filter(field: np.ndarray, radius: float) -> np.ndarray:
    """Weighted neighbourhood mean with weights max(0, radius - distance).

    The window is truncated at the domain boundary and the weights are
    renormalised over the part that lies inside.
    """
    rr = int(np.ceil(radius)) - 1
    off = np.arange(-rr, rr + 1)
    dy, dx = np.meshgrid(off, off, indexing="ij")
    w = np.maximum(0.0, radius - np.sqrt(dx * dx + dy * dy))
    num = scipy.ndimage.convolve(field, w, mode="constant", cval=0.0)
    den = scipy.ndimage.convolve(np.ones_like(field), w, mode="constant", cval=0.0)
    return num / den


def density_random_cone(n: int, seed: int, rng: Optional[np.random.Generator] = None,
                        m: int = 3, radius: float = 2.0) -> np.ndarray:
    """Uniform noise on m+1 channels, cone-filtered, normalised to sum 1.

    The first m channels are the solid phases; the last is the void share.
    """
    rng = np.random.default_rng(seed) if rng is None else rng
    w = rng.random((m + 1, n, n))
    w = np.stack([cone_filter(w[c], radius) for c in range(m + 1)])
    w /= w.sum(axis=0, keepdims=True)
    return np.ascontiguousarray(np.moveaxis(w[:m], 0, -1))


def density_binary_contrast(n: int, seed: int, m: int = 3):
    """One-hot solid or void per element, with probability 1/2 each.

    The solid phase of an element is the argmax of the cone-filtered field;
    the top (loaded) and bottom (clamped) element rows are always solid so
    the load path never hangs on the void modulus.  Returns (x, solid_mask,
    rng) so callers can keep drawing from the same stream.
    """
    rng = np.random.default_rng(seed)
    base = density_random_cone(n, seed, rng=rng, m=m)
    d = np.argmax(base, axis=2)
    b = rng.random((n, n))
    solid = b < 0.5
    solid[0, :] = True
    solid[-1, :] = True
    x = np.zeros((n, n, m))
    jj, ii = np.nonzero(solid)
    x[jj, ii, d[jj, ii]] = 1.0
    return x, solid, d, rng


def density_gaussian_sum(nelx: int, nely: int, seed: int, m: int = 3,
                         n_gauss: int = 32) -> np.ndarray:
    """Sum of n_gauss seeded Gaussians per phase, clipped and normalised.

    For each phase the centres, widths and amplitudes are drawn in that
    order; the field is clipped to [1e-3, 1] and divided by max(1, sum over
    phases) so the solid share of every element is at most 1.
    """
    rng = np.random.default_rng(seed)
    h = 1.0 / nelx
    xc = (np.arange(nelx) + 0.5) * h
    yc = (np.arange(nely) + 0.5) * h
    g = np.zeros((m, nely, nelx))
    for ph in range(m):
        cen = rng.random((n_gauss, 2))
        sig = rng.uniform(0.03, 0.15, n_gauss)
        amp = rng.uniform(0.5, 1.0, n_gauss)
        for k in range(n_gauss):
            gx = np.exp(-((xc - cen[k, 0]) ** 2) / (2 * sig[k] ** 2))
            gy = np.exp(-((yc - cen[k, 1]) ** 2) / (2 * sig[k] ** 2))
            g[ph] += amp[k] * gy[:, None] * gx[None, :]
    g = np.clip(g, 1e-3, 1.0)
    g /= np.maximum(1.0, g.sum(axis=0, keepdims=True))
    return np.ascontiguousarray(np.moveaxis(g, 0, -1))


def density_near_binary(n: int, seed: int, m: int = 4, quantile: float = 0.30):
    """Thresholded smooth noise: near-binary multi-phase layout.

    Each phase gets Gaussian-smoothed noise (sigma = n/128); the phase of an
    element is the argmax, and the element is solid iff that maximum reaches
    the given quantile.  Top and bottom rows are solid.  Solid elements take
    1 - 3e-3 on their phase and 1e-3 on the others; void elements take 1e-3
    everywhere.  If the solid set does not connect the top and bottom edges
    the seed is moved by 100 (returned so the caller can record it).
    """
    for s in (seed, seed + 100, seed + 200):
        rng = np.random.default_rng(s)
        sm = np.stack([scipy.ndimage.gaussian_filter(rng.random((n, n)), sigma=n / 128.0,
                                                     mode="reflect") for _ in range(m)])
        d = np.argmax(sm, axis=0)
        mx = np.max(sm, axis=0)
        solid = mx >= np.quantile(mx, quantile)
        solid[0, :] = True
        solid[-1, :] = True
        lab, _ = scipy.ndimage.label(solid)
        if np.intersect1d(lab[0][lab[0] > 0], lab[-1][lab[-1] > 0]).size:
            break
    x = np.full((n, n, m), 1e-3)
    jj, ii = np.nonzero(solid)
    x[jj, ii, d[jj, ii]] = 1.0 - 3e-3
    return x, s


# ----------------------------------------------------------------------------
# loads (consistent nodal forces, total magnitude 1)
# ----------------------------------------------------------------------------

def load_top_traction(nelx: int, nely: int) -> np.ndarray:
    """Uniform downward traction on the top edge, total force 1."""
    F = np.zeros((nely + 1, nelx + 1, 2))
    h = 1.0 / nelx
    F[nely, :, 1] = -h
    F[nely, 0, 1] = -h / 2
    F[nely, nelx, 1] = -h / 2
    return F


def load_point(nelx: int, nely: int, i: int, j: int) -> np.ndarray:
    """Downward unit point load at node (i, j)."""
    F = np.zeros((nely + 1, nelx + 1, 2))
    F[j, i, 1] = -1.0
    return F


def load_left_traction(nelx: int, nely: int) -> np.ndarray:
    """Uniform downward (shear) traction on the left edge, total force 1."""
    F = np.zeros((nely + 1, nelx + 1, 2))
    F[:, 0, 1] = -1.0 / nely
    F[0, 0, 1] = -0.5 / nely
    F[nely, 0, 1] = -0.5 / nely
    return F


def four_load_cases(nelx: int, nely: int) -> np.ndarray:
    """Top traction, top-right point load, left-edge shear, top-mid point load."""
    return np.stack([
        load_top_traction(nelx, nely),
        load_point(nelx, nely, nelx, nely),
        load_left_traction(nelx, nely),
        load_point(nelx, nely, nelx // 2, nely),
    ])


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

def _phys(**kw):
    p = dict(PHYSICS)
    p.update(kw)
    return p


def make_problem(name: str, n: Optional[int] = None, levels: Optional[int] = None,
                 mixed: Optional[bool] = None) -> Problem:
    """Build one named square-wall workload.

    Names: "wall64" (random cone field, 3 levels), "wall256" (binary 1e9
    contrast, 5 levels), "wall1024" (smooth Gaussian field, 7 levels, FP32
    V-cycle), "wall2048" (near-binary 4-phase, 8 levels, FP32 V-cycle).  The
    optional n / levels / mixed arguments rescale a recipe, e.g. for small
    parity cases.
    """
    if name == "wall64":
        n = n or 64
        x = density_random_cone(n, 0)
        ph = _phys()
        prob = Problem(name, n, n, x, np.array(ph["E_phase"]), ph["E_min"], ph["penal"], ph["nu"],
                       load_top_traction(n, n)[None], levels or 3, mixed=bool(mixed), seed=0)
    elif name == "wall256":
        n = n or 256
        x, solid, d, rng = density_binary_contrast(n, 1)
        flat = np.flatnonzero(solid.ravel())
        k = min(64, flat.size)
        el = rng.choice(flat, k, replace=False)
        fd = np.stack([el, d.ravel()[el]], axis=1)
        z = rng.choice(flat, 8, replace=False)
        zp = np.stack([z, (d.ravel()[z] + 1) % 3], axis=1)
        ph = _phys()
        prob = Problem(name, n, n, x, np.array(ph["E_phase"]), ph["E_min"], ph["penal"], ph["nu"],
                       load_top_traction(n, n)[None], levels or 5, mixed=bool(mixed),
                       fd_elements=fd, fd_zero_pairs=zp, seed=1)
    elif name == "wall1024":
        n = n or 1024
        x = density_gaussian_sum(n, n, 2)
        ph = _phys()
        prob = Problem(name, n, n, x, np.array(ph["E_phase"]), ph["E_min"], ph["penal"], ph["nu"],
                       load_top_traction(n, n)[None], levels or 7,
                       mixed=True if mixed is None else mixed, seed=2)
    elif name == "wall2048":
        n = n or 2048
        x, s = density_near_binary(n, 3)
        ph = _phys(E_phase=(1.0, 0.7, 0.4, 0.1))
        prob = Problem(name, n, n, x, np.array(ph["E_phase"]), ph["E_min"], ph["penal"], ph["nu"],
                       load_top_traction(n, n)[None], levels or 8,
                       mixed=True if mixed is None else mixed, seed=s)
    else:
        raise ValueError(f"unknown workload {name!r}")
    return prob


def batched_design(d: int, sizes: Sequence[int] = (128, 384, 768), per_size: int = 16,
                   levels: Sequence[int] = (4, 5, 6)) -> Problem:
    """Design d of ``batched_designs`` (same sizes and per_size), built alone."""
    if not 0 <= d < per_size * len(sizes):
        raise IndexError(f"design {d} out of range")
    n, lv = sizes[d // per_size], levels[d // per_size]
    x = density_gaussian_sum(n, n, 1000 + d)
    ph = _phys()
    return Problem(f"batch{d}", n, n, x, np.array(ph["E_phase"]), ph["E_min"], ph["penal"], ph["nu"],
                   four_load_cases(n, n), lv, mixed=True, seed=1000 + d)


def batched_designs(sizes: Sequence[int] = (128, 384, 768), per_size: int = 16,
                    levels: Sequence[int] = (4, 5, 6)) -> List[Problem]:
    """Many independent smooth 3-phase designs, four load cases each."""
    return [batched_design(d, sizes, per_size, levels) for d in range(per_size * len(sizes))]
