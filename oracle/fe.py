"""Finite-element model of the multi-material plane-stress wall (Section 3).

Everything here is FP64 and written as the plain definition:

* the multi-phase SIMP modulus of Eq. (5), read with an implicit void phase
  E = E_min + sum_i x_i^p (E_i - E_min) (the form whose derivative is
  p x_i^(p-1) (E_i - E_min));
* the element stiffness K^e = integral of B^T D B (Eq. 7) with the
  plane-stress D (Eq. 8) and the bilinear strain-displacement B (Eq. 9),
  integrated by 2x2 Gauss quadrature, which is exact for these polynomial
  products;
* assembly of K = sum_e E_e A_e^T K^0 A_e, the clamped bottom edge of the
  wall (Eq. 10, u = 0 on Gamma_u), compliance C = F^T U = U^T K U (Eq. 6)
  and its element-wise gradient (the sensitivity step of Section 4).

Grid conventions: element (i, j) is j*nelx + i with nodes (i,j), (i+1,j),
(i+1,j+1), (i,j+1) counter-clockwise; node (i, j) owns DOFs 2*(j*(nelx+1)+i)
and +1; nodes with j = 0 are clamped.  Parity unpinned: none — every
function below is checked by a test against closed forms or invariants.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def constitutive_matrix(nu: float) -> np.ndarray:
    """Plane-stress material matrix of Eq. (8) for unit modulus."""
    return np.array([[1.0, nu, 0.0],
                     [nu, 1.0, 0.0],
                     [0.0, 0.0, (1.0 - nu) / 2.0]]) / (1.0 - nu * nu)


def shape_gradients(xi: float, eta: float):
    """Derivatives of the four bilinear shape functions on the unit square.

    Local nodes: 0 (0,0), 1 (1,0), 2 (1,1), 3 (0,1).  Returns (dN/dxi,
    dN/deta), each of length 4.
    """
    dxi = np.array([-(1.0 - eta), (1.0 - eta), eta, -eta])
    deta = np.array([-(1.0 - xi), -xi, xi, (1.0 - xi)])
    return dxi, deta


def strain_displacement(xi: float, eta: float, h: float = 1.0) -> np.ndarray:
    """The 3x8 matrix B of Eq. (9) at a local point of a square element of side h."""
    dxi, deta = shape_gradients(xi, eta)
    B = np.zeros((3, 8))
    B[0, 0::2] = dxi / h
    B[1, 1::2] = deta / h
    B[2, 0::2] = deta / h
    B[2, 1::2] = dxi / h
    return B


def element_stiffness(nu: float, h: float = 1.0) -> np.ndarray:
    """Unit-modulus element stiffness K^0 = integral over the element of B^T D B (Eq. 7).

    Thickness 1, square element of side h (the 2D result does not depend on
    h).  2x2 Gauss points integrate the quadratic integrand exactly.
    """
    D = constitutive_matrix(nu)
    g = (0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0))
    K = np.zeros((8, 8))
    for xi in g:
        for eta in g:
            B = strain_displacement(xi, eta, h)
            K += 0.25 * (h * h) * (B.T @ D @ B)
    return K


def interpolate_modulus(x: np.ndarray, E_phase, E_min: float, penal: float) -> np.ndarray:
    """Element modulus from phase densities, Eq. (5) with an implicit void phase.

    x has shape [..., m]; returns E_min + sum_i x_i^p (E_i - E_min).
    """
    E_phase = np.asarray(E_phase, dtype=np.float64)
    return E_min + np.sum(np.power(x, penal) * (E_phase - E_min), axis=-1)


def element_dof_map(nelx: int, nely: int) -> np.ndarray:
    """[nelx*nely, 8] global DOF indices of each element, local order of K^0."""
    j, i = np.meshgrid(np.arange(nely, dtype=np.int32), np.arange(nelx, dtype=np.int32),
                       indexing="ij")
    n0 = (j * (nelx + 1) + i).ravel()
    n1 = n0 + 1
    n2 = n0 + (nelx + 1) + 1
    n3 = n0 + (nelx + 1)
    nodes = np.stack([n0, n1, n2, n3], axis=1)
    dofs = np.empty((nodes.shape[0], 8), dtype=np.int32)
    dofs[:, 0::2] = 2 * nodes
    dofs[:, 1::2] = 2 * nodes + 1
    return dofs


def assemble_stiffness(nelx: int, nely: int, E: np.ndarray, nu: float) -> sp.csr_matrix:
    """Global (unconstrained) stiffness K = sum_e E_e A_e^T K^0 A_e as CSR."""
    KE = element_stiffness(nu)
    dofs = element_dof_map(nelx, nely)
    Ef = np.asarray(E, dtype=np.result_type(E, np.float64)).reshape(-1)
    rows = np.repeat(dofs, 8, axis=1).ravel()
    cols = np.tile(dofs, (1, 8)).ravel()
    vals = (Ef[:, None] * KE.ravel()[None, :]).ravel()
    n = 2 * (nelx + 1) * (nely + 1)
    K = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    K.sum_duplicates()
    return K


def free_dofs(nelx: int, nely: int) -> np.ndarray:
    """DOFs not on the clamped bottom edge (Eq. 10, u = 0 on Gamma_u)."""
    return np.arange(2 * (nelx + 1), 2 * (nelx + 1) * (nely + 1))


def restrict_to_free(K: sp.spmatrix, free: np.ndarray) -> sp.csr_matrix:
    """K_ff: rows and columns of the free DOFs."""
    return K.tocsr()[free][:, free].tocsr()


def compliance(F: np.ndarray, U: np.ndarray) -> float:
    """C = F^T U, which equals U^T K U at equilibrium (Eq. 6)."""
    return float(np.dot(np.ravel(F), np.ravel(U)))


def element_energies(U: np.ndarray, nelx: int, nely: int, nu: float) -> np.ndarray:
    """u_e^T K^0 u_e per element, shape [nely, nelx]."""
    KE = element_stiffness(nu)
    ue = np.ravel(U)[element_dof_map(nelx, nely)]
    return np.einsum("ea,ab,eb->e", ue, KE, ue).reshape(nely, nelx)


def compliance_gradient(x: np.ndarray, U: np.ndarray, E_phase, E_min: float, penal: float,
                        nu: float) -> np.ndarray:
    """dC/dx_{e,i} = -p x_{e,i}^(p-1) (E_i - E_min) u_e^T K^0 u_e.

    Compliance is self-adjoint (the adjoint state is -U), so the derivative
    of C = F^T U with K(x) U = F is -U^T (dK/dx) U element by element.
    """
    nely, nelx, _ = x.shape
    w = element_energies(U, nelx, nely, nu)
    dE = penal * np.power(x, penal - 1.0) * (np.asarray(E_phase) - E_min)
    return -dE * w[:, :, None]


def rigid_body_modes(nelx: int, nely: int, h: float) -> np.ndarray:
    """The three in-plane rigid motions sampled at the nodes, [3, n_dof]."""
    j, i = np.meshgrid(np.arange(nely + 1), np.arange(nelx + 1), indexing="ij")
    X = (i * h).ravel()
    Y = (j * h).ravel()
    n = X.size
    R = np.zeros((3, 2 * n))
    R[0, 0::2] = 1.0
    R[1, 1::2] = 1.0
    R[2, 0::2] = -Y
    R[2, 1::2] = X
    return R
