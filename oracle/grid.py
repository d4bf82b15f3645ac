"""Discrete gradient, penalty R(f) and the prior matrix M_f on a voxel grid.

The paper discretises (1.12) with P1 finite elements on an unstructured mesh
(Section 5.2). On the structured grids used here (arrays of shape (nz, ny, nx),
x fastest, voxel size h = 1) the reading is:

* gradient G: forward differences, (G f)_{j,a} = f_{j+e_a} - f_j when j+e_a is
  inside the grid and 0 otherwise (the natural, Neumann, condition of the weak
  form (1.12)); a grid with nz = 1 is 2D and its z-differences vanish;
* |grad f|_j = sqrt(sum_a (G f)_{j,a}^2) per voxel;
* R(f) = sum_j r(|grad f|_j), the discretisation of (1.2);
* M_f = G^T diag(kappa (x) 1_d) G + eps I, the discretisation of the diffusion
  operator (1.13) with c_f = kappa(|grad f|) evaluated per voxel, shifted by
  eps so that it is SPD (the constant vector is otherwise in its null space).

All operators are built as explicit scipy sparse matrices so that each one is
its definition.
"""

import numpy as np
import scipy.sparse as sp

from . import regularizers


def _diff1d(n):
    """n x n forward difference with a zero last row."""
    if n == 1:
        return sp.csr_matrix((1, 1))
    main = -np.ones(n)
    main[-1] = 0.0
    return sp.diags([main, np.ones(n - 1)], [0, 1], shape=(n, n), format="csr")


def gradient_matrix(shape):
    """Sparse G of shape (3 n, n) for a grid of array shape (nz, ny, nx)."""
    nz, ny, nx = shape
    Ix, Iy, Iz = sp.identity(nx), sp.identity(ny), sp.identity(nz)
    gx = sp.kron(Iz, sp.kron(Iy, _diff1d(nx)))
    gy = sp.kron(Iz, sp.kron(_diff1d(ny), Ix))
    gz = sp.kron(_diff1d(nz), sp.kron(Iy, Ix))
    return sp.vstack([gx, gy, gz]).tocsr()


def grad(f):
    """(3, nz, ny, nx) forward differences of f (x, y, z components)."""
    f = np.asarray(f, dtype=np.float64)
    q = gradient_matrix(f.shape) @ f.ravel()
    return q.reshape((3,) + f.shape)


def grad_T(q):
    """Adjoint of grad: maps (3, nz, ny, nx) to (nz, ny, nx)."""
    q = np.asarray(q, dtype=np.float64)
    shape = q.shape[1:]
    return (gradient_matrix(shape).T @ q.ravel()).reshape(shape)


def grad_norm(f):
    q = grad(f)
    return np.sqrt(q[0] ** 2 + q[1] ** 2 + q[2] ** 2)


def penalty(f, kind, T):
    """R(f) = sum over voxels of r(|grad f|)."""
    return float(np.sum(regularizers.penalty_density(kind, grad_norm(f), T)))


def prior_matrix(kappa, eps):
    """Sparse M = G^T diag(kappa, kappa, kappa) G + eps I for per-voxel diffusivity kappa."""
    kappa = np.asarray(kappa, dtype=np.float64)
    G = gradient_matrix(kappa.shape)
    k = kappa.ravel()
    D = sp.diags(np.concatenate([k, k, k]))
    n = k.size
    return (G.T @ D @ G + eps * sp.identity(n)).tocsr()
