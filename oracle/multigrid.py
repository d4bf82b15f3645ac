"""Geometric multigrid V-cycle: a fixed, symmetric positive definite approximation of M^{-1}.

Section 4.2 asks for a preconditioner solve that is a *fixed* symmetric
operator (same smoother and number of steps before and after the coarse-grid
correction, fixed grid transfers), so that it can priorcondition MLSQR. The
paper uses algebraic multigrid on its FEM mesh; on a structured grid the
reading here is:

* cell-centred 2:1 coarsening of every axis of extent > 1 (x, y, and z for 3D);
* piecewise-constant prolongation P (a coarse value is copied to its 2^d
  children), restriction P^T, and Galerkin coarse operators A_{l+1} = P^T A_l P;
* zero initial guess on every level; nu_pre pre-smoothing steps, the residual
  restricted, the correction solved recursively and prolongated, nu_post
  post-smoothing steps;
* smoothers: damped Jacobi x <- x + omega D^{-1} (b - A x), or a Chebyshev
  polynomial of degree m in D^{-1} A on [lo, hi] (three-term recurrence of the
  Chebyshev acceleration method), the same polynomial before and after;
* the coarsest level is solved exactly with a dense FP64 Cholesky factor.
"""

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def _interp1d(n, coarsen):
    if not coarsen:
        return sp.identity(n, format="csr")
    if n % 2:
        raise ValueError(f"cannot coarsen an axis of odd length {n}")
    rows = np.arange(n)
    return sp.csr_matrix((np.ones(n), (rows, rows // 2)), shape=(n, n // 2))


def prolongation(shape):
    """Sparse P mapping a coarse grid to ``shape`` = (nz, ny, nx) by piecewise-constant copy."""
    nz, ny, nx = shape
    return sp.kron(_interp1d(nz, nz > 1), sp.kron(_interp1d(ny, ny > 1), _interp1d(nx, nx > 1))).tocsr()


def coarse_shape(shape):
    nz, ny, nx = shape
    return (nz // 2 if nz > 1 else 1, ny // 2 if ny > 1 else 1, nx // 2 if nx > 1 else 1)


class Hierarchy:
    """Galerkin hierarchy A_0 = M, A_{l+1} = P_l^T A_l P_l, with a Cholesky factor of the last."""

    def __init__(self, M, shape, levels):
        if levels < 1:
            raise ValueError("need at least one level")
        self.shapes = [tuple(shape)]
        self.A = [sp.csr_matrix(M)]
        self.P = []
        for _ in range(levels - 1):
            P = prolongation(self.shapes[-1])
            self.P.append(P)
            self.A.append((P.T @ self.A[-1] @ P).tocsr())
            self.shapes.append(coarse_shape(self.shapes[-1]))
        self.D = [np.asarray(A.diagonal()) for A in self.A]
        self.coarse_dense = self.A[-1].toarray()
        self.chol = sla.cho_factor(self.coarse_dense, lower=True)

    @property
    def levels(self):
        return len(self.A)


def jacobi(A, D, b, x, steps, omega):
    for _ in range(steps):
        x = x + omega * (b - A @ x) / D
    return x


def chebyshev(A, D, b, x, degree, lo, hi):
    """Degree-``degree`` Chebyshev polynomial smoother in D^{-1} A on [lo, hi]."""
    theta = 0.5 * (hi + lo)
    delta = 0.5 * (hi - lo)
    sigma = theta / delta
    r = b - A @ x
    rho = 1.0 / sigma
    d = (r / D) / theta
    for _ in range(degree):
        x = x + d
        r = r - A @ d
        rho_next = 1.0 / (2.0 * sigma - rho)
        d = rho_next * rho * d + (2.0 * rho_next / delta) * (r / D)
        rho = rho_next
    return x


class Smoother:
    def __init__(self, kind="jacobi", nu_pre=2, nu_post=2, omega=0.8, degree=3, lo=1.0 / 3.0,
                 hi=2.0):
        if kind not in ("jacobi", "chebyshev"):
            raise ValueError(kind)
        self.kind, self.nu_pre, self.nu_post = kind, nu_pre, nu_post
        self.omega, self.degree, self.lo, self.hi = omega, degree, lo, hi

    def __call__(self, A, D, b, x, steps):
        if self.kind == "jacobi":
            return jacobi(A, D, b, x, steps, self.omega)
        for _ in range(steps):
            x = chebyshev(A, D, b, x, self.degree, self.lo, self.hi)
        return x


def vcycle(h, b, smoother, level=0):
    """One V-cycle for A_level x = b from x = 0."""
    if level == h.levels - 1:
        return sla.cho_solve(h.chol, b)
    A, D = h.A[level], h.D[level]
    x = smoother(A, D, b, np.zeros_like(b), smoother.nu_pre)
    r = b - A @ x
    e = vcycle(h, h.P[level].T @ r, smoother, level + 1)
    x = x + h.P[level] @ e
    return smoother(A, D, b, x, smoother.nu_post)
