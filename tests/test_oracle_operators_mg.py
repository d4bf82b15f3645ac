"""Pins for the oracle's forward maps and its multigrid V-cycle.

* Blur: equals an explicit matrix built entry by entry from the definition,
  equals ``scipy.ndimage.correlate`` with the tensor-product kernel, and
  satisfies the adjoint identity (also for asymmetric taps).
* Dense: adjoint identity.
* Multigrid: the Galerkin coarse operator equals the face-weight construction
  written out cell by cell; the V-cycle formed as a dense matrix is symmetric
  positive definite; iterating x <- x + B (b - M x) converges to a sparse
  direct solve; the smoothers match their closed-form error polynomials.
"""

import itertools

import numpy as np
import pytest
import scipy.sparse.linalg as spla
from numpy.polynomial import chebyshev as C
from scipy import ndimage

from oracle import grid, multigrid, operators


def _brute_blur_matrix(w, shape):
    r = (len(w) - 1) // 2
    nz, ny, nx = shape
    n = nx * ny * nz
    A = np.zeros((n, n))
    for j in range(n):
        x, y, z = j % nx, (j // nx) % ny, j // (nx * ny)
        # tensor product: sum over (kx, ky, kz) inside the grid of w_kx w_ky w_kz
        rx = range(-r, r + 1) if nx > 1 else [0]
        ry = range(-r, r + 1) if ny > 1 else [0]
        rz = range(-r, r + 1) if nz > 1 else [0]
        for kx, ky, kz in itertools.product(rx, ry, rz):
            xx, yy, zz = x + kx, y + ky, z + kz
            if 0 <= xx < nx and 0 <= yy < ny and 0 <= zz < nz:
                c = ((w[kx + r] if nx > 1 else 1.0) * (w[ky + r] if ny > 1 else 1.0)
                     * (w[kz + r] if nz > 1 else 1.0))
                A[j, xx + nx * (yy + ny * zz)] += c
    return A


@pytest.mark.parametrize("shape,r", [((1, 12, 12), 4), ((10, 10, 10), 3), ((3, 5, 4), 6)])
def test_blur_equals_brute_force_matrix(shape, r, rng):
    w = rng.uniform(0.1, 1.0, size=2 * r + 1)
    op = operators.Blur(w, shape)
    A = _brute_blur_matrix(w, shape)
    x = rng.standard_normal(shape)
    np.testing.assert_allclose(op.apply(x).ravel(), A @ x.ravel(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(op.apply_T(x).ravel(), A.T @ x.ravel(), rtol=1e-12, atol=1e-12)


def test_blur_equals_ndimage_correlate(rng):
    shape, r = (9, 11, 13), 4
    w = rng.uniform(0.1, 1.0, size=2 * r + 1)
    kernel = w[:, None, None] * w[None, :, None] * w[None, None, :]
    x = rng.standard_normal(shape)
    ref = ndimage.correlate(x, kernel, mode="constant", cval=0.0)
    np.testing.assert_allclose(operators.Blur(w, shape).apply(x), ref, rtol=1e-12, atol=1e-12)


def test_blur_adjoint_identity(rng):
    shape = (6, 7, 8)
    w = rng.uniform(0.0, 1.0, size=7)          # asymmetric on purpose
    op = operators.Blur(w, shape)
    x, y = rng.standard_normal(shape), rng.standard_normal(shape)
    assert np.vdot(op.apply(x), y) == pytest.approx(np.vdot(x, op.apply_T(y)), rel=1e-12)


def test_dense_adjoint_identity(rng):
    shape = (3, 4, 5)
    A = rng.standard_normal((17, 60))
    op = operators.Dense(A, shape)
    x, y = rng.standard_normal(shape), rng.standard_normal(17)
    assert np.vdot(op.apply(x), y) == pytest.approx(np.vdot(x, op.apply_T(y)), rel=1e-12)


def _face_weight_coarse(Wf, shape, eps):
    """Coarse operator written out from the fine face weights (Wf[a][z,y,x], face j -> j+e_a)."""
    nz, ny, nx = shape
    cz = 2 if nz > 1 else 1
    d = 3 if nz > 1 else 2
    cs = (nz // cz, ny // 2, nx // 2)
    n = cs[0] * cs[1] * cs[2]
    A = np.zeros((n, n))
    idx = lambda z, y, x: x + cs[2] * (y + cs[1] * z)  # noqa: E731
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        for a, (dz, dy, dx) in enumerate([(0, 0, 1), (0, 1, 0), (1, 0, 0)]):
            zu, yu, xu = z + dz, y + dy, x + dx
            if not (zu < nz and yu < ny and xu < nx):
                continue
            I, J = idx(z // cz, y // 2, x // 2), idx(zu // cz, yu // 2, xu // 2)
            if I == J:
                continue
            wgt = Wf[a][z, y, x]
            A[I, I] += wgt
            A[J, J] += wgt
            A[I, J] -= wgt
            A[J, I] -= wgt
    A += (2 ** d) * eps * np.eye(n)
    return A


@pytest.mark.parametrize("shape", [(4, 8, 6), (1, 8, 10)])
def test_galerkin_equals_face_sums(shape, rng):
    kappa = rng.uniform(0.2, 2.0, size=shape)
    eps = 1e-2
    M = grid.prior_matrix(kappa, eps)
    h = multigrid.Hierarchy(M, shape, 2)
    nz, ny, nx = shape
    Wf = [kappa.copy(), kappa.copy(), kappa.copy()]
    Wf[0][:, :, -1] = 0.0
    Wf[1][:, -1, :] = 0.0
    Wf[2][-1, :, :] = 0.0
    ref = _face_weight_coarse(Wf, shape, eps)
    np.testing.assert_allclose(h.A[1].toarray(), ref, rtol=1e-13, atol=1e-13)


def _dense_vcycle(h, sm):
    n = h.A[0].shape[0]
    B = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        B[:, j] = multigrid.vcycle(h, e, sm)
    return B


@pytest.mark.parametrize("shape,levels,sm", [
    ((1, 8, 8), 3, multigrid.Smoother("jacobi", 2, 2, 0.8)),
    ((8, 8, 8), 3, multigrid.Smoother("jacobi", 2, 2, 0.8)),
    ((8, 8, 8), 2, multigrid.Smoother("chebyshev", 1, 1, degree=3, lo=1 / 3, hi=2.0)),
])
def test_vcycle_is_symmetric_positive_definite(shape, levels, sm, rng):
    kappa = np.exp(rng.uniform(-3, 3, size=shape))     # strongly varying diffusivity
    M = grid.prior_matrix(kappa, 1e-6)
    h = multigrid.Hierarchy(M, shape, levels)
    B = _dense_vcycle(h, sm)
    asym = np.abs(B - B.T).max() / np.abs(B).max()
    assert asym < 1e-12
    Bs = 0.5 * (B + B.T)
    assert np.linalg.eigvalsh(Bs).min() > 0.0


@pytest.mark.parametrize("sm", [multigrid.Smoother("jacobi", 2, 2, 0.8),
                                multigrid.Smoother("chebyshev", 1, 1, degree=3, lo=1 / 3, hi=2.0)])
def test_vcycle_iteration_converges_to_direct_solve(sm, rng):
    shape = (8, 16, 16)
    kappa = np.exp(rng.uniform(-2, 2, size=shape))
    M = grid.prior_matrix(kappa, 1e-3)
    h = multigrid.Hierarchy(M, shape, 3)
    b = rng.standard_normal(M.shape[0])
    ref = spla.spsolve(M.tocsc(), b)
    x = np.zeros_like(b)
    # piecewise-constant transfers give a modest factor (about 0.8 per cycle
    # with this strongly varying kappa), so iterate long enough to reach 1e-10.
    for _ in range(150):
        x = x + multigrid.vcycle(h, b - M @ x, sm)
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-10


def test_jacobi_closed_form(rng):
    # Two damped Jacobi sweeps from 0: x = (I - S^2) A^{-1} b with S = I - omega D^{-1} A.
    shape = (3, 4, 5)
    M = grid.prior_matrix(rng.uniform(0.5, 2.0, size=shape), 0.1).toarray()
    D = np.diag(M).copy()
    b = rng.standard_normal(M.shape[0])
    S = np.eye(len(b)) - 0.8 * M / D[:, None]
    ref = (np.eye(len(b)) - S @ S) @ np.linalg.solve(M, b)
    x = multigrid.jacobi(M, D, b, np.zeros_like(b), 2, 0.8)
    np.testing.assert_allclose(x, ref, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("degree", [1, 2, 3, 4])
def test_chebyshev_error_polynomial(degree, rng):
    # Error after the smoother: e = p(D^{-1} A) e0 with p(l) = T_m((theta - l)/delta) / T_m(theta/delta).
    shape = (3, 4, 5)
    A = grid.prior_matrix(rng.uniform(0.5, 2.0, size=shape), 0.1).toarray()
    D = np.diag(A).copy()
    lo, hi = 0.3, 2.0
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    b = rng.standard_normal(A.shape[0])
    x0 = rng.standard_normal(A.shape[0])
    xs = np.linalg.solve(A, b)
    x = multigrid.chebyshev(A, D, b, x0, degree, lo, hi)
    # evaluate p on the (similar-to-symmetric) matrix D^{-1} A through its eigen-decomposition
    Dh = np.sqrt(D)
    Sym = A / Dh[:, None] / Dh[None, :]
    lam, Q = np.linalg.eigh(Sym)
    coef = np.zeros(degree + 1)
    coef[-1] = 1.0
    p = C.chebval((theta - lam) / delta, coef) / C.chebval(theta / delta, coef)
    P = (Q * p) @ Q.T                              # p(D^{-1/2} A D^{-1/2})
    e_ref = (P @ (Dh * (x0 - xs))) / Dh            # p(D^{-1} A) = D^{-1/2} p(Sym) D^{1/2}
    np.testing.assert_allclose(x - xs, e_ref, rtol=1e-8, atol=1e-10)
