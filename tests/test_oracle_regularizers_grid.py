"""Pins for the oracle's diffusivities, penalty, gradient and prior matrix.

Nothing here compares the oracle with itself: the checks are closed forms,
difference quotients, hand-computed sums and brute-force loops written from the
definitions (forward differences with a zero at the upper boundary).
"""

import itertools

import numpy as np
import pytest

from oracle import grid, regularizers

KINDS = regularizers.KINDS


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("T", [0.01, 0.05, 1.0])
def test_kappa_is_difference_quotient_of_r(kind, T):
    # kappa(t) = r'(t) / t, eq. (1.12)-(1.13): compare with a central difference of r.
    for t in [1e-3, 0.03, 0.2, 1.5]:
        h = 1e-3 * t
        rp = (regularizers.penalty_density(kind, t + h, T)
              - regularizers.penalty_density(kind, t - h, T)) / (2 * h)
        k = regularizers.diffusivity(kind, t, T)
        assert abs(rp / t - k) <= 1e-5 * max(1.0, abs(k)), (kind, T, t, rp / t, k)


def test_kappa_limits_at_zero():
    T = 0.07
    assert regularizers.diffusivity("tikhonov", 0.0, T) == 1.0
    assert regularizers.diffusivity("stv", 0.0, T) == pytest.approx(1.0 / T, rel=1e-15)
    assert regularizers.diffusivity("pm_log", 0.0, T) == 1.0
    assert regularizers.diffusivity("pm_exp", 0.0, T) == 1.0


def test_penalty_values_hand_computed():
    # r(t) at points where the closed forms reduce to simple numbers.
    T = 0.5
    assert regularizers.penalty_density("tikhonov", 3.0, T) == 4.5
    assert regularizers.penalty_density("stv", 0.0, T) == pytest.approx(T)
    assert regularizers.penalty_density("stv", T, T) == pytest.approx(T * np.sqrt(2.0))
    assert regularizers.penalty_density("pm_log", T, T) == pytest.approx(0.5 * T * T * np.log(2.0))
    assert regularizers.penalty_density("pm_exp", T, T) == pytest.approx(0.5 * T * T * (1 - np.exp(-1)))


def _brute_grad(f):
    nz, ny, nx = f.shape
    q = np.zeros((3,) + f.shape)
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        if x + 1 < nx:
            q[0, z, y, x] = f[z, y, x + 1] - f[z, y, x]
        if y + 1 < ny:
            q[1, z, y, x] = f[z, y + 1, x] - f[z, y, x]
        if z + 1 < nz:
            q[2, z, y, x] = f[z + 1, y, x] - f[z, y, x]
    return q


@pytest.mark.parametrize("shape", [(3, 4, 5), (1, 6, 7), (2, 1, 3)])
def test_gradient_matches_brute_force(shape, rng):
    f = rng.standard_normal(shape)
    np.testing.assert_array_equal(grid.grad(f), _brute_grad(f))


def test_gradient_adjoint_identity(rng):
    shape = (4, 5, 6)
    x = rng.standard_normal(shape)
    q = rng.standard_normal((3,) + shape)
    lhs = np.vdot(grid.grad(x), q)
    rhs = np.vdot(x, grid.grad_T(q))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_penalty_linear_ramp():
    # f = a x: |grad f| = a except on the last x-layer, where the Neumann
    # difference is 0, so R = (nx-1) ny nz r(a) + ny nz r(0).
    nz, ny, nx, a = 3, 4, 6, 0.3
    f = a * np.broadcast_to(np.arange(nx, dtype=float), (nz, ny, nx)).copy()
    for kind, T in [("tikhonov", 1.0), ("stv", 0.1), ("pm_log", 0.2), ("pm_exp", 0.2)]:
        expect = ((nx - 1) * ny * nz * regularizers.penalty_density(kind, a, T)
                  + ny * nz * regularizers.penalty_density(kind, 0.0, T))
        assert grid.penalty(f, kind, T) == pytest.approx(float(expect), rel=1e-13)


@pytest.mark.parametrize("kind", KINDS)
def test_gradient_of_penalty_is_prior_operator(kind, rng):
    # d R / d f = G^T diag(kappa(t)) G f = (M - eps I) f, checked by central differences of R.
    shape, T, eps = (3, 4, 5), 0.4, 1e-3
    f = rng.standard_normal(shape)
    kappa = regularizers.diffusivity(kind, grid.grad_norm(f), T)
    Mf = grid.prior_matrix(kappa, eps) @ f.ravel() - eps * f.ravel()
    h = 1e-6
    num = np.empty(f.size)
    for j in range(f.size):
        e = np.zeros(f.size)
        e[j] = h
        num[j] = (grid.penalty(f + e.reshape(shape), kind, T)
                  - grid.penalty(f - e.reshape(shape), kind, T)) / (2 * h)
    np.testing.assert_allclose(num, Mf, rtol=1e-5, atol=1e-7)


def _brute_M(kappa, eps, x):
    # (M x)_j = eps x_j + sum_a [k_j (x_j - x_{j+e_a}) 1(j+e_a in) + k_{j-e_a} (x_j - x_{j-e_a}) 1(j-e_a in)]
    nz, ny, nx = x.shape
    y = eps * x.copy()
    for z, yy, xx in itertools.product(range(nz), range(ny), range(nx)):
        for dz, dy, dx in [(0, 0, 1), (0, 1, 0), (1, 0, 0)]:
            zu, yu, xu = z + dz, yy + dy, xx + dx
            if zu < nz and yu < ny and xu < nx:
                y[z, yy, xx] += kappa[z, yy, xx] * (x[z, yy, xx] - x[zu, yu, xu])
            zl, yl, xl = z - dz, yy - dy, xx - dx
            if zl >= 0 and yl >= 0 and xl >= 0:
                y[z, yy, xx] += kappa[zl, yl, xl] * (x[z, yy, xx] - x[zl, yl, xl])
    return y


@pytest.mark.parametrize("shape", [(3, 4, 5), (1, 5, 6)])
def test_prior_matrix_properties(shape, rng):
    kappa = rng.uniform(0.1, 3.0, size=shape)
    eps = 1e-3
    M = grid.prior_matrix(kappa, eps)
    x = rng.standard_normal(shape)
    np.testing.assert_allclose(M @ x.ravel(), _brute_M(kappa, eps, x).ravel(), rtol=1e-13, atol=1e-13)
    Md = M.toarray()
    np.testing.assert_array_equal(Md, Md.T)
    np.testing.assert_allclose(M @ np.ones(M.shape[0]), eps * np.ones(M.shape[0]), atol=1e-13)
    assert np.linalg.eigvalsh(Md).min() > 0.0
