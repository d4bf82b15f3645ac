"""Pins for the oracle's multi-tau solve (Section 3.3: one bidiagonalisation, the projected
problem (3.6) solved for each damping).

References (none of them is the multi-tau code path):
* SciPy's LSQR with damp = sqrt(tau), identity priorconditioner, for several step counts;
* the oracle's recurrence form mlsqr() (Givens rotations with the damping rotation, pinned
  elsewhere) run separately for each tau, with a V-cycle priorconditioner;
* with as many steps as unknowns and an exact prior, the dense normal equations
  (A^T A + tau M) f = A^T g.
"""

import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import gen
from oracle import grid, lagged, mlsqr, multigrid, regularizers


@pytest.mark.parametrize("iters", [1, 3, 8])
def test_identity_prior_equals_damped_lsqr_for_every_tau(rng, iters):
    A = rng.standard_normal((30, 24)) / 5.0
    g = rng.standard_normal(30)
    taus = [0.0, 0.3, 5.0]
    fs, k = mlsqr.mlsqr_taus(lambda x: A @ x, lambda y: A.T @ y, lambda p: p, g, taus, iters)
    assert k == iters
    for tau, f in zip(taus, fs):
        ref = spla.lsqr(A, g, damp=math.sqrt(tau), atol=0.0, btol=0.0, conlim=1e300,
                        iter_lim=iters)[0]
        np.testing.assert_allclose(f, ref, rtol=1e-9, atol=1e-12)


def test_vcycle_prior_equals_separate_recurrence_runs():
    p = gen.small_blur_case(5, (12, 10, 4), reg="stv", T=0.05, tau=1.0, outer=1, inner=7,
                            levels=2)
    shape = (4, 10, 12)
    op = lagged.make_operator("blur", shape, taps=p.taps)
    g = np.asarray(p.g, dtype=np.float64).reshape(shape)
    kappa = regularizers.diffusivity("stv", grid.grad_norm(np.zeros(shape)), 0.05)
    h = multigrid.Hierarchy(grid.prior_matrix(kappa, 1e-3), shape, 2)
    sm = multigrid.Smoother("jacobi", 2, 2, 0.8, 3, 1 / 3, 2.0)

    def Minv(v):
        return multigrid.vcycle(h, np.ravel(v), sm).reshape(shape)

    taus = [0.0, 0.5, 4.0, 100.0]
    fs, k = mlsqr.mlsqr_taus(op.apply, op.apply_T, Minv, g, taus, 7)
    assert k == 7
    for tau, f in zip(taus, fs):
        ref, done = mlsqr.mlsqr(op.apply, op.apply_T, Minv, g, tau, 7)
        assert done == 7
        assert np.linalg.norm(np.ravel(f) - np.ravel(ref)) <= 1e-9 * np.linalg.norm(ref)


def test_converged_iterates_solve_the_normal_equations(rng):
    shape = (1, 3, 4)
    n = 12
    A = rng.standard_normal((16, n))
    g = rng.standard_normal(16)
    kappa = rng.uniform(0.5, 2.0, size=shape)
    M = grid.prior_matrix(kappa, 0.1).toarray()
    taus = [0.05, 1.0, 20.0]
    fs, _ = mlsqr.mlsqr_taus(lambda x: A @ np.ravel(x), lambda y: A.T @ y,
                             lambda q: np.linalg.solve(M, np.ravel(q)), g, taus, 3 * n)
    for tau, f in zip(taus, fs):
        ref = np.linalg.solve(A.T @ A + tau * M, A.T @ g)
        np.testing.assert_allclose(np.ravel(f), ref, rtol=1e-6, atol=1e-9)


def test_zero_data_gives_zero_for_every_tau():
    A = np.eye(4)
    fs, k = mlsqr.mlsqr_taus(lambda x: A @ x, lambda y: A.T @ y, lambda p: p, np.zeros(4),
                             [0.0, 1.0], 5)
    assert k == 0 and all(np.all(f == 0.0) for f in fs)


def test_lagged_multi_tau_last_step_equals_separate_runs():
    """Outer steps 1..K-1 at the problem's tau, then the last step for several taus: each
    result equals Algorithm 3 run with tau for the first K-1 steps and tau_t in the last."""
    p = gen.small_blur_case(9, (12, 8, 1), reg="pm_log", T=0.05, tau=2.0, outer=3, inner=6,
                            levels=2)
    shape = (1, 8, 12)
    op = lagged.make_operator("blur", shape, taps=p.taps)
    sm = multigrid.Smoother("jacobi", 2, 2, 0.8, 3, 1 / 3, 2.0)
    g = np.asarray(p.g, dtype=np.float64).reshape(shape)
    taus = [0.5, 2.0, 30.0]
    fs, done = lagged.solve_taus(shape, op, g, p.reg, p.T, p.tau, p.eps, 3, 6, 2, sm, taus)
    assert done == 6
    f2, _ = lagged.solve(shape, op, g, p.reg, p.T, p.tau, p.eps, 2, 6, 2, sm)
    kappa = regularizers.diffusivity(p.reg, grid.grad_norm(f2), p.T)
    h = multigrid.Hierarchy(grid.prior_matrix(kappa, p.eps), shape, 2)
    for tau, f in zip(taus, fs):
        ref, _ = mlsqr.mlsqr(op.apply, op.apply_T,
                             lambda q: multigrid.vcycle(h, np.ravel(q), sm).reshape(shape),
                             g, tau, 6)
        assert np.linalg.norm(f - ref) <= 1e-9 * np.linalg.norm(ref)
    f_same, _ = lagged.solve(shape, op, g, p.reg, p.T, p.tau, p.eps, 3, 6, 2, sm)
    assert np.linalg.norm(fs[1] - f_same) <= 1e-9 * np.linalg.norm(f_same)
