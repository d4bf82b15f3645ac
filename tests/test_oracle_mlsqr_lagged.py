"""Pins for the oracle's MLSQR (Algorithm 2 with damping) and the lagged-diffusivity loop.

References used (none of them is the oracle's own code path):
* SciPy's LSQR with ``damp`` (the priorconditioner set to the identity);
* LSQR on the standard-form problem A L^{-1} (Algorithm 1 with explicit L, run
  by SciPy), mapped back by L^{-1} -- this fixes the normalisation of p in the
  initialisation;
* a textbook preconditioned CG on (A^T A + tau M) f = A^T g with preconditioner M^{-1}
  (Section 3: the method is analytically PCG on the normal equations);
* dense solves of the normal equations and a dense least-squares solve of the
  stacked problem (1.8) with the explicit non-square factor;
* invariants: alpha and beta do not depend on tau (Section 3.1), phibar is
  non-increasing, and for tau = 0 it equals ||g - A f_i|| (Section 3.4).
"""

import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import gen
from oracle import grid, lagged, multigrid, mlsqr, regularizers
from oracle.operators import Blur, Dense


def _small_problem(rng, nY=30, shape=(1, 5, 6)):
    n = int(np.prod(shape))
    A = rng.standard_normal((nY, n)) / math.sqrt(n)
    g = rng.standard_normal(nY)
    return A, g, shape


def _lsqr_iterates(Ahat, g, damp, iters):
    out = []
    for i in range(1, iters + 1):
        x = spla.lsqr(Ahat, g, damp=damp, atol=0.0, btol=0.0, conlim=1e300, iter_lim=i)[0]
        out.append(x)
    return out


@pytest.mark.parametrize("tau", [0.0, 0.3, 5.0])
def test_identity_priorconditioner_is_damped_lsqr(tau, rng):
    A, g, shape = _small_problem(rng)
    ref = _lsqr_iterates(A, g, math.sqrt(tau), 8)
    for i in range(1, 9):
        f, done = mlsqr.mlsqr(lambda x: A @ x, lambda y: A.T @ y, lambda p: p, g, tau, i)
        assert done == i
        np.testing.assert_allclose(f, ref[i - 1], rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("tau", [0.0, 2.0])
def test_exact_priorconditioner_is_lsqr_on_standard_form(tau, rng):
    A, g, shape = _small_problem(rng, nY=45)
    kappa = rng.uniform(0.3, 3.0, size=shape)
    M = grid.prior_matrix(kappa, 0.05).toarray()
    L = np.linalg.cholesky(M).T                     # M = L^T L, L upper triangular
    Linv = np.linalg.inv(L)
    # Krylov iterates are ill-conditioned functions of the data (the difference
    # between two exact-arithmetic-equivalent runs grows ~50x per step here), so
    # compare the first six steps, where rounding stays below 1e-9.
    ref = _lsqr_iterates(A @ Linv, g, math.sqrt(tau), 6)
    for i in range(1, 7):
        f, _ = mlsqr.mlsqr(lambda x: A @ x, lambda y: A.T @ y,
                           lambda p: np.linalg.solve(M, p), g, tau, i)
        ref_f = Linv @ ref[i - 1]
        assert np.linalg.norm(f - ref_f) <= 1e-9 * np.linalg.norm(ref_f)


def _pcg_iterates(K, b, Minv, iters):
    x = np.zeros_like(b)
    r = b.copy()
    z = Minv(r)
    p = z.copy()
    rz = r @ z
    out = []
    for _ in range(iters):
        Kp = K @ p
        a = rz / (p @ Kp)
        x = x + a * p
        r = r - a * Kp
        z = Minv(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
        out.append(x.copy())
    return out


def test_mlsqr_is_pcg_on_normal_equations(rng):
    A, g, shape = _small_problem(rng)
    tau = 0.7
    M = grid.prior_matrix(rng.uniform(0.3, 3.0, size=shape), 0.05).toarray()
    K = A.T @ A + tau * M
    ref = _pcg_iterates(K, A.T @ g, lambda r: np.linalg.solve(M, r), 6)
    for i in range(1, 7):
        f, _ = mlsqr.mlsqr(lambda x: A @ x, lambda y: A.T @ y,
                           lambda p: np.linalg.solve(M, p), g, tau, i)
        np.testing.assert_allclose(f, ref[i - 1], rtol=1e-7, atol=1e-10)


def test_converged_mlsqr_solves_regularised_problem(rng):
    A, g, shape = _small_problem(rng)
    tau = 0.4
    kappa = rng.uniform(0.3, 3.0, size=shape)
    eps = 0.05
    M = grid.prior_matrix(kappa, eps)
    Md = M.toarray()
    n = Md.shape[0]
    f, _ = mlsqr.mlsqr(lambda x: A @ x, lambda y: A.T @ y, lambda p: np.linalg.solve(Md, p),
                       g, tau, 3 * n)
    ref = np.linalg.solve(A.T @ A + tau * Md, A.T @ g)
    np.testing.assert_allclose(f, ref, rtol=1e-8, atol=1e-10)
    # the same point from the stacked least-squares problem (1.8) with the explicit
    # non-square factor Lhat = [diag(sqrt(kappa)) G ; sqrt(eps) I], Lhat^T Lhat = M
    G = grid.gradient_matrix(shape).toarray()
    k = np.tile(kappa.ravel(), 3)
    Lhat = np.vstack([np.sqrt(k)[:, None] * G, math.sqrt(eps) * np.eye(n)])
    stacked = np.vstack([A, math.sqrt(tau) * Lhat])
    rhs = np.concatenate([g, np.zeros(Lhat.shape[0])])
    ls = np.linalg.lstsq(stacked, rhs, rcond=None)[0]
    np.testing.assert_allclose(f, ls, rtol=1e-8, atol=1e-10)


def test_converged_with_vcycle_priorconditioner(rng):
    # With a V-cycle B standing in for M^{-1}, the limit solves (A^T A + tau B^{-1}) f = A^T g.
    shape = (1, 8, 8)
    n = 64
    A = rng.standard_normal((50, n)) / 8.0
    g = rng.standard_normal(50)
    M = grid.prior_matrix(rng.uniform(0.3, 3.0, size=shape), 1e-2)
    h = multigrid.Hierarchy(M, shape, 2)
    sm = multigrid.Smoother("jacobi", 2, 2, 0.8)
    B = np.column_stack([multigrid.vcycle(h, e, sm) for e in np.eye(n)])
    tau = 0.5
    f, _ = mlsqr.mlsqr(lambda x: A @ x, lambda y: A.T @ y,
                       lambda p: multigrid.vcycle(h, p, sm), g, tau, 4 * n)
    ref = np.linalg.solve(A.T @ A + tau * np.linalg.inv(0.5 * (B + B.T)), A.T @ g)
    np.testing.assert_allclose(f, ref, rtol=1e-7, atol=1e-9)


def test_invariants(rng):
    A, g, shape = _small_problem(rng, nY=40, shape=(1, 6, 6))
    M = grid.prior_matrix(rng.uniform(0.3, 3.0, size=shape), 0.05).toarray()
    hs = {}
    for tau in (0.0, 50.0):
        hist = []
        mlsqr.mlsqr(lambda x: A @ x, lambda y: A.T @ y, lambda p: np.linalg.solve(M, p), g, tau,
                    12, hist)
        hs[tau] = hist
    # alpha, beta independent of tau (bitwise: the bidiagonalisation never sees tau)
    assert [h["alpha"] for h in hs[0.0]] == [h["alpha"] for h in hs[50.0]]
    assert [h["beta"] for h in hs[0.0]] == [h["beta"] for h in hs[50.0]]
    # |phibar| is non-increasing (its sign may alternate with the sign of rho_bar)
    for tau in (0.0, 50.0):
        pb = [abs(h["phibar"]) for h in hs[tau]]
        assert all(b <= a * (1 + 1e-12) for a, b in zip(pb, pb[1:]))
    # tau = 0: |phibar_{i+1}| = ||g - A f_i||
    for i in range(1, 10):
        f, _ = mlsqr.mlsqr(lambda x: A @ x, lambda y: A.T @ y,
                           lambda p: np.linalg.solve(M, p), g, 0.0, i)
        assert np.linalg.norm(g - A @ f) == pytest.approx(abs(hs[0.0][i]["phibar"]), rel=1e-9)


def test_zero_data_gives_zero(rng):
    A, g, shape = _small_problem(rng)
    f, done = mlsqr.mlsqr(lambda x: A @ x, lambda y: A.T @ y, lambda p: p, np.zeros_like(g),
                          1.0, 5)
    assert done == 0 and not np.any(f)


def test_not_spd_raises(rng):
    A, g, shape = _small_problem(rng)
    with pytest.raises(mlsqr.NotSPD):
        mlsqr.mlsqr(lambda x: A @ x, lambda y: A.T @ y, lambda p: -p, g, 1.0, 3)


def _tiny_blur_problem(reg, T, tau, outer, inner, levels, seed=3):
    p = gen.small_blur_case(seed, (8, 8, 1), sigma=1.0, radius=2, reg=reg, T=T, tau=tau,
                            outer=outer, inner=inner, levels=levels)
    return p


def test_tikhonov_outer_iterates_identical():
    p = _tiny_blur_problem("tikhonov", 1.0, 0.5, 3, 10, 2)
    hist = []
    shape = (1, 8, 8)
    op = Blur(p.taps, shape)
    sm = multigrid.Smoother("jacobi", 2, 2, 0.8)
    fs = []
    for K in (1, 2, 3):
        f, _ = lagged.solve(shape, op, p.g.astype(float), "tikhonov", 1.0, 0.5, 1e-6, K, 10, 2, sm, hist)
        fs.append(f)
    np.testing.assert_array_equal(fs[0], fs[1])
    np.testing.assert_array_equal(fs[0], fs[2])


def test_tikhonov_exact_prior_matches_normal_equations():
    shape = (1, 8, 8)
    p = _tiny_blur_problem("tikhonov", 1.0, 0.5, 1, 64 * 3, 1)
    op = Blur(p.taps, shape)
    sm = multigrid.Smoother("jacobi", 2, 2, 0.8)
    eps = 1e-2
    f, _ = lagged.solve(shape, op, p.g.astype(float), "tikhonov", 1.0, 0.5, eps, 1, 64 * 3, 1, sm)
    Ad = np.column_stack([op.apply(e.reshape(shape)).ravel() for e in np.eye(64)])
    G = grid.gradient_matrix(shape).toarray()
    K = Ad.T @ Ad + 0.5 * (G.T @ G + eps * np.eye(64))
    ref = np.linalg.solve(K, Ad.T @ p.g.astype(float).ravel())
    np.testing.assert_allclose(f.ravel(), ref, rtol=1e-7, atol=1e-9)


def test_first_outer_iterates_of_pm_equal_tikhonov():
    shape = (1, 8, 8)
    p = _tiny_blur_problem("tikhonov", 1.0, 0.5, 1, 12, 2)
    op = Blur(p.taps, shape)
    sm = multigrid.Smoother("jacobi", 2, 2, 0.8)
    g = p.g.astype(float)
    f_t, _ = lagged.solve(shape, op, g, "tikhonov", 1.0, 0.5, 1e-6, 1, 12, 2, sm)
    f_l, _ = lagged.solve(shape, op, g, "pm_log", 0.05, 0.5, 1e-6, 1, 12, 2, sm)
    f_e, _ = lagged.solve(shape, op, g, "pm_exp", 0.05, 0.5, 1e-6, 1, 12, 2, sm)
    np.testing.assert_array_equal(f_t, f_l)
    np.testing.assert_array_equal(f_t, f_e)


def test_first_outer_iterate_of_stv_is_scaled_laplacian():
    shape = (1, 8, 8)
    T, tau, eps = 0.1, 0.5, 1e-2
    p = _tiny_blur_problem("stv", T, tau, 1, 64 * 3, 1)
    op = Blur(p.taps, shape)
    sm = multigrid.Smoother("jacobi", 2, 2, 0.8)
    g = p.g.astype(float)
    f, _ = lagged.solve(shape, op, g, "stv", T, tau, eps, 1, 64 * 3, 1, sm)
    Ad = np.column_stack([op.apply(e.reshape(shape)).ravel() for e in np.eye(64)])
    G = grid.gradient_matrix(shape).toarray()
    K = Ad.T @ Ad + tau * ((1.0 / T) * G.T @ G + eps * np.eye(64))
    ref = np.linalg.solve(K, Ad.T @ g.ravel())
    np.testing.assert_allclose(f.ravel(), ref, rtol=1e-7, atol=1e-9)
    assert regularizers.diffusivity("stv", 0.0, T) == pytest.approx(1.0 / T)


def test_dense_operator_solve_runs_and_records():
    p = gen.small_dense_case(4, 8, outer=3, inner=6)
    f, rec = lagged.solve_problem(p)
    assert f.shape == (8, 8, 8)
    assert [r["inner_done"] for r in rec] == [6, 6, 6]
    A = p.A.astype(float)
    assert rec[-1]["resid"] == pytest.approx(np.linalg.norm(p.g - A @ f.ravel()), rel=1e-12)
    assert rec[-1]["penalty"] == pytest.approx(grid.penalty(f, p.reg, p.T), rel=1e-12)


def test_restart_residual_each_outer():
    # every outer iteration restarts MLSQR at f = 0: phibar_1 = ||g|| each time
    p = _tiny_blur_problem("pm_log", 0.05, 0.1, 3, 6, 2)
    hist = []
    lagged.solve_problem(p, history=hist)
    for inner in hist:
        assert inner[0]["phibar"] == pytest.approx(np.linalg.norm(p.g.astype(float)), rel=1e-14)


@pytest.mark.slow
def test_method_reduces_error_and_penalty_on_small_tv_problem():
    # qualitative claims of Sections 4.3/5.3: error vs the truth falls over the
    # outer iterations, and R(f^k) falls after the first iterate
    p = gen.small_blur_case(7, (32, 32, 1), sigma=1.5, radius=3, reg="stv", T=0.01, tau=0.002,
                            outer=6, inner=25, levels=3)
    errs = []
    for K in (1, 6):
        f, rec = lagged.solve_problem(p, outer=K)
        errs.append(np.linalg.norm(f - p.f_true) / np.linalg.norm(p.f_true))
    assert errs[1] < errs[0]
    assert rec[-1]["penalty"] < rec[1]["penalty"]


@pytest.mark.parametrize("reg,T,tau,outer", [("stv", 0.05, 0.2, 60), ("pm_log", 0.3, 0.1, 120)])
def test_lagged_diffusivity_fixed_point_is_stationary(reg, T, tau, outer):
    """Section 4.1: the outer loop is the lagged-diffusivity fixed-point iteration for the
    stationarity condition (4.1)/(4.2) of the MAP functional. With an exact prior solve (one
    multigrid level: the Cholesky solve of M) and converged inner solves, each outer step
    returns argmin ||g - A f||^2 + tau f^T M_{f^{k-1}} f, so a fixed point f* satisfies
    A^T (A f* - g) + tau (G^T diag(kappa(|grad f*|)) G + eps I) f* = 0, which is the gradient of
        J(f) = 1/2 ||g - A f||^2 + tau R(f) + 1/2 tau eps ||f||^2
    (dR/df = G^T diag(r'(t)/t) G f). The gradient is taken here by central differences of J
    (no diffusivity formula enters), so a kappa formed from the wrong iterate or the wrong
    formula leaves a non-zero gradient at the limit. The first iterate (kappa from f^0 = 0) is
    far from stationary, which shows the check has teeth."""
    p = gen.small_blur_case(3, (7, 6, 1), sigma=1.2, radius=2, reg=reg, T=T, tau=tau, levels=1,
                            eps=1e-3)
    shape = (1, 6, 7)
    op = Blur(p.taps, shape)
    g = p.g.astype(float).reshape(shape)
    sm = multigrid.Smoother("jacobi", 2, 2, 0.8)
    f, _ = lagged.solve(shape, op, g, reg, T, tau, p.eps, outer, 150, 1, sm)
    f_next, _ = lagged.solve(shape, op, g, reg, T, tau, p.eps, outer + 1, 150, 1, sm)
    assert np.linalg.norm(f_next - f) <= 1e-8 * np.linalg.norm(f)      # the iteration has settled

    def J(x):
        x = x.reshape(shape)
        return (0.5 * np.sum((g - op.apply(x)) ** 2) + tau * grid.penalty(x, reg, T)
                + 0.5 * tau * p.eps * np.sum(x * x))

    def grad_J(x, h=1e-6):
        x = x.ravel()
        out = np.zeros(x.size)
        for j in range(x.size):
            e = np.zeros(x.size)
            e[j] = h
            out[j] = (J(x + e) - J(x - e)) / (2.0 * h)
        return out

    scale = np.linalg.norm(op.apply_T(g))
    assert np.linalg.norm(grad_J(f_next)) <= 1e-7 * scale
    f1, _ = lagged.solve(shape, op, g, reg, T, tau, p.eps, 1, 150, 1, sm)
    assert np.linalg.norm(grad_J(f1)) >= 1e-3 * scale
