"""Pins for the oracle's adaptive stopping rules (Section 3.4, S4; Algorithm 3, step 5).

References used (none of them is the oracle's stopping code):
* S4 with the identity priorconditioner and tau = 0: SciPy's LSQR run for a fixed number of
  steps i = 1, 2, ..., the residual g - A x_i formed with the explicit matrix; the first i that
  meets ||g - A x_i|| <= eta * delta is the step S4 must stop at;
* S4 with damping and a V-cycle: the oracle's own fixed-count runs (pinned elsewhere against
  SciPy, PCG and dense solves), residuals formed with the explicit matrix -- the stopped run
  must equal the fixed-count run of the same length, meet the test there and fail it one step
  earlier (brute force over the step count);
* outer stop, closed form: for the Tikhonov regulariser the diffusivity is constant, so every
  outer iterate is the same vector and R never decreases: the loop stops exactly at k_min;
* outer stop, brute force: the penalties of a fixed-count run give the first k >= k_min at
  which R(f^k) - R(f^{k-1}) >= -rtol R(f^{k-1}); the adaptive run must stop there with the
  fixed-count iterate of that length.
"""

import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import gen
from oracle import lagged, multigrid, mlsqr


def _toeplitz_blur(n, sigma):
    """Explicit 1D Gaussian blur matrix (an ill-posed operator) built entry by entry."""
    A = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            A[i, j] = math.exp(-0.5 * ((i - j) / sigma) ** 2)
    return A / A.sum(axis=1, keepdims=True)


def _deconv_case(seed, n=80, sigma=2.5, noise=0.01):
    rng = np.random.default_rng(seed)
    A = _toeplitz_blur(n, sigma)
    x = np.zeros(n)
    x[n // 5:n // 2] = 1.0
    x[3 * n // 5:4 * n // 5] = 0.5
    e = rng.normal(0.0, noise, size=n)
    return A, A @ x + e, float(np.linalg.norm(e))


@pytest.mark.parametrize("seed,eta", [(0, 1.1), (1, 1.5), (2, 1.05)])
def test_s4_identity_prior_stops_where_lsqr_first_meets_the_discrepancy(seed, eta):
    A, g, delta = _deconv_case(seed)
    thr = eta * delta
    resid, xs = [], []
    for i in range(1, 61):
        x = spla.lsqr(A, g, damp=0.0, atol=0.0, btol=0.0, conlim=1e300, iter_lim=i)[0]
        xs.append(x)
        resid.append(float(np.linalg.norm(g - A @ x)))
    first = next(i for i, r in enumerate(resid, start=1) if r <= thr)
    # not a near tie, so that rounding cannot move the crossing
    assert resid[first - 1] < thr * (1 - 1e-6) and resid[first - 2] > thr * (1 + 1e-6)
    f, done = mlsqr.mlsqr(lambda v: A @ v, lambda u: A.T @ u, lambda p: p, g, 0.0, 60,
                          resid_stop=thr)
    assert done == first
    np.testing.assert_allclose(f, xs[first - 1], rtol=1e-8, atol=1e-10)


def test_s4_cap_and_unreachable_level():
    A, g, delta = _deconv_case(3)
    # a level below what LSQR reaches in 12 steps: the cap decides
    f, done = mlsqr.mlsqr(lambda v: A @ v, lambda u: A.T @ u, lambda p: p, g, 0.0, 12,
                          resid_stop=1e-3 * delta)
    f12, d12 = mlsqr.mlsqr(lambda v: A @ v, lambda u: A.T @ u, lambda p: p, g, 0.0, 12)
    assert done == d12 == 12
    assert np.array_equal(f, f12)
    # a level above ||g||: S4 holds after the first step
    _, done = mlsqr.mlsqr(lambda v: A @ v, lambda u: A.T @ u, lambda p: p, g, 0.0, 12,
                          resid_stop=2.0 * np.linalg.norm(g))
    assert done == 1


@pytest.mark.parametrize("tau", [0.0, 1e-3])
def test_s4_damped_vcycle_brute_force(tau):
    p = gen.small_blur_case(11, (12, 10, 1), reg="stv", T=0.05, tau=tau, outer=1, inner=30,
                            levels=2, noise_frac=0.02)
    shape = (1, 10, 12)
    op = lagged.make_operator("blur", shape, taps=p.taps)
    Adense = np.stack([op.apply(e.reshape(shape)).ravel() for e in np.eye(120)], axis=1)
    g = np.asarray(p.g, dtype=np.float64).reshape(shape)
    sm = multigrid.Smoother("jacobi", 2, 2, 0.8, 3, 1 / 3, 2.0)
    from oracle import grid, regularizers
    kappa = regularizers.diffusivity("stv", grid.grad_norm(np.zeros(shape)), 0.05)
    h = multigrid.Hierarchy(grid.prior_matrix(kappa, 1e-6), shape, 2)

    def Minv(v):
        return multigrid.vcycle(h, np.ravel(v), sm).reshape(shape)

    def run(iters, stop=None):
        return mlsqr.mlsqr(op.apply, op.apply_T, Minv, g, tau, iters, resid_stop=stop)

    def resid(f):
        return float(np.linalg.norm(g.ravel() - Adense @ np.ravel(f)))

    fixed = [resid(run(i)[0]) for i in range(1, 31)]
    # a level that the iteration crosses strictly inside the cap, away from a tie
    i_star = next(i for i in range(3, 30) if fixed[i - 1] < fixed[i - 2] * 0.999)
    thr = 0.5 * (fixed[i_star - 1] + fixed[i_star - 2])
    expect = next(i for i, r in enumerate(fixed, start=1) if r <= thr)
    f, done = run(30, thr)
    assert done == expect
    f_fixed, _ = run(done)
    assert np.array_equal(np.ravel(f), np.ravel(f_fixed))
    assert resid(f) <= thr < resid(run(done - 1)[0])


def _outer_case(reg, T=0.05, outer=6, inner=10, tau=5.0):
    return gen.small_blur_case(4, (16, 12, 1), reg=reg, T=T, tau=tau, outer=outer, inner=inner,
                               levels=3, noise_frac=0.01)


@pytest.mark.parametrize("k_min", [2, 3, 4])
def test_outer_stop_tikhonov_stops_at_first_check(k_min):
    p = _outer_case("tikhonov", T=1.0)
    f_fixed, rec_fixed = lagged.solve_problem(p, outer=1)
    p.stop_outer, p.outer_rtol, p.outer_min = True, 0.0, k_min
    f, rec = lagged.solve_problem(p)
    assert len(rec) == k_min
    assert np.array_equal(f, f_fixed)
    assert all(r["penalty"] == rec[0]["penalty"] for r in rec)


@pytest.mark.parametrize("reg,rtol,k_min", [("stv", 0.0, 3), ("stv", 0.02, 2), ("pm_log", 0.01, 3)])
def test_outer_stop_brute_force(reg, rtol, k_min):
    p = _outer_case(reg, outer=8)
    _, rec_fixed = lagged.solve_problem(p)
    R = [r["penalty"] for r in rec_fixed]
    expect = len(R)
    for k in range(k_min, len(R) + 1):
        change = R[k - 1] - R[k - 2]
        assert abs(change + rtol * R[k - 2]) > 1e-9 * R[k - 2]     # not a tie
        if change >= -rtol * R[k - 2]:
            expect = k
            break
    p.stop_outer, p.outer_rtol, p.outer_min = True, rtol, k_min
    f, rec = lagged.solve_problem(p)
    assert len(rec) == expect
    f_fixed, _ = lagged.solve_problem(p.__class__(**{**p.__dict__, "stop_outer": False}),
                                      outer=expect)
    assert np.array_equal(f, f_fixed)


def test_outer_stop_rejects_k_min_below_two():
    p = _outer_case("stv", outer=3)
    p.stop_outer, p.outer_rtol, p.outer_min = True, 0.0, 1
    with pytest.raises(ValueError):
        lagged.solve_problem(p)


def test_s4_and_outer_stop_together_record_inner_counts():
    # the regime of Section 5.3: the cap binds in the first outer step, S4 in later ones, and
    # the outer loop ends once R stops decreasing
    p = _outer_case("stv", T=0.01, outer=8, inner=20, tau=1e-3)
    p.stop_s4, p.eta = True, 1.1
    p.stop_outer, p.outer_rtol, p.outer_min = True, 0.0, 3
    f, rec = lagged.solve_problem(p)
    for r in rec:
        # each outer step either met the discrepancy level or used the whole cap
        assert r["inner_done"] == 20 or r["resid"] <= p.eta * p.delta
    assert rec[0]["inner_done"] == 20 and rec[0]["resid"] > p.eta * p.delta
    assert any(r["inner_done"] < 20 for r in rec)
    assert len(rec) < 8 and rec[-1]["penalty"] >= rec[-2]["penalty"]
