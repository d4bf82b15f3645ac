"""Algorithm 3: the priorconditioned lagged-diffusivity solver (Section 4.1).

Outer iteration k (k = 1..K, starting from f^0 = 0):
  1. form M_{f^{k-1}} from the current iterate: kappa = r'(t)/t at t = |grad f^{k-1}|
     (eq. (1.12)-(1.13)), once per outer iteration, fixed during the inner solve;
  2. solve the damped priorconditioned problem (4.3) with MLSQR (Algorithm 2),
     restarted from f = 0 (Section 4.3 notes every outer step restarts the residual at ||g||),
     with the V-cycle standing in for M^{-1};
  3. record ||g - A f^k|| and R(f^k) (the quantities the paper monitors for the
     discrepancy principle S4 and the outer stopping rule).

By default the counts are fixed (K outer x m inner). The paper's adaptive stops are
optional:
  * inner: the discrepancy principle S4 (Section 3.4), ||g - A f_i|| <= eta * delta,
    with m as the global cap on MLSQR steps per outer step (Section 4.1);
  * outer: step 5 of Algorithm 3, break once R(f^k) does not decrease fast enough. The
    reading used: stop after outer step k >= k_min when
        R(f^k) - R(f^{k-1}) >= -rtol * R(f^{k-1}),
    i.e. the relative decrease is at most rtol (Section 4.3 uses a 15% threshold, Section
    5.3 stops once R stops decreasing: rtol = 0, where an unchanged R also stops). The first comparison is made at
    k_min >= 2 (k_min = 3 by default: Section 5.3 observes that the first damped iterate
    is flattened, so R(f^1) is not on the trend). The iterate returned is f^k, the last
    one computed.
"""

import numpy as np

from . import grid, multigrid, mlsqr, regularizers
from .operators import Blur, Dense


def make_operator(op_kind, shape, taps=None, A=None):
    if op_kind == "blur":
        return Blur(taps, shape)
    if op_kind == "dense":
        return Dense(A, shape)
    raise ValueError(op_kind)


def solve(shape, op, g, reg, T, tau, eps, outer, inner, levels, smoother, history=None,
          s4=None, outer_stop=None):
    """Return the last iterate f^k (array of ``shape``) and a per-outer record list.

    ``shape`` is (nz, ny, nx); ``op`` has ``apply``/``apply_T``; ``smoother`` is a
    ``multigrid.Smoother``. ``s4`` = (eta, delta) turns on the S4 inner stop;
    ``outer_stop`` = (rtol, k_min) turns on the penalty-based outer stop.
    """
    g = np.asarray(g, dtype=np.float64)
    resid_stop = None if s4 is None else float(s4[0]) * float(s4[1])
    if outer_stop is not None and int(outer_stop[1]) < 2:
        raise ValueError("the outer stop compares R(f^k) with R(f^{k-1}) for k >= 2")
    f = np.zeros(shape)
    records = []
    for k in range(1, outer + 1):
        kappa = regularizers.diffusivity(reg, grid.grad_norm(f), T)
        M = grid.prior_matrix(kappa, eps)
        h = multigrid.Hierarchy(M, shape, levels)

        def apply_Minv(p, h=h):
            return multigrid.vcycle(h, np.asarray(p).ravel(), smoother).reshape(shape)

        inner_hist = [] if history is not None else None
        f, done = mlsqr.mlsqr(op.apply, op.apply_T, apply_Minv, g, tau, inner, inner_hist,
                              resid_stop=resid_stop)
        f = np.asarray(f).reshape(shape)
        resid = float(np.linalg.norm(g.ravel() - np.asarray(op.apply(f)).ravel()))
        records.append(dict(k=k, inner_done=done, resid=resid, penalty=grid.penalty(f, reg, T)))
        if history is not None:
            history.append(inner_hist)
        if outer_stop is not None and k >= int(outer_stop[1]):
            r_now, r_prev = records[-1]["penalty"], records[-2]["penalty"]
            if r_now - r_prev >= -float(outer_stop[0]) * r_prev:
                break
    return f, records


def solve_taus(shape, op, g, reg, T, tau, eps, outer, inner, levels, smoother, taus):
    """Algorithm 3 with the damping tau for outer steps 1..K-1, then the last outer step's
    MLSQR solve for every damping in ``taus`` from one bidiagonalisation (Section 3.3):
    returns the list of f^K(tau_t) and the iterations completed in the last step."""
    g = np.asarray(g, dtype=np.float64)
    f = np.zeros(shape)
    if outer > 1:
        f, _ = solve(shape, op, g, reg, T, tau, eps, outer - 1, inner, levels, smoother)
    kappa = regularizers.diffusivity(reg, grid.grad_norm(f), T)
    h = multigrid.Hierarchy(grid.prior_matrix(kappa, eps), shape, levels)

    def apply_Minv(p):
        return multigrid.vcycle(h, np.asarray(p).ravel(), smoother).reshape(shape)

    fs, done = mlsqr.mlsqr_taus(op.apply, op.apply_T, apply_Minv, g, taus, inner)
    return [np.asarray(x).reshape(shape) for x in fs], done


def solve_problem(prob, history=None, outer=None, inner=None):
    """Convenience wrapper taking a ``gen.Problem``-like object (fields only, no behaviour)."""
    nx, ny, nz = prob.dims
    shape = (nz, ny, nx)
    op = make_operator(prob.op_kind, shape, taps=prob.taps, A=prob.A)
    sm = multigrid.Smoother(prob.smoother, prob.nu_pre, prob.nu_post, prob.omega,
                            prob.cheb_degree, prob.cheb_lo, prob.cheb_hi)
    g = np.asarray(prob.g, dtype=np.float64).reshape(shape if prob.op_kind == "blur" else (-1,))
    s4 = (prob.eta, prob.delta) if getattr(prob, "stop_s4", False) else None
    ostop = (prob.outer_rtol, prob.outer_min) if getattr(prob, "stop_outer", False) else None
    return solve(shape, op, g, prob.reg, prob.T, prob.tau, prob.eps,
                 prob.outer if outer is None else outer, prob.inner if inner is None else inner,
                 prob.levels, sm, history, s4=s4, outer_stop=ostop)
