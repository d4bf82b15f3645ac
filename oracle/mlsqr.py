"""Algorithm 2 (MLSQR, factorization-free priorconditioned LSQR) with damping.

Bidiagonalisation (Section 3.2): the Golub-Kahan process of Section 3.1 run in
the M-weighted inner product, keeping p = M v so that only solves with M are
needed, never products with M or a factor of it.

Damping (Section 3.3): the projected problem (3.6) stacks sqrt(tau) I under the
bidiagonal B_i. Its QR factorisation, updated one column at a time, first
rotates the new damping row into rho_bar (c1, s1 below) and then applies the
usual Givens rotation with beta_{i+1} (the orthogonal transformation of
Algorithm 1). For tau = 0 the first rotation is the identity.

Readings of points the paper leaves open:
* initialisation normalises p by alpha_1 as well as v (the in-loop update of p
  needs p = M v_1, and the initial step has the same form as the loop step);
* if beta or alpha falls to <= 1e-300 the iteration stops and keeps the last
  completed f (exact termination of the Krylov process);
* alpha^2 < 0 means the preconditioner is not positive definite: an error.

``apply_Minv`` is any fixed SPD operator standing for M^{-1} (a V-cycle, an
exact solve, or the identity, which gives plain damped LSQR).

Stopping (Section 3.4): besides the iteration cap, the Morozov discrepancy
principle S4 ends the iteration at the first i with ||g - A f_i|| <= eta * delta.
The residual is formed here from its definition, one extra product with A per
iteration, checked after the update of f (the test closes each loop pass of
Algorithm 2).
"""

import math

import numpy as np

TINY = 1e-300


class NotSPD(ArithmeticError):
    pass


def mlsqr(apply_A, apply_AT, apply_Minv, g, tau, iters, history=None, resid_stop=None):
    """Run at most ``iters`` MLSQR iterations from f = 0; returns (f, iterations completed).

    ``resid_stop`` (eta * delta of S4, or None): stop after the first iteration whose
    iterate has ||g - A f_i|| <= resid_stop."""
    lam = math.sqrt(tau)
    g = np.asarray(g, dtype=np.float64)
    beta = float(np.linalg.norm(g))
    if beta <= TINY:
        return np.zeros_like(apply_AT(g)), 0
    u = g / beta
    p = apply_AT(u)
    v = apply_Minv(p)
    a2 = float(np.vdot(v, p))
    if a2 < 0.0:
        raise NotSPD(a2)
    alpha = math.sqrt(a2)
    if alpha <= TINY:
        return np.zeros_like(p), 0
    p = p / alpha
    v = v / alpha
    w = v.copy()
    f = np.zeros_like(v)
    phibar, rhobar = beta, alpha
    if history is not None:
        history.append(dict(i=0, alpha=alpha, beta=beta, phibar=phibar))
    done = 0
    for i in range(1, iters + 1):
        # bidiagonalisation
        u = apply_A(v) - alpha * u
        beta = float(np.linalg.norm(u))
        if beta <= TINY:
            break
        u = u / beta
        p = apply_AT(u) - beta * p
        v = apply_Minv(p)
        a2 = float(np.vdot(v, p))
        if a2 < 0.0:
            raise NotSPD(a2)
        alpha = math.sqrt(a2)
        if alpha <= TINY:
            break
        p = p / alpha
        v = v / alpha
        # damping rotation, then the Givens rotation of the bidiagonal
        rhohat = math.hypot(rhobar, lam)
        c1, s1 = rhobar / rhohat, lam / rhohat
        phibar = c1 * phibar
        rho = math.hypot(rhohat, beta)
        c, s = rhohat / rho, beta / rho
        theta = s * alpha
        rhobar = -c * alpha
        phi = c * phibar
        phibar = s * phibar
        # update
        f = f + (phi / rho) * w
        w = v - (theta / rho) * w
        done = i
        resid = None
        if resid_stop is not None:
            resid = float(np.linalg.norm(np.ravel(g) - np.ravel(apply_A(f))))
        if history is not None:
            history.append(dict(i=i, alpha=alpha, beta=beta, phibar=phibar, rho=rho, phi=phi,
                                theta=theta, s1=s1, resid=resid))
        if resid is not None and resid <= resid_stop:
            break
    return f, done
