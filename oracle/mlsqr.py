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


def mlsqr_taus(apply_A, apply_AT, apply_Minv, g, taus, iters):
    """The iterate after ``iters`` steps for every damping tau in ``taus`` from one Krylov run.

    Section 3.3: the bidiagonalisation does not depend on tau, so the basis (here the
    M-weighted vectors v_i that MLSQR combines into f) and the bidiagonal B_i are formed once;
    for each tau the projected problem (3.6),
        min_y || [B_i; sqrt(tau) I] y - beta_1 e_1 ||,
    is solved (a dense least-squares solve of the stacked (2i+1) x i matrix, its definition)
    and f(tau) = V_i y. Returns (list of f, iterations completed).
    """
    g = np.asarray(g, dtype=np.float64)
    beta = float(np.linalg.norm(g))
    shape = np.shape(apply_AT(g))
    if beta <= TINY:
        return [np.zeros(shape) for _ in taus], 0
    u = g / beta
    p = apply_AT(u)
    v = apply_Minv(p)
    a2 = float(np.vdot(v, p))
    if a2 < 0.0:
        raise NotSPD(a2)
    alpha = math.sqrt(a2)
    if alpha <= TINY:
        return [np.zeros(shape) for _ in taus], 0
    p = p / alpha
    v = v / alpha
    alphas, betas, basis = [alpha], [beta], [v]
    done = 0
    for i in range(1, iters + 1):
        # the steps of mlsqr() (same stops): step i needs beta_{i+1} and alpha_{i+1}, and f_i
        # combines v_1..v_i
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
        betas.append(beta)                      # beta_{i+1}
        alphas.append(alpha)                    # alpha_{i+1}
        basis.append(v)                         # v_{i+1} (used from step i+1 on)
        done = i
    k = done
    if k == 0:
        return [np.zeros(shape) for _ in taus], 0
    B = np.zeros((k + 1, k))
    for c in range(k):
        B[c, c] = alphas[c]
        B[c + 1, c] = betas[c + 1]
    rhs = np.zeros(2 * k + 1)
    rhs[0] = betas[0]
    V = np.stack([np.ravel(b) for b in basis[:k]], axis=1)
    out = []
    for tau in taus:
        S = np.vstack([B, math.sqrt(tau) * np.eye(k)])
        y = np.linalg.lstsq(S, rhs, rcond=None)[0]
        out.append((V @ y).reshape(shape))
    return out, k
