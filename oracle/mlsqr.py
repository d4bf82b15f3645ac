"""MLSQR (factorization-free priorconditioned LSQR, Section 3.2) with damping (Section 3.3).

The method is two independent pieces, composed by ``mlsqr``:

* ``Bidiag`` -- the Golub-Kahan bidiagonalisation of A (Section 3.1) run in the M-weighted
  inner product on the domain (Section 3.2): beta_1 u_1 = g, alpha_1 v_1 = M^{-1} A^T u_1, and
  for j >= 1
      beta_{j+1} u_{j+1} = A v_j - alpha_j u_j,
      alpha_{j+1} v_{j+1} = M^{-1} A^T u_{j+1} - beta_{j+1} v_j,
  with ||u||_2 = 1 and ||v||_M = 1. Only solves with M appear: the vector q = M v is carried
  alongside v (q_{j+1} is formed from A^T u_{j+1} - beta_{j+1} q_j, then v = M^{-1} q and
  alpha = sqrt(v . q) = ||v||_M before the normalisation).
* ``DampedQR`` -- the QR factorisation of the damped projected problem (3.6),
      min_y || [B_k; sqrt(tau) I] y - beta_1 e_1 ||,
  updated one column of the lower bidiagonal B_k at a time: the new damping row is rotated
  into the running diagonal entry rho_bar (c1, s1), then the subdiagonal beta_{k+1} (c, s),
  giving R's diagonal rho_k, its superdiagonal theta_{k+1} and the rotated right-hand side
  phi_k; |phi_bar| is the norm of the projected residual. For tau = 0 the first rotation is
  the identity and this is the QR update of plain LSQR (Section 3.1).

The iterate f_k = V_k y_k is accumulated without storing V_k, through the directions
W_k = V_k R_k^{-1}: f_k = f_{k-1} + (phi_k / rho_k) w_k and w_{k+1} = v_{k+1} - (theta_{k+1} /
rho_k) w_k.

Readings of points the paper leaves open:
* the first right vector is normalised like every later one (q_1 = A^T u_1 / alpha_1 as well
  as v_1), so that q_j = M v_j holds from the start;
* if beta or alpha falls to <= 1e-300 the iteration stops and keeps the last completed f
  (exact termination of the Krylov process);
* alpha^2 = v . q < 0 means the preconditioner is not positive definite: an error.

``apply_Minv`` is any fixed SPD operator standing for M^{-1} (a V-cycle, an exact solve, or
the identity, which gives plain damped LSQR).

Stopping (Section 3.4): besides the iteration cap, the Morozov discrepancy principle S4 ends
the iteration at the first k with ||g - A f_k|| <= eta * delta. The residual is formed here
from its definition, one extra product with A per iteration, checked once f_k is formed.
"""

import math

import numpy as np

TINY = 1e-300


class NotSPD(ArithmeticError):
    pass


class Bidiag:
    """Golub-Kahan bidiagonalisation of A in the M-inner product (Sections 3.1-3.2).

    After construction (``ok`` true) it holds beta_1, u_1, alpha_1, v_1 and q_1 = M v_1;
    each ``advance()`` forms beta_{j+1}, u_{j+1}, alpha_{j+1}, v_{j+1}, q_{j+1} and returns
    False (changing nothing) when the process terminates exactly."""

    def __init__(self, apply_A, apply_AT, apply_Minv, g):
        self.A, self.AT, self.Minv = apply_A, apply_AT, apply_Minv
        g = np.asarray(g, dtype=np.float64)
        self.ok = False
        self.beta = float(np.linalg.norm(g))
        self.shape = None
        if self.beta <= TINY:
            self.shape = np.shape(apply_AT(g))
            return
        self.u = g / self.beta
        right = self._right(self.AT(self.u))
        if right is None:
            return
        self.alpha, self.q, self.v = right
        self.ok = True

    def _right(self, q):
        """M-normalise a new right vector given as q = M (alpha v): (alpha, q, v), or None at
        exact termination (the shape is then recorded)."""
        v = self.Minv(q)
        a2 = float(np.vdot(v, q))
        if a2 < 0.0:
            raise NotSPD(a2)
        alpha = math.sqrt(a2)
        if alpha <= TINY:
            self.shape = np.shape(q)
            return None
        return alpha, q / alpha, v / alpha

    def advance(self):
        u = self.A(self.v) - self.alpha * self.u
        beta = float(np.linalg.norm(u))
        if beta <= TINY:
            return False
        u = u / beta
        right = self._right(self.AT(u) - beta * self.q)
        if right is None:
            return False
        self.u, self.beta = u, beta
        self.alpha, self.q, self.v = right
        return True


class DampedQR:
    """QR of [B_k; lam I] (eq. (3.6)) one column at a time; see the module docstring."""

    def __init__(self, beta1, alpha1, lam):
        self.lam = lam
        self.rhobar = alpha1       # diagonal entry of the column not yet rotated
        self.phibar = beta1        # rotated right-hand side entry not yet final

    def column(self, beta_next, alpha_next):
        """Close column k with its subdiagonal beta_{k+1} (and the damping entry), opening
        column k+1 with alpha_{k+1}: returns (rho_k, theta_{k+1}, phi_k, s1)."""
        # the damping row of column k into rho_bar
        rhohat = math.hypot(self.rhobar, self.lam)
        c1, s1 = self.rhobar / rhohat, self.lam / rhohat
        self.phibar = c1 * self.phibar
        # the subdiagonal beta_{k+1}
        rho = math.hypot(rhohat, beta_next)
        c, s = rhohat / rho, beta_next / rho
        theta = s * alpha_next
        self.rhobar = -c * alpha_next
        phi = c * self.phibar
        self.phibar = s * self.phibar
        return rho, theta, phi, s1


def mlsqr(apply_A, apply_AT, apply_Minv, g, tau, iters, history=None, resid_stop=None):
    """At most ``iters`` MLSQR iterations from f = 0; returns (f, iterations completed).

    ``resid_stop`` (eta * delta of S4, or None): stop after the first iteration whose iterate
    has ||g - A f_k|| <= resid_stop. ``history`` (a list) receives one record per iteration:
    alpha and beta of the bidiagonalisation step it used, phibar, and the rotation values."""
    gk = Bidiag(apply_A, apply_AT, apply_Minv, g)
    if not gk.ok:
        return np.zeros(gk.shape), 0
    qr = DampedQR(gk.beta, gk.alpha, math.sqrt(tau))
    f = np.zeros_like(gk.v)
    w = gk.v.copy()
    if history is not None:
        history.append(dict(i=0, alpha=gk.alpha, beta=gk.beta, phibar=qr.phibar))
    g_flat = np.ravel(np.asarray(g, dtype=np.float64))
    done = 0
    for k in range(1, iters + 1):
        if not gk.advance():
            break
        rho, theta, phi, s1 = qr.column(gk.beta, gk.alpha)
        f = f + (phi / rho) * w
        w = gk.v - (theta / rho) * w
        done = k
        resid = None
        if resid_stop is not None:
            resid = float(np.linalg.norm(g_flat - np.ravel(apply_A(f))))
        if history is not None:
            history.append(dict(i=k, alpha=gk.alpha, beta=gk.beta, phibar=qr.phibar, rho=rho,
                                phi=phi, theta=theta, s1=s1, resid=resid))
        if resid is not None and resid <= resid_stop:
            break
    return f, done


def mlsqr_taus(apply_A, apply_AT, apply_Minv, g, taus, iters):
    """The iterate after ``iters`` steps for every damping tau in ``taus`` from one Krylov run.

    Section 3.3: the bidiagonalisation does not depend on tau, so the basis (here the
    M-weighted vectors v_j that MLSQR combines into f) and the bidiagonal B_k are formed once;
    for each tau the projected problem (3.6),
        min_y || [B_k; sqrt(tau) I] y - beta_1 e_1 ||,
    is solved (a dense least-squares solve of the stacked (2k+1) x k matrix, its definition)
    and f(tau) = V_k y. The same steps and stops as ``mlsqr``: step k needs beta_{k+1} and
    alpha_{k+1}, and f_k combines v_1..v_k. Returns (list of f, iterations completed)."""
    gk = Bidiag(apply_A, apply_AT, apply_Minv, g)
    if not gk.ok:
        return [np.zeros(gk.shape) for _ in taus], 0
    shape = np.shape(gk.v)
    alphas, betas, basis = [gk.alpha], [gk.beta], [gk.v]
    k = 0
    while k < iters and gk.advance():
        betas.append(gk.beta)                   # beta_{k+2}
        alphas.append(gk.alpha)                 # alpha_{k+2}
        basis.append(gk.v)                      # v_{k+2}
        k += 1
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
