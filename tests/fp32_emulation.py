"""Float32 emulation of the method, for locating where float32 vector arithmetic meets the
parity bar (test infrastructure, CPU only; no part of the HIP path).

It runs the oracle's algorithm with the number formats of the library's single-precision
path: vectors, blur products, multigrid level operators and smoother arithmetic in float32;
inner products and norms accumulated in float64; Krylov scalars (alpha, beta, rotations) in
float64; the coarsest-grid solve in float64. The operators are the oracle's own matrices
(Galerkin hierarchy, gradient, blur definition) cast to float32, so any difference from the
FP64 oracle is rounding, not a different method.
"""

import math

import numpy as np
import scipy.linalg as sla

from oracle import grid, multigrid, regularizers
from oracle.operators import _correlate_axis

F32 = np.float32


def _blur32(x, taps, shape):
    y = np.asarray(x, dtype=F32).reshape(shape)
    w = np.asarray(taps, dtype=F32)
    for axis in (2, 1, 0):
        if shape[axis] > 1:
            y = _correlate_axis(y, w, axis).astype(F32)
    return y.ravel()


def _dot(a, b):
    return float(np.dot(np.asarray(a, np.float64), np.asarray(b, np.float64)))


def _vcycle32(h, A32, D32, P32, b, sm, level=0):
    if level == h.levels - 1:
        return sla.cho_solve(h.chol, np.asarray(b, np.float64)).astype(F32)
    A, D = A32[level], D32[level]

    def smooth(x, steps):
        for _ in range(steps):
            if sm.kind == "jacobi":
                x = (x + F32(sm.omega) * ((b - A @ x) / D)).astype(F32)
            else:
                theta, delta = 0.5 * (sm.hi + sm.lo), 0.5 * (sm.hi - sm.lo)
                sigma = theta / delta
                r = (b - A @ x).astype(F32)
                rho = 1.0 / sigma
                d = ((r / D) / F32(theta)).astype(F32)
                for _ in range(sm.degree):
                    x = (x + d).astype(F32)
                    r = (r - A @ d).astype(F32)
                    rn = 1.0 / (2.0 * sigma - rho)
                    d = (F32(rn * rho) * d + F32(2.0 * rn / delta) * (r / D)).astype(F32)
                    rho = rn
        return x

    x = smooth(np.zeros_like(b), sm.nu_pre)
    r = (b - A @ x).astype(F32)
    e = _vcycle32(h, A32, D32, P32, (P32[level].T @ r).astype(F32), sm, level + 1)
    x = (x + P32[level] @ e).astype(F32)
    return smooth(x, sm.nu_post)


def solve_blur(p, sm):
    """f^K of a blur problem (``gen.Problem``) with float32 vectors and float64 scalars."""
    nx, ny, nz = p.dims
    shape = (nz, ny, nx)
    taps = np.asarray(p.taps, F32)
    fwd = lambda x: _blur32(x, taps, shape)
    adj = lambda y: _blur32(y, taps[::-1], shape)
    g = np.asarray(p.g, F32).ravel()
    lam = math.sqrt(p.tau)
    f = np.zeros(nx * ny * nz, F32)
    for _ in range(p.outer):
        kappa = regularizers.diffusivity(p.reg, grid.grad_norm(f.reshape(shape).astype(float)), p.T)
        h = multigrid.Hierarchy(grid.prior_matrix(kappa.astype(F32).astype(float), p.eps), shape,
                                p.levels)
        A32 = [A.astype(F32) for A in h.A]
        D32 = [d.astype(F32) for d in h.D]
        P32 = [P.astype(F32) for P in h.P]
        B = lambda q: _vcycle32(h, A32, D32, P32, q, sm)
        beta = math.sqrt(_dot(g, g))
        u = (g / F32(beta)).astype(F32)
        q = adj(u)
        v = B(q)
        alpha = math.sqrt(_dot(v, q))
        q = (q / F32(alpha)).astype(F32)
        v = (v / F32(alpha)).astype(F32)
        w = v.copy()
        f = np.zeros_like(v)
        phibar, rhobar = beta, alpha
        for _ in range(p.inner):
            u = (fwd(v) - F32(alpha) * u).astype(F32)
            beta = math.sqrt(_dot(u, u))
            u = (u / F32(beta)).astype(F32)
            q = (adj(u) - F32(beta) * q).astype(F32)
            v = B(q)
            alpha = math.sqrt(_dot(v, q))
            q = (q / F32(alpha)).astype(F32)
            v = (v / F32(alpha)).astype(F32)
            rhohat = math.hypot(rhobar, lam)
            phibar = (rhobar / rhohat) * phibar
            rho = math.hypot(rhohat, beta)
            c, s = rhohat / rho, beta / rho
            theta = s * alpha
            rhobar = -c * alpha
            phi = c * phibar
            phibar = s * phibar
            f = (f + F32(phi / rho) * w).astype(F32)
            w = (v - F32(theta / rho) * w).astype(F32)
    return f.reshape(shape)
