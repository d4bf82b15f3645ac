"""Penalty densities r(t) and diffusivities kappa(t) = r'(t)/t.

r(t) is given by eq. (1.3) (first-order Tikhonov), the smoothed form of (1.4)
(total variation with smoothing parameter T) and both forms of (1.5)
(Perona-Malik, log and exponential). The diffusivity c_f = r'(|grad f|)/|grad f|
comes from the Frechet derivative (1.12), the coefficient of the diffusion
operator (1.13). Each kappa below is r'(t)/t simplified by hand so that it is
finite at t = 0; a CPU test checks it against a difference quotient of r.
"""

import numpy as np

KINDS = ("tikhonov", "stv", "pm_log", "pm_exp")


def penalty_density(kind, t, T):
    t = np.asarray(t, dtype=np.float64)
    if kind == "tikhonov":          # r = t^2 / 2                     (1.3)
        return 0.5 * t * t
    if kind == "stv":               # r = T sqrt(1 + (t/T)^2)         (1.4), smoothed TV
        return T * np.sqrt(1.0 + (t / T) ** 2)
    if kind == "pm_log":            # r = T^2/2 log(1 + (t/T)^2)      (1.5), left
        return 0.5 * T * T * np.log1p((t / T) ** 2)
    if kind == "pm_exp":            # r = T^2/2 (1 - exp(-t^2/T^2))   (1.5), right
        return 0.5 * T * T * (1.0 - np.exp(-(t * t) / (T * T)))
    raise ValueError(f"unknown regulariser {kind!r}")


def diffusivity(kind, t, T):
    t = np.asarray(t, dtype=np.float64)
    if kind == "tikhonov":          # r' = t
        return np.ones_like(t)
    if kind == "stv":               # r' = t / sqrt(T^2 + t^2)
        return 1.0 / np.sqrt(T * T + t * t)
    if kind == "pm_log":            # r' = t / (1 + t^2/T^2)
        return 1.0 / (1.0 + (t * t) / (T * T))
    if kind == "pm_exp":            # r' = t exp(-t^2/T^2)
        return np.exp(-(t * t) / (T * T))
    raise ValueError(f"unknown regulariser {kind!r}")
