"""Where float32 vector arithmetic meets the 1e-3 parity bar (CPU, no GPU).

The library's single-precision path keeps vectors, stencils and products in float32 and the
Krylov scalars in float64. With eps << 1 the constant vector is an eigenvector of M with
eigenvalue eps, so A L^{-1} (M = L^T L) has one singular value about eps^{-1/2} times the rest;
without enough damping tau, Krylov rounding is amplified along it. A float32 emulation of the
oracle (``fp32_emulation``: the oracle's own matrices cast to float32, float64 reductions and
scalars) is compared here with the FP64 oracle across (tau, eps) on a blur problem scaled as
the configured workloads are (normalised taps, so ||A|| <= 1; Perona-Malik and Tikhonov
diffusivities <= 1, the least damped prior). This pins the region where a GPU parity test
against the 1e-3 bar is meaningful:

* every damping tau >= 10 at eps = 1e-6 (the configured workloads use tau in [10, 100],
  eps = 1e-6) stays two orders of magnitude inside the bar;
* undamped or weakly damped solves (tau <= 1) at eps <= 1e-4 miss it in float32 by itself,
  so the GPU's undamped tests run at eps = 0.1, where the emulation meets the bar.
"""

import numpy as np
import pytest

import fp32_emulation as E
import gen
from oracle import lagged, multigrid


def _err(reg, T, tau, eps, inner=12, dims=(24, 24, 1), levels=3, seed=16):
    p = gen.small_blur_case(seed, dims, reg=reg, T=T, tau=tau, outer=2, inner=inner,
                            levels=levels, eps=eps)
    sm = multigrid.Smoother(p.smoother, p.nu_pre, p.nu_post, p.omega)
    f_ref, _ = lagged.solve_problem(p)
    f32 = E.solve_blur(p, sm)
    return float(np.linalg.norm(f32 - f_ref) / np.linalg.norm(f_ref))


def test_emulation_is_float32_rounding_only():
    # well damped: the emulation sits at float32 resolution of the oracle
    assert _err("pm_log", 0.05, 100.0, 1e-6) <= 1e-6


@pytest.mark.parametrize("reg,T", [("pm_log", 0.05), ("tikhonov", 1.0)])
@pytest.mark.parametrize("tau", [10.0, 20.0, 100.0])
def test_configured_damping_is_inside_the_bar(reg, T, tau):
    assert _err(reg, T, tau, 1e-6) <= 1e-5


@pytest.mark.parametrize("tau,eps", [(0.0, 1e-6), (0.1, 1e-6), (1.0, 1e-6), (1.0, 1e-4)])
def test_weak_damping_small_eps_misses_the_bar_in_float32(tau, eps):
    assert _err("pm_log", 0.05, tau, eps) > 1e-3


def test_undamped_gpu_test_regime_is_inside_the_bar():
    # the GPU's undamped parity case: tau = 0, eps = 0.1, 2 x 6 iterations
    assert _err("pm_log", 0.05, 0.0, 0.1, inner=6) <= 1e-4


def test_three_dimensional_configured_regime():
    assert _err("stv", 0.02, 20.0, 1e-6, dims=(16, 16, 16), levels=3) <= 1e-5


def test_early_iterates_of_a_weakly_regularised_3d_solve():
    """The float32 deviation is a transient of the first MLSQR steps, not of the converged
    solve: on a 48^3 Tikhonov blur problem (eps = 1e-6, tau = 54.5, the served stream's
    regime) the emulation misses the oracle by about 1e-3 after 4 inner steps and sits at
    float32 resolution from 8 steps on. Parity tests of such problems therefore run at least
    8 inner steps (the served stream runs 40)."""
    import math
    rng = np.random.default_rng(924)
    sigma = float(rng.uniform(1.5, 3.5))
    tau = float(rng.uniform(10, 100))
    errs = {}
    for inner in (4, 8):
        p = gen.small_blur_case(924, (48, 48, 48), sigma=sigma, radius=int(math.ceil(3 * sigma)),
                                reg="tikhonov", T=1.0, tau=tau, outer=2, inner=inner,
                                levels=gen.auto_levels((48, 48, 48)))
        sm = multigrid.Smoother(p.smoother, p.nu_pre, p.nu_post, p.omega)
        f_ref, _ = lagged.solve_problem(p)
        errs[inner] = float(np.linalg.norm(E.solve_blur(p, sm) - f_ref) / np.linalg.norm(f_ref))
    assert errs[4] > 3e-4
    assert errs[8] <= 5e-6


def test_three_dimensional_tikhonov_edge_of_the_region():
    # the region's edge depends on the problem: a 32 x 32 x 16 Tikhonov case with a Chebyshev
    # V-cycle misses the bar in float32 at tau = 5 and is an order inside it at tau = 20 (the
    # GPU's batch test of this shape uses tau >= 20)
    kw = dict(dims=(32, 32, 16), levels=3, inner=9, seed=72)
    p5 = _err_cheb("tikhonov", 1.0, 5.0, 1e-6, **kw)
    p20 = _err_cheb("tikhonov", 1.0, 20.0, 1e-6, **kw)
    assert p5 > 1e-3 and p20 < 1e-4, (p5, p20)


def _err_cheb(reg, T, tau, eps, inner, dims, levels, seed):
    p = gen.small_blur_case(seed, dims, reg=reg, T=T, tau=tau, outer=2, inner=inner,
                            levels=levels, eps=eps, smoother="chebyshev", nu_pre=1, nu_post=1)
    sm = multigrid.Smoother(p.smoother, p.nu_pre, p.nu_post, p.omega)
    f_ref, _ = lagged.solve_problem(p)
    f32 = E.solve_blur(p, sm)
    return float(np.linalg.norm(f32 - f_ref) / np.linalg.norm(f_ref))
