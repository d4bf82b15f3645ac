"""Workload recipes: the five synthetic problem families and small test cases.

Each recipe fixes the grid, the phantom family, the forward operator, the noise
level, the regulariser (kind, T, tau), the fixed outer x inner iteration counts
and the multigrid/smoother settings, then draws phantom and noise from one seed.

Families (sizes are the defaults; tests shrink them):
  C1  2D 64^2 blur (sigma 2, radius 4), 8 rectangles, 1% noise, smoothed TV
      T=0.01, tau=50, 10 x 50, 4 levels, Jacobi V(2,2) omega 0.8.
  C2  3D 64^3, dense ring sensitivity 4096 x 262144, 5 ellipsoids, 1% noise,
      Perona-Malik (log) T=0.05, tau=20, 8 x 40, 5 levels, Jacobi V(2,2).
  C3  3D 128^3 blur (sigma 3, 19 taps), 20 boxes/spheres, 0.5% noise, smoothed
      TV T=0.02, tau=100, 10 x 60, 6 levels, Chebyshev(3) on [1/3, 2].
  C4  64 instances of 64^3 sharing one 8192 x 262144 sensitivity (8 source
      rings), regulariser drawn per instance from {sTV 0.02, PM-log 0.05},
      tau=20, 8 x 40.
  C5  request stream: Poisson arrivals (mean gap 20 ms), grid size uniform over
      {32,48,64,96,128}^3, blur sigma ~ U(1.5,3.5) with radius ceil(3 sigma),
      10 boxes/spheres scaled by n/128, 1% noise, regulariser uniform over
      {Tikhonov, sTV 0.02, PM-log 0.05}, tau ~ U(10,100), 8 x 40.
"""

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from . import operators as ops
from . import phantoms

REG_KINDS = ("tikhonov", "stv", "pm_log", "pm_exp")


@dataclass
class Problem:
    name: str
    dims: tuple                       # (nx, ny, nz)
    f_true: np.ndarray                # (nz, ny, nx) float64
    g: np.ndarray                     # float32 data, (n_Y,) dense or (nz, ny, nx) blur
    op_kind: str                      # "blur" | "dense"
    taps: Optional[np.ndarray] = None   # float32, 2*radius+1 (blur)
    A: Optional[np.ndarray] = None      # float32 row-major (n_Y, n_X) (dense)
    reg: str = "stv"
    T: float = 0.01
    tau: float = 50.0
    eps: float = 1e-6
    outer: int = 10
    inner: int = 50
    levels: int = 4
    smoother: str = "jacobi"          # "jacobi" | "chebyshev"
    nu_pre: int = 2
    nu_post: int = 2
    omega: float = 0.8
    cheb_degree: int = 3
    cheb_lo: float = 1.0 / 3.0
    cheb_hi: float = 2.0
    noise_sd: float = 0.0
    delta: float = 0.0                # Euclidean norm of the noise actually drawn (noise level)
    # adaptive stopping (off by default: fixed outer x inner counts)
    stop_s4: bool = False             # stop MLSQR once ||g - A f_i|| <= eta * delta
    eta: float = 1.1
    stop_outer: bool = False          # stop the outer loop once R(f^k) no longer falls by
    outer_rtol: float = 0.0           #   more than outer_rtol * R(f^{k-1}) (checked for k >=
    outer_min: int = 3                #   outer_min)
    extra: dict = field(default_factory=dict)

    @property
    def n_x(self):
        nx, ny, nz = self.dims
        return nx * ny * nz

    @property
    def n_y(self):
        return self.A.shape[0] if self.op_kind == "dense" else self.n_x

    @property
    def radius(self):
        return (len(self.taps) - 1) // 2 if self.taps is not None else 0


def auto_levels(dims, max_levels=16):
    """Number of grids: keep halving while every coarsened axis is even and > 4."""
    nx, ny, nz = dims
    axes = [nx, ny] + ([nz] if nz > 1 else [])
    levels = 1
    while levels < max_levels and all(a % 2 == 0 and a > 4 for a in axes):
        axes = [a // 2 for a in axes]
        levels += 1
    return levels


def make_blur_problem(name, f_true, rng, sigma, radius, noise_frac, **kw):
    taps = ops.gaussian_taps(sigma, radius)
    g, sd, delta = ops.blur_data(rng, f_true, taps, noise_frac)
    nz, ny, nx = f_true.shape
    return Problem(name=name, dims=(nx, ny, nz), f_true=f_true, g=g, op_kind="blur", taps=taps,
                   noise_sd=sd, delta=delta, extra={"sigma": sigma}, **kw)


def make_dense_problem(name, f_true, rng, A, noise_frac, ring=None, **kw):
    """``ring`` = (sources, detectors, mu) of the sensitivity A, kept for the matrix-free form."""
    g, sd, delta = ops.dense_data(rng, A, f_true, noise_frac)
    nz, ny, nx = f_true.shape
    extra = {"ring": ring} if ring is not None else {}
    return Problem(name=name, dims=(nx, ny, nz), f_true=f_true, g=g, op_kind="dense", A=A,
                   noise_sd=sd, delta=delta, extra=extra, **kw)


def config_c1(seed=0, n=64, outer=10, inner=50):
    rng = np.random.default_rng(seed)
    f = phantoms.rectangles_2d(rng, n, count=8, side_lo=max(1, n // 16), side_hi=max(2, n // 2))
    return make_blur_problem("c1", f, rng, sigma=2.0, radius=4, noise_frac=0.01, reg="stv",
                             T=0.01, tau=50.0, eps=1e-6, outer=outer, inner=inner,
                             levels=4, smoother="jacobi", nu_pre=2,
                             nu_post=2, omega=0.8)


def config_c2(seed=1, n=64, outer=8, inner=40, A=None):
    rng = np.random.default_rng(seed)
    f = phantoms.ellipsoids_3d(rng, n, count=5)
    mu = 0.5 * 64.0 / n
    if A is None:
        A = ops.dense_sensitivity(n, mu=mu)
    return make_dense_problem("c2", f, rng, A, noise_frac=0.01, ring=(*ops.ring_points(n), mu),
                              reg="pm_log", T=0.05, tau=20.0,
                              eps=1e-6, outer=outer, inner=inner, levels=auto_levels((n, n, n)),
                              smoother="jacobi", nu_pre=2, nu_post=2, omega=0.8)


def config_c3(seed=2, n=128, outer=10, inner=60, smoother="chebyshev"):
    rng = np.random.default_rng(seed)
    s = n / 128.0
    f = phantoms.boxes_spheres_3d(rng, n, count=20, edge_lo=max(1, round(8 * s)),
                                  edge_hi=max(2, round(40 * s)), rad_lo=4.0 * s, rad_hi=20.0 * s)
    return make_blur_problem("c3", f, rng, sigma=3.0, radius=9, noise_frac=0.005, reg="stv",
                             T=0.02, tau=100.0, eps=1e-6, outer=outer, inner=inner,
                             levels=auto_levels((n, n, n)), smoother=smoother, nu_pre=1,
                             nu_post=1, omega=0.8, cheb_degree=3, cheb_lo=1.0 / 3.0, cheb_hi=2.0)


def c4_matrix(n=64):
    """Shared sensitivity for the batched family: 8 source rings x 16, 4 detector rings x 16."""
    return ops.dense_sensitivity(n, mu=0.5 * 64.0 / n, n_src_rings=8, n_det_rings=4)


def config_c4(i, A, n=64, outer=8, inner=40):
    rng = np.random.default_rng(1000 + i)
    if rng.uniform() < 0.5:
        reg, T = "stv", 0.02
    else:
        reg, T = "pm_log", 0.05
    f = phantoms.ellipsoids_3d(rng, n, count=5)
    return make_dense_problem(f"c4_{i}", f, rng, A, noise_frac=0.01,
                              ring=(*ops.ring_points(n, 8, 4), 0.5 * 64.0 / n), reg=reg, T=T, tau=20.0,
                              eps=1e-6, outer=outer, inner=inner, levels=auto_levels((n, n, n)),
                              smoother="jacobi", nu_pre=2, nu_post=2, omega=0.8)


def config_c4_batch(A, count=64, n=64, outer=8, inner=40, chunk=256):
    """Instances 0..count-1 of the batched family, equal to ``config_c4(i, A)`` one by one
    (same seeds and draw order: regulariser, phantom, then noise per instance), with the clean
    data of all instances formed in one pass over A: each float64 row chunk of A multiplies the
    matrix of all phantoms (the one-at-a-time recipe converts A once per instance)."""
    rngs, meta, F = [], [], []
    for i in range(count):
        rng = np.random.default_rng(1000 + i)
        if rng.uniform() < 0.5:
            reg, T = "stv", 0.02
        else:
            reg, T = "pm_log", 0.05
        f = phantoms.ellipsoids_3d(rng, n, count=5)
        rngs.append(rng)
        meta.append((reg, T, f))
        F.append(f.ravel())
    F = np.stack(F, axis=1)                                  # n^3 x count, float64
    clean = np.empty((A.shape[0], count))
    for r0 in range(0, A.shape[0], chunk):
        clean[r0:r0 + chunk] = A[r0:r0 + chunk].astype(np.float64) @ F
    ring = (*ops.ring_points(n, 8, 4), 0.5 * 64.0 / n)
    out = []
    for i, (rng, (reg, T, f)) in enumerate(zip(rngs, meta)):
        g, sd, delta = ops.add_noise(rng, clean[:, i], 0.01)
        nz, ny, nx = f.shape
        out.append(Problem(name=f"c4_{i}", dims=(nx, ny, nz), f_true=f, g=g, op_kind="dense", A=A,
                           noise_sd=sd, delta=delta, extra={"ring": ring}, reg=reg, T=T, tau=20.0,
                           eps=1e-6, outer=outer, inner=inner, levels=auto_levels((n, n, n)),
                           smoother="jacobi", nu_pre=2, nu_post=2, omega=0.8))
    return out


C5_SIZES = (32, 48, 64, 96, 128)


def c5_request(r, sizes=C5_SIZES, outer=8, inner=40):
    """Request r of the served stream (its own seed 5000 + r)."""
    rng = np.random.default_rng(5000 + r)
    n = int(sizes[rng.integers(0, len(sizes))])
    sigma = float(rng.uniform(1.5, 3.5))
    radius = ops.radius_for_sigma(sigma)
    reg = ("tikhonov", "stv", "pm_log")[rng.integers(0, 3)]
    T = {"tikhonov": 1.0, "stv": 0.02, "pm_log": 0.05}[reg]
    tau = float(rng.uniform(10.0, 100.0))
    s = n / 128.0
    f = phantoms.boxes_spheres_3d(rng, n, count=10, edge_lo=max(1, round(8 * s)),
                                  edge_hi=max(2, round(40 * s)), rad_lo=4.0 * s, rad_hi=20.0 * s)
    return make_blur_problem(f"c5_{r}", f, rng, sigma=sigma, radius=radius, noise_frac=0.01,
                             reg=reg, T=T, tau=tau, eps=1e-6, outer=outer, inner=inner,
                             levels=auto_levels((n, n, n)), smoother="jacobi", nu_pre=2,
                             nu_post=2, omega=0.8)


def config_c5_requests(count=2000, seed=5, mean_gap_s=0.020):
    """Arrival times (seconds from stream start) of ``count`` Poisson requests."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(mean_gap_s, size=count)
    return np.cumsum(gaps) - gaps[0]


def small_blur_case(seed, dims, sigma=1.5, radius=3, reg="stv", T=0.05, tau=10.0, outer=3,
                    inner=8, levels=None, smoother="jacobi", nu_pre=2, nu_post=2, omega=0.8,
                    eps=1e-6, noise_frac=0.01, cheb_lo=1.0 / 3.0, cheb_hi=2.0, cheb_degree=3):
    """Small blur problem on an arbitrary (nx, ny, nz) grid with a random-box phantom."""
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    f = np.zeros((nz, ny, nx))
    for _ in range(6):
        c = [rng.integers(0, m) for m in (nx, ny, nz)]
        e = [rng.integers(1, max(2, m // 2) + 1) for m in (nx, ny, nz)]
        f[c[2]:c[2] + e[2], c[1]:c[1] + e[1], c[0]:c[0] + e[0]] += rng.uniform(0.0, 1.0)
    if levels is None:
        levels = auto_levels(dims)
    return make_blur_problem(f"blur_{nx}x{ny}x{nz}_s{seed}", f, rng, sigma=sigma, radius=radius,
                             noise_frac=noise_frac, reg=reg, T=T, tau=tau, eps=eps, outer=outer,
                             inner=inner, levels=levels, smoother=smoother, nu_pre=nu_pre,
                             nu_post=nu_post, omega=omega, cheb_lo=cheb_lo, cheb_hi=cheb_hi,
                             cheb_degree=cheb_degree)


def small_dense_case(seed, n, reg="pm_log", T=0.05, tau=20.0, outer=3, inner=8, levels=None,
                     smoother="jacobi", n_src_rings=2, n_det_rings=2, noise_frac=0.01,
                     eps=1e-6, A=None):
    """Small cubic dense problem (ring sensitivity scaled to n) with an ellipsoid phantom."""
    rng = np.random.default_rng(seed)
    f = phantoms.ellipsoids_3d(rng, n, count=3)
    mu = 0.5 * 64.0 / n / 4.0
    if A is None:
        A = ops.dense_sensitivity(n, mu=mu, n_src_rings=n_src_rings, n_det_rings=n_det_rings)
    if levels is None:
        levels = auto_levels((n, n, n))
    return make_dense_problem(f"dense_{n}_s{seed}", f, rng, A, noise_frac=noise_frac,
                              ring=(*ops.ring_points(n, n_src_rings, n_det_rings), mu), reg=reg,
                              T=T, tau=tau, eps=eps, outer=outer, inner=inner, levels=levels,
                              smoother=smoother, nu_pre=2, nu_post=2, omega=0.8)
