"""Piecewise-constant phantoms on a zero background (shapes summed where they overlap).

Arrays are returned with shape ``(nz, ny, nx)`` (x fastest), float64. A 2D image
has ``nz == 1``. These stand in for the paper's fluorescent inclusions on a zero
background (Section 5.2); the shape mix and value ranges are this project's.
"""

import numpy as np


def rectangles_2d(rng, n, count=8, side_lo=4, side_hi=32):
    """``count`` axis-aligned rectangles, corner ~ U{0..n-1}^2, sides ~ U{lo..hi}, value U(0,1)."""
    f = np.zeros((1, n, n))
    for _ in range(count):
        cx, cy = rng.integers(0, n, size=2)
        sx, sy = rng.integers(side_lo, side_hi + 1, size=2)
        val = rng.uniform(0.0, 1.0)
        f[0, cy:cy + sy, cx:cx + sx] += val
    return f


def _coords(n):
    z, y, x = np.meshgrid(np.arange(n, dtype=np.float64), np.arange(n, dtype=np.float64),
                          np.arange(n, dtype=np.float64), indexing="ij")
    return x, y, z


def ellipsoids_3d(rng, n, count=5, centre_lo=None, centre_hi=None, axis_lo=4.0, axis_hi=14.0,
                  val_lo=0.5, val_hi=1.0):
    """``count`` axis-aligned ellipsoids; centre ~ U(lo,hi)^3, semi-axes ~ U(axis_lo,axis_hi)^3.

    Defaults reproduce the 64^3 recipe (centre U(12,52)); other sizes scale the
    centre range and semi-axes by n/64.
    """
    s = n / 64.0
    if centre_lo is None:
        centre_lo = 12.0 * s
    if centre_hi is None:
        centre_hi = 52.0 * s
    x, y, z = _coords(n)
    f = np.zeros((n, n, n))
    for _ in range(count):
        c = rng.uniform(centre_lo, centre_hi, size=3)
        a = rng.uniform(axis_lo * s, axis_hi * s, size=3)
        val = rng.uniform(val_lo, val_hi)
        inside = ((x - c[0]) / a[0]) ** 2 + ((y - c[1]) / a[1]) ** 2 + ((z - c[2]) / a[2]) ** 2 <= 1.0
        f[inside] += val
    return f


def boxes_spheres_3d(rng, n, count=20, edge_lo=8, edge_hi=40, rad_lo=4.0, rad_hi=20.0):
    """``count`` shapes, each a box (probability 1/2) or a sphere, value U(0,1).

    Box: corner ~ U{0..n-1}^3, edges ~ U{edge_lo..edge_hi}. Sphere: centre ~
    U(0,n)^3, radius ~ U(rad_lo, rad_hi). Sizes are given for n = 128; callers
    scale them for other grids.
    """
    x, y, z = _coords(n)
    f = np.zeros((n, n, n))
    for _ in range(count):
        is_box = rng.uniform() < 0.5
        if is_box:
            c = rng.integers(0, n, size=3)
            e = rng.integers(edge_lo, edge_hi + 1, size=3)
            val = rng.uniform(0.0, 1.0)
            f[c[2]:c[2] + e[2], c[1]:c[1] + e[1], c[0]:c[0] + e[0]] += val
        else:
            c = rng.uniform(0.0, float(n), size=3)
            r = rng.uniform(rad_lo, rad_hi)
            val = rng.uniform(0.0, 1.0)
            inside = (x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2 <= r * r
            f[inside] += val
    return f
