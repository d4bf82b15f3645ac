"""Forward-operator definitions and noisy data.

* Gaussian blur: 1D taps w_k proportional to exp(-k^2 / (2 sigma^2)), |k| <= radius,
  normalised to sum 1 and rounded to float32; 2D/3D blurs are tensor products
  with zero padding (same-size output). These are the operator's definition;
  the solver applies them itself.
* Dense sensitivity: A[s*n_det + d, j] = exp(-mu (d_sj + d_dj)) / (d_sj d_dj + 1)
  with d_sj, d_dj the Euclidean distances from voxel centre j to source s and
  detector d, which sit on rings around the volume on the square side walls
  x, y in {-0.5, n-0.5}. This stands in for the fDOT sensitivity of Section 5.1
  (sources and detectors on rings around the object, Section 5.2); the kernel
  formula and the ring layout are this project's synthetic choice.

Data g = A f_true + noise is formed in float64 with library routines
(``scipy.ndimage.correlate1d`` for the blur, a BLAS product for dense A) and
rounded to float32.
"""

import concurrent.futures as _cf
import math

import numpy as np
from scipy import ndimage


def gaussian_taps(sigma, radius):
    k = np.arange(-radius, radius + 1, dtype=np.float64)
    w = np.exp(-(k * k) / (2.0 * sigma * sigma))
    w /= w.sum()
    return w.astype(np.float32)


def _perimeter_point(s, n):
    """Point at arc length s on the square wall [-0.5, n-0.5]^2, counter-clockwise from (-0.5,-0.5)."""
    lo, side = -0.5, float(n)
    s = s % (4.0 * side)
    if s < side:
        return lo + s, lo
    if s < 2 * side:
        return lo + side, lo + (s - side)
    if s < 3 * side:
        return lo + side - (s - 2 * side), lo + side
    return lo, lo + side - (s - 3 * side)


def ring_geometry(n, src_rings, det_rings, per_ring=16):
    """Source and detector positions (x, y, z) for rings of ``per_ring`` points.

    ``src_rings`` / ``det_rings`` list the ring heights z. Along each ring,
    with spacing = 4n/per_ring, sources sit at arc length spacing*k + spacing/4
    and detectors at spacing*k + 3*spacing/4 (for n = 64: 16k+4 and 16k+12).
    """
    spacing = 4.0 * n / per_ring
    src, det = [], []
    for z in src_rings:
        for k in range(per_ring):
            x, y = _perimeter_point(spacing * k + spacing / 4.0, n)
            src.append((x, y, float(z)))
    for z in det_rings:
        for k in range(per_ring):
            x, y = _perimeter_point(spacing * k + 3.0 * spacing / 4.0, n)
            det.append((x, y, float(z)))
    return np.array(src), np.array(det)


def default_rings(n, n_src_rings=4, n_det_rings=4):
    """Ring heights: k rings evenly spaced, z = (n/k) r + n/(2k) - 0.5."""
    src = [(n / n_src_rings) * r + n / (2.0 * n_src_rings) - 0.5 for r in range(n_src_rings)]
    det = [(n / n_det_rings) * r + n / (2.0 * n_det_rings) - 0.5 for r in range(n_det_rings)]
    return src, det


def _voxel_distances(points, n):
    z, y, x = np.meshgrid(np.arange(n, dtype=np.float64), np.arange(n, dtype=np.float64),
                          np.arange(n, dtype=np.float64), indexing="ij")
    x, y, z = x.ravel(), y.ravel(), z.ravel()
    out = np.empty((len(points), n * n * n))
    for i, (px, py, pz) in enumerate(points):
        out[i] = np.sqrt((x - px) ** 2 + (y - py) ** 2 + (z - pz) ** 2)
    return out


def ring_points(n, n_src_rings=4, n_det_rings=4, per_ring=16):
    """Source and detector positions of the default ring layout."""
    src_z, det_z = default_rings(n, n_src_rings, n_det_rings)
    return ring_geometry(n, src_z, det_z, per_ring)


def dense_sensitivity(n, mu=0.5, n_src_rings=4, n_det_rings=4, per_ring=16, threads=8):
    """Row-major float32 matrix of shape (n_src*n_det, n^3); row index = s*n_det + d."""
    src, det = ring_points(n, n_src_rings, n_det_rings, per_ring)
    ds = _voxel_distances(src, n)
    dd = _voxel_distances(det, n)
    es, ed = np.exp(-mu * ds), np.exp(-mu * dd)
    n_s, n_d, n_x = len(src), len(det), n ** 3
    A = np.empty((n_s * n_d, n_x), dtype=np.float32)

    def fill(s):
        num = es[s][None, :] * ed
        den = ds[s][None, :] * dd + 1.0
        A[s * n_d:(s + 1) * n_d] = (num / den).astype(np.float32)

    with _cf.ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        list(ex.map(fill, range(n_s)))
    return A


def add_noise(rng, clean, noise_frac):
    """Returns (float32 data, noise standard deviation, Euclidean norm of the drawn noise)."""
    sd = noise_frac * float(np.max(np.abs(clean)))
    e = rng.normal(0.0, sd, size=clean.shape)
    return (clean + e).astype(np.float32), sd, float(np.linalg.norm(e))


def blur_data(rng, f_true, taps, noise_frac):
    """g = blur(f_true) + N(0, (noise_frac * max|blur f|)^2), float32, same shape as f_true;
    returns (g, noise sd, noise norm)."""
    w = np.asarray(taps, dtype=np.float64)
    clean = np.asarray(f_true, dtype=np.float64)
    for ax in range(3):
        if clean.shape[ax] > 1:
            clean = ndimage.correlate1d(clean, w, axis=ax, mode="constant", cval=0.0)
    return add_noise(rng, clean, noise_frac)


def dense_data(rng, A, f_true, noise_frac, chunk=512):
    """g = A f_true + noise (float32, length n_Y), A given as float32 rows."""
    x = np.asarray(f_true, dtype=np.float64).ravel()
    clean = np.empty(A.shape[0])
    for r0 in range(0, A.shape[0], chunk):
        clean[r0:r0 + chunk] = A[r0:r0 + chunk].astype(np.float64) @ x
    return add_noise(rng, clean, noise_frac)


def radius_for_sigma(sigma):
    return int(math.ceil(3.0 * sigma))
