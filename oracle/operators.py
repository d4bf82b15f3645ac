"""Forward maps A and their adjoints (the method only needs their action, Section 1).

* ``Blur``: separable correlation with 1D taps w_{-r..r} along every grid axis
  of extent > 1, zero outside the grid (same-size output):
  (A x)_j = sum_k w_k x_{j + k e_a}, one axis after another. The adjoint
  correlates with the reversed taps; for symmetric taps A = A^T.
* ``Dense``: an explicit matrix (n_Y x n_X) acting on the raveled grid.
"""

import numpy as np


def _correlate_axis(x, w, axis):
    r = (len(w) - 1) // 2
    n = x.shape[axis]
    out = np.zeros_like(x)
    for k in range(-r, r + 1):
        lo, hi = max(0, -k), min(n, n - k)      # output j with j + k inside [0, n)
        if hi <= lo:
            continue
        dst = [slice(None)] * x.ndim
        src = [slice(None)] * x.ndim
        dst[axis] = slice(lo, hi)
        src[axis] = slice(lo + k, hi + k)
        out[tuple(dst)] += w[k + r] * x[tuple(src)]
    return out


class Blur:
    def __init__(self, taps, shape):
        self.w = np.asarray(taps, dtype=np.float64)
        self.shape = tuple(shape)            # (nz, ny, nx)

    def _apply(self, x, w):
        y = np.asarray(x, dtype=np.float64).reshape(self.shape)
        for axis in (2, 1, 0):               # x, then y, then z
            if self.shape[axis] > 1:
                y = _correlate_axis(y, w, axis)
        return y

    def apply(self, x):
        return self._apply(x, self.w)

    def apply_T(self, y):
        return self._apply(y, self.w[::-1])


class Dense:
    def __init__(self, A, shape):
        self.A = np.asarray(A, dtype=np.float64)
        self.shape = tuple(shape)

    def apply(self, x):
        return self.A @ np.asarray(x, dtype=np.float64).ravel()

    def apply_T(self, y):
        return (self.A.T @ np.asarray(y, dtype=np.float64).ravel()).reshape(self.shape)
