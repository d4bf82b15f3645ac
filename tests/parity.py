"""Parity bars shared by the GPU tests (HIP path against the FP64 oracle).

Two bars at the same tolerance ``tol`` (1e-3 for the float32 path, 5e-3 for BF16 products with
refinement):
* relative L2 over the whole grid, ||f - f_ref|| / ||f_ref|| <= tol;
* element-wise, max |f - f_ref| <= tol * max |f_ref|, so that an error confined to a few
  voxels (a wrong edge line or face of a tile) cannot hide inside a small L2 norm.
"""

import numpy as np


def rel_l2(a, b):
    a = np.asarray(a, float).ravel()
    b = np.asarray(b, float).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def max_rel(a, b):
    a = np.asarray(a, float).ravel()
    b = np.asarray(b, float).ravel()
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def assert_parity(f, f_ref, tol, what=""):
    """Both bars; returns the relative L2 error."""
    f = np.asarray(f, float)
    assert np.all(np.isfinite(f)), what
    err, emax = rel_l2(f, f_ref), max_rel(f, f_ref)
    assert err <= tol, (what, "rel L2", err)
    assert emax <= tol, (what, "max element", emax)
    return err
