"""ctypes binding of ``libplsqr.so`` (argument marshalling only).

The functions carry the C names and follow the C ABI of ``include/plsqr.h``. Calls that
fail with a negative status raise ``PlsqrError``; ``plsqr_poll`` returns the status of a
finished request (it only raises for an unknown ticket or a bad engine). Device memory
and streams come from PyTorch: pass ``tensor.data_ptr()`` and
``torch.cuda.current_stream().cuda_stream``.

Importing this module loads the library and fails loudly if it is missing: there is no
fallback implementation.
"""

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime the library then shares with torch)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libplsqr.so")

PLSQR_OK = 0
PLSQR_PENDING = 1
PLSQR_E_INVALID = -1
PLSQR_E_NOMEM = -2
PLSQR_E_BUDGET = -3
PLSQR_E_HIP = -4
PLSQR_E_NOT_SPD = -5
PLSQR_E_NONFINITE = -6
PLSQR_E_UNKNOWN_TICKET = -7

PLSQR_OP_BLUR = 1
PLSQR_OP_DENSE = 2
PLSQR_OP_RING = 3
PLSQR_REG_TIKHONOV, PLSQR_REG_STV, PLSQR_REG_PM_LOG, PLSQR_REG_PM_EXP = 0, 1, 2, 3
PLSQR_SMOOTH_JACOBI, PLSQR_SMOOTH_CHEBYSHEV = 0, 1
PLSQR_VCYCLE_FUSED, PLSQR_VCYCLE_PER_SWEEP = 0, 1
PLSQR_UPDATE_AUTO, PLSQR_UPDATE_PRODUCT, PLSQR_UPDATE_TAIL = 0, 1, 2
PLSQR_PREC_FP32, PLSQR_PREC_BF16_REFINED, PLSQR_PREC_BF16 = 0, 1, 2
PLSQR_ENGINE_SERVE = 1
PLSQR_FLAG_TIME_PRODUCTS = 1
PLSQR_FLAG_NO_GRAPHS = 2
PLSQR_FLAG_STOP_S4 = 4
PLSQR_FLAG_STOP_OUTER = 8
PLSQR_STATIC_SCRATCH_BYTES = 64 << 20
PLSQR_FLAG_TIME_PHASES = 16
PLSQR_MAX_LEVELS = 12
PLSQR_MAX_OUTER = 64
PLSQR_MAX_RADIUS = 16
PLSQR_MAX_COARSE = 512

REG_CODES = {"tikhonov": PLSQR_REG_TIKHONOV, "stv": PLSQR_REG_STV, "pm_log": PLSQR_REG_PM_LOG,
             "pm_exp": PLSQR_REG_PM_EXP}
SMOOTHER_CODES = {"jacobi": PLSQR_SMOOTH_JACOBI, "chebyshev": PLSQR_SMOOTH_CHEBYSHEV}

EXPORTED = ("plsqr_create", "plsqr_set_operator", "plsqr_solve", "plsqr_solve_batch", "plsqr_poll",
            "plsqr_solve_taus", "plsqr_solve_static",
            "plsqr_wait_all",
            "plsqr_destroy", "plsqr_last_error", "plsqr_auto_levels", "plsqr_workspace_bytes")


class plsqr_operator(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("radius", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("taps", ctypes.POINTER(ctypes.c_float)), ("n_y", ctypes.c_int64),
                ("A_dev", ctypes.c_void_p), ("A_hi_dev", ctypes.c_void_p),
                ("A_lo_dev", ctypes.c_void_p), ("n_src", ctypes.c_int32), ("n_det", ctypes.c_int32),
                ("src_xyz", ctypes.POINTER(ctypes.c_float)),
                ("det_xyz", ctypes.POINTER(ctypes.c_float)), ("mu", ctypes.c_double)]


class plsqr_problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("reg", ctypes.c_int32), ("T", ctypes.c_double), ("tau", ctypes.c_double),
                ("eps", ctypes.c_double), ("outer", ctypes.c_int32), ("inner", ctypes.c_int32),
                ("mg_levels", ctypes.c_int32), ("smoother", ctypes.c_int32),
                ("nu_pre", ctypes.c_int32), ("nu_post", ctypes.c_int32), ("omega", ctypes.c_double),
                ("cheb_degree", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("cheb_lo", ctypes.c_double), ("cheb_hi", ctypes.c_double),
                ("flags", ctypes.c_uint32), ("tune_gemv_rows", ctypes.c_int32),
                ("tune_col_chunks", ctypes.c_int32),
                ("eta", ctypes.c_double), ("delta", ctypes.c_double),
                ("outer_rtol", ctypes.c_double), ("outer_min", ctypes.c_int32),
                ("tune_blur_window", ctypes.c_int32), ("tune_blur_xgroups", ctypes.c_int32),
                ("tune_vcycle", ctypes.c_int32), ("tune_zm_ty", ctypes.c_int32),
                ("tune_zm_zc", ctypes.c_int32), ("tune_zm_v", ctypes.c_int32),
                ("tune_tail_cells", ctypes.c_int32), ("tune_update_site", ctypes.c_int32)]


class plsqr_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("outer_done", ctypes.c_int32),
                ("levels", ctypes.c_int32), ("mixed_steps", ctypes.c_int32),
                ("inner_done", ctypes.c_int32 * PLSQR_MAX_OUTER),
                ("resid", ctypes.c_double * PLSQR_MAX_OUTER),
                ("penalty", ctypes.c_double * PLSQR_MAX_OUTER),
                ("submit_to_done_ms", ctypes.c_double), ("device_ms", ctypes.c_double),
                ("forward_ms", ctypes.c_double), ("forward_launches", ctypes.c_int64),
                ("adjoint_ms", ctypes.c_double), ("adjoint_launches", ctypes.c_int64),
                ("workspace_bytes", ctypes.c_int64),
                ("setup_ms", ctypes.c_double), ("vcycle_ms", ctypes.c_double),
                ("update_ms", ctypes.c_double), ("diag_ms", ctypes.c_double),
                ("phase_launches", ctypes.c_int64)]


class PlsqrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"plsqr error {code}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1308_6634_amd.build` "
                          "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    lib.plsqr_create.argtypes = [P(ctypes.c_void_p), ctypes.c_int, ctypes.c_uint64, ctypes.c_void_p,
                                 ctypes.c_uint32]
    lib.plsqr_set_operator.argtypes = [ctypes.c_void_p, P(plsqr_operator), P(ctypes.c_int32)]
    lib.plsqr_solve.argtypes = [ctypes.c_void_p, ctypes.c_int32, P(plsqr_problem), ctypes.c_void_p,
                                ctypes.c_void_p, P(ctypes.c_uint64)]
    lib.plsqr_solve_taus.argtypes = [ctypes.c_void_p, ctypes.c_int32, P(plsqr_problem),
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                     P(ctypes.c_double), ctypes.c_void_p, P(ctypes.c_uint64)]
    lib.plsqr_solve_batch.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                      P(plsqr_problem), P(ctypes.c_void_p), P(ctypes.c_void_p),
                                      P(ctypes.c_uint64)]
    lib.plsqr_solve_static.argtypes = [ctypes.c_void_p, ctypes.c_int32, P(plsqr_problem),
                                       ctypes.c_void_p, ctypes.c_void_p, P(plsqr_result)]
    lib.plsqr_poll.argtypes = [ctypes.c_void_p, ctypes.c_uint64, P(plsqr_result)]
    lib.plsqr_wait_all.argtypes = [ctypes.c_void_p]
    lib.plsqr_destroy.argtypes = [ctypes.c_void_p]
    lib.plsqr_last_error.argtypes = [ctypes.c_void_p]
    lib.plsqr_last_error.restype = ctypes.c_char_p
    lib.plsqr_auto_levels.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    lib.plsqr_workspace_bytes.argtypes = [P(plsqr_problem), ctypes.c_int32, ctypes.c_int64]
    lib.plsqr_workspace_bytes.restype = ctypes.c_uint64
    for name in EXPORTED:
        getattr(lib, name).restype = getattr(lib, name).restype or ctypes.c_int
    return lib


_lib = _load()


def _check(rc, eng=None):
    if rc < 0:
        raise PlsqrError(rc, _lib.plsqr_last_error(eng).decode())
    return rc


def plsqr_create(device=0, hbm_budget_bytes=0, hip_stream=None, flags=0):
    eng = ctypes.c_void_p()
    _check(_lib.plsqr_create(ctypes.byref(eng), device, hbm_budget_bytes, hip_stream, flags))
    return eng


def plsqr_set_operator(eng, op):
    op_id = ctypes.c_int32()
    _check(_lib.plsqr_set_operator(eng, ctypes.byref(op), ctypes.byref(op_id)), eng)
    return op_id.value


def plsqr_solve(eng, op_id, prob, g_dev, f_dev):
    ticket = ctypes.c_uint64()
    _check(_lib.plsqr_solve(eng, op_id, ctypes.byref(prob), g_dev, f_dev, ctypes.byref(ticket)), eng)
    return ticket.value


def plsqr_solve_taus(eng, op_id, prob, g_dev, f_dev, taus, f_taus_dev):
    n = len(taus)
    arr = (ctypes.c_double * n)(*[float(t) for t in taus])
    ticket = ctypes.c_uint64()
    _check(_lib.plsqr_solve_taus(eng, op_id, ctypes.byref(prob), g_dev, f_dev, n, arr, f_taus_dev,
                                 ctypes.byref(ticket)), eng)
    return ticket.value


def plsqr_solve_batch(eng, op_id, probs, g_devs, f_devs):
    n = len(probs)
    arr = (plsqr_problem * n)(*probs)
    gs = (ctypes.c_void_p * n)(*g_devs)
    fs = (ctypes.c_void_p * n)(*f_devs)
    tickets = (ctypes.c_uint64 * n)()
    _check(_lib.plsqr_solve_batch(eng, op_id, n, arr, gs, fs, tickets), eng)
    return list(tickets)


def plsqr_solve_static(eng, op_id, prob, g_dev, f_dev, want_result=True):
    """The no-allocation entry point. With want_result, waits and returns (status, result);
    otherwise returns (PLSQR_OK, None) once the work is enqueued. Argument errors raise; a
    request that fails on the device returns its status."""
    res = plsqr_result() if want_result else None
    rc = _lib.plsqr_solve_static(eng, op_id, ctypes.byref(prob), g_dev, f_dev,
                                 ctypes.byref(res) if want_result else None)
    if rc < 0 and (res is None or res.status != rc):
        _check(rc, eng)
    return rc, res


def plsqr_poll(eng, ticket):
    """Returns (status, plsqr_result or None). status is PLSQR_PENDING, PLSQR_OK or a
    request error; an unknown ticket raises."""
    res = plsqr_result()
    rc = _lib.plsqr_poll(eng, ticket, ctypes.byref(res))
    if rc in (PLSQR_E_UNKNOWN_TICKET, PLSQR_E_INVALID):
        _check(rc, eng)
    return rc, (None if rc == PLSQR_PENDING else res)


def plsqr_wait_all(eng):
    return _check(_lib.plsqr_wait_all(eng), eng)


def plsqr_destroy(eng):
    return _check(_lib.plsqr_destroy(eng))


def plsqr_last_error(eng=None):
    return _lib.plsqr_last_error(eng).decode()


def plsqr_auto_levels(nx, ny, nz):
    return _lib.plsqr_auto_levels(nx, ny, nz)


def plsqr_workspace_bytes(prob, op_kind, n_y):
    return _lib.plsqr_workspace_bytes(ctypes.byref(prob), op_kind, n_y)


# ---- marshalling helpers -----------------------------------------------------------

def blur_operator(dims, taps):
    """plsqr_operator for a separable blur on dims = (nx, ny, nz); taps is a float32 array."""
    import numpy as np
    t = np.ascontiguousarray(taps, dtype=np.float32)
    op = plsqr_operator()
    op.kind = PLSQR_OP_BLUR
    op.nx, op.ny, op.nz = dims
    op.radius = (len(t) - 1) // 2
    op.taps = t.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    op._keep = t
    return op


def dense_operator(dims, n_y, A_dev, A_hi_dev=None, A_lo_dev=None):
    op = plsqr_operator()
    op.kind = PLSQR_OP_DENSE
    op.nx, op.ny, op.nz = dims
    op.n_y = n_y
    op.A_dev = A_dev
    op.A_hi_dev = A_hi_dev
    op.A_lo_dev = A_lo_dev
    return op


def ring_operator(dims, src_xyz, det_xyz, mu):
    """plsqr_operator for the matrix-free ring sensitivity: src_xyz (n_src, 3) and det_xyz
    (n_det, 3) positions in voxel units, attenuation mu."""
    import numpy as np
    s = np.ascontiguousarray(src_xyz, dtype=np.float32).reshape(-1, 3)
    d = np.ascontiguousarray(det_xyz, dtype=np.float32).reshape(-1, 3)
    op = plsqr_operator()
    op.kind = PLSQR_OP_RING
    op.nx, op.ny, op.nz = dims
    op.n_src, op.n_det = s.shape[0], d.shape[0]
    op.n_y = s.shape[0] * d.shape[0]
    op.src_xyz = s.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    op.det_xyz = d.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    op.mu = float(mu)
    op._keep = (s, d)
    return op


def make_problem(dims, reg="stv", T=0.01, tau=1.0, eps=1e-6, outer=1, inner=1, levels=0,
                 smoother="jacobi", nu_pre=2, nu_post=2, omega=0.8, cheb_degree=3,
                 cheb_lo=1.0 / 3.0, cheb_hi=2.0, precision=PLSQR_PREC_FP32, flags=0,
                 eta=1.1, delta=0.0, outer_rtol=0.0, outer_min=3):
    """plsqr_problem; the stop parameters matter only with PLSQR_FLAG_STOP_S4 (eta, delta)
    and PLSQR_FLAG_STOP_OUTER (outer_rtol, outer_min)."""
    pb = plsqr_problem()
    pb.nx, pb.ny, pb.nz = dims
    pb.reg = REG_CODES[reg] if isinstance(reg, str) else int(reg)
    pb.T, pb.tau, pb.eps = T, tau, eps
    pb.outer, pb.inner, pb.mg_levels = outer, inner, levels
    pb.smoother = SMOOTHER_CODES[smoother] if isinstance(smoother, str) else int(smoother)
    pb.nu_pre, pb.nu_post, pb.omega = nu_pre, nu_post, omega
    pb.cheb_degree, pb.cheb_lo, pb.cheb_hi = cheb_degree, cheb_lo, cheb_hi
    pb.precision, pb.flags = precision, flags
    pb.eta, pb.delta, pb.outer_rtol, pb.outer_min = eta, delta, outer_rtol, outer_min
    return pb
