"""Convenience layer over the C ABI: device buffers from torch, blocking waits.

Only marshalling and bookkeeping: every step of the method runs in ``libplsqr.so``.
"""

import time

import numpy as np
import torch

from . import plsqr as P


def problem_struct(p, flags=0, precision=P.PLSQR_PREC_FP32, knobs=None):
    """plsqr_problem from any object with the problem fields (dims, reg, T, tau, eps, outer,
    inner, levels, smoother, nu_pre, nu_post, omega, cheb_degree, cheb_lo, cheb_hi, and
    optionally the stop fields stop_s4, eta, delta, stop_outer, outer_rtol, outer_min);
    ``knobs`` sets tiling fields (tune_*)."""
    stop = 0
    if getattr(p, "stop_s4", False):
        stop |= P.PLSQR_FLAG_STOP_S4
    if getattr(p, "stop_outer", False):
        stop |= P.PLSQR_FLAG_STOP_OUTER
    pb = P.make_problem(tuple(p.dims), reg=p.reg, T=p.T, tau=p.tau, eps=p.eps, outer=p.outer,
                        inner=p.inner, levels=p.levels, smoother=p.smoother, nu_pre=p.nu_pre,
                        nu_post=p.nu_post, omega=p.omega, cheb_degree=p.cheb_degree,
                        cheb_lo=p.cheb_lo, cheb_hi=p.cheb_hi, precision=precision,
                        flags=flags | stop, eta=getattr(p, "eta", 1.1),
                        delta=getattr(p, "delta", 0.0), outer_rtol=getattr(p, "outer_rtol", 0.0),
                        outer_min=getattr(p, "outer_min", 3))
    for k, v in (knobs or {}).items():
        if k.startswith("tune_"):
            setattr(pb, k, int(v))
    return pb


class Engine:
    def __init__(self, device=0, hbm_budget_bytes=0, stream=None, flags=0):
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.handle = P.plsqr_create(device, hbm_budget_bytes, self.stream.cuda_stream, flags)
        self._keep = {}

    def close(self):
        if self.handle is not None:
            P.plsqr_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # operators -------------------------------------------------------------------
    def blur_operator(self, dims, taps):
        op_id = P.plsqr_set_operator(self.handle, P.blur_operator(dims, taps))
        return op_id

    def ring_operator(self, dims, src_xyz, det_xyz, mu):
        """Matrix-free ring sensitivity (entries recomputed in every product)."""
        return P.plsqr_set_operator(self.handle, P.ring_operator(dims, src_xyz, det_xyz, mu))

    def dense_operator(self, dims, A, A_hi=None, A_lo=None):
        """A: float32 (n_Y, n_X) numpy array or CUDA tensor (kept alive by the engine)."""
        if not torch.is_tensor(A):
            A = torch.from_numpy(np.ascontiguousarray(A, dtype=np.float32)).to(self.device)
        A = A.contiguous()
        op = P.dense_operator(dims, A.shape[0], A.data_ptr(),
                              None if A_hi is None else A_hi.data_ptr(),
                              None if A_lo is None else A_lo.data_ptr())
        op_id = P.plsqr_set_operator(self.handle, op)
        self._keep[("op", op_id)] = (A, A_hi, A_lo)
        return op_id

    # requests --------------------------------------------------------------------
    def submit(self, op_id, prob, g, f):
        """g, f: contiguous float32 CUDA tensors (borrowed until the request completes)."""
        assert g.dtype == torch.float32 and f.dtype == torch.float32
        assert g.is_cuda and f.is_cuda and g.is_contiguous() and f.is_contiguous()
        t = P.plsqr_solve(self.handle, op_id, prob, g.data_ptr(), f.data_ptr())
        self._keep[("req", t)] = (g, f)
        return t

    def submit_taus(self, op_id, prob, g, f, taus, f_taus):
        """One request plus f for every damping in taus (Section 3.3); f_taus: contiguous
        float32 CUDA tensor of len(taus) x n_X."""
        for x in (g, f, f_taus):
            assert x.dtype == torch.float32 and x.is_cuda and x.is_contiguous()
        t = P.plsqr_solve_taus(self.handle, op_id, prob, g.data_ptr(), f.data_ptr(), list(taus),
                               f_taus.data_ptr())
        self._keep[("req", t)] = (g, f, f_taus)
        return t

    def submit_batch(self, op_id, probs, gs, fs):
        """Lockstep batch; returns one ticket per instance."""
        for g, f in zip(gs, fs):
            assert g.dtype == torch.float32 and f.dtype == torch.float32
            assert g.is_cuda and f.is_cuda and g.is_contiguous() and f.is_contiguous()
        ts = P.plsqr_solve_batch(self.handle, op_id, probs, [g.data_ptr() for g in gs],
                                 [f.data_ptr() for f in fs])
        for t, g, f in zip(ts, gs, fs):
            self._keep[("req", t)] = (g, f)
        return ts

    def poll(self, ticket):
        st, res = P.plsqr_poll(self.handle, ticket)
        if st != P.PLSQR_PENDING:
            self._keep.pop(("req", ticket), None)
        return st, res

    def wait(self, ticket, timeout_s=600.0, sleep_s=0.0005):
        t0 = time.time()
        while True:
            st, res = self.poll(ticket)
            if st != P.PLSQR_PENDING:
                return st, res
            if time.time() - t0 > timeout_s:
                raise TimeoutError(f"request {ticket} not finished after {timeout_s} s")
            time.sleep(sleep_s)

    def wait_all(self):
        P.plsqr_wait_all(self.handle)


def solve(problem, device=0, flags=0, engine=None, knobs=None, matrix_free=False):
    """Run one problem (a gen.Problem-like object) and return (f as numpy, plsqr_result).
    ``knobs``: tiling fields (tune_*) for the problem struct; ``matrix_free``: apply a dense
    ring sensitivity through its geometry (problem.extra["ring"]) instead of the matrix."""
    own = engine is None
    eng = engine or Engine(device)
    try:
        dev = eng.device
        if problem.op_kind == "blur":
            op_id = eng.blur_operator(tuple(problem.dims), problem.taps)
        elif matrix_free:
            op_id = eng.ring_operator(tuple(problem.dims), *problem.extra["ring"])
        else:
            op_id = eng.dense_operator(tuple(problem.dims), problem.A)
        g = torch.from_numpy(np.ascontiguousarray(problem.g, dtype=np.float32).ravel()).to(dev)
        f = torch.zeros(problem.n_x, dtype=torch.float32, device=dev)
        t = eng.submit(op_id, problem_struct(problem, flags=flags, knobs=knobs), g, f)
        st, res = eng.wait(t)
        if st != P.PLSQR_OK:
            raise P.PlsqrError(st, P.plsqr_last_error(eng.handle))
        nx, ny, nz = problem.dims
        return f.cpu().numpy().reshape(nz, ny, nx), res
    finally:
        if own:
            eng.close()
