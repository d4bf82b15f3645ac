"""Autotuner for the library's tiling knobs and the Chebyshev smoother interval.

Tiling knobs (``tune_gemv_rows``, ``tune_col_chunks``, ``tune_blur_window``) only change how
the kernels split their work; the autotuner times each candidate with short solves (first
outer iteration, a few inner iterations) through the C ABI and keeps the fastest, one knob
at a time (coordinate descent), using the HIP-event product timings the library reports.

The Chebyshev interval is a choice of the method (it changes the priorconditioner B and so
the iterates): candidates for its lower end are compared by the data residual
||g - A f^1|| after the same short solve (a better B reduces it faster at equal cost), ties
broken by time. The chosen interval is returned with the knobs and must be used by any
reference computation of the tuned problem.
"""

import dataclasses
import json

from . import plsqr as P

DENSE_KNOBS = {"tune_gemv_rows": (1, 2, 4, 8), "tune_col_chunks": (4, 8, 16, 32, 64)}
BLUR_KNOBS = {"tune_blur_window": (8, 16), "tune_blur_xgroups": (1, 2, 4)}
CHEB_LO = (1.0 / 8.0, 1.0 / 4.0, 1.0 / 3.0, 1.0 / 2.0)


def coordinate_descent(knobs, measure, start=None):
    """Minimise ``measure(settings)`` one knob at a time over the candidate values.

    ``knobs`` maps a knob name to its candidates; ``measure`` returns a cost (lower is
    better). Returns (best settings, list of (settings, cost) evaluated).
    """
    best = dict(start or {k: v[0] for k, v in knobs.items()})
    log = []
    cache = {}

    def cost(s):
        key = tuple(sorted(s.items()))
        if key not in cache:
            cache[key] = measure(dict(s))
            log.append((dict(s), cache[key]))
        return cache[key]

    best_cost = cost(best)
    for name, values in knobs.items():
        for v in values:
            trial = dict(best)
            trial[name] = v
            c = cost(trial)
            if c < best_cost:
                best, best_cost = trial, c
    return best, log


def _short(problem, inner):
    return dataclasses.replace(problem, outer=1, inner=inner)


def tune(problem, engine, inner=4, repeats=3, tune_cheb=True):
    """Return (settings dict, report dict) for a gen.Problem-like ``problem``."""
    import numpy as np
    import torch
    from .engine import problem_struct

    dev = engine.device
    if problem.op_kind == "dense":
        op = engine.dense_operator(tuple(problem.dims), problem.A)
        knobs = dict(DENSE_KNOBS)
    else:
        op = engine.blur_operator(tuple(problem.dims), problem.taps)
        knobs = dict(BLUR_KNOBS)
    g = torch.from_numpy(np.ascontiguousarray(problem.g, dtype=np.float32).ravel()).to(dev)
    f = torch.zeros(problem.n_x, dtype=torch.float32, device=dev)
    short = _short(problem, inner)

    def run(p, settings, flags):
        pb = problem_struct(p, flags=flags)
        for k, v in settings.items():
            setattr(pb, k, int(v))
        st, res = engine.wait(engine.submit(op, pb, g, f))
        if st != P.PLSQR_OK:
            raise P.PlsqrError(st, P.plsqr_last_error(engine.handle))
        return res

    def measure(settings):
        best = float("inf")
        for _ in range(repeats):
            res = run(short, settings, P.PLSQR_FLAG_TIME_PRODUCTS)
            best = min(best, res.forward_ms + res.adjoint_ms)
        return best

    settings, log = {}, []
    if knobs:
        start = {k: v[min(len(v) - 1, len(v) // 2)] for k, v in knobs.items()}
        settings, log = coordinate_descent(knobs, measure, start)
    report = {"knob_trials": [{"settings": s, "product_ms": c} for s, c in log]}

    if tune_cheb and problem.smoother == "chebyshev":
        trials = []
        for lo in CHEB_LO:
            p = dataclasses.replace(short, cheb_lo=lo)
            res = run(p, settings, 0)
            trials.append({"cheb_lo": lo, "resid": res.resid[0], "device_ms": res.device_ms})
        best = min(trials, key=lambda t: (round(t["resid"], 12), t["device_ms"]))
        settings["cheb_lo"] = best["cheb_lo"]
        report["cheb_trials"] = trials
    return settings, report


def apply(problem, settings):
    """The problem with a tuned (result-affecting) Chebyshev interval, if any."""
    if "cheb_lo" in settings:
        return dataclasses.replace(problem, cheb_lo=settings["cheb_lo"])
    return problem


def knob_fields(settings):
    return {k: v for k, v in settings.items() if k.startswith("tune_")}


def save(path, settings, report):
    with open(path, "w") as fh:
        json.dump({"settings": settings, "report": report}, fh, indent=1)
