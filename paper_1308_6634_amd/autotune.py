"""Autotuner for the library's tiling knobs, the V-cycle launch schedule and the Chebyshev
smoother interval.

Tiling knobs (``tune_gemv_rows``, ``tune_col_chunks``, ``tune_blur_window``) only change how
the kernels split their work; the autotuner times each candidate with short solves (first
outer iteration, a few inner iterations) through the C ABI and keeps the fastest, one knob
at a time (coordinate descent), using the HIP-event product timings the library reports.

The V-cycle knobs (``tune_vcycle``: fused level kernels or one launch per sweep,
``tune_zm_v``: voxels per thread of the fused kernels, ``tune_zm_zc``: planes per block,
``tune_tail_cells``: the largest level of the one-workgroup tail) are chosen the same way by
the V-cycle phase time (PLSQR_FLAG_TIME_PHASES), on the request or on the whole lockstep batch
it will run in, since a batch fills the chip differently from one instance. They change only the
order in which the alpha = sqrt(v . p) partial sums are added.

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
# V-cycle knobs, the library default first (0 = chosen per level). Voxels per thread and planes
# per block are searched jointly (one favours the other: four voxels per thread pay off with
# deep plane chunks), as one knob whose values are (tune_zm_v, tune_zm_zc) pairs.
VCYCLE_SHAPES = tuple((v, zc) for v in (0, 4, 1) for zc in (0, 16, 8, 4))
VCYCLE_KNOBS = {"zm_shape": VCYCLE_SHAPES, "tune_tail_cells": (0, 512), "tune_vcycle": (0, 1)}


def _expand(settings):
    out = {k: v for k, v in settings.items() if k != "zm_shape"}
    if "zm_shape" in settings:
        out["tune_zm_v"], out["tune_zm_zc"] = settings["zm_shape"]
    return out


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


def tune(problem, engine, inner=4, repeats=3, tune_cheb=True, tune_vcycle_knobs=True):
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

    if tune_vcycle_knobs:
        def vcycle_ms(vs):
            res = run(short, {**settings, **vs}, P.PLSQR_FLAG_TIME_PHASES)
            return res.vcycle_ms
        vs, vrep = tune_vcycle(vcycle_ms)
        settings.update(vs)
        report.update(vrep)

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


def tune_vcycle(run_vcycle_ms, knobs=None, repeats=2):
    """Coordinate descent over the V-cycle knobs. ``run_vcycle_ms(settings)`` runs a short solve
    (one request or a whole batch) with PLSQR_FLAG_TIME_PHASES and the given tune_* settings
    and returns its V-cycle phase time. Returns (settings, report)."""
    knobs = knobs or VCYCLE_KNOBS

    def measure(settings):
        s = _expand(settings)
        return min(run_vcycle_ms(s) for _ in range(repeats))

    start = {k: v[0] for k, v in knobs.items()}
    settings, log = coordinate_descent(knobs, measure, start)
    settings = {k: v for k, v in _expand(settings).items() if v}
    return settings, {"vcycle_trials": [{"settings": _expand(s), "vcycle_ms": c} for s, c in log]}


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
