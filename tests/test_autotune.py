"""Autotuner search logic (host only): coordinate descent over tiling knobs."""

import pytest

pytest.importorskip("torch")


def test_coordinate_descent_finds_separable_minimum():
    from paper_1308_6634_amd.autotune import coordinate_descent
    knobs = {"a": (1, 2, 4, 8), "b": (4, 8, 16, 32, 64)}
    calls = []

    def cost(s):
        calls.append(dict(s))
        return (s["a"] - 2) ** 2 + (s["b"] - 16) ** 2 / 100.0

    best, log = coordinate_descent(knobs, cost, start={"a": 4, "b": 32})
    assert best == {"a": 2, "b": 16}
    # every distinct setting is measured once
    keys = [tuple(sorted(c.items())) for c in calls]
    assert len(keys) == len(set(keys)) == len(log)


def test_coordinate_descent_keeps_start_when_flat():
    from paper_1308_6634_amd.autotune import coordinate_descent
    best, _ = coordinate_descent({"k": (16, 32, 64)}, lambda s: 1.0, start={"k": 32})
    assert best == {"k": 32}


def test_apply_sets_only_the_interval():
    import gen
    from paper_1308_6634_amd.autotune import apply, knob_fields
    p = gen.config_c3(n=16, outer=1, inner=2)
    q = apply(p, {"cheb_lo": 0.25, "tune_blur_window": 16})
    assert q.cheb_lo == 0.25 and q.cheb_hi == p.cheb_hi and q.g is p.g
    assert knob_fields({"cheb_lo": 0.25, "tune_blur_window": 16}) == {"tune_blur_window": 16}


def test_vcycle_tuning_starts_at_the_defaults_and_drops_them():
    from paper_1308_6634_amd.autotune import VCYCLE_KNOBS, tune_vcycle
    seen = []

    def vcycle_ms(s):
        seen.append(dict(s))
        if s["tune_zm_v"] == 4:
            return 4.0 if s["tune_zm_zc"] == 16 else 6.0      # worse than the default alone
        return 5.0

    settings, report = tune_vcycle(vcycle_ms, repeats=1)
    # the first trial is the library's default schedule (every knob 0); the joint shape knob
    # finds four voxels per thread with 16-plane chunks although neither wins alone here
    assert seen[0] == {"tune_zm_v": 0, "tune_zm_zc": 0, "tune_tail_cells": 0, "tune_vcycle": 0}
    assert set(VCYCLE_KNOBS) == {"zm_shape", "tune_tail_cells", "tune_vcycle"}
    assert settings == {"tune_zm_v": 4, "tune_zm_zc": 16}      # zero (default) knobs left out
    assert len(report["vcycle_trials"]) == len(seen)
