"""Seeded input generators: determinism, shapes, value ranges, operator definitions."""

import math

import numpy as np
import pytest

import gen
from gen import operators as gops


def test_taps_normalised_symmetric():
    w = gen.gaussian_taps(2.0, 4)
    assert w.dtype == np.float32 and len(w) == 9
    assert abs(float(w.astype(np.float64).sum()) - 1.0) < 1e-6
    np.testing.assert_array_equal(w, w[::-1])
    assert w[4] == w.max()


def test_ring_geometry_n64():
    src, det = gops.ring_geometry(64, [7.5], [7.5])
    # first source at arc length 4 on the y = -0.5 wall, first detector at 12
    assert tuple(src[0]) == (3.5, -0.5, 7.5)
    assert tuple(det[0]) == (11.5, -0.5, 7.5)
    assert len(src) == 16 and len(det) == 16
    assert np.all((np.abs(src[:, 0] + 0.5) < 1e-12) | (np.abs(src[:, 0] - 63.5) < 1e-12)
                  | (np.abs(src[:, 1] + 0.5) < 1e-12) | (np.abs(src[:, 1] - 63.5) < 1e-12))


def test_dense_entries_match_formula():
    n, mu = 6, 0.7
    A = gen.dense_sensitivity(n, mu=mu, n_src_rings=2, n_det_rings=2, per_ring=4)
    src_z, det_z = gops.default_rings(n, 2, 2)
    src, det = gops.ring_geometry(n, src_z, det_z, 4)
    assert A.shape == (len(src) * len(det), n ** 3)
    rng = np.random.default_rng(0)
    for _ in range(50):
        s, d, j = rng.integers(len(src)), rng.integers(len(det)), rng.integers(n ** 3)
        x, y, z = j % n, (j // n) % n, j // (n * n)
        ds = math.dist((x, y, z), src[s])
        dd = math.dist((x, y, z), det[d])
        ref = math.exp(-mu * (ds + dd)) / (ds * dd + 1.0)
        assert A[s * len(det) + d, j] == pytest.approx(ref, rel=1e-6)


def test_configs_deterministic_and_shaped():
    a, b = gen.config_c1(), gen.config_c1()
    np.testing.assert_array_equal(a.g, b.g)
    np.testing.assert_array_equal(a.f_true, b.f_true)
    assert a.g.shape == (1, 64, 64) and a.g.dtype == np.float32
    assert a.levels == 4 and a.outer == 10 and a.inner == 50
    c = gen.config_c1(seed=1)
    assert not np.array_equal(a.g, c.g)
    assert 0.0 <= a.f_true.min() and a.f_true.max() > 0.0


def test_auto_levels_rule():
    assert [gen.auto_levels((n, n, n)) for n in (32, 48, 64, 96, 128)] == [4, 5, 5, 6, 6]
    assert gen.auto_levels((64, 64, 1)) == 5
    assert gen.auto_levels((6, 6, 6)) == 2 and gen.auto_levels((5, 8, 8)) == 1


def test_small_cases_and_noise_level():
    p = gen.small_blur_case(1, (16, 12, 8))
    assert p.g.shape == (8, 12, 16) and p.f_true.shape == (8, 12, 16)
    d = gen.small_dense_case(2, 8)
    assert d.A.shape == (32 * 32, 512) and d.g.shape == (1024,)
    assert d.noise_sd > 0.0


def test_c5_requests_and_arrivals():
    t = gen.config_c5_requests(count=200)
    assert t[0] == 0.0 and np.all(np.diff(t) >= 0.0)
    assert 0.01 < np.mean(np.diff(t)) < 0.03
    r = gen.configs.c5_request(3, sizes=(32,))
    assert r.dims == (32, 32, 32) and r.levels == 4
    assert r.radius == math.ceil(3 * r.extra["sigma"]) and 1.5 <= r.extra["sigma"] <= 3.5


def test_c4_batch_generator_equals_one_at_a_time():
    """The batched family's generator that forms every instance's clean data in one pass over A
    gives the same instances as the one-at-a-time recipe (same seeds and draw order)."""
    from gen import operators as ops
    from gen.configs import config_c4, config_c4_batch
    A = ops.dense_sensitivity(8, mu=4.0, n_src_rings=8, n_det_rings=4)
    one = [config_c4(i, A, n=8) for i in range(6)]
    many = config_c4_batch(A, 6, n=8)
    for a, b in zip(one, many):
        assert (a.reg, a.T, a.tau, a.levels) == (b.reg, b.T, b.tau, b.levels)
        np.testing.assert_array_equal(a.f_true, b.f_true)
        np.testing.assert_array_equal(a.g, b.g)
        assert a.delta == pytest.approx(b.delta, rel=1e-12)
