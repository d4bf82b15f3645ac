"""GPU parity of the matrix-free ring sensitivity (PLSQR_OP_RING): the same reconstructions as
with the stored dense matrix, where every product regenerates the entries from the source and
detector positions.

References: the FP64 oracle with the dense matrix (from the generators, or built here entry by
entry from the formula exp(-mu (r_s + r_d)) / (r_s r_d + 1)), and the GPU's stored-matrix path.
Bar: relative L2 <= 1e-3 against the oracle (FP32 vectors; the regenerated entries carry the
hardware exponential / reciprocal / square-root rounding, ~1e-6 relative).
"""

import math
import sys

import numpy as np
import pytest

import gen
from oracle import lagged
from parity import assert_parity

pytestmark = pytest.mark.gpu

TOL = 1e-3


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def engine():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1308_6634_amd.engine import Engine
    eng = Engine(0)
    yield eng
    eng.close()


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, float) - np.asarray(b, float)) /
                 max(np.linalg.norm(np.asarray(b, float)), 1e-300))


def _entrywise_matrix(dims, src, det, mu):
    """The sensitivity written out entry by entry in FP64 (voxel centres at integer
    coordinates, x fastest; row s * n_det + d)."""
    nx, ny, nz = dims
    A = np.empty((len(src) * len(det), nx * ny * nz))
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                j = x + nx * (y + ny * z)
                for s, ps in enumerate(src):
                    rs = math.dist((x, y, z), ps)
                    for d, pd in enumerate(det):
                        rd = math.dist((x, y, z), pd)
                        A[s * len(det) + d, j] = math.exp(-mu * (rs + rd)) / (rs * rd + 1.0)
    return A


@pytest.mark.parametrize("n,reg", [(8, "pm_log"), (16, "stv")])
def test_ring_matches_oracle_and_stored_matrix(engine, n, reg):
    from paper_1308_6634_amd.engine import solve
    p = gen.small_dense_case(40 + n, n, reg=reg, outer=3, inner=10)
    _say(f"[ring] {p.name} n_y={p.A.shape[0]} {p.outer}x{p.inner}")
    f_ring, res = solve(p, engine=engine, matrix_free=True)
    f_ref, rec = lagged.solve_problem(p)
    err = assert_parity(f_ring, f_ref, TOL, p.name)
    f_dense, _ = solve(p, engine=engine)
    diff = _rel(f_ring, f_dense)
    _say(f"[ring] {p.name}: rel L2 vs oracle {err:.3e}, vs stored matrix {diff:.3e}")
    assert diff <= 1e-4
    for k, r in enumerate(rec):
        assert abs(res.resid[k] - r["resid"]) <= TOL * r["resid"]


def test_ring_irregular_counts_against_entrywise_matrix(engine):
    """5 sources x 7 detectors (tiles and register groups partly empty) around an 8 x 6 x 4
    grid, positions drawn at random outside the box; the oracle's matrix is built entry by
    entry from the formula."""
    from paper_1308_6634_amd.engine import solve
    rng = np.random.default_rng(77)
    dims = (8, 6, 4)
    src = rng.uniform(-3.0, 11.0, size=(5, 3))
    det = rng.uniform(-3.0, 11.0, size=(7, 3))
    mu = 0.3
    A = _entrywise_matrix(dims, src, det, mu)
    f_true = np.zeros((4, 6, 8))
    f_true[1:3, 2:5, 2:6] = 1.0
    g = A @ f_true.ravel()
    g = (g + rng.normal(0.0, 0.01 * np.abs(g).max(), size=g.shape)).astype(np.float32)
    p = gen.Problem(name="ring_irregular", dims=dims, f_true=f_true, g=g, op_kind="dense",
                    A=A.astype(np.float32), reg="pm_log", T=0.05, tau=2.0, eps=1e-2, outer=2,
                    inner=8, levels=2, extra={"ring": (src, det, mu)})
    f_ring, _ = solve(p, engine=engine, matrix_free=True)
    p_ref = gen.Problem(**{**p.__dict__, "A": A})
    f_ref, _ = lagged.solve_problem(p_ref)
    err = assert_parity(f_ring, f_ref, TOL, "ring irregular")
    _say(f"[ring] irregular 5 x 7: rel L2 vs oracle {err:.3e}")


def test_ring_batch_equals_alone(engine):
    import torch
    from paper_1308_6634_amd.engine import problem_struct, solve
    A = gen.operators.dense_sensitivity(8, mu=0.5 * 64.0 / 8 / 4.0, n_src_rings=2, n_det_rings=2)
    probs = [gen.small_dense_case(60 + i, 8, outer=2, inner=6, A=A) for i in range(3)]
    alone = [solve(p, engine=engine, matrix_free=True)[0] for p in probs]
    op = engine.ring_operator(probs[0].dims, *probs[0].extra["ring"])
    gs = [torch.from_numpy(np.ascontiguousarray(p.g, dtype=np.float32)).cuda() for p in probs]
    fs = [torch.zeros(p.n_x, device="cuda") for p in probs]
    ts = engine.submit_batch(op, [problem_struct(p) for p in probs], gs, fs)
    for (st, _), f, a in zip([engine.wait(t) for t in ts], fs, alone):
        assert st == 0
        np.testing.assert_array_equal(f.cpu().numpy().reshape(a.shape), a)


def test_full_size_c2_ring_first_iterations_match_stored_matrix(engine):
    """The c2 workload (64^3, 64 x 64 ring, n_y = 4096) through the regenerated entries agrees
    with the stored-matrix path (itself checked against the oracle at this size)."""
    import dataclasses
    from paper_1308_6634_amd.engine import solve
    p = dataclasses.replace(gen.config_c2(), outer=1, inner=3)
    f_ring, r_ring = solve(p, engine=engine, matrix_free=True)
    f_dense, r_dense = solve(p, engine=engine)
    diff = _rel(f_ring, f_dense)
    _say(f"[ring] c2 1x3: rel L2 ring vs stored matrix {diff:.3e}")
    assert diff <= 1e-4
    assert abs(r_ring.resid[0] - r_dense.resid[0]) <= 1e-4 * r_dense.resid[0]


def test_ring_operator_arguments_are_validated(engine):
    from paper_1308_6634_amd import plsqr as P
    src = np.zeros((4, 3), np.float32) - 1.0
    det = np.zeros((4, 3), np.float32) + 9.0
    for s, d, mu in ((src, det, 0.0), (src, det, -1.0), (np.zeros((0, 3), np.float32), det, 0.5),
                     (np.zeros((129, 3), np.float32), np.zeros((128, 3), np.float32), 0.5),
                     (np.full((4, 3), np.nan, np.float32), det, 0.5)):
        with pytest.raises(P.PlsqrError):
            engine.ring_operator((8, 8, 8), s, d, mu)
