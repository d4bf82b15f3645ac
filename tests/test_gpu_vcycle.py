"""The fused level kernels of the V-cycle (one launch per level for the whole pre-smoothing with
the residual restriction, one for the prolongation with the whole post-smoothing) against the
per-sweep kernels and the FP64 oracle.

Both launch schedules compute every voxel with the same formulas in the same order; only the
alpha = sqrt(v . p) partial sums are grouped by different blocks, so whole solves agree to
float32 rounding propagated through the Krylov recurrence (bar 2e-5), and each meets the oracle
bar. The cases cover every fused depth (Jacobi sweeps 1-4, Chebyshev degree 1-4), 2D and 3D,
tiles that leave ragged edges in x, y and z (grids not multiples of the tile, knobs that force
small tiles), levels whose coarse grid has one z-plane, and a batch.
"""

import sys

import numpy as np
import pytest

import gen
from oracle import lagged
from parity import assert_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def engine():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1308_6634_amd.engine import Engine
    eng = Engine(0)
    yield eng
    eng.close()


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


CASES = [
    # dims, levels, smoother, nu, degree, ty, zc, voxels per thread (0: the default, which on
    # these grids is one; 4: groups of four)
    ((40, 24, 12), 3, "jacobi", 2, 3, 0, 0, 0),
    ((40, 24, 12), 3, "jacobi", 2, 3, 0, 0, 4),
    ((40, 24, 12), 3, "jacobi", 2, 3, 6, 4, 4),
    ((96, 20, 8), 3, "jacobi", 1, 3, 4, 2, 4),
    ((96, 20, 8), 3, "jacobi", 1, 3, 4, 2, 1),
    ((32, 16, 8), 3, "jacobi", 3, 3, 0, 0, 0),
    ((24, 16, 8), 3, "jacobi", 4, 3, 2, 2, 4),
    ((24, 16, 8), 3, "jacobi", 4, 3, 2, 2, 1),
    ((32, 32, 16), 3, "chebyshev", 1, 3, 0, 0, 0),
    ((32, 32, 16), 3, "chebyshev", 1, 3, 0, 0, 4),
    ((32, 32, 16), 3, "chebyshev", 1, 3, 10, 6, 1),
    ((36, 12, 4), 2, "chebyshev", 1, 1, 0, 0, 4),
    ((36, 12, 4), 2, "chebyshev", 1, 1, 0, 0, 0),
    ((48, 16, 4), 3, "chebyshev", 1, 2, 0, 0, 0),
    ((40, 16, 8), 3, "chebyshev", 1, 4, 6, 2, 4),
    ((40, 16, 8), 3, "chebyshev", 1, 4, 6, 2, 1),
    # four levels: the LDS-resident tail holds two smoothed levels and the coarsest, so a
    # prolongation reads a level whose iterate is in either array of its pair
    ((32, 32, 16), 4, "jacobi", 2, 3, 0, 0, 0),
    ((32, 32, 16), 4, "jacobi", 1, 3, 0, 0, 4),
    ((32, 32, 16), 4, "jacobi", 3, 3, 0, 0, 1),
    ((32, 32, 16), 4, "chebyshev", 1, 2, 0, 0, 0),
    ((64, 48, 1), 4, "jacobi", 2, 3, 0, 0, 0),
    ((64, 48, 1), 4, "jacobi", 1, 3, 0, 0, 0),
    ((64, 48, 1), 4, "chebyshev", 1, 3, 8, 0, 4),
    ((16, 16, 2), 2, "jacobi", 2, 3, 0, 0, 0),
    ((70, 14, 4), 2, "chebyshev", 1, 3, 0, 0, 1),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}-{c[2]}{c[3] if c[2] == 'jacobi' else c[4]}-t{c[5]}z{c[6]}v{c[7]}")
def test_fused_equals_per_sweep_and_oracle(engine, case):
    from paper_1308_6634_amd import plsqr as P
    from paper_1308_6634_amd.engine import solve
    dims, levels, sm, nu, deg, ty, zc, v = case
    p = gen.small_blur_case(300 + sum(dims), dims, sigma=1.5, radius=3, reg="pm_log", T=0.05,
                            tau=20.0, outer=2, inner=6, levels=levels, smoother=sm, nu_pre=nu,
                            nu_post=nu, cheb_degree=deg, eps=1e-2)
    _say(f"[vcycle] {p.name} {sm} nu={nu} deg={deg} ty={ty} zc={zc} v={v}")
    fused, _ = solve(p, engine=engine, knobs={"tune_zm_ty": ty, "tune_zm_zc": zc, "tune_zm_v": v})
    sweep, _ = solve(p, engine=engine, knobs={"tune_vcycle": P.PLSQR_VCYCLE_PER_SWEEP})
    rel = float(np.linalg.norm(fused - sweep) / np.linalg.norm(sweep))
    assert rel <= 2e-5, rel
    f_ref, _ = lagged.solve_problem(p)
    err = assert_parity(fused, f_ref, 1e-3, p.name)
    _say(f"[vcycle]   fused vs per-sweep {rel:.2e}, vs oracle {err:.2e}")


def test_fused_batch_equals_alone(engine):
    """A lockstep batch through the fused kernels gives each instance its solo result."""
    import torch
    from paper_1308_6634_amd.engine import problem_struct, solve
    probs = [gen.small_blur_case(330 + i, (32, 24, 16), reg=r, T=0.05, tau=20.0, outer=2, inner=5,
                                 levels=3, smoother="chebyshev", nu_pre=1, nu_post=1)
             for i, r in enumerate(["stv", "pm_log", "tikhonov"])]
    alone = [solve(p, engine=engine)[0] for p in probs]
    op = engine.blur_operator(probs[0].dims, probs[0].taps)
    gs = [torch.from_numpy(np.ascontiguousarray(p.g, np.float32).ravel()).cuda() for p in probs]
    fs = [torch.zeros(p.n_x, device="cuda") for p in probs]
    ts = engine.submit_batch(op, [problem_struct(p) for p in probs], gs, fs)
    for t, f, a in zip(ts, fs, alone):
        st, _ = engine.wait(t)
        assert st == 0
        np.testing.assert_array_equal(f.cpu().numpy().reshape(a.shape), a)
