"""Host-side pieces of bench.py: the HBM traffic record built from rocprofv3 counter CSVs,
the algorithmic byte counts of the dominant kernels and the one-GPU guard."""

import argparse
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _csv(folder, rows):
    os.makedirs(folder, exist_ok=True)
    with open(os.path.join(folder, "x_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(FIELDS, r)))


def test_write_traffic_scales_by_copy(tmp_path):
    k2 = "void plsqr::k_gemv_rows<2>(plsqr::InstDesc* const*, int, int)"
    k4 = "void plsqr::k_gemv_rows<4>(plsqr::InstDesc* const*, int, int)"
    other = "void plsqr::k_gemv_cols(plsqr::InstDesc* const*)"
    # two dispatches of <2> (one of them split over two rows), one of <4>, one unrelated kernel
    _csv(tmp_path / "f", [(1, k2, "FETCH_SIZE", 1000.0), (2, k2, "FETCH_SIZE", 600.0),
                          (2, k2, "FETCH_SIZE", 600.0), (3, k4, "FETCH_SIZE", 3000.0),
                          (4, other, "FETCH_SIZE", 9e9)])
    _csv(tmp_path / "w", [(1, k2, "WRITE_SIZE", 10.0), (2, k2, "WRITE_SIZE", 30.0),
                          (3, k4, "WRITE_SIZE", 8.0)])
    cp = "__amd_rocclr_copyBuffer"
    _csv(tmp_path / "cf", [(1, cp, "FETCH_SIZE", 524288.0), (2, cp, "FETCH_SIZE", 524288.0)])
    _csv(tmp_path / "cw", [(1, cp, "WRITE_SIZE", 1048576.0)])
    args = argparse.Namespace(write_traffic=[str(tmp_path / d) for d in ("f", "w", "cf", "cw")],
                              traffic_kernel="k_gemv_rows", traffic_sequence=None,
                              traffic_key=None, workload="c2")
    out = tmp_path / "traffic.json"
    bench.write_traffic(args, out=str(out))
    rec = json.load(open(out))
    assert set(rec["variants"]) == {"2", "4"}
    v2, v4 = rec["variants"]["2"], rec["variants"]["4"]
    assert v2["launches"] == 2 and v4["launches"] == 1
    assert rec["copy_calibration"]["fetch_scale"] == pytest.approx(2.0)
    assert rec["copy_calibration"]["write_scale"] == pytest.approx(1.0)
    assert v2["fetch_bytes_per_launch"] == pytest.approx(1100.0 * 1024 * 2.0)
    assert v2["write_bytes_per_launch"] == pytest.approx(20.0 * 1024)
    assert v4["bytes_per_launch"] == pytest.approx(3000.0 * 1024 * 2.0 + 8.0 * 1024)
    assert rec["source_sha"] == bench.kernel_source_hash(bench.KERNEL_SOURCES["c2"])


def test_write_traffic_sums_a_dispatch_sequence(tmp_path):
    """The c4 forward product is three consecutive dispatches (pack, GEMM, reduce); the adjoint
    reuses the pack kernel before another GEMM variant, which must not be counted."""
    pk = "void plsqr::k_pack_split(plsqr::InstDesc* const*, int, int, long long)"
    gf = "void plsqr::k_gemm_bf16<2, true, false>(plsqr::GemmArgs)"
    ga = "void plsqr::k_gemm_bf16<2, true, true>(plsqr::GemmArgs)"
    rd = "void plsqr::k_fwd_reduce(plsqr::InstDesc* const*, float const*, int)"
    seq = [(pk, 5.0), (gf, 100.0), (rd, 2.0), (pk, 7.0), (ga, 300.0)] * 2
    _csv(tmp_path / "f", [(i + 1, k, "FETCH_SIZE", v) for i, (k, v) in enumerate(seq)])
    _csv(tmp_path / "w", [(i + 1, k, "WRITE_SIZE", v / 10) for i, (k, v) in enumerate(seq)])
    cp = "__amd_rocclr_copyBuffer"
    _csv(tmp_path / "cf", [(1, cp, "FETCH_SIZE", 1048576.0)])
    _csv(tmp_path / "cw", [(1, cp, "WRITE_SIZE", 1048576.0)])
    args = argparse.Namespace(write_traffic=[str(tmp_path / d) for d in ("f", "w", "cf", "cw")],
                              traffic_kernel=None,
                              traffic_sequence="k_pack_split;k_gemm_bf16<2, true, false>;k_fwd_reduce",
                              traffic_key="forward_bf16_refined", workload="c4")
    out = tmp_path / "traffic_c4.json"
    bench.write_traffic(args, out=str(out))
    v = json.load(open(out))["variants"]["forward_bf16_refined"]
    assert v["launches"] == 2
    assert v["fetch_bytes_per_launch"] == pytest.approx(107.0 * 1024)
    assert v["write_bytes_per_launch"] == pytest.approx(10.7 * 1024)


def test_dominant_bytes():
    class P:
        pass

    p = P()
    # blur: algorithmic bytes are v read, u read and written; the kernels move 2k + 1 vectors
    p.dims, p.op_kind = (8, 8, 8), "blur"
    b, _, k = bench.dominant_bytes(p)
    assert b == 4 * 512 * 3 and k == 4 * 512 * 7          # 3 passes
    p.dims = (6, 8, 1)
    b, _, k = bench.dominant_bytes(p)
    assert b == 4 * 48 * 3 and k == 4 * 48 * 5            # 2 passes
    p.dims = (16, 1, 1)
    b, _, k = bench.dominant_bytes(p)
    assert b == 4 * 16 * 3 and k == 4 * 16 * 3            # 1 pass
    # with the previous step's f, w update (f and w read and written, in inner - 1 of every
    # inner products; the pass that applies it reads v again)
    p.dims, p.inner = (8, 8, 8), 5
    b, _, k = bench.dominant_bytes(p, update_fused=True)
    assert b == 12 * 512 + 16 * 512 * 4 // 5 and k == 28 * 512 + 20 * 512 * 4 // 5
    assert bench.blur_update_fused(p, {}) and not bench.blur_update_fused(p, {"tune_vcycle": 1})
    p.dims = (6, 8, 8)
    assert not bench.blur_update_fused(p, {})               # the x pass takes 4-voxel groups only
    # above the tail the update runs in the V-cycle tail launch, unless the batch is large or
    # the knob puts it in the product
    p.dims, p.levels, p.smoother, p.nu_pre, p.cheb_degree = (64, 64, 64), 5, "chebyshev", 1, 3
    assert bench.update_in_tail(p, {}) and not bench.blur_update_fused(p, {})
    assert bench.blur_update_fused(p, {"tune_update_site": 1})
    assert bench.blur_update_fused(p, {}, batch=17) and not bench.update_in_tail(p, {}, 17)
    assert bench.update_in_tail(p, {"tune_update_site": 2}, 17)
    p.nu_pre = 2                                            # Chebyshev level kernels: one polynomial
    assert bench.blur_update_fused(p, {})
    import numpy as np
    p.dims, p.op_kind, p.A = (4, 4, 2), "dense", np.zeros((10, 32), np.float32)
    b, _, k = bench.dominant_bytes(p)
    assert b == k == 4 * 10 * 32 + 4 * 32 + 8 * 10


def test_more_than_one_gpu_exits():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout
