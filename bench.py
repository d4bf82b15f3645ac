#!/usr/bin/env python
"""Throughput benchmark: voxel-LSQR-iterations per second on one MI355X.

Workload (default): a 64^3 grid reconstructed from a dense 4096 x 262144 float32 ring
sensitivity matrix (64 sources x 64 detectors on four rings), five ellipsoid
inclusions, 1% noise, Perona-Malik (log) diffusivity T = 0.05, tau = 20, 8 outer x 40
inner iterations, 5-level Jacobi V(2,2) priorconditioner. A step is one whole
reconstruction (all outer and inner iterations, setup and diagnostics included) with
inputs already resident in HBM.

value = n_X * outer * inner * steps / wall seconds of the timed steps.

Beside it: the roofline of the dominant kernel (the dense forward product, timed with
HIP events on the stream it runs on) and the FP64 oracle timed on the host cores on a
bounded sample of the same workload.
"""

import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, 8 TB/s
FP32_VECTOR_PEAK_TFLOPS = 157.3
# Matrix-free ring product: 6 flops per entry (r_s r_d, + 1, 1/t, a c, * v, + acc). The issue
# model: 256 CUs x 4 SIMDs at 2.4 GHz; the 157.3 TFLOP/s FP32 vector peak counts packed (two per
# lane) FMAs on 16 lanes per SIMD per clock, so unpacked FP32 operations (the library is
# compiled without packed FP32) run 16 lanes per SIMD per clock and the reciprocal, a transcendental, at
# a quarter of that. An entry takes 3 unpacked operations and one reciprocal, 3/16 + 1/4
# SIMD-clocks per lane, so at most 256 * 4 * 2.4e9 / (3/16 + 1/4) = 5.6e12 entries/s.
RING_FLOPS_PER_ENTRY = 6
RING_ENTRY_PEAK = 256 * 4 * 2.4e9 / (3.0 / 16.0 + 1.0 / 4.0)
# HBM traffic records (rocprofv3 FETCH_SIZE / WRITE_SIZE passes, copy-calibrated), one file per
# workload, keyed by a hash of the sources that determine the counted kernels' device code.
def traffic_file(workload):
    return os.path.join(ROOT, "profiles", f"traffic_{workload}.json")


# Sources that determine the device code of each workload's dominant kernel: HBM traffic counted
# for it stays valid while these and the device compile flags are unchanged. (kernels.hpp only
# declares host launchers and constants the kernels do not use.)
KERNEL_SOURCES = {"c2": ("dense.hip", "device_common.hpp", "plsqr_internal.hpp"),
                  "c4": ("gemm_bf16.hip", "device_common.hpp", "plsqr_internal.hpp")}


def kernel_source_hash(files):
    """Hash of the sources and of the device compile flags that determine the kernel's code."""
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "_plsqr_build_flags", os.path.join(ROOT, "paper_1308_6634_amd", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    h = hashlib.sha256(" ".join(mod.DEVICE_FLAGS).encode())
    for name in files:
        with open(os.path.join(ROOT, "paper_1308_6634_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_for(workload, key):
    """HBM bytes per launch of variant ``key`` from the workload's traffic record, or None when
    there is none or the kernel's sources have changed since the counters were taken."""
    fn = traffic_file(workload)
    if not os.path.exists(fn):
        return None
    try:
        tr = json.load(open(fn))
        var = tr.get("variants", {}).get(str(key))
        if var is None or tr.get("source_sha") != kernel_source_hash(tuple(tr["source_files"])):
            return None
        return var["bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        return None


def workload(name):
    import gen
    if name == "c2":
        p = gen.config_c2()
        desc = ("64^3 grid, dense ring sensitivity 4096x262144 fp32 (64 src x 64 det, 4 rings, "
                "mu=0.5), 5 ellipsoids, 1% noise, Perona-Malik log T=0.05, tau=20, 8 outer x 40 "
                "inner, 5-level Jacobi V(2,2) omega=0.8, eps=1e-6")
    elif name == "c3":
        p = gen.config_c3()
        desc = ("128^3 grid, separable Gaussian blur sigma=3 (19 taps), 20 boxes/spheres, 0.5% "
                "noise, smoothed TV T=0.02, tau=100, 10 outer x 60 inner, 6-level Chebyshev(3)")
    elif name == "c1":
        p = gen.config_c1()
        desc = ("64^2 image, Gaussian blur sigma=2 (9 taps), 8 rectangles, 1% noise, smoothed TV "
                "T=0.01, tau=50, 10 outer x 50 inner, 4-level Jacobi V(2,2)")
    else:
        raise SystemExit(f"unknown workload {name}")
    return p, desc


def update_in_tail(p, settings, batch=1):
    """Whether the library runs the previous inner step's f, w update in extra workgroups of the
    V-cycle tail launch (tune_update_site; by default where that applies and the batch holds at
    most 2^22 voxels): a blur operator with nx % 4 == 0 on a grid of more than one row, no S4
    recurrence, and a fused V-cycle of two or more levels whose finest level runs as fused
    level kernels above the tail (Jacobi with at most 4 sweeps, or Chebyshev of degree <= 4 with
    one polynomial per side)."""
    s = settings or {}
    site = s.get("tune_update_site", 0)
    nx, ny, nz = p.dims
    n = nx * ny * nz
    if site == 1 or p.op_kind != "blur" or nx % 4 or s.get("tune_vcycle", 0):
        return False
    if n <= (s.get("tune_tail_cells", 0) or 4096):   # the finest level is in the tail
        return False
    if getattr(p, "stop_s4", False) or (ny < 2 and nz < 2) or p.levels == 1:
        return False
    if p.smoother == "jacobi" and p.nu_pre > 4:
        return False
    if p.smoother != "jacobi" and (p.nu_pre != 1 or p.cheb_degree > 4):
        return False
    return site == 2 or batch * n <= 1 << 22


def blur_update_fused(p, settings, batch=1):
    """Whether the library applies the previous inner step's f, w update inside the forward blur
    product (the fused update: a four-voxel x pass, the fused V-cycle, no S4 recurrence), rather
    than in the V-cycle tail launch (update_in_tail) or a launch of its own."""
    return (p.op_kind == "blur" and p.dims[0] % 4 == 0 and not getattr(p, "stop_s4", False)
            and not (settings or {}).get("tune_vcycle", 0)
            and not update_in_tail(p, settings, batch))


def dominant_bytes(p, update_fused=False):
    """Algorithmic HBM bytes of one dominant-kernel launch (the forward product u <- A v - alpha u:
    read A (dense), read v, read and write u), its name, and the bytes its kernels move.
    update_fused: the blur product also applies the previous step's f, w update (read and write
    f and w: 16 bytes per voxel in inner - 1 of every inner products; its pass reads v again)."""
    nx, ny, nz = p.dims
    n = nx * ny * nz
    if p.op_kind == "dense":
        m = p.A.shape[0]
        b = 4 * m * n + 4 * n + 8 * m
        return b, "k_gemv_rows (dense forward product A v, u update)", b
    # blur: one 1D pass per axis of extent > 1; each pass reads and writes one vector (halo
    # re-reads come from cache) and the last one also reads u, so 2 k + 1 vectors move for k
    # passes, against 3 vectors (v in, u in and out) for the product itself
    k = max(1, sum(1 for e in (nx, ny, nz) if e > 1))
    names = ("k_blur_xg" if nx % 4 == 0 else "k_blur_x") + (" + k_blur_win" if k > 1 else "")
    upd = (p.inner - 1) / p.inner if update_fused else 0.0
    return int(12 * n + 16 * n * upd), \
        f"{names} (forward blur product, {k} pass{'es' if k > 1 else ''}" + \
        (", with the previous step's f, w update)" if update_fused else ")"), \
        int(4 * n * (2 * k + 1) + 20 * n * upd)


def cpu_baseline(p, target_s=20.0):
    """The FP64 oracle on a bounded sample of about target_s seconds: the first K outer
    iterations with all their inner iterations when one outer iteration fits the budget,
    otherwise the first outer iteration with S inner iterations. Returns (record, K, S, f)."""
    import numpy as np
    from threadpoolctl import threadpool_info
    from oracle import lagged

    nx, ny, nz = p.dims
    shape = (nz, ny, nx)
    op = lagged.make_operator(p.op_kind, shape, taps=p.taps, A=p.A)   # input prep, untimed
    from oracle import multigrid
    sm = multigrid.Smoother(p.smoother, p.nu_pre, p.nu_post, p.omega, p.cheb_degree, p.cheb_lo,
                            p.cheb_hi)
    g = np.asarray(p.g, dtype=np.float64).reshape(shape if p.op_kind == "blur" else (-1,))

    def run(outer, inner):
        t0 = time.perf_counter()
        f, _ = lagged.solve(shape, op, g, p.reg, p.T, p.tau, p.eps, outer, inner, p.levels, sm)
        return time.perf_counter() - t0, f

    t2, _ = run(1, 2)
    per_iter = max(t2 / 3.0, 1e-3)
    if per_iter * p.inner <= target_s / 2:
        K, S = int(min(p.outer, max(1, round(target_s / (per_iter * p.inner))))), p.inner
    else:
        K, S = 1, int(min(p.inner, max(4, target_s / per_iter)))
    t, f = run(K, S)
    threads = [i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"]
    cores = max(threads) if threads else 1
    n = nx * ny * nz
    what = (f"first {K} outer iterations x {S} inner iterations" if K > 1
            else f"first outer iteration with {S} inner iterations")
    return {"value": n * K * S / t, "unit": "voxel-iter/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{what} (setup included), {t:.1f} s, FP64 NumPy/SciPy, "
                      f"host cores: {len(os.sched_getaffinity(0))}"}, K, S, f


def _counter_rows(folder, counter):
    """[(dispatch key, short kernel name, value)] of one rocprofv3 counter, in dispatch order."""
    import csv
    import glob
    vals = {}
    files = glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {folder}")
    for fn in sorted(files):
        with open(fn, newline="") as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") != counter:
                    continue
                did = row.get("Dispatch_Id") or row.get("Correlation_Id")
                key = (fn, int(did) if did and did.isdigit() else did)
                name = _short_kernel(row.get("Kernel_Name", ""))
                old = vals.get(key, (name, 0.0))
                vals[key] = (name, old[1] + float(row["Counter_Value"]))
    return [(k, v[0], v[1]) for k, v in sorted(vals.items(), key=lambda kv: kv[0])]


def _counter_per_dispatch(folder, counter, match):
    """{kernel name: per-dispatch values} of one rocprofv3 counter, for kernels whose (short)
    name satisfies match."""
    out = {}
    for _, name, v in _counter_rows(folder, counter):
        if match(name):
            out.setdefault(name, []).append(v)
    return out


def _sequence_sums(folder, counter, seq):
    """Per occurrence of the consecutive dispatch sequence ``seq`` (exact short kernel names),
    the counter summed over its dispatches."""
    rows = _counter_rows(folder, counter)
    sums, i = [], 0
    while i + len(seq) <= len(rows):
        if all(rows[i + k][1] == seq[k] for k in range(len(seq))):
            sums.append(sum(rows[i + k][2] for k in range(len(seq))))
            i += len(seq)
        else:
            i += 1
    return sums


def _short_kernel(full):
    """'void plsqr::k_gemv_rows<2>(plsqr::InstDesc* const*, int, int)' -> 'k_gemv_rows<2>'."""
    s = full.split("(")[0].replace("void ", "").strip()
    return s.split("::")[-1] if "::" in s.split("<")[0] else s


def write_traffic(args, out=None):
    """HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE passes (KiB per dispatch),
    each scaled so that a plain 1 GiB device copy reads and writes 1 GiB. Either every template
    variant of one kernel (--traffic-kernel, e.g. each k_gemv_rows<R> the autotuner ran), or one
    sequence of consecutive dispatches that make up one product (--traffic-sequence, comma
    separated exact names, recorded under --traffic-key)."""
    import re
    fdir, wdir, cfdir, cwdir = args.write_traffic
    cfetch = sum(_counter_per_dispatch(cfdir, "FETCH_SIZE", lambda k: "copyBuffer" in k).values(), [])
    cwrite = sum(_counter_per_dispatch(cwdir, "WRITE_SIZE", lambda k: "copyBuffer" in k).values(), [])
    if not (cfetch and cwrite):
        raise SystemExit("the copy calibration passes hold no copy dispatch")
    gib_kib = float(1 << 20)
    fscale = gib_kib / (sum(cfetch) / len(cfetch))
    wscale = gib_kib / (sum(cwrite) / len(cwrite))
    groups = {}          # key -> (name, fetch values, write values)
    if args.traffic_sequence:
        seq = [x.strip() for x in args.traffic_sequence.split(";")]
        key = args.traffic_key or "sequence"
        groups[key] = (" + ".join(seq), _sequence_sums(fdir, "FETCH_SIZE", seq),
                       _sequence_sums(wdir, "WRITE_SIZE", seq))
        base = " + ".join(seq)
    elif args.traffic_kernel:
        base = args.traffic_kernel.split("<")[0]

        def is_kernel(k):
            return k == base or k.startswith(base + "<")

        fetch = _counter_per_dispatch(fdir, "FETCH_SIZE", is_kernel)
        write = _counter_per_dispatch(wdir, "WRITE_SIZE", is_kernel)
        for name in sorted(set(fetch) & set(write)):
            m = re.search(r"<(\d+)>", name)
            groups[m.group(1) if m else name] = (name, fetch[name], write[name])
    else:
        raise SystemExit("--write-traffic needs --traffic-kernel or --traffic-sequence")
    variants = {}
    for key, (name, fv, wv) in groups.items():
        if not (fv and wv):
            raise SystemExit(f"a counter pass holds no dispatch of {name}")
        f_kib, w_kib = sum(fv) / len(fv), sum(wv) / len(wv)
        fb, wb = f_kib * 1024 * fscale, w_kib * 1024 * wscale
        variants[key] = {"kernel": name, "launches": len(fv),
                         "fetch_kib_per_launch_raw": f_kib, "write_kib_per_launch_raw": w_kib,
                         "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
                         "bytes_per_launch": fb + wb}
        print(f"{name}: {len(fv)} launches; FETCH_SIZE {f_kib:.1f} KiB raw x {fscale:.5f}, "
              f"WRITE_SIZE {w_kib:.1f} KiB raw x {wscale:.5f} -> {(fb + wb) / 1e9:.4f} GB per launch")
    files = KERNEL_SOURCES[args.workload]
    rec = {"workload": args.workload, "kernel": base, "variants": variants,
           "source_sha": kernel_source_hash(files), "source_files": list(files),
           "copy_calibration": {"bytes": 1 << 30, "fetch_kib_raw": sum(cfetch) / len(cfetch),
                                "write_kib_raw": sum(cwrite) / len(cwrite), "fetch_scale": fscale,
                                "write_scale": wscale, "launches": len(cfetch)}}
    with open(out or traffic_file(args.workload), "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c4", choices=["c2", "c3", "c1", "c4", "c5"])
    ap.add_argument("--latency-solves", type=int, default=20,
                    help="c1-c3: solves issued one at a time after the timed run for the p50/p99 "
                         "solve latency (0: skip)")
    ap.add_argument("--requests", type=int, default=2000, help="c5 only: requests in the stream")
    ap.add_argument("--templates", type=int, default=200,
                    help="c5 only: distinct pre-generated reconstructions the stream cycles through")
    ap.add_argument("--plain-requests", type=int, default=300,
                    help="c5 only: prefix of the stream replayed on the plain one-at-a-time path")
    ap.add_argument("--precision", default="bf16_refined", choices=["bf16_refined", "bf16"],
                    help="c4 only: BF16 product mode of the batched path")
    ap.add_argument("--plain-sample", type=int, default=2,
                    help="c4 only: instances run one at a time on the FP32 path for comparison")
    ap.add_argument("--batch", type=int, default=1,
                    help="c3 only: run this many 128^3 instances (seeds 2, 3, ...) as one lockstep "
                         "FP32 batch, so that every stencil and multigrid launch moves B vectors")
    ap.add_argument("--no-graphs", action="store_true",
                    help="launch every kernel eagerly (for hardware-counter profiling, which "
                         "does not see kernels replayed from HIP graphs)")
    ap.add_argument("--stop", action="store_true",
                    help="c1-c3: also time the same reconstruction with the paper's adaptive stops "
                         "(S4 with eta = 1.1 and the drawn noise norm as delta, the configured "
                         "inner count as the cap; outer stop once R(f^k) stops decreasing, checked "
                         "from k = 3) and compare its result with the fixed-count one")
    ap.add_argument("--matrix-free", action="store_true",
                    help="c2: apply the ring sensitivity through its geometry (entries recomputed "
                         "in every product) instead of the stored 4096 x 262144 matrix")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--counts", default=None, metavar="OUTER,INNER",
                    help="c1-c3: override the workload's outer x inner iteration counts (for "
                         "profiler runs, which slow every launch; the record's workload text "
                         "states the override)")
    ap.add_argument("--knob", action="append", default=[], metavar="NAME=VALUE",
                    help="set a tiling knob of the problem struct (tune_*), after any autotuning; "
                         "repeatable")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the (untimed) autotuning of tiling knobs before the warm-up")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy 3 times (HBM counter calibration)")
    ap.add_argument("--write-traffic", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPYF_DIR", "COPYW_DIR"),
                    help="host only: turn four rocprofv3 --pmc CSV output folders (FETCH_SIZE and "
                         "WRITE_SIZE of a bench run, then of --copy-calibration) into the HBM "
                         "traffic record of --traffic-kernel read by later bench runs")
    ap.add_argument("--stream", action="store_true",
                    help="practical HBM ceiling: a 2 GiB device copy and a 4 GiB read-only sum "
                         "(library kernels of PyTorch), timed with events")
    ap.add_argument("--traffic-kernel", default=None,
                    help="kernel for --write-traffic: every template variant of it is recorded, "
                         "e.g. 'k_gemv_rows'")
    ap.add_argument("--traffic-sequence", default=None,
                    help="for --write-traffic: ';'-separated exact short names of consecutive "
                         "dispatches forming one product, e.g. 'k_pack_split;k_gemm_bf16<2, true, "
                         "false>;k_fwd_reduce'")
    ap.add_argument("--traffic-key", default=None,
                    help="record key of --traffic-sequence (c4: forward_bf16_refined)")
    args = ap.parse_args()
    args.knobs = {}
    for kv in args.knob:
        name, _, val = kv.partition("=")
        if not name.startswith("tune_") or not val:
            raise SystemExit(f"--knob takes tune_NAME=VALUE, got {kv!r}")
        args.knobs[name] = int(val)
    if args.write_traffic:
        return write_traffic(args)
    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 1 << 30, "copy_bytes_written": 1 << 30, "launches": 3}))
        return
    if args.stream:
        return stream_ceiling()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU only; --gpus must be 1 "
                                   "(instances shard across GPUs without communication, see the "
                                   "design notes)"}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1308_6634_amd import plsqr as P
    from paper_1308_6634_amd.engine import Engine, problem_struct

    if args.workload == "c4":
        return bench_c4(args)
    if args.workload == "c5":
        return bench_c5(args)
    if args.batch > 1:
        if args.workload != "c3":
            raise SystemExit("--batch applies to the c3 workload only")
        return bench_c3_batch(args)
    p, desc = workload(args.workload)
    if args.counts:
        k_out, k_in = (int(x) for x in args.counts.split(","))
        p = dataclasses.replace(p, outer=k_out, inner=k_in)
        desc += f" [counts overridden: {k_out} outer x {k_in} inner]"
    nx, ny, nz = p.dims
    n = nx * ny * nz
    print(f"[bench] workload {args.workload}: {desc}", file=sys.stderr, flush=True)
    eng = Engine(0)
    settings, tune_report = {}, None
    if not args.no_tune and not args.matrix_free:   # no tiling knob applies to the ring products
        from paper_1308_6634_amd import autotune
        settings, tune_report = autotune.tune(p, eng)
        p = autotune.apply(p, settings)
        print(f"[bench] autotuned: {settings}", file=sys.stderr, flush=True)
    settings.update(args.knobs)
    if p.op_kind == "dense" and args.matrix_free:
        op = eng.ring_operator(p.dims, *p.extra["ring"])
    elif p.op_kind == "dense":
        op = eng.dense_operator(p.dims, p.A)
    else:
        op = eng.blur_operator(p.dims, p.taps)
    g = torch.from_numpy(np.ascontiguousarray(p.g, dtype=np.float32).ravel()).cuda()
    f = torch.zeros(n, dtype=torch.float32, device="cuda")
    # the timed steps carry no timing events (every inner iteration replays as one graph); the
    # products are timed with events in one more solve afterwards, for the roofline figure
    graphs_flag = P.PLSQR_FLAG_NO_GRAPHS if args.no_graphs else 0
    pb = problem_struct(p, flags=graphs_flag, knobs=settings)

    for _ in range(args.warmup):
        st, _ = eng.wait(eng.submit(op, pb, g, f))
        assert st == 0, P.plsqr_last_error(eng.handle)
    print("[bench] warmup done", file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tickets = [eng.submit(op, pb, g, f) for _ in range(args.steps)]
    results = [eng.wait(t) for t in tickets]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for st, _ in results:
        assert st == 0
    iters = n * p.outer * p.inner * args.steps
    value = iters / elapsed
    st, timed = eng.wait(eng.submit(op, problem_struct(p, flags=graphs_flag |
                                                       P.PLSQR_FLAG_TIME_PRODUCTS,
                                                       knobs=settings), g, f))
    assert st == 0
    fwd_ms, fwd_n = timed.forward_ms, timed.forward_launches
    adj_ms, adj_n = timed.adjoint_ms, timed.adjoint_launches
    avg_fwd_s = fwd_ms / max(fwd_n, 1) / 1e3
    nbytes, kname, pass_bytes = dominant_bytes(p, blur_update_fused(p, settings))
    achieved = nbytes / avg_fwd_s / 1e9 if avg_fwd_s > 0 else None
    roofline = None
    if args.matrix_free:
        # ALU-bound: per entry r_s r_d + 1 (FMA), 1/t, a c (multiply), times v, accumulate
        entries = int(p.n_y) * n
        # peak: the entry issue limit (3 unpacked FP32 operations and a reciprocal per entry)
        # expressed in the same 6 flops per entry as the achieved figure
        alu_peak = RING_FLOPS_PER_ENTRY * RING_ENTRY_PEAK / 1e12
        alu = RING_FLOPS_PER_ENTRY * entries / avg_fwd_s / 1e12
        roofline = {"bound": "alu", "kernel": "k_ring_fwd + k_ring_fwd_sum + k_ring_fwd_reduce "
                    "(forward product, entries regenerated)", "achieved": alu, "peak": alu_peak,
                    "unit": "TFLOP/s", "frac": alu / alu_peak,
                    "fp32_vector_peak_tflops": FP32_VECTOR_PEAK_TFLOPS,
                    "frac_of_fp32_vector_peak": alu / FP32_VECTOR_PEAK_TFLOPS,
                    "traffic": None, "entries_per_launch": entries,
                    "entries_per_s": entries / avg_fwd_s, "entry_peak_per_s": RING_ENTRY_PEAK,
                    "entry_frac": entries / avg_fwd_s / RING_ENTRY_PEAK,
                    "avg_launch_ms": avg_fwd_s * 1e3, "launches": int(fwd_n)}
    traffic = None
    if p.op_kind == "dense" and not args.matrix_free:
        traffic = traffic_for(args.workload, settings.get("tune_gemv_rows"))
    print(f"[bench] timed {args.steps} steps in {elapsed:.3f} s; forward product avg "
          f"{avg_fwd_s * 1e3:.3f} ms, adjoint avg {adj_ms / max(adj_n, 1):.3f} ms (one more "
          f"solve with product timing)", file=sys.stderr, flush=True)

    out = {
        "metric": "voxel-LSQR-iters/s",
        "value": value,
        "unit": "voxel-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}" + (
                       "; matrix-free: entries regenerated from the source/detector positions in "
                       "every product" if args.matrix_free else ""), "n_x": n, "n_y": int(p.n_y),
                   "outer": p.outer, "inner": p.inner, "precision": "fp32 vectors, fp64 scalars",
                   "autotuned": settings},
        "roofline": roofline or {
            "bound": "hbm", "kernel": kname, "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
            "traffic": traffic, "bytes_per_launch": nbytes, "kernel_bytes_per_launch": pass_bytes,
            "avg_launch_ms": avg_fwd_s * 1e3, "launches": int(fwd_n)},
    }
    if args.latency_solves > 0:
        pb_plain = problem_struct(p, flags=P.PLSQR_FLAG_NO_GRAPHS if args.no_graphs else 0,
                                  knobs=settings)   # products inside the graphs, no events
        out["latency_ms"] = solve_latency(args.latency_solves, eng, op, pb_plain, g, f)
    if args.stop:
        out["adaptive"] = adaptive_run(args, eng, op, p, settings, g, f)
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on a sample", file=sys.stderr, flush=True)
        cb, K, S, f_ref = cpu_baseline(p)
        out["cpu_baseline"] = cb
        # the same sample on the GPU, for a parity figure at full size
        q = dataclasses.replace(p, outer=K, inner=S)
        st, _ = eng.wait(eng.submit(op, problem_struct(q, knobs=settings), g, f))
        assert st == 0
        fg = f.cpu().numpy().astype(np.float64).reshape(f_ref.shape)
        out["parity_sample_rel_l2"] = float(np.linalg.norm(fg - f_ref) / np.linalg.norm(f_ref))
    eng.close()
    print(json.dumps(out), flush=True)


def stream_ceiling(reps=10):
    """STREAM-like practical ceiling of HBM bandwidth on this GPU: a device-to-device copy of
    2 GiB (reads and writes 2 GiB each) and a sum over 4 GiB (reads 4 GiB), both far larger than
    the last-level cache, timed with events on the current stream."""
    import torch
    n = 1 << 29                                   # 2 GiB of float32
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    big = torch.ones(2 * n, dtype=torch.float32, device="cuda")
    out = {}
    for name, fn, nbytes in (("copy", lambda: dst.copy_(src), 2 * 4 * n),
                             ("read_sum", lambda: big.sum(), 4 * 2 * n)):
        for _ in range(2):
            fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        out[name] = {"bytes": nbytes, "ms": ms, "GB_per_s": nbytes / ms / 1e6,
                     "frac_of_8TBps": nbytes / ms / 1e6 / HBM_PEAK_GBS}
    print(json.dumps({"stream_ceiling": out, "reps": reps}), flush=True)


def solve_latency(k, eng, op, pb, g, f):
    """p50 / p99 of the host wall time from plsqr_solve to completion over k solves issued one
    at a time (nothing else queued), after the throughput run."""
    import numpy as np
    lat = []
    for _ in range(k):
        t = time.perf_counter()
        st, _ = eng.wait(eng.submit(op, pb, g, f))
        lat.append((time.perf_counter() - t) * 1e3)
        assert st == 0
    print(f"[bench] latency over {k} solves: p50 {np.percentile(lat, 50):.2f} ms, p99 "
          f"{np.percentile(lat, 99):.2f} ms", file=sys.stderr, flush=True)
    return {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
            "min": float(min(lat)), "max": float(max(lat)), "n": k,
            "mode": "one solve at a time, submit to completion"}


def adaptive_run(args, eng, op, p, settings, g, f):
    """The workload with the adaptive stops against its fixed-count result (already in f)."""
    import numpy as np
    import torch
    from paper_1308_6634_amd.engine import problem_struct
    q = dataclasses.replace(p, stop_s4=True, eta=1.1, stop_outer=True, outer_rtol=0.0, outer_min=3)
    f_fixed = f.clone()
    fa = torch.zeros_like(f)
    pb = problem_struct(q, knobs=settings)
    st, res = eng.wait(eng.submit(op, pb, g, fa))            # warm-up
    assert st == 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [eng.wait(eng.submit(op, pb, g, fa)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / args.steps
    res = results[-1][1]
    inner = [int(res.inner_done[k]) for k in range(res.outer_done)]
    n = p.n_x
    nx, ny, nz = p.dims
    truth = np.asarray(p.f_true, dtype=np.float64).ravel()
    a = fa.cpu().numpy().astype(np.float64)
    b = f_fixed.cpu().numpy().astype(np.float64)
    return {"ms_per_reconstruction": el * 1e3, "outer_done": int(res.outer_done),
            "inner_done": inner, "voxel_iters": n * sum(inner),
            "voxel_iters_per_s": n * sum(inner) / el,
            "fixed_count_voxel_iters": n * p.outer * p.inner,
            "rel_l2_vs_fixed_count": float(np.linalg.norm(a - b) / np.linalg.norm(b)),
            "rel_error_vs_truth": float(np.linalg.norm(a - truth) / np.linalg.norm(truth)),
            "fixed_count_rel_error_vs_truth": float(np.linalg.norm(b - truth) / np.linalg.norm(truth)),
            "rule": "S4 eta=1.1, delta=noise norm, inner cap as configured; outer stop rtol=0 from k=3"}


C4_A_BYTES_PER_VOXEL_ITER = {"bf16_refined": 1024, "bf16": 512}   # A_hi (+ A_lo) per product pair
STENCIL_BYTES_PER_VOXEL_ITER = 75                                   # vectors, multigrid, update


def c4_oracle_sample(probs, A, which=(0, 63), target_s=15.0):
    """The FP64 oracle on instances of the batched family: its first outer iteration with S
    inner iterations, S sized so that one instance takes about target_s seconds. Returns
    (cpu_baseline record, S, {instance: f})."""
    import numpy as np
    from threadpoolctl import threadpool_info
    from oracle import lagged, multigrid
    from oracle.operators import Dense

    p0 = probs[which[0]]
    nx, ny, nz = p0.dims
    shape = (nz, ny, nx)
    op = Dense(A, shape)                       # one FP64 copy of A serves every sample (untimed)
    sm = multigrid.Smoother(p0.smoother, p0.nu_pre, p0.nu_post, p0.omega)

    def run(p, inner):
        t0 = time.perf_counter()
        f, _ = lagged.solve(shape, op, np.asarray(p.g, dtype=np.float64), p.reg, p.T, p.tau, p.eps,
                            1, inner, p.levels, sm)
        return time.perf_counter() - t0, f

    t2, _ = run(p0, 2)
    per_iter = max(t2 / 3.0, 1e-3)            # setup and initialisation cost about one step
    S = int(min(p0.inner, max(4, round(target_s / per_iter) - 1)))
    refs, times = {}, []
    for i in which:
        t, refs[i] = run(probs[i], S)
        times.append(t)
        print(f"[bench] oracle instance {i}: 1 x {S} in {t:.1f} s", file=sys.stderr, flush=True)
    threads = [x.get("num_threads", 1) for x in threadpool_info() if x.get("user_api") == "blas"]
    n = nx * ny * nz
    rec = {"value": n * S * len(which) / sum(times), "unit": "voxel-iter/s",
           "cores": int(max(threads) if threads else 1), "kind": "oracle",
           "sample": f"instances {', '.join(map(str, which))} one at a time, first outer iteration "
                     f"with {S} inner iterations each (setup included), {sum(times):.1f} s, FP64 "
                     f"NumPy/SciPy on the FP64 matrix, host cores: {len(os.sched_getaffinity(0))}"}
    return rec, S, refs


def c5_oracle_sample(temps, sizes=(32, 32, 48)):
    """The FP64 oracle on whole requests of the served family (their full outer x inner counts):
    the first templates of the given grid sizes, one at a time. Returns (cpu_baseline record,
    {template index: f})."""
    from threadpoolctl import threadpool_info
    from oracle import lagged

    picks, want = [], list(sizes)
    for k, p in enumerate(temps):
        if p.dims[0] in want:
            picks.append(k)
            want.remove(p.dims[0])
    refs, work, t_all = {}, 0, 0.0
    for k in picks:
        p = temps[k]
        t0 = time.perf_counter()
        refs[k], _ = lagged.solve_problem(p)
        t = time.perf_counter() - t0
        t_all += t
        work += p.n_x * p.outer * p.inner
        print(f"[bench] oracle request template {k} ({p.dims[0]}^3, {p.outer} x {p.inner}): "
              f"{t:.1f} s", file=sys.stderr, flush=True)
    threads = [x.get("num_threads", 1) for x in threadpool_info() if x.get("user_api") == "blas"]
    rec = {"value": work / t_all, "unit": "voxel-iter/s",
           "cores": int(max(threads) if threads else 1), "kind": "oracle",
           "sample": f"requests of {', '.join(f'{temps[k].dims[0]}^3' for k in picks)} one at a "
                     f"time at their full counts ({temps[picks[0]].outer} x "
                     f"{temps[picks[0]].inner}, setup included), {t_all:.1f} s, FP64 NumPy/SciPy, "
                     f"host cores: {len(os.sched_getaffinity(0))}"}
    return rec, refs


def bench_c4(args):
    """64 reconstructions of 64^3 sharing one 8192 x 262144 sensitivity, batched in lockstep
    with the dense products on MFMA (BF16 split products), against the same instances run
    one at a time on the FP32 path; the FP64 oracle timed on a sample and compared with the
    batched GPU result on the same sample."""
    import numpy as np
    import torch
    from gen.configs import c4_matrix, config_c4_batch
    from paper_1308_6634_amd import plsqr as P
    from paper_1308_6634_amd.engine import Engine, problem_struct

    B = 64
    t_gen = time.perf_counter()
    A = c4_matrix(64)
    probs = config_c4_batch(A, B)
    p0 = probs[0]
    n, m = p0.n_x, A.shape[0]
    print(f"[bench] c4 inputs generated in {time.perf_counter() - t_gen:.1f} s", file=sys.stderr,
          flush=True)
    prec = P.PLSQR_PREC_BF16_REFINED if args.precision == "bf16_refined" else P.PLSQR_PREC_BF16
    desc = (f"c4: 64 instances x 64^3, shared dense ring sensitivity {m}x{n} (8 source rings x 16, "
            f"4 detector rings x 16, mu=0.5), own ellipsoid phantom / noise / regulariser "
            f"(sTV 0.02 or PM-log 0.05), tau=20, 8 outer x 40 inner, 5-level Jacobi V(2,2); "
            f"products {args.precision} on MFMA")
    print(f"[bench] workload {desc}", file=sys.stderr, flush=True)
    eng = Engine(0)
    A_dev = torch.from_numpy(A).cuda()
    op = eng.dense_operator(p0.dims, A_dev)
    gs = [torch.from_numpy(np.ascontiguousarray(p.g, dtype=np.float32)).cuda() for p in probs]
    fs = [torch.zeros(n, device="cuda") for _ in probs]

    def run_batch(pbs):
        ts = eng.submit_batch(op, pbs, gs, fs)
        res = [eng.wait(t) for t in ts]
        for st, _ in res:
            assert st == 0, P.plsqr_last_error(eng.handle)
        return res

    settings = {}
    if not args.no_tune:
        # V-cycle launch schedule for this batch, by the V-cycle phase time of a short batch
        # (8 V-cycles per trial, the better of two runs)
        from paper_1308_6634_amd import autotune
        short = [dataclasses.replace(p, outer=1, inner=8) for p in probs]

        def vcycle_ms(vs):
            res = run_batch([problem_struct(p, flags=P.PLSQR_FLAG_TIME_PHASES, precision=prec,
                                            knobs=vs) for p in short])
            return res[0][1].vcycle_ms
        settings, _ = autotune.tune_vcycle(vcycle_ms, repeats=2)
        print(f"[bench] autotuned V-cycle: {settings}", file=sys.stderr, flush=True)
    settings.update(args.knobs)
    pbs = [problem_struct(p, precision=prec, knobs=settings) for p in probs]
    for _ in range(args.warmup):
        run_batch(pbs)
    print("[bench] warmup done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [run_batch(pbs) for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = B * n * p0.outer * p0.inner * args.steps / elapsed
    # one more batch with every phase timed (not part of the timed steps): the product launch
    # times of the roofline and the phase split
    ph = run_batch([problem_struct(p, flags=P.PLSQR_FLAG_TIME_PHASES, precision=prec,
                                   knobs=settings)
                    for p in probs])[0][1]
    fwd_ms = ph.forward_ms / max(ph.forward_launches, 1)
    adj_ms = ph.adjoint_ms / max(ph.adjoint_launches, 1)
    lo = 2 if prec == P.PLSQR_PREC_BF16_REFINED else 1
    # A (hi and lo parts) and the packed right operand, plus the previous step's f, w update that
    # the packing applies (16 B per voxel and instance, every inner step but the first of an
    # outer iteration)
    fwd_bytes = (lo * 2 * m * n + 2 * 2 * 64 * n
                 + 16 * B * n * (p0.inner - 1) / p0.inner)
    fwd_flops = 2.0 * m * n * 64 * (lo + 1)
    print(f"[bench] batched: {elapsed / args.steps * 1e3:.1f} ms per batch; forward product "
          f"{fwd_ms:.3f} ms, adjoint {adj_ms:.3f} ms", file=sys.stderr, flush=True)

    phases = {"setup_ms": ph.setup_ms, "forward_ms": ph.forward_ms, "adjoint_ms": ph.adjoint_ms,
              "vcycle_ms": ph.vcycle_ms, "update_ms": ph.update_ms, "diag_ms": ph.diag_ms,
              "device_ms": ph.device_ms, "inner_steps": int(ph.phase_launches)}

    # plain comparison: the same instances one at a time, FP32 products
    pl = [problem_struct(p, flags=0) for p in probs[:args.plain_sample]]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for i, pb in enumerate(pl):
        st, _ = eng.wait(eng.submit(op, pb, gs[i], torch.zeros(n, device="cuda")))
        assert st == 0
    torch.cuda.synchronize()
    plain_s = (time.perf_counter() - t1) / len(pl) if pl else None
    plain_value = n * p0.outer * p0.inner / plain_s if pl else None
    bpvi = C4_A_BYTES_PER_VOXEL_ITER[args.precision] + STENCIL_BYTES_PER_VOXEL_ITER
    out = {
        "metric": "voxel-LSQR-iters/s", "value": value, "unit": "voxel-iter/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": desc, "instances": B, "n_x": n, "n_y": m, "outer": p0.outer,
                   "inner": p0.inner, "precision": args.precision + " products, fp32 vectors, "
                   "fp64 scalars", "autotuned": settings},
        "roofline": {"bound": "hbm", "kernel": "forward product (k_pack_split + k_gemm_bf16 + "
                     "k_fwd_reduce)", "achieved": fwd_bytes / (fwd_ms / 1e3) / 1e9,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": fwd_bytes / (fwd_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                     "traffic": traffic_for("c4", "forward_" + args.precision), "bytes_per_launch": fwd_bytes,
                     "avg_launch_ms": fwd_ms, "adjoint_avg_launch_ms": adj_ms,
                     "mfma_tflops": fwd_flops / (fwd_ms / 1e3) / 1e12, "mfma_peak_tflops": 2500.0,
                     "whole_step": {"bytes_per_voxel_iter": bpvi,
                                    "achieved_GBps": value * bpvi / 1e9,
                                    "frac": value * bpvi / 1e9 / HBM_PEAK_GBS}},
        "phases_ms_one_batch": phases,
        "plain_fp32_one_at_a_time": {"value": plain_value, "unit": "voxel-iter/s",
                                     "sample": f"instances 0..{len(pl) - 1} of the {B}, FP32 "
                                               f"products", "s_per_instance": plain_s}
        if pl else None,
        "batched_over_plain": value / plain_value if pl else None,
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on a sample", file=sys.stderr, flush=True)
        cb, S, refs = c4_oracle_sample(probs, A)
        out["cpu_baseline"] = cb
        # the same sample on the GPU: the whole batch at 1 outer x S inner, same precision
        run_batch([problem_struct(dataclasses.replace(p, outer=1, inner=S), precision=prec,
                                  knobs=settings)
                   for p in probs])
        errs = {}
        for i, f_ref in refs.items():
            fg = fs[i].cpu().numpy().astype(np.float64).reshape(f_ref.shape)
            errs[str(i)] = float(np.linalg.norm(fg - f_ref) / np.linalg.norm(f_ref))
        out["parity_sample_rel_l2"] = max(errs.values())
        out["parity_sample"] = {"instances": errs, "outer": 1, "inner": S, "bar": 5e-3}
    eng.close()
    print(json.dumps(out), flush=True)


def bench_c3_batch(args):
    """B reconstructions of the c3 workload (own phantom and noise per seed) advanced in
    lockstep: one launch of every stencil, blur and multigrid kernel serves all B instances,
    so each launch moves B times the single-instance bytes (for B >= 4 the vectors no longer
    fit the 256 MB last-level cache)."""
    import numpy as np
    import torch
    import gen
    from paper_1308_6634_amd import plsqr as P
    from paper_1308_6634_amd.engine import Engine, problem_struct

    B = args.batch
    print(f"[bench] c3 batch: generating {B} instances", file=sys.stderr, flush=True)
    probs = [gen.config_c3(seed=2 + i) for i in range(B)]
    p0 = probs[0]
    n = p0.n_x
    _, desc = workload("c3")
    eng = Engine(0)
    settings = {}
    if not args.no_tune:
        from paper_1308_6634_amd import autotune
        settings, _ = autotune.tune(p0, eng)
        probs = [autotune.apply(p, settings) for p in probs]
        print(f"[bench] autotuned on instance 0: {settings}", file=sys.stderr, flush=True)
    op = eng.blur_operator(p0.dims, p0.taps)
    gs = [torch.from_numpy(np.ascontiguousarray(p.g, dtype=np.float32).ravel()).cuda() for p in probs]
    fs = [torch.zeros(n, device="cuda") for _ in probs]
    flags = P.PLSQR_FLAG_TIME_PRODUCTS | (P.PLSQR_FLAG_NO_GRAPHS if args.no_graphs else 0)
    pbs = [problem_struct(p, flags=flags, knobs=settings) for p in probs]

    def run_batch():
        ts = eng.submit_batch(op, pbs, gs, fs)
        res = [eng.wait(t) for t in ts]
        for st, _ in res:
            assert st == 0, P.plsqr_last_error(eng.handle)
        return res

    for _ in range(args.warmup):
        run_batch()
    print("[bench] warmup done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [run_batch() for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = B * n * p0.outer * p0.inner * args.steps / elapsed
    r0 = [res[0][1] for res in results]
    fwd_s = sum(r.forward_ms for r in r0) / max(sum(r.forward_launches for r in r0), 1) / 1e3
    nbytes, kname, pass_bytes = dominant_bytes(p0, blur_update_fused(p0, settings, B))
    nbytes *= B
    pass_bytes *= B
    achieved = nbytes / fwd_s / 1e9
    out = {
        "metric": "voxel-LSQR-iters/s", "value": value, "unit": "voxel-iter/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"c3 x {B} lockstep: {desc}; seeds 2..{1 + B}", "instances": B,
                   "n_x": n, "n_y": n, "outer": p0.outer, "inner": p0.inner,
                   "precision": "fp32 vectors, fp64 scalars", "autotuned": settings},
        "roofline": {"bound": "hbm", "kernel": kname + f" over {B} instances", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "bytes_per_launch": nbytes,
                     "kernel_bytes_per_launch": pass_bytes, "avg_launch_ms": fwd_s * 1e3,
                     "launches": int(sum(r.forward_launches for r in r0))},
    }
    eng.close()
    print(json.dumps(out), flush=True)


def _replay(eng, arrivals, reqs, poll_sleep=0.002):
    """Submit reqs[i] at arrivals[i] seconds from now (one thread) while another thread
    polls; returns per-request (latency ms, status) and the wall span."""
    import threading
    n = len(reqs)
    tickets = [None] * n
    done = [None] * n
    t0 = time.perf_counter()
    t_sub = [0.0] * n

    def submitter():
        for i, (op, pb, g, f) in enumerate(reqs):
            dt = t0 + arrivals[i] - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            t_sub[i] = time.perf_counter()
            tickets[i] = eng.submit(op, pb, g, f)

    th = threading.Thread(target=submitter)
    th.start()
    remaining = set(range(n))
    while remaining:
        for i in list(remaining):
            if tickets[i] is None:
                continue
            st, res = eng.poll(tickets[i])
            if st != 1:
                # latency from the scheduled arrival (a late submit counts against the path)
                t_end = t_sub[i] + (res.submit_to_done_ms / 1e3 if res is not None else 0.0)
                mixed = res.mixed_steps if res is not None else 0
                done[i] = ((t_end - (t0 + arrivals[i])) * 1e3, st, t_end, mixed)
                remaining.discard(i)
        time.sleep(poll_sleep)
    th.join()
    span = max(d[2] for d in done) - t0
    return done, span


def bench_c5(args):
    """Served stream: Poisson arrivals (mean 20 ms), grid sizes 32..128^3, blur sigma
    U(1.5,3.5), regulariser and tau per request, 8 x 40; continuous batching engine
    against the plain one-request-at-a-time path on a prefix of the same stream."""
    import numpy as np
    import torch
    import gen
    from gen.configs import c5_request
    from paper_1308_6634_amd import plsqr as P
    from paper_1308_6634_amd.engine import Engine, problem_struct

    N, NT = args.requests, args.templates
    arrivals = gen.config_c5_requests(count=N)
    print(f"[bench] c5: generating {NT} request templates", file=sys.stderr, flush=True)
    temps = [c5_request(r) for r in range(NT)]
    desc = (f"{N} Poisson requests (mean gap 20 ms) cycling through {NT} seeded reconstructions: "
            f"grid uniform over {{32,48,64,96,128}}^3, blur sigma U(1.5,3.5) radius ceil(3 sigma), "
            f"10 boxes/spheres, 1% noise, Tikhonov / sTV 0.02 / PM-log 0.05, tau U(10,100), 8x40, "
            f"auto levels, Jacobi V(2,2); HBM budget 200 GB")
    gs = [torch.from_numpy(np.ascontiguousarray(p.g, dtype=np.float32).ravel()).cuda() for p in temps]
    work = [p.n_x * p.outer * p.inner for p in temps]

    def build(eng, count):
        ops = [eng.blur_operator(p.dims, p.taps) for p in temps]
        pbs = [problem_struct(p) for p in temps]
        out = []
        for i in range(count):
            k = i % NT
            out.append((ops[k], pbs[k], gs[k], torch.zeros(temps[k].n_x, device="cuda")))
        return out

    srv = Engine(0, hbm_budget_bytes=200 * 10**9, flags=P.PLSQR_ENGINE_SERVE)
    warm = build(srv, NT)
    _replay(srv, np.zeros(NT), warm)            # warm-up: every template once
    reqs = build(srv, N)
    torch.cuda.synchronize()
    print("[bench] c5: serving the stream", file=sys.stderr, flush=True)
    done, span = _replay(srv, arrivals, reqs)
    srv.close()
    lat = np.array([d[0] for d in done])
    assert all(d[1] == 0 for d in done)
    total = sum(work[i % NT] for i in range(N))
    served_value = total / span
    # inner steps that ran in launches shared with requests of other grids
    mixed_share = sum(d[3] for d in done) / sum(temps[i % NT].outer * temps[i % NT].inner
                                                for i in range(N))

    plain = Engine(0, hbm_budget_bytes=200 * 10**9)
    M = min(args.plain_requests, N)
    preqs = build(plain, M)
    print(f"[bench] c5: plain path on the first {M} requests", file=sys.stderr, flush=True)
    pdone, pspan = _replay(plain, arrivals[:M], preqs)
    plain.close()
    plat = np.array([d[0] for d in pdone])
    ptotal = sum(work[i % NT] for i in range(M))
    out = {
        "metric": "voxel-LSQR-iters/s", "value": served_value, "unit": "voxel-iter/s",
        "n_gpus": 1, "steps": N, "warmup": NT, "ms_per_step": span / N * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic", "config": {"workload": f"c5: {desc}"},
        "served": {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                   "requests": N, "span_s": span, "voxel_iters_per_s": served_value,
                   "mixed_grid_step_share": mixed_share},
        "plain": {"p50_ms": float(np.percentile(plat, 50)), "p99_ms": float(np.percentile(plat, 99)),
                  "requests": M, "span_s": pspan, "voxel_iters_per_s": ptotal / pspan},
        "served_over_plain_throughput": served_value / (ptotal / pspan),
    }
    if not args.no_cpu_baseline:
        # the oracle on a few whole requests of the stream, timed, and compared with what the
        # served path returned for the same requests (request k of the stream is template k)
        print("[bench] c5: timing the FP64 oracle on whole requests", file=sys.stderr, flush=True)
        cb, refs = c5_oracle_sample(temps)
        out["cpu_baseline"] = cb
        errs = {}
        for k, f_ref in refs.items():
            got = reqs[k][3].cpu().numpy().astype(np.float64).reshape(f_ref.shape)
            errs[f"template {k} ({temps[k].dims[0]}^3)"] = float(
                np.linalg.norm(got - f_ref) / np.linalg.norm(f_ref))
        out["parity_sample_rel_l2"] = max(errs.values())
        out["parity_sample"] = {"requests": errs, "outer": temps[0].outer, "inner": temps[0].inner,
                                "bar": 1e-3, "path": "served"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
