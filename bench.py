"""Benchmark: randomized streaming SVD on one MI355X.

Workload: one GPU's row share of the randomized streaming SVD -- M = 1,048,576
rows, batches of N = 256 FP32 snapshots (16 distinct batches, cycled), K = 50
modes, oversampling p = 10, q = 2 power iterations, forget factor 0.95,
planted spectrum sigma_j = j^-1.5 over 200 modes plus Gaussian noise of
standard deviation 1e-5 (seeded synthetic data resident in HBM).

One step = one streaming update (incorporate_data) of one batch: sketch,
power iterations, projection, small SVD, lift -- every row of the hot path.

Reported: snapshot GB/s ingested by the mixed-precision path (value), the
plain FP64 GPU path on the same batches (speedup), the live roofline of the
dominant kernel from HIP events on the library's stream, and the FP64 CPU
oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COPY_BYTES = 1 << 30
MFMA_PEAK_TFLOPS = {"bf16": 2500.0, "f32": 157.3, "f64": 78.6}
FP64_VECTOR_TFLOPS = 78.6      # MI355X vector FP64 (256 CUs at 2.4 GHz)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=32)
    ap.add_argument("--warmup", type=int, default=24)   # past the clock ramp of the first updates
    ap.add_argument("--precision", default="mixed", choices=["mixed", "bf16", "fp32", "fp64"])
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-rows", type=int, default=0, help="rows of the oracle sample (0: all M rows)")
    ap.add_argument("--M", type=int, default=1 << 20)
    ap.add_argument("--graph", action="store_true",
                    help="launch each update's kernels as one captured hipGraph instead of one by one")
    ap.add_argument("--workload", default="randomized",
                    choices=["randomized", "mixed_wide", "partitioned", "burgers", "gradient", "apmos"],
                    help="randomized: the headline mixed-precision randomized stream (M = 2^20, batches of "
                         "256, K = 50, p = 10, q = 2); mixed_wide: the widest mixed-precision configuration "
                         "(M = 2^22, batches of 512, K = 100, p = 20, q = 1); partitioned: the "
                         "partitioned streaming SVD (APMOS initialisation, partition QR combination); burgers: "
                         "the partitioned stream over the closed-form Burgers snapshots (16384 x 800, FP64); "
                         "gradient: loss and reverse-mode gradient of the streamed truncated SVD (M = 2^18, "
                         "4 batches of 64, K = 20, FP32); apmos: batched APMOS over 64 row partitions "
                         "(16384 .. 262144 rows each, N = 128 FP32, r = 20, K = 20, one hipGraph)")
    ap.add_argument("--partitions", type=int, default=8)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (calibration of the HBM byte counters)")
    return ap.parse_args()


def copy_probe(reps=4):
    """A plain copy of known size: reads and writes COPY_BYTES per launch.  Under
    rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE it gives the factor between the
    counters and HBM bytes."""
    n = COPY_BYTES // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        dst.copy_(src)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    print(json.dumps({"copy_bytes_read": COPY_BYTES, "copy_bytes_written": COPY_BYTES, "launches": reps,
                      "ms_per_copy": ms, "GB_per_s_read_plus_write": 2 * COPY_BYTES / (ms * 1e-3) / 1e9}), flush=True)


def run_stream(P, w, batches, precision, steps, warmup, profile, graph=True):
    """Warm up, then time exactly `steps` updates; returns (ms/step, svd, stats).
    Every precision draws the same BF16-valued test matrices, so their results
    differ only by their arithmetic."""
    svd = P.StreamingSVD(w.M, w.K, ff=w.ff, oversampling=w.oversampling, power_iters=w.power_iters,
                         randomized=True, precision=precision, seed=w.seed, async_updates=True, profile=profile,
                         graph=graph, omega_bf16=True)
    nb = len(batches)
    views = [b.t() for b in batches]
    for i in range(warmup):
        svd.incorporate_data(views[i % nb])
    torch.cuda.synchronize()
    svd.stats()
    svd.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(warmup, warmup + steps):
        svd.incorporate_data(views[i % nb])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = svd.stats()
    return (t1 - t0) * 1e3 / steps, svd, st


def cpu_baseline(w, rows, min_seconds=10.0, max_updates=8):
    """The oracle, as it stands, on a bounded sample: steady-state updates on
    `rows` rows, repeated until `min_seconds` of CPU work (at most `max_updates`)."""
    import oracle
    import synth
    ws = synth.scaled(w, M=rows, batches=3)
    bs = synth.planted_stream(ws)
    so = oracle.StreamOracle(rows, w.K, ff=w.ff, oversampling=w.oversampling, power_iters=w.power_iters,
                             randomized=True, seed=w.seed, omega_precision=oracle.PREC_BF16)
    so.incorporate(synth.numpy_cm(bs[0]))          # initialisation, untimed
    As = [synth.numpy_cm(b) for b in bs[1:]]
    del bs
    dt, n = 0.0, 0
    while n < max_updates and (n == 0 or dt < min_seconds):
        A = As[n % len(As)]
        t0 = time.perf_counter()
        so.incorporate(A)
        dt += time.perf_counter() - t0
        n += 1
    gbs = n * rows * w.N * 4 / dt / 1e9
    return {"value": gbs, "unit": "GB/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{n} steady-state randomized updates (panel {w.K}+{w.N} columns, p={w.oversampling}, "
                      f"q={w.power_iters}) on {rows} of the {w.M} rows, FP32 snapshots; {dt:.2f} s in total",
            "seconds": dt, "updates": n}


PART_CPU_ROWS = 1 << 17


def partition_sizes(M, P, seed=7):
    """Uneven row partitions summing to M (each within +-25% of M / P, multiples of 4)."""
    g = np.random.default_rng(seed)
    w = g.uniform(0.75, 1.25, P)
    sizes = [int(4 * round(M * x / w.sum() / 4)) for x in w]
    sizes[-1] += M - sum(sizes)
    return sizes


def bench_partitioned(args):
    """Partitioned streaming SVD (the parallel variant over row partitions) on one
    GPU: FP32 deterministic updates (the QR + SVD(R) step of Algorithm 1, as the
    parallel variant runs it) with batches of 64 snapshots and K = 10 (the
    deterministic workload's panel, n = 74) on M = 2^20 rows in uneven row
    partitions; one JSON line."""
    import synth
    import paper_2108_08845_amd as P
    w = synth.scaled(synth.c1_plain_fp64(), M=args.M, batches=16, ff=0.95, dtype=torch.float32, precision="fp32")
    sizes = partition_sizes(w.M, args.partitions)
    log(f"generating {w.batches} batches of {w.M} x {w.N}; partitions {sizes}")
    batches = synth.planted_stream(w, device="cuda")
    views = []
    for b in batches:
        o, parts = 0, []
        for m in sizes:
            parts.append(b[:, o: o + m].t())
            o += m
        views.append(parts)
    torch.cuda.synchronize()
    svd = P.PartitionedStreamingSVD(sizes, w.K, ff=w.ff, r_local=w.K, precision="fp32", profile=True)
    nb = len(views)
    for i in range(args.warmup + 1):               # the first call is the APMOS initialisation
        svd.incorporate_data(views[i % nb])
    torch.cuda.synchronize()
    svd.reset_stats()
    t0 = time.perf_counter()
    for i in range(args.warmup + 1, args.warmup + 1 + args.steps):
        svd.incorporate_data(views[i % nb])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    st = svd.stats()
    kern = st["kernels"]
    dom = max(kern, key=lambda k: kern[k]["ms"])
    avg_ms = kern[dom]["ms"] / max(1, kern[dom]["launches"])
    n = w.K + w.N
    if dom == "small_svd":   # Cholesky + Jacobi SVD of the n x n R in one work-group (per launch, two per update)
        flops = 2.0 * n ** 3 + 4.0 * max(1, st["last_sweeps"]) * n ** 3
        roof = {"bound": "alu", "achieved": flops / (avg_ms * 1e-3) / 1e12, "peak": FP64_VECTOR_TFLOPS,
                "unit": "TFLOP/s"}
    elif dom == "tn":    # FP64 Gram of the panel (or of Q1): M n (n + 1) flops per pass, FP64 matrix cores
        roof = {"bound": "mfma", "achieved": w.M * n * (n + 1) / (avg_ms * 1e-3) / 1e12,
                "peak": MFMA_PEAK_TFLOPS["f64"], "unit": "TFLOP/s"}
    elif dom == "nn":    # Q1 = C R1^-1 over all partitions: reads the panel, writes Q1 (FP32)
        roof = {"bound": "hbm", "achieved": 2 * w.M * n * 4 / (avg_ms * 1e-3) / 1e9,
                "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    else:                # lift U_i = Q1_i T: reads Q1, writes U
        roof = {"bound": "hbm", "achieved": w.M * (n + w.K) * 4 / (avg_ms * 1e-3) / 1e9,
                "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = None
    roof["kernel"] = dom
    roof["avg_launch_ms"] = avg_ms
    per_kernel = {k: {"launches": v["launches"], "avg_ms": (v["ms"] / v["launches"]) if v["launches"] else 0.0}
                  for k, v in kern.items() if v["launches"]}
    svd.close()
    value = w.M * w.N * 4 / (ms * 1e-3) / 1e9
    out = {
        "metric": "snapshot GB/s ingested (partitioned streaming SVD)",
        "value": value, "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 data / f64 grams and small core", "data": "synthetic",
        "config": {"workload": f"partitioned_streaming_M{w.M}_P{len(sizes)}_N{w.N}x{w.batches}_K{w.K}_fp32", "M": w.M,
                   "partitions": sizes, "N": w.N, "K": w.K, "ff": w.ff, "parallelism": "single GPU"},
        "roofline": roof, "kernels": per_kernel,
    }
    del batches, views
    torch.cuda.empty_cache()
    if not args.no_cpu:
        import oracle
        rows = args.cpu_rows or PART_CPU_ROWS
        ws = synth.scaled(w, M=rows, batches=3)
        psz = partition_sizes(rows, args.partitions)
        bs = [synth.numpy_cm(b) for b in synth.planted_stream(ws)]
        po = oracle.PartitionedStreamOracle(psz, w.K, ff=w.ff, r_local=w.K)
        split = lambda A: [np.asfortranarray(A[sum(psz[:i]): sum(psz[:i]) + m]) for i, m in enumerate(psz)]
        po.incorporate(split(bs[0]))
        dt, nup = 0.0, 0
        while nup < 6 and (nup == 0 or dt < 10.0):
            t0 = time.perf_counter()
            po.incorporate(split(bs[1 + nup % 2]))
            dt += time.perf_counter() - t0
            nup += 1
        out["cpu_baseline"] = {"value": nup * rows * w.N * 4 / dt / 1e9, "unit": "GB/s", "cores": oracle.num_threads(),
                               "kind": "oracle",
                               "sample": f"{nup} partitioned updates on {rows} of the {w.M} rows ({len(psz)} "
                                         f"partitions, panel {w.K}+{w.N} columns); {dt:.2f} s in total"}
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


def bench_burgers(args):
    """The paper's first experiment: Burgers snapshots (Eq. (13), 16384 points x
    800 snapshots, FP64) streamed in 8 batches of 100 on 4 row partitions (K =
    20, ff = 1): APMOS initialisation, then 7 partitioned updates.  A step is one
    whole pass over the 800 snapshots; one JSON line."""
    import synth
    import paper_2108_08845_amd as P
    nx, nt, nb, K, parts = 16384, 800, 100, 20, 4
    sizes = [nx // parts] * parts
    u = synth.burgers_snapshots(nx, nt).to("cuda")
    blocks = []
    for b in range(nt // nb):
        blk = u[b * nb:(b + 1) * nb]
        blocks.append([blk[:, i * sizes[0]:(i + 1) * sizes[0]].t() for i in range(parts)])
    torch.cuda.synchronize()

    def one_pass(profile):
        svd = P.PartitionedStreamingSVD(sizes, K, ff=1.0, r_local=nb, precision="fp64", profile=profile)
        for bl in blocks:
            svd.incorporate_data(bl)
        return svd

    for _ in range(args.warmup):
        one_pass(False).close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        svd = one_pass(False)
        s = svd.singular_values
        svd.close()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    svd = one_pass(True)
    st = svd.stats()
    kern = st["kernels"]
    dom = max(kern, key=lambda k: kern[k]["ms"])
    avg_ms = kern[dom]["ms"] / max(1, kern[dom]["launches"])
    n = K + nb
    if dom == "small_svd":   # Cholesky + Jacobi SVD of the n x n R in one work-group (per launch, two per update)
        flops = 2.0 * n ** 3 + 4.0 * max(1, st["last_sweeps"]) * n ** 3
        roof = {"bound": "alu", "achieved": flops / (avg_ms * 1e-3) / 1e12, "peak": FP64_VECTOR_TFLOPS,
                "unit": "TFLOP/s"}
    elif dom == "tn":
        roof = {"bound": "mfma", "achieved": nx * n * (n + 1) / (avg_ms * 1e-3) / 1e12,
                "peak": MFMA_PEAK_TFLOPS["f64"], "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": nx * n * 8 * 2 / (avg_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                "unit": "GB/s"}
    roof.update({"frac": roof["achieved"] / roof["peak"], "traffic": None, "kernel": dom, "avg_launch_ms": avg_ms})
    per_kernel = {k: {"launches": v["launches"], "avg_ms": (v["ms"] / v["launches"]) if v["launches"] else 0.0}
                  for k, v in kern.items() if v["launches"]}
    svd.close()
    out = {
        "metric": "snapshot GB/s ingested (partitioned streaming SVD, Burgers snapshots)",
        "value": nx * nt * 8 / (ms * 1e-3) / 1e9, "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "strong",
        "vs_baseline": None, "dtype": "f64", "data": "closed-form Burgers solution (Eq. 13)",
        "config": {"workload": f"burgers_partitioned_stream_{nx}x{nt}_P{parts}_batches{nb}_K{K}_fp64",
                   "grid_points": nx, "snapshots": nt, "batch": nb, "partitions": sizes, "K": K, "ff": 1.0,
                   "parallelism": "single GPU"},
        "sigma_1_2": [float(x) for x in s[:2]],
        "roofline": roof, "kernels": per_kernel,
    }
    del blocks, u
    torch.cuda.empty_cache()
    if not args.no_cpu:
        import oracle
        A = synth.numpy_cm(synth.burgers_snapshots(nx, nt))
        dt, npass = 0.0, 0
        while npass < 20 and (npass == 0 or dt < 10.0):
            po = oracle.PartitionedStreamOracle(sizes, K, ff=1.0, r_local=nb)
            t0 = time.perf_counter()
            for b in range(nt // nb):
                po.incorporate([np.asfortranarray(A[i * sizes[0]:(i + 1) * sizes[0], b * nb:(b + 1) * nb])
                                for i in range(parts)])
            dt += time.perf_counter() - t0
            npass += 1
        out["cpu_baseline"] = {"value": npass * nx * nt * 8 / dt / 1e9, "unit": "GB/s", "cores": oracle.num_threads(),
                               "kind": "oracle",
                               "sample": f"{npass} whole passes of the oracle's partitioned stream over the same "
                                         f"snapshots; {dt:.2f} s in total"}
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


def bench_gradient(args):
    """Loss L = ||A - U U^T A||_F^2 + sum_j w_j s_j of the deterministic stream and
    its gradient dL/dA (M = 2^18 rows, 4 batches of 64 FP32 snapshots, K = 20,
    spectral gap s_20 / s_21 = 4): forward (loss only) and forward + backward
    (the backward recomputes every batch's panel from the stored incoming state)
    timed on the device; one JSON line (time-like: lower is better)."""
    import synth
    import paper_2108_08845_amd as P
    w = synth.c5_gradient()
    bs = synth.planted_stream(w, device="cuda")
    A = torch.cat(bs, dim=0).t()                  # M x (B Nb), column-major
    wt = synth.loss_weights(w)
    del bs
    torch.cuda.synchronize()

    def timed(want_grad):
        for _ in range(args.warmup):
            P.loss_and_grad(A, w.batches, w.K, w.ff, wt, want_grad=want_grad)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            L, G = P.loss_and_grad(A, w.batches, w.K, w.ff, wt, want_grad=want_grad)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / args.steps, L

    fwd_ms, L = timed(False)
    fb_ms, _ = timed(True)
    n = w.K + w.N
    panel = w.M * n * 4
    # stored between the passes: the state entering every batch (U: M x K FP32, s: K FP64)
    stored = w.batches * (w.M * w.K * 4 + w.K * 8)
    # algorithmic bytes of the forward: per batch the Gram, the second Gram (Q1), the
    # Q1 product and the lift read the panel (4 reads; Q1 written and read once more)
    fwd_bytes = w.batches * (4 * panel + 2 * w.M * n * 4)
    out = {
        "metric": "loss + gradient of the streamed truncated SVD, ms per stream (forward + backward)",
        "value": fb_ms, "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": fb_ms, "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
        "dtype": "f32 (tall products) / f64 small core", "data": "synthetic",
        "config": {"workload": w.name, "M": w.M, "N": w.N, "batches": w.batches, "K": w.K, "ff": w.ff,
                   "parallelism": "single GPU"},
        "forward_ms": fwd_ms, "forward_backward_ms": fb_ms, "stored_state_bytes": stored, "loss": L,
        "roofline": {"bound": "hbm", "achieved": fwd_bytes / (fwd_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": fwd_bytes / (fwd_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "whole forward stream (algorithmic bytes of its tall passes / stream time)"},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def bench_apmos(args):
    """Batched APMOS (Algorithm 2) on one GPU's share: 64 row partitions with
    row counts uniform in [16384, 262144], N = 128 FP32 snapshots each, local
    truncation r = 20, global K = 20, the whole sequence one captured hipGraph
    (replayed on every call after the first).  One JSON line: snapshot bytes
    per second through the call (the partitions stay resident in HBM)."""
    import synth
    import paper_2108_08845_amd as P
    w = synth.c4_apmos()
    sizes = synth.partition_sizes(w)
    parts = [p.t() for p in synth.apmos_partitions(w, device="cuda", sizes=sizes)]   # M_i x N column-major
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        P.apmos_batched(parts, w.local_rank, w.K, stream=stream)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        U, Lam, X = P.apmos_batched(parts, w.local_rank, w.K, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    rows = int(sum(sizes))
    snap_bytes = rows * w.N * 4
    # algorithmic bytes: the local Grams and the lift each read every partition
    # once; the lift writes the K local modes
    alg_bytes = 2 * snap_bytes + rows * w.K * 4
    out = {
        "metric": "batched APMOS snapshot GB/s (local Grams, eigen-decompositions, global SVD, lift; one hipGraph)",
        "value": snap_bytes / (ms * 1e-3) / 1e9, "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 (tall products) / f64 small core", "data": "synthetic",
        "config": {"workload": w.name, "partitions": w.partitions, "rows_total": rows, "N": w.N,
                   "local_rank": w.local_rank, "K": w.K, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": alg_bytes / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": alg_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "whole call (algorithmic bytes of its tall passes / call time)"},
        "global_singular_values_head": [float(x) for x in Lam[:5]],
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU per process; --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "partitioned":
        bench_partitioned(args)
        return
    if args.workload == "burgers":
        bench_burgers(args)
        return
    if args.workload == "gradient":
        bench_gradient(args)
        return
    if args.workload == "apmos":
        bench_apmos(args)
        return
    import synth
    import paper_2108_08845_amd as P

    if args.workload == "mixed_wide":
        # 8 batches of 2^22 x 512 FP32 (69 GB) resident; fewer steps (tens of ms each)
        w = synth.c3_mixed()
        args.steps = min(args.steps, 8)
        args.warmup = min(args.warmup, 2)
    else:
        w = synth.scaled(synth.c2_randomized_fp32(), M=args.M)
    log(f"generating {w.batches} batches of {w.M} x {w.N} on the GPU")
    batches = synth.planted_stream(w, device="cuda")
    torch.cuda.synchronize()
    bytes_per_step = w.M * w.N * 4

    log(f"timing {args.precision}: warmup {args.warmup}, steps {args.steps}")
    ms, svd, _ = run_stream(P, w, batches, args.precision, args.steps, args.warmup, profile=False,
                            graph=args.graph)
    s_main = svd.singular_values
    svd.close()
    value = bytes_per_step / (ms * 1e-3) / 1e9
    # Per-kernel device times from a second run of the same steps with the
    # library's event pairs around its launches (kept out of the timed run).
    log("per-kernel times (event-timed run)")
    _, svd, st = run_stream(P, w, batches, args.precision, args.steps, args.warmup, profile=True)

    # Roofline of the dominant kernel class (largest total device time).
    n = w.K + w.N
    ell = w.K + w.oversampling
    kern = st["kernels"]
    dom = max(kern, key=lambda k: kern[k]["ms"])
    avg_ms = kern[dom]["ms"] / max(1, kern[dom]["launches"])
    panel_bytes = w.M * n * 4
    if dom == "fused_bf16":
        roof = {"bound": "hbm", "achieved": panel_bytes / (avg_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    elif dom == "split":
        # split-BF16 final pass: reads the panel, writes the kept sketch Y (M x l FP32)
        roof = {"bound": "hbm", "achieved": (panel_bytes + w.M * ell * 4) / (avg_ms * 1e-3) / 1e9,
                "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    elif dom == "fused_f32":
        # power passes P = C^T (C X) on the FP32 matrix cores (the class average; the
        # FP32 precision's final pass adds 2 M l^2 for G, not counted)
        flops = 4.0 * w.M * n * ell
        roof = {"bound": "mfma", "achieved": flops / (avg_ms * 1e-3) / 1e12, "peak": MFMA_PEAK_TFLOPS["f32"],
                "unit": "TFLOP/s"}
    elif dom == "split3":
        # FP32-accurate power passes on three-term BF16 splits: the method's six
        # BF16 term products per FP32 product, 6 x 4 M n l, on the BF16 matrix cores
        flops = 6.0 * 4.0 * w.M * n * ell
        roof = {"bound": "mfma", "achieved": flops / (avg_ms * 1e-3) / 1e12, "peak": MFMA_PEAK_TFLOPS["bf16"],
                "unit": "TFLOP/s"}
    elif dom == "wide":
        # wide panels: Y = C X and C^T Y on the FP32 matrix cores, one read of the
        # panel each, 2 M n l algorithmic flops per launch
        roof = {"bound": "mfma", "achieved": 2.0 * w.M * n * ell / (avg_ms * 1e-3) / 1e12,
                "peak": MFMA_PEAK_TFLOPS["f32"], "unit": "TFLOP/s"}
    elif dom == "nn":
        # generic Y = C X (panel read, sketch written)
        roof = {"bound": "hbm", "achieved": (panel_bytes + w.M * ell * 4) / (avg_ms * 1e-3) / 1e9,
                "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    elif dom == "tn":
        # generic reductions over the rows: C^T Y (panel and sketch read) and Y^T Y
        roof = {"bound": "hbm", "achieved": (panel_bytes + w.M * ell * 4) / (avg_ms * 1e-3) / 1e9,
                "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    elif dom == "lift":
        roof = {"bound": "hbm", "achieved": (panel_bytes + w.M * w.K * 4) / (avg_ms * 1e-3) / 1e9,
                "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    elif dom in ("small", "small_svd"):
        # one work-group FP64 kernels: counted FP64 flops against the vector FP64 peak
        ncol = n
        if dom == "small":      # Cholesky-QR re-orthonormalisation of the n x l sketch
            flops = 4.0 * ncol * ell * ell + 2.0 * ell ** 3 / 3.0
        else:                   # final small SVD: three n x l products, Cholesky, inverses, Jacobi sweeps
            flops = (6.0 * ncol * ell * ell + 5.0 * ell ** 3 / 3.0 + 6.0 * ell ** 3
                     + 4.0 * max(1, st["last_sweeps"]) * ell ** 3)
        roof = {"bound": "alu", "achieved": flops / (avg_ms * 1e-3) / 1e12, "peak": FP64_VECTOR_TFLOPS,
                "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": panel_bytes / (avg_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    # HBM bytes per launch from the committed counter record of this kernel, if
    # its source has not changed since the counters were taken (else null).
    from paper_2108_08845_amd import pmc_traffic
    rec = pmc_traffic.load_current(os.path.join(ROOT, "profiles"), dom, w.name)
    roof["traffic"] = rec["traffic_bytes_per_launch"] if rec else None
    roof["kernel"] = dom
    roof["avg_launch_ms"] = avg_ms
    per_kernel = {k: {"launches": v["launches"], "avg_ms": (v["ms"] / v["launches"]) if v["launches"] else 0.0}
                  for k, v in kern.items() if v["launches"]}
    per_kernel["jacobi_sweeps_last"] = st["last_sweeps"]
    svd.close()

    out = {
        "metric": "snapshot GB/s ingested vs HBM peak; mixed vs FP64 speedup at fixed sigma error",
        "value": value,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"mixed": "bf16 pairs (mfma, f32 accumulate) / f64 small core",
                  "bf16": "bf16+f32 (mfma) / f64 small core", "fp32": "f32 (mfma) / f64 small core",
                  "fp64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": w.name, "M": w.M, "N": w.N, "batches_cycled": w.batches, "K": w.K,
                   "oversampling": w.oversampling, "power_iters": w.power_iters, "ff": w.ff,
                   "precision": args.precision, "launch": "hipGraph" if args.graph else "stream",
                   "parallelism": "single GPU"},
        "frac_of_hbm_peak_ingest": value / HBM_PEAK_GBS,
        "roofline": roof,
        "kernels": per_kernel,
    }

    if not args.no_fp64 and args.precision != "fp64":
        # "At fixed sigma error": the FP64 path runs the same algorithm on the same
        # test matrices; the sigma difference over every retained mode is the
        # error of this precision, reported beside the speedup.
        log("timing the FP64 GPU path on the same batches")
        ms64, svd64, st64 = run_stream(P, w, batches, "fp64", args.steps, args.warmup, profile=False,
                                       graph=args.graph)
        s64 = svd64.singular_values
        svd64.close()
        out["fp64_ms_per_step"] = ms64
        out["speedup_vs_fp64"] = ms64 / ms
        out["sigma_rel_diff_vs_fp64_path"] = {"modes": int(len(s64)),
                                              "max_all": float(np.max(np.abs(s_main - s64) / s64))}
        if args.precision == "mixed":
            # the unrefined BF16 sketch (plain BF16 power passes), for comparison
            log("timing the unrefined BF16 sketch on the same batches")
            msb, svdb, _ = run_stream(P, w, batches, "bf16", args.steps, args.warmup, profile=False,
                                      graph=args.graph)
            sb = svdb.singular_values
            svdb.close()
            out["bf16_sketch"] = {"ms_per_step": msb, "GB_per_s": bytes_per_step / (msb * 1e-3) / 1e9,
                                  "speedup_vs_fp64": ms64 / msb,
                                  "sigma_rel_diff_vs_fp64_path_max_all": float(np.max(np.abs(sb - s64) / s64))}

    del batches
    torch.cuda.empty_cache()
    if not args.no_cpu:
        # the wide workload's oracle update takes ~90 s on all 2^22 rows: a 2^16-row sample
        rows = args.cpu_rows or (w.M if args.workload == "randomized" else 1 << 16)
        log(f"oracle CPU baseline on {rows} rows")
        out["cpu_baseline"] = cpu_baseline(w, rows)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
