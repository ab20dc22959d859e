"""Benchmark: exact multidimensional range queries on one MI355X.

Default workload: 10^8 rows x 17 float32 columns (8 uniform, 8 Gaussian-mixture,
1 Zipf) and 1,000 queries on 2-8 dims with target selectivity log-uniform in
[1e-5, 0.2].  One step answers the whole query set (count + ascending uint32 ids per
query) through the C ABI; data are resident in HBM before timing starts.

Prints one JSON line.  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "tuples/s & HBM GB/s per query; batched+learned vs plain queries/s; p99 latency"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def source_hash(path: str) -> str:
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def counters_traffic(kernel_src: str, workload: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were taken
    on the current kernel source; otherwise None."""
    path = os.path.join(ROOT, "profiles", f"scan_{workload}_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        c = json.load(f)
    if c.get("kernel_source_sha256_16") != source_hash(kernel_src):
        return None
    return c.get("hbm_bytes_per_launch")


COPY_BYTES = 1 << 30   # calibration copy for the HBM byte counters


def summarize(outdir: str, workload: str):
    """Turn rocprofv3 CSV output under `outdir` (kernel stats, and FETCH_SIZE /
    WRITE_SIZE counter runs) into the short summaries kept under profiles/.  Counter
    values are scaled by what the same counter reads for the calibration copy of
    COPY_BYTES bytes."""
    import csv
    import glob

    prof = os.path.join(ROOT, "profiles")
    os.makedirs(prof, exist_ok=True)
    cmd = os.environ.get("MDRQ_PROFILE_CMD", "")
    for path in glob.glob(os.path.join(outdir, "**", "*kernel_stats.csv"), recursive=True):
        with open(path) as f:
            rows = list(csv.DictReader(f))
        kind = {"c3": "batch", "c4": "learned", "c5": "serve"}.get(workload, "scan")
        out = os.path.join(prof, f"{kind}_{workload}_kernel_stats.txt")
        with open(out, "w") as f:
            f.write("rocprofv3 --kernel-trace --stats summary\n")
            f.write(f"command: {cmd}\n")
            if kind in ("batch", "learned", "serve"):
                f.write("note: the first shared scan of each batch shape runs every autotuner "
                        "candidate once; the shared-scan kernels with more calls than the "
                        "others are the configurations it kept\n")
            f.write("\n")
            f.write(f"{'kernel':72s} {'calls':>7s} {'avg_us':>10s} {'total_ms':>10s} {'pct':>6s}\n")
            for r in rows:
                f.write(f"{r.get('Name', '')[:72]:72s} {int(r.get('Calls', 0)):7d} "
                        f"{float(r.get('AverageNs', 0)) / 1e3:10.2f} "
                        f"{float(r.get('TotalDurationNs', 0)) / 1e6:10.3f} "
                        f"{float(r.get('Percentage', 0)):6.2f}\n")
        log("wrote", out)
    per = {}       # (counter, kernel) -> values in KiB per dispatch
    calib = {}     # counter -> largest copy-kernel value (the calibration copy)
    for path in glob.glob(os.path.join(outdir, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as f:
            for r in csv.DictReader(f):
                c, k, v = r["Counter_Name"], r["Kernel_Name"], float(r["Counter_Value"])
                per.setdefault((c, k), []).append(v)
                if "copyBuffer" in k:
                    calib[c] = max(calib.get(c, 0.0), v)
    if not per:
        return
    factor = {c: COPY_BYTES / 1024 / v for c, v in calib.items() if v > 0}
    out = os.path.join(prof, f"scan_{workload}_counters.txt")
    summary = {"kernel_source_sha256_16": source_hash(os.path.join(
        ROOT, "paper_1801_03644_amd", "csrc", "scan.hip")), "scale": factor,
        "copy_bytes": COPY_BYTES, "per_kernel_bytes": {}}
    with open(out, "w") as f:
        f.write("rocprofv3 --pmc summary (KiB per dispatch, then bytes after scaling by the "
                f"calibration copy of {COPY_BYTES} bytes)\n")
        f.write(f"command: {cmd}\n")
        f.write(f"scale factors: {json.dumps(factor)}\n\n")
        for (c, k), v in sorted(per.items()):
            mean = float(np.mean(v))
            scaled = mean * 1024 * factor.get(c, 1.0)
            summary["per_kernel_bytes"].setdefault(k, {})[c] = scaled
            f.write(f"{k[:72]:72s} {c:10s} n={len(v):4d} mean={mean:14.1f} KiB "
                    f"-> {scaled / 1e9:9.4f} GB\n")
    for k, d in summary["per_kernel_bytes"].items():
        if k.startswith("void mdrq::(anonymous namespace)::scan_kernel<3, 8>"):
            summary["hbm_bytes_per_launch"] = d.get("FETCH_SIZE", 0.0) + d.get("WRITE_SIZE", 0.0)
    with open(os.path.join(prof, f"scan_{workload}_counters.json"), "w") as f:
        json.dump(summary, f, indent=1)
    log("wrote", out)


def cpu_baseline(cols_raw, queries, n_rows, budget_s: float, all_cores: bool = True):
    """The oracle on the host: single-threaded over the first queries for about
    budget_s seconds; then (all_cores) the same unchanged single-threaded oracle on
    one query per thread, all host threads (at most 16), for about half that."""
    import threading

    import oracle

    cols = oracle.prepare(cols_raw)
    t0 = time.perf_counter()
    done = 0
    for q in queries:
        oracle.count(cols, q)
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    line = {"value": n_rows * done / dt, "unit": "tuples/s", "cores": 1, "kind": "oracle",
            "sample": f"first {done} of the {len(queries)} queries on the full {n_rows}-row data, "
                      f"single-threaded oracle scan ({dt:.1f} s)",
            "queries_per_s": done / dt}
    if all_cores:
        # The oracle's C scan runs outside the interpreter lock, so threads scale.
        n_threads = max(1, min(16, os.cpu_count() or 1))
        lock = threading.Lock()
        state = {"next": 0, "done": 0}
        stop_at = time.perf_counter() + budget_s / 2

        def worker():
            while time.perf_counter() < stop_at:
                with lock:
                    i = state["next"]
                    state["next"] += 1
                oracle.count(cols, queries[i % len(queries)])
                with lock:
                    state["done"] += 1

        t1 = time.perf_counter()
        threads = [threading.Thread(target=worker) for _ in range(n_threads)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        dt1 = time.perf_counter() - t1
        line["all_cores"] = {"value": n_rows * state["done"] / dt1, "unit": "tuples/s",
                             "cores": n_threads, "queries_per_s": state["done"] / dt1,
                             "sample": f"{state['done']} queries, one per thread, "
                                       f"{n_threads} threads ({dt1:.1f} s)"}
    return line


def device_info():
    """The GPU the line was measured on (torch's view of it)."""
    import torch

    p = torch.cuda.get_device_properties(0)
    info = {"name": p.name, "arch": getattr(p, "gcnArchName", ""),
            "compute_units": p.multi_processor_count, "memory_gib": round(p.total_memory / 2**30, 1)}
    for k in ("L2_cache_size", "shared_memory_per_block", "shared_memory_per_multiprocessor",
              "clock_rate"):
        if hasattr(p, k):
            info[k] = getattr(p, k)
    return info


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4", "c5", "syntuni"])
    ap.add_argument("--rows", type=int, default=None, help="override the row count")
    ap.add_argument("--queries", type=int, default=None)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-earlyout", action="store_true")
    ap.add_argument("--unroll", type=int, default=None)
    ap.add_argument("--blocks-per-cu", type=int, default=None,
                    help="single-query scans: workgroups per CU (MDRQ_OPT_BLOCKS_PER_CU)")
    ap.add_argument("--graphs", type=int, default=None,
                    help="MDRQ_OPT_GRAPHS: bit 0 single queries, bit 1 shared scans replayed from graphs")
    ap.add_argument("--counters", type=int, default=0, metavar="Q",
                    help="counter-collection run: Q queries once (c3: three shared scans of Q "
                         "queries with ids output), plus a plain copy of known size for "
                         "calibration; prints no bench line")
    ap.add_argument("--summarize", metavar="DIR", default=None,
                    help="summarise rocprofv3 CSV output found under DIR into profiles/")
    ap.add_argument("--train-queries", type=int, default=200_000, help="c4: training queries")
    ap.add_argument("--test-queries", type=int, default=10_000, help="c4: held-out queries")
    ap.add_argument("--epochs", type=int, default=20, help="c4/c5: estimator epochs")
    ap.add_argument("--rates", default="2000,10000,50000", help="c5: arrival rates (queries/s)")
    ap.add_argument("--serve-seconds", type=float, default=2.0, help="c5: seconds per rate")
    ap.add_argument("--segments", default="4",
                    help="c5: circular-scan parts per pass to serve each rate with as well (comma list)")
    ap.add_argument("--circular-modes", default="4,0",
                    help="c5: MDRQ_OPT_CIRCULAR values to serve the circular scan with (comma list)")
    args = ap.parse_args()
    if args.summarize:
        summarize(args.summarize, args.workload)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(row sharding across GPUs is a design note, not code).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1801_03644_amd import datagen as dg
    from paper_1801_03644_amd import mdrq
    from paper_1801_03644_amd.metrics import HBM_PEAK_GBPS

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.workload in ("c3", "c4", "c5", "syntuni"):
        import bench_extra

        line = {"c3": bench_extra.batched, "c4": bench_extra.learned,
                "c5": bench_extra.serving, "syntuni": bench_extra.paper}[args.workload](args)
        if line is None:   # a counter-collection run
            return
        line["device"] = device_info()
        print(json.dumps(line), flush=True)
        return
    w = dg.workload(args.workload, args.rows)
    n_q = args.queries or (100 if args.workload == "c1" else 1000)
    log(f"generating {w.name}: {w.n_rows} x {w.n_dims}")
    t0 = time.perf_counter()
    raw = w.columns()
    log(f"generated in {time.perf_counter() - t0:.1f}s; drawing {n_q} queries")
    queries = dg.workload_queries(w, n_q)
    log("loading into HBM")
    ds = mdrq.Dataset.from_host(raw)
    if args.unroll:
        ds.set_option(mdrq.OPT_UNROLL, args.unroll)
    if args.graphs is not None:
        ds.set_option(mdrq.OPT_GRAPHS, args.graphs)
    if args.blocks_per_cu:
        ds.set_option(mdrq.OPT_BLOCKS_PER_CU, args.blocks_per_cu)
    flags = mdrq.Q_NO_EARLYOUT if args.no_earlyout else 0
    out = torch.empty(w.n_rows, dtype=torch.int32, device="cuda:0")
    prepared = [mdrq.make_query(q, flags) for q in queries]
    lib = mdrq.load_library()
    import ctypes

    stream = mdrq._stream_handle(torch.cuda.current_stream())
    res = mdrq.Result()
    res.mode, res.mem, res.buf, res.buf_bytes = mdrq.OUT_IDS, mdrq.MEM_DEVICE, out.data_ptr(), out.numel() * 4
    counts = np.zeros(n_q, dtype=np.int64)
    lat = np.zeros(n_q)

    def step(record: bool):
        for i, (q, keep) in enumerate(prepared):
            t = time.perf_counter()
            rc = lib.mdrq_query(ds.handle, ctypes.byref(q), ctypes.byref(res), stream)
            if record:
                lat[i] = time.perf_counter() - t
            if rc not in (mdrq.OK, mdrq.EOVERFLOW):
                raise mdrq.MdrqError(rc, mdrq.last_error())
            counts[i] = res.count

    if args.counters:
        for q, keep in prepared[:args.counters]:
            rc = lib.mdrq_query(ds.handle, ctypes.byref(q), ctypes.byref(res), stream)
            if rc not in (mdrq.OK, mdrq.EOVERFLOW):
                raise mdrq.MdrqError(rc, mdrq.last_error())
        src = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        ks = [len(q[0]) for q in queries[:args.counters]]
        log(f"counters run done: {args.counters} queries, mean k {np.mean(ks):.3f}; "
            f"copy of {COPY_BYTES} bytes")
        ds.close()
        return

    for s in range(args.warmup):
        step(False)
        log(f"warmup step {s + 1}/{args.warmup} done")
    ds.set_profiling(True)
    ds.reset_profile()
    lat_all = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(True)
        lat_all.append(lat.copy())
        log(f"step {s + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    launches, scan_ms, total_ms = ds.profile()
    # The same queries with early-out off: every queried column is read in full, so the
    # algorithmic read bytes are exactly the bytes the scan must fetch.
    n_ne = min(n_q, 200)
    ne = [mdrq.make_query(q, mdrq.Q_NO_EARLYOUT) for q in queries[:n_ne]]
    ds.reset_profile()
    counts_ne = np.zeros(n_ne, dtype=np.int64)
    for i, (q, keep) in enumerate(ne):
        lib.mdrq_query(ds.handle, ctypes.byref(q), ctypes.byref(res), stream)
        counts_ne[i] = res.count
    launches_ne, scan_ms_ne, total_ms_ne = ds.profile()
    ds.set_profiling(False)
    if not np.array_equal(counts_ne, counts[:n_ne]):
        raise RuntimeError("early-out changed a result count")

    ks = np.array([len(q[0]) for q in queries])
    n_words = (w.n_rows + 63) // 64
    unroll = ds.get_option(mdrq.OPT_UNROLL)      # tile height in use (x 256 rows)
    n_tiles = (w.n_rows + 256 * unroll - 1) // (256 * unroll)   # wave tiles
    # Scan kernel writes per launch: the staged result bitmap (1 bit per row) and the
    # per-tile counts.
    write_bytes = 8 * n_words + 4 * n_tiles
    # Algorithmic reads of the early-break scan (the method's own bytes): per predicate
    # in evaluation order, the 128-byte column lines holding a row every earlier
    # predicate accepted (measured on the device, outside the timed region).
    log("measuring the early break's column bytes per query")
    read_q = np.array([ds.read_bytes(q, flags=flags) for q in queries], dtype=np.float64)
    scan_bytes_q = read_q + write_bytes
    # Logical view: every queried column read in full (no early break).
    dense_bytes_q = 4.0 * w.n_rows * ks + write_bytes
    # Whole query: the scan plus the compaction (bitmap read back, 4 B per id).
    query_bytes_q = scan_bytes_q + 8 * n_words + 4 * counts
    total_q = n_q * args.steps
    tuples_per_s = w.n_rows * total_q / elapsed
    lat_us = np.concatenate(lat_all) * 1e6
    avg_scan_s = scan_ms / 1e3 / launches
    avg_query_s = total_ms / 1e3 / launches
    achieved = scan_bytes_q.mean() / avg_scan_s / 1e9
    kernel_src = os.path.join(ROOT, "paper_1801_03644_amd", "csrc", "scan.hip")
    traffic = counters_traffic(kernel_src, w.name)
    # Streaming-read ceiling of the scan's launch shape on the same columns, this run.
    probe_dims = list(range(min(8, w.n_dims)))
    probe_ms = ds.probe_bandwidth(probe_dims, iters=5)
    probe_gbps = 4.0 * w.n_rows * len(probe_dims) / (probe_ms / 1e3) / 1e9
    sel = counts / w.n_rows
    line = {
        "metric": METRIC,
        "value": tuples_per_s,
        "unit": "tuples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.n_rows} rows x {w.n_dims} float32 columns, "
                               f"{n_q} queries per step, ids output",
                   "n_rows": w.n_rows, "n_dims": w.n_dims, "queries_per_step": n_q,
                   "mean_queried_dims": float(ks.mean()), "mean_selectivity": float(sel.mean()),
                   "early_out": not args.no_earlyout, "graphs": args.graphs or 0,
                   "unroll": unroll, "blocks_per_cu": args.blocks_per_cu or 3,
                   "data_seed": w.data_seed,
                   "query_seed": w.query_seed},
        "queries_per_s": total_q / elapsed,
        "hbm_gbps_logical": float(query_bytes_q.mean() / avg_query_s / 1e9),
        "query_device_us": avg_query_s * 1e6,
        "p50_us": float(np.percentile(lat_us, 50)),
        "p99_us": float(np.percentile(lat_us, 99)),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                     "kernel": f"scan_kernel<stage,{unroll}>", "avg_kernel_us": avg_scan_s * 1e6,
                     "algorithmic_bytes_per_launch": float(scan_bytes_q.mean()),
                     "probe_gbps": probe_gbps, "frac_of_probe": achieved / probe_gbps,
                     "logical_bytes_per_launch": float(dense_bytes_q.mean()),
                     "logical_gbps": float(dense_bytes_q.mean() / avg_scan_s / 1e9),
                     "note": "algorithmic bytes = the early break's column reads (per predicate, "
                             "the 128-byte lines holding a row every earlier predicate "
                             "accepted, measured per query by mdrq_query_read_bytes) + the "
                             "staged bitmap and tile counts written; probe = streaming read "
                             "of 8 full columns with the scan's launch shape, same run; "
                             "logical = every queried column read in full"},
    }
    if traffic:
        line["roofline"]["frac_counters"] = traffic / avg_scan_s / 1e9 / HBM_PEAK_GBPS
    bytes_ne = dense_bytes_q[:n_ne].mean()
    ach_ne = bytes_ne / (scan_ms_ne / 1e3 / launches_ne) / 1e9
    line["roofline_no_earlyout"] = {
        "bound": "hbm", "achieved": ach_ne, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
        "frac": ach_ne / HBM_PEAK_GBPS, "avg_kernel_us": scan_ms_ne / launches_ne * 1e3,
        "query_device_us": total_ms_ne / launches_ne * 1e3, "queries": n_ne}
    if not args.no_cpu_baseline:
        log("timing the CPU oracle baseline")
        line["cpu_baseline"] = cpu_baseline(raw, queries, w.n_rows, args.cpu_budget)
    line["device"] = device_info()
    ds.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
