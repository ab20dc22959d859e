"""The batched, learned, serving and paper-shaped workloads of bench.py
(--workload c3 / c4 / c5 / syntuni).

Each function returns one JSON-ready dict in the same form as bench.py's line: `value`
is the configuration's headline throughput, with inputs already resident in HBM and
outputs written to HBM.  Every compared variant must return identical counts (and,
where checked, identical ids); a mismatch raises.
"""
from __future__ import annotations

import ctypes
import math
import sys
import time

import numpy as np

METRIC = "tuples/s & HBM GB/s per query; batched+learned vs plain queries/s; p99 latency"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def _line(value, unit, config, steps, warmup, ms_per_step, extra):
    d = {"metric": METRIC, "value": value, "unit": unit, "n_gpus": 1, "steps": steps,
         "warmup": warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
         "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
         "config": config}
    d.update(extra)
    return d


class Runner:
    """Prepared single-query and batch calls through the C ABI (no per-call Python
    marshalling in the timed loops).  Query i writes its ids into its own region of one
    device buffer, caps[i] ids long; the regions of each window of `window` consecutive
    queries (a batch) are disjoint, and windows reuse the buffer."""

    def __init__(self, ds, queries, caps, stream, window=1024):
        import torch

        from paper_1801_03644_amd import mdrq

        self.mdrq = mdrq
        self.lib = mdrq.load_library()
        self.ds = ds
        self.stream = stream
        self.n = len(queries)
        self.window = window
        self.caps = np.maximum(np.asarray(caps, dtype=np.int64), 1)
        off = np.zeros(self.n, dtype=np.int64)
        need = 1
        for a in range(0, self.n, window):
            c = self.caps[a:a + window]
            off[a:a + window] = np.concatenate([[0], np.cumsum(c)[:-1]])
            need = max(need, int(c.sum()))
        self.buf = torch.empty(need, dtype=torch.int32, device="cuda:0")
        self.off = off
        self.ptrs = (self.buf.data_ptr() + 4 * off).astype(np.uint64)
        self.bytes = (4 * self.caps).astype(np.uint64)
        self.keep = []
        self.q = {}
        for flags in (0, mdrq.Q_ORDER_ESTIMATED, mdrq.Q_ORDER_ESTIMATED | mdrq.Q_SIZE_ESTIMATED):
            arr = (mdrq.Query * self.n)()
            for i, q in enumerate(queries):
                qq, k = mdrq.make_query(q, flags)
                arr[i] = qq
                self.keep.append(k)
            self.q[flags] = arr
        # Result records as numpy fields, set and read per batch without a Python loop.
        self.rrec = np.zeros(self.n, dtype=mdrq._RESULT_DT)
        self.r = (mdrq.Result * self.n).from_buffer(self.rrec)
        self.counts = np.zeros(self.n, dtype=np.int64)
        self.written = np.zeros(self.n, dtype=np.int64)

    def ids(self, i):
        """The ids query i wrote in the last call that answered it."""
        return self.buf[self.off[i]:self.off[i] + int(self.written[i])]

    def check_complete(self):
        if (self.written != self.counts).any():
            raise RuntimeError("an output buffer was too small: work would be skipped")

    def plain(self, flags=0, lo=0, hi=None):
        hi = self.n if hi is None else hi
        for i in range(lo, hi):
            r = self.r[i]
            r.mode, r.mem = self.mdrq.OUT_IDS, self.mdrq.MEM_DEVICE
            r.buf = int(self.ptrs[i])
            r.buf_bytes = int(self.bytes[i])
            rc = self.lib.mdrq_query(self.ds.handle, ctypes.byref(self.q[flags][i]), ctypes.byref(r),
                                     self.stream)
            if rc not in (0, self.mdrq.EOVERFLOW):
                raise self.mdrq.MdrqError(rc, self.mdrq.last_error())
            self.counts[i] = r.count
            self.written[i] = r.written
        return self.counts[lo:hi].copy()

    def batch(self, flags=0, lo=0, hi=None, size=1024):
        hi = self.n if hi is None else hi
        for a in range(lo, hi, size):
            b = min(hi, a + size)
            rec = self.rrec[a:b]
            rec["mode"] = self.mdrq.OUT_IDS
            rec["mem"] = self.mdrq.MEM_DEVICE
            rec["buf"] = self.ptrs[a:b]
            rec["buf_bytes"] = self.bytes[a:b]
            qp = ctypes.cast(ctypes.byref(self.q[flags], a * ctypes.sizeof(self.mdrq.Query)),
                             ctypes.POINTER(self.mdrq.Query))
            rp = ctypes.cast(ctypes.byref(self.r, a * ctypes.sizeof(self.mdrq.Result)),
                             ctypes.POINTER(self.mdrq.Result))
            rc = self.lib.mdrq_query_batch(self.ds.handle, qp, b - a, rp, self.stream)
            if rc not in (0, self.mdrq.EOVERFLOW):
                raise self.mdrq.MdrqError(rc, self.mdrq.last_error())
            self.counts[a:b] = rec["count"]
            self.written[a:b] = rec["written"]
        return self.counts[lo:hi].copy()


def _exact_counts(ds, queries):
    """Exact result sizes (count-only shared scans), to size the output buffers."""
    out = []
    for a in range(0, len(queries), 1024):
        out += [x.count for x in ds.query_batch(queries[a:a + 1024], None, "count")]
    return np.array(out, dtype=np.int64)


def _setup(name, rows, graphs=None):
    import torch

    from paper_1801_03644_amd import datagen as dg
    from paper_1801_03644_amd import mdrq

    w = dg.workload(name, rows)
    log(f"generating {w.name}: {w.n_rows} x {w.n_dims}")
    t0 = time.perf_counter()
    raw = w.columns()
    log(f"generated in {time.perf_counter() - t0:.1f}s; loading into HBM")
    ds = mdrq.Dataset.from_host(raw)
    if graphs is not None:
        ds.set_option(mdrq.OPT_GRAPHS, graphs)
    stream = mdrq._stream_handle(torch.cuda.current_stream())
    return w, raw, ds, stream


def _timed(fn, reps=1):
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = fn()
    torch.cuda.synchronize()
    return out, (time.perf_counter() - t0) / reps


def _cpu(raw, queries, n_rows, budget):
    import bench

    return bench.cpu_baseline(raw, queries, n_rows, budget)


def _batch_counters_run(ds, queries, stream):
    """Counter-collection run of one shared scan: the queries' exact counts (a count-only
    batch), then three batches with ids output through the rank kernel with a fixed launch
    shape (8 waves, 512-row chunks, groups of 128), then a plain copy of known size for the
    byte counters' calibration.  Prints no bench line."""
    import torch

    from paper_1801_03644_amd import mdrq

    counts = _exact_counts(ds, queries)
    for o, v in ((mdrq.OPT_AUTOTUNE, 0), (mdrq.OPT_BATCH_VARIANT, 5), (mdrq.OPT_BATCH_WAVES, 8),
                 (mdrq.OPT_BATCH_ROWS, 8)):
        ds.set_option(o, v)
    run = Runner(ds, queries, counts, stream)
    for _ in range(3):
        run.batch(0, 0, len(queries), len(queries))
    run.check_complete()
    src = torch.empty((1 << 30) // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"counters run done: {len(queries)} queries, {int(counts.sum())} ids per batch; "
        f"copy of {1 << 30} bytes")
    return None


def batched(args):
    """c3: batches of 64, 256 and 1024 queries answered by one shared scan each, against
    the same queries one at a time through mdrq_query; ids output in both."""
    import torch

    from paper_1801_03644_amd import datagen as dg
    from paper_1801_03644_amd.metrics import (ALU_COMPARES_PEAK, COMPARES_PER_TEST, LDS_PEAK_GBPS,
                                              RANK_LDS_BYTES_PER_LOOKUP)

    w, raw, ds, stream = _setup("c3", args.rows, args.graphs)
    n_q = 1024
    queries = dg.workload_queries(w, n_q)
    ks = np.array([len(q[0]) for q in queries])
    if args.counters:
        return _batch_counters_run(ds, queries[:args.counters], stream)
    run = Runner(ds, queries, _exact_counts(ds, queries), stream)
    reps = max(1, args.steps)
    res = {}
    for Q in (64, 256, 1024):
        log(f"batch size {Q}: plain")
        run.plain(0, 0, Q)                                   # warm-up
        c_plain, t_plain = _timed(lambda: run.plain(0, 0, Q), reps)
        log(f"batch size {Q}: shared scan (the first call autotunes)")
        run.batch(0, 0, Q, Q)
        ds.reset_profile()
        c_batch, t_batch = _timed(lambda: run.batch(0, 0, Q, Q), reps)
        scans, dev_ms = ds.batch_profile()
        lookups, col_bytes, scan_ms = ds.batch_work()
        if not np.array_equal(c_plain, c_batch):
            raise RuntimeError("batched counts differ from single-query counts")
        tests = float(ks[:Q].sum()) * w.n_rows
        res[Q] = {"plain_queries_per_s": Q / t_plain, "batched_queries_per_s": Q / t_batch,
                  "speedup": t_plain / t_batch, "batch_ms": t_batch * 1e3,
                  "shared_scans_per_batch": scans / reps, "device_ms_per_batch": dev_ms / reps,
                  "row_tests_per_s": tests / (dev_ms / reps / 1e3),
                  "scan_kernel_ms_per_batch": scan_ms / reps, "rank_lookups_per_batch": lookups / reps,
                  "column_bytes_per_batch": col_bytes / reps}
        log(f"Q={Q}: plain {Q / t_plain:.0f} q/s, batched {Q / t_batch:.0f} q/s")
    # ids of a few queries of the largest batch against their single-query ids
    run.batch(0, 0, n_q, n_q)
    run.check_complete()
    check = [0, 17, 511, 1023]
    got = [run.ids(i).clone() for i in check]
    for j, i in enumerate(check):
        run.plain(0, i, i + 1)
        if not torch.equal(got[j], run.ids(i)):
            raise RuntimeError("batched ids differ from single-query ids")
    big = res[1024]
    ach = COMPARES_PER_TEST * big["row_tests_per_s"]
    lds_ach = big["rank_lookups_per_batch"] * RANK_LDS_BYTES_PER_LOOKUP / (big["scan_kernel_ms_per_batch"] / 1e3) / 1e9
    # HBM view of the same batch: every column of the union read once, ids written.
    union = len({int(d) for q in queries for d in q[0]})
    hbm_bytes = 4.0 * w.n_rows * union + 4.0 * float(run.counts.sum())
    hbm_ach = hbm_bytes / (big["device_ms_per_batch"] / 1e3) / 1e9
    line = _line(big["batched_queries_per_s"], "queries/s",
                 {"workload": f"c3: {w.n_rows} rows x {w.n_dims} float32 columns, batches of "
                              f"64/256/1024 queries (k 1..8, s 1e-5..0.2), ids output",
                  "n_rows": w.n_rows, "n_dims": w.n_dims, "mean_queried_dims": float(ks.mean()),
                  "data_seed": w.data_seed, "query_seed": w.query_seed},
                 reps, 1, big["batch_ms"],
                 {"batches": {str(k): v for k, v in res.items()},
                  "plain_queries_per_s": big["plain_queries_per_s"],
                  "roofline": {"bound": "lds", "achieved": lds_ach, "peak": LDS_PEAK_GBPS, "unit": "GB/s",
                               "frac": lds_ach / LDS_PEAK_GBPS, "traffic": None,
                               "kernel": "batch_rank_kernel (the shared scan alone, without the finish)",
                               "avg_kernel_ms": big["scan_kernel_ms_per_batch"],
                               "note": "work = per row and (group of up to 128 queries, column) one "
                                       "4-byte bucket word and one 16-byte row of query bitsets read "
                                       "from LDS (the search probes inside a bucket are data-dependent "
                                       "and not counted); peak = 128 B per clock per CU x 256 CUs x "
                                       "2.4 GHz"},
                  "roofline_alu": {"bound": "alu", "achieved": ach, "peak": ALU_COMPARES_PEAK,
                               "unit": "compares/s", "frac": ach / ALU_COMPARES_PEAK,
                               "traffic": None, "kernel": "shared scan, autotuned variant (+ finish)",
                               "note": "work = 2 compares (lo <= x, x <= hi) per row-predicate "
                                       "test, tests = sum over queries of (queried dims x rows), "
                                       "the work without early-out; peak = one 32-bit compare "
                                       "per lane and clock (256 CUs x 64 lanes x 2.4 GHz). This "
                                       "is the roof of the variants that test every (row, "
                                       "predicate); the rank variant looks each row up once per "
                                       "group of up to 128 queries and column, so its frac can "
                                       "exceed 1"},
                  "roofline_hbm": {"bound": "hbm", "achieved": hbm_ach, "peak": 8000.0,
                                   "unit": "GB/s", "frac": hbm_ach / 8000.0, "traffic": None,
                                   "note": "bytes = 4 N x union columns (each read once) + 4 x "
                                           "ids written, over the device time of the batch"}})
    if not args.no_cpu_baseline:
        log("timing the CPU oracle baseline")
        line["cpu_baseline"] = _cpu(raw, queries, w.n_rows, args.cpu_budget)
    ds.close()
    return line


def _qerror(est, true, n_rows):
    e = np.maximum(np.asarray(est, dtype=np.float64), 1.0 / n_rows)
    t = np.maximum(np.asarray(true, dtype=np.float64), 1.0 / n_rows)
    return np.maximum(e / t, t / e)


def _qstats(q):
    return {"median": float(np.median(q)), "p90": float(np.percentile(q, 90)),
            "p99": float(np.percentile(q, 99)), "max": float(q.max()),
            "geometric_mean": float(np.exp(np.log(q).mean()))}


def learned(args):
    """c4: the estimator trained on scan-labelled queries and gated on a held-out
    validation split (an output keeps its learned correction only where it lowers the
    validation error); q-error against the histogram estimates and their independence
    product (the untrained estimator returns exactly those); and queries/s of the
    held-out queries one at a time in given order, in the untrained estimator's
    (histogram) order and in the trained one's, and in shared scans of 1024 in given
    order and with the trained estimator's order and scratch sizing.  Every query's
    output buffer holds its whole result (no work skipped)."""
    from paper_1801_03644_amd import datagen as dg
    from paper_1801_03644_amd import mdrq

    w, raw, ds, stream = _setup("c4", args.rows, args.graphs)
    samp = w.sampler()
    n_tr, n_te = args.train_queries, args.test_queries
    n_va = max(1000, n_te // 2)
    train_q = dg.quantile_queries(samp, n_tr, (1, 10), (1e-5, 0.2), w.split_seed)
    val_q = dg.quantile_queries(samp, n_va, (1, 10), (1e-5, 0.2), w.split_seed + 1)
    test_q = dg.quantile_queries(samp, n_te, (3, 10), (1e-5, 0.2), w.query_seed)
    log(f"labelling {n_tr} + {n_va} + {n_te} queries with shared count scans")
    t0 = time.perf_counter()
    parts = []
    for a in range(0, n_tr, 20_000):
        parts.append(ds.label_selectivities(train_q[a:a + 20_000]))
        log(f"labelled {min(n_tr, a + 20_000)} training queries ({time.perf_counter() - t0:.1f}s)")
    s_train = np.concatenate(parts)
    s_val = ds.label_selectivities(val_q)
    s_test = ds.label_selectivities(test_q)
    t_label = time.perf_counter() - t0
    hist_est = mdrq.Estimator(ds, seed=1)              # untrained: histogram estimates
    est = mdrq.Estimator(ds, seed=1)
    base = hist_est.predict(test_q)
    log(f"training {args.epochs} epochs")
    t0 = time.perf_counter()
    losses = est.train(train_q, s_train, epochs=args.epochs, batch=256, lr=1e-3,
                       seed=w.split_seed)
    t_train = time.perf_counter() - t0
    ungated = est.predict(test_q)
    kept = est.gate(val_q, s_val)
    pred = est.predict(test_q)
    n = w.n_rows
    mask = s_test[:, :-1] >= 0
    qerr = {"joint_learned": _qstats(_qerror(pred[:, -1], s_test[:, -1], n)),
            "joint_independence": _qstats(_qerror(base[:, -1], s_test[:, -1], n)),
            "per_dim_learned": _qstats(_qerror(pred[:, :-1][mask], s_test[:, :-1][mask], n)),
            "per_dim_learned_before_gating": _qstats(_qerror(ungated[:, :-1][mask], s_test[:, :-1][mask], n)),
            "per_dim_histogram": _qstats(_qerror(base[:, :-1][mask], s_test[:, :-1][mask], n)),
            "outputs_kept": [int(j) for j in np.flatnonzero(kept)]}
    counts = _exact_counts(ds, test_q)
    run = Runner(ds, test_q, counts, stream)
    G, E = 0, mdrq.Q_ORDER_ESTIMATED
    ES = mdrq.Q_ORDER_ESTIMATED | mdrq.Q_SIZE_ESTIMATED
    variants = {}
    log("warm-up (the first shared scan of each batch shape autotunes its launch)")
    ds.attach_estimator(est)
    run.plain(G, 0, 200)
    run.plain(E, 0, 200)
    run.batch(G)
    run.batch(ES)
    ds.set_profiling(True)
    for name, fn, e in (("plain_given_order", lambda: run.plain(G), est),
                        ("plain_histogram_order", lambda: run.plain(E), hist_est),
                        ("plain_learned_order", lambda: run.plain(E), est),
                        ("batched_given_order", lambda: run.batch(G), est),
                        ("batched_learned_order", lambda: run.batch(E), est),
                        ("batched_learned_order_and_sizing", lambda: run.batch(ES), est)):
        log(name)
        ds.attach_estimator(e)
        ds.reset_profile()
        c, t = _timed(fn)
        run.check_complete()
        launches, scan_ms, total_ms = ds.profile()
        variants[name] = {"queries_per_s": n_te / t, "seconds": t, "counts": c}
        if launches:
            variants[name]["scan_kernel_us_per_query"] = scan_ms / launches * 1e3
        sized, reruns = ds.sizing_profile()
        if sized:
            variants[name]["sized_by_estimate"] = sized
            variants[name]["answered_again"] = reruns
        log(f"{name}: {n_te / t:.0f} queries/s")
    ds.set_profiling(False)
    ref = variants["plain_given_order"]["counts"]
    for name, v in variants.items():
        if not np.array_equal(v.pop("counts"), ref):
            raise RuntimeError(f"{name}: counts differ")
    if not np.array_equal(ref, counts):
        raise RuntimeError("counts differ from the count-only scans")
    lab = s_test[:, -1].astype(np.float64) * n
    if np.abs(lab - ref).max() > 1e-6 * n + 1:   # labels are float32 count / N
        raise RuntimeError("labels disagree with the scan counts")
    best = max(variants["batched_learned_order"]["queries_per_s"],
               variants["batched_learned_order_and_sizing"]["queries_per_s"])
    # Scratch the shared scans reserve for the held-out queries: a bitmap row and its
    # chunk marks each (worst case), against the estimate-sized room where it is smaller
    # (the serving loop's admission sizes).
    nw = (n + 63) // 64
    dense_b = nw * 8 + ((n + 255) // 256) * 2
    nch = (n + 511) // 512
    est_rows = pred[:, -1].astype(np.float64) * n
    want = np.minimum(nch, np.ceil(4.0 * est_rows) + 64)
    sparse_b = nch * 4 + want * 64
    sized_b = np.where(sparse_b < nw * 8 + nch * 2, sparse_b, dense_b)
    scratch = {"worst_case_bytes_per_query": float(dense_b), "estimate_sized_mean_bytes": float(sized_b.mean()),
               "estimate_sized_median_bytes": float(np.median(sized_b)),
               "queries_sized": int((sparse_b < nw * 8 + nch * 2).sum())}
    line = _line(best, "queries/s",
                 {"workload": f"c4: {n} rows x {w.n_dims} float32 columns (10 correlated pairs), "
                              f"{n_tr} training / {n_va} validation / {n_te} held-out queries, ids output",
                  "n_rows": n, "n_dims": w.n_dims, "train_queries": n_tr, "validation_queries": n_va,
                  "test_queries": n_te, "hidden": 64, "epochs": args.epochs, "data_seed": w.data_seed,
                  "query_seed": w.query_seed, "split_seed": w.split_seed},
                 1, 0, n_te / best * 1e3,
                 {"variants": variants, "q_error": qerr, "scratch_reservation": scratch,
                  "speedup_vs_plain_given_order": best / variants["plain_given_order"]["queries_per_s"],
                  "learned_vs_histogram_order_plain": variants["plain_learned_order"]["queries_per_s"]
                  / variants["plain_histogram_order"]["queries_per_s"],
                  "label_seconds": t_label, "train_seconds": t_train,
                  "epoch_loss_first_last": [float(losses[0]), float(losses[-1])]})
    if not args.no_cpu_baseline:
        log("timing the CPU oracle baseline")
        line["cpu_baseline"] = _cpu(raw, test_q, n, args.cpu_budget)
    ds.attach_estimator(None)
    est.close()
    hist_est.close()
    ds.close()
    return line


def serving(args):
    """c5: Poisson arrivals at each rate replayed through mdrq_serve (2 streams, shared
    scans of up to 256), results in device memory; with the estimator's order and
    estimate-sized admission, and, for comparison, its order with worst-case
    reservations."""
    import torch

    from paper_1801_03644_amd import datagen as dg
    from paper_1801_03644_amd import mdrq

    w, raw, ds, stream = _setup("c5", args.rows, args.graphs)
    samp = w.sampler()
    pool = dg.workload_queries(w, 4096, sampler=samp)
    train_q = dg.quantile_queries(samp, 20_000, (1, 6), (1e-6, 0.1), w.split_seed)
    val_q = dg.quantile_queries(samp, 4_000, (1, 6), (1e-6, 0.1), w.split_seed + 1)
    log("labelling, training and gating the estimator")
    est = mdrq.Estimator(ds, seed=1)
    est.train(train_q, ds.label_selectivities(train_q), epochs=args.epochs, batch=256, lr=1e-3)
    kept = est.gate(val_q, ds.label_selectivities(val_q))
    ds.attach_estimator(est)
    log("pool counts (single queries)")
    pool_counts = np.array([ds.query(q, None, mode="count").count for q in pool])
    n_words = (w.n_rows + 63) // 64
    n_buf = 1024
    bufs = torch.empty((n_buf, 2 * n_words), dtype=torch.int32, device="cuda:0")
    rng = np.random.default_rng(w.split_seed)
    rates = [float(r) for r in args.rates.split(",")]
    budget = 8 << 30

    def serve(rate, seconds, seed, use_estimator=3, segments=0):
        n = max(1, int(rate * seconds))
        r = np.random.default_rng(seed)
        arrivals = np.cumsum(r.exponential(1e9 / rate, size=n)).astype(np.uint64)
        pick = r.integers(0, len(pool), size=n)
        qs = [pool[i] for i in pick]
        # output buffers are reused cyclically; only counts are checked here
        outs = [bufs[i % n_buf] for i in range(n)]
        answers, lat, st = ds.serve(arrivals, qs, outs, "auto", max_batch=256, n_streams=2,
                                    budget_bytes=budget, use_estimator=use_estimator, segments=segments)
        counts = np.array([a.count for a in answers])
        if not np.array_equal(counts, pool_counts[pick]):
            raise RuntimeError("served counts differ from single-query counts")
        return st

    log("warm-up")
    serve(rates[0], 0.2, 1)
    per_rate = {}
    keys = ("completed", "scans", "wall_s", "qps", "p50_us", "p99_us", "mean_us", "max_us", "mean_batch",
            "hbm_gbps", "sized_by_estimate", "overflow_reruns")
    for i, rate in enumerate(rates):
        log(f"rate {rate:.0f}/s for {args.serve_seconds}s: learned order and sizing")
        st = serve(rate, args.serve_seconds, 100 + i, 3)
        per_rate[str(int(rate))] = {k: st[k] for k in keys}
        log(f"rate {rate:.0f}: {st['qps']:.0f} q/s, p50 {st['p50_us']:.0f} us, p99 {st['p99_us']:.0f} us")
        log(f"rate {rate:.0f}/s: learned order, worst-case reservations")
        st1 = serve(rate, args.serve_seconds, 100 + i, 1)
        per_rate[str(int(rate))]["order_only"] = {k: st1[k] for k in keys}
        log(f"rate {rate:.0f} (order only): {st1['qps']:.0f} q/s, p50 {st1['p50_us']:.0f} us, "
            f"p99 {st1['p99_us']:.0f} us")
        for seg in [int(x) for x in args.segments.split(",") if x]:
            for cm in [int(x) for x in args.circular_modes.split(",") if x]:
                ds.set_option(mdrq.OPT_CIRCULAR, cm)
                name = f"circular_{seg}" if cm == 4 else f"circular_{seg}_mode{cm}"
                log(f"rate {rate:.0f}/s: circular scan, {seg} parts per pass, mode {cm}")
                st2 = serve(rate, args.serve_seconds, 100 + i, 0, seg)
                per_rate[str(int(rate))][name] = {k: st2[k] for k in keys}
                log(f"rate {rate:.0f} ({name}): {st2['qps']:.0f} q/s, p50 {st2['p50_us']:.0f} us, "
                    f"p99 {st2['p99_us']:.0f} us, {st2['mean_batch']:.1f} active per step")
            ds.set_option(mdrq.OPT_CIRCULAR, 4)
    top = per_rate[str(int(rates[-1]))]
    line = _line(top["qps"], "queries/s",
                 {"workload": f"c5: {w.n_rows} rows x {w.n_dims} float32 columns resident, Poisson "
                              f"arrivals at {args.rates}/s for {args.serve_seconds}s each, pool of "
                              f"4096 queries (k 1..6, s 1e-6..0.1), auto output",
                  "n_rows": w.n_rows, "n_dims": w.n_dims, "max_batch": 256, "n_streams": 2,
                  "result_budget_bytes": budget, "data_seed": w.data_seed,
                  "query_seed": w.query_seed},
                 1, 0, top["wall_s"] * 1e3,
                 {"rates": per_rate, "p50_us": top["p50_us"], "p99_us": top["p99_us"],
                  "estimator_outputs_kept": [int(j) for j in np.flatnonzero(kept)]})
    if not args.no_cpu_baseline:
        log("timing the CPU oracle baseline")
        line["cpu_baseline"] = _cpu(raw, pool, w.n_rows, args.cpu_budget)
    ds.attach_estimator(None)
    est.close()
    ds.close()
    return line


def paper(args):
    """SYNT-UNI in the paper's terms (section 7.2.1): queries/s of 1000 two-object
    queries (complete match) per point, hot caches (one untimed pass first), for the
    dimensionality sweep of Figure 5 (10^6 objects, 5..100 dims) and the size sweep of
    Figure 7 (5 dims, 10^4..10^7 objects); one at a time and as shared scans."""
    import torch

    from paper_1801_03644_amd import datagen as dg
    from paper_1801_03644_amd import mdrq

    stream = mdrq._stream_handle(torch.cuda.current_stream())
    n_q = 1000

    def point(n, d):
        w = dg.workload(f"syntuni{d}", n)
        raw = w.columns()
        qs = dg.two_object_queries(raw, n_q, seed=w.query_seed)
        ds = mdrq.Dataset.from_host(raw)
        run = Runner(ds, qs, _exact_counts(ds, qs), stream)
        run.plain()
        c_plain, t_plain = _timed(run.plain)
        run.batch()
        c_batch, t_batch = _timed(run.batch)
        if not np.array_equal(c_plain, c_batch):
            raise RuntimeError("batched counts differ from single-query counts")
        run.check_complete()
        sel = c_plain / n
        ds.close()
        del run
        r = {"n_rows": n, "dims": d, "plain_queries_per_s": n_q / t_plain,
             "batched_queries_per_s": n_q / t_batch, "mean_selectivity_percent": 100 * float(sel.mean()),
             "sigma_selectivity_percent": 100 * float(sel.std())}
        log(f"N={n} d={d}: plain {r['plain_queries_per_s']:.0f} q/s, batched "
            f"{r['batched_queries_per_s']:.0f} q/s, selectivity {r['mean_selectivity_percent']:.5f}%")
        return r

    fig5 = [point(1_000_000, d) for d in (5, 10, 20, 50, 100)]
    fig7 = [point(n, 5) for n in (10_000, 100_000, 1_000_000, 10_000_000)]
    best = max(p["batched_queries_per_s"] for p in fig5 if p["dims"] == 5)
    return _line(best, "queries/s",
                 {"workload": "syntuni: SYNT-UNI grid data, 1000 two-object queries per point; "
                              "Figure 5 (10^6 x 5..100) and Figure 7 (10^4..10^7 x 5)",
                  "n_queries": n_q},
                 1, 1, n_q / best * 1e3,
                 {"figure5_dimensionality": fig5, "figure7_dataset_size": fig7,
                  "note": "value = batched queries/s at 10^6 x 5; the paper prints no numbers "
                          "for these figures, so there is no vs_baseline"})
