"""GPU parity of the serving loop (mdrq_serve): every request's result is the oracle's
and the same as the query alone, whatever it was batched with; admission respects the
result-memory budget."""
import numpy as np
import pytest

import oracle
from paper_1801_03644_amd import datagen as dg
from paper_1801_03644_amd import mdrq
from tests.gpu_helpers import bitmap_to_ids, device, run

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def outputs(n_rows, modes, caps=None):
    import torch

    outs = []
    for i, m in enumerate(modes):
        cap = None if caps is None else caps[i]
        if m == "count":
            outs.append(None)
        elif m == "bitmap":
            n = (n_rows + 63) // 64 if cap is None else cap
            outs.append(torch.full((max(1, n),), -1, dtype=torch.int64, device=device())[:n])
        else:
            n = max(n_rows, 2 * ((n_rows + 63) // 64)) if cap is None else cap
            outs.append(torch.full((max(1, n),), -1, dtype=torch.int32, device=device())[:n])
    return outs


def payload(out, ans, n_rows):
    a = out.cpu().numpy().view(np.uint8)
    if ans.mode == "bitmap":
        return bitmap_to_ids(a[:8 * ans.written].view(np.uint64), n_rows)[0]
    return a[:4 * ans.written].view(np.uint32)


def poisson(n, rate_per_s, seed):
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1e9 / rate_per_s, size=n)).astype(np.uint64)


def c5_small(n_rows):
    w = dg.workload("c5", n_rows)
    return w, w.columns()


def check(ds, cols, qs, modes, outs, answers, label):
    for i, (q, m, o, a) in enumerate(zip(qs, modes, outs, answers)):
        st, cnt, want = oracle.query(cols, q)
        assert a.count == cnt, (label, i)
        if m == "count":
            assert a.mode == "count"
            continue
        assert a.status == mdrq.OK, (label, i)
        assert np.array_equal(payload(o, a, ds.n_rows), want), (label, i, m)


def test_serve_results_match_oracle_and_alone():
    w, raw = c5_small(300_007)
    cols = oracle.prepare(raw)
    pool = dg.workload_queries(w, 64, sampler=w.sampler(sample_rows=1 << 16))
    pool[0] = dg.make_query([])                       # every row
    pool[1] = dg.make_query([(2, 0.6, 0.1)])          # empty interval
    pool[2] = dg.make_query([(j, -np.inf, np.inf) for j in range(12)])
    rng = np.random.default_rng(1)
    n = 400
    qs = [pool[i] for i in rng.integers(0, len(pool), size=n)]
    modes = [["ids", "bitmap", "count", "auto"][i % 4] for i in range(n)]
    arrivals = poisson(n, 40_000, seed=2)
    with mdrq.Dataset.from_host(raw) as ds:
        outs = outputs(ds.n_rows, modes)
        _print("serve 400 requests")
        answers, lat, stats = ds.serve(arrivals, qs, outs, modes, max_batch=64, n_streams=2,
                                       budget_bytes=1 << 26)
        _print(stats)
        check(ds, cols, qs, modes, outs, answers, "mix")
        assert stats["completed"] == n and stats["scans"] >= 1
        assert stats["p50_us"] <= stats["p99_us"] <= stats["max_us"]
        assert (lat > 0).all()
        assert stats["mean_batch"] >= 1.0
        # the same queries alone
        for i in range(0, n, 37):
            if modes[i] != "ids":
                continue
            a1, ids1 = run(ds, qs[i])
            assert a1.count == answers[i].count
            assert np.array_equal(ids1, payload(outs[i], answers[i], ds.n_rows))


@pytest.mark.parametrize("segments,mode", [(1, 0), (3, 0), (8, 0), (200, 0), (3, 3), (8, 1), (8, 2), (3, 4),
                                            (200, 4), (8, 7)])
def test_circular_scan_results_match_oracle_and_alone(segments, mode):
    """The circular scan: requests join the running scan at whatever part of the rows
    comes next and finish after one pass; every result is the oracle's and the query's
    alone (mixed output modes, every row, an empty interval, an unrestricted query, a
    ragged last tile; 200 parts are more than the 74 tiles: one per tile), with steps
    pipelined or not, with or without separate scans for few requests, and with steps of
    few requests by single-query scans into the slots (mode bits)."""
    w, raw = c5_small(300_007)
    cols = oracle.prepare(raw)
    pool = dg.workload_queries(w, 64, sampler=w.sampler(sample_rows=1 << 16))
    pool[0] = dg.make_query([])                       # every row
    pool[1] = dg.make_query([(2, 0.6, 0.1)])          # empty interval
    pool[2] = dg.make_query([(j, -np.inf, np.inf) for j in range(12)])
    rng = np.random.default_rng(4)
    n = 300
    qs = [pool[i] for i in rng.integers(0, len(pool), size=n)]
    modes = [["ids", "bitmap", "count", "auto"][i % 4] for i in range(n)]
    # bursts of 1..24 requests (the first of 24) at Poisson times: bursts start passes,
    # later ones join them, lone requests may be answered by their own scans
    sizes = np.concatenate([[24], rng.integers(1, 25, size=n)])
    burst_of = np.repeat(np.arange(len(sizes)), sizes)[:n]
    arrivals = poisson(len(sizes), 3_000, seed=5)[burst_of] - poisson(len(sizes), 3_000, seed=5)[0]
    with mdrq.Dataset.from_host(raw) as ds:
        ds.set_option(mdrq.OPT_CIRCULAR, mode)
        outs = outputs(ds.n_rows, modes)
        _print("circular serve", n, "requests, segments", segments, "mode", mode)
        answers, lat, stats = ds.serve(arrivals, qs, outs, modes, max_batch=64, n_streams=2,
                                       budget_bytes=1 << 26, segments=segments)
        _print(stats)
        check(ds, cols, qs, modes, outs, answers, "circular")
        assert stats["completed"] == n and stats["scans"] >= 1
        assert stats["mean_batch"] >= 1.0
        assert stats["p50_us"] <= stats["p99_us"] <= stats["max_us"]
        for i in range(0, n, 23):
            if modes[i] != "ids":
                continue
            a1, ids1 = run(ds, qs[i])
            assert a1.count == answers[i].count
            assert np.array_equal(ids1, payload(outs[i], answers[i], ds.n_rows))


def test_circular_scan_slots_and_union_limit():
    """Circular-scan admission: with a share of two query slots per stream no step scans
    more than two requests per worker; lone requests on an idle server get their own
    scans; on 128 columns, requests restricting 50 columns each wait while their union
    would not fit one scan, and a request on 110 columns is answered by its own scan;
    all results are the oracle's."""
    w, raw = c5_small(100_000)
    cols = oracle.prepare(raw)
    qs = dg.workload_queries(w, 40, sampler=w.sampler(sample_rows=1 << 16))
    row = 8 * ((100_000 + 63) // 64)
    with mdrq.Dataset.from_host(raw) as ds:
        modes = ["ids", "auto"] * 20
        outs = outputs(ds.n_rows, modes)
        answers, lat, stats = ds.serve(np.zeros(40, dtype=np.uint64), qs, outs, modes, max_batch=64,
                                       n_streams=2, budget_bytes=2 * 3 * row, segments=4)
        _print(stats)
        check(ds, cols, qs, modes, outs, answers, "slots")
        assert 1.0 <= stats["mean_batch"] <= 2.0
        # requests arriving one at a time with idle gaps, separate scans allowed: each
        # answered by its own scan (cheaper than a pass), no pass started
        ds.set_option(mdrq.OPT_CIRCULAR, 2)
        answers, lat, stats = ds.serve(np.arange(8, dtype=np.uint64) * 3_000_000, qs[:8], outs[:8], modes[:8],
                                       max_batch=64, n_streams=1, budget_bytes=1 << 26, segments=4)
        _print(stats)
        check(ds, cols, qs[:8], modes[:8], outs[:8], answers, "separate")
        assert stats["scans"] == 0
        ds.set_option(mdrq.OPT_CIRCULAR, 4)
        with pytest.raises(mdrq.MdrqError) as e:
            ds.serve([0], qs[:1], outputs(ds.n_rows, ["ids"]), "ids", n_streams=1,
                     budget_bytes=row, segments=4)
        assert e.value.code == mdrq.EBUSY
        for kwargs in ({"segments": 4097}, {"segments": 2, "use_estimator": 2}):
            with pytest.raises(mdrq.MdrqError) as e:
                ds.serve([0], qs[:1], outputs(ds.n_rows, ["ids"]), "ids", **kwargs)
            assert e.value.code == mdrq.EINVAL

    n, d = 20_000, 128
    raw = [dg.column(41, j, dg.uniform(), n) for j in range(d)]
    cols = oracle.prepare(raw)
    rng = np.random.default_rng(6)
    qs = []
    for i in range(24):
        k = 110 if i == 7 else 50
        dims = rng.choice(d, size=k, replace=False)
        qs.append(dg.make_query([(int(j), 0.0, 0.995) for j in dims]))
    modes = ["ids", "count", "bitmap"] * 8
    with mdrq.Dataset.from_host(raw) as ds:
        outs = outputs(ds.n_rows, modes)
        answers, lat, stats = ds.serve(np.zeros(24, dtype=np.uint64), qs, outs, modes, max_batch=64,
                                       n_streams=1, budget_bytes=1 << 26, segments=3)
        _print(stats)
        check(ds, cols, qs, modes, outs, answers, "union limit")
        # at most two 50-column requests fit one scan's union (three cover about 99 of
        # 128 columns, over the limit most of the time): steps carry few of the 24
        assert stats["mean_batch"] < 6


def test_circular_scan_edge_datasets():
    """The circular scan on a dataset of one ragged tile (more parts asked than tiles),
    on special values (+-0, +-inf, subnormals, bounds at them) and on an empty dataset
    (every request answered at admission)."""
    special = np.array([-np.inf, -2.5, -1.0, -1e-45, -0.0, 0.0, 1e-45, 1.1754942e-38,
                        0.25, 0.5, 1.0, 3.0e38, np.inf], dtype=np.float32)
    rng = np.random.default_rng(8)
    cases = [
        ("one tile", [rng.random(1000, dtype=np.float32) for _ in range(4)],
         [(j, lo, hi) for j in range(4) for lo, hi in ((0.1, 0.7), (0.0, 0.05), (0.5, 1.0))]),
        ("special", [special[rng.integers(0, len(special), size=30_000)] for _ in range(3)],
         [(j, lo, hi) for j in range(3) for lo, hi in ((-0.0, 0.0), (0.0, np.inf), (-np.inf, -0.0),
                                                        (1e-45, 1.0), (-1e-45, 1e-45), (-2.5, 0.25))]),
    ]
    for (label, raw, preds), mode in [(case, m) for case in cases for m in (0, 4)]:
        cols = oracle.prepare(raw)
        qs = [dg.make_query([preds[i], preds[(3 * i + 1) % len(preds)]])
              if preds[i][0] != preds[(3 * i + 1) % len(preds)][0] else dg.make_query([preds[i]])
              for i in range(len(preds))]
        qs.append(dg.make_query([]))
        modes = [["ids", "bitmap", "count", "auto"][i % 4] for i in range(len(qs))]
        with mdrq.Dataset.from_host(raw) as ds:
            ds.set_option(mdrq.OPT_CIRCULAR, mode)
            outs = outputs(ds.n_rows, modes)
            answers, lat, stats = ds.serve(np.zeros(len(qs), dtype=np.uint64), qs, outs, modes,
                                           max_batch=64, n_streams=1, budget_bytes=1 << 26, segments=4)
            _print(label, "mode", mode, stats)
            check(ds, cols, qs, modes, outs, answers, label)
    raw = [np.empty(0, dtype=np.float32)] * 2
    with mdrq.Dataset.from_host(raw) as ds:
        modes = ["ids", "bitmap", "count", "auto"]
        qs = [dg.make_query([(0, 0.0, 1.0)])] * 4
        answers, lat, stats = ds.serve(np.zeros(4, dtype=np.uint64), qs, [None] * 4, modes,
                                       max_batch=8, n_streams=1, budget_bytes=1 << 20, segments=3)
        assert all(a.count == 0 and a.status == mdrq.OK for a in answers)
        assert stats["completed"] == 4 and stats["scans"] == 0


def test_admission_by_result_memory():
    """Each stream's share holds exactly 3 bitmap rows: no worker batch carries more
    than 3 requests that need one, count-only requests need none."""
    w, raw = c5_small(100_000)
    cols = oracle.prepare(raw)
    qs = dg.workload_queries(w, 60, sampler=w.sampler(sample_rows=1 << 16))
    row = 8 * ((100_000 + 63) // 64)
    with mdrq.Dataset.from_host(raw) as ds:
        modes = ["ids"] * 60
        outs = outputs(ds.n_rows, modes)
        answers, lat, stats = ds.serve(np.zeros(60, dtype=np.uint64), qs, outs, modes,
                                       max_batch=64, n_streams=2, budget_bytes=2 * 3 * row + 100)
        check(ds, cols, qs, modes, outs, answers, "admission")
        assert stats["mean_batch"] <= 3.0 and stats["mean_batch"] >= 1.0
        cmodes = ["count"] * 60
        answers, lat, stats = ds.serve(np.zeros(60, dtype=np.uint64), qs, [None] * 60, cmodes,
                                       max_batch=64, n_streams=2, budget_bytes=0)
        check(ds, cols, qs, cmodes, [None] * 60, answers, "count only")
        with pytest.raises(mdrq.MdrqError) as e:
            ds.serve([0], qs[:1], outputs(ds.n_rows, ["ids"]), "ids", n_streams=2,
                     budget_bytes=row)
        assert e.value.code == mdrq.EBUSY


def test_serve_overflow_and_invalid():
    w, raw = c5_small(50_000)
    cols = oracle.prepare(raw)
    q = dg.make_query([(0, 0.1, 0.8)])
    st, cnt, want = oracle.query(cols, q)
    with mdrq.Dataset.from_host(raw) as ds:
        outs = outputs(ds.n_rows, ["ids", "ids"], caps=[10, None])
        answers, lat, stats = ds.serve([0, 0], [q, q], outs, "ids", n_streams=1)
        assert answers[0].status == mdrq.EOVERFLOW and answers[0].count == cnt
        assert answers[0].written == 10
        assert np.array_equal(payload(outs[0], answers[0], ds.n_rows), want[:10])
        assert answers[1].status == mdrq.OK
        assert np.array_equal(payload(outs[1], answers[1], ds.n_rows), want)
        host = [np.zeros(ds.n_rows, dtype=np.uint32)]
        for kwargs in ({"max_batch": 0}, {"n_streams": 9}, {"use_estimator": True}):
            with pytest.raises(mdrq.MdrqError) as e:
                ds.serve([0], [q], outputs(ds.n_rows, ["ids"]), "ids", **kwargs)
            assert e.value.code == mdrq.EINVAL
        with pytest.raises(mdrq.MdrqError) as e:
            ds.serve([0], [q], host, "ids")
        assert e.value.code == mdrq.EINVAL


def test_serve_with_estimated_order_is_exact():
    w, raw = c5_small(200_000)
    cols = oracle.prepare(raw)
    samp = w.sampler(sample_rows=1 << 16)
    train = dg.workload_queries(w, 2000, sampler=samp, seed=5)
    qs = dg.workload_queries(w, 120, sampler=samp, seed=6)
    modes = ["ids", "count", "auto"] * 40
    with mdrq.Dataset.from_host(raw) as ds, mdrq.Estimator(ds) as est:
        est.train(train, ds.label_selectivities(train), epochs=5, batch=256, lr=2e-3)
        ds.attach_estimator(est)
        outs = outputs(ds.n_rows, modes)
        answers, lat, stats = ds.serve(poisson(120, 50_000, 3), qs, outs, modes, max_batch=32,
                                       n_streams=3, budget_bytes=1 << 26, use_estimator=True)
        check(ds, cols, qs, modes, outs, answers, "estimated")
        ds.attach_estimator(None)


def test_full_size_c5_served_sampled():
    """The serving shape at full size (2*10^8 x 12 resident), as the bench runs it:
    requests replayed through the serving loop with estimated order (an untrained
    estimator: the histogram ranking) and AUTO outputs; every count and a sample of
    results equal the oracle's."""
    from paper_1801_03644_amd.mdrq import Estimator
    from tests.gpu_helpers import oracle_counts

    w = dg.workload("c5")
    _print("c5 full size: generating")
    raw = w.columns()
    cols = oracle.prepare(raw)
    qs = dg.workload_queries(w, 40)
    modes = ["auto"] * len(qs)
    with mdrq.Dataset.from_host(raw) as ds:
        est = Estimator(ds)
        ds.attach_estimator(est)
        outs = outputs(ds.n_rows, modes, caps=[ds.n_rows] * len(qs))
        _print("c5 full size: serve", len(qs))
        answers, lat, stats = ds.serve(poisson(len(qs), 20_000, seed=5), qs, outs, modes,
                                       max_batch=32, n_streams=2, budget_bytes=2 << 30,
                                       use_estimator=True)
        assert stats["completed"] == len(qs)
        _print("c5 full size: oracle counts of all", len(qs))
        assert [a.count for a in answers] == oracle_counts(cols, qs)
        for i in (0, 7, 19):
            _print("c5 full size: oracle", i)
            st, cnt, want = oracle.query(cols, qs[i])
            assert answers[i].count == cnt
            assert answers[i].status == mdrq.OK
            assert np.array_equal(payload(outs[i], answers[i], ds.n_rows), want), i
        ds.attach_estimator(None)
        est.close()


def test_serving_with_estimate_sized_scratch():
    """Serving with estimated order and sizing (use_estimator = 3): requests are
    admitted by the scratch their estimate
    needs (smaller than a bitmap row for small results), so more of them share a scan;
    with the reserve factor forced to 10^-6 most of them outgrow their room and are
    answered again.  Every result equals the oracle's."""
    from paper_1801_03644_amd.mdrq import Estimator

    w = dg.workload("c5", 2_000_003)
    raw = w.columns()
    cols = oracle.prepare(raw)
    qs = dg.workload_queries(w, 120, sampler=w.sampler(sample_rows=1 << 15), seed=9)
    modes = [("ids", "auto", "bitmap")[i % 3] for i in range(len(qs))]
    want = [oracle.query(cols, q) for q in qs]
    with mdrq.Dataset.from_host(raw) as ds:
        est = Estimator(ds)
        ds.attach_estimator(est)
        row_bytes = 8 * ((ds.n_rows + 63) // 64)
        for factor in (4_000_000, 1):
            ds.set_option(mdrq.OPT_RESERVE_FACTOR, factor)
            outs = outputs(ds.n_rows, modes)
            # a burst: every request waits at once, so batches are bounded by memory
            answers, lat, stats = ds.serve(poisson(len(qs), 100_000_000, seed=3), qs, outs, modes,
                                           max_batch=64, n_streams=2, budget_bytes=8 * row_bytes,
                                           use_estimator=3)
            _print("factor", factor, "mean batch", stats["mean_batch"], "sized", stats["sized_by_estimate"],
                   "reruns", stats["overflow_reruns"])
            assert stats["completed"] == len(qs) and stats["sized_by_estimate"] > 0
            if factor == 1:
                assert stats["overflow_reruns"] > 0
            else:
                # a stream's share holds three bitmap rows with their marks; estimates
                # admit more requests per scan
                assert stats["mean_batch"] > 3
            for i, (a, o) in enumerate(zip(answers, outs)):
                st, cnt, ids = want[i]
                assert a.count == cnt and a.status == mdrq.OK, i
                assert np.array_equal(payload(o, a, ds.n_rows), ids), (factor, i)
        ds.attach_estimator(None)
        est.close()
