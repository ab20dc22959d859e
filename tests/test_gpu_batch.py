"""GPU parity of the batched shared scan (mdrq_query_batch).

Each query of a batch must give exactly what the oracle gives for it alone (and what
mdrq_query gives for it alone): identical counts and ascending id lists, bitmaps that
decode to the same ids.
"""
import numpy as np
import pytest

import oracle
from paper_1801_03644_amd import datagen as dg
from paper_1801_03644_amd import mdrq
from tests.gpu_helpers import bitmap_to_ids, device, run

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def make_outs(n_rows, modes, caps=None):
    import torch

    outs = []
    for i, m in enumerate(modes):
        if m == "count":
            outs.append(None)
            continue
        if m == "bitmap":
            n = (n_rows + 63) // 64 if caps is None or caps[i] is None else caps[i]
            outs.append(torch.full((max(1, n),), -1, dtype=torch.int64, device=device())[:n])
        else:  # ids or auto: room for every row (ids) or the bitmap, whichever is larger
            n = max(n_rows, 2 * ((n_rows + 63) // 64)) if caps is None or caps[i] is None else caps[i]
            outs.append(torch.full((max(1, n),), -1, dtype=torch.int32, device=device())[:n])
    return outs


def payload(out, ans, n_rows):
    if out is None:
        return None
    a = out.cpu().numpy().view(np.uint8)
    if ans.mode == "bitmap":
        return bitmap_to_ids(a[:8 * ans.written].view(np.uint64), n_rows)[0]
    return a[:4 * ans.written].view(np.uint32)


def check_batch(ds, cols, queries, modes, label="", caps=None):
    outs = make_outs(ds.n_rows, modes, caps)
    answers = ds.query_batch(queries, outs, modes)
    for i, (q, m, a, o) in enumerate(zip(queries, modes, answers, outs)):
        st, cnt, want = oracle.query(cols, q)
        assert a.count == cnt, (label, i, m, a.count, cnt)
        got = payload(o, a, ds.n_rows)
        if m == "count":
            assert a.mode == "count"
            continue
        if m == "auto":
            assert a.mode in ("ids", "bitmap")
            nw = (ds.n_rows + 63) // 64
            if a.mode == "bitmap":
                assert 8 * nw < 4 * cnt or 4 * cnt > o.numel() * 4, (label, i)
        cap = None if caps is None else caps[i]
        if cap is None:
            assert a.status == mdrq.OK
            assert np.array_equal(got, want), (label, i, m)
        else:
            if a.mode == "ids":
                assert a.written == min(cap, cnt)
                assert np.array_equal(got, want[:cap]), (label, i)
                assert a.status == (mdrq.EOVERFLOW if cnt > cap else mdrq.OK)
    return answers


def c3_like(n_rows, seed=0):
    w = dg.workload("c3", n_rows)
    raw = w.columns()
    return w, raw


def test_batch_matches_oracle_and_singles():
    w, raw = c3_like(300_001)
    cols = oracle.prepare(raw)
    qs = dg.workload_queries(w, 64, sampler=w.sampler(sample_rows=1 << 16))
    modes = ["ids", "bitmap", "count", "auto"] * 16
    with mdrq.Dataset.from_host(raw) as ds:
        _print("batch 64 on", w.n_rows)
        check_batch(ds, cols, qs, modes, "c3-like")
        # the same queries one at a time through mdrq_query
        for q in qs[:16]:
            a1, ids1 = run(ds, q)
            outs = make_outs(ds.n_rows, ["ids"])
            (a2,) = ds.query_batch([q], outs, ["ids"])
            assert a1.count == a2.count
            assert np.array_equal(ids1, payload(outs[0], a2, ds.n_rows))


@pytest.mark.parametrize("n", [1, 63, 100, 255, 256, 4095, 4096, 4097, 70001])
def test_batch_sizes_and_ragged_tails(n):
    raw = [dg.column(21, j, dg.uniform(), n) for j in range(4)]
    cols = oracle.prepare(raw)
    rng = np.random.default_rng(n)
    qs = [dg.make_query([]), dg.make_query([(0, 0.0, 1.0)])]
    for _ in range(14):
        k = int(rng.integers(1, 5))
        dims = rng.permutation(4)[:k]
        wdt = float(rng.choice([0.9, 0.5, 0.2, 0.05]))
        preds = []
        for j in dims:
            lo = float(rng.uniform(0, 1 - wdt))
            preds.append((int(j), lo, lo + wdt))
        qs.append(dg.make_query(preds))
    with mdrq.Dataset.from_host(raw) as ds:
        for variant in (0, 4, 5):   # autotuned; slot-mask records; ranks and bitsets
            ds.set_option(mdrq.OPT_BATCH_VARIANT, variant)
            for Q in (1, 7, 16):
                modes = (["ids", "bitmap", "count", "auto"] * 4)[:Q]
                check_batch(ds, cols, qs[:Q], modes, f"n={n} Q={Q} variant={variant}")
        for buckets in (1, 2):      # rank variant, each bucket map forced
            ds.set_option(mdrq.OPT_RANK_BUCKETS, buckets)
            modes = ["ids", "bitmap", "count", "auto"] * 4
            check_batch(ds, cols, qs, modes, f"n={n} rank buckets={buckets}")
        ds.set_option(mdrq.OPT_RANK_BUCKETS, 0)


@pytest.mark.parametrize("n", [128 * 4096 + 1, 5 * 128 * 4096, 5 * 128 * 4096 - 4095])
def test_finish_chunk_boundaries(n):
    """The finish sums tile counts per chunk of 128 tiles (a chunk per wave, four per
    workgroup) and emits each chunk's tiles from its position: a last chunk of one tile,
    chunk counts that leave waves of the sum pass idle, a ragged last tile.  Interval
    widths give tiles of thousands of ids (direct writes), of hundreds (staged in LDS)
    and of a few (direct writes again); capped outputs stop inside each kind."""
    raw = [dg.column(31, j, dg.uniform(), n) for j in range(4)]
    cols = oracle.prepare(raw)
    rng = np.random.default_rng(n % 1000)
    qs, caps = [], []
    for wdt in (0.95, 0.9, 0.3, 0.1, 0.02, 0.004, 0.0005):
        for k in (1, 2):
            dims = rng.permutation(4)[:k]
            preds = []
            for j in dims:
                lo = float(rng.uniform(0, 1 - wdt ** (1.0 / k)))
                preds.append((int(j), lo, lo + wdt ** (1.0 / k)))
            qs.append(dg.make_query(preds))
    counts = [oracle.count(cols, q) for q in qs]
    modes = (["ids", "auto", "bitmap", "count"] * 4)[:len(qs)]
    caps = [None] * len(qs)
    # ids outputs capped inside a dense tile, a staged tile and a sparse tile
    extra = [(0, 4096 * 3 + 17), (6, 999), (10, 31)]
    for i, cap in extra:
        qs.append(qs[i])
        modes.append("ids")
        caps.append(min(cap, max(1, counts[i] - 1)))
    with mdrq.Dataset.from_host(raw) as ds:
        for variant in (0, 5):
            ds.set_option(mdrq.OPT_BATCH_VARIANT, variant)
            _print("finish chunks", n, "variant", variant, "queries", len(qs))
            check_batch(ds, cols, qs, modes, f"n={n} variant={variant}", caps=caps)


def test_batch_special_values_degenerate_and_invalid():
    vals = np.array([-np.inf, -1.0, -0.0, 0.0, 1e-45, 1.1754944e-38, 0.5, 1.0, np.inf],
                    dtype=np.float32)
    rng = np.random.default_rng(8)
    n = 9000
    raw = [vals[rng.integers(0, len(vals), size=n)].astype(np.float32) for _ in range(3)]
    cols = oracle.prepare(raw)
    cands = sorted({float(x) for v in vals for x in
                    (v, np.nextafter(v, np.float32(np.inf)), np.nextafter(v, np.float32(-np.inf)))})
    qs = [dg.make_query([(0, 0.5, 0.2)]),                     # empty interval
          dg.make_query([]),                                   # all rows
          dg.make_query([(j, -np.inf, np.inf) for j in range(3)]),
          dg.make_query([(1, -0.0, 0.0)]),
          dg.make_query([(2, 0.0, -0.0), (0, -np.inf, 0.5)])]
    for _ in range(59):
        k = int(rng.integers(1, 4))
        dims = rng.permutation(3)[:k]
        qs.append(dg.make_query([(int(j), cands[rng.integers(len(cands))],
                                  cands[rng.integers(len(cands))]) for j in dims]))
    modes = (["ids", "bitmap", "auto", "count"] * 16)
    with mdrq.Dataset.from_host(raw) as ds:
        for variant in (5, 4, 3, 2, 1, 0):
            ds.set_option(mdrq.OPT_BATCH_VARIANT, variant)
            check_batch(ds, cols, qs, modes, f"special variant={variant}")
        ds.set_option(mdrq.OPT_BATCH_VARIANT, 5)
        for buckets in (1, 2):   # the rank search's buckets by key, then by float value
            ds.set_option(mdrq.OPT_RANK_BUCKETS, buckets)
            check_batch(ds, cols, qs, modes, f"special rank buckets={buckets}")
        ds.set_option(mdrq.OPT_RANK_BUCKETS, 0)
        with pytest.raises(mdrq.MdrqError) as e:
            ds.set_option(mdrq.OPT_RANK_BUCKETS, 3)
        assert e.value.code == mdrq.EINVAL
        with pytest.raises(mdrq.MdrqError) as e:
            ds.query_batch([qs[3], dg.make_query([(1, np.nan, 1.0)])], None, "count")
        assert e.value.code == mdrq.EINVAL
        with pytest.raises(mdrq.MdrqError) as e:
            ds.query_batch([dg.make_query([(0, 0.0, 1.0), (0, 0.1, 0.2)])], None, "count")
        assert e.value.code == mdrq.EINVAL


def test_union_beyond_register_slots_and_long_queries():
    """20 columns: batches whose union exceeds the 16 register slots are split into
    several shared scans; a query on more than 16 columns runs alone."""
    w = dg.workload("c4", 50_000)
    raw = w.columns()
    cols = oracle.prepare(raw)
    rng = np.random.default_rng(4)
    qs = []
    for i in range(40):
        k = 18 if i % 13 == 0 else int(rng.integers(1, 6))
        dims = rng.permutation(20)[:k]
        preds = []
        for j in dims:
            lo = float(rng.uniform(0, 0.4))
            preds.append((int(j), lo, lo + (0.6 if k > 10 else 0.4)))
        qs.append(dg.make_query(preds))
    with mdrq.Dataset.from_host(raw) as ds:
        for variant in (0, 4, 5):
            ds.set_option(mdrq.OPT_BATCH_VARIANT, variant)
            check_batch(ds, cols, qs, ["ids", "auto"] * 20, f"union variant={variant}")


@pytest.mark.parametrize("variant", [0, 2, 3, 4, 5])
def test_wide_unions_share_one_scan(variant):
    """40 columns: the union of all 40 is staged in LDS and the batch shares one scan
    (forced LDS variant, or autotuned).  Ragged row count."""
    n = 70_001
    raw = [dg.column(44, j, dg.uniform() if j % 2 == 0 else dg.gmm(), n) for j in range(40)]
    cols = oracle.prepare(raw)
    rng = np.random.default_rng(9)
    qs = []
    for i in range(48):
        k = 34 if i % 11 == 0 else int(rng.integers(1, 24))
        dims = rng.permutation(40)[:k]
        preds = []
        for j in dims:
            lo = float(rng.uniform(0, 0.3))
            preds.append((int(j), lo, lo + float(rng.uniform(0.5, 0.7))))
        qs.append(dg.make_query(preds))
    with mdrq.Dataset.from_host(raw) as ds:
        ds.set_option(mdrq.OPT_BATCH_VARIANT, variant)
        check_batch(ds, cols, qs, ["ids", "bitmap", "count", "auto"] * 12, f"wide {variant}")


def test_batch_overflow_and_host_outputs():
    w, raw = c3_like(120_000)
    cols = oracle.prepare(raw)
    q = dg.make_query([(0, 0.1, 0.7), (5, 0.0, 0.9)])
    st, cnt, want = oracle.query(cols, q)
    with mdrq.Dataset.from_host(raw) as ds:
        for variant in (0, 5):   # autotuned; ranks and bitsets
            ds.set_option(mdrq.OPT_BATCH_VARIANT, variant)
            caps = [0, 1, cnt // 2, cnt - 1, cnt, None]
            check_batch(ds, cols, [q] * len(caps), ["ids"] * len(caps), f"overflow variant={variant}",
                        caps=caps)
            outs = [np.zeros(w.n_rows, dtype=np.uint32), np.zeros((w.n_rows + 63) // 64, dtype=np.uint64)]
            a = ds.query_batch([q, q], outs, ["ids", "bitmap"])
            assert a[0].count == cnt and np.array_equal(outs[0][:a[0].written], want)
            assert np.array_equal(bitmap_to_ids(outs[1], w.n_rows)[0], want)


def test_launch_configurations_give_identical_results():
    w, raw = c3_like(200_000)
    cols = oracle.prepare(raw)
    qs = dg.workload_queries(w, 48, sampler=w.sampler(sample_rows=1 << 16))
    with mdrq.Dataset.from_host(raw) as ds:
        ref = None
        for waves, group, tune, variant, rows in [
                (0, 0, 1, 0, 0), (4, 0, 0, 1, 0), (8, 0, 0, 1, 0), (4, 16, 0, 1, 0), (8, 24, 0, 1, 0),
                (4, 0, 0, 2, 2), (4, 0, 0, 2, 4), (8, 0, 0, 2, 8), (4, 16, 0, 2, 8), (8, 24, 0, 2, 4),
                (4, 0, 0, 3, 8), (8, 0, 0, 3, 8), (4, 16, 0, 3, 16), (4, 0, 0, 2, 1),
                (4, 0, 0, 4, 8), (8, 0, 0, 4, 8), (4, 16, 0, 4, 16), (8, 24, 0, 4, 4),
                (4, 0, 0, 4, 4), (4, 0, 0, 5, 8), (8, 0, 0, 5, 4), (4, 20, 0, 5, 8),
                (8, 40, 0, 5, 4), (4, 0, 0, 5, 16), (0, 0, 1, 0, 0)]:
            ds.set_option(mdrq.OPT_BATCH_WAVES, waves)
            ds.set_option(mdrq.OPT_BATCH_GROUP, group)
            ds.set_option(mdrq.OPT_AUTOTUNE, tune)
            ds.set_option(mdrq.OPT_BATCH_VARIANT, variant)
            ds.set_option(mdrq.OPT_BATCH_ROWS, rows)
            outs = make_outs(ds.n_rows, ["ids"] * len(qs))
            ans = ds.query_batch(qs, outs, "ids")
            got = [(a.count, payload(o, a, ds.n_rows).tobytes()) for a, o in zip(ans, outs)]
            if ref is None:
                ref = got
                for q, (c, _) in zip(qs, got):
                    assert c == oracle.count(cols, q)
            assert got == ref, (waves, group, tune, variant, rows)


def test_full_size_c3_batch_sampled():
    """The c3 shape at full size (5*10^7 x 8): one batch of 256 queries in AUTO mode;
    every count and the results of a sample of queries against the oracle."""
    from tests.gpu_helpers import oracle_counts, oracle_queries

    w = dg.workload("c3")
    _print("c3 full size: generating")
    raw = w.columns()
    cols = oracle.prepare(raw)
    qs = dg.workload_queries(w, 256)
    modes = ["auto"] * 256
    with mdrq.Dataset.from_host(raw) as ds:
        outs = make_outs(ds.n_rows, ["ids"] * 256, caps=[4_000_000] * 256)
        _print("c3 full size: batch")
        ans = ds.query_batch(qs, outs, modes)
        rng = np.random.default_rng(0)
        pick = rng.choice(256, size=8, replace=False)
        for i, (st, cnt, want) in zip(pick, oracle_queries(cols, [qs[i] for i in pick])):
            assert ans[i].count == cnt
            got = payload(outs[i], ans[i], ds.n_rows)
            if ans[i].status == mdrq.OK:
                assert np.array_equal(got, want)
            else:
                assert np.array_equal(got, want[:len(got)])
        _print("c3 full size: oracle counts of all 256")
        assert [a.count for a in ans] == oracle_counts(cols, qs)


def test_full_size_c3_headline_batch():
    """The c3 headline batch as the bench runs it: 5*10^7 x 8, 1024 queries in one call
    (eight rank groups of 128 under the autotuned launch), ids output into 12 M-id
    buffers.  The autotuning call and a repeat both give every count equal to the
    oracle's (host threads, one query each), and 16 sampled id lists equal the
    oracle's."""
    import torch

    from tests.gpu_helpers import oracle_counts, oracle_queries

    w = dg.workload("c3")
    _print("c3 headline: generating")
    raw = w.columns()
    cols = oracle.prepare(raw)
    qs = dg.workload_queries(w, 1024)
    cap = 12_000_000
    with mdrq.Dataset.from_host(raw) as ds:
        out = torch.full((1024, cap), -1, dtype=torch.int32, device=device())
        outs = [out[i] for i in range(1024)]
        _print("c3 headline: oracle counts (host threads)")
        want_counts = oracle_counts(cols, qs)
        assert max(want_counts) <= cap  # no overflow: the bench's outputs hold every id
        for rep in range(2):
            _print("c3 headline: batch", rep)
            ans = ds.query_batch(qs, outs, "ids")
            assert [a.count for a in ans] == want_counts, rep
            assert all(a.status == mdrq.OK and a.mode == "ids" for a in ans)
        rng = np.random.default_rng(1)
        pick = sorted(set(rng.choice(1024, size=14, replace=False).tolist()) | {0, 1023})
        _print("c3 headline: oracle ids of", len(pick), "queries")
        for i, (st, cnt, want) in zip(pick, oracle_queries(cols, [qs[i] for i in pick])):
            got = out[i, :ans[i].written].cpu().numpy().view(np.uint32)
            assert ans[i].written == cnt and np.array_equal(got, want), i


@pytest.mark.parametrize("factor", [4_000_000, 1])
def test_estimate_sized_scratch_is_exact_and_falls_back(factor):
    """Batches with MDRQ_Q_SIZE_ESTIMATED: queries predicted to have small results keep
    only their chunks with a hit, in room for the reserve factor times the estimate
    (default four times); at a factor of 10^-6 nearly every such query outgrows its room
    and is answered again by the single-query scan.  Either way every count, id list
    and bitmap equals the oracle's, in every output mode and on a ragged row count."""
    from paper_1801_03644_amd.mdrq import Estimator

    w = dg.workload("c5", 1_000_003)
    raw = w.columns()
    cols = oracle.prepare(raw)
    qs = dg.workload_queries(w, 96, sampler=w.sampler(sample_rows=1 << 15), seed=4)
    qs[0] = dg.make_query([(0, 0.5, 0.4)])            # empty
    qs[1] = dg.make_query([])                          # every row
    qs[2] = dg.make_query([(1, 0.3, 0.3000001)])       # (nearly) a point
    modes = [("ids", "bitmap", "auto", "count")[i % 4] for i in range(len(qs))]
    with mdrq.Dataset.from_host(raw) as ds, Estimator(ds) as est:
        ds.attach_estimator(est)
        ds.set_option(mdrq.OPT_RESERVE_FACTOR, factor)
        ds.reset_profile()
        outs = make_outs(ds.n_rows, modes)
        ans = ds.query_batch(qs, outs, modes, flags=mdrq.Q_SIZE_ESTIMATED | mdrq.Q_ORDER_ESTIMATED)
        sized, reruns = ds.sizing_profile()
        _print("factor", factor, "sized by estimate", sized, "answered again", reruns)
        assert sized > 0
        if factor == 1:
            assert reruns > 0
        for i, (q, m, a, o) in enumerate(zip(qs, modes, ans, outs)):
            st, cnt, want = oracle.query(cols, q)
            assert a.count == cnt, (i, m)
            if m == "count":
                continue
            got = payload(o, a, ds.n_rows)
            assert np.array_equal(got, want), (i, m, a.mode)
        ds.attach_estimator(None)


def test_batch_graph_replays_match_direct_launches():
    """Shared scans replay a graph per scan kernel with each batch's arguments, grid and
    buffers: batches of different sizes, unions and modes alternate through the graphs,
    with other device work between them, then the same batches with direct launches;
    every result equals the oracle's."""
    import torch

    w = dg.workload("c3", 400_009)
    raw = w.columns()
    cols = oracle.prepare(raw)
    samp = w.sampler(sample_rows=1 << 14)
    batches = [dg.workload_queries(w, n, sampler=samp, seed=s) for n, s in ((40, 1), (7, 2), (130, 3), (40, 4))]
    with mdrq.Dataset.from_host(raw) as ds:
        for graphs in (2, 0):
            ds.set_option(mdrq.OPT_GRAPHS, graphs)   # bit 1: shared scans
            for rep in range(2):
                for b, qs in enumerate(batches):
                    x = torch.randn(1 << 16, device=device())
                    _ = (x * 3).sum().item()
                    modes = [("ids", "bitmap", "auto", "count")[(i + rep + b) % 4] for i in range(len(qs))]
                    check_batch(ds, cols, qs, modes, label=f"graphs={graphs} rep={rep} batch={b}")
