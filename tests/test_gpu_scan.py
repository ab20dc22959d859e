"""GPU parity of the single-query scan (mdrq_query) against the CPU oracle.

Integer results, so the bar is bit-exact: identical counts and identical ascending
identifier lists; bitmaps decode to the same identifiers with zero padding bits.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_1801_03644_amd import datagen as dg
from paper_1801_03644_amd import mdrq
from tests.gpu_helpers import bitmap_to_ids, device, run

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def assert_same(ds, cols, q, modes=("ids", "bitmap", "count"), flags=0, label=""):
    st_, want_cnt, want = oracle.query(cols, q)
    assert st_ == oracle.OK
    for mode in modes:
        a, got = run(ds, q, mode=mode, flags=flags)
        assert a.count == want_cnt, (label, mode, a.count, want_cnt)
        assert a.status == mdrq.OK
        if mode == "ids":
            assert a.written == want_cnt
            assert np.array_equal(got, want), (label, mode)
        elif mode == "bitmap":
            ids, pad = bitmap_to_ids(got, ds.n_rows)
            assert np.array_equal(ids, want), (label, mode)
            assert not pad.any(), (label, "bits past n_rows must be zero")


@pytest.fixture(scope="module")
def c1():
    w = dg.workload("c1")
    raw = w.columns()
    _print("c1: loading", w.n_rows, "x", w.n_dims)
    ds = mdrq.Dataset.from_host(raw)
    yield w, raw, oracle.prepare(raw), ds
    ds.close()


def test_c1_all_queries_bit_exact(c1):
    w, raw, cols, ds = c1
    qs = dg.workload_queries(w, 100)
    for i, q in enumerate(qs):
        assert_same(ds, cols, q, modes=("ids",) if i % 10 else ("ids", "bitmap", "count"),
                    label=f"c1 q{i}")


def test_column_ranges_found_at_load(c1):
    w, raw, cols, ds = c1
    rc, mn, mx = oracle.validate_columns(cols)
    for j in range(w.n_dims):
        assert ds.column_range(j) == (mn[j], mx[j])


SIZES = [1, 3, 4, 5, 63, 64, 65, 255, 256, 257, 1023, 1024, 1025, 4095, 4096, 4097, 8191, 8193,
         32769, 300001]


@pytest.mark.parametrize("unroll", [0, 1, 2, 4, 8])
def test_sizes_tiles_and_ragged_tails(unroll):
    """unroll 0: the tile height chosen by rows per CU (2 below 6144, 4 below 65536)."""
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    for n in SIZES:
        _print("sizes: unroll", unroll, "n", n)
        raw = [dg.column(11, j, dg.uniform(), n) for j in range(3)]
        cols = oracle.prepare(raw)
        with mdrq.Dataset.from_host(raw) as ds:
            ds.set_option(mdrq.OPT_UNROLL, unroll)
            per_cu = n // cus
            want_u = unroll or (2 if per_cu < 6144 else 4 if per_cu < 65536 else 8)
            assert ds.get_option(mdrq.OPT_UNROLL) == want_u
            rng = np.random.default_rng(n + unroll)
            qs = [dg.make_query([]), dg.make_query([(0, 0.0, 1.0)])]
            for s in (0.5, 0.05, 0.001):
                for _ in range(2):
                    k = int(rng.integers(1, 4))
                    dims = rng.permutation(3)[:k]
                    w = s ** (1 / k)
                    preds = []
                    for j in dims:
                        lo = float(rng.uniform(0, 1 - w))
                        preds.append((int(j), lo, lo + w))
                    qs.append(dg.make_query(preds))
            for i, q in enumerate(qs):
                assert_same(ds, cols, q, label=f"n={n} U={unroll} q{i}")


def test_empty_dataset():
    raw = [np.empty(0, dtype=np.float32)] * 2
    with mdrq.Dataset.from_host(raw) as ds:
        for mode in ("ids", "bitmap", "count"):
            a, got = run(ds, dg.make_query([(0, 0.0, 1.0)]), mode=mode, cap=0)
            assert a.count == 0 and a.status == mdrq.OK


SPECIAL = np.array([-np.inf, -2.5, -1.0, -1e-45, -0.0, 0.0, 1e-45, 1.1754942e-38,
                    1.1754944e-38, 0.25, 0.5, 1.0, 3.0e38, np.inf], dtype=np.float32)


def test_special_values_and_neighbouring_bounds():
    """+-0, +-inf, subnormals and the smallest normal in data and in bounds; bounds equal
    to data values and to their float32 neighbours; lo > hi included."""
    n = 20000
    rng = np.random.default_rng(5)
    raw = [SPECIAL[rng.integers(0, len(SPECIAL), size=n)].astype(np.float32) for _ in range(3)]
    cols = oracle.prepare(raw)
    cands = sorted({float(x) for v in SPECIAL for x in
                    (v, np.nextafter(v, np.float32(np.inf)), np.nextafter(v, np.float32(-np.inf)))})
    with mdrq.Dataset.from_host(raw) as ds:
        for i in range(400):
            k = int(rng.integers(1, 4))
            dims = rng.permutation(3)[:k]
            preds = [(int(j), cands[rng.integers(len(cands))], cands[rng.integers(len(cands))])
                     for j in dims]
            assert_same(ds, cols, dg.make_query(preds),
                        modes=("ids", "bitmap") if i % 4 == 0 else ("ids",), label=f"special {i}")


def test_degenerate_and_invalid_queries():
    n = 5000
    raw = [dg.column(12, j, dg.uniform(), n) for j in range(3)]
    cols = oracle.prepare(raw)
    with mdrq.Dataset.from_host(raw) as ds:
        # lo > hi: empty, including in bitmap mode (all words zero)
        for mode in ("ids", "bitmap", "count"):
            a, got = run(ds, dg.make_query([(0, 0.7, 0.2), (1, 0.0, 1.0)]), mode=mode)
            assert a.count == 0 and a.status == mdrq.OK
            if mode == "bitmap":
                assert a.written == (n + 63) // 64 and not got.any()
        # no predicate / all [-inf, inf]: every row
        assert_same(ds, cols, dg.make_query([]))
        assert_same(ds, cols, dg.make_query([(j, -np.inf, np.inf) for j in range(3)]))
        assert_same(ds, cols, dg.make_query([(1, -np.inf, np.inf), (2, 0.1, 0.2)]))
        bad = [[(0, np.nan, 1.0)], [(0, 0.0, np.nan)], [(3, 0.0, 1.0)],
               [(1, 0.0, 1.0), (1, 0.2, 0.3)]]
        for preds in bad:
            with pytest.raises(mdrq.MdrqError) as e:
                ds.query(dg.make_query(preds), None, mode="count")
            assert e.value.code == mdrq.EINVAL


def test_nan_data_rejected_at_load():
    raw = [dg.column(13, 0, dg.uniform(), 1000)]
    raw[0][777] = np.nan
    with pytest.raises(mdrq.MdrqError) as e:
        mdrq.Dataset.from_host(raw)
    assert e.value.code == mdrq.EINVAL


def test_overflow_returns_exact_count_and_prefix():
    n = 100000
    raw = [dg.column(14, j, dg.uniform(), n) for j in range(2)]
    cols = oracle.prepare(raw)
    q = dg.make_query([(0, 0.1, 0.6), (1, 0.2, 0.9)])
    st_, cnt, want = oracle.query(cols, q)
    with mdrq.Dataset.from_host(raw) as ds:
        for cap in (0, 1, cnt // 3, cnt - 1):
            a, got = run(ds, q, mode="ids", cap=cap)
            assert a.status == mdrq.EOVERFLOW and a.count == cnt and a.written == cap
            assert np.array_equal(got, want[:cap])
        a, got = run(ds, q, mode="ids", cap=cnt)
        assert a.status == mdrq.OK and np.array_equal(got, want)
        a, got = run(ds, q, mode="bitmap", cap=10)
        assert a.status == mdrq.EOVERFLOW and a.count == cnt and a.written == 10
        ids, _ = bitmap_to_ids(got, 640)
        assert np.array_equal(ids, want[want < 640])


def test_predicate_order_and_early_out_do_not_change_results():
    w = dg.workload("c2", 200_000)
    raw = w.columns()
    cols = oracle.prepare(raw)
    qs = dg.workload_queries(w, 12, sampler=w.sampler(sample_rows=1 << 16))
    with mdrq.Dataset.from_host(raw) as ds:
        for i, q in enumerate(qs):
            st_, cnt, want = oracle.query(cols, q)
            k = len(q[0])
            perms = list(itertools.permutations(range(k)))
            rng = np.random.default_rng(i)
            for pi in rng.permutation(len(perms))[:6]:
                p = np.array(perms[pi])
                qq = (q[0][p], q[1][p], q[2][p])
                for flags in (0, mdrq.Q_NO_EARLYOUT):
                    a, got = run(ds, qq, flags=flags)
                    assert a.count == cnt and np.array_equal(got, want)


def test_host_outputs_and_borrowed_columns():
    import torch

    n = 70001
    raw = [dg.column(15, j, dg.gmm(), n) for j in range(4)]
    cols = oracle.prepare(raw)
    q = dg.make_query([(3, 0.2, 0.8), (0, 0.3, 0.95)])
    st_, cnt, want = oracle.query(cols, q)
    with mdrq.Dataset.from_host(raw) as ds:
        a, got = run(ds, q, mode="ids", host=True)
        assert a.count == cnt and np.array_equal(got, want)
        a, got = run(ds, q, mode="bitmap", host=True)
        assert np.array_equal(bitmap_to_ids(got, n)[0], want)
    tens = [torch.from_numpy(c).to(device()) for c in raw]
    for borrow in (False, True):
        with mdrq.Dataset.from_device(tens, borrow=borrow) as ds:
            assert_same(ds, cols, q, label=f"borrow={borrow}")


@pytest.mark.parametrize("grid", [1, 2, 7, 64, 0])
def test_launch_shapes_and_repeat_runs_are_deterministic(grid):
    """Any number of workgroups (down to one) gives the same ordered result; a tiny
    grid makes every workgroup run a long segment of tiles, whose offsets the
    compaction's segment sums must carry."""
    n = 1_000_003
    raw = [dg.column(16, j, dg.uniform(), n) for j in range(2)]
    cols = oracle.prepare(raw)
    q = dg.make_query([(0, 0.05, 0.75), (1, 0.5, 0.9)])
    st_, cnt, want = oracle.query(cols, q)
    with mdrq.Dataset.from_host(raw) as ds:
        for unroll in (1, 8):
            ds.set_option(mdrq.OPT_UNROLL, unroll)
            ds.set_option(mdrq.OPT_GRID, grid)
            for _ in range(3):
                a, got = run(ds, q)
                assert a.count == cnt and np.array_equal(got, want)


def test_gpu_invariants():
    """Intersection of single-dim results, monotonicity and the full domain, on the GPU."""
    n = 250_000
    raw = [dg.column(17, j, dg.gmm(), n) for j in range(3)]
    with mdrq.Dataset.from_host(raw) as ds:
        rng = np.random.default_rng(3)
        for _ in range(10):
            preds = [(j, float(a), float(a + rng.uniform(0.05, 0.6)))
                     for j, a in zip(range(3), rng.uniform(0, 0.5, size=3))]
            ids = set(run(ds, dg.make_query(preds))[1].tolist())
            inter = set(range(n))
            for p in preds:
                inter &= set(run(ds, dg.make_query([p]))[1].tolist())
            assert ids == inter
            wider = [(j, a - 0.01, b + 0.01) for j, a, b in preds]
            assert ids <= set(run(ds, dg.make_query(wider))[1].tolist())
        mn_mx = [ds.column_range(j) for j in range(3)]
        full = run(ds, dg.make_query([(j, a, b) for j, (a, b) in enumerate(mn_mx)]), mode="count")[0]
        assert full.count == n


@pytest.mark.parametrize("host", [False, True])
def test_auto_output_picks_the_smaller_exact_result(host):
    """MDRQ_OUT_AUTO on a single query: the bitmap when it is smaller than the ids
    (selectivity above 1/32) and the buffer holds it, otherwise the ids; decided on the
    device from the exact count.  Both decode to the oracle's ids."""
    import torch

    n = 300_001
    raw = [dg.column(61, j, dg.uniform(), n) for j in range(3)]
    cols = oracle.prepare(raw)
    n_words = (n + 63) // 64
    cases = [((0, 0.0, 0.5),), ((0, 0.0, 0.001),), ((1, 0.2, 0.9), (2, 0.0, 0.3)),
             ((1, 0.5, 0.2),), ((0, 0.0, 1.0), (1, 0.0, 1.0))]
    with mdrq.Dataset.from_host(raw) as ds:
        for preds in cases:
            q = dg.make_query(list(preds))
            st, cnt, want = oracle.query(cols, q)
            for n_bytes in (8 * n_words, 4 * n, 8 * n_words - 8):
                if host:
                    out = np.zeros(n_bytes // 4, dtype=np.uint32)
                else:
                    out = torch.full((n_bytes // 4,), -1, dtype=torch.int32, device=device())
                a = ds.query(q, out, mode="auto")
                buf = (out if host else out.cpu().numpy()).view(np.uint8)
                assert a.count == cnt
                bitmap_wins = 8 * n_words < 4 * cnt or n_bytes < 4 * cnt
                if n_bytes >= 8 * n_words and bitmap_wins:
                    assert a.mode == "bitmap" and a.written == n_words
                    assert np.array_equal(bitmap_to_ids(buf[:8 * n_words].view(np.uint64), n)[0], want)
                else:
                    assert a.mode == "ids"
                    got = buf[:4 * a.written].view(np.uint32)
                    assert np.array_equal(got, want[:len(got)])
                    assert a.status == (mdrq.EOVERFLOW if cnt > n_bytes // 4 else mdrq.OK)


def test_full_size_c2_sampled():
    """The headline shape at full size (10^8 x 17), in the bench's launch configuration
    (ids output, default tile and grid): the first bench queries against the oracle,
    identifier for identifier; two of them also without early break and as bitmaps."""
    w = dg.workload("c2")
    _print("c2 full size: generating")
    raw = w.columns()
    cols = oracle.prepare(raw)
    qs = dg.workload_queries(w, 1000)[:5]
    with mdrq.Dataset.from_host(raw) as ds:
        for i, q in enumerate(qs):
            _print("c2 full size: query", i, "k =", len(q[0]))
            modes = ("ids", "bitmap") if i < 2 else ("ids",)
            assert_same(ds, cols, q, modes=modes, label=f"c2 full {i}")
            if i < 2:
                assert_same(ds, cols, q, modes=("ids",), flags=mdrq.Q_NO_EARLYOUT,
                            label=f"c2 full {i} no early break")


def _lines_reference(raw, query, early_out=True):
    """128-byte lines (32 rows) per predicate, in the given order, holding a row that
    every earlier predicate accepted (numpy, from the definition of the early break)."""
    n = len(raw[0])
    n_lines = (n + 31) // 32
    alive = np.ones(n, dtype=bool)
    total = 0
    for j, lo, hi in zip(*query):
        if lo == -np.inf and hi == np.inf:
            continue
        if lo > hi:
            return 0
        pad = np.zeros(n_lines * 32, dtype=bool)
        pad[:n] = alive if early_out else True
        total += int(pad.reshape(n_lines, 32).any(axis=1).sum())
        x = raw[j]
        alive &= (np.float32(lo) <= x) & (x <= np.float32(hi))
    return 128 * total


def test_read_bytes_measurement():
    """mdrq_query_read_bytes (the early break's own column bytes, for the roofline)
    equals the line count taken from the definition, with and without early-out, on
    ragged row counts and over wide and narrow predicates."""
    for n in (1, 31, 33, 200_017):
        w = dg.workload("c2", n)
        raw = w.columns()
        qs = dg.workload_queries(w, 12, sampler=w.sampler(sample_rows=min(n, 1 << 14)))
        qs.append(dg.make_query([(0, -np.inf, np.inf), (3, 0.2, 0.9), (5, 0.1, 0.15)]))
        qs.append(dg.make_query([(2, 0.5, 0.4)]))
        qs.append(dg.make_query([]))
        with mdrq.Dataset.from_host(raw) as ds:
            for q in qs:
                assert ds.read_bytes(q) == _lines_reference(raw, q), (n, q)
                assert ds.read_bytes(q, flags=mdrq.Q_NO_EARLYOUT) == _lines_reference(raw, q, False)


def test_graph_replays_match_direct_launches():
    """Single queries replay a captured graph per launch shape with each query's
    arguments: different queries and modes alternate through the same graphs, with
    other device work and synchronisations between replays, with profiling events on
    and off; every replay equals the oracle and the directly launched kernels."""
    import torch

    w = dg.workload("c2", 300_007)
    raw = w.columns()
    cols = oracle.prepare(raw)
    qs = dg.workload_queries(w, 10, sampler=w.sampler(sample_rows=1 << 14))
    want = [oracle.query(cols, q) for q in qs]
    with mdrq.Dataset.from_host(raw) as ds:
        results = {}
        for graphs in (1, 0):
            ds.set_option(mdrq.OPT_GRAPHS, graphs)   # bit 0: single queries
            for rep in range(3):
                ds.set_profiling(rep == 1)
                for i, q in enumerate(qs):
                    x = torch.randn(1 << 16, device=device())
                    _ = (x * 2).sum().item()            # unrelated work between replays
                    a, ids = run(ds, q)
                    st, cnt, ref = want[i]
                    assert a.count == cnt and np.array_equal(ids, ref), (graphs, rep, i)
                    b, words = run(ds, q, mode="bitmap")
                    assert np.array_equal(bitmap_to_ids(words, ds.n_rows)[0], ref), (graphs, rep, i)
                    c, _ = run(ds, q, mode="count")
                    assert c.count == cnt
                    results[(graphs, rep, i)] = (a.count, ids.tobytes(), words.tobytes())
            ds.set_profiling(False)
        for key, val in results.items():
            assert val == results[(0, key[1], key[2])], key
        launches, scan_ms, total_ms = ds.profile()
        assert launches > 0 and 0 < scan_ms <= total_ms


@pytest.mark.parametrize("unroll", [0, 1, 8])
def test_dense_chunks_and_caps(unroll):
    """Chunks of 4096 rows with more than 2048 hits (written word by word, one bit per
    lane) next to sparser ones (staged in LDS), whole and cut by the output's capacity
    inside a chunk."""
    n = 1_000_003
    raw = [dg.column(23, j, dg.uniform(), n) for j in range(2)]
    cols = oracle.prepare(raw)
    with mdrq.Dataset.from_host(raw) as ds:
        ds.set_option(mdrq.OPT_UNROLL, unroll)
        for preds in ([(0, 0.0, 1.0)], [(0, 0.0, 0.9)], [(0, 0.2, 0.75)], [(0, 0.0, 0.52)],
                      [(0, 0.1, 0.99), (1, 0.0, 0.97)]):
            q = dg.make_query(preds)
            st_, cnt, want = oracle.query(cols, q)
            _print("dense: unroll", unroll, preds, cnt)
            a, got = run(ds, q)
            assert a.count == cnt and np.array_equal(got, want)
            for cap in (cnt // 2 + 37, 3 * 4096 + 5):
                a, got = run(ds, q, cap=cap)
                assert a.status == mdrq.EOVERFLOW and a.count == cnt and a.written == cap
                assert np.array_equal(got, want[:cap])
