"""The binding's batch marshalling: the query records built for a whole batch as numpy
fields (one predicate array, per-query offsets) equal, query by query, the records that
make_query builds one at a time -- for queries given as three arrays or as (dim, lo,
hi) tuples, empty queries, NaN and infinite bounds, float64 bounds that round, and
out-of-range dimensions (passed through for the library to reject)."""
import ctypes

import numpy as np

from paper_1801_03644_amd import mdrq


def _queries(rng, n):
    qs = []
    for i in range(n):
        k = int(rng.integers(0, 6))
        dims = rng.permutation(12)[:k].astype(np.uint32)
        lo = rng.uniform(-1, 1, size=k)
        hi = lo + rng.uniform(0, 1, size=k)
        if i % 5 == 0:
            qs.append((dims, lo.astype(np.float32), hi.astype(np.float32)))
        elif i % 5 == 1:
            qs.append([(int(d), float(a), float(b)) for d, a, b in zip(dims, lo, hi)])
        elif i % 5 == 2:
            qs.append((dims, lo, hi))              # float64 bounds: rounded to float32
        elif i % 5 == 3:
            qs.append([])                          # every row
        else:
            qs.append([(3, float("nan"), 1.0), (70, -np.inf, np.inf), (-1, 0.5, 0.25)])
    return qs


def _same(a, b):
    return a == b or (np.isnan(a) and np.isnan(b))


def test_batch_records_equal_single_records():
    rng = np.random.default_rng(7)
    qs = _queries(rng, 400)
    for flags in (0, mdrq.Q_NO_EARLYOUT, mdrq.Q_ORDER_ESTIMATED):
        arr, keep = mdrq._query_array(qs, flags)
        assert len(arr) == len(qs)
        for i, q in enumerate(qs):
            ref, _ = mdrq.make_query(q, flags)
            got = arr[i]
            assert got.n_preds == ref.n_preds and got.flags == ref.flags, i
            if ref.n_preds == 0:
                assert not got.preds, i
            for j in range(ref.n_preds):
                a, b = got.preds[j], ref.preds[j]
                assert a.dim == b.dim and _same(a.lo, b.lo) and _same(a.hi, b.hi), (i, j)


def test_empty_batch_and_result_records():
    arr, keep = mdrq._query_array([], 0)
    assert len(arr) == 1 and arr[0].n_preds == 0
    assert mdrq._RESULT_DT.itemsize == ctypes.sizeof(mdrq.Result)
    rec = np.zeros(3, dtype=mdrq._RESULT_DT)
    rarr = (mdrq.Result * 3).from_buffer(rec)
    rarr[1].count = 12345
    rarr[2].status = -7
    assert rec["count"][1] == 12345 and rec["status"][2] == -7
