"""mdrq_query_noalloc (the library's fixed per-GPU scratch instead of the dataset's
workspace) against mdrq_query and the oracle: identical counts, ascending ids and
bitmap words, on two calls in a row whose second input is smaller than the first (the
scratch keeps the first call's contents), in every output mode."""
import numpy as np
import pytest

import oracle
from paper_1801_03644_amd import datagen as dg
from paper_1801_03644_amd import mdrq
from tests.gpu_helpers import bitmap_to_ids, device

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def _both(ds, q, mode, cap=None):
    """(answer, payload) of mdrq_query and of mdrq_query_noalloc on the same query."""
    import torch

    out = []
    for fn in (ds.query, ds.query_noalloc):
        if mode == "count":
            out.append((fn(q, None, mode="count"), None))
            continue
        if mode == "bitmap":
            n = (ds.n_rows + 63) // 64 if cap is None else cap
            buf = torch.full((max(1, n),), -1, dtype=torch.int64, device=device())[:n]
        else:
            n = max(ds.n_rows, 2 * ((ds.n_rows + 63) // 64)) if cap is None else cap
            buf = torch.full((max(1, n),), -1, dtype=torch.int32, device=device())[:n]
        a = fn(q, buf, mode=mode)
        raw = buf.cpu().numpy().view(np.uint8)
        if a.mode == "bitmap":
            out.append((a, bitmap_to_ids(raw[:8 * a.written].view(np.uint64), ds.n_rows)[0]))
        else:
            out.append((a, raw[:4 * a.written].view(np.uint32).copy()))
    return out


@pytest.mark.parametrize("mode", ["ids", "bitmap", "count", "auto"])
def test_noalloc_matches_query_on_a_larger_then_a_smaller_input(mode):
    for n, seed in ((3_000_017, 0), (70_001, 1)):
        w = dg.workload("c2", n)
        raw = w.columns()
        cols = oracle.prepare(raw)
        qs = dg.workload_queries(w, 6, sampler=w.sampler(sample_rows=1 << 14), seed=seed)
        qs.append(dg.make_query([(1, 0.0, 1.0)]))          # nearly every row
        qs.append(dg.make_query([]))                       # every row
        qs.append(dg.make_query([(2, 0.6, 0.3)]))          # empty interval
        with mdrq.Dataset.from_host(raw) as ds:
            for i, q in enumerate(qs):
                _print("noalloc", mode, n, i)
                (a, got), (b, got_na) = _both(ds, q, mode)
                st, cnt, want = oracle.query(cols, q)
                assert a.count == b.count == cnt, (n, i)
                assert (a.mode, a.written, a.status) == (b.mode, b.written, b.status), (n, i)
                if mode != "count":
                    assert np.array_equal(got_na, want), (n, i)
                    assert np.array_equal(got, got_na), (n, i)


def test_noalloc_overflow_and_limits():
    import torch

    w = dg.workload("c2", 500_003)
    raw = w.columns()
    cols = oracle.prepare(raw)
    q = dg.make_query([(0, 0.1, 0.6)])
    st, cnt, want = oracle.query(cols, q)
    with mdrq.Dataset.from_host(raw) as ds:
        # a buffer too small: exact count, the first ids, EOVERFLOW
        (a, got), (b, got_na) = _both(ds, q, "ids", cap=1000)
        assert b.count == cnt and b.status == mdrq.EOVERFLOW and np.array_equal(got_na, want[:1000])
        (a, got), (b, got_na) = _both(ds, q, "bitmap", cap=7)
        assert b.count == cnt and b.status == mdrq.EOVERFLOW and b.written == 7
        # host outputs and estimated order are not served here
        with pytest.raises(mdrq.MdrqError) as e:
            ds.query_noalloc(q, np.zeros(10, dtype=np.uint32), mode="ids")
        assert e.value.code == mdrq.EINVAL
        with pytest.raises(mdrq.MdrqError) as e:
            ds.query_noalloc(q, None, mode="count", flags=mdrq.Q_ORDER_ESTIMATED)
        assert e.value.code == mdrq.ENOTSUP
    # a dataset larger than the fixed scratch is refused with a clear error
    big = torch.zeros(300_000_000, dtype=torch.float32, device=device())
    with mdrq.Dataset.from_device([big], borrow=True) as ds:
        with pytest.raises(mdrq.MdrqError) as e:
            ds.query_noalloc(dg.make_query([(0, 0.0, 1.0)]), None, mode="count")
        assert e.value.code == mdrq.ENOTSUP and "scratch" in str(e.value)
        assert ds.query(dg.make_query([(0, 0.0, 1.0)]), None, mode="count").count == 300_000_000
