"""GPU parity of the live server (mdrq_serve_open / submit / poll / close): every
request's result is the oracle's whatever it was batched with, admission control
rejects submissions beyond the queue bound, and closing answers everything that was
accepted."""
import time

import numpy as np
import pytest

import oracle
from paper_1801_03644_amd import datagen as dg
from paper_1801_03644_amd import mdrq
from tests.gpu_helpers import run
from tests.test_gpu_serve import c5_small, check, outputs

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("segments", [0, 5])
def test_live_server_results_match_oracle(segments):
    """Continuous batching (segments 0) and the circular scan (5 parts per pass), with
    submissions in bursts while earlier requests are being scanned."""
    w, raw = c5_small(300_007)
    cols = oracle.prepare(raw)
    pool = dg.workload_queries(w, 48, sampler=w.sampler(sample_rows=1 << 16))
    pool[0] = dg.make_query([])                       # every row
    pool[1] = dg.make_query([(2, 0.6, 0.1)])          # empty interval
    rng = np.random.default_rng(3)
    n = 240
    qs = [pool[i] for i in rng.integers(0, len(pool), size=n)]
    modes = [["ids", "bitmap", "count", "auto"][i % 4] for i in range(n)]
    with mdrq.Dataset.from_host(raw) as ds:
        outs = outputs(ds.n_rows, modes)
        answers = [None] * n
        with ds.serve_open(max_batch=32, n_streams=2, budget_bytes=1 << 26, segments=segments) as srv:
            _print("live: submitting", n, "segments", segments)
            tickets = {}
            for i in range(n):
                tickets[srv.submit(qs[i], outs[i], modes[i])] = i
                if i % 16 == 15:   # bursts, with polls in between
                    for t, a in srv.poll():
                        answers[tickets[t]] = a
                    time.sleep(0.0005)
            assert sorted(tickets) == list(range(n))   # tickets in submission order
            deadline = time.time() + 60
            while any(a is None for a in answers) and time.time() < deadline:
                for t, a in srv.poll(wait_s=0.05):
                    answers[tickets[t]] = a
            stats = srv.close()
        _print(stats)
        assert all(a is not None for a in answers)
        check(ds, cols, qs, modes, outs, answers, "live")
        assert stats["completed"] == n and stats["scans"] >= 1
        assert stats["p50_us"] <= stats["p99_us"] <= stats["max_us"]
        # the same queries alone
        for i in range(0, n, 29):
            if modes[i] == "ids":
                a1, ids1 = run(ds, qs[i])
                assert a1.count == answers[i].count


def test_live_server_admission_and_close():
    """One stream, at most one waiting request: while the worker scans, a third rapid
    submission is refused with EBUSY; everything accepted is answered, also when the
    server is closed before it was polled."""
    w, raw = c5_small(2_000_000)
    cols = oracle.prepare(raw)
    qs = dg.workload_queries(w, 40, sampler=w.sampler(sample_rows=1 << 16))
    with mdrq.Dataset.from_host(raw) as ds:
        srv = ds.serve_open(max_batch=8, n_streams=1, budget_bytes=1 << 26, max_queue=1)
        accepted, busy = [], 0
        for i, q in enumerate(qs):
            try:
                srv.submit(q, None, "count")
                accepted.append(i)
            except mdrq.MdrqError as e:
                assert e.code == mdrq.EBUSY
                busy += 1
        stats = srv.close()
        res = srv.results()
        assert busy >= 1 and len(accepted) >= 2
        assert stats["completed"] == len(accepted) == len(res)
        for (t, a), i in zip(res, accepted):
            assert a.count == oracle.count(cols, qs[i]), i
        with pytest.raises(mdrq.MdrqError) as e:   # one bitmap row exceeds the share
            with ds.serve_open(n_streams=2, budget_bytes=8 * ((ds.n_rows + 63) // 64)) as s2:
                s2.submit(qs[0], outputs(ds.n_rows, ["ids"])[0], "ids")
        assert e.value.code == mdrq.EBUSY
        with ds.serve_open(n_streams=1) as s3:     # host-memory results are refused
            with pytest.raises(mdrq.MdrqError) as e:
                s3.submit(qs[0], np.zeros(ds.n_rows, dtype=np.uint32), "ids")
            assert e.value.code == mdrq.EINVAL


def test_circular_live_server_close_answers_everything():
    """A circular-scan server closed right after a burst of submissions (none polled):
    close waits for every pass, and every accepted request holds the oracle's answer."""
    w, raw = c5_small(1_000_003)
    cols = oracle.prepare(raw)
    qs = dg.workload_queries(w, 30, sampler=w.sampler(sample_rows=1 << 16))
    modes = ["ids", "count", "bitmap"] * 10
    with mdrq.Dataset.from_host(raw) as ds:
        outs = outputs(ds.n_rows, modes)
        srv = ds.serve_open(max_batch=16, n_streams=2, budget_bytes=1 << 26, segments=6)
        tickets = [srv.submit(q, o, m) for q, o, m in zip(qs, outs, modes)]
        stats = srv.close()
        res = dict(srv.results())
        assert stats["completed"] == len(qs) and sorted(res) == sorted(tickets)
        check(ds, cols, qs, modes, outs, [res[t] for t in tickets], "circular close")


def test_live_server_alongside_single_queries():
    """mdrq_query on the same dataset while a server is open (other stream, no lock on
    the dataset held by the server); the dataset closes an open server first."""
    w, raw = c5_small(200_003)
    cols = oracle.prepare(raw)
    qs = dg.workload_queries(w, 24, sampler=w.sampler(sample_rows=1 << 16))
    ds = mdrq.Dataset.from_host(raw)
    srv = ds.serve_open(max_batch=16, n_streams=2, budget_bytes=1 << 26)
    outs = outputs(ds.n_rows, ["ids"] * len(qs))
    tickets = [srv.submit(q, o, "ids") for q, o in zip(qs, outs)]
    for q in qs[:6]:
        a1, ids1 = run(ds, q)
        st, cnt, want = oracle.query(cols, q)
        assert a1.count == cnt and np.array_equal(ids1, want)
    got = {}
    deadline = time.time() + 60
    while len(got) < len(tickets) and time.time() < deadline:
        got.update(dict(srv.poll(wait_s=0.05)))
    answers = [got[t] for t in tickets]
    check(ds, cols, qs, ["ids"] * len(qs), outs, answers, "alongside")
    srv.submit(qs[0], outs[0], "ids")   # left open: closing the dataset closes it
    ds.close()
