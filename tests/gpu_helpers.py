"""Helpers for GPU parity tests: run the library through its C ABI and fetch results."""
import numpy as np

from paper_1801_03644_amd import mdrq


def device():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("GPU test needs a GPU")
    return torch.device("cuda:0")


def run(ds, q, mode="ids", cap=None, flags=0, host=False):
    """(Answer, payload): payload is the uint32 ids, the uint64 words or None."""
    import torch

    if mode == "count":
        return ds.query(q, None, mode="count", flags=flags), None
    if mode == "ids":
        cap = ds.n_rows if cap is None else cap
        if host:
            out = np.zeros(cap, dtype=np.uint32)
        else:
            out = torch.full((cap,), -1, dtype=torch.int32, device=device())
        a = ds.query(q, out, mode="ids", flags=flags)
        got = out if host else out.cpu().numpy().view(np.uint32)
        return a, got[:a.written].copy()
    words = (ds.n_rows + 63) // 64 if cap is None else cap
    if host:
        out = np.zeros(words, dtype=np.uint64)
    else:
        out = torch.full((words,), -1, dtype=torch.int64, device=device())
    a = ds.query(q, out, mode="bitmap", flags=flags)
    got = out if host else out.cpu().numpy().view(np.uint64)
    return a, got[:a.written].copy()


def bitmap_to_ids(words, n_rows):
    bits = np.unpackbits(np.ascontiguousarray(words).view(np.uint8), bitorder="little")
    return np.flatnonzero(bits[:n_rows]).astype(np.uint32), bits[n_rows:]


def oracle_counts(cols, queries, threads=None):
    """Oracle counts of many queries on host threads (each call is the unchanged
    single-threaded oracle; ctypes releases the interpreter lock during it)."""
    import os
    from concurrent.futures import ThreadPoolExecutor

    import oracle

    oracle._load()  # once, before the threads
    threads = threads or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(threads) as ex:
        return list(ex.map(lambda q: oracle.count(cols, q), queries))


def oracle_queries(cols, queries, threads=None):
    """(status, count, ids) of each query from the oracle, on host threads."""
    import os
    from concurrent.futures import ThreadPoolExecutor

    import oracle

    oracle._load()
    threads = threads or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(threads) as ex:
        return list(ex.map(lambda q: oracle.query(cols, q), queries))
