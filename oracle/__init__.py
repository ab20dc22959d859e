"""CPU oracle for exact multidimensional range queries.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's CPU
baseline may use this package; the product library never imports, links or calls it.
It shares no code with the GPU path (only the seeded input generators feed both).

The scan itself is plain C in ``mdrq_oracle.c`` (the paper's problem definition,
section 2.1, evaluated as its sequential scan with early break, section 2.2.4, on
column arrays as in section 5.5).  This module loads it through ctypes and adds the
definitions built directly on top of it: selectivity and per-dimension selectivity
(section 2.1), and batches answered query by query.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mdrq_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, EINVAL, EOVERFLOW = 0, -1, -3


def build() -> str:
    """Compile the oracle with gcc (-O2, IEEE semantics, no fast-math)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-std=c99", "-O2", "-fno-fast-math", "-fPIC", "-shared",
                           "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.POINTER
    colsT = P(P(ctypes.c_float))
    u32, u64 = ctypes.c_uint32, ctypes.c_uint64
    common = [colsT, u32, u64, P(u32), P(ctypes.c_float), P(ctypes.c_float), u32]
    lib.oracle_query.argtypes = common + [P(u32), u64, P(u64)]
    lib.oracle_bitmap.argtypes = common + [P(u64), P(u64)]
    lib.oracle_count.argtypes = common + [P(u64)]
    lib.oracle_match_row.argtypes = common + [u64]
    lib.oracle_validate_columns.argtypes = [colsT, u32, u64, P(ctypes.c_float), P(ctypes.c_float)]
    for f in (lib.oracle_query, lib.oracle_bitmap, lib.oracle_count, lib.oracle_match_row,
              lib.oracle_validate_columns):
        f.restype = ctypes.c_int
    _lib = lib
    return lib


class _Cols:
    """Keeps the float32 column arrays alive and exposes a float** for C."""

    def __init__(self, cols):
        self.arrays = [np.ascontiguousarray(c, dtype=np.float32) for c in cols]
        n = {a.size for a in self.arrays}
        if len(n) > 1:
            raise ValueError("columns differ in length")
        self.n_rows = n.pop() if n else 0
        FP = ctypes.POINTER(ctypes.c_float)
        self.ptrs = (FP * max(1, len(self.arrays)))(*[a.ctypes.data_as(FP) for a in self.arrays])

    @property
    def n_dims(self):
        return len(self.arrays)


def _as_cols(cols):
    return cols if isinstance(cols, _Cols) else _Cols(cols)


def prepare(cols) -> _Cols:
    """Wrap column arrays once so repeated oracle calls do not re-marshal them."""
    return _as_cols(cols)


def _qargs(query):
    dims, lo, hi = query
    dims = np.ascontiguousarray(dims, dtype=np.uint32)
    lo = np.ascontiguousarray(lo, dtype=np.float32)
    hi = np.ascontiguousarray(hi, dtype=np.float32)
    if not (dims.size == lo.size == hi.size):
        raise ValueError("query arrays differ in length")
    P = ctypes.POINTER
    return (dims, lo, hi), (dims.ctypes.data_as(P(ctypes.c_uint32)),
                            lo.ctypes.data_as(P(ctypes.c_float)),
                            hi.ctypes.data_as(P(ctypes.c_float)), dims.size)


def query(cols, query, capacity: int | None = None):
    """(status, count, ids): ascending uint32 identifiers of the qualifying objects.
    With capacity=None the buffer holds every identifier."""
    lib = _load()
    c = _as_cols(cols)
    keep, qa = _qargs(query)
    cnt = ctypes.c_uint64(0)
    if capacity is None:
        rc = lib.oracle_count(c.ptrs, c.n_dims, c.n_rows, *qa, ctypes.byref(cnt))
        if rc != OK:
            return rc, 0, np.empty(0, dtype=np.uint32)
        capacity = cnt.value
    ids = np.empty(max(1, capacity), dtype=np.uint32)
    rc = lib.oracle_query(c.ptrs, c.n_dims, c.n_rows, *qa,
                          ids.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), capacity,
                          ctypes.byref(cnt))
    if rc == EINVAL:
        return rc, 0, np.empty(0, dtype=np.uint32)
    return rc, cnt.value, ids[:min(capacity, cnt.value)].copy()


def count(cols, query) -> int:
    lib = _load()
    c = _as_cols(cols)
    keep, qa = _qargs(query)
    cnt = ctypes.c_uint64(0)
    rc = lib.oracle_count(c.ptrs, c.n_dims, c.n_rows, *qa, ctypes.byref(cnt))
    if rc != OK:
        raise ValueError(f"invalid query (status {rc})")
    return cnt.value


def bitmap(cols, query):
    """(status, count, words): uint64 words, bit i%64 of word i//64 <=> object i qualifies."""
    lib = _load()
    c = _as_cols(cols)
    keep, qa = _qargs(query)
    words = np.zeros(max(1, (c.n_rows + 63) // 64), dtype=np.uint64)
    cnt = ctypes.c_uint64(0)
    rc = lib.oracle_bitmap(c.ptrs, c.n_dims, c.n_rows, *qa,
                           words.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), ctypes.byref(cnt))
    return rc, cnt.value, words[:(c.n_rows + 63) // 64]


def match_row(cols, query, row: int) -> bool:
    lib = _load()
    c = _as_cols(cols)
    keep, qa = _qargs(query)
    rc = lib.oracle_match_row(c.ptrs, c.n_dims, c.n_rows, *qa, row)
    if rc < 0:
        raise ValueError(f"invalid query or row (status {rc})")
    return bool(rc)


def validate_columns(cols):
    """(status, min[d], max[d]); status EINVAL if any value is NaN."""
    lib = _load()
    c = _as_cols(cols)
    mn = np.empty(max(1, c.n_dims), dtype=np.float32)
    mx = np.empty(max(1, c.n_dims), dtype=np.float32)
    FP = ctypes.POINTER(ctypes.c_float)
    rc = lib.oracle_validate_columns(c.ptrs, c.n_dims, c.n_rows, mn.ctypes.data_as(FP),
                                     mx.ctypes.data_as(FP))
    return rc, mn[:c.n_dims], mx[:c.n_dims]


def selectivity(cols, query) -> float:
    """sel(MDRQ): fraction of objects that qualify (section 2.1)."""
    c = _as_cols(cols)
    return count(c, query) / c.n_rows if c.n_rows else 0.0


def dim_selectivities(cols, query) -> np.ndarray:
    """sel_j(MDRQ) for each predicate of the query, in the query's order (section 2.1)."""
    c = _as_cols(cols)
    dims, lo, hi = query
    return np.array([count(c, (dims[i:i + 1], lo[i:i + 1], hi[i:i + 1])) / c.n_rows
                     for i in range(len(dims))], dtype=np.float64)


def batch(cols, queries, capacity: int | None = None):
    """Each query of a batch answered on its own: a query's result does not depend on
    the other queries it is batched or served with."""
    c = _as_cols(cols)
    return [query(c, q, capacity) for q in queries]
