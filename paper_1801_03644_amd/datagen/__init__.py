"""Seeded synthetic columns and range queries.

This module draws inputs only; it contains none of the range-query arithmetic.  The
GPU path and the CPU oracle both consume its output and share nothing else.

Column values come from ``datagen.c`` (counter-based SplitMix64, one value per
(seed, column, row), identical for any thread count).  Queries are drawn with
numpy's PCG64 generator from a fixed seed.

Workload shapes follow the paper's data sets (Table 2, section 7.2) and the five
synthetic configurations built from them:

* ``c1`` 10^6 x 3 uniform columns, 100 queries on all dims at ~1% selectivity.
* ``c2`` 10^8 x 17 columns (8 uniform, 8 Gaussian-mixture, 1 Zipf), 1,000 queries
  on 2-8 dims, target selectivity log-uniform in [1e-5, 0.2].
* ``c3`` 5*10^7 x 8 columns (4 uniform, 4 Gaussian-mixture), batches of queries on
  1-8 dims.
* ``c4`` 10^8 x 20 columns in 10 correlated pairs.
* ``c5`` 2*10^8 x 12 columns (4 uniform, 4 Gaussian-mixture, 4 Zipf).
* ``syntuni`` the paper's SYNT-UNI: uniform [0,1] on 10^6 + 1 levels, queries
  spanned by two random data objects (section 7.2.1).
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(os.path.dirname(_HERE), "lib", "libmdrq_datagen.so")
_lib = None

UNIFORM24, GMM, ZIPF, CORR, GRID = 0, 1, 2, 3, 4


class _Spec(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("iparam", ctypes.c_int32), ("fparam", ctypes.c_double)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from .. import build as _build

        _build.build_datagen()
    lib = ctypes.CDLL(_LIB_PATH)
    u64, u32, i32 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
    fptr = ctypes.POINTER(ctypes.c_float)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.dg_column.argtypes = [u64, u32, ctypes.POINTER(_Spec), u64, u64, fptr, i32]
    lib.dg_column.restype = i32
    lib.dg_column_at.argtypes = [u64, u32, ctypes.POINTER(_Spec), u64p, u64, fptr, i32]
    lib.dg_column_at.restype = i32
    lib.dg_rows.argtypes = [u64, u64, u64, u64, u64p]
    lib.dg_rows.restype = i32
    lib.dg_raw.argtypes = [u64, u64, u64, u64, u64p]
    lib.dg_raw.restype = i32
    _lib = lib
    return lib


def _threads() -> int:
    for var in ("MDRQ_GEN_THREADS", "OMP_NUM_THREADS"):
        v = os.environ.get(var)
        if v and v.isdigit() and int(v) > 0:
            return int(v)
    return max(1, min(16, os.cpu_count() or 1))


@dataclass(frozen=True)
class ColumnSpec:
    kind: int
    iparam: int = 0
    fparam: float = 0.0

    def _c(self) -> _Spec:
        return _Spec(self.kind, self.iparam, self.fparam)


def uniform() -> ColumnSpec:
    return ColumnSpec(UNIFORM24)


def gmm(components: int = 32, sigma: float = 0.02) -> ColumnSpec:
    return ColumnSpec(GMM, components, sigma)


def zipf(n: int = 10_000, s: float = 1.1) -> ColumnSpec:
    return ColumnSpec(ZIPF, n, s)


def corr(source: int, sigma: float = 0.05) -> ColumnSpec:
    return ColumnSpec(CORR, source, sigma)


def grid(levels: int = 1_000_000) -> ColumnSpec:
    return ColumnSpec(GRID, levels, 0.0)


def column(seed: int, col: int, spec: ColumnSpec, n: int, row0: int = 0, out=None) -> np.ndarray:
    """float32 values of column ``col`` for rows row0 .. row0+n-1."""
    lib = _load()
    if out is None:
        out = np.empty(n, dtype=np.float32)
    assert out.dtype == np.float32 and out.flags.c_contiguous and out.size >= n
    if n:
        rc = lib.dg_column(seed, col, ctypes.byref(spec._c()), row0, n,
                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), _threads())
        if rc != 0:
            raise ValueError(f"dg_column failed ({rc}) for {spec}")
    return out


def column_at(seed: int, col: int, spec: ColumnSpec, rows: np.ndarray) -> np.ndarray:
    """float32 values of column ``col`` at the given row indices."""
    lib = _load()
    rows = np.ascontiguousarray(rows, dtype=np.uint64)
    out = np.empty(rows.size, dtype=np.float32)
    if rows.size:
        rc = lib.dg_column_at(seed, col, ctypes.byref(spec._c()),
                              rows.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), rows.size,
                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), _threads())
        if rc != 0:
            raise ValueError(f"dg_column_at failed ({rc})")
    return out


def random_rows(seed: int, stream: int, n_rows: int, n: int) -> np.ndarray:
    lib = _load()
    out = np.empty(n, dtype=np.uint64)
    rc = lib.dg_rows(seed, stream, n_rows, n, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    if rc != 0:
        raise ValueError("dg_rows failed")
    return out


def raw(seed: int, stream: int, n: int, ctr0: int = 0) -> np.ndarray:
    lib = _load()
    out = np.empty(n, dtype=np.uint64)
    lib.dg_raw(seed, stream, ctr0, n, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    return out


# --------------------------------------------------------------------------------------
# Queries.  A query is a tuple (dims uint32[k], lo float32[k], hi float32[k]).
# --------------------------------------------------------------------------------------

def make_query(preds) -> tuple:
    dims = np.array([p[0] for p in preds], dtype=np.uint32)
    lo = np.array([p[1] for p in preds], dtype=np.float32)
    hi = np.array([p[2] for p in preds], dtype=np.float32)
    return dims, lo, hi


def box_queries(n_queries: int, n_dims: int, selectivity: float, seed: int) -> list:
    """Queries on every dim of uniform [0,1) data, each interval of width
    selectivity**(1/n_dims) with a uniform random start chosen so the box fits in [0,1)."""
    rng = np.random.default_rng(seed)
    w = selectivity ** (1.0 / n_dims)
    out = []
    for _ in range(n_queries):
        lo = rng.uniform(0.0, 1.0 - w, size=n_dims).astype(np.float32)
        hi = (lo.astype(np.float64) + w).astype(np.float32)
        out.append((np.arange(n_dims, dtype=np.uint32), lo, hi))
    return out


@dataclass
class QuantileSampler:
    """Sorted seeded row samples of each column: empirical quantile functions."""
    samples: list = field(default_factory=list)

    @classmethod
    def build(cls, seed: int, specs, n_rows: int, sample_rows: int = 1 << 20, stream: int = 77):
        m = min(sample_rows, n_rows)
        rows = random_rows(seed, stream, n_rows, m)
        return cls([np.sort(column_at(seed, j, s, rows)) for j, s in enumerate(specs)])

    def q(self, j: int, p: np.ndarray | float):
        s = self.samples[j]
        idx = np.minimum(len(s) - 1, np.floor(np.asarray(p) * len(s)).astype(np.int64))
        return s[np.maximum(idx, 0)]


def quantile_queries(sampler: QuantileSampler, n_queries: int, k_range, s_range, seed: int,
                     dims_pool=None) -> list:
    """Queries on a random k-subset of dims (k uniform in k_range, inclusive) with a target
    selectivity s log-uniform in s_range, split unevenly as s_j = s**w_j with
    w ~ Dirichlet(1,...,1); per dim the interval spans the empirical quantiles
    [Q_j(u), Q_j(u + s_j)] with u ~ U[0, 1 - s_j]."""
    rng = np.random.default_rng(seed)
    d = len(sampler.samples)
    pool = np.arange(d) if dims_pool is None else np.asarray(dims_pool)
    kmin, kmax = k_range
    smin, smax = s_range
    out = []
    for _ in range(n_queries):
        k = int(rng.integers(kmin, kmax + 1))
        dims = rng.choice(pool, size=k, replace=False).astype(np.uint32)
        s = math.exp(rng.uniform(math.log(smin), math.log(smax)))
        w = rng.dirichlet(np.ones(k))
        sj = s ** w
        lo = np.empty(k, dtype=np.float32)
        hi = np.empty(k, dtype=np.float32)
        for i, j in enumerate(dims):
            u = rng.uniform(0.0, 1.0 - sj[i])
            lo[i] = sampler.q(int(j), u)
            hi[i] = sampler.q(int(j), u + sj[i])
        out.append((dims, lo, hi))
    return out


def two_object_queries(cols, n_queries: int, seed: int) -> list:
    """Paper section 7.2.1: pick two distinct data objects at random and use them as
    the lower/upper corners (per dim: lb = min, ub = max) of a complete-match query."""
    rng = np.random.default_rng(seed)
    n = len(cols[0])
    d = len(cols)
    out = []
    for _ in range(n_queries):
        a, b = rng.choice(n, size=2, replace=False)
        va = np.array([c[a] for c in cols], dtype=np.float32)
        vb = np.array([c[b] for c in cols], dtype=np.float32)
        out.append((np.arange(d, dtype=np.uint32), np.minimum(va, vb), np.maximum(va, vb)))
    return out


# --------------------------------------------------------------------------------------
# Workload configurations.
# --------------------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    n_rows: int
    specs: list
    data_seed: int
    query_seed: int
    split_seed: int

    @property
    def n_dims(self) -> int:
        return len(self.specs)

    def columns(self, n_rows: int | None = None) -> list:
        n = self.n_rows if n_rows is None else n_rows
        return [column(self.data_seed, j, s, n) for j, s in enumerate(self.specs)]

    def fill(self, out2d: np.ndarray) -> np.ndarray:
        """Fill a (d, n) float32 array (e.g. pinned host memory) with the columns."""
        d, n = out2d.shape
        assert d == self.n_dims and out2d.dtype == np.float32
        for j, s in enumerate(self.specs):
            column(self.data_seed, j, s, n, out=out2d[j])
        return out2d

    def sampler(self, n_rows: int | None = None, sample_rows: int = 1 << 20) -> QuantileSampler:
        n = self.n_rows if n_rows is None else n_rows
        return QuantileSampler.build(self.data_seed, self.specs, n, sample_rows)


def workload(name: str, n_rows: int | None = None) -> Workload:
    """The named configuration; ``n_rows`` overrides the row count (same column mix)."""
    if name == "c1":
        specs, n = [uniform()] * 3, 1_000_000
    elif name == "c2":
        specs, n = [uniform()] * 8 + [gmm()] * 8 + [zipf()], 100_000_000
    elif name == "c3":
        specs, n = [uniform()] * 4 + [gmm()] * 4, 50_000_000
    elif name == "c4":
        specs = []
        for k in range(10):
            specs += [uniform(), corr(2 * k)]
        n = 100_000_000
    elif name == "c5":
        specs, n = [uniform()] * 4 + [gmm()] * 4 + [zipf()] * 4, 200_000_000
    elif name.startswith("syntuni"):
        # syntuni<d>: the paper's SYNT-UNI with d dims (default 5)
        d = int(name[7:] or 5)
        specs, n = [grid()] * d, 1_000_000
    else:
        raise KeyError(name)
    num = {"c1": 1, "c2": 2, "c3": 3, "c4": 4, "c5": 5}.get(name, 6)
    return Workload(name, n if n_rows is None else n_rows, list(specs), 1000 + num, 2000 + num,
                    3000 + num)


def workload_queries(w: Workload, n_queries: int, sampler: QuantileSampler | None = None,
                     seed: int | None = None) -> list:
    """The query mix of a configuration."""
    seed = w.query_seed if seed is None else seed
    if w.name == "c1":
        return box_queries(n_queries, 3, 0.01, seed)
    sampler = sampler or w.sampler()
    if w.name == "c2":
        return quantile_queries(sampler, n_queries, (2, 8), (1e-5, 0.2), seed)
    if w.name == "c3":
        return quantile_queries(sampler, n_queries, (1, 8), (1e-5, 0.2), seed)
    if w.name == "c4":
        return quantile_queries(sampler, n_queries, (3, 10), (1e-5, 0.2), seed)
    if w.name == "c5":
        return quantile_queries(sampler, n_queries, (1, 6), (1e-6, 0.1), seed)
    raise KeyError(w.name)
