"""Python binding of libmdrq (argument marshalling only).

Every step of a query runs in the library's HIP kernels; this module only converts
Python and torch objects to the C ABI declared in ``include/mdrq.h``.  torch provides
device memory and streams.  There is no fallback: if the library or a GPU is missing,
calls raise.
"""
from __future__ import annotations

import ctypes
import os
import weakref
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libmdrq.so")

OK, EINVAL, ENOMEM, EOVERFLOW, EDEVICE, EBUSY, ENOTSUP = 0, -1, -2, -3, -4, -5, -6
MEM_HOST, MEM_DEVICE, BORROW = 0, 1, 2
OUT_IDS, OUT_BITMAP, OUT_COUNT, OUT_AUTO = 0, 1, 2, 3
Q_ORDER_GIVEN, Q_ORDER_ESTIMATED, Q_NO_EARLYOUT, Q_SIZE_ESTIMATED = 0, 1, 2, 4
MAX_DIMS, MAX_BATCH = 128, 1024
_MODES = {"ids": OUT_IDS, "bitmap": OUT_BITMAP, "count": OUT_COUNT, "auto": OUT_AUTO}
_MODE_NAMES = {v: k for k, v in _MODES.items()}

EXPORTS = ["mdrq_load_columns", "mdrq_query", "mdrq_query_batch", "mdrq_serve", "mdrq_free",
           "mdrq_last_error", "mdrq_dataset_info", "mdrq_column_range", "mdrq_set_profiling",
           "mdrq_get_profile", "mdrq_reset_profile", "mdrq_set_option", "mdrq_get_option",
           "mdrq_probe_bandwidth", "mdrq_get_batch_profile", "mdrq_version",
           "mdrq_estimator_create", "mdrq_estimator_free", "mdrq_estimator_histograms",
           "mdrq_estimator_features", "mdrq_estimator_param_count", "mdrq_estimator_get_params",
           "mdrq_estimator_set_params", "mdrq_label_selectivities", "mdrq_estimator_gradient",
           "mdrq_estimator_train", "mdrq_estimator_predict", "mdrq_attach_estimator",
           "mdrq_estimator_activations", "mdrq_query_read_bytes", "mdrq_estimator_gate",
           "mdrq_get_sizing_profile", "mdrq_get_batch_work", "mdrq_query_noalloc",
           "mdrq_serve_open", "mdrq_serve_submit", "mdrq_serve_poll", "mdrq_serve_close"]
EST_BINS = 16
EST_FEATS = EST_BINS + 3  # per dimension: H(lo), H(hi), histogram estimate, bins
OPT_UNROLL, OPT_GRID, OPT_BLOCKS_PER_CU = 1, 2, 3
OPT_BATCH_WAVES, OPT_BATCH_GROUP, OPT_AUTOTUNE, OPT_BATCH_ROWS = 4, 5, 6, 7
OPT_BATCH_VARIANT = 8
OPT_RANK_BUCKETS = 9
OPT_GRAPHS = 10
OPT_RESERVE_FACTOR = 11
OPT_CIRCULAR = 12


class MdrqError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mdrq error {code}: {msg}")
        self.code = code


class Pred(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_uint32), ("lo", ctypes.c_float), ("hi", ctypes.c_float)]


class Query(ctypes.Structure):
    _fields_ = [("preds", ctypes.POINTER(Pred)), ("n_preds", ctypes.c_uint32),
                ("flags", ctypes.c_uint32)]


class Result(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_uint32), ("mem", ctypes.c_uint32), ("buf", ctypes.c_void_p),
                ("buf_bytes", ctypes.c_uint64), ("count", ctypes.c_uint64),
                ("written", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("reserved", ctypes.c_uint32)]


class ServeConfig(ctypes.Structure):
    _fields_ = [("result_budget_bytes", ctypes.c_uint64), ("max_batch", ctypes.c_uint32),
                ("n_streams", ctypes.c_uint32), ("use_estimator", ctypes.c_uint32),
                ("max_queue", ctypes.c_uint32), ("segments", ctypes.c_uint32)]


class EstimatorConfig(ctypes.Structure):
    _fields_ = [("hidden", ctypes.c_uint32), ("sample_rows", ctypes.c_uint32),
                ("seed", ctypes.c_uint64)]


class TrainConfig(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_uint32), ("batch", ctypes.c_uint32), ("lr", ctypes.c_float),
                ("reserved", ctypes.c_uint32), ("seed", ctypes.c_uint64)]


class Request(ctypes.Structure):
    _fields_ = [("arrival_ns", ctypes.c_uint64), ("query", Query)]


class ServeStats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_uint64), ("scans", ctypes.c_uint64),
                ("wall_s", ctypes.c_double), ("qps", ctypes.c_double),
                ("p50_us", ctypes.c_double), ("p99_us", ctypes.c_double),
                ("mean_us", ctypes.c_double), ("max_us", ctypes.c_double),
                ("mean_batch", ctypes.c_double), ("hbm_gbps", ctypes.c_double),
                ("overflow_reruns", ctypes.c_uint64), ("sized_by_estimate", ctypes.c_uint64)]


_lib = None


def _hip_runtimes() -> set:
    try:
        with open("/proc/self/maps") as f:
            return {ln.split()[-1] for ln in f if "libamdhip64" in ln}
    except OSError:
        return set()


def load_library(path: str = LIB_PATH):
    """Load libmdrq.so (building it first only if no build exists).

    torch is imported first so that the library binds to the HIP runtime torch
    already loaded (same soname): one runtime per process, shared device memory and
    streams.  A second HIP runtime in the process is an error."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (loads the process's HIP runtime)

    if not os.path.exists(path):
        from . import build as _build

        _build.build_mdrq()
    lib = ctypes.CDLL(path)
    runtimes = _hip_runtimes()
    if len(runtimes) > 1:
        raise RuntimeError(f"two HIP runtimes loaded in one process: {sorted(runtimes)}")
    P, vp, u32, u64, i32 = ctypes.POINTER, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    lib.mdrq_load_columns.argtypes = [P(vp), u32, u64, u32, vp, P(vp)]
    lib.mdrq_query.argtypes = [vp, P(Query), P(Result), vp]
    lib.mdrq_query_batch.argtypes = [vp, P(Query), u32, P(Result), vp]
    lib.mdrq_serve.argtypes = [vp, P(ServeConfig), P(Request), u32, P(Result), P(u64), P(ServeStats)]
    lib.mdrq_serve_open.argtypes = [vp, P(ServeConfig), P(vp)]
    lib.mdrq_serve_submit.argtypes = [vp, P(Query), P(Result), vp, P(u64)]
    lib.mdrq_serve_poll.argtypes = [vp, P(u64), u32, P(u32), u64]
    lib.mdrq_serve_close.argtypes = [vp, P(ServeStats)]
    lib.mdrq_free.argtypes = [vp]
    lib.mdrq_free.restype = None
    lib.mdrq_last_error.restype = ctypes.c_char_p
    lib.mdrq_dataset_info.argtypes = [vp, P(u64), P(u32)]
    lib.mdrq_column_range.argtypes = [vp, u32, P(ctypes.c_float), P(ctypes.c_float)]
    lib.mdrq_set_profiling.argtypes = [vp, i32]
    lib.mdrq_get_profile.argtypes = [vp, P(u64), P(ctypes.c_double), P(ctypes.c_double)]
    lib.mdrq_reset_profile.argtypes = [vp]
    lib.mdrq_version.restype = ctypes.c_char_p
    lib.mdrq_set_option.argtypes = [vp, u32, ctypes.c_int64]
    lib.mdrq_get_option.argtypes = [vp, u32, P(ctypes.c_int64)]
    lib.mdrq_probe_bandwidth.argtypes = [vp, P(u32), u32, u32, vp, P(ctypes.c_double)]
    lib.mdrq_get_batch_profile.argtypes = [vp, P(u64), P(ctypes.c_double)]
    fp, u16p = P(ctypes.c_float), P(ctypes.c_uint16)
    lib.mdrq_estimator_create.argtypes = [vp, P(EstimatorConfig), P(vp)]
    lib.mdrq_estimator_free.argtypes = [vp]
    lib.mdrq_estimator_free.restype = None
    lib.mdrq_estimator_histograms.argtypes = [vp, fp]
    lib.mdrq_estimator_features.argtypes = [vp, P(Query), u32, u16p]
    lib.mdrq_estimator_param_count.argtypes = [vp, P(u64)]
    lib.mdrq_estimator_get_params.argtypes = [vp, fp]
    lib.mdrq_estimator_set_params.argtypes = [vp, fp]
    lib.mdrq_label_selectivities.argtypes = [vp, P(Query), u32, fp]
    lib.mdrq_estimator_gradient.argtypes = [vp, P(Query), u32, fp, fp, fp]
    lib.mdrq_estimator_train.argtypes = [vp, P(Query), u32, fp, P(TrainConfig), fp]
    lib.mdrq_estimator_predict.argtypes = [vp, P(Query), u32, fp]
    lib.mdrq_attach_estimator.argtypes = [vp, vp]
    lib.mdrq_estimator_activations.argtypes = [vp, P(Query), u32, u16p, u16p, fp]
    lib.mdrq_query_read_bytes.argtypes = [vp, P(Query), P(u64), vp]
    lib.mdrq_estimator_gate.argtypes = [vp, P(Query), u32, fp, P(u32)]
    lib.mdrq_get_sizing_profile.argtypes = [vp, P(u64), P(u64)]
    lib.mdrq_get_batch_work.argtypes = [vp, P(u64), P(u64), P(ctypes.c_double)]
    lib.mdrq_query_noalloc.argtypes = [vp, P(Query), P(Result), vp]
    for f in ("mdrq_load_columns", "mdrq_query", "mdrq_query_batch", "mdrq_serve",
              "mdrq_dataset_info", "mdrq_column_range", "mdrq_set_profiling",
              "mdrq_get_profile", "mdrq_reset_profile", "mdrq_set_option", "mdrq_get_option",
              "mdrq_probe_bandwidth", "mdrq_get_batch_profile", "mdrq_estimator_create", "mdrq_estimator_histograms",
              "mdrq_estimator_features", "mdrq_estimator_param_count", "mdrq_estimator_get_params",
              "mdrq_estimator_set_params", "mdrq_label_selectivities", "mdrq_estimator_gradient",
              "mdrq_estimator_train", "mdrq_estimator_predict", "mdrq_attach_estimator",
              "mdrq_estimator_activations", "mdrq_query_read_bytes", "mdrq_estimator_gate",
              "mdrq_get_sizing_profile", "mdrq_get_batch_work", "mdrq_query_noalloc"):
        getattr(lib, f).restype = i32
    _lib = lib
    return lib


def last_error() -> str:
    return load_library().mdrq_last_error().decode()


def _check(rc: int, allow=(OK,)):
    if rc not in allow:
        raise MdrqError(rc, last_error())
    return rc


def _stream_handle(stream) -> ctypes.c_void_p:
    if stream is None:
        import torch

        stream = torch.cuda.current_stream()
    if hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    return ctypes.c_void_p(int(stream) if stream else 0)


# numpy views of the records above, for building whole batches without a Python loop
# over predicates.
_PRED_DT = np.dtype([("dim", "<u4"), ("lo", "<f4"), ("hi", "<f4")])
_QUERY_DT = np.dtype([("preds", "<u8"), ("n_preds", "<u4"), ("flags", "<u4")])
_RESULT_DT = np.dtype([("mode", "<u4"), ("mem", "<u4"), ("buf", "<u8"), ("buf_bytes", "<u8"),
                       ("count", "<u8"), ("written", "<u8"), ("status", "<i4"),
                       ("reserved", "<u4")])
assert _PRED_DT.itemsize == ctypes.sizeof(Pred)
assert _QUERY_DT.itemsize == ctypes.sizeof(Query)
assert _RESULT_DT.itemsize == ctypes.sizeof(Result)


def make_query(query, flags: int = 0):
    """(dims, lo, hi) arrays or [(dim, lo, hi), ...] -> (Query, keepalive)."""
    if isinstance(query, tuple) and len(query) == 3 and hasattr(query[0], "__len__") \
            and not isinstance(query[0], tuple):
        dims, lo, hi = query
        preds = list(zip([int(d) for d in dims], [float(x) for x in lo], [float(x) for x in hi]))
    else:
        preds = [(int(d), float(a), float(b)) for d, a, b in query]
    arr = (Pred * max(1, len(preds)))(*[Pred(d, a, b) for d, a, b in preds])
    return Query(arr if preds else None, len(preds), flags), arr


@dataclass
class Answer:
    count: int
    written: int
    status: int
    mode: str


def _out_spec(out):
    """(memory kind, address, bytes) of an output buffer."""
    if out is None:
        return MEM_DEVICE, 0, 0
    if isinstance(out, np.ndarray):
        if not out.flags.c_contiguous:
            raise ValueError("output array must be contiguous")
        return MEM_HOST, out.ctypes.data, out.nbytes
    if not out.is_contiguous():  # torch tensor
        raise ValueError("output tensor must be contiguous")
    return (MEM_DEVICE if out.is_cuda else MEM_HOST), out.data_ptr(), out.numel() * out.element_size()


def _result_for(out, mode: str) -> Result:
    r = Result()
    r.mode = _MODES[mode]
    r.mem, buf, r.buf_bytes = _out_spec(out)
    r.buf = buf or None
    return r


class Dataset:
    """Columns resident in HBM; answers queries with the library's scan kernels."""

    def __init__(self, handle: int, n_rows: int, n_dims: int, keepalive=None):
        self._h = ctypes.c_void_p(handle)
        self.n_rows = n_rows
        self.n_dims = n_dims
        self._keep = keepalive
        self._estimators = weakref.WeakSet()  # released before the dataset
        self._servers = weakref.WeakSet()     # closed before the dataset

    @classmethod
    def from_host(cls, cols, stream=None) -> "Dataset":
        """Copy host float32 columns (a list of 1-D arrays or a (d, n) array) into HBM."""
        lib = load_library()
        arrs = [np.ascontiguousarray(c, dtype=np.float32) for c in cols]
        n = arrs[0].size if arrs else 0
        if any(a.size != n for a in arrs):
            raise ValueError("columns differ in length")
        ptrs = (ctypes.c_void_p * max(1, len(arrs)))(*[a.ctypes.data for a in arrs])
        h = ctypes.c_void_p()
        _check(lib.mdrq_load_columns(ptrs, len(arrs), n, MEM_HOST, _stream_handle(stream),
                                     ctypes.byref(h)))
        return cls(h.value, n, len(arrs))

    @classmethod
    def from_device(cls, tensors, borrow: bool = False, stream=None) -> "Dataset":
        """Use float32 CUDA tensors (one per column): copied, or borrowed in place."""
        lib = load_library()
        ts = list(tensors)
        n = ts[0].numel() if ts else 0
        for t in ts:
            if not (t.is_cuda and t.is_contiguous() and str(t.dtype) == "torch.float32"):
                raise ValueError("columns must be contiguous float32 CUDA tensors")
            if t.numel() != n:
                raise ValueError("columns differ in length")
        ptrs = (ctypes.c_void_p * max(1, len(ts)))(*[t.data_ptr() for t in ts])
        h = ctypes.c_void_p()
        flags = MEM_DEVICE | (BORROW if borrow else 0)
        _check(lib.mdrq_load_columns(ptrs, len(ts), n, flags, _stream_handle(stream),
                                     ctypes.byref(h)))
        return cls(h.value, n, len(ts), keepalive=ts if borrow else None)

    def close(self):
        if self._h and self._h.value:
            for srv in list(self._servers):
                srv.close()
            for est in list(self._estimators):
                est.close()
            load_library().mdrq_free(self._h)
            self._h = ctypes.c_void_p()
            self._keep = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        return self._h

    def column_range(self, dim: int):
        lo, hi = ctypes.c_float(), ctypes.c_float()
        _check(load_library().mdrq_column_range(self._h, dim, ctypes.byref(lo), ctypes.byref(hi)))
        return lo.value, hi.value

    def query(self, query, out=None, mode: str = "ids", flags: int = 0, stream=None) -> Answer:
        """Answer one query.  `out` is a CUDA tensor, a host numpy array or None (count
        only / nothing written).  Raises on errors other than overflow."""
        lib = load_library()
        q, keep = make_query(query, flags)
        r = _result_for(out, mode)
        rc = lib.mdrq_query(self._h, ctypes.byref(q), ctypes.byref(r), _stream_handle(stream))
        _check(rc, (OK, EOVERFLOW))
        return Answer(r.count, r.written, r.status, _MODE_NAMES[r.mode])

    def query_noalloc(self, query, out=None, mode: str = "ids", flags: int = 0, stream=None) -> Answer:
        """As query(), through mdrq_query_noalloc: the library's fixed per-GPU scratch
        instead of the dataset's workspace (device outputs, given order)."""
        lib = load_library()
        q, keep = make_query(query, flags)
        r = _result_for(out, mode)
        rc = lib.mdrq_query_noalloc(self._h, ctypes.byref(q), ctypes.byref(r), _stream_handle(stream))
        _check(rc, (OK, EOVERFLOW))
        return Answer(r.count, r.written, r.status, _MODE_NAMES[r.mode])

    def read_bytes(self, query, flags: int = 0, stream=None) -> int:
        """Column bytes the scan of `query` must read (128-byte lines that hold a row
        every earlier predicate accepted)."""
        q, keep = make_query(query, flags)
        b = ctypes.c_uint64()
        _check(load_library().mdrq_query_read_bytes(self._h, ctypes.byref(q), ctypes.byref(b),
                                                    _stream_handle(stream)))
        return b.value

    def query_batch(self, queries, outs=None, modes="ids", flags: int = 0, stream=None):
        lib = load_library()
        n = len(queries)
        qarr, keep = _query_array(queries, flags)
        rec = np.zeros(max(1, n), dtype=_RESULT_DT)
        if isinstance(modes, str):
            rec["mode"][:n] = _MODES[modes]
        else:
            rec["mode"][:n] = [_MODES[m] for m in modes]
        if outs is None:
            rec["mem"][:n] = MEM_DEVICE
        else:
            spec = [_out_spec(o) for o in outs]
            rec["mem"][:n] = [m for m, _, _ in spec]
            rec["buf"][:n] = [a for _, a, _ in spec]
            rec["buf_bytes"][:n] = [b for _, _, b in spec]
        rarr = (Result * max(1, n)).from_buffer(rec)
        rc = lib.mdrq_query_batch(self._h, qarr, n, rarr, _stream_handle(stream))
        _check(rc, (OK, EOVERFLOW))
        return [Answer(c, w, st, _MODE_NAMES[m]) for c, w, st, m in
                zip(rec["count"][:n].tolist(), rec["written"][:n].tolist(),
                    rec["status"][:n].tolist(), rec["mode"][:n].tolist())]

    def set_option(self, option: int, value: int):
        _check(load_library().mdrq_set_option(self._h, option, value))

    def get_option(self, option: int) -> int:
        v = ctypes.c_int64()
        _check(load_library().mdrq_get_option(self._h, option, ctypes.byref(v)))
        return v.value

    def probe_bandwidth(self, dims, iters: int = 5, stream=None) -> float:
        """Mean ms of one full read of the listed columns (no predicate, no output)."""
        arr = (ctypes.c_uint32 * len(dims))(*[int(d) for d in dims])
        ms = ctypes.c_double()
        _check(load_library().mdrq_probe_bandwidth(self._h, arr, len(dims), iters,
                                                   _stream_handle(stream), ctypes.byref(ms)))
        return ms.value

    def set_profiling(self, on: bool = True):
        _check(load_library().mdrq_set_profiling(self._h, 1 if on else 0))

    def profile(self):
        """(timed queries, scan-kernel ms, whole-query device ms)."""
        n, ms1, ms2 = ctypes.c_uint64(), ctypes.c_double(), ctypes.c_double()
        _check(load_library().mdrq_get_profile(self._h, ctypes.byref(n), ctypes.byref(ms1),
                                               ctypes.byref(ms2)))
        return n.value, ms1.value, ms2.value

    def batch_profile(self):
        """(shared scans, their summed device ms) since the last reset."""
        n, ms = ctypes.c_uint64(), ctypes.c_double()
        _check(load_library().mdrq_get_batch_profile(self._h, ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value

    def batch_work(self):
        """(rank lookups, column bytes, scan-kernel ms) of the shared scans since the last
        reset."""
        a, b, ms = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_double()
        _check(load_library().mdrq_get_batch_work(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(ms)))
        return a.value, b.value, ms.value

    def sizing_profile(self):
        """(queries whose scratch was sized by estimate, of those answered again) since the
        last reset."""
        a, b = ctypes.c_uint64(), ctypes.c_uint64()
        _check(load_library().mdrq_get_sizing_profile(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def reset_profile(self):
        _check(load_library().mdrq_reset_profile(self._h))

    def serve(self, arrivals_ns, queries, outs, modes="ids", max_batch: int = 256,
              n_streams: int = 2, budget_bytes: int = 1 << 30, use_estimator: int = 0,
              segments: int = 0):
        """Replay requests (arrival time in ns, query) through the serving loop
        (segments > 0: the circular scan with that many parts per pass).
        Returns (answers, latencies in ns, stats dict)."""
        lib = load_library()
        n = len(queries)
        modes = [modes] * n if isinstance(modes, str) else list(modes)
        qarr, keep = _query_array(queries, 0)
        reqs = (Request * max(1, n))()
        for i in range(n):
            reqs[i].arrival_ns = int(arrivals_ns[i])
            reqs[i].query = qarr[i]
        rarr = (Result * max(1, n))(*[_result_for(o, m) for o, m in zip(outs, modes)])
        lat = (ctypes.c_uint64 * max(1, n))()
        st = ServeStats()
        cfg = ServeConfig(int(budget_bytes), max_batch, n_streams, int(use_estimator), 0, int(segments))
        rc = lib.mdrq_serve(self._h, ctypes.byref(cfg), reqs, n, rarr, lat, ctypes.byref(st))
        _check(rc, (OK, EOVERFLOW))
        answers = [Answer(r.count, r.written, r.status, _MODE_NAMES[r.mode]) for r in rarr[:n]]
        stats = {name: getattr(st, name) for name, _ in ServeStats._fields_}
        return answers, np.array(lat[:n], dtype=np.uint64), stats

    def serve_open(self, max_batch: int = 256, n_streams: int = 2, budget_bytes: int = 1 << 30,
                   use_estimator: int = 0, max_queue: int = 0, segments: int = 0) -> "Server":
        """A live server on this dataset (submit / poll / close)."""
        return Server(self, max_batch, n_streams, budget_bytes, use_estimator, max_queue, segments)

    def label_selectivities(self, queries) -> np.ndarray:
        """Exact selectivities (n, n_dims + 1): each predicate alone, then the query;
        -1 where a query does not restrict a dimension."""
        qarr, keep = _query_array(queries, 0)
        out = np.empty((len(queries), self.n_dims + 1), dtype=np.float32)
        _check(load_library().mdrq_label_selectivities(self._h, qarr, len(queries), _fptr(out)))
        return out

    def attach_estimator(self, est):
        """Order MDRQ_Q_ORDER_ESTIMATED queries by `est` (None detaches)."""
        _check(load_library().mdrq_attach_estimator(self._h, est.handle if est else None))


def _query_parts(query):
    """(dims, lo, hi) of a query given as three arrays or as [(dim, lo, hi), ...]."""
    if isinstance(query, tuple) and len(query) == 3 and hasattr(query[0], "__len__") \
            and not isinstance(query[0], tuple):
        return query
    q = list(query)
    return [p[0] for p in q], [p[1] for p in q], [p[2] for p in q]


def _query_array(queries, flags: int):
    """ctypes array of mdrq_query over numpy records: all predicates in one array, each
    query pointing at its run (NULL when it has none).  Returns (array, keepalive)."""
    n = len(queries)
    parts = [_query_parts(q) for q in queries]
    counts = np.fromiter((len(p[0]) for p in parts), dtype=np.int64, count=n)
    total = int(counts.sum())
    preds = np.zeros(max(1, total), dtype=_PRED_DT)
    if total:
        preds["dim"][:total] = np.concatenate([p[0] for p in parts]).astype(np.int64).astype(np.uint32)
        preds["lo"][:total] = np.concatenate([p[1] for p in parts]).astype(np.float32)
        preds["hi"][:total] = np.concatenate([p[2] for p in parts]).astype(np.float32)
    rec = np.zeros(max(1, n), dtype=_QUERY_DT)
    if n:
        offs = np.cumsum(counts) - counts
        rec["preds"][:n] = np.where(counts > 0, preds.ctypes.data + offs * _PRED_DT.itemsize, 0)
        rec["n_preds"][:n] = counts
        rec["flags"][:n] = flags
    return (Query * max(1, n)).from_buffer(rec), (preds, rec)


def _fptr(a: np.ndarray):
    assert a.dtype == np.float32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


class Server:
    """Live serving loop (mdrq_serve_open): requests are submitted one at a time and
    answered by continuous batching; poll() reports the completed ones."""

    def __init__(self, ds: Dataset, max_batch: int, n_streams: int, budget_bytes: int,
                 use_estimator: int, max_queue: int, segments: int = 0):
        cfg = ServeConfig(int(budget_bytes), max_batch, n_streams, int(use_estimator),
                          int(max_queue), int(segments))
        h = ctypes.c_void_p()
        _check(load_library().mdrq_serve_open(ds.handle, ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self.ds = ds
        ds._servers.add(self)
        self._pending = {}   # ticket -> (result record, output buffer): alive until polled

    def submit(self, query, out=None, mode: str = "ids", stream=None) -> int:
        """Queue one request; returns its ticket.  The request's scan runs after the work
        queued so far on `stream` (default: torch's current stream), e.g. a fill of
        `out`.  Raises MdrqError (code EBUSY) when the queue is full."""
        q, keep = make_query(query, 0)
        r = _result_for(out, mode)
        t = ctypes.c_uint64()
        _check(load_library().mdrq_serve_submit(self._h, ctypes.byref(q), ctypes.byref(r),
                                                _stream_handle(stream), ctypes.byref(t)))
        self._pending[t.value] = (r, out)
        return t.value

    def poll(self, max_tickets: int = 1024, wait_s: float = 0.0):
        """Completed requests since the last poll: list of (ticket, Answer)."""
        buf = (ctypes.c_uint64 * max(1, max_tickets))()
        n = ctypes.c_uint32()
        rc = load_library().mdrq_serve_poll(self._h, buf, max_tickets, ctypes.byref(n),
                                            int(wait_s * 1e9))
        done = []
        for t in buf[:n.value]:
            r, _ = self._pending.pop(t)
            done.append((t, Answer(r.count, r.written, r.status, _MODE_NAMES[r.mode])))
        _check(rc)
        return done

    def close(self):
        """Answer everything submitted, stop, and return the summary statistics."""
        if not (self._h and self._h.value):
            return None
        st = ServeStats()
        rc = load_library().mdrq_serve_close(self._h, ctypes.byref(st))
        self._h = ctypes.c_void_p()
        _check(rc, (OK, EOVERFLOW))
        return {name: getattr(st, name) for name, _ in ServeStats._fields_}

    def results(self):
        """Answers of requests completed but not yet polled (after close)."""
        out = [(t, Answer(r.count, r.written, r.status, _MODE_NAMES[r.mode]))
               for t, (r, _) in sorted(self._pending.items())]
        self._pending.clear()
        return out

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Estimator:
    """Learned selectivity estimator of a dataset (histograms + MLP on the GPU)."""

    def __init__(self, ds: Dataset, hidden: int = 64, sample_rows: int = 0, seed: int = 0):
        cfg = EstimatorConfig(hidden, sample_rows, seed)
        h = ctypes.c_void_p()
        _check(load_library().mdrq_estimator_create(ds.handle, ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self.ds = ds
        ds._estimators.add(self)
        self.n_dims = ds.n_dims
        self.hidden = hidden or 64
        n = ctypes.c_uint64()
        _check(load_library().mdrq_estimator_param_count(self._h, ctypes.byref(n)))
        self.n_params = n.value

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h and self._h.value:
            load_library().mdrq_estimator_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def histograms(self) -> np.ndarray:
        out = np.empty((self.n_dims, EST_BINS + 1), dtype=np.float32)
        _check(load_library().mdrq_estimator_histograms(self._h, _fptr(out)))
        return out

    def features(self, queries) -> np.ndarray:
        """bfloat16 bit patterns (n, n_dims * EST_FEATS) as uint16."""
        qarr, keep = _query_array(queries, 0)
        out = np.empty((len(queries), self.n_dims * EST_FEATS), dtype=np.uint16)
        _check(load_library().mdrq_estimator_features(
            self._h, qarr, len(queries), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16))))
        return out

    def _shapes(self):
        F, H, O = self.n_dims * EST_FEATS, self.hidden, self.n_dims + 1
        return [("W1", (F, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, O)),
                ("b3", (O,))]

    def unpack(self, flat: np.ndarray) -> dict:
        out, at = {}, 0
        for name, shape in self._shapes():
            n = int(np.prod(shape))
            out[name] = flat[at:at + n].reshape(shape)
            at += n
        return out

    def pack(self, params: dict) -> np.ndarray:
        return np.concatenate([np.asarray(params[name], dtype=np.float32).reshape(-1)
                               for name, _ in self._shapes()])

    def get_params(self) -> dict:
        flat = np.empty(self.n_params, dtype=np.float32)
        _check(load_library().mdrq_estimator_get_params(self._h, _fptr(flat)))
        return self.unpack(flat)

    def set_params(self, params: dict):
        flat = np.ascontiguousarray(self.pack(params))
        _check(load_library().mdrq_estimator_set_params(self._h, _fptr(flat)))

    def gradient(self, queries, sel):
        """(loss, gradient dict) of the current parameters on one batch."""
        qarr, keep = _query_array(queries, 0)
        sel = np.ascontiguousarray(sel, dtype=np.float32)
        loss = np.zeros(1, dtype=np.float32)
        grad = np.empty(self.n_params, dtype=np.float32)
        _check(load_library().mdrq_estimator_gradient(self._h, qarr, len(queries), _fptr(sel),
                                                      _fptr(loss), _fptr(grad)))
        return float(loss[0]), self.unpack(grad)

    def train(self, queries, sel, epochs: int = 10, batch: int = 256, lr: float = 1e-3,
              seed: int = 0) -> np.ndarray:
        """Adam on the labelled queries; returns the mean loss of each epoch."""
        qarr, keep = _query_array(queries, 0)
        sel = np.ascontiguousarray(sel, dtype=np.float32)
        cfg = TrainConfig(epochs, batch, lr, 0, seed)
        losses = np.zeros(epochs, dtype=np.float32)
        _check(load_library().mdrq_estimator_train(self._h, qarr, len(queries), _fptr(sel),
                                                    ctypes.byref(cfg), _fptr(losses)))
        return losses

    def gate(self, queries, sel) -> np.ndarray:
        """Remove the learned correction of every output that does not lower the held-out
        error on these labelled queries; returns the kept mask (n_dims + 1,)."""
        qarr, keep = _query_array(queries, 0)
        sel = np.ascontiguousarray(sel, dtype=np.float32)
        kept = np.zeros(self.n_dims + 1, dtype=np.uint32)
        _check(load_library().mdrq_estimator_gate(
            self._h, qarr, len(queries), _fptr(sel), kept.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))))
        return kept.astype(bool)

    def activations(self, queries):
        """(h1, h2, y): the hidden layers' bfloat16 bit patterns (n, hidden) as uint16 and
        the output layer (n, n_dims + 1) as float32, before clamping."""
        qarr, keep = _query_array(queries, 0)
        n = len(queries)
        h1 = np.empty((n, self.hidden), dtype=np.uint16)
        h2 = np.empty((n, self.hidden), dtype=np.uint16)
        y = np.empty((n, self.n_dims + 1), dtype=np.float32)
        u16 = ctypes.POINTER(ctypes.c_uint16)
        _check(load_library().mdrq_estimator_activations(
            self._h, qarr, n, h1.ctypes.data_as(u16), h2.ctypes.data_as(u16), _fptr(y)))
        return h1, h2, y

    def predict(self, queries) -> np.ndarray:
        qarr, keep = _query_array(queries, 0)
        out = np.empty((len(queries), self.n_dims + 1), dtype=np.float32)
        _check(load_library().mdrq_estimator_predict(self._h, qarr, len(queries), _fptr(out)))
        return out


def version() -> str:
    return load_library().mdrq_version().decode()
