"""Host-side checks of the C ABI library (no GPU needed): it loads, exports every
function the header declares, and rejects invalid arguments before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1801_03644_amd import mdrq

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "mdrq.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mdrq_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = mdrq.load_library()
    names = header_functions()
    assert "mdrq_query" in names and "mdrq_load_columns" in names
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(mdrq.EXPORTS) == names


def test_version():
    assert re.fullmatch(r"\d+\.\d+\.\d+", mdrq.version())


def test_load_rejects_bad_arguments_without_a_device():
    lib = mdrq.load_library()
    h = ctypes.c_void_p()
    col = np.zeros(8, dtype=np.float32)
    ptrs = (ctypes.c_void_p * 1)(col.ctypes.data)
    assert lib.mdrq_load_columns(ptrs, 0, 8, 0, None, ctypes.byref(h)) == mdrq.EINVAL
    assert "n_dims" in mdrq.last_error()
    assert lib.mdrq_load_columns(ptrs, 129, 8, 0, None, ctypes.byref(h)) == mdrq.EINVAL
    assert lib.mdrq_load_columns(ptrs, 1, 1 << 32, 0, None, ctypes.byref(h)) == mdrq.EINVAL
    assert lib.mdrq_load_columns(None, 1, 8, 0, None, ctypes.byref(h)) == mdrq.EINVAL
    assert lib.mdrq_load_columns(ptrs, 1, 8, 0, None, None) == mdrq.EINVAL
    assert lib.mdrq_load_columns(ptrs, 1, 8, mdrq.BORROW, None, ctypes.byref(h)) == mdrq.EINVAL
    assert lib.mdrq_load_columns(ptrs, 1, 8, 8, None, ctypes.byref(h)) == mdrq.EINVAL
    nulls = (ctypes.c_void_p * 1)(None)
    assert lib.mdrq_load_columns(nulls, 1, 8, 0, None, ctypes.byref(h)) == mdrq.EINVAL
    odd = (ctypes.c_void_p * 1)(col.ctypes.data + 4)
    assert lib.mdrq_load_columns(odd, 1, 8, mdrq.MEM_DEVICE | mdrq.BORROW, None,
                                 ctypes.byref(h)) == mdrq.EINVAL
    assert "aligned" in mdrq.last_error()


def test_calls_on_null_dataset_are_rejected():
    lib = mdrq.load_library()
    q, keep = mdrq.make_query([(0, 0.0, 1.0)])
    r = mdrq.Result()
    assert lib.mdrq_query(None, ctypes.byref(q), ctypes.byref(r), None) == mdrq.EINVAL
    assert lib.mdrq_query_batch(None, ctypes.byref(q), 1, ctypes.byref(r), None) == mdrq.EINVAL
    cfg = mdrq.ServeConfig(1 << 20, 16, 1, 0, 0)
    req = mdrq.Request(0, q)
    assert lib.mdrq_serve(None, ctypes.byref(cfg), ctypes.byref(req), 1, ctypes.byref(r), None,
                          None) == mdrq.EINVAL
    assert lib.mdrq_dataset_info(None, None, None) == mdrq.EINVAL
    assert lib.mdrq_column_range(None, 0, None, None) == mdrq.EINVAL
    assert lib.mdrq_set_option(None, mdrq.OPT_UNROLL, 4) == mdrq.EINVAL
    assert lib.mdrq_get_option(None, mdrq.OPT_UNROLL, None) == mdrq.EINVAL
    lib.mdrq_free(None)


def test_estimator_calls_reject_null_arguments():
    lib = mdrq.load_library()
    q, keep = mdrq.make_query([(0, 0.0, 1.0)])
    f = (ctypes.c_float * 8)()
    n = ctypes.c_uint64()
    h = ctypes.c_void_p()
    cfg = mdrq.EstimatorConfig(64, 0, 0)
    tc = mdrq.TrainConfig(1, 16, 1e-3, 0, 0)
    assert lib.mdrq_estimator_create(None, ctypes.byref(cfg), ctypes.byref(h)) == mdrq.EINVAL
    assert lib.mdrq_estimator_histograms(None, f) == mdrq.EINVAL
    assert lib.mdrq_estimator_features(None, ctypes.byref(q), 1, None) == mdrq.EINVAL
    assert lib.mdrq_estimator_param_count(None, ctypes.byref(n)) == mdrq.EINVAL
    assert lib.mdrq_estimator_get_params(None, f) == mdrq.EINVAL
    assert lib.mdrq_estimator_set_params(None, f) == mdrq.EINVAL
    assert lib.mdrq_label_selectivities(None, ctypes.byref(q), 1, f) == mdrq.EINVAL
    assert lib.mdrq_estimator_gradient(None, ctypes.byref(q), 1, f, f, f) == mdrq.EINVAL
    assert lib.mdrq_estimator_train(None, ctypes.byref(q), 1, f, ctypes.byref(tc), f) == mdrq.EINVAL
    assert lib.mdrq_estimator_predict(None, ctypes.byref(q), 1, f) == mdrq.EINVAL
    assert lib.mdrq_attach_estimator(None, None) == mdrq.EINVAL
    lib.mdrq_estimator_free(None)


def test_error_message_is_thread_local():
    import threading

    lib = mdrq.load_library()
    h = ctypes.c_void_p()
    col = np.zeros(8, dtype=np.float32)
    ptrs = (ctypes.c_void_p * 1)(col.ctypes.data)
    assert lib.mdrq_load_columns(ptrs, 0, 8, 0, None, ctypes.byref(h)) == mdrq.EINVAL
    seen = []
    t = threading.Thread(target=lambda: seen.append(mdrq.last_error()))
    t.start()
    t.join()
    assert seen == [""]
    assert mdrq.last_error() != ""


def test_live_server_calls_reject_null_arguments():
    lib = mdrq.load_library()
    q, keep = mdrq.make_query([(0, 0.0, 1.0)])
    r = mdrq.Result()
    cfg = mdrq.ServeConfig(1 << 20, 16, 1, 0, 0)
    h = ctypes.c_void_p()
    t = ctypes.c_uint64()
    n = ctypes.c_uint32()
    tickets = (ctypes.c_uint64 * 4)()
    assert lib.mdrq_serve_open(None, ctypes.byref(cfg), ctypes.byref(h)) == mdrq.EINVAL
    assert lib.mdrq_serve_submit(None, ctypes.byref(q), ctypes.byref(r), None, ctypes.byref(t)) == mdrq.EINVAL
    assert lib.mdrq_serve_poll(None, tickets, 4, ctypes.byref(n), 0) == mdrq.EINVAL
    assert lib.mdrq_serve_close(None, None) == mdrq.EINVAL
