"""The C-ABI library loads and exports every symbol include/slim.h declares;
argument checks that need no GPU reject bad calls."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "slim.h")


def declared_symbols():
    text = open(HEADER).read()
    return re.findall(r"^SLIM_API\s+[\w\s\*]*?\b(slim_\w+)\s*\(", text, flags=re.M)


def test_header_declares_the_abi():
    syms = declared_symbols()
    for s in ("slim_load_csr", "slim_triangle_reduce", "slim_edge_sample", "slim_graph_free",
              "slim_workspace_size", "slim_last_error"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    from paper_1912_08950_amd import slim
    lib = ctypes.CDLL(slim.LIB_PATH)
    for s in declared_symbols():
        assert hasattr(lib, s), s
    assert set(declared_symbols()) == set(slim.SYMBOLS)


def test_errors_without_gpu():
    from paper_1912_08950_amd import slim
    L = slim._lib
    h = ctypes.c_void_p()
    assert L.slim_load_csr(None, None, 5, 0, 0, None, ctypes.byref(h)) == slim.EINVAL
    assert b"NULL" in L.slim_last_error()
    assert L.slim_load_csr(1, 1, 5, 3, 0, None, ctypes.byref(h)) == slim.EINVAL  # odd nnz
    assert L.slim_load_csr(1, 1, 2**32, 2, 0, None, ctypes.byref(h)) == slim.EINVAL
    assert L.slim_triangle_reduce(None, 0.5, 1, None, 0, None, None, None, None) == slim.EINVAL
    assert L.slim_edge_sample(None, 0.5, 1, None, 0, None, None, None, None) == slim.EINVAL
    b = ctypes.c_uint64()
    assert L.slim_workspace_size(None, 1, ctypes.byref(b)) == slim.EINVAL
    assert L.slim_strerror(slim.ENOMEM) == b"SLIM_ENOMEM"
    L.slim_graph_free(None)


def test_degree_kl_errors_without_gpu():
    from paper_1912_08950_amd import slim
    L = slim._lib
    b = ctypes.c_uint64()
    assert L.slim_degree_kl_workspace(1000, ctypes.byref(b)) == slim.OK
    assert b.value >= 2 * 8 * 1001 and b.value % 256 == 0
    assert L.slim_degree_kl_workspace(2**32, ctypes.byref(b)) == slim.EINVAL
    assert L.slim_degree_kl_workspace(5, None) == slim.EINVAL
    assert L.slim_degree_kl(1, 1, 4, None, 0, None, None) == slim.EINVAL  # d_out NULL
    assert L.slim_degree_kl(None, 1, 4, None, 0, 8, None) == slim.EINVAL
    assert L.slim_degree_kl(1, 1, 4, 256, 16, 8, None) == slim.ENOMEM


def test_tuning_knobs():
    from paper_1912_08950_amd import slim
    for k, v in (("eo_rounds", 3), ("tri_tile", 256), ("eo_list_try", 0), ("eo_list_try", 100000)):
        old = slim.tune_get(k)
        slim.tune_set(k, v)
        assert slim.tune_get(k) == v
        slim.tune_set(k, old)
    with pytest.raises(slim.SlimError):
        slim.tune_set("eo_rounds", 0)
    with pytest.raises(slim.SlimError):
        slim.tune_set("eo_list_try", 100001)
    assert slim.tune_get("eo_list_try") == 250
    old = slim.tune_get("tri_chunk")
    slim.tune_set("tri_chunk", 64)
    assert slim.tune_get("tri_chunk") == 64
    slim.tune_set("tri_chunk", old)
    with pytest.raises(slim.SlimError):
        slim.tune_set("tri_chunk", 5000)
    with pytest.raises(slim.SlimError):
        slim.tune_set("no_such_knob", 1)


def test_batch_and_serve_errors_without_gpu():
    from paper_1912_08950_amd import slim
    L = slim._lib
    h = ctypes.c_void_p()
    assert L.slim_batch_create(None, None, 0, ctypes.byref(h)) == slim.EINVAL
    b = ctypes.c_uint64()
    assert L.slim_batch_workspace_size(None, ctypes.byref(b)) == slim.EINVAL
    assert L.slim_batch_run(None, None, 0, None, None) == slim.EINVAL
    L.slim_batch_free(None)
    assert L.slim_serve_create(None, ctypes.byref(h)) == slim.EINVAL
    cfg = slim.ServeCfg(0, 0, 0, 0, 0)
    assert L.slim_serve_create(ctypes.byref(cfg), ctypes.byref(h)) == slim.EINVAL
    cfg = slim.ServeCfg(1 << 30, 0, 17, 0, 0)
    assert L.slim_serve_create(ctypes.byref(cfg), ctypes.byref(h)) == slim.EINVAL
    t = ctypes.c_uint64()
    assert L.slim_serve_submit(None, None, ctypes.byref(t)) == slim.EINVAL
    assert L.slim_result_release(None, 1) == slim.EINVAL
    L.slim_serve_destroy(None)
