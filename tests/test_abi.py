"""Host-side checks of the C ABI: the library loads, exports every entry point that
include/tdb.h declares, its struct layout matches the binding, and argument
validation rejects bad configurations (no device needed for any of this)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tdb.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tdb_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    from paper_2201_06958_amd import tdb
    lib = tdb.load_library()
    names = _declared_functions()
    assert "tdb_init" in names and "tdb_ingest_snapshot" in names
    for name in names:
        assert hasattr(lib, name), name


def test_struct_layout_matches_binding():
    from paper_2201_06958_amd import tdb
    lib = tdb.load_library()
    a, b = ctypes.c_int64(), ctypes.c_int64()
    lib.tdb_struct_sizes(ctypes.byref(a), ctypes.byref(b))
    assert a.value == ctypes.sizeof(tdb.TdbConfig)
    assert b.value == ctypes.sizeof(tdb.TdbStats)


@pytest.mark.parametrize("field,value,code", [
    ("order", 1, 1), ("order", 9, 1), ("order", 5, 6), ("dt", 0.0, 1), ("data_dtype", 7, 1),
    ("precision", 9, 1), ("slope_window", 1, 1), ("snapshot_mode", 5, 1), ("integrator", 2, 1),
    ("fd_order", 3, 1), ("fd_order", -1, 1),
])
def test_invalid_config_is_rejected_before_any_device_work(field, value, code):
    from paper_2201_06958_amd import tdb
    lib = tdb.load_library()
    cfg = tdb.TdbConfig()
    cfg.order = 3
    for n in range(3):
        cfg.dims[n] = 8
        cfg.rank_max[n] = 2
    cfg.dt = 0.1
    cfg.eps_th = 1e-3
    cfg.adaptive = 1
    setattr(cfg, field, value)
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(1)   # never dereferenced: validation fails first
    st = lib.tdb_init(ctypes.byref(cfg), dummy, None, ctypes.byref(h))
    assert st == code
    assert not h.value
    assert lib.tdb_last_error(None)


def test_null_handle_calls_fail_cleanly():
    from paper_2201_06958_amd import tdb
    lib = tdb.load_library()
    assert lib.tdb_ingest_snapshot(None, None, None) == tdb.EINVAL
    assert lib.tdb_ingest_with_derivative(None, None, None, None) == tdb.EINVAL
    assert lib.tdb_set_threshold(None, 1.0, 0.0) == tdb.EINVAL
    s = tdb.TdbStats()
    assert lib.tdb_get_stats(None, ctypes.byref(s)) == tdb.EINVAL
    assert lib.tdb_gate_load(None, None, None, 0, 0) == tdb.EINVAL
    lib.tdb_destroy(None)


def test_noalloc_reconstruct_validates_before_device_work():
    """tdb_reconstruct_noalloc refuses bad arguments and intermediates larger than half
    its fixed scratch before any HIP call (the pointers here are never dereferenced)."""
    from paper_2201_06958_amd import tdb
    lib = tdb.load_library()
    dummy = ctypes.c_void_p(1)
    uptr = (ctypes.c_void_p * 8)(1, 1, 1, None, None, None, None, None)
    out = ctypes.c_void_p(1)

    def call(order, dims, ranks, dtype=tdb.F64):
        d = (ctypes.c_int64 * 8)(*(list(dims) + [0] * (8 - len(dims))))
        r = (ctypes.c_int32 * 8)(*(list(ranks) + [0] * (8 - len(ranks))))
        return lib.tdb_reconstruct_noalloc(order, d, r, dummy, uptr, dtype, out, None)

    assert call(1, (4,), (2,)) == tdb.EINVAL
    assert call(3, (4, 4, 4), (5, 2, 2)) == tdb.EINVAL            # rank above the mode size
    assert call(3, (4, 4, 4), (2, 2, 2), dtype=7) == tdb.EINVAL
    # 2048 x 2048 x 4 doubles after the first product: above TDB_NOALLOC_SCRATCH / 2
    assert call(3, (2048, 2048, 4), (2048, 2048, 4)) == tdb.EINVAL
    assert b"scratch" in lib.tdb_last_error(None)


def _cfg3(tdb):
    cfg = tdb.TdbConfig()
    cfg.order = 3
    for n in range(3):
        cfg.dims[n] = 8
        cfg.rank_max[n] = 2
    cfg.dt = 0.1
    cfg.eps_th = 1e-3
    cfg.adaptive = 1
    return cfg


@pytest.mark.parametrize("case,code", [("n0", 1), ("order4", 6), ("plain", 6), ("mixed_dtype", 1), ("dt0", 1),
                                       ("mixed_precision", 1)])
def test_batch_create_validates_before_device_work(case, code):
    from paper_2201_06958_amd import tdb
    lib = tdb.load_library()
    cfgs = (tdb.TdbConfig * 2)(_cfg3(tdb), _cfg3(tdb))
    n = 2
    if case == "n0":
        n = 0
    elif case == "order4":
        cfgs[1].order = 4
        cfgs[1].dims[3] = 2
        cfgs[1].rank_max[3] = 1
    elif case == "plain":
        cfgs[0].path = 1
    elif case == "mixed_dtype":
        cfgs[1].data_dtype = 1
    elif case == "dt0":
        cfgs[0].dt = 0.0
    elif case == "mixed_precision":
        cfgs[0].precision = 1
        cfgs[1].precision = 2
    ptrs = (ctypes.c_void_p * 2)(1, 1)   # never dereferenced: validation fails first
    b = ctypes.c_void_p()
    st = lib.tdb_batch_create(n, cfgs, ptrs, None, ctypes.byref(b))
    assert st == code
    assert not b.value
    assert lib.tdb_batch_last_error(None)


def test_batch_null_handle_calls():
    from paper_2201_06958_amd import tdb
    lib = tdb.load_library()
    out = ctypes.c_void_p()
    assert lib.tdb_batch_ingest(None, None, None) == 1
    assert lib.tdb_batch_stream(None, 0, ctypes.byref(out)) == 1
    assert lib.tdb_batch_profile_enable(None, 1) == 1
    lib.tdb_batch_destroy(None)
