"""The C-ABI library loads and exports every symbol include/rf.h declares;
host-side argument checks reject bad descriptors without touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rf.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rf_[a-z_]+)\s*\(", text)))


def lib():
    from paper_1802_03084_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("librf.so not built")
    return _lib.load()


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ("rf_dedisperse", "rf_resample", "rf_grid", "rf_image", "rf_search",
                 "rf_search_segment", "rf_plan_create"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    L = lib()
    for name in declared_symbols():
        assert hasattr(L, name), name


def test_binding_covers_every_declared_symbol():
    from paper_1802_03084_amd import _lib
    assert set(declared_symbols()) == set(_lib.SIGNATURES)


def test_status_strings():
    L = lib()
    assert L.rf_status_string(0) == b"ok"
    assert L.rf_status_string(-4).startswith(b"workspace")


def _desc(**over):
    from paper_1802_03084_amd import _lib
    keep = {}
    freq = np.linspace(1.0, 2.0, 8)
    uvw = np.zeros((3, 3))
    dm = np.array([0.0, 10.0])
    width = np.array([1, 2], np.int32)
    keep.update(freq=freq, uvw=uvw, dm=dm, width=width)
    d = _lib.PlanDesc()
    d.nint, d.nbl, d.nchan, d.npol, d.vis_dtype = 16, 3, 8, 2, 0
    d.tint_s = 0.005
    d.freq_ghz = freq.ctypes.data_as(_lib.c_dp)
    d.uvw_m = uvw.ctypes.data_as(_lib.c_dp)
    d.dm = dm.ctypes.data_as(_lib.c_dp)
    d.ndm = 2
    d.width = width.ctypes.data_as(_lib.c_ip)
    d.nwidth = 2
    d.npix = 64
    d.du = d.dv = 10.0
    d.kdm = 4.15e-3
    d.threshold = 6.0
    d.t_begin, d.t_end = 0, 16
    for k, v in over.items():
        setattr(d, k, v)
    return d, keep


@pytest.mark.parametrize("field,value,status", [
    ("npix", 100, -3), ("npix", 32, -3), ("npix", 4096, -3), ("npol", 3, -2), ("nint", 0, -2),
    ("tint_s", 0.0, -3), ("du", -1.0, -3), ("vis_dtype", 7, -1), ("t_end", 17, -3),
    ("t_begin", 5, None), ("ndm", 0, -2),
])
def test_table_bytes_validates(field, value, status):
    from paper_1802_03084_amd import _lib
    L = lib()
    d, keep = _desc(**{field: value})
    n = _lib.c_size(0)
    st = L.rf_plan_table_bytes(ctypes.byref(d), ctypes.byref(n))
    if status is None:
        assert st == 0 and n.value > 0
    else:
        assert st == status


def test_negative_dm_and_bad_width_rejected():
    from paper_1802_03084_amd import _lib
    L = lib()
    d, keep = _desc()
    keep["dm"][1] = -1.0
    n = _lib.c_size(0)
    assert L.rf_plan_table_bytes(ctypes.byref(d), ctypes.byref(n)) == -3
    d, keep = _desc()
    keep["width"][1] = 17
    assert L.rf_plan_table_bytes(ctypes.byref(d), ctypes.byref(n)) == -3


def test_null_arguments_rejected_without_gpu():
    from paper_1802_03084_amd import _lib
    L = lib()
    out = ctypes.c_void_p()
    assert L.rf_plan_create(None, None, 0, None, ctypes.byref(out)) == -1
    d, keep = _desc()
    assert L.rf_plan_create(ctypes.byref(d), None, 0, None, ctypes.byref(out)) == -1
    assert L.rf_plan_create(ctypes.byref(d), ctypes.c_void_p(1), 16, None, ctypes.byref(out)) == -4
    assert out.value is None
    assert L.rf_dedisperse(None, 0, None, None, None) == -1
    assert L.rf_search_segment(None, None, None, 0, None, None, None, 0, None) == -1
    assert L.rf_plan_destroy(None) == 0


def test_server_arguments_rejected_without_gpu():
    """Serving entry points validate on the host before any HIP call."""
    L = lib()
    out = ctypes.c_void_p(123)
    n = ctypes.c_size_t(0)
    t = ctypes.c_int64(0)
    k = ctypes.c_int32(0)
    assert L.rf_server_request_bytes(None, 0, ctypes.byref(n)) == -1
    assert L.rf_server_create(None, 1 << 20, 2, ctypes.byref(out)) == -1
    assert out.value is None  # *out cleared on error
    assert L.rf_server_create(ctypes.c_void_p(4096), 0, 2, ctypes.byref(out)) == -1
    assert L.rf_server_create(ctypes.c_void_p(4096), 1 << 20, 0, ctypes.byref(out)) == -3
    assert L.rf_server_create(ctypes.c_void_p(4096), 1 << 20, 17, ctypes.byref(out)) == -3
    assert L.rf_server_create(ctypes.c_void_p(4097), 1 << 20, 2, ctypes.byref(out)) == -1
    assert L.rf_server_create(ctypes.c_void_p(4096), 1 << 20, 2, None) == -1
    assert L.rf_server_submit(None, None, None, 0, 0, ctypes.byref(t)) == -1
    assert L.rf_server_wait(None, 1, None, 0, ctypes.byref(k), None) == -1
    assert L.rf_server_destroy(None) == -1


def test_segment_begin_end_arguments_rejected_without_gpu():
    L = lib()
    job = ctypes.c_void_p(123)
    assert L.rf_search_segment_begin(None, None, None, 0, None, None, None, 0, None,
                                     ctypes.byref(job)) == -1
    assert job.value is None  # *job cleared on error
    assert L.rf_search_segment_begin(None, None, None, 0, None, None, None, 0, None, None) == -1
    assert L.rf_search_segment_end(None) == -1


def test_tuning_and_batch_arguments_rejected_without_gpu():
    L = lib()
    out = ctypes.c_void_p(123)
    n = ctypes.c_size_t(0)
    assert L.rf_plan_set_tuning(None, 2, 240) == -1
    assert L.rf_batch_workspace_bytes(None, 1, ctypes.byref(n)) == -1
    assert L.rf_batch_create(None, 1, None, None, None, None, None, None, 0, 0,
                             ctypes.byref(out)) == -1
    assert out.value is None
    assert L.rf_batch_graph_nodes(None, ctypes.byref(n)) == -1
    assert L.rf_batch_run(None, None) == -1
    assert L.rf_batch_destroy(None) == -1


def test_mock_and_noise_arguments_rejected_without_gpu():
    from paper_1802_03084_amd import _lib
    L = lib()
    mk = (_lib.Mock * 1)()
    assert L.rf_inject(None, mk, 1, 0, ctypes.c_void_p(4096), None) == -1
    assert L.rf_noise(None, 1, 0, 0, ctypes.c_void_p(4096), None) == -1


def test_products_arguments_rejected_without_gpu():
    L = lib()
    n = ctypes.c_size_t(0)
    assert L.rf_products_workspace_bytes(None, 16, ctypes.byref(n)) == -1
    assert L.rf_candidate_products(None, None, None, 0, 8, 16, None, None, None, 0, None) == -1


def test_periodic_arguments_rejected_without_gpu():
    L = lib()
    n = ctypes.c_size_t(0)
    assert L.rf_periodic_workspace_bytes(None, ctypes.byref(n)) == -1
    assert L.rf_search_periodic(None, None, None, 0, None, None, None, 0, None) == -1


def test_select_tier_keeps_rows_above_the_second_threshold():
    """rf_select_tier (host only): rows with snr strictly above the tier's
    threshold, in order; the count is the true count when cap is short; in
    place works; bad arguments are rejected."""
    L = lib()
    import paper_1802_03084_amd as rf
    rows = np.zeros(6, dtype=rf.CAND_DTYPE)
    rows["snr"] = [5.0, 7.5, 7.0, 9.0, 6.9, 12.0]
    rows["dm_idx"] = np.arange(6)
    got = rf.second_tier(rows, 7.0)
    assert list(got["dm_idx"]) == [1, 3, 5]
    out = np.zeros(2, dtype=rf.CAND_DTYPE)
    k = ctypes.c_int32()
    vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    assert L.rf_select_tier(vp(rows), 6, ctypes.c_float(7.0), vp(out), 2, ctypes.byref(k)) == 0
    assert k.value == 3 and list(out["dm_idx"]) == [1, 3]
    inplace = rows.copy()
    assert L.rf_select_tier(vp(inplace), 6, ctypes.c_float(6.0), vp(inplace), 6, ctypes.byref(k)) == 0
    assert k.value == 5 and list(inplace["dm_idx"][:5]) == [1, 2, 3, 4, 5]
    assert L.rf_select_tier(None, 0, ctypes.c_float(7.0), None, 0, ctypes.byref(k)) == 0 and k.value == 0
    assert L.rf_select_tier(vp(rows), -1, ctypes.c_float(7.0), vp(out), 2, ctypes.byref(k)) == -3
    assert L.rf_select_tier(vp(rows), 6, ctypes.c_float(float("nan")), vp(out), 2, ctypes.byref(k)) == -3
    assert L.rf_select_tier(vp(rows), 6, ctypes.c_float(7.0), None, 2, ctypes.byref(k)) == -1
