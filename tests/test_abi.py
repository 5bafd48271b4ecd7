"""C-ABI surface checks that need no GPU: exports, argument validation, error strings."""
import ctypes as C
import os
import re

import pytest

from tests.libutil import ROOT, ensure_built

INCLUDE = os.path.join(ROOT, "include")


def declared_functions():
    """Every bm_* function declared in include/*.h (comments stripped)."""
    names = set()
    for f in sorted(os.listdir(INCLUDE)):
        if f.endswith(".h"):
            txt = re.sub(r"/\*.*?\*/", "", open(os.path.join(INCLUDE, f)).read(), flags=re.S)
            names |= set(re.findall(r"\b(bm_[a-z_]+)\s*\(", txt))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["bm_plan", "bm_plan_info", "bm_match", "bm_match_batch", "bm_plan_destroy",
              "bm_server_create", "bm_submit", "bm_poll", "bm_cancel", "bm_server_destroy",
              "bm_status_str", "bm_last_error", "bm_norms", "bm_batch_workspace",
              "bm_peak_mfma", "bm_peak_copy"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    bm = ensure_built()
    h = C.CDLL(bm.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(h, n)]
    assert not missing, missing


def test_status_strings():
    bm = ensure_built()
    assert bm.bm_status_str(0) == "BM_OK"
    assert bm.bm_status_str(bm.BM_EINVAL) == "BM_EINVAL"
    assert bm.bm_status_str(bm.BM_EBUSY) == "BM_EBUSY"
    assert bm.bm_status_str(12345) == "BM_UNKNOWN"


@pytest.mark.parametrize("field,value,needle", [
    ("height", 0, "height"), ("channels", 9, "channels"), ("patch", 0, "patch"),
    ("patch", 17, "patch"), ("stride", 0, "stride"), ("window", 0, "window must"), ("window", -3, "window must"),
    ("k", 0, "k must"), ("k", 65, "k must"), ("precision", 7, "precision"), ("flags", 8, "flag"),
])
def test_invalid_descriptors_rejected_on_host(field, value, needle):
    bm = ensure_built()
    d = bm.make_desc(64, 64, 1, 8, 3, 21, 16)
    setattr(d, field, value)
    with pytest.raises(bm.BMError) as ei:
        bm.bm_plan(d)
    assert ei.value.status == bm.BM_EINVAL
    assert needle in str(ei.value)


def test_patch_larger_than_image_rejected():
    bm = ensure_built()
    with pytest.raises(bm.BMError) as ei:
        bm.bm_plan(bm.make_desc(5, 40, 1, 8, 1, 3, 4))
    assert ei.value.status == bm.BM_EINVAL


def test_unsupported_contraction_is_enotsup():
    bm = ensure_built()
    with pytest.raises(bm.BMError) as ei:
        bm.bm_plan(bm.make_desc(64, 64, 8, 8, 1, 3, 4))  # 8 * 16 steps > 64
    assert ei.value.status == bm.BM_ENOTSUP


def test_null_arguments():
    bm = ensure_built()
    lib = bm.lib()
    assert lib.bm_plan(None, None) == bm.BM_EINVAL
    assert lib.bm_plan_info(None, None, None) == bm.BM_EINVAL
    assert lib.bm_match(None, None, None, None, None, None) == bm.BM_EINVAL
    assert lib.bm_plan_destroy(None) == bm.BM_EINVAL
    assert "NULL" in bm.bm_last_error()


def test_batch_arguments_checked_on_host():
    import ctypes as C
    bm = ensure_built()
    lib = bm.lib()
    # an empty batch is a no-op and needs no workspace
    assert lib.bm_match_batch(0, None, None, None, None, None, None) == bm.BM_OK
    out = C.c_int64(-1)
    assert lib.bm_batch_workspace(0, None, C.byref(out)) == bm.BM_OK and out.value == 0
    assert lib.bm_match_batch(-1, None, None, None, None, None, None) == bm.BM_EINVAL
    assert lib.bm_match_batch(2, None, None, None, None, None, None) == bm.BM_EINVAL
    nulls = (C.c_void_p * 2)(None, None)
    assert lib.bm_match_batch(2, nulls, nulls, nulls, nulls, None, None) == bm.BM_EINVAL
    assert "NULL" in bm.bm_last_error()
    assert lib.bm_batch_workspace(2, nulls, C.byref(out)) == bm.BM_EINVAL
    assert lib.bm_batch_workspace(1, nulls, None) == bm.BM_EINVAL


def test_server_arguments_checked_on_host():
    import ctypes as C
    bm = ensure_built()
    lib = bm.lib()
    out = C.c_void_p()
    assert lib.bm_server_create(None, C.byref(out)) == bm.BM_EINVAL
    bad = bm.bm_server_cfg(0, 1, 1)  # budget below the minimum
    assert lib.bm_server_create(C.byref(bad), C.byref(out)) == bm.BM_EINVAL
    bad = bm.bm_server_cfg(1 << 30, 0, 1)
    assert lib.bm_server_create(C.byref(bad), C.byref(out)) == bm.BM_EINVAL
    t = C.c_uint64()
    assert lib.bm_submit(None, None, None, C.byref(t)) == bm.BM_EINVAL
    assert lib.bm_poll(None, 1, None, None, None) == bm.BM_EINVAL
    assert lib.bm_cancel(None, 1) == bm.BM_EINVAL
    assert lib.bm_server_destroy(None) == bm.BM_EINVAL


def test_ncc_with_centring_rejected_on_host():
    bm = ensure_built()
    with pytest.raises(bm.BMError) as ei:
        bm.bm_plan(bm.make_desc(64, 64, 1, 8, 3, 39, 16, "fp32", bm.BM_FLAG_NCC | bm.BM_FLAG_CENTER))
    assert ei.value.status == bm.BM_EINVAL
    with pytest.raises(bm.BMError) as ei:
        bm.bm_plan(bm.make_desc(64, 64, 1, 8, 3, 39, 16, "fp32", 4))
    assert ei.value.status == bm.BM_EINVAL


def test_nlm_arguments_checked_on_host():
    bm = ensure_built()
    lib = bm.lib()
    assert lib.bm_nlm(None, None, 1.0, None, None, None, None) == bm.BM_EINVAL


def test_group_arguments_checked_on_host():
    import ctypes as C
    bm = ensure_built()
    lib = bm.lib()
    assert lib.bm_gather(None, None, None, None, None) == bm.BM_EINVAL
    assert lib.bm_aggregate(None, None, None, None, None, None) == bm.BM_EINVAL
    out = C.c_int64()
    assert lib.bm_aggregate_workspace(None, C.byref(out)) == bm.BM_EINVAL


@pytest.mark.parametrize("pd,wd,channels,status,needle", [
    (1, 0, 4, "BM_EINVAL", "window_depth"), (0, 3, 4, "BM_EINVAL", "patch_depth"),
    (5, 3, 4, "BM_EINVAL", "patch_depth"), (2, -1, 4, "BM_EINVAL", "window_depth"),
    (5, 2, 8, "BM_ENOTSUP", "patch_depth <= 4"), (2, 3, 70000, "BM_EINVAL", "volume planes"),
])
def test_3d_descriptors_checked_on_host(pd, wd, channels, status, needle):
    """3D fields: both 0 (2D) or window_depth >= 1 with 1 <= patch_depth <= channels; the
    kernels take patch_depth <= 4."""
    bm = ensure_built()
    d = bm.make_desc(8, 8, channels, 3, 1, 3, 4, "fp32", 0, pd, wd)
    with pytest.raises(bm.BMError) as ei:
        bm.bm_plan(d)
    assert ei.value.status == getattr(bm, status)
    assert needle in str(ei.value)


@pytest.mark.parametrize("flags", [1, 2])
def test_3d_takes_no_flags(flags):
    bm = ensure_built()
    with pytest.raises(bm.BMError) as ei:
        bm.bm_plan(bm.make_desc(64, 64, 6, 6, 2, 15, 16, "fp32", flags, 2, 3))
    assert ei.value.status == bm.BM_ENOTSUP


def test_3d_descriptor_layout():
    """The two depth fields follow flags in the C struct (9 + 2 int32 fields)."""
    bm = ensure_built()
    import ctypes as C
    assert C.sizeof(bm.bm_desc) == 44
    assert bm.bm_desc.patch_depth.offset == 36 and bm.bm_desc.window_depth.offset == 40
