"""The C ABI library loads without a GPU and exports every declared symbol."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(contour_[A-Za-z0-9_]+)\s*\(",
                            text, flags=re.M)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = declared_functions()
    for need in ("contour_cc", "contour_cc_ex", "contour_batch_plan_create",
                 "contour_batch_plan_launch", "contour_batch_plan_destroy", "contour_cc_batched",
                 "contour_status_string", "contour_last_hip_error", "contour_default_opts",
                 "contour_cc_add_edges", "contour_group_edges"):
        assert need in names


def test_library_exports_every_declared_symbol():
    import paper_2311_02811_amd as contour
    lib = ctypes.CDLL(contour.lib_path())
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_only_calls_work_without_gpu():
    import paper_2311_02811_amd as contour
    lib = contour.load()
    assert lib.contour_status_string(0) == b"ok"
    assert lib.contour_status_string(2).startswith(b"edge id")
    o = contour.make_opts()
    assert o.order == 0 and o.write_mode == 0 and o.driver == 0   # 0: the default order
    assert contour.make_opts(order="full").order == -1
    assert b"gfx950" in lib.contour_version()


def test_argument_errors_are_synchronous_without_touching_the_device():
    import paper_2311_02811_amd as contour
    lib = contour.load()
    # negative sizes and NULL arrays are rejected before any HIP call
    assert lib.contour_cc(None, None, -1, 4, None, None) == contour.EINVAL
    assert lib.contour_cc(None, None, 5, 4, None, None) == contour.EINVAL
    assert lib.contour_cc(None, None, 0, -3, None, None) == contour.EINVAL
    o = contour.make_opts()
    o.order = 5000
    assert lib.contour_cc_ex(None, None, 0, 0, None, ctypes.byref(o), None, None) == contour.EINVAL
    o = contour.make_opts(update="sync")
    assert lib.contour_cc_ex(None, None, 0, 0, None, ctypes.byref(o), None, None) == contour.ENOTSUP


def test_package_fails_loudly_without_library(tmp_path, monkeypatch):
    import paper_2311_02811_amd._lib as L
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        L.load()


def test_add_edges_argument_errors_without_touching_the_device():
    import paper_2311_02811_amd as contour
    lib = contour.load()
    assert lib.contour_cc_add_edges(None, None, -1, 4, None, None, None, None) == contour.EINVAL
    assert lib.contour_cc_add_edges(None, None, 3, 4, None, None, None, None) == contour.EINVAL
    assert lib.contour_cc_add_edges(None, None, 0, 4, None, None, None, None) == contour.EINVAL
    # the augmented list has 3m edges, which must fit int32 slots
    assert lib.contour_cc_add_edges(ctypes.c_void_p(16), ctypes.c_void_p(16), 1 << 30, 4,
                                    ctypes.c_void_p(16), None, None, None) == contour.EINVAL
    o = contour.make_opts()
    o.order = 0x7fff
    assert lib.contour_cc_add_edges(None, None, 0, 0, None, ctypes.byref(o), None, None) == contour.EINVAL


def test_group_edges_argument_errors_without_touching_the_device():
    import paper_2311_02811_amd as contour
    lib = contour.load()
    p = ctypes.c_void_p(16)
    assert lib.contour_group_edges(None, None, -1, 4, None, None, None) == contour.EINVAL
    assert lib.contour_group_edges(p, p, 3, 0, p, p, None) == contour.EINVAL
    assert lib.contour_group_edges(p, p, 3, -2, p, p, None) == contour.EINVAL
    assert lib.contour_group_edges(None, p, 3, 4, p, p, None) == contour.EINVAL
    assert lib.contour_group_edges(p, p, 3, 4, p, None, None) == contour.EINVAL
    # slots of the grouped copy are int32
    assert lib.contour_group_edges(p, p, 0x7fffffff, 4, p, p, None) == contour.EINVAL
    # nothing to do
    assert lib.contour_group_edges(None, None, 0, 4, None, None, None) == contour.OK


def test_reserve_and_noalloc_argument_errors_without_touching_the_device():
    import paper_2311_02811_amd as contour
    lib = contour.load()
    assert lib.contour_reserve(-1, 4, None, None) == contour.EINVAL
    assert lib.contour_reserve(4, -1, None, None) == contour.EINVAL
    o = contour.make_opts()
    o.order = 5000
    assert lib.contour_reserve(4, 4, ctypes.byref(o), None) == contour.EINVAL
    assert lib.contour_cc_noalloc(None, None, -1, 4, None, None, None, None) == contour.EINVAL
    assert lib.contour_cc_noalloc(None, None, 3, 4, None, None, None, None) == contour.EINVAL
    assert lib.contour_cc_noalloc(None, None, 0, 4, None, None, None, None) == contour.EINVAL
    assert lib.contour_cc_noalloc(None, None, 0, 0, None, ctypes.byref(o), None, None) == contour.EINVAL
    assert lib.contour_status_string(contour.ETOOBIG).startswith(b"input needs more")


def test_gather_ceiling_and_count_reads_argument_errors_without_touching_the_device():
    import paper_2311_02811_amd as contour
    lib = contour.load()
    p = ctypes.c_void_p(16)
    assert lib.contour_gather_ceiling(p, p, 5, p, 4, 0, None, None) == contour.EINVAL   # no sink
    assert lib.contour_gather_ceiling(p, p, 5, p, 4, 3, p, None) == contour.EINVAL      # bad mode
    assert lib.contour_gather_ceiling(None, None, 5, p, 4, 1, p, None) == contour.EINVAL
    assert lib.contour_gather_ceiling(None, None, 0, None, 0, 0, p, None) == contour.OK
    assert lib.contour_merge_min(p, p, -1, None, None) == contour.EINVAL
    assert lib.contour_merge_min(None, p, 5, None, None) == contour.EINVAL
    assert lib.contour_merge_min(p, None, 5, None, None) == contour.EINVAL
    assert lib.contour_merge_min(None, None, 0, None, None) == contour.OK
    assert lib.contour_cc_count_reads(None, None, 0, 0, None, None, None, None, None) == contour.EINVAL
    assert lib.contour_cc_count_reads(None, None, -1, 4, None, None, None, p, None) == contour.EINVAL
