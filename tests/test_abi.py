"""CPU-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments without touching a device."""
import ctypes as C
import os
import re

import pytest

import paper_1708_02574_amd as tpa

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_header_symbol():
    lib = tpa.load_library()
    names = tpa.header_symbols()
    assert len(names) >= 18
    for name in names:
        assert hasattr(lib, name), name
        assert name in tpa._SIGS, f"binding lacks {name}"


def test_status_strings():
    lib = tpa.load_library()
    for code in tpa.STATUS:
        s = lib.tpa_status_string(code).decode()
        assert s and s != "unknown status"
    assert lib.tpa_status_string(42).decode() == "unknown status"


def test_header_status_codes_match_binding():
    txt = open(os.path.join(ROOT, "include", "tpa.h")).read()
    for name, val in re.findall(r"(TPA_[A-Z_]+)\s*=\s*(-?\d+)", txt):
        assert tpa.STATUS[int(val)] == name


@pytest.mark.parametrize("call", [
    lambda L: L.tpa_graph_info(None, None, None, None),
    lambda L: L.tpa_preprocess(None, 0.15, 10, None),
    lambda L: L.tpa_preprocess_ex(None, 0.15, 10, 1e-9, None),
    lambda L: L.tpa_query(None, None, 1, 0.15, 5, 10, None, None),
    lambda L: L.tpa_query_packed(None, None, 1, 0.15, 5, 10, None, None),
    lambda L: L.tpa_stranger(None, None, None),
    lambda L: L.tpa_set_tuning(None, 0, 0),
    lambda L: L.tpa_get_tuning(None, None, None),
    lambda L: L.tpa_set_push_limit(None, -1),
    lambda L: L.tpa_get_push_limit(None, None),
    lambda L: L.tpa_set_tile_push_limit(None, -1),
    lambda L: L.tpa_get_tile_push_limit(None, None),
    lambda L: L.tpa_set_third_push_limit(None, -1),
    lambda L: L.tpa_get_third_push_limit(None, None),
    lambda L: L.tpa_set_gather_layout(None, 1),
    lambda L: L.tpa_cpi(None, 0, None, 0.15, 0, -1, 1e-9, None, None),
    lambda L: L.tpa_topk(None, 1, 10, 0, None, None, None),
    lambda L: L.tpa_topk(None, 1, 10, 3, None, None, None),
    lambda L: L.tpa_row_l1(None, None, -1, 10, 1.0, None, None),
    lambda L: L.tpa_row_l1(None, None, 2, 10, 1.0, None, None),
    lambda L: L.tpa_get_gather_layout(None, None),
    lambda L: L.tpa_set_sliced_sweep(None, 1),
    lambda L: L.tpa_get_sliced_sweep(None, None, None),
    lambda L: L.tpa_graph_device_bytes(None, None),
    lambda L: L.tpa_graph_blocks(None, None),
    lambda L: L.tpa_graph_export(None, 0, None, None, None, None),
    lambda L: L.tpa_graph_padded(None, None, None),
    lambda L: L.tpa_graph_set_logits(None, None, None),
    lambda L: L.tpa_reserve(None, 1),
    lambda L: L.tpa_query_workspace_size(None, 1, None),
    lambda L: L.tpa_set_keep_iterates(None, 1),
    lambda L: L.tpa_cpi_batch(None, None, None, 1, 0.15, 0, -1, 1e-9, None, None),
    lambda L: L.tpa_get_device_error(None, None),
    lambda L: L.tpa_graph_pack(None, 0, None, None),
    lambda L: L.tpa_query_dense(None, None, 1, 0.15, 5, 10, None, None),
    lambda L: L.tpa_backward(None, None, None, 1, 0, 0.15, 5, 10, None, None, None, 0, None),
    lambda L: L.tpa_query_graph_create(None, None, None, 1, 0, 0.15, 5, 10, None, None, C.byref(C.c_void_p())),
    lambda L: L.tpa_query_graph_launch(None, None),
    lambda L: L.tpa_autotune(None, None, 1, 0.15, 5, 10, None, None, None, None, None),
])
def test_null_handles_are_invalid_arg(call):
    lib = tpa.load_library()
    assert call(lib) == -1
    assert lib.tpa_last_error_message().decode()


def test_constructor_argument_checks():
    lib = tpa.load_library()
    h = C.c_void_p()
    assert lib.tpa_graph_rmat(0, 0, 10, 1, 0.57, 0.19, 0.19, None, C.byref(h)) == -1
    assert lib.tpa_graph_rmat(32, 0, 10, 1, 0.57, 0.19, 0.19, None, C.byref(h)) == -1
    assert lib.tpa_graph_rmat(10, 0, -1, 1, 0.57, 0.19, 0.19, None, C.byref(h)) == -1
    assert lib.tpa_graph_rmat(10, 0, 10, 1, 0.7, 0.3, 0.3, None, C.byref(h)) == -1
    assert lib.tpa_graph_rmat(10, 2000, 10, 1, 0.57, 0.19, 0.19, None, C.byref(h)) == -1
    assert lib.tpa_graph_from_edges(0, 0, None, None, 0, None, C.byref(h)) == -1
    assert lib.tpa_graph_from_edges(1 << 31, 0, None, None, 0, None, C.byref(h)) == -6
    assert lib.tpa_graph_from_edges(10, 5, None, None, 0, None, C.byref(h)) == -1
    assert lib.tpa_graph_rmat(10, 0, 10, 1, 0.57, 0.19, 0.19, None, None) == -1
    assert not h.value


def test_profile_argument_checks():
    lib = tpa.load_library()
    assert lib.tpa_profile_enable(1, 0, 1) == -1
    assert lib.tpa_profile_enable(1, 1 << 21, 1) == -1
    assert lib.tpa_profile_enable(1, 16, 0) == -1
    assert lib.tpa_profile_read(128, None, None) == -1
    assert lib.tpa_profile_read(-1, None, None) == -1
    assert tpa.profile_code(1, 0, False, False) == 0
    assert tpa.profile_code(64, 0, True, True) == 16 * 6 + 3
    assert tpa.profile_code(1, 1, False, False) == 4
