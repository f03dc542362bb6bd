"""CPU checks of the C ABI boundary: the library loads and exports every declared symbol."""
import ctypes

import paper_1901_01652_amd as rt


def test_header_declares_the_four_stage_calls():
    syms = rt.header_symbols()
    for name in ("rtr_sketch", "rtr_compress", "rtr_decompose", "rtr_backproject"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    syms = rt.header_symbols()
    assert len(syms) >= 12
    for name in syms:
        assert hasattr(rt.lib, name), name


def test_null_handle_is_rejected_without_touching_a_device():
    assert rt.lib.rtr_sketch(None, None, 0, 0, None, None, 0, 0, 0, 0, None, None) == 1
    assert rt.lib.rtr_destroy(None) == 0
    assert rt.lib.rtr_last_error(None) == b"invalid handle"
    assert rt.lib.rtr_profile_enable(None, 1) == 1


def test_status_strings():
    assert rt.status_string(0) == "RTR_OK"
    assert rt.status_string(2) == "RTR_ERR_UNSUPPORTED"
    assert rt.status_string(5) == "RTR_ERR_NUMERICAL"
