"""The C-ABI library loads and exports every function the public header
declares (no device calls), and host-side argument checks return the
documented status without touching the GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ddhf.h")
LIB = os.path.join(ROOT, "paper_2603_08386_amd", "libddhf.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(ddhf_[a-z0-9_]+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__.build()
    return C.CDLL(LIB)


def test_header_declares_the_four_hot_path_calls():
    names = declared_functions()
    for n in ["ddhf_build_pixel_index", "ddhf_ndft_power", "ddhf_comb_score", "ddhf_detect"]:
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings(lib):
    lib.ddhf_status_string.restype = C.c_char_p
    assert lib.ddhf_status_string(0) == b"ok"
    assert lib.ddhf_status_string(2) == b"workspace too small"
    assert lib.ddhf_status_string(99) == b"unknown status"


def test_host_side_validation_needs_no_gpu(lib):
    b = C.c_size_t(0)
    assert lib.ddhf_build_pixel_index_workspace_size(C.c_int64(-1), 4, 4, C.c_int64(10), 0, C.byref(b)) == 1
    assert lib.ddhf_build_pixel_index_workspace_size(C.c_int64(1000), 64, 64, C.c_int64(20000), 1, C.byref(b)) == 0
    assert b.value > 0
    assert lib.ddhf_detect_workspace_size(0, 4, C.byref(b)) == 1

    class Grid(C.Structure):
        _fields_ = [("f0", C.c_int64), ("df", C.c_int64), ("K", C.c_int32), ("mode", C.c_int32),
                    ("T_w_us", C.c_int64)]
    bad = Grid(1 << 40, 1, 4, 0, 0)  # f_max * 2^32 would overflow
    assert lib.ddhf_ndft_workspace_size(1, C.c_int64(1), C.byref(bad), None, C.byref(b)) == 1
    good = Grid(1000, 1000, 1024, 0, 20000)
    assert lib.ddhf_ndft_workspace_size(1, C.c_int64(1), C.byref(good), None, C.byref(b)) == 0
    # zero active pixels is a no-op that needs no pointers
    assert lib.ddhf_ndft_power(None, None, None, None, 0, C.c_int64(0), C.byref(good), None, None,
                               None, C.c_size_t(0), None) == 0


def test_detect_noalloc_refuses_oversized_frames_on_the_host(lib):
    """Frames above DDHF_DETECT_NOALLOC_MAX_PIXELS are refused before any device call."""
    class Grid(C.Structure):
        _fields_ = [("f0", C.c_int64), ("df", C.c_int64), ("K", C.c_int32), ("mode", C.c_int32),
                    ("T_w_us", C.c_int64)]
    g = Grid(10_000, 500, 3981, 0, 0)
    rc = lib.ddhf_detect_noalloc(None, None, None, None, None, 0, 2048, 1024, C.byref(g), None,
                                 None, None, None, 0, None, None)
    assert rc == 2
    assert lib.ddhf_detect_noalloc(None, None, None, None, None, 0, 0, 4, C.byref(g), None,
                                   None, None, None, 0, None, None) == 1


def test_fused_call_validates_on_the_host(lib):
    """ddhf_ndft_comb refuses grids beyond the fused kernel's reach before any
    device call, and zero active pixels need no pointers."""
    class Grid(C.Structure):
        _fields_ = [("f0", C.c_int64), ("df", C.c_int64), ("K", C.c_int32), ("mode", C.c_int32),
                    ("T_w_us", C.c_int64)]

    class Params(C.Structure):
        _fields_ = [("tau_sf", C.c_float), ("tau_comb", C.c_float), ("alpha", C.c_float),
                    ("eps_rel", C.c_float), ("M", C.c_int32), ("dk", C.c_int32),
                    ("h_min", C.c_int32), ("n_min", C.c_int32), ("a_min", C.c_int32),
                    ("reserved", C.c_int32)]
    prm = Params(0.89, 1.5, 19.05, 1e-6, 4, 3, 4, 6, 147, 0)
    ok = Grid(10_000, 1000, 3991, 0, 0)
    assert lib.ddhf_ndft_comb(None, None, None, None, 0, C.byref(ok), C.byref(prm), None, None,
                              None, None, None) == 0
    too_long = Grid(10_000, 1000, 4097, 0, 0)
    assert lib.ddhf_ndft_comb(None, None, None, None, 0, C.byref(too_long), C.byref(prm), None,
                              None, None, None, None) == 1
    wide = Params(0.89, 1.5, 19.05, 1e-6, 32, 16, 1, 6, 147, 0)  # band of 1585 ranks
    assert lib.ddhf_ndft_comb(None, None, None, None, 0, C.byref(ok), C.byref(wide), None, None,
                              None, None, None) == 1
    assert lib.ddhf_ndft_comb(None, None, None, None, 5, C.byref(ok), C.byref(prm), None, None,
                              None, None, None) == 1
