"""CPU-side checks of the C ABI: the built library exports every function
that include/tga.h declares, and the binding knows all of them.  No device
call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tga.h")
LIB = os.path.join(ROOT, "paper_2506_17357_amd", "libtga.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tga_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_four_core_calls():
    names = declared_functions()
    for core in ("tga_load_instance", "tga_set_solution", "tga_eval_neighborhood", "tga_apply_move"):
        assert core in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtga.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_2506_17357_amd import tga
    assert sorted(tga.EXPORTS) == declared_functions()


def test_workspace_size_queries_need_no_device():
    if not os.path.exists(LIB):
        pytest.skip("libtga.so not built")
    lib = ctypes.CDLL(LIB)
    lib.tga_solution_workspace_bytes.restype = ctypes.c_size_t
    lib.tga_instance_workspace_bytes.restype = ctypes.c_size_t
    assert lib.tga_solution_workspace_bytes(1000, 50) > 0
    assert lib.tga_solution_workspace_bytes(14000, 655) == 0  # n + R > 14654
    assert lib.tga_solution_workspace_bytes(10, 0) == 0
    assert lib.tga_instance_workspace_bytes(0) == 0


def test_static_scratch_size_matches_header():
    text = open(HEADER).read()
    m = re.search(r"#define TGA_STATIC_SCRATCH_BYTES \((\d+)u << (\d+)\)", text)
    assert m
    from paper_2506_17357_amd import tga
    assert tga.STATIC_SCRATCH_BYTES == int(m.group(1)) << int(m.group(2))


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtga.so not built")
def test_tuning_table_validation_needs_no_device():
    """tga_set_tuning is host-only: malformed entries are refused, a good
    table and an empty one are accepted."""
    lib = ctypes.CDLL(LIB)

    class E(ctypes.Structure):
        _fields_ = [("has_tw", ctypes.c_int32), ("n_max", ctypes.c_int32), ("plain_rows", ctypes.c_int32),
                    ("item_rows", ctypes.c_int32)]

    lib.tga_set_tuning.restype = ctypes.c_int
    lib.tga_set_tuning.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    good = (E * 3)(E(1, 1000, 4, 16), E(0, 300, 1, 0), E(0, 14654, 2, 32))
    assert lib.tga_set_tuning(good, 3) == 0
    for bad in (E(2, 100, 1, 1), E(0, 0, 1, 1), E(0, 100, -1, 0), E(1, 100, 0, -3)):
        arr = (E * 1)(bad)
        assert lib.tga_set_tuning(arr, 1) != 0
    assert lib.tga_set_tuning(None, -1) != 0
    assert lib.tga_set_tuning(None, 0) == 0
