"""The C ABI: libbl.so loads without a GPU and exports every function include/bl.h declares."""
import ctypes
import os
import re

import paper_1701_05936_amd as bl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "bl.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bl_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_named_entry_points():
    names = declared_functions()
    for required in ("bl_standardize", "bl_lambda_max", "bl_screen", "bl_cd_solve", "bl_kkt_check", "bl_fit_path"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(bl.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(bl.EXPORTS) == declared_functions()


def test_binding_declares_signatures_without_touching_the_device():
    L = bl.load_library()
    assert L.bl_last_error(None) == b"null context"
    # a null context is rejected before any device work
    assert L.bl_fit_path(None, None, None, None, None) == bl.BL_ERR_INVALID


def test_struct_layouts_match_header_sizes():
    # bl_matrix: ptr, int32 (+pad), 3 x int64, ptr
    assert ctypes.sizeof(bl._Matrix) == 48
    assert ctypes.sizeof(bl._PathOpts) == 48
