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


def test_struct_layouts_match_the_header(tmp_path):
    """Offsets and sizes of every ctypes mirror equal what a C compiler gives for include/bl.h."""
    import subprocess
    mirrors = {"bl_matrix": bl._Matrix, "bl_screen_state": bl._ScreenState, "bl_path_opts": bl._PathOpts,
               "bl_path_result": bl._PathResult, "bl_kernel_profile": bl._KernelProfile, "bl_batch": bl._Batch,
               "bl_batch_result": bl._BatchResult, "bl_mlp_train_opts": bl._MlpTrainOpts,
               "bl_mlp_train_result": bl._MlpTrainResult, "bl_limits": bl._Limits, "bl_cv": bl._Cv,
               "bl_cv_result": bl._CvResult, "bl_host_stream": bl._HostStream}
    renames = {"lambda_": "lambda"}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "bl.h"', "int main(void) {"]
    for cname, cls in mirrors.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            c_field = renames.get(fname, fname)
            lines.append(f'printf("{cname}.{fname} %zu\\n", offsetof({cname}, {c_field}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = dict(line.rsplit(" ", 1) for line in out if line)
    for cname, cls in mirrors.items():
        assert int(got[f"{cname} size"]) == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert int(got[f"{cname}.{fname}"]) == getattr(cls, fname).offset, f"{cname}.{fname}"
