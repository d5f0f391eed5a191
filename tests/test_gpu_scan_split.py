"""White-box check of the batched scans' work split (tests/native/scan_split_check.hip).

Both batched scans split a column list over as many workgroups as the device holds at once: whole tiles
first, then the tiles left over cut by rows and joined in row order.  The check program calls the
library's launchers directly: the FP64 matrix-core scan (modes 0-2, all six variants) against FP64 dot
products on the CPU for sampled columns (to 1e-12 of sum |x b|), the BF16 scans (two and three pieces)
against the FP64 scan within the stated BF16 bound, for list lengths that cut every tile, give each
workgroup whole tiles and a leftover, or fill it exactly, with the length on the host and on the device;
each run is repeated (equal bit for bit) and entries outside the list must stay untouched.
"""
import importlib.util
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def _program() -> str:
    exe = os.path.join(HERE, "native", "scan_split_check")
    if not os.path.exists(exe):   # __graft_entry__.build() builds it; here only if it is missing
        spec = importlib.util.spec_from_file_location("native_build", os.path.join(HERE, "native", "build.py"))
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        mod.build(force=False)
    return exe


def test_batched_scan_work_split():
    r = subprocess.run([_program()], capture_output=True, text=True, timeout=240)
    print(r.stdout)
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), r.stdout + r.stderr
