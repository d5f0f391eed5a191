"""Compile the white-box GPU check programs under tests/native against the built libbl.so."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
PKG = os.path.join(ROOT, "paper_1701_05936_amd")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
PROGRAMS = ["scan_split_check"]


def build(force: bool = True) -> list[str]:
    out = []
    for name in PROGRAMS:
        exe = os.path.join(HERE, name)
        out.append(exe)
        if not force and os.path.exists(exe):
            continue
        cmd = [HIPCC, "--offload-arch=gfx950", "-O2", "-std=c++17",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-I", os.path.join(PKG, "csrc"), "-I", os.path.join(ROOT, "include"),
               os.path.join(HERE, name + ".hip"), "-L", PKG, "-lbl",
               "-Wl,-rpath,$ORIGIN/../../paper_1701_05936_amd", "-o", exe + ".tmp"]
        subprocess.run(cmd, check=True)
        os.replace(exe + ".tmp", exe)
    return out


if __name__ == "__main__":
    print(build())
