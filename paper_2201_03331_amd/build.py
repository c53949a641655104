"""Builds libfiuncho.so (gfx950) in-tree with hipcc.

    python -m paper_2201_03331_amd.build        # or build() from Python
"""
from __future__ import annotations

import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libfiuncho.so")
SOURCES = ["api.hip", "pack.hip", "scan.hip", "mfma.hip", "select.hip", "io.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=off",
    "-Wall", "-Wno-unused-result",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


# Kernels that address their dynamic LDS from address 0 (lds_window in
# mfma.hip): they must declare no static LDS, which the compiler's resource
# remarks for mfma.hip confirm at every build.
LDS_WINDOW_KERNELS = re.compile(r"_ZN7fiuncho(11mfma_kernelILi[23]ELi[123]E|15mfma_sub_kernelI)")
REMARKS = "-Rpass-analysis=kernel-resource-usage"


def check_lds_window(text: str) -> None:
    """Raises unless every kernel of LDS_WINDOW_KERNELS reports 0 bytes of static LDS."""
    sizes, name = {}, None
    for line in text.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
        m = re.search(r"LDS Size \[bytes/block\]: (\d+)", line)
        if m and name:
            sizes[name] = int(m.group(1))
    checked = {k: v for k, v in sizes.items() if LDS_WINDOW_KERNELS.match(k)}
    if not checked:
        raise RuntimeError("no resource remarks for the kernels that address LDS from 0")
    bad = {k: v for k, v in checked.items() if v != 0}
    if bad:
        raise RuntimeError(f"kernels addressing LDS from 0 declare static LDS: {bad}")


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        cmd = [HIPCC, *FLAGS, *([REMARKS] if src == "mfma.hip" else []), "-c", os.path.join(CSRC, src),
               "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        lines = [l for l in text.splitlines()
                 if "packed-fp32-ops" not in l and "kernel-resource-usage" not in l and l.strip()]
        if p.returncode != 0:
            failed.append(src)
            print("\n".join(lines), file=sys.stderr)
        elif src == "mfma.hip":
            check_lds_window(text)
        elif verbose and lines:
            print("\n".join(lines))
    if failed:
        raise RuntimeError("hipcc failed for " + ", ".join(failed))
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
