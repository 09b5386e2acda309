"""Build the gfx950 shared library libgp.so in-tree with hipcc.

The library is C++/HIP only; this module just drives the compiler.  Every
evaluation kernel must keep its stack in registers: the build fails if the
compiler reports private (scratch) memory for any of them.
"""
from __future__ import annotations

import os
import re
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libgp.so")
SOURCES = [os.path.join(CSRC, "gp_device.hip"), os.path.join(CSRC, "gp_mutate.hip"), os.path.join(CSRC, "gp_host.cpp")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # every float operation rounds on its own: no contraction into FMA
    "-ffp-contract=off",
    # no packed-FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # leave regions whose branches are all wave-uniform unstructured: the
    # evaluation kernel's dispatch on a scalar opcode then compiles to plain
    # compare-and-branch trees, without the exec-mask flag bookkeeping the
    # structurizer adds (about 30% fewer scalar instructions per dispatch)
    "-mllvm", "-structurizecfg-skip-uniform-regions=true",
    "-Rpass-analysis=kernel-resource-usage",
]


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-o", tmp, *SOURCES]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stderr[-6000:])
    usage = parse_resource_usage(res.stderr)
    bad = [k for k, v in usage.items() if v.get("scratch", 0) > 0]
    if bad:
        raise RuntimeError("kernels spill to scratch memory: " + ", ".join(bad))
    os.replace(tmp, LIB)
    if verbose:
        for k, v in usage.items():
            print(k, v)
    return LIB


def parse_resource_usage(text: str) -> dict:
    """Per-kernel VGPRs / scratch bytes / occupancy from the compiler's
    kernel-resource-usage remarks."""
    out, cur = {}, None
    for line in text.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            out[cur] = {}
            continue
        if cur is None:
            continue
        for key, pat in (("vgpr", r"\bVGPRs: (\d+)"), ("scratch", r"ScratchSize \[bytes/lane\]: (\d+)"),
                         ("occupancy", r"Occupancy \[waves/SIMD\]: (\d+)")):
            m = re.search(pat, line)
            if m:
                out[cur][key] = int(m.group(1))
    return out


if __name__ == "__main__":
    print(build(verbose=True))
