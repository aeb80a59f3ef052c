"""Builds libxdrop.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC_DIR = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libxdrop.so")
ARCH = os.environ.get("XDROP_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    "--offload-arch=" + ARCH,
    # keep hipcc from forming packed fp32 instructions (no float math here,
    # but the flag applies to every HIP build of this project)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
    "-I" + SRC_DIR,
]


def sources():
    return [os.path.join(SRC_DIR, f) for f in sorted(os.listdir(SRC_DIR)) if f.endswith(".hip")]


# instrumented variant: per-wave busy intervals of the extension kernels
# (xd_debug_stamps_arm / xd_debug_stamps_count), loaded when XDROP_LIB=stamps
VARIANTS = {"": [], "stamps": ["-DXD_WAVE_STAMPS"]}


def lib_path(variant: str = "") -> str:
    return os.path.join(HERE, "libxdrop%s.so" % ("_" + variant if variant else ""))


def build(verbose: bool = False, variants=("", "stamps")) -> str:
    """Compile every HIP source into one shared library per variant (in
    parallel); always rebuilds.  Returns the product library's path."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    procs = []
    for v in variants:
        dst = lib_path(v)
        tmp = dst + ".tmp%d" % os.getpid()
        cmd = [hipcc] + HIPCC_FLAGS + VARIANTS[v] + ["-o", tmp] + sources()
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((dst, tmp, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                 stderr=subprocess.STDOUT, text=True)))
    failed = []
    for dst, tmp, pr in procs:
        text, _ = pr.communicate()
        out = "\n".join(l for l in text.splitlines()
                        if "packed-fp32-ops" not in l and "hip-link" not in l)
        if pr.returncode != 0:
            failed.append("%s:\n%s" % (os.path.basename(dst), out))
        else:
            os.replace(tmp, dst)
    if failed:
        raise RuntimeError("hipcc failed:\n" + "\n".join(failed))
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
