"""Compile the HIP library libaeraunfold.so for gfx950, in-tree.

Every HIP source is compiled with packed-FP32 instruction selection turned
off (-Xclang -target-feature -Xclang -packed-fp32-ops); hipcc's host pass
warns that it does not know the feature, which is harmless.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libaeraunfold.so")
SOURCES = ["aeraunfold.hip", "au_server.hip"]
# the device generator of the synthetic trace stream: a library of its own
SYNTH_LIB = os.path.join(PKG, "libausynth.so")
SYNTH_SOURCES = ["au_synth.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def flags(debug: bool = False):
    f = ["--offload-arch=" + ARCH, "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + INCLUDE, "-I" + CSRC]
    f += ["-O0", "-g"] if debug else ["-O3"]
    return f


def build(verbose: bool = True, jobs: int = 4) -> str:
    """Build the unfolding library and the synthetic-stream generator library."""
    build_lib(LIB, SOURCES, verbose)
    build_lib(SYNTH_LIB, SYNTH_SOURCES, verbose)
    return LIB


def build_lib(lib_path: str, sources, verbose: bool = True) -> str:
    """Compile every source to an object in parallel, then link the shared library."""
    cc = hipcc()
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    srcs = [s for s in sources if os.path.exists(os.path.join(CSRC, s))]
    procs = []
    objs = []
    for s in srcs:
        obj = os.path.join(objdir, os.path.splitext(s)[0] + ".o")
        objs.append(obj)
        cmd = [cc] + flags() + ["-c", os.path.join(CSRC, s), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((s, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for s, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln]
        if lines and verbose:
            print("\n".join(lines), flush=True)
        if p.returncode != 0:
            failed.append(s)
    if failed:
        raise RuntimeError("hipcc failed for " + ", ".join(failed))
    tmp = lib_path + ".tmp%d" % os.getpid()
    cmd = [cc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, lib_path)
    return lib_path


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
