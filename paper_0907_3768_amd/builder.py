"""Compile libdust.so for gfx950 with hipcc (in-tree, no JIT cache).

Every translation unit under csrc/ is compiled to an object in parallel and
linked into paper_0907_3768_amd/libdust.so.  The measurement-only ALU probes
under measure/ become a library of their own, libdust_probe.so, which only
the benchmark loads.  Packed FP32 instructions are disabled for the device
code (-packed-fp32-ops): the kernels are written with ordinary scalar float
arithmetic.

Machine-level loop-invariant code motion is disabled (-disable-machine-licm):
it hoists the constants of the tile bodies' rarely taken FP64 paths (the
series coefficients of the exact fallback) out of the enclosing loops, where
they hold registers for the whole tile and push the kernels that ask for six
resident waves into spilling (the fused kernel 80 bytes per lane, the
persistent batch kernel over a kilobyte).  Without it the fused kernels do
not spill (the four-tile form a few registers), and measured 1-3 % faster.
"""
from __future__ import annotations

import concurrent.futures
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
MEASURE = os.path.join(HERE, "measure")
LIB = os.path.join(HERE, "libdust.so")
PROBE_LIB = os.path.join(HERE, "libdust_probe.so")
ARCH = os.environ.get("DUST_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags(licm: bool = False):
    """Device-code flags of libdust (machine LICM off); licm=True keeps the
    pass, for the ALU probes, whose loops must hold only the instructions
    they time (without it the compiler rebuilds a constant in every
    iteration of the FMA chain)."""
    return (["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] +
            ([] if licm else ["-mllvm", "-disable-machine-licm"]) +
            ["-Wall", "-Wno-unused-result", "-I", INCLUDE, "-I", CSRC])


def _compile_link(srcs, lib, objdir, extra_inc, verbose, licm=False):
    cc = hipcc()
    os.makedirs(objdir, exist_ok=True)

    def compile_one(src):
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        cmd = [cc] + flags(licm) + extra_inc + ["-c", src, "-o", obj]
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{out}")
        if verbose and out.strip():
            print(out, file=sys.stderr)
        return obj

    workers = min(len(srcs), max(1, min(8, os.cpu_count() or 1)))
    with concurrent.futures.ThreadPoolExecutor(workers) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [cc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout)
    os.replace(tmp, lib)
    return lib


def build(verbose: bool = False) -> str:
    """Build libdust.so and the benchmark's libdust_probe.so; returns the
    path of libdust.so."""
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    _compile_link(srcs, LIB, os.path.join(ROOT, "_build", "obj"), [], verbose)
    _compile_link(sorted(glob.glob(os.path.join(MEASURE, "*.hip"))), PROBE_LIB,
                  os.path.join(ROOT, "_build", "obj_probe"), ["-I", MEASURE], verbose, licm=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
