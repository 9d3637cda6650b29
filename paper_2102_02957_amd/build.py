"""Build libqsv.so (gfx950) in-tree with hipcc.

Usage: python -m paper_2102_02957_amd.build [--incremental]  (or build() from Python).
By default every source is recompiled; sources are compiled in parallel.
"""

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libqsv.so")
OBJDIR = os.path.join(HERE, "_build")

SOURCES = ["gates.cpp", "planner.cpp", "density.cpp", "runtime.hip", "section_kernel.hip", "section_c128.hip", "section_c64.hip", "section_lds.hip", "section_paired.hip",
           "pergate_kernels.hip", "misc_kernels.hip", "batch.hip", "adjoint.hip", "autotune.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-I" + INCLUDE, "-I" + CSRC,
          "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]
# Packed FP32 instructions are kept out of the device code.  Common-code sinking
# is off: it merges the per-position branches of the register kernels into one
# with runtime-selected register addresses, which sends the amplitude array to
# scratch memory.
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-mllvm", "-simplifycfg-sink-common=false"]


def _stale(obj, src_path):
    """Object older than its source or than any header (headers are not tracked
    per source: a header change rebuilds everything)."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    heads = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))]
    heads += [os.path.join(INCLUDE, f) for f in os.listdir(INCLUDE)]
    return any(os.path.getmtime(f) > t for f in [src_path] + heads)


def _compile(src, incremental=False):
    path = os.path.join(CSRC, src)
    obj = os.path.join(OBJDIR, src + ".o")
    if incremental and not _stale(obj, path):
        return obj, ""
    if src.endswith(".hip"):
        cmd = [HIPCC, "-x", "hip"] + DEVICE + COMMON + ["-c", path, "-o", obj]
    else:
        cmd = [HIPCC, "-x", "c++"] + COMMON + ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (src, " ".join(cmd), msg))
    return obj, msg


def build(verbose=False, incremental=False):
    """Compile every source (incremental=True: only sources whose object is
    older than the source or any header) and link libqsv.so."""
    os.makedirs(OBJDIR, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        results = list(ex.map(lambda f: _compile(f, incremental), SOURCES))
    for obj, msg in results:
        if verbose and msg.strip():
            print(msg)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + [o for o, _ in results]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stdout + r.stderr))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv))
