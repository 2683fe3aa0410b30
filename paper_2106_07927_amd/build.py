"""Build libsgm.so (the gfx950 HIP kernels and the C ABI of include/sgm.h).

    python -m paper_2106_07927_amd.build [--incremental]

Every source is compiled by hipcc for gfx950 only, in-tree, into
``paper_2106_07927_amd/libsgm.so``.  Packed-FP32 instruction selection is
switched off for the device code.  ``paths.hip`` (the path pass) is compiled
once per lane layout (-DSGM_PATH_LAYOUT=k) and per form (-DSGM_PATH_PART=0
for the single-frame kernels, 1 for the work-list kernels), so its kernels
build in parallel.
"""
from __future__ import annotations

import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libsgm.so")

HIP_SOURCES = ["census.hip", "cost.hip", "ncc.hip", "aggregate.hip", "wta_lrc.hip", "noalloc.hip"]
CPP_SOURCES = ["sgm_capi.cpp", "batch.cpp"]
PATH_LAYOUTS = 12          # entries of kPathLayouts in sgm_internal.h
# (source, object, extra flags) of every translation unit
UNITS = ([(s, s + ".o", []) for s in HIP_SOURCES + CPP_SOURCES] +
         [("paths.hip", f"paths_{k}_{part}.hip.o", [f"-DSGM_PATH_LAYOUT={k}", f"-DSGM_PATH_PART={part}"])
          for k in range(PATH_LAYOUTS) for part in (0, 1)])

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
          "-I", INCLUDE, "-I", CSRC]
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _hipcc():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    path = os.path.join(rocm, "bin", "hipcc")
    return path if os.path.exists(path) else "hipcc"


def _compile(unit) -> str:
    src, objname, extra = unit
    obj = os.path.join(BUILD, objname)
    cmd = [_hipcc(), *COMMON, *extra]
    if src.endswith(".hip"):
        cmd += ["-x", "hip", *DEVICE, "-Rpass-analysis=kernel-resource-usage"]
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stderr}")
    if src.endswith(".hip"):
        _check_resources(src, res.stderr)
    return obj


def _check_resources(src: str, remarks: str) -> None:
    """Every kernel keeps its state in registers: a kernel with per-lane
    scratch (spills or private arrays) fails the build."""
    name = None
    bad = []
    for line in remarks.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and int(m.group(1)) > 0:
            bad.append(f"{name}: {m.group(1)} bytes/lane")
    if bad:
        raise RuntimeError(f"{src}: kernels with scratch memory:\n  " + "\n  ".join(bad))


def _stale(unit) -> bool:
    """True when the unit's object is missing or older than its source or any
    header."""
    src, objname, _ = unit
    obj = os.path.join(BUILD, objname)
    if not os.path.exists(obj):
        return True
    deps = [os.path.join(CSRC, src)]
    deps += [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".h")]
    deps += [os.path.join(INCLUDE, h) for h in os.listdir(INCLUDE) if h.endswith(".h")]
    return max(os.path.getmtime(d) for d in deps) > os.path.getmtime(obj)


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every source (with incremental=True: only those whose object is
    out of date) and link libsgm.so; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    todo = [u for u in UNITS if not incremental or _stale(u)]
    # the path-pass objects take longest: start them first
    todo.sort(key=lambda u: 0 if u[0] == "paths.hip" else 1)
    workers = max(1, min(len(todo), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(max_workers=workers) as pool:
        list(pool.map(_compile, todo))
    objs = [os.path.join(BUILD, u[1]) for u in UNITS]
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True, incremental="--incremental" in sys.argv[1:])
    sys.exit(0)
