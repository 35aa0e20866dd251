"""Build libdirac.so (HIP, gfx950) in-tree.

    python -m paper_2112_14640_amd.build [--jobs N] [--verbose]

Every ``csrc/*.hip`` file is compiled to an object under ``_build/`` with hipcc
for gfx950 only, then linked into ``paper_2112_14640_amd/libdirac.so``; the
measurement probes (``measure/probe.hip``) become ``measure/libdirac_probe.so``.  The
build always recompiles (it is the "does it build" check); objects of
unchanged sources are reused only when ``incremental=True``.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libdirac.so")
# measurement probes: a library of their own, sharing no code with the operator library
PROBE_SRC = os.path.join(PKG, "measure", "probe.hip")
PROBE_LIB = os.path.join(PKG, "measure", "libdirac_probe.so")
ARCH = "gfx950"

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

COMMON_FLAGS = [
    "-O3",
    "-std=c++17",
    "-fPIC",
    f"--offload-arch={ARCH}",
    # no packed FP32 instructions (v_pk_*_f32) anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
    "-Wall",
    "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"),
]


def _compile(src: str, verbose: bool, obj: str | None = None) -> str:
    obj = obj or os.path.join(BUILD, os.path.basename(src).replace(".hip", ".o"))
    cmd = [HIPCC, *COMMON_FLAGS, "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stdout}\n{res.stderr}")
    if verbose and res.stderr.strip():
        print(res.stderr, file=sys.stderr)
    return obj


def build(jobs: int | None = None, verbose: bool = False, incremental: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    sources = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    if not sources:
        raise RuntimeError("no HIP sources found")
    headers = glob.glob(os.path.join(CSRC, "*.h")) + [os.path.join(ROOT, "include", "dirac.h")]
    newest_header = max(os.path.getmtime(h) for h in headers)

    def stale(src):
        obj = os.path.join(BUILD, os.path.basename(src).replace(".hip", ".o"))
        if not incremental or not os.path.exists(obj):
            return True
        return os.path.getmtime(obj) < max(os.path.getmtime(src), newest_header)

    todo = [s for s in sources if stale(s)]
    jobs = jobs or min(len(todo) or 1, os.cpu_count() or 4, 8)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda s: _compile(s, verbose), todo))
    objs = [os.path.join(BUILD, os.path.basename(s).replace(".hip", ".o")) for s in sources]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    _link(_compile(PROBE_SRC, verbose, os.path.join(BUILD, "measure_probe.o")), PROBE_LIB, verbose)
    return LIB


def _link(obj: str, lib: str, verbose: bool) -> None:
    tmp = lib + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", obj, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, lib)


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--incremental", action="store_true")
    a = ap.parse_args()
    print(build(a.jobs, a.verbose, a.incremental))


if __name__ == "__main__":
    main()
