"""Build libhologen.so for gfx950 in-tree with hipcc.

    python -m paper_2006_10509_amd.build

Always recompiles: one object per transform length (csrc/length.hip with
-DHG_LEN=N) plus the host runtime (csrc/hologen.hip), compiled in parallel and
linked into paper_2006_10509_amd/libhologen.so.  Packed-FP32 instructions are
disabled for the device code; the host pass warns that it does not know that
target feature, which is harmless.
"""
from __future__ import annotations

import os
import re
import shutil
import subprocess
import sys
import tempfile
import time
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libhologen.so")
ARCH = os.environ.get("HG_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found")
    return path


def lengths(csrc: str = CSRC) -> list:
    text = open(os.path.join(csrc, "sizes.hpp")).read()
    block = text[text.index("#define HG_FOR_EACH_LENGTH"):]
    block = block[:block.index("\n\n")]
    return [int(n) for n in re.findall(r"X\((\d+)\)", block)]


def common_flags() -> list:
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include")]


def _run(cmd):
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + proc.stdout + proc.stderr)
    return proc.stderr


def build_library(csrc: str, out: str, jobs: int = 0) -> str:
    """Compile the sources in csrc (the lengths its sizes.hpp lists) into out."""
    jobs = jobs or min(16, os.cpu_count() or 4)
    with tempfile.TemporaryDirectory(prefix="hg_build_") as tmp:
        jobs_list = []
        for n in lengths(csrc):
            obj = os.path.join(tmp, f"len_{n}.o")
            jobs_list.append([hipcc(), *common_flags(), f"-DHG_LEN={n}", "-c",
                              os.path.join(csrc, "length.hip"), "-o", obj])
        host_obj = os.path.join(tmp, "hologen.o")
        jobs_list.append([hipcc(), *common_flags(), "-c", os.path.join(csrc, "hologen.hip"), "-o", host_obj])
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            list(ex.map(_run, jobs_list))
        objs = [j[-1] for j in jobs_list]
        out_tmp = out + ".tmp"
        _run([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", out_tmp])
        os.replace(out_tmp, out)
    return out


def build(verbose: bool = False, jobs: int = 0) -> str:
    t0 = time.time()
    build_library(CSRC, LIB, jobs)
    if verbose:
        print(f"built {LIB} ({len(lengths())} transform lengths) in {time.time() - t0:.1f} s")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
