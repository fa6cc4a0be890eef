"""Build libwdg.so (HIP for gfx950) in-tree.

    python -m paper_1607_03399_amd.build

Every source is compiled with hipcc for gfx950, with packed FP32 VALU
instructions disabled, then linked into paper_1607_03399_amd/libwdg.so.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libwdg.so")
SOURCES = ["wedge_stage.hip", "wedge_node.hip", "tet_stage.hip", "mortar.hip", "adjoint.hip", "batch.hip", "noalloc.hip", "setup.hip", "api.cpp", "refops.cpp"]
ARCH = "gfx950"


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found")
    return exe


def common_flags(opt: str = "-O3"):
    return [opt, "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-I", os.path.join(ROOT, "include"), "-I", BUILD,
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall", "-Wno-unused-function"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    # hipcc's host pass does not know the packed-fp32 feature; that warning is expected
    out = "\n".join(l for l in proc.stdout.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if proc.returncode != 0:
        raise RuntimeError(f"command failed ({proc.returncode}): {' '.join(cmd)}\n{out}")
    if verbose and out:
        print(out)


def generate_tables(verbose: bool = False) -> None:
    """Compile and run gen_tables (host C++ only) to write ref_tables.inc, the
    reference operators that the stage kernels compile in as literals."""
    gen = os.path.join(BUILD, "gen_tables")
    cxx = shutil.which("g++") or "g++"
    _run([cxx, "-O2", "-std=c++17", os.path.join(CSRC, "gen_tables.cpp"), os.path.join(CSRC, "refops.cpp"),
          "-I", CSRC, "-o", gen], verbose)
    proc = subprocess.run([gen], stdout=subprocess.PIPE, text=True, check=True)
    out = os.path.join(BUILD, "ref_tables.inc")
    with open(out + ".tmp", "w") as fh:
        fh.write(proc.stdout)
    os.replace(out + ".tmp", out)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    generate_tables(verbose)
    cc = hipcc()
    jobs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        jobs.append([cc, *common_flags(), "-c", os.path.join(CSRC, src), "-o", obj])
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        list(ex.map(lambda c: _run(c, verbose), jobs))
    tmp = LIB + ".tmp"
    _run([cc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
