"""Builds libmhd.so (HIP, gfx950) in-tree: one object per grid size plus the
host/C-ABI object, compiled in parallel with hipcc.

    python -m paper_1810_12707_amd.build_lib [--jobs J] [--sizes 8,16,32]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIBDIR = os.path.join(HERE, "_lib")
LIB = os.path.join(LIBDIR, "libmhd.so")
SIZES = (8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024)
SCHED1_SIZES = (32, 64, 96, 128)  # sizes with an alternative-schedule build (the ensemble's)
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libmhd)")


def flags() -> list[str]:
    return [
        "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
        # keep the compiler from emitting packed FP32 VALU ops
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
        "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    ]


def _compile(src: str, obj: str, extra: list[str]) -> str:
    cmd = [hipcc(), *flags(), *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int | None = None, sizes=SIZES, verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 1)
    tasks = [(os.path.join(CSRC, "mhd_host.hip"), os.path.join(BUILD, "mhd_host.o"), [])]
    sz = set(sizes)
    for n in SIZES:
        # sizes left out still need their registration symbol: build them as empty stubs
        if n in sz:
            tasks.append((os.path.join(CSRC, "mhd_inst.hip"), os.path.join(BUILD, f"mhd_inst_{n}.o"), [f"-DMHD_N={n}"]))
        else:
            tasks.append((os.path.join(CSRC, "mhd_stub.hip"), os.path.join(BUILD, f"mhd_stub_{n}.o"), [f"-DMHD_N={n}"]))
    for n in SCHED1_SIZES:
        src = "mhd_inst.hip" if n in sz else "mhd_stub.hip"
        tasks.append((os.path.join(CSRC, src), os.path.join(BUILD, f"{src[:-4]}_s1_{n}.o"),
                      [f"-DMHD_N={n}", "-DMHD_SCHED=1"]))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = [ex.submit(_compile, *t) for t in tasks]
        objs = [f.result() for f in futs]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--sizes", type=str, default=None)
    a = ap.parse_args(argv)
    sizes = SIZES if not a.sizes else tuple(int(s) for s in a.sizes.split(","))
    build(a.jobs, sizes)


if __name__ == "__main__":
    sys.exit(main())
