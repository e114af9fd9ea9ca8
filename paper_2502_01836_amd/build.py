"""Build libleafi.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2502_01836_amd.build [--jobs N] [--debug]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libleafi.so")
BUILD = os.path.join(HERE, "_build")
SOURCES = ["api.hip", "serve.hip", "noalloc.hip", "k_prep.hip", "k_rounds.hip", "k_scan.hip", "k_rerank.hip", "k_mlp.hip", "k_cnn.hip", "tree.cpp",
           "calib.cpp"]
ARCH = os.environ.get("LEAFI_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libleafi)")


def _flags(debug: bool):
    f = ["-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result"]
    f += ["-O1", "-g"] if debug else ["-O3"]
    return f


def build(jobs: int = 0, debug: bool = False, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    cc = hipcc()
    objs = []

    def compile_one(src):
        path = os.path.join(CSRC, src)
        obj = os.path.join(BUILD, src + ".o")
        cmd = [cc] + _flags(debug) + ["-I", CSRC]
        if src.endswith(".hip"):
            # packed FP32 instructions stay off in device code
            cmd += ["-x", "hip", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
        else:
            cmd += ["-D__HIP_PLATFORM_AMD__"]
        cmd += ["-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        errs = "\n".join(l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l)
        if res.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{errs}")
        if errs.strip() and verbose:
            print(errs)
        return obj

    n = jobs or min(len(SOURCES), max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(max_workers=n) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = OUT + ".tmp"
    link = [cc, "-shared", f"--offload-arch={ARCH}", "-o", tmp] + objs + ["-lamdhip64"]
    res = subprocess.run(link, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + res.stderr)
    os.replace(tmp, OUT)
    return OUT


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=0)
    ap.add_argument("--debug", action="store_true")
    ap.add_argument("-v", "--verbose", action="store_true")
    a = ap.parse_args(argv)
    print(build(a.jobs, a.debug, a.verbose))


if __name__ == "__main__":
    sys.exit(main())
