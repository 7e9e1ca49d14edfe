"""Build libkrig.so (HIP, gfx950) in-tree.

    python -m paper_2605_29284_amd.build [-j JOBS]

Every transform length listed in csrc/fft_sizes.h gets its own small generated
translation unit so the instantiations compile in parallel; all objects are
linked into paper_2605_29284_amd/libkrig.so.
"""
from __future__ import annotations

import argparse
import os
import re
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
ROOT = os.path.dirname(PKG)
BUILD = os.path.join(ROOT, "_build", "krig")
LIB = os.path.join(PKG, "libkrig.so")

ARCH = os.environ.get("KRIG_OFFLOAD_ARCH", "gfx950")
FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
    # hand-written packed FP32 forms are avoided and the compiler may not form them
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def fft_sizes():
    txt = open(os.path.join(CSRC, "fft_sizes.h")).read()
    return [tuple(int(v) for v in m) for m in re.findall(r"X\((\d+),\s*(\d+),\s*(\d+)\)", txt)]


def hipcc():
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc") or ""):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return cmd[-1]


def build(jobs: int = 8, verbose: bool = False) -> str:
    os.makedirs(os.path.join(BUILD, "gen"), exist_ok=True)
    cc = hipcc()
    units = []
    for a, b, c in fft_sizes():
        src = os.path.join(BUILD, "gen", f"fft_{a}x{b}x{c}.hip")
        body = f'#include "{CSRC}/fft_passes.h"\nKRIG_FFT_SIZE({a}, {b}, {c})\n'
        if not os.path.exists(src) or open(src).read() != body:
            with open(src, "w") as f:
                f.write(body)
        units.append(src)
    for name in ("dense.hip", "setup.hip", "exact.hip", "interp.hip", "mixture.hip", "universal.hip", "plan.cpp", "fft_registry.cpp"):
        path = os.path.join(CSRC, name)
        if os.path.exists(path):
            units.append(path)
    cmds = []
    objs = []
    for u in units:
        obj = os.path.join(BUILD, os.path.basename(u) + ".o")
        lang = ["-x", "hip"] if u.endswith(".cpp") else []
        cmds.append([cc] + FLAGS + lang + ["-c", u, "-o", obj])
        objs.append(obj)
    # largest units first
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        for done in ex.map(_run, cmds):
            if verbose:
                print("built", done, flush=True)
    tmp = LIB + ".tmp"
    _run([cc, "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", "--jobs", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("-v", "--verbose", action="store_true")
    a = ap.parse_args(argv)
    print(build(a.jobs, a.verbose))


if __name__ == "__main__":
    sys.exit(main())
