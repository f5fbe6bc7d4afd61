"""Builds libdsoar.so (HIP for gfx950) in the package directory, and
libdsoar_chaos.so: the same sources compiled with DSOAR_CHAOS, which puts
short hash-chosen pauses into the heap's race windows for the stress tests."""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(os.path.dirname(HERE), "_build")
LIB = os.path.join(HERE, "libdsoar.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall",
         "-Wno-unused-command-line-argument"]


def sources() -> list[str]:
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


VARIANTS = {"release": ("libdsoar.so", []), "chaos": ("libdsoar_chaos.so", ["-DDSOAR_CHAOS"])}


def _compile(src: str, variant: str) -> str:
    out_dir = os.path.join(BUILD, variant)
    obj = os.path.join(out_dir, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, *VARIANTS[variant][1], "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src} ({variant}):\n{r.stderr}")
    return obj


def _link(objs: list[str], lib: str) -> str:
    tmp = lib + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, lib)
    return lib


def build(jobs: int = 8, variants=("release", "chaos")) -> str:
    """Compiles every variant (all sources of all variants in one pool) and
    returns the release library's path."""
    for v in variants:
        os.makedirs(os.path.join(BUILD, v), exist_ok=True)
    work = [(src, v) for v in variants for src in sources()]
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda a: _compile(*a), work))
    for v in variants:
        _link([o for o, (_, ov) in zip(objs, work) if ov == v], os.path.join(HERE, VARIANTS[v][0]))
    return LIB


if __name__ == "__main__":
    print(build(int(sys.argv[1]) if len(sys.argv) > 1 else 8))
