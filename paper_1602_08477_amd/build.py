"""Compiles libmg.so (HIP for gfx950) in-tree.

Every source under csrc/ is compiled with hipcc to an object in _build/ (in
parallel), then linked into paper_1602_08477_amd/libmg.so; each program under
drivers/ becomes paper_1602_08477_amd/mg_<name>, linked against it.  The same
sources built with -DMG_LDS_POISON (objects in _build/poison/) give the debug
library paper_1602_08477_amd/libmg_poison.so, whose kernels fill every LDS
stage with 0xFF bytes before refilling it (load it with MG_LIBRARY set to
its path).  Always rebuilds.
"""

from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libmg.so")
LIB_POISON = os.path.join(HERE, "libmg_poison.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

ARCH = "gfx950"
CXXFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-I" + os.path.join(ROOT, "include"),
]


def _compile(src: str, verbose: bool, poison: bool = False) -> str:
    out_dir = os.path.join(BUILD, "poison") if poison else BUILD
    obj = os.path.join(out_dir, os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith((".hip", ".cpp")) else []
    cmd = [HIPCC, *lang, *CXXFLAGS, *(["-DMG_LDS_POISON"] if poison else []), "-c", src,
           "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    # the host pass does not know the packed-fp32 feature name; that warning is harmless
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in r.stderr.splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{err}")
    if err.strip() and verbose:
        print(err)
    return obj


def drivers() -> list[str]:
    """Measurement programs linked against libmg.so (one executable each)."""
    return sorted(glob.glob(os.path.join(HERE, "drivers", "*.hip")))


def driver_path(src: str) -> str:
    return os.path.join(HERE, "mg_" + os.path.splitext(os.path.basename(src))[0])


def _build_driver(src: str, verbose: bool) -> str:
    out = driver_path(src)
    cmd = [HIPCC, "-x", "hip", *CXXFLAGS, src, "-o", out + ".tmp", "-L" + HERE, "-lmg",
           "-Wl,-rpath,$ORIGIN"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    os.replace(out + ".tmp", out)
    return out


def sources() -> list[str]:
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def _link(objs: list[str], lib: str, verbose: bool) -> None:
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", lib + ".tmp", *objs,
           "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(lib + ".tmp", lib)


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(os.path.join(BUILD, "poison"), exist_ok=True)
    srcs = sources()
    jobs = jobs or min(8, os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
        pobjs = list(ex.map(lambda s: _compile(s, verbose, True), srcs))
    _link(objs, LIB, verbose)
    _link(pobjs, LIB_POISON, verbose)
    with cf.ThreadPoolExecutor(jobs) as ex:
        list(ex.map(lambda s: _build_driver(s, verbose), drivers()))
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
