"""Build libmmot.so for gfx950 with hipcc (in-tree, next to the package).

    python -m paper_2405_19246_amd.csrc.build        # or build() from Python

Every translation unit is compiled in parallel into _build/, then linked into
paper_2405_19246_amd/libmmot.so.  Packed-FP32 instructions are disabled for all
device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
BUILD = os.path.join(ROOT, "_build")
OUT = os.path.join(PKG, "libmmot.so")
ARCH = os.environ.get("MMOT_OFFLOAD_ARCH", "gfx950")
LMAX = 6   # the one-wavefront and register-resident kernels
WMAX = 10  # the team-layout kernels (l = 7 .. WMAX)

COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + HERE, "-I" + os.path.join(ROOT, "include")]


def _hipcc() -> str:
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(h):
        raise RuntimeError("hipcc not found")
    return h


def _units():
    units = []
    for l in range(2, LMAX + 1):
        units.append((os.path.join(HERE, "k_single.hip"), "k_single_l%d.o" % l, ["-DMMOT_L=%d" % l]))
    for l in range(7, WMAX + 1):
        units.append((os.path.join(HERE, "k_wide.hip"), "k_wide_l%d.o" % l, ["-DMMOT_L=%d" % l]))
    for l in range(2, WMAX + 1):
        units.append((os.path.join(HERE, "k_tile.hip"), "k_tile_l%d.o" % l, ["-DMMOT_L=%d" % l]))
    units.append((os.path.join(HERE, "k_batch.hip"), "k_batch.o", []))
    units.append((os.path.join(HERE, "api.cpp"), "api.o", ["-x", "hip"]))
    units.append((os.path.join(HERE, "serve.cpp"), "serve.o", ["-x", "hip"]))
    units.append((os.path.join(HERE, "tile.cpp"), "tile.o", ["-x", "hip"]))
    units.append((os.path.join(HERE, "noalloc.cpp"), "noalloc.o", ["-x", "hip"]))
    units.append((os.path.join(HERE, "twod.cpp"), "twod.o", ["-x", "hip"]))
    units.append((os.path.join(HERE, "k_2d.hip"), "k_2d.o", []))
    units.append((os.path.join(HERE, "k_dense.hip"), "k_dense.o", []))
    units.append((os.path.join(HERE, "tables.cpp"), "tables.o", []))
    return units


def _includes(path: str, seen: set) -> set:
    """Files of this directory (and include/) that path includes, transitively."""
    import re
    for name in re.findall(r'#include\s+"([^"]+)"', open(path).read()):
        for d in (HERE, os.path.join(ROOT, "include")):
            f = os.path.join(d, name)
            if os.path.exists(f) and f not in seen:
                seen.add(f)
                _includes(f, seen)
    return seen


def _stale(unit) -> bool:
    """True if the unit's object is missing or older than its source or a header it includes."""
    src, obj, _ = unit
    path = os.path.join(BUILD, obj)
    if not os.path.exists(path):
        return True
    t = os.path.getmtime(path)
    deps = _includes(src, {src})
    return any(os.path.getmtime(f) > t for f in deps)


def _compile(args):
    src, obj, extra = args
    cmd = [_hipcc()] + COMMON + extra + ["-c", src, "-o", os.path.join(BUILD, obj)]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    msgs = [ln for ln in r.stdout.splitlines() if "packed-fp32-ops" not in ln]
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), "\n".join(msgs)))
    return obj


def build(jobs: int | None = None, verbose: bool = True, only_stale: bool = False) -> str:
    """Compile every unit (only_stale: only units older than a source) and link libmmot.so."""
    os.makedirs(BUILD, exist_ok=True)
    units = _units()
    if only_stale:
        keep = [u for u in units if not _stale(u)]
        units = [u for u in units if _stale(u)]
    else:
        keep = []
    jobs = jobs or max(1, min(len(units), os.cpu_count() or 4))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, units)) + [u[1] for u in keep]
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = [_hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + \
          [os.path.join(BUILD, o) for o in objs] + ["-lpthread"]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout)
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(only_stale="--stale" in sys.argv)
    sys.exit(0)
