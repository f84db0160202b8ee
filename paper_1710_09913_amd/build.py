"""Build libdogip.so (HIP for gfx950) in-tree.

    python -m paper_1710_09913_amd.build [-j N] [-v]

Every source under csrc/ is compiled with hipcc into _build/, then linked into
paper_1710_09913_amd/libdogip.so.  Objects are rebuilt when a source or any
header is newer than the object.
"""

from __future__ import annotations

import argparse
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libdogip.so")
ARCH = os.environ.get("DOGIP_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-fPIC",
    "-std=c++20",
    "-munsafe-fp-atomics",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fconstexpr-steps=400000000",
    "-Wno-unused-command-line-argument",
    f"-I{INCLUDE}",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def _headers_mtime():
    hs = glob.glob(os.path.join(CSRC, "*.hpp")) + glob.glob(os.path.join(INCLUDE, "*.h"))
    return max((os.path.getmtime(h) for h in hs), default=0.0)


# the sources the element-wise apply is built from: its tile and finish kernels, their
# headers and B^ tables, the host code that plans the tiles and launches them, and the
# compiler flags in this file
APPLY_SOURCES = ("kern_apply.hpp", "kern_apply_u2.hip", "kern_apply_u3.hip", "kern_apply_l2.hip",
                 "kern_apply_l3.hip", "kern_aux.hip", "kern_common.hpp", "reftab.hpp", "internal.hpp", "setup.cpp",
                 "op.cpp")


def apply_hash() -> str:
    """SHA-256 over the apply's sources (identifies the kernels that counter summaries
    were taken on)."""
    import hashlib

    h = hashlib.sha256()
    for f in sorted(os.path.join(CSRC, n) for n in APPLY_SOURCES) + [os.path.abspath(__file__)]:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def source_hash() -> str:
    """SHA-256 over the kernel and host sources and the public header (identifies a build)."""
    import hashlib

    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(CSRC, "*")) + glob.glob(os.path.join(INCLUDE, "*.h")))
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _compile(src: str, force: bool, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if not force and os.path.exists(obj):
        if os.path.getmtime(obj) >= max(os.path.getmtime(src), _headers_mtime()):
            return obj
    cmd = [hipcc()] + FLAGS + ["-c", src, "-o", obj + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {os.path.basename(src)}:\n{r.stdout}\n{r.stderr}")
    os.replace(obj + ".tmp", obj)
    return obj


def build(force: bool = True, jobs: int | None = None, verbose: bool = False) -> str:
    """Compile and link; returns the library path.  force=True recompiles everything."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = _sources()
    jobs = jobs or min(8, os.cpu_count() or 4)
    # largest translation units first
    srcs.sort(key=lambda s: -os.path.getsize(s) - (10 ** 6 if "_u" in os.path.basename(s) else 0))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, force, verbose), srcs))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs + ["-Wl,-rpath,/opt/rocm/lib"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=None)
    ap.add_argument("-v", action="store_true")
    ap.add_argument("--incremental", action="store_true", help="only rebuild out-of-date objects")
    a = ap.parse_args(argv)
    path = build(force=not a.incremental, jobs=a.j, verbose=a.v)
    print(path)


if __name__ == "__main__":
    sys.exit(main())
