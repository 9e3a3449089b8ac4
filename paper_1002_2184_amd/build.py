"""Compile libhaar.so (every HIP source under csrc/) for gfx950, in-tree.

    python -m paper_1002_2184_amd.build [--force] [-j N]

Each source is compiled to an object in parallel, then linked into
``paper_1002_2184_amd/libhaar.so``.  Always rebuilds when called through
``build(force=True)``.
"""
from __future__ import annotations

import argparse
import glob
import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libhaar.so")
ARCH = "gfx950"

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off",                       # arithmetic exactly as written (pair sums)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = sources() + glob.glob(os.path.join(CSRC, "*.h")) + [os.path.join(INCLUDE, "haar.h")]
    return any(os.path.getmtime(d) > t for d in deps)


def build(force: bool = True, jobs: int = 8, verbose: bool = False, defines=(), out: str = LIB,
          extra_flags=(), link_flags=()) -> str:
    """Compile and link; `defines` adds -D flags, `out` redirects the library,
    `extra_flags` / `link_flags` go to every compile / the link (the tests'
    host-sanitizer build uses them)."""
    if not force and not _stale() and out == LIB and not defines and not extra_flags:
        return LIB
    tmp = tempfile.mkdtemp(prefix="haarbuild_")
    try:
        def compile_one(src):
            obj = os.path.join(tmp, os.path.basename(src) + ".o")
            cmd = [HIPCC, *FLAGS, *extra_flags, *[f"-D{d}" for d in defines], "-c", src, "-o", obj]
            r = subprocess.run(cmd, capture_output=True, text=True)
            if r.returncode != 0:
                raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
            if verbose and r.stderr.strip():
                print(r.stderr, file=sys.stderr)
            return obj

        with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
            objs = list(ex.map(compile_one, sources()))
        out_tmp = out + f".tmp{os.getpid()}"
        cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *link_flags, "-o", out_tmp, *objs]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed:\n{r.stderr}")
        os.replace(out_tmp, out)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--force", action="store_true")
    ap.add_argument("-j", type=int, default=8)
    ap.add_argument("-v", action="store_true")
    ap.add_argument("-D", action="append", default=[], help="extra preprocessor define")
    ap.add_argument("-o", default=LIB, help="output library path")
    a = ap.parse_args()
    print(build(force=True, jobs=a.j, verbose=a.v, defines=a.D, out=a.o))


if __name__ == "__main__":
    main()
