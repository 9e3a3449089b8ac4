"""Host-side sanitizer runs (no GPU needed).

* The FP64 oracle, built with gcc's AddressSanitizer and
  UndefinedBehaviorSanitizer together with tests/sanitize/oracle_driver.c,
  which calls every oracle entry point on odd and even sizes at every depth.
* The C ABI's host code: libhaar rebuilt with the sanitizers on its host
  pass only (the gfx950 device code is compiled as usual), linked into
  tests/sanitize/abi_driver.cpp, which runs every validation path, the
  host-only queries, plan creation and the tuning table's JSON round trip.
  Nothing in it reaches a HIP call, so it runs on a machine without a GPU.

Any sanitizer report aborts the driver (no recovery), so a clean exit is the
pass condition.  The library build takes about a minute and a half; it is
cached under _build/sanitize/ keyed by a hash of the sources and flags."""
import glob
import hashlib
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CACHE = os.path.join(ROOT, "_build", "sanitize")

# host-pass sanitizer flags of the HIP build (device code is not instrumented)
HOST_SAN = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=all",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]
HOST_SAN_LINK = ["-Xarch_host", "-fsanitize=address,undefined", "-shared-libsan"]


def _run(cmd, env=None, cwd=None):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, cwd=cwd, timeout=900)
    return r.returncode, r.stdout + r.stderr


def test_oracle_under_asan_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_driver")
    rc, out = _run([gcc, "-std=c11", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", os.path.join(SAN, "oracle_driver.c"),
                    os.path.join(ROOT, "oracle", "haar_oracle.c"), "-lm", "-o", exe])
    assert rc == 0, out
    rc, out = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    assert rc == 0 and "all calls clean" in out, out


def _clang_rt_dir():
    hits = glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    return os.path.dirname(hits[0]) if hits else None


def _sanitized_library():
    from paper_1002_2184_amd import build as B
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(B.CSRC, "*"))) + [os.path.join(B.INCLUDE, "haar.h")]:
        with open(p, "rb") as f:
            h.update(f.read())
    h.update(" ".join(B.FLAGS + HOST_SAN + HOST_SAN_LINK).encode())
    d = os.path.join(CACHE, h.hexdigest()[:16])
    lib = os.path.join(d, "libhaar_san.so")
    if not os.path.exists(lib):
        shutil.rmtree(CACHE, ignore_errors=True)
        os.makedirs(d)
        B.build(force=True, out=lib, extra_flags=HOST_SAN, link_flags=HOST_SAN_LINK)
    return lib


@pytest.mark.slow
def test_abi_host_code_under_asan_ubsan(tmp_path):
    from paper_1002_2184_amd import build as B
    rt = _clang_rt_dir()
    if rt is None:
        pytest.skip("clang sanitizer runtime not found")
    lib = _sanitized_library()
    exe = str(tmp_path / "abi_driver")
    rc, out = _run([B.HIPCC, *HOST_SAN, "-shared-libsan", f"-I{B.INCLUDE}", os.path.join(SAN, "abi_driver.cpp"),
                    "-o", exe, f"-L{os.path.dirname(lib)}", "-lhaar_san", f"-Wl,-rpath,{os.path.dirname(lib)}"])
    assert rc == 0, out
    env = dict(os.environ, LD_LIBRARY_PATH=rt + os.pathsep + os.environ.get("LD_LIBRARY_PATH", ""),
               ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    rc, out = _run([exe, str(tmp_path / "table.json")], env=env)
    assert rc == 0 and "all calls clean" in out, out
    assert "runtime error" not in out, out
