"""Host-side sanitizer run: AddressSanitizer + UndefinedBehaviorSanitizer
builds of the library's host code (argument validation, plan and table
building, the C ABI) and of the C oracle, and the CPU test suite
(pytest -m "not gpu") run against them.

GPU code is built as usual (device code is not instrumented: the sanitizer
flags reach the host pass only).  Both libraries are compiled with the ROCm
clang so that one sanitizer runtime serves the process; it is preloaded into
the Python interpreter, which is not instrumented itself (leak reports are
off: the interpreter keeps its allocations to the end).  Any report aborts
the run with a non-zero status.

    python paper_2007_12065_amd/sanitize.py [extra pytest arguments]
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
OUT = os.path.join(HERE, "_build", "sanitize")
CLANG = "/opt/rocm/llvm/bin/clang"
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer"]


def runtime() -> str:
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not found:
        raise RuntimeError("the clang AddressSanitizer runtime is not installed")
    return found[-1]


def build_library() -> str:
    sys.path.insert(0, HERE)
    import build as hip_build
    extra = []
    for f in SAN:
        extra += ["-Xarch_host", f]
    lib = os.path.join(OUT, "libpl.so")
    os.makedirs(OUT, exist_ok=True)
    hip_build.build(out=lib, build_dir=os.path.join(OUT, "obj"), extra=extra)
    return lib


def build_oracle() -> str:
    lib = os.path.join(OUT, "liboracle.so")
    os.makedirs(OUT, exist_ok=True)
    subprocess.check_call([CLANG, "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                           "-ffp-contract=off", "-fno-fast-math", *SAN,
                           "-o", lib, os.path.join(ROOT, "oracle", "pl_oracle.c"), "-lm"])
    return lib


def main(argv) -> int:
    lib, orc = build_library(), build_oracle()
    env = dict(os.environ)
    env.update(PL_LIBRARY=lib, PL_ORACLE_LIBRARY=orc, LD_PRELOAD=runtime(),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    cmd = [sys.executable, "-m", "pytest", os.path.join(ROOT, "tests"), "-q", "-m", "not gpu",
           "-p", "no:cacheprovider", *argv]
    print("sanitized libraries:", lib, orc, flush=True)
    return subprocess.call(cmd, cwd=ROOT, env=env)


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
