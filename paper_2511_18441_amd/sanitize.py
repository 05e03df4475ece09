"""Host-code sanitizer run (CPU only): AddressSanitizer and UndefinedBehaviorSanitizer
builds of the FP64 oracle and of the host side of librecogs.so (argument checks,
workspace carving, launch set-up; the gfx950 device code is built as usual), then the
CPU test suite against them.

    python paper_2511_18441_amd/sanitize.py [pytest args...]

Both libraries are built with the ROCm clang, so one ASan runtime (preloaded into the
Python process, which is not instrumented itself) serves both. Builds go to _build/san/
(git-ignored); the in-tree libraries are not touched. Leak detection is off: the
interpreter and torch keep allocations alive until exit by design.
"""
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
OUT = os.path.join(ROOT, "_build", "san")
CLANG = "/opt/rocm/llvm/bin/clang"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]


def asan_runtime() -> str:
    libs = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not libs:
        raise RuntimeError("no clang ASan runtime under /opt/rocm/llvm")
    return libs[-1]


def build() -> tuple:
    os.makedirs(OUT, exist_ok=True)
    orc = os.path.join(OUT, "liborc_san.so")
    subprocess.run([CLANG, "-O1", "-std=gnu11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", *SAN,
                    "-o", orc, os.path.join(ROOT, "oracle", "recogs_oracle.c"), "-lm"], check=True)
    lib = os.path.join(OUT, "librecogs_san.so")
    host = [x for f in SAN for x in ("-Xarch_host", f)]
    srcs = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-O1", "-std=c++17", "-fPIC", "-shared",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-munsafe-fp-atomics",
                    "-Wno-unused-command-line-argument", *host, "-I", os.path.join(ROOT, "include"), *srcs, "-o", lib],
                   check=True)
    return orc, lib


def main(argv) -> int:
    orc, lib = build()
    env = dict(os.environ)
    env.update(RECOGS_ORACLE_LIB=orc, RECOGS_LIB=lib, LD_PRELOAD=asan_runtime(),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    cmd = [sys.executable, "-m", "pytest", os.path.join(ROOT, "tests"), "-q", "-m", "not gpu", "-p", "no:cacheprovider",
           *argv]
    print(" ".join(cmd), flush=True)
    return subprocess.run(cmd, env=env, cwd=ROOT).returncode


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
