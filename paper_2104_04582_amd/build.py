"""Build libfew.so for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libfew.so")
SOURCES = ["kernels.hip", "few_api.cpp", "host_core.cpp"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed binary32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", "-Wno-unused-value",
]


# Host-code checking build: AddressSanitizer and UndefinedBehaviorSanitizer on
# the host pass only (the GPU code is not instrumented); any report aborts.
SAN_OUT = os.path.join(HERE, "libfew_san.so")
SAN_FLAGS = [
    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
    "-g",
]


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """Compile libfew.so (or, sanitize=True, libfew_san.so)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    out = SAN_OUT if sanitize else OUT
    cmd = [hipcc] + HIPCC_FLAGS + (SAN_FLAGS if sanitize else []) + ["-o", out + ".tmp"] + \
        [os.path.join(CSRC, s) for s in SOURCES] + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed with status {r.returncode}")
    os.replace(out + ".tmp", out)
    return out


def sanitizer_runtime() -> str:
    """Path of the compiler's AddressSanitizer runtime, to be preloaded into
    the Python process that loads libfew_san.so."""
    clang = os.environ.get("HIP_CLANG", "/opt/rocm/llvm/bin/clang++")
    r = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True, check=True)
    return r.stdout.strip()


def run_host_tests_sanitized(pytest_args=("tests/test_host_core.py", "-q")) -> int:
    """Build libfew_san.so and run the host-side CPU tests against it in a
    child process with the sanitizer runtime preloaded.  Returns pytest's status."""
    lib = build(sanitize=True)
    env = dict(os.environ)
    env["LD_PRELOAD"] = sanitizer_runtime()
    env["FEW_LIBRARY"] = lib
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    root = os.path.dirname(HERE)
    try:
        return subprocess.run([sys.executable, "-m", "pytest", *pytest_args,
                               "-p", "no:cacheprovider"], cwd=root, env=env).returncode
    finally:
        os.remove(lib)          # a checking build only: nothing else loads it


if __name__ == "__main__":
    if "--sanitize-check" in sys.argv:
        sys.exit(run_host_tests_sanitized())
    print(build(verbose=True, sanitize="--sanitize" in sys.argv))
