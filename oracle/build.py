"""Compile the CPU oracle (test infrastructure) into ``oracle/libtsds_oracle.so``.

Plain gcc, ``-O2 -ffp-contract=off``: no fused multiply-add, so every floating
point expression in the oracle is rounded exactly as it is written.  With
TSDS_SANITIZE=1 the oracle is built with ASan/UBSan instead (CPU runs only).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tsds_oracle.c")
LIB = os.path.join(HERE, "libtsds_oracle.so")


LIB_SAN = os.path.join(HERE, "libtsds_oracle_san.so")
# AddressSanitizer + UndefinedBehaviorSanitizer build of the same source (CPU
# test runs only): ROCm's clang, so that one sanitizer runtime serves both the
# oracle and the sanitized host code of the GPU library in one process.
CLANG = "/opt/rocm/llvm/bin/clang"
SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined", "-shared-libsan"]


def sanitize_requested() -> bool:
    return os.environ.get("TSDS_SANITIZE", "") == "1"


def build(force: bool = True, sanitize: bool = None) -> str:
    sanitize = sanitize_requested() if sanitize is None else sanitize
    lib = LIB_SAN if sanitize else LIB
    if not force and os.path.exists(lib) and os.path.getmtime(lib) >= os.path.getmtime(SRC):
        return lib
    tmp = lib + ".tmp"
    if sanitize:
        cmd = [CLANG, *SAN_FLAGS, "-ffp-contract=off", "-fPIC", "-shared", "-Wall", "-Wextra", "-pthread",
               "-o", tmp, SRC, "-lm"]
    else:
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
               "-Wall", "-Wextra", "-pthread", "-o", tmp, SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build())
