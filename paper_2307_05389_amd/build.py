"""Build libtsds.so (all HIP kernels + the C ABI) for gfx950 with hipcc.

Every translation unit is compiled separately (``-ffp-contract=off`` so that
no multiply-add is fused anywhere, packed FP32 instructions disabled) and the
objects are linked into ``paper_2307_05389_amd/libtsds.so`` in place.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libtsds.so")

SOURCES = ["scan.hip", "select.hip", "window.hip", "pick.hip", "nan.hip", "lttb.hip", "api.cpp", "batch.hip",
           "batch_lttb.hip", "api_batch.cpp", "noalloc.hip"]
EXTRA_SOURCES = ["serve.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("TSDS_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-I", INCLUDE, "-I", CSRC,
    "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
]


def _sources():
    srcs = list(SOURCES)
    for s in EXTRA_SOURCES:
        if os.path.exists(os.path.join(CSRC, s)):
            srcs.append(s)
    return srcs


# The argmin/argmax scan compares values only and y holds no NaN by contract,
# so its unit drops IEEE-mode NaN quieting in front of every min/max.
PER_FILE = {"scan.hip": ["-fno-honor-nans", "-mno-amdgpu-ieee"],
            "select.hip": ["-fno-honor-nans", "-mno-amdgpu-ieee"],
            "batch.hip": ["-fno-honor-nans", "-mno-amdgpu-ieee"]}


# ASan/UBSan on the host code only (argument checks, planning, scheduler):
# every flag is handed to the host pass, the device code is built as usual.
LIB_SAN = os.path.join(HERE, "libtsds_san.so")
HOST_SAN = ("-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined "
            "-Xarch_host -fno-sanitize-recover=undefined -Xarch_host -shared-libsan "
            "-Xarch_host -fno-omit-frame-pointer").split()


def _compile(src, sanitize=False):
    obj = os.path.join(BUILD, os.path.basename(src) + (".san.o" if sanitize else ".o"))
    cmd = [HIPCC, "-x", "hip", *FLAGS, *PER_FILE.get(src, []), *(HOST_SAN if sanitize else []), "-c",
           os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj, r.stderr


def build(verbose=False, sanitize=None):
    """Build libtsds.so; with sanitize (default: TSDS_SANITIZE=1 in the
    environment) build libtsds_san.so, the same library with ASan/UBSan on its
    host code, for CPU test runs."""
    if sanitize is None:
        sanitize = os.environ.get("TSDS_SANITIZE", "") == "1"
    os.makedirs(BUILD, exist_ok=True)
    srcs = _sources()
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        results = list(ex.map(lambda f: _compile(f, sanitize), srcs))
    if verbose:
        for _, err in results:
            if err.strip():
                print(err, file=sys.stderr)
    lib = LIB_SAN if sanitize else LIB
    tmp = lib + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + [o for o, _ in results] + \
        ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"] + (HOST_SAN if sanitize else [])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True, sanitize="--sanitize" in sys.argv[1:] or None))
