"""Build the gfx950 HIP library ``libhj.so`` in-tree with hipcc.

    python -m paper_2012_04011_amd.build
    python -m paper_2012_04011_amd.build --sanitize

``--sanitize`` builds ``libhj_san.so`` instead: the host side compiled with
AddressSanitizer and UndefinedBehaviorSanitizer (clang's runtime, shared),
the device code as usual.  The binding loads it when HJ_SANITIZE=1, with
that runtime preloaded into the process (see ``sanitizer_runtime()``).
"""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhj.so")
LIB_SAN = os.path.join(HERE, "libhj_san.so")
SOURCES = ["hj_kernels.hip", "hj_abi.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    "-Wno-unused-function",
    # keep packed FP32 instructions out of the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


# host-only sanitizers: each -fsanitize= follows -Xarch_host, so the device
# code is built as in the plain library
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-shared-libsan",
             "-Xarch_host", "-fno-omit-frame-pointer", "-g"]


def sanitizer_runtime() -> str:
    """The shared ASan + UBSan runtime the sanitized builds link against
    (to be preloaded into an unsanitized interpreter)."""
    clang = os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "llvm", "bin", "clang")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang"
    return subprocess.check_output([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], text=True).strip()


def build(verbose: bool = False, sanitize: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    out = LIB_SAN if sanitize else LIB
    tmp = out + ".tmp"
    cmd = [HIPCC, *FLAGS, *(SAN_FLAGS if sanitize else []), "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd, cwd=CSRC)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True, sanitize="--sanitize" in sys.argv[1:]))
    sys.exit(0)
