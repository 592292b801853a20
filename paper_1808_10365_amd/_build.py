"""Build step for the HIP library (hipcc, gfx950 only). Always recompiles."""
from __future__ import annotations

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(_HERE)
CSRC = os.path.join(_HERE, "csrc")
LIB = os.path.join(_HERE, "libsk.so")

SOURCES = ["sk_pass_a.hip", "sk_pass_b.hip", "sk_api.hip", "sk_batch.hip", "sk_server.hip", "sk_diag.hip", "sk_mc.hip", "sk_probe.hip", "sk_calib.cpp", "sk_fap.cpp"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # Packed FP32 ops are kept out of the generated code.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    return "hipcc"


def build_library(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    extra = [s for s in sorted(os.listdir(CSRC)) if s.endswith((".hip", ".cpp")) and s not in SOURCES]
    srcs += [os.path.join(CSRC, s) for s in extra]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    env = dict(os.environ)
    subprocess.run(cmd, check=True, env=env)
    os.replace(tmp, LIB)
    return LIB


C_ABI_CHECK_SRC = os.path.join(ROOT, "tests", "c_abi", "sk_c_abi_check.c")
C_ABI_CHECK_BIN = os.path.join(ROOT, "tests", "c_abi", "sk_c_abi_check")


def build_c_abi_check(verbose: bool = False) -> str:
    """Compile the plain C client of the library (gcc; links libsk.so and the
    HIP runtime's C API)."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    tmp = C_ABI_CHECK_BIN + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(rocm, "include"),
           "-I", os.path.join(ROOT, "include"), C_ABI_CHECK_SRC, "-o", tmp,
           "-L", _HERE, "-lsk", "-L", os.path.join(rocm, "lib"), "-lamdhip64",
           "-Wl,-rpath," + _HERE, "-Wl,-rpath,$ORIGIN/../../paper_1808_10365_amd", "-Wl,-rpath," + os.path.join(rocm, "lib")]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, C_ABI_CHECK_BIN)
    return C_ABI_CHECK_BIN
