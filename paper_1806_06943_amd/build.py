"""Compile the HIP library ``liblbm_hip.so`` for gfx950 with hipcc (in-tree)."""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
TARGET = os.path.join(PKG, "liblbm_hip.so")
SOURCES = ["lbm_kernels.hip", "lbm_adjoint.hip", "lbm_pressure.hip", "lbm_capi.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # contraction only within one source expression: every template instance
    # of a kernel rounds the same way (strip shapes give bitwise equal results)
    "-ffp-contract=on",
    # packed FP32 instructions are kept out of every code object
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
]


# the checked build: the fused step counts out-of-range LDS indices
# (lbm_lds_checks); load it with LBM_HIP_SO
CHECKED = os.path.join(PKG, "liblbm_hip_check.so")


def build(verbose: bool = False, checked: bool = True) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    for target, extra in ((TARGET, []), (CHECKED, ["-DLBM_CHECK_LDS"])):
        if extra and not checked:
            continue
        tmp = target + ".tmp"
        cmd = [HIPCC] + FLAGS + extra + srcs + ["-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(tmp, target)
    return TARGET


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
