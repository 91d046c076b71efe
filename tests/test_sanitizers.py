"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle is built a second time with -fsanitize=address,undefined and the
fast oracle pins (tables, moments, brute force, stepping with and without
walls on small and aliasing lattices, single-node steps, forces, the pressure
tensor, the adjoint) run against that build in a child process with the
sanitizer runtime preloaded.  Any out-of-bounds access, use after free or
undefined arithmetic in the oracle ends the child with a report.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

FAST_PINS = ("tests/test_oracle_pins.py", "tests/test_oracle_pressure_pins.py",
             "tests/test_oracle_shift.py", "tests/test_oracle_adjoint.py")
DESELECT = ("laplace or poiseuille or flat_interface or slab or original or scales "
            "or run_gradient or thirty")


def asan_runtime():
    out = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = out.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_pins_under_address_and_ub_sanitizers(tmp_path):
    rt = asan_runtime()
    if rt is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    sys.path.insert(0, ROOT)
    from oracle import build as B
    so = B.build_sanitized(str(tmp_path / "_lbm_oracle_asan.so"))
    env = dict(os.environ)
    env.update(LBM_ORACLE_SO=so, LD_PRELOAD=rt, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
           "-k", f"not ({DESELECT})", *FAST_PINS]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    log = r.stdout + r.stderr
    assert "AddressSanitizer" not in log and "runtime error:" not in log, log[-4000:]
    assert r.returncode == 0, log[-4000:]
    assert " passed" in log, log[-2000:]


def clang_asan_runtime():
    import glob
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_c_abi_host_code_under_address_and_ub_sanitizers(tmp_path):
    """The HIP library's host code (argument validation, workspace layout, the
    strip planners) built with AddressSanitizer and UndefinedBehaviorSanitizer for
    the host pass only, then the host C-ABI tests against it (no device code runs)."""
    rt = clang_asan_runtime()
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if rt is None or not os.path.exists(hipcc):
        pytest.skip("hipcc or clang's AddressSanitizer runtime is not installed")
    sys.path.insert(0, ROOT)
    from paper_1806_06943_amd import build as HB
    so = str(tmp_path / "liblbm_hip_asan.so")
    host_sanitizers = ["-Xarch_host", "-fsanitize=address",
                       "-Xarch_host", "-fsanitize=undefined",
                       "-Xarch_host", "-fno-sanitize-recover=undefined",
                       "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = [f for f in HB.FLAGS if f != "-O3"] + ["-O1", "-g"] + host_sanitizers
    srcs = [os.path.join(HB.CSRC, s) for s in HB.SOURCES]
    subprocess.run([hipcc] + flags + srcs + ["-o", so], check=True, capture_output=True)
    env = dict(os.environ)
    env.update(LBM_HIP_SO=so, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
           "tests/test_capi_host.py"]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    log = r.stdout + r.stderr
    assert "AddressSanitizer" not in log and "runtime error:" not in log, log[-4000:]
    assert r.returncode == 0 and " passed" in log, log[-4000:]
