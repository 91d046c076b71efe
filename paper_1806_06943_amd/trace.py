"""roctx ranges for profilers (rocprofv3 --marker-trace shows them on the host
timeline): ``with trace.range("adjoint window 3"): ...``.

Uses the ROCm profiler SDK's roctx library (or the older libroctx64) through
ctypes; without either, or with LBM_ROCTX=0, every range is a no-op.
"""
from __future__ import annotations

import contextlib
import ctypes
import os

_lib = None
_tried = False


def _load():
    global _lib, _tried
    if _tried:
        return _lib
    _tried = True
    if os.environ.get("LBM_ROCTX", "1") == "0":
        return None
    root = os.environ.get("ROCM_PATH", "/opt/rocm")
    for name in ("librocprofiler-sdk-roctx.so.1", "libroctx64.so.4", "libroctx64.so"):
        try:
            L = ctypes.CDLL(os.path.join(root, "lib", name))
            L.roctxRangePushA.argtypes = [ctypes.c_char_p]
            L.roctxRangePushA.restype = ctypes.c_int
            L.roctxRangePop.restype = ctypes.c_int
            _lib = L
            break
        except OSError:
            continue
    return _lib


def push(name: str) -> None:
    L = _load()
    if L is not None:
        L.roctxRangePushA(name.encode())


def pop() -> None:
    L = _load()
    if L is not None:
        L.roctxRangePop()


@contextlib.contextmanager
def range(name: str):  # noqa: A001 - the profiler's own term
    push(name)
    try:
        yield
    finally:
        pop()
