"""Edge-parallel FP64 GEE on the host's cores: the CPU timing baseline.

TIMING BASELINE ONLY: ``bench.py`` times it beside the GPU path and the FP64 oracle, and
``tests/test_cpu_baseline.py`` checks it against the oracle. It is neither the oracle (it
shares no code with it) nor part of the GPU library. It follows the paper's parallel
design (Section III): records in parallel, lock-free atomic adds into Z.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gee_cpu.c")
_LIB = os.path.join(_HERE, "libgeecpu.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile with gcc: -O3 -fopenmp, no fast-math."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared",
                               "-std=c11", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        vp, i64, i32, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int
        lib.cpu_zero.restype = None
        lib.cpu_zero.argtypes = [vp, i64, ci]
        lib.cpu_embed_atomic.restype = ci
        lib.cpu_embed_atomic.argtypes = [i64, i64, vp, vp, vp, vp, i32, ci, vp, ci]
        _lib = lib
    return _lib


def host_threads() -> int:
    """Threads for the baseline: the CPUs this process may run on, capped by OMP_NUM_THREADS."""
    n = len(os.sched_getaffinity(0))
    cap = os.environ.get("OMP_NUM_THREADS", "")
    if cap.isdigit() and int(cap) > 0:
        n = min(n, int(cap))
    return max(1, n)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def zeros(n: int, K: int, threads: int) -> np.ndarray:
    """An n x K FP64 array, zeroed by the threads (its pages are brought in here)."""
    Z = np.empty((n, K), np.float64)
    _load().cpu_zero(Z.ctypes.data, Z.size, threads)
    return Z


def embed_atomic(n: int, src, dst, w, Y, K: int, laplacian: bool = False, threads: int | None = None,
                 Z: np.ndarray | None = None) -> np.ndarray:
    """Z (n x K, FP64) by the edge-parallel atomic pass. A given Z must be zero."""
    threads = threads or host_threads()
    src = np.ascontiguousarray(src, np.int32)
    dst = np.ascontiguousarray(dst, np.int32)
    w = None if w is None else np.ascontiguousarray(w, np.float32)
    Y = np.ascontiguousarray(Y, np.int32)
    if Z is None:
        Z = zeros(n, K, threads)
    assert Z.dtype == np.float64 and Z.flags.c_contiguous and Z.size == n * K
    rc = _load().cpu_embed_atomic(n, src.shape[0], src.ctypes.data, dst.ctypes.data,
                                  None if w is None else w.ctypes.data, Y.ctypes.data, K, 1 if laplacian else 0,
                                  Z.ctypes.data, threads)
    if rc != 0:
        raise RuntimeError(f"cpu_embed_atomic failed ({rc})")
    return Z
