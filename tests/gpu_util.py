"""Helpers shared by the GPU tests (imported by test modules; not a test file)."""
import sys

import numpy as np

TOL = 1e-5  # max relative error per row, FP32 Z against the FP64 oracle


def row_rel_err(Zg, Zo) -> float:
    """max_u max_k |Zg - Zo| / max_k |Zo|; a zero oracle row must be exactly zero."""
    Zg = np.asarray(Zg, np.float64)
    Zo = np.asarray(Zo, np.float64)
    den = np.abs(Zo).max(axis=1) if Zo.shape[1] else np.zeros(Zo.shape[0])
    num = np.abs(Zg - Zo).max(axis=1) if Zo.shape[1] else np.zeros(Zo.shape[0])
    zero = den == 0
    if np.any(num[zero] != 0):
        return float("inf")
    if not np.any(~zero):
        return 0.0
    return float((num[~zero] / den[~zero]).max())


def assert_parity(Zg, Zo, tol=TOL, what=""):
    e = row_rel_err(Zg, Zo)
    assert e <= tol, f"{what}: row relative error {e:.3e} > {tol:g}"
    return e


def announce(msg: str):
    print(f"[gpu] {msg}", file=sys.__stderr__, flush=True)


def random_multigraph(rng, n, s, weighted, loops=True):
    src = rng.integers(0, n, s).astype(np.int32)
    dst = rng.integers(0, n, s).astype(np.int32)
    if loops and s >= 8:
        src[: s // 8] = dst[: s // 8]
    if s >= 16:
        src[s // 8: s // 8 + s // 16] = src[: s // 16]
        dst[s // 8: s // 8 + s // 16] = dst[: s // 16]
    w = None
    if weighted:
        w = ((rng.integers(0, 1 << 24, s) + 1) * 2.0 ** -24).astype(np.float32)
    return src, dst, w


def random_labels(rng, n, K, unknown=0.1):
    Y = rng.integers(1, K + 1, n).astype(np.int32)
    Y[rng.random(n) < unknown] = 0
    return Y
