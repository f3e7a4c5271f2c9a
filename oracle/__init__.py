"""FP64 CPU oracle for one-hot graph encoder embedding (GEE).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg are the only users. The GPU library never imports, links or runs
anything here, and the two share no code.

* ``counts / weights / degrees / embed / embed_rows`` wrap ``gee_oracle.c``: plain C,
  FP64, single thread, Algorithm 1 of the paper (Section II) taken step by step.
* ``argmax_labels`` / ``refine``: labels from an embedding (the class of a row's largest
  entry) and the loop that re-embeds with them until they stop changing; NumPy over
  ``embed``.
* ``csr`` builds the symmetric CSR of S = A + A^T with NumPy: row u lists, for every
  record (u, v, w), the entry (v, w) and, for every record (v, u, w), the entry (v, w);
  a self-loop therefore appears twice in its row. Rows are sorted by (column, bit
  pattern of w), which makes the result independent of record order. This is the
  per-vertex edge list that the paper's edge-map walks (Section III).

Every function is pinned by the ``-m "not gpu"`` tests against closed forms, exact
rational brute force, invariants and hand-worked graphs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gee_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

I32P = ctypes.POINTER(ctypes.c_int32)
I64P = ctypes.POINTER(ctypes.c_int64)
F32P = ctypes.POINTER(ctypes.c_float)
F64P = ctypes.POINTER(ctypes.c_double)

OK, EINVAL, ELABEL, EVERTEX, ENEGW, ENOMEM = 0, -1, -2, -3, -4, -8


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle error {code}")
        self.code = code


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: -O2, no fast-math, no OpenMP (single thread)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fPIC",
                               "-shared", "-std=c11", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _bind(lib):
    """Declare the C signatures on a loaded oracle library."""
    i64, i32, ci = ctypes.c_int64, ctypes.c_int32, ctypes.c_int
    lib.oracle_counts.restype = ci
    lib.oracle_counts.argtypes = [i64, I32P, i32, I64P]
    lib.oracle_weights.restype = ci
    lib.oracle_weights.argtypes = [I64P, i32, F64P]
    lib.oracle_degrees.restype = ci
    lib.oracle_degrees.argtypes = [i64, i64, I32P, I32P, F32P, F64P]
    lib.oracle_embed.restype = ci
    lib.oracle_embed.argtypes = [i64, i64, I32P, I32P, F32P, I32P, i32, ci, F64P]
    lib.oracle_embed_rows.restype = ci
    lib.oracle_embed_rows.argtypes = [i64, i64, I32P, I32P, F32P, I32P, i32, ci, i64, I64P, F64P]
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def _c(a, dtype):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=dtype)
    return a


def _p(a, t):
    return a.ctypes.data_as(t) if a is not None else None


def _check(rc):
    if rc != OK:
        raise OracleError(rc)


def counts(Y, K: int) -> np.ndarray:
    """n_k for k = 0..K (int64; index 0 counts unknown labels)."""
    Y = _c(Y, np.int32)
    out = np.zeros(K + 1, np.int64)
    _check(_load().oracle_counts(Y.shape[0], _p(Y, I32P), K, _p(out, I64P)))
    return out


def weights(cnt, K: int) -> np.ndarray:
    """inv[k] = 1/n_k (0 for k = 0 and for empty classes), FP64."""
    cnt = _c(cnt, np.int64)
    out = np.zeros(K + 1, np.float64)
    _check(_load().oracle_weights(_p(cnt, I64P), K, _p(out, F64P)))
    return out


def degrees(n: int, src, dst, w=None) -> np.ndarray:
    src, dst, w = _c(src, np.int32), _c(dst, np.int32), _c(w, np.float32)
    out = np.zeros(n, np.float64)
    _check(_load().oracle_degrees(n, src.shape[0], _p(src, I32P), _p(dst, I32P), _p(w, F32P),
                                  _p(out, F64P)))
    return out


def embed(n: int, src, dst, w, Y, K: int, laplacian: bool = False) -> np.ndarray:
    """Z (n x K, FP64) by Algorithm 1; ``laplacian`` scales each record by (d_u d_v)^-1/2."""
    src, dst, w, Y = _c(src, np.int32), _c(dst, np.int32), _c(w, np.float32), _c(Y, np.int32)
    Z = np.zeros((n, K), np.float64)
    _check(_load().oracle_embed(n, src.shape[0], _p(src, I32P), _p(dst, I32P), _p(w, F32P),
                                _p(Y, I32P), K, 1 if laplacian else 0, _p(Z, F64P)))
    return Z


def embed_rows(n: int, src, dst, w, Y, K: int, laplacian: bool, rows) -> np.ndarray:
    """Rows ``rows`` (distinct ids) of the Z that ``embed`` returns, one streaming pass."""
    src, dst, w, Y = _c(src, np.int32), _c(dst, np.int32), _c(w, np.float32), _c(Y, np.int32)
    rows = _c(rows, np.int64)
    Z = np.zeros((rows.shape[0], K), np.float64)
    _check(_load().oracle_embed_rows(n, src.shape[0], _p(src, I32P), _p(dst, I32P), _p(w, F32P),
                                     _p(Y, I32P), K, 1 if laplacian else 0, rows.shape[0],
                                     _p(rows, I64P), _p(Z, F64P)))
    return Z


def argmax_labels(Z, prev=None):
    """Labels from an embedding: 1 + the first k of row u's largest entry when it is above
    zero, else 0 (each vertex takes the class to which it has the most weight per class
    member; Section II allows labels derived from a clustering). The decision is taken on
    FP32 values, the precision of the library's Z, so that both sides compare the same
    numbers; numpy's argmax returns the first maximum. With prev, also the number of
    labels that differ from it."""
    Zf = np.asarray(Z, dtype=np.float64).astype(np.float32)
    lab = (np.argmax(Zf, axis=1) + 1).astype(np.int32)
    lab[Zf.max(axis=1) <= 0] = 0
    if prev is None:
        return lab
    return lab, int(np.count_nonzero(lab != np.asarray(prev)))


def refine(n: int, src, dst, Y, K: int, max_iter: int = 50):
    """Repeat (embed with the current labels, argmax_labels) until no label changes, until a
    round changes no fewer labels than the round two before it (synchronous updates that
    have settled into a cycle), or max_iter rounds; returns (labels, rounds, changes per
    round). Unit weights, adjacency version."""
    Y = np.asarray(Y, dtype=np.int32).copy()
    history = []
    for _ in range(max_iter):
        Y, ch = argmax_labels(embed(n, src, dst, None, Y, K), Y)
        history.append(ch)
        if ch == 0 or (len(history) >= 3 and history[-1] >= history[-3]):
            break
    return Y, len(history), history


def csr(n: int, src, dst, w=None):
    """Symmetric CSR of S = A + A^T: (row_ptr int64[n+1], col int32[2s], val float32[2s] or None).

    Row u holds (v, w) for each record (u, v, w) and (v, w) for each record (v, u, w);
    entries of a row are sorted by column, then by the bit pattern of w."""
    src = np.asarray(src, np.int64)
    dst = np.asarray(dst, np.int64)
    rows = np.concatenate([src, dst])
    cols = np.concatenate([dst, src])
    if rows.size and (rows.min() < 0 or rows.max() >= n):
        raise OracleError(EVERTEX)
    if w is not None:
        wv = np.concatenate([np.asarray(w, np.float32)] * 2)
        wbits = wv.view(np.uint32)
        order = np.lexsort((wbits, cols, rows))
        val = wv[order]
    else:
        order = np.lexsort((cols, rows))
        val = None
    col = cols[order].astype(np.int32)
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=row_ptr[1:])
    return row_ptr, col, val
