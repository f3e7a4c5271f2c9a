"""Seeded synthetic graphs and label vectors for GEE (one-hot graph encoder embedding).

The edge lists and labels written here feed both the FP64 oracle and the GPU path;
this package contains none of the embedding's arithmetic. Every generator is a pure
function of its seed (counter-based SplitMix64 streams), so any run regenerates
byte-identical inputs regardless of thread count.

Workload recipes (the paper's graphs are public datasets that are not available
here; these synthetic graphs stand in with comparable shapes):

* ``sbm_small``  — SBM n=10,000, 5 equal blocks, p_in=0.05, p_out=0.005, unit
  weights, labels = block+1 with exactly 1,000 (10%) set to 0, K=5.
* ``er_weighted`` — Erdős–Rényi G(n, m), n=2^22, m=2^26 records, weights on the
  2^-24 grid in (0, 1], labels uniform over 1..50 with exactly 5% set to 0
  (the paper's weak-scaling family, Section IV / Fig. 4).
* ``rmat_paper_scale`` — R-MAT (0.57, 0.19, 0.19, 0.05), scale 27, edge factor 14
  (1,879,048,192 records, about Friendster's 1.8B edges of Table I), unit weights,
  ids scrambled by a seeded bijection, labels 1 + hash mod 50 with 1% set to 0.
* ``rmat_batched`` — R-MAT scale 24, edge factor 16 (268,435,456 records), unit
  weights, and 64 label vectors on it: K_b = floor(exp(U[ln 2, ln 257))) in
  [2, 256], unknown fraction f_b ~ U[0, 0.5) (Bernoulli per vertex), even b the
  adjacency version and odd b the Laplacian version (many label vectors sharing
  one graph: labels from ground truth or from clusterings, Section II).

The paper's label protocol (Section IV) draws labels uniformly at random; here the
class of a labelled vertex is uniform over 1..K and a fixed fraction is unknown (0).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gee_gen.c")
_LIB = os.path.join(_HERE, "libgeegen.so")
_lib = None

I32P = ctypes.POINTER(ctypes.c_int32)
F32P = ctypes.POINTER(ctypes.c_float)


def build(force: bool = True) -> str:
    """Compile the generator library with gcc (OpenMP, -O2)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        i64, u64, f64, i32 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_int32
        lib.gen_rng_at.restype = u64
        lib.gen_rng_at.argtypes = [u64, u64, u64]
        lib.gen_scramble.restype = u64
        lib.gen_scramble.argtypes = [ctypes.c_int, u64, u64]
        lib.gen_er.restype = None
        lib.gen_er.argtypes = [i64, i64, u64, I32P, I32P, F32P]
        lib.gen_grid_weights.restype = None
        lib.gen_grid_weights.argtypes = [i64, u64, F32P]
        lib.gen_rmat.restype = None
        lib.gen_rmat.argtypes = [ctypes.c_int, i64, f64, f64, f64, u64, ctypes.c_int, I32P, I32P]
        lib.gen_sbm.restype = i64
        lib.gen_sbm.argtypes = [i64, i64, f64, f64, u64, i64, I32P, I32P]
        lib.gen_sbm_records.restype = None
        lib.gen_sbm_records.argtypes = [i64, i64, f64, i64, u64, I32P, I32P]
        lib.gen_labels_uniform.restype = None
        lib.gen_labels_uniform.argtypes = [i64, i32, u64, I32P]
        lib.gen_unlabel_exact.restype = ctypes.c_int
        lib.gen_unlabel_exact.argtypes = [i64, i64, u64, I32P]
        lib.gen_unlabel_bernoulli.restype = None
        lib.gen_unlabel_bernoulli.argtypes = [i64, f64, u64, I32P]
        lib.gen_shuffle_records.restype = None
        lib.gen_shuffle_records.argtypes = [i64, u64, I32P, I32P, F32P]
        _lib = lib
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t) if a is not None else None


@dataclass
class Graph:
    """An edge list of s records (src[i], dst[i], w[i]) over vertices [0, n).

    ``w is None`` means unit weights. Arrays are contiguous int32 / float32."""

    n: int
    src: np.ndarray
    dst: np.ndarray
    w: np.ndarray | None = None

    @property
    def s(self) -> int:
        return int(self.src.shape[0])


def rng_at(seed: int, stream: int, ctr: int) -> int:
    return int(_load().gen_rng_at(seed, stream, ctr))


def er(n: int, s: int, seed: int, weighted: bool) -> Graph:
    src = np.empty(s, np.int32)
    dst = np.empty(s, np.int32)
    w = np.empty(s, np.float32) if weighted else None
    _load().gen_er(n, s, seed, _p(src, I32P), _p(dst, I32P), _p(w, F32P))
    return Graph(n, src, dst, w)


def grid_weights(s: int, seed: int) -> np.ndarray:
    w = np.empty(s, np.float32)
    _load().gen_grid_weights(s, seed, _p(w, F32P))
    return w


def rmat(scale: int, s: int, seed: int, a=0.57, b=0.19, c=0.19, scramble: bool = True) -> Graph:
    src = np.empty(s, np.int32)
    dst = np.empty(s, np.int32)
    _load().gen_rmat(scale, s, a, b, c, seed, 1 if scramble else 0, _p(src, I32P), _p(dst, I32P))
    return Graph(1 << scale, src, dst, None)


def scramble(scale: int, seed: int, v: int) -> int:
    return int(_load().gen_scramble(scale, seed, v))


def sbm(n: int, nb: int, p_in: float, p_out: float, seed: int) -> Graph:
    exp = 0.5 * n * n * max(p_in, p_out)
    cap = int(exp * 1.2 + 1024)
    src = np.empty(cap, np.int32)
    dst = np.empty(cap, np.int32)
    s = _load().gen_sbm(n, nb, p_in, p_out, seed, cap, _p(src, I32P), _p(dst, I32P))
    if s < 0:
        raise RuntimeError("sbm: record count exceeded capacity")
    return Graph(n, src[:s].copy(), dst[:s].copy(), None)


def sbm_records(n: int, nb: int, ratio: float, s: int, seed: int) -> Graph:
    """SBM with nb equal blocks by record sampling: s records, density inside blocks
    ratio times the density between them (repeats possible)."""
    sizes = np.diff((np.arange(nb + 1, dtype=np.int64) * n + nb - 1) // nb)
    W = float((sizes * (sizes - 1) // 2).sum())
    B = n * (n - 1) / 2 - W
    p_within = ratio * W / (ratio * W + B) if (ratio * W + B) > 0 else 1.0
    src = np.empty(s, np.int32)
    dst = np.empty(s, np.int32)
    _load().gen_sbm_records(n, nb, p_within, s, seed, _p(src, I32P), _p(dst, I32P))
    return Graph(n, src, dst, None)


def labels_uniform(n: int, K: int, seed: int) -> np.ndarray:
    Y = np.empty(n, np.int32)
    _load().gen_labels_uniform(n, K, seed, _p(Y, I32P))
    return Y


def unlabel_exact(Y: np.ndarray, m: int, seed: int) -> np.ndarray:
    if _load().gen_unlabel_exact(Y.shape[0], m, seed, _p(Y, I32P)) != 0:
        raise ValueError("unlabel_exact: bad count")
    return Y


def unlabel_bernoulli(Y: np.ndarray, f: float, seed: int) -> np.ndarray:
    _load().gen_unlabel_bernoulli(Y.shape[0], f, seed, _p(Y, I32P))
    return Y


def shuffle_records(g: Graph, seed: int) -> Graph:
    src, dst = g.src.copy(), g.dst.copy()
    w = g.w.copy() if g.w is not None else None
    _load().gen_shuffle_records(g.s, seed, _p(src, I32P), _p(dst, I32P), _p(w, F32P))
    return Graph(g.n, src, dst, w)


# ----------------------------------------------------------------- recipes ----

@dataclass
class Workload:
    name: str
    graph: Graph
    labels: np.ndarray
    K: int


def sbm_small(seed: int = 1) -> Workload:
    """SBM n=10,000, five blocks of 2,000, p_in 0.05, p_out 0.005, K=5, 10% unknown."""
    n, nb = 10_000, 5
    g = sbm(n, nb, 0.05, 0.005, seed)
    Y = (np.arange(n, dtype=np.int64) * nb // n + 1).astype(np.int32)
    unlabel_exact(Y, n // 10, seed)
    return Workload("sbm-n10000-K5", g, Y, 5)


def er_weighted(seed: int = 2, log2n: int = 22, log2s: int = 26, K: int = 50) -> Workload:
    """Erdős–Rényi n=2^log2n, s=2^log2s, grid weights in (0,1], K uniform classes, 5% unknown."""
    n, s = 1 << log2n, 1 << log2s
    g = er(n, s, seed, weighted=True)
    Y = labels_uniform(n, K, seed)
    unlabel_exact(Y, (5 * n) // 100, seed)
    return Workload(f"er-n2^{log2n}-s2^{log2s}-K{K}-weighted", g, Y, K)


def er_unit(seed: int = 2, log2n: int = 22, log2s: int = 26, K: int = 50) -> Workload:
    """Erdős–Rényi n=2^log2n, s=2^log2s, unit weights, K uniform classes, 5% unknown."""
    n, s = 1 << log2n, 1 << log2s
    g = er(n, s, seed, weighted=False)
    Y = labels_uniform(n, K, seed)
    unlabel_exact(Y, (5 * n) // 100, seed)
    return Workload(f"er-n2^{log2n}-s2^{log2s}-K{K}-unit", g, Y, K)


def rmat_paper_scale(seed: int = 3, scale: int = 27, edge_factor: int = 14, K: int = 50,
                     unlabeled: float = 0.01) -> Workload:
    """R-MAT (0.57,0.19,0.19,0.05), 2^scale vertices, edge_factor*2^scale records, unit weights."""
    n = 1 << scale
    g = rmat(scale, edge_factor * n, seed)
    Y = labels_uniform(n, K, seed)
    unlabel_bernoulli(Y, unlabeled, seed)
    return Workload(f"rmat-s{scale}-ef{edge_factor}-K{K}", g, Y, K)


BATCH_PARAM_STREAM = 13  # counter stream of the per-vector (K_b, f_b) draws


def _unit(seed: int, stream: int, ctr: int) -> float:
    return (rng_at(seed, stream, ctr) >> 11) * 2.0 ** -53


def batch_params(B: int, seed: int, k_lo: int = 2, k_hi: int = 256):
    """Per-vector (K_b, f_b, laplacian_b): K log-uniform on [k_lo, k_hi], f ~ U[0, 0.5), odd b Laplacian."""
    Ks, fs, laps = [], [], []
    lo, hi = np.log(k_lo), np.log(k_hi + 1)
    for b in range(B):
        K = int(np.floor(np.exp(lo + _unit(seed, BATCH_PARAM_STREAM, 2 * b) * (hi - lo))))
        Ks.append(min(max(K, k_lo), k_hi))
        fs.append(0.5 * _unit(seed, BATCH_PARAM_STREAM, 2 * b + 1))
        laps.append(b % 2 == 1)
    return Ks, fs, laps


@dataclass
class BatchWorkload:
    name: str
    graph: Graph
    labels: np.ndarray  # [B, n] int32
    Ks: list
    fs: list
    laps: list


def batch_labels(n: int, Ks, fs, seed: int) -> np.ndarray:
    Y = np.empty((len(Ks), n), np.int32)
    for b, (K, f) in enumerate(zip(Ks, fs)):
        sb = seed * 1_000_003 + b
        Y[b] = labels_uniform(n, K, sb)
        unlabel_bernoulli(Y[b], f, sb)
    return Y


def rmat_batched(seed: int = 4, scale: int = 24, edge_factor: int = 16, B: int = 64) -> BatchWorkload:
    """R-MAT (0.57,0.19,0.19,0.05) 2^scale vertices, edge_factor*2^scale records; B label vectors."""
    n = 1 << scale
    g = rmat(scale, edge_factor * n, seed)
    Ks, fs, laps = batch_params(B, seed)
    return BatchWorkload(f"rmat-s{scale}-ef{edge_factor}-B{B}", g, batch_labels(n, Ks, fs, seed), Ks, fs, laps)


# ----------------------------------------------------------- serving mix ----

SERVE_STREAM = 17  # counter stream of the serving mix draws


def _normal(seed: int, stream: int, ctr: int) -> float:
    u1 = max(_unit(seed, stream, 2 * ctr), 2.0 ** -53)
    u2 = _unit(seed, stream, 2 * ctr + 1)
    return float(np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2))


@dataclass
class PoolGraph:
    gid: int
    kind: str  # "sbm" or "rmat"
    n: int
    s: int
    seed: int

    def make(self) -> Graph:
        if self.kind == "sbm":
            return sbm_records(self.n, 10, 10.0, self.s, self.seed)
        return rmat(int(self.n).bit_length() - 1, self.s, self.seed)


@dataclass
class Job:
    jid: int
    gid: int
    Ks: list
    fs: list
    laplacian: bool
    seed: int

    def labels(self, n: int) -> np.ndarray:
        return batch_labels(n, self.Ks, self.fs, self.seed)


def serve_pool(seed: int = 5, graphs: int = 100, mu: float = 12.32, sigma: float = 1.80,
               s_min: int = 1_000, s_max: int = 50_000_000):
    """Graphs of uneven size: s ~ log-normal(mu, sigma) truncated to [s_min, s_max]; even ids
    SBM (10 blocks, inside/between density 10, mean degree 16: n = s / 8), odd ids R-MAT
    (edge factor 16: n = the power of two nearest s / 16)."""
    pool = []
    for g in range(graphs):
        x = int(round(np.exp(mu + sigma * _normal(seed, SERVE_STREAM, g))))
        s = min(max(x, s_min), s_max)
        if g % 2 == 0:
            pool.append(PoolGraph(g, "sbm", max(s // 8, 16), s, seed * 1_000 + g))
        else:
            scale = max(int(round(np.log2(max(s / 16, 2)))), 4)
            pool.append(PoolGraph(g, "rmat", 1 << scale, s, seed * 1_000 + g))
    return pool


def serve_jobs(pool, seed: int = 6, jobs: int = 2000, zipf: float = 1.1, k_lo: int = 2, k_hi: int = 128):
    """Jobs on the pool: graph by Zipf(zipf) over the pool ids (id 0 most popular), 1..8
    vectors, K log-uniform on [k_lo, k_hi], unknown fraction U[0, 0.5), version
    Bernoulli(1/2) per job."""
    w = 1.0 / np.arange(1, len(pool) + 1, dtype=np.float64) ** zipf
    cdf = np.cumsum(w / w.sum())
    out = []
    lo, hi = np.log(k_lo), np.log(k_hi + 1)
    for j in range(jobs):
        g = int(np.searchsorted(cdf, _unit(seed, SERVE_STREAM + 1, 4 * j), side="right"))
        g = min(g, len(pool) - 1)
        B = 1 + int(_unit(seed, SERVE_STREAM + 1, 4 * j + 1) * 8)
        lap = _unit(seed, SERVE_STREAM + 1, 4 * j + 2) < 0.5
        Ks, fs = [], []
        for b in range(B):
            c = (j * 8 + b) * 2
            Ks.append(min(max(int(np.floor(np.exp(lo + _unit(seed, SERVE_STREAM + 2, c) * (hi - lo)))), k_lo), k_hi))
            fs.append(0.5 * _unit(seed, SERVE_STREAM + 2, c + 1))
        out.append(Job(j, g, Ks, fs, lap, seed * 1_000_003 + j))
    return out


def poisson_arrivals(rate: float, jobs: int, seed: int = 7) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate."""
    gaps = np.array([-np.log(max(1.0 - _unit(seed, SERVE_STREAM + 3, j), 2.0 ** -53)) / rate for j in range(jobs)])
    return np.cumsum(gaps)
