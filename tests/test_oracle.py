"""Pins of the FP64 oracle (CPU only).

The paper prints no embedding values and no worked example, so every pin here is
mathematical: exact rational brute force, hand-worked closed forms, invariants,
special cases that reduce to a library routine, and equivariances. Each is chosen so
that a plausible slip in the oracle (a dropped update, a swapped endpoint, the wrong
class index, a missing self-loop term, a mis-scaled Laplacian) fails at least one.
"""
import itertools
import json
import math
import os
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest

import gen
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def _rand_graph(rng, n, s, weighted=True, self_loops=True):
    src = rng.integers(0, n, s, dtype=np.int32)
    dst = rng.integers(0, n, s, dtype=np.int32)
    if not self_loops:
        keep = src != dst
        src, dst = src[keep], dst[keep]
    w = None
    if weighted:
        w = ((rng.integers(0, 1 << 24, src.size) + 1) * 2.0 ** -24).astype(np.float32)
    return src, dst, w


def _S_times(n, src, dst, w, x):
    """(A + A^T) x from the records, by two weighted histograms."""
    ww = np.ones(src.size) if w is None else w.astype(np.float64)
    return (np.bincount(src, weights=ww * x[dst], minlength=n)
            + np.bincount(dst, weights=ww * x[src], minlength=n))


# ------------------------------------------------------------------ counts, W

def test_counts_match_bincount():
    rng = np.random.default_rng(0)
    for n, K in [(1, 1), (17, 3), (1000, 50), (4096, 255)]:
        Y = rng.integers(0, K + 1, n, dtype=np.int32)
        c = oracle.counts(Y, K)
        assert np.array_equal(c, np.bincount(Y, minlength=K + 1))
        assert c.sum() == n


def test_weights_are_ieee_reciprocals():
    cnt = np.array([7, 1, 3, 0, 5, 1 << 20, 123457], np.int64)
    K = cnt.size - 1
    inv = oracle.weights(cnt, K)
    assert inv[0] == 0.0
    assert inv[3] == 0.0  # empty class
    for k in [1, 2, 4, 5, 6]:
        assert inv[k] == np.float64(1.0) / np.float64(cnt[k])
    # correctly rounded: the exact rational 1/c lies within half an ulp
    for k in [2, 6]:
        exact = Fraction(1, int(cnt[k]))
        assert abs(Fraction(inv[k]) - exact) <= Fraction(np.spacing(inv[k])) / 2


def test_degrees_match_histograms():
    rng = np.random.default_rng(1)
    n = 500
    src, dst, w = _rand_graph(rng, n, 4000)
    d = oracle.degrees(n, src, dst, w)
    ref = np.bincount(src, weights=w, minlength=n) + np.bincount(dst, weights=w, minlength=n)
    assert np.array_equal(d, ref)  # grid weights: every partial sum is exact
    assert d.sum() == 2 * w.astype(np.float64).sum()
    # a self-loop counts twice
    d1 = oracle.degrees(3, np.array([1], np.int32), np.array([1], np.int32), np.array([0.5], np.float32))
    assert d1.tolist() == [0.0, 1.0, 0.0]
    du = oracle.degrees(n, src, dst, None)
    assert np.array_equal(du, np.bincount(src, minlength=n) + np.bincount(dst, minlength=n))


# ------------------------------------------------------- exact brute force

PAIRS4 = list(itertools.combinations(range(4), 2))


def _exact_adjacency(n, edges, Y, K):
    cnt = [sum(1 for y in Y if y == k) for k in range(K + 1)]
    S = [[Fraction(0)] * n for _ in range(n)]
    for u, v in edges:
        S[u][v] += 1
        S[v][u] += 1
    Z = [[Fraction(0)] * K for _ in range(n)]
    for u in range(n):
        for k in range(1, K + 1):
            if cnt[k] == 0:
                continue
            Z[u][k - 1] = sum((S[u][v] for v in range(n) if Y[v] == k), Fraction(0)) / cnt[k]
    return Z


def _exact_laplacian(n, edges, Y, K):
    getcontext().prec = 50
    cnt = [sum(1 for y in Y if y == k) for k in range(K + 1)]
    S = [[0] * n for _ in range(n)]
    for u, v in edges:
        S[u][v] += 1
        S[v][u] += 1
    d = [sum(S[u]) for u in range(n)]
    r = [Decimal(1) / Decimal(x).sqrt() if x > 0 else Decimal(0) for x in d]
    Z = [[Decimal(0)] * K for _ in range(n)]
    for u in range(n):
        for k in range(1, K + 1):
            if cnt[k] == 0:
                continue
            acc = sum((S[u][v] * r[v] for v in range(n) if Y[v] == k), Decimal(0))
            Z[u][k - 1] = r[u] * acc / cnt[k]
    return Z


def test_exact_bruteforce_all_graphs_on_4_vertices():
    """All 64 simple graphs on 4 vertices x all 81 labelings (K=2), both variants."""
    rng = np.random.default_rng(2)
    K, n = 2, 4
    labelings = list(itertools.product(range(K + 1), repeat=n))
    for mask in range(1 << len(PAIRS4)):
        edges = [PAIRS4[b] for b in range(len(PAIRS4)) if mask >> b & 1]
        # store each pair once, with a random orientation
        oriented = [(v, u) if rng.integers(2) else (u, v) for u, v in edges]
        src = np.array([e[0] for e in oriented], np.int32)
        dst = np.array([e[1] for e in oriented], np.int32)
        for Y in labelings:
            Ya = np.array(Y, np.int32)
            Za = oracle.embed(n, src, dst, None, Ya, K)
            exact = _exact_adjacency(n, edges, Y, K)
            for u in range(n):
                for k in range(K):
                    assert abs(Fraction(Za[u, k]) - exact[u][k]) <= Fraction(1, 1 << 50)
            if mask % 4 == 0 or mask == 63:  # Laplacian on a spread of the graphs
                Zl = oracle.embed(n, src, dst, None, Ya, K, laplacian=True)
                exl = _exact_laplacian(n, edges, Y, K)
                for u in range(n):
                    for k in range(K):
                        assert abs(Decimal(float(Zl[u, k])) - exl[u][k]) <= Decimal("1e-15")


# ------------------------------------------------------------- hand-worked

def _golden_cases():
    with open(os.path.join(HERE, "golden", "hand_worked.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _golden_cases(), ids=lambda c: c["name"])
@pytest.mark.parametrize("laplacian", [False, True])
def test_hand_worked_graphs(case, laplacian):
    n, K = case["n"], case["K"]
    e = np.array(case["edges"], np.int32).reshape(-1, 2)
    Y = np.array(case["labels"], np.int32)
    want = np.array([[a / (b * math.sqrt(c)) for a, b, c in row]
                     for row in case["laplacian" if laplacian else "adjacency"]])
    for s_, d_ in [(e[:, 0], e[:, 1]), (e[:, 1], e[:, 0])]:  # both orientations
        Z = oracle.embed(n, s_, d_, None, Y, K, laplacian)
        np.testing.assert_allclose(Z, want, rtol=1e-15, atol=0)


@pytest.mark.parametrize("n", [2, 5, 9])
def test_complete_graph_closed_form(n):
    rng = np.random.default_rng(n)
    K = 3
    Y = rng.integers(0, K + 1, n, dtype=np.int32)
    pairs = np.array(list(itertools.combinations(range(n), 2)), np.int32)
    Z = oracle.embed(n, pairs[:, 0], pairs[:, 1], None, Y, K)
    nk = np.bincount(Y, minlength=K + 1)
    for u in range(n):
        for k in range(1, K + 1):
            want = 0.0 if nk[k] == 0 else (nk[k] - (Y[u] == k)) / nk[k]
            assert Z[u, k - 1] == pytest.approx(want, rel=1e-15, abs=0)
    Zl = oracle.embed(n, pairs[:, 0], pairs[:, 1], None, Y, K, laplacian=True)
    np.testing.assert_allclose(Zl, Z / (n - 1), rtol=1e-14, atol=0)


# ------------------------------------------------------------ invariants

@pytest.mark.parametrize("seed", [3, 4, 5])
def test_row_and_column_sums(seed):
    rng = np.random.default_rng(seed)
    n, K = 300, 7
    src, dst, w = _rand_graph(rng, n, 3000)
    src[:20] = dst[:20]  # self-loops
    src[20:40], dst[20:40] = src[40:60], dst[40:60]  # repeated records
    Y = rng.integers(0, K + 1, n, dtype=np.int32)
    nk = np.bincount(Y, minlength=K + 1)
    inv = np.where(nk > 0, 1.0 / np.maximum(nk, 1), 0.0)
    inv[0] = 0.0
    ell = inv[Y]
    d = np.bincount(src, weights=w, minlength=n) + np.bincount(dst, weights=w, minlength=n)
    Z = oracle.embed(n, src, dst, w, Y, K)
    np.testing.assert_allclose(Z.sum(1), _S_times(n, src, dst, w, ell), rtol=1e-12, atol=1e-12)
    for k in range(1, K + 1):
        want = d[Y == k].sum() / nk[k] if nk[k] else 0.0
        assert Z[:, k - 1].sum() == pytest.approx(want, rel=1e-12)
    # Laplacian: row sums r_u (S (r * ell))_u; column sums weighted by sqrt(d)
    r = np.where(d > 0, 1.0 / np.sqrt(np.where(d > 0, d, 1.0)), 0.0)
    Zl = oracle.embed(n, src, dst, w, Y, K, laplacian=True)
    np.testing.assert_allclose(Zl.sum(1), r * _S_times(n, src, dst, w, r * ell), rtol=1e-12, atol=1e-14)
    for k in range(1, K + 1):
        want = np.sqrt(d[Y == k]).sum() / nk[k] if nk[k] else 0.0
        assert (np.sqrt(d) * Zl[:, k - 1]).sum() == pytest.approx(want, rel=1e-12)


def test_dense_definition_small():
    """Z equals the dense products S M and R S R M on small random multigraphs."""
    rng = np.random.default_rng(6)
    for n, s, K in [(1, 3, 1), (8, 30, 3), (64, 700, 5)]:
        src, dst, w = _rand_graph(rng, n, s)
        Y = rng.integers(0, K + 1, n, dtype=np.int32)
        A = np.zeros((n, n))
        np.add.at(A, (src, dst), w.astype(np.float64))
        S = A + A.T
        nk = np.bincount(Y, minlength=K + 1)
        M = np.zeros((n, K))
        for v in range(n):
            if Y[v] > 0:
                M[v, Y[v] - 1] = 1.0 / nk[Y[v]]
        np.testing.assert_allclose(oracle.embed(n, src, dst, w, Y, K), S @ M, rtol=1e-13, atol=1e-15)
        d = S.sum(1)
        R = np.diag(np.where(d > 0, 1 / np.sqrt(np.where(d > 0, d, 1)), 0))
        np.testing.assert_allclose(oracle.embed(n, src, dst, w, Y, K, True), R @ S @ R @ M,
                                   rtol=1e-13, atol=1e-15)


# -------------------------------------------------------- special cases

def test_all_unknown_labels_give_zero():
    rng = np.random.default_rng(7)
    n = 200
    src, dst, w = _rand_graph(rng, n, 1000)
    Y = np.zeros(n, np.int32)
    assert not oracle.embed(n, src, dst, w, Y, 4).any()
    assert not oracle.embed(n, src, dst, w, Y, 4, laplacian=True).any()


def test_single_class_gives_degree_over_n():
    rng = np.random.default_rng(8)
    n = 150
    src, dst, w = _rand_graph(rng, n, 900)
    Y = np.ones(n, np.int32)
    Z = oracle.embed(n, src, dst, w, Y, 1)
    d = np.bincount(src, weights=w, minlength=n) + np.bincount(dst, weights=w, minlength=n)
    np.testing.assert_allclose(Z[:, 0], d / n, rtol=1e-13)


@pytest.mark.parametrize("n", [3, 10, 101])
def test_regular_graph_laplacian_is_adjacency_over_degree(n):
    rng = np.random.default_rng(n)
    Y = rng.integers(0, 4, n, dtype=np.int32)
    src = np.arange(n, dtype=np.int32)
    dst = ((src + 1) % n).astype(np.int32)  # cycle: 2-regular
    Z = oracle.embed(n, src, dst, None, Y, 3)
    Zl = oracle.embed(n, src, dst, None, Y, 3, laplacian=True)
    np.testing.assert_allclose(Zl, Z / 2, rtol=1e-15, atol=0)


def test_big_star_hub_sum():
    """m = 2^20 + 3 unit leaves of class 2 around a class-1 centre: Z[centre] = [0, 1]."""
    m = (1 << 20) + 3
    src = np.zeros(m, np.int32)
    dst = np.arange(1, m + 1, dtype=np.int32)
    Y = np.full(m + 1, 2, np.int32)
    Y[0] = 1
    Z = oracle.embed(m + 1, src, dst, None, Y, 2)
    assert Z[0, 0] == 0.0 and abs(Z[0, 1] - 1.0) < 1e-9
    assert np.all(Z[1:, 0] == 1.0) and np.all(Z[1:, 1] == 0.0)
    Zl = oracle.embed(m + 1, src, dst, None, Y, 2, laplacian=True)
    assert abs(Zl[0, 1] - 1 / math.sqrt(m)) < 1e-9 / math.sqrt(m)
    np.testing.assert_allclose(Zl[1:, 0], 1 / math.sqrt(m), rtol=1e-15)


def test_power_of_two_classes_are_exact():
    """Unit weights and n_k = 2^j: every addend is dyadic, so Z is the exact count / n_k."""
    rng = np.random.default_rng(9)
    n, K = 64, 3
    Y = np.zeros(n, np.int32)
    Y[:32], Y[32:48], Y[48:56] = 1, 2, 3  # n_k = 32, 16, 8; 8 unknown
    rng.shuffle(Y)
    src, dst, _ = _rand_graph(rng, n, 2000, weighted=False)
    cnt = np.zeros((n, K + 1), np.int64)
    np.add.at(cnt, (src, Y[dst]), 1)
    np.add.at(cnt, (dst, Y[src]), 1)
    want = cnt[:, 1:] / np.array([32.0, 16.0, 8.0])
    assert np.array_equal(oracle.embed(n, src, dst, None, Y, K), want)


def test_linearity_in_the_edge_set():
    rng = np.random.default_rng(10)
    n, K = 120, 4
    Y = rng.integers(0, K + 1, n, dtype=np.int32)
    s1, d1, w1 = _rand_graph(rng, n, 500)
    s2, d2, w2 = _rand_graph(rng, n, 700)
    Z12 = oracle.embed(n, np.r_[s1, s2], np.r_[d1, d2], np.r_[w1, w2], Y, K)
    np.testing.assert_allclose(Z12, oracle.embed(n, s1, d1, w1, Y, K) + oracle.embed(n, s2, d2, w2, Y, K),
                               rtol=1e-13, atol=1e-15)


def test_equivariances():
    rng = np.random.default_rng(11)
    n, K = 90, 5
    src, dst, w = _rand_graph(rng, n, 800)
    Y = rng.integers(0, K + 1, n, dtype=np.int32)
    for lap in (False, True):
        Z = oracle.embed(n, src, dst, w, Y, K, lap)
        # vertex permutation -> row permutation
        p = rng.permutation(n).astype(np.int32)
        Yp = np.empty_like(Y)
        Yp[p] = Y
        Zp = oracle.embed(n, p[src], p[dst], w, Yp, K, lap)
        np.testing.assert_allclose(Zp[p], Z, rtol=1e-13, atol=1e-15)
        # class permutation -> column permutation
        sigma = np.r_[0, rng.permutation(K) + 1].astype(np.int32)
        Zs = oracle.embed(n, src, dst, w, sigma[Y], K, lap)
        np.testing.assert_allclose(Zs[:, sigma[1:] - 1], Z, rtol=1e-13, atol=1e-15)
        # record order, record orientation, weight split
        q = rng.permutation(src.size)
        np.testing.assert_allclose(oracle.embed(n, src[q], dst[q], w[q], Y, K, lap), Z, rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(oracle.embed(n, dst, src, w, Y, K, lap), Z, rtol=1e-13, atol=1e-15)
        half = (w / 2).astype(np.float32)
        np.testing.assert_allclose(oracle.embed(n, np.r_[src, src], np.r_[dst, dst], np.r_[half, half], Y, K, lap),
                                   Z, rtol=1e-13, atol=1e-15)


def test_unknown_class_update_is_skipped_but_other_side_kept():
    # record (0, 1) with Y(0) = 0: Z(1, .) gets nothing, Z(0, Y(1)) gets 1/n_{Y(1)}
    Z = oracle.embed(2, np.array([0], np.int32), np.array([1], np.int32), None, np.array([0, 1], np.int32), 1)
    assert Z.tolist() == [[1.0], [0.0]]


# ------------------------------------------------------------ sampled rows

def test_embed_rows_equals_full_rows():
    wl = gen.er_weighted(seed=12, log2n=12, log2s=16, K=9)
    g = wl.graph
    rows = np.array([0, 5, 4095, 77, 1234], np.int64)
    for lap in (False, True):
        Z = oracle.embed(g.n, g.src, g.dst, g.w, wl.labels, wl.K, lap)
        Zr = oracle.embed_rows(g.n, g.src, g.dst, g.w, wl.labels, wl.K, lap, rows)
        assert np.array_equal(Zr, Z[rows])


# ------------------------------------------------------------- error paths

def test_error_codes():
    s = np.array([0, 1], np.int32)
    d = np.array([1, 2], np.int32)
    with pytest.raises(oracle.OracleError) as e:
        oracle.embed(3, s, d, None, np.array([0, 1, 3], np.int32), 2)
    assert e.value.code == oracle.ELABEL
    with pytest.raises(oracle.OracleError) as e:
        oracle.embed(3, s, d, None, np.array([0, -1, 1], np.int32), 2)
    assert e.value.code == oracle.ELABEL
    with pytest.raises(oracle.OracleError) as e:
        oracle.embed(2, s, d, None, np.array([0, 1], np.int32), 2)
    assert e.value.code == oracle.EVERTEX
    with pytest.raises(oracle.OracleError) as e:
        oracle.embed(3, s, d, np.array([1.0, -0.5], np.float32), np.array([1, 1, 2], np.int32), 2, True)
    assert e.value.code == oracle.ENEGW
    with pytest.raises(oracle.OracleError) as e:
        oracle.embed(3, s, d, None, np.array([0, 0, 0], np.int32), 0)
    assert e.value.code == oracle.EINVAL
    # negative weights are fine for the adjacency version
    Z = oracle.embed(3, s, d, np.array([1.0, -0.5], np.float32), np.array([1, 1, 2], np.int32), 2)
    assert Z[2, 0] == -0.25  # W(1, 1) * w = (1/2) * (-0.5)


# -------------------------------------------------------------------- CSR

def test_csr_matches_adjacency_lists():
    rng = np.random.default_rng(13)
    for n, s, weighted in [(1, 0, False), (1, 4, True), (6, 25, False), (40, 300, True)]:
        src, dst, w = _rand_graph(rng, n, s, weighted=weighted)
        if weighted:  # force ties in (row, col) with different weights
            src, dst = np.r_[src, src[:3]], np.r_[dst, dst[:3]]
            w = np.r_[w, w[:3][::-1] * 0.5].astype(np.float32)
        row_ptr, col, val = oracle.csr(n, src, dst, w)
        lists = [[] for _ in range(n)]
        for i in range(src.size):
            x = float(w[i]) if w is not None else 1.0
            lists[src[i]].append((int(dst[i]), np.float32(x).view(np.uint32)))
            lists[dst[i]].append((int(src[i]), np.float32(x).view(np.uint32)))
        assert row_ptr[0] == 0 and row_ptr[-1] == 2 * src.size
        for u in range(n):
            got = list(zip(col[row_ptr[u]:row_ptr[u + 1]].tolist(),
                           (val[row_ptr[u]:row_ptr[u + 1]].view(np.uint32).tolist() if val is not None
                            else [np.float32(1.0).view(np.uint32)] * int(row_ptr[u + 1] - row_ptr[u]))))
            assert got == sorted(lists[u])
        q = rng.permutation(src.size)
        r2, c2, v2 = oracle.csr(n, src[q], dst[q], w[q] if w is not None else None)
        assert np.array_equal(r2, row_ptr) and np.array_equal(c2, col)
        if w is not None:
            assert np.array_equal(v2.view(np.uint32), val.view(np.uint32))
