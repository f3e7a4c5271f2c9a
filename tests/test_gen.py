"""Seeded input generators: determinism and the statistics of each recipe (CPU only)."""
import os
import subprocess
import sys

import numpy as np
import pytest

import gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_streams_are_deterministic_and_distinct():
    a = [gen.rng_at(7, 1, i) for i in range(4)]
    assert a == [gen.rng_at(7, 1, i) for i in range(4)]
    assert len(set(a)) == 4
    assert gen.rng_at(7, 2, 0) != a[0] and gen.rng_at(8, 1, 0) != a[0]


def test_sbm_small_recipe():
    wl = gen.sbm_small()
    g = wl.graph
    # E[s] = 5 * C(2000, 2) * 0.05 + 10 * 2000^2 * 0.005 = 699,750; sd about 821
    assert abs(g.s - 699_750) < 5 * 821
    assert np.all(g.src != g.dst)
    lo, hi = np.minimum(g.src, g.dst).astype(np.int64), np.maximum(g.src, g.dst).astype(np.int64)
    assert np.unique(lo * g.n + hi).size == g.s  # each pair stored once
    same = (lo // 2000) == (hi // 2000)
    # within-block share: 0.05*5*C(2000,2) / 699,750 = 0.714
    assert abs(same.mean() - 0.714) < 0.01
    assert (wl.labels == 0).sum() == 1000
    assert wl.K == 5 and wl.labels.max() == 5
    kept = wl.labels > 0
    assert np.all(wl.labels[kept] == np.arange(g.n)[kept] // 2000 + 1)
    again = gen.sbm_small()
    assert np.array_equal(again.graph.src, g.src) and np.array_equal(again.labels, wl.labels)


def test_er_weighted_small():
    wl = gen.er_weighted(seed=2, log2n=14, log2s=18, K=50)
    g = wl.graph
    assert g.s == 1 << 18 and g.n == 1 << 14
    assert g.src.min() >= 0 and g.src.max() < g.n
    assert np.all(g.w > 0) and np.all(g.w <= 1)
    grid = g.w.astype(np.float64) * 2.0 ** 24
    assert np.array_equal(grid, np.round(grid))  # on the 2^-24 grid
    assert (wl.labels == 0).sum() == (5 * g.n) // 100
    assert set(np.unique(wl.labels)) == set(range(51))
    # endpoints roughly uniform
    h = np.bincount(g.src >> 10, minlength=16)
    assert np.all(np.abs(h - g.s / 16) < 6 * np.sqrt(g.s / 16))


def test_rmat_quadrant_frequencies():
    g = gen.rmat(12, 1 << 18, seed=5, scramble=False)
    for level in (11, 5, 0):
        bu = (g.src >> level) & 1
        bv = (g.dst >> level) & 1
        q = np.bincount(bu * 2 + bv, minlength=4) / g.s
        np.testing.assert_allclose(q, [0.57, 0.19, 0.19, 0.05], atol=0.005)


def test_rmat_scramble_is_a_bijection():
    for scale in (1, 7, 16):
        vals = np.array([gen.scramble(scale, 3, v) for v in range(1 << min(scale, 12))])
        assert vals.max() < (1 << scale)
        assert np.unique(vals).size == vals.size
    g0 = gen.rmat(10, 5000, seed=4, scramble=False)
    g1 = gen.rmat(10, 5000, seed=4, scramble=True)
    m = np.array([gen.scramble(10, 4, v) for v in range(1 << 10)])
    assert np.array_equal(m[g0.src], g1.src) and np.array_equal(m[g0.dst], g1.dst)


def test_rmat_recipe_labels():
    wl = gen.rmat_paper_scale(scale=16, edge_factor=14)
    assert wl.graph.s == 14 << 16
    frac0 = (wl.labels == 0).mean()
    assert abs(frac0 - 0.01) < 5 * np.sqrt(0.01 * 0.99 / wl.graph.n)
    assert wl.labels.max() == 50 and wl.labels.min() == 0


def test_output_independent_of_thread_count():
    code = ("import sys; sys.path.insert(0, %r); import gen, hashlib;"
            "g = gen.rmat(14, 200000, 9); w = gen.er(1000, 100000, 9, True);"
            "print(hashlib.sha256(g.src.tobytes() + g.dst.tobytes() + w.w.tobytes()).hexdigest())") % ROOT
    outs = []
    for t in ("1", "3"):
        env = dict(os.environ, OMP_NUM_THREADS=t)
        outs.append(subprocess.check_output([sys.executable, "-c", code], env=env).strip())
    assert outs[0] == outs[1]


def test_serving_mix_recipe():
    """Pool sizes within the truncation, both graph kinds, Zipf-skewed job placement,
    K and vector counts in range, reproducible draws."""
    pool = gen.serve_pool()
    assert len(pool) == 100 and {p.kind for p in pool} == {"sbm", "rmat"}
    assert all(1_000 <= p.s <= 50_000_000 for p in pool)
    jobs = gen.serve_jobs(pool, jobs=500)
    assert all(1 <= len(j.Ks) <= 8 and all(2 <= k <= 128 for k in j.Ks) for j in jobs)
    assert all(0.0 <= f < 0.5 for j in jobs for f in j.fs)
    counts = np.bincount([j.gid for j in jobs], minlength=100)
    assert counts[0] == counts.max() and counts[0] > 3 * counts[10]
    again = gen.serve_jobs(gen.serve_pool(), jobs=500)
    assert [(j.gid, j.Ks, j.laplacian) for j in jobs] == [(j.gid, j.Ks, j.laplacian) for j in again]
    g = gen.sbm_records(10_000, 10, 10.0, 200_000, seed=3)
    blk_u, blk_v = g.src * 10 // 10_000, g.dst * 10 // 10_000
    within = np.mean(blk_u == blk_v)
    assert abs(within - 10 * 0.1 / (10 * 0.1 + 0.9)) < 0.01  # inside/between density ratio 10
    t = gen.poisson_arrivals(100.0, 2000)
    assert np.all(np.diff(t) > 0) and abs(t[-1] / 2000 - 0.01) < 0.001
