"""The CPU timing baseline (edge-parallel FP64 atomic adds on all host threads) computes
the oracle's Z: every row within 1e-12 relative (FP64 sums in another order), integer
class counts exact, and the same errors (CPU only)."""
import numpy as np
import pytest

import cpu_baseline
import gen
import oracle
from gpu_util import random_labels, random_multigraph, row_rel_err


@pytest.mark.parametrize("weighted,lap", [(False, False), (True, False), (True, True), (False, True)])
def test_matches_oracle(weighted, lap):
    rng = np.random.default_rng(5)
    n, s, K = 3000, 40_000, 9
    src, dst, w = random_multigraph(rng, n, s, weighted)
    Y = random_labels(rng, n, K)
    Zo = oracle.embed(n, src, dst, w, Y, K, laplacian=lap)
    for threads in (1, 4):
        Zc = cpu_baseline.embed_atomic(n, src, dst, w, Y, K, laplacian=lap, threads=threads)
        assert row_rel_err(Zc, Zo) <= 1e-12


def test_rmat_hubs_match_oracle():
    g = gen.rmat(12, 60_000, 3)
    rng = np.random.default_rng(6)
    Y = random_labels(rng, g.n, 50, unknown=0.01)
    Zo = oracle.embed(g.n, g.src, g.dst, None, Y, 50)
    Zc = cpu_baseline.embed_atomic(g.n, g.src, g.dst, None, Y, 50, threads=4)
    assert row_rel_err(Zc, Zo) <= 1e-12


def test_errors():
    n, K = 10, 3
    src = np.array([0, 1, 2], np.int32)
    dst = np.array([1, 2, 3], np.int32)
    Y = np.array([1, 2, 3, 0, 1, 2, 3, 0, 1, 2], np.int32)
    with pytest.raises(RuntimeError, match="-2"):
        cpu_baseline.embed_atomic(n, src, dst, None, np.where(Y == 3, 4, Y), K)
    with pytest.raises(RuntimeError, match="-3"):
        cpu_baseline.embed_atomic(n, src, np.array([1, 2, 10], np.int32), None, Y, K)
    with pytest.raises(RuntimeError, match="-4"):
        cpu_baseline.embed_atomic(n, src, dst, np.array([1, -1, 1], np.float32), Y, K, laplacian=True)
