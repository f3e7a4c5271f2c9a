"""Pins of the oracle's labels-from-embedding step and its refinement loop (CPU)."""
import numpy as np

import oracle


def test_argmax_rule_by_hand():
    Z = np.array([[0, 0, 0], [1, 2, 2], [3, 1, 0], [0, 0.5, 0]], dtype=np.float64)
    assert oracle.argmax_labels(Z).tolist() == [0, 2, 1, 2]  # empty row -> 0, ties -> first
    lab, ch = oracle.argmax_labels(Z, prev=np.array([0, 3, 1, 1]))
    assert lab.tolist() == [0, 2, 1, 2] and ch == 2


def test_argmax_brute_force():
    rng = np.random.default_rng(0)
    Z = rng.integers(0, 4, (500, 7)).astype(np.float64) / rng.integers(1, 9, 7)
    got = oracle.argmax_labels(Z)
    for u in range(Z.shape[0]):
        row = Z[u].astype(np.float32)
        m = max(row)
        want = 0 if m <= 0 else 1 + [k for k in range(7) if row[k] == m][0]
        assert got[u] == want


def test_argmax_decides_in_fp32():
    # 1 and 1 + 1e-12 differ in FP64 but not in FP32: the first class wins
    assert oracle.argmax_labels(np.array([[1.0, 1.0 + 1e-12]])).tolist() == [1]


def _two_cliques():
    A = [(i, j) for i in range(5) for j in range(i + 1, 5)]
    B = [(i + 5, j + 5) for i, j in A]
    e = np.array(A + B + [(4, 5)], dtype=np.int32)
    return 10, e[:, 0].copy(), e[:, 1].copy()


def test_refine_two_cliques():
    n, src, dst = _two_cliques()
    truth = np.array([1] * 5 + [2] * 5, dtype=np.int32)
    # two labels flipped: one round puts every vertex back in its clique, the next changes nothing
    Y0 = truth.copy()
    Y0[0], Y0[9] = 2, 1
    Y, rounds, hist = oracle.refine(n, src, dst, Y0, 2)
    assert Y.tolist() == truth.tolist() and rounds == 2 and hist == [2, 0]
    # the truth is a fixed point
    Y, rounds, hist = oracle.refine(n, src, dst, truth, 2)
    assert Y.tolist() == truth.tolist() and hist == [0]


def test_refine_stops_on_a_cycle():
    """A path of two vertices with swapped labels swaps back and forth forever under
    synchronous updates: the loop stops once a round changes as many labels as the round
    two before it."""
    Y, rounds, hist = oracle.refine(2, np.array([0], np.int32), np.array([1], np.int32),
                                    np.array([1, 2], np.int32), 2)
    assert hist == [2, 2, 2] and rounds == 3 and Y.tolist() == [2, 1]  # three swaps
