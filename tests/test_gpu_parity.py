"""Parity of the HIP path with the FP64 oracle on the GPU, through the C ABI.

Counts, weights, degrees and the CSR are compared bit for bit; Z within 1e-5 max
relative error per row (zero rows exactly zero); unit-weight adjacency results whose
sums are dyadic are compared bit for bit.
"""
import json
import math
import os

import numpy as np
import pytest
import torch

import gen
import oracle
import paper_2402_04403_amd as gee
from gpu_util import announce, assert_parity, random_labels, random_multigraph, row_rel_err

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]
DEV = torch.device("cuda:0")
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(autouse=True)
def _announce(request):
    announce(request.node.nodeid)
    yield
    torch.cuda.synchronize()


def dev(a, dtype=None):
    t = torch.as_tensor(a)
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV).contiguous()


def run_both_forms(n, src, dst, w, Y, K, lap, seg_lens=(0,), rws=(0,)):
    """Yield (label, Z as numpy) for the push form and every requested pull configuration."""
    coo = gee.to_device(n, src, dst, w, device=DEV)
    labels = dev(Y, torch.int32)
    yield "push", gee.embed(labels, K, coo=coo, laplacian=lap).cpu().numpy()
    csr = gee.csr_build(coo)
    for L in seg_lens:
        for rw in rws:
            Z = gee.embed(labels, K, csr=csr, laplacian=lap, seg_len=L, rows_per_window=rw)
            yield f"pull(L={L},rw={rw})", Z.cpu().numpy()
    hot = gee.csr_build(coo, hot_budget=max(1, n // 10))
    yield "pull(hot)", gee.embed(labels, K, csr=hot, laplacian=lap).cpu().numpy()


# ---------------------------------------------------------------- W, counts --

@pytest.mark.parametrize("K", [1, 5, 50, 255, 256, 4000, 65535])
def test_counts_and_weights_bit_exact(K):
    rng = np.random.default_rng(K)
    n = 100_003
    Y = rng.integers(0, K + 1, n).astype(np.int32)
    c = gee.counts(dev(Y), K)
    want = oracle.counts(Y, K)
    assert np.array_equal(c.cpu().numpy(), want)
    inv = gee.weights(c, K).cpu().numpy()
    assert np.array_equal(inv.view(np.uint64), oracle.weights(want, K).view(np.uint64))


# ------------------------------------------------------------------ degrees --

@pytest.mark.parametrize("weighted", [False, True])
def test_degrees_bit_exact(weighted):
    rng = np.random.default_rng(3)
    n, s = 20_000, 300_001
    src, dst, w = random_multigraph(rng, n, s, weighted)
    want = oracle.degrees(n, src, dst, w)
    coo = gee.to_device(n, src, dst, w, device=DEV)
    d_coo = gee.degrees(coo=coo).cpu().numpy()
    assert np.array_equal(d_coo, want)
    csr = gee.csr_build(coo)
    d_csr = gee.degrees(csr=csr).cpu().numpy()
    assert np.array_equal(d_csr, want)


# ---------------------------------------------------------------------- CSR --

@pytest.mark.parametrize("n,s,weighted", [(1, 0, False), (1, 5, True), (7, 40, False), (5000, 100_003, True),
                                          (300_000, 50_000, False), (4096, 1 << 20, True)])
def test_csr_build_matches_oracle(n, s, weighted):
    rng = np.random.default_rng(n + s)
    src, dst, w = random_multigraph(rng, n, s, weighted)
    if weighted and s > 10:  # repeated (row, col) with different weights: ties broken by w bits
        src[-5:], dst[-5:] = src[:5], dst[:5]
        w[-5:] = w[:5] * np.float32(0.5)
    rp, col, val = oracle.csr(n, src, dst, w)
    csr = gee.csr_build(gee.to_device(n, src, dst, w, device=DEV))
    assert np.array_equal(csr.row_ptr.cpu().numpy(), rp)
    assert np.array_equal(csr.col.cpu().numpy(), col)
    if weighted:
        assert np.array_equal(csr.val.cpu().numpy().view(np.uint32), val.view(np.uint32))


@pytest.mark.parametrize("n,s,weighted", [(1 << 24, 1 << 24, False), (1 << 22, 1 << 23, True)])
def test_csr_build_matches_oracle_large(n, s, weighted):
    """Keys of 44 and 48 bits (more radix passes than the small cases) and scans over
    many blocks."""
    rng = np.random.default_rng(n + s + 1)
    src, dst, w = random_multigraph(rng, n, s, weighted)
    rp, col, val = oracle.csr(n, src, dst, w)
    csr = gee.csr_build(gee.to_device(n, src, dst, w, device=DEV))
    assert np.array_equal(csr.row_ptr.cpu().numpy(), rp)
    assert np.array_equal(csr.col.cpu().numpy(), col)
    if weighted:
        assert np.array_equal(csr.val.cpu().numpy().view(np.uint32), val.view(np.uint32))


def test_csr_build_rmat_skew_large():
    """Scale-21 R-MAT (2^24 records), hot slots on: the plain columns match the oracle."""
    g = gen.rmat(21, 8 << 21, seed=23)
    rp, col, _ = oracle.csr(g.n, g.src, g.dst)
    csr = gee.csr_build(gee.to_device(g.n, g.src, g.dst, device=DEV), hot_budget=1 << 16)
    assert np.array_equal(csr.row_ptr.cpu().numpy(), rp)
    assert np.array_equal(csr.plain_col().cpu().numpy(), col)


def test_csr_build_rmat_skew():
    g = gen.rmat(16, 14 << 16, seed=21)
    rp, col, _ = oracle.csr(g.n, g.src, g.dst)
    csr = gee.csr_build(gee.to_device(g.n, g.src, g.dst, device=DEV))
    assert np.array_equal(csr.row_ptr.cpu().numpy(), rp)
    assert np.array_equal(csr.col.cpu().numpy(), col)


def _expected_hot(rp, H):
    """Top-H vertices in slot order: degree capped at 4095 descending, then id ascending."""
    deg = np.diff(rp)
    bucket = np.minimum(deg, 4095)
    order = np.lexsort((np.arange(deg.size), -bucket))
    return order[:H]


@pytest.mark.parametrize("n,s,weighted,H", [(1, 3, False, 1), (500, 20_000, True, 37), (1 << 14, 1 << 18, False, 1000),
                                            (5000, 100, False, 4999), (300, 4000, False, 300)])
def test_csr_hot_slots(n, s, weighted, H):
    rng = np.random.default_rng(n + H)
    if n == 1 << 14:
        g = gen.rmat(14, s, seed=31)
        src, dst, w = g.src, g.dst, None
    else:
        src, dst, w = random_multigraph(rng, n, s, weighted)
    rp, col, val = oracle.csr(n, src, dst, w)
    csr = gee.csr_build(gee.to_device(n, src, dst, w, device=DEV), hot_budget=H)
    hot_ids = csr.hot_ids.cpu().numpy()
    assert np.array_equal(hot_ids, _expected_hot(rp, min(H, n)))
    assert np.array_equal(csr.row_ptr.cpu().numpy(), rp)
    c = csr.col.cpu().numpy()
    assert np.array_equal(csr.plain_col().cpu().numpy(), col)
    is_hot = np.zeros(n, bool)
    is_hot[hot_ids] = True
    assert np.array_equal(c < 0, is_hot[col])  # exactly the hot columns are encoded
    if weighted:
        assert np.array_equal(csr.val.cpu().numpy().view(np.uint32), val.view(np.uint32))


@pytest.mark.parametrize("lap", [False, True])
@pytest.mark.parametrize("weighted", [False, True])
def test_hot_slots_do_not_change_z(lap, weighted):
    """The gather source is the only difference: Z is bit-identical with and without hot slots."""
    rng = np.random.default_rng(41)
    g = gen.rmat(15, 12 << 15, seed=42)
    w = ((rng.integers(0, 1 << 24, g.s) + 1) * 2.0 ** -24).astype(np.float32) if weighted else None
    Y = random_labels(rng, g.n, 50)
    coo = gee.to_device(g.n, g.src, g.dst, w, device=DEV)
    labels = dev(Y)
    plain = gee.csr_build(coo)
    Zo = oracle.embed(g.n, g.src, g.dst, w, Y, 50, lap)
    for H in (1, 1000, 1 << 14, g.n):
        hot = gee.csr_build(coo, hot_budget=H)
        for L in (0, 256):
            Za = gee.embed(labels, 50, csr=plain, laplacian=lap, seg_len=L)
            Zb = gee.embed(labels, 50, csr=hot, laplacian=lap, seg_len=L)
            assert torch.equal(Za.view(torch.int32), Zb.view(torch.int32)), (H, L)
        assert_parity(Zb.cpu().numpy(), Zo, what=f"hot H={H}")


# -------------------------------------------------------------- hand-worked --

def _golden():
    with open(os.path.join(HERE, "golden", "hand_worked.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _golden(), ids=lambda c: c["name"])
@pytest.mark.parametrize("lap", [False, True])
def test_hand_worked(case, lap):
    e = np.array(case["edges"], np.int32).reshape(-1, 2)
    Y = np.array(case["labels"], np.int32)
    want = np.array([[a / (b * math.sqrt(c)) for a, b, c in row] for row in case["laplacian" if lap else "adjacency"]])
    for name, Z in run_both_forms(case["n"], e[:, 0], e[:, 1], None, Y, case["K"], lap, seg_lens=(0, 64), rws=(0, 1)):
        assert_parity(Z, want, what=f"{case['name']} {name}")


# ---------------------------------------------------------- random graphs --

GRAPHS = [
    # n, s, weighted, K
    (1, 0, False, 1),
    (1, 3, True, 2),
    (17, 0, False, 3),
    (300, 5_000, False, 7),
    (300, 5_000, True, 7),
    (2_000, 65_537, False, 50),
    (2_000, 65_537, True, 50),
    (50_000, 20_011, False, 5),  # mostly isolated vertices
    (3_000, 200_000, False, 300),  # 16-bit labels
    (10_000, 100_000, True, 1000),
]


@pytest.mark.parametrize("n,s,weighted,K", GRAPHS)
@pytest.mark.parametrize("lap", [False, True])
def test_random_graphs(n, s, weighted, K, lap):
    rng = np.random.default_rng(n * 31 + s)
    src, dst, w = random_multigraph(rng, n, s, weighted)
    Y = random_labels(rng, n, K)
    Zo = oracle.embed(n, src, dst, w, Y, K, lap)
    for name, Z in run_both_forms(n, src, dst, w, Y, K, lap, seg_lens=(0, 64, 1000), rws=(0, 3)):
        assert_parity(Z, Zo, what=f"n={n} s={s} w={weighted} K={K} lap={lap} {name}")


@pytest.mark.parametrize("lap", [False, True])
@pytest.mark.parametrize("weighted", [False, True])
def test_hubs_split_across_segments(lap, weighted):
    """A star of 50,000 leaves plus an R-MAT: hub rows span hundreds of segments at L=64."""
    rng = np.random.default_rng(5)
    g = gen.rmat(13, 8 << 13, seed=6)
    m = 50_000
    n = max(g.n, m + 1)
    src = np.r_[g.src, np.zeros(m, np.int32)].astype(np.int32)
    dst = np.r_[g.dst, np.arange(1, m + 1, dtype=np.int32)].astype(np.int32)
    w = ((rng.integers(0, 1 << 24, src.size) + 1) * 2.0 ** -24).astype(np.float32) if weighted else None
    Y = random_labels(rng, n, 11)
    Zo = oracle.embed(n, src, dst, w, Y, 11, lap)
    results = {}
    for name, Z in run_both_forms(n, src, dst, w, Y, 11, lap, seg_lens=(0, 64, 4099), rws=(0, 1, 64)):
        assert_parity(Z, Zo, what=f"hubs lap={lap} w={weighted} {name}")
        results[name] = Z
    if not weighted and not lap:  # exact integer sums: every form and split agrees bit for bit
        ref = results["push"]
        for name, Z in results.items():
            assert np.array_equal(Z.view(np.uint32), ref.view(np.uint32)), name


@pytest.mark.parametrize("seg_len", [0, 64])
def test_negative_weights_pull(seg_len):
    """Adjacency weights of both signs: the pull form's FP32 bins hold only segments without
    a negative weight, the others are summed again in FP64. Half of the rows see only
    positive weights, so both passes run; every row is within the bar, and the result is
    bit-reproducible."""
    rng = np.random.default_rng(21)
    n, s, K = 30_000, 600_000, 17
    src, dst, _ = random_multigraph(rng, n, s, False)
    w = ((rng.integers(0, 1 << 24, s) + 1) * 2.0 ** -24).astype(np.float32)
    neg = (src < n // 2) & (rng.random(s) < 0.3)
    w[neg] = -w[neg]
    hub = np.arange(1, 3001, dtype=np.int32)  # a hub row longer than a segment's FP32 window
    src = np.r_[src, np.full(hub.size, n - 1, np.int32)].astype(np.int32)
    dst = np.r_[dst, hub].astype(np.int32)
    w = np.r_[w, np.linspace(0.25, 1.0, hub.size, dtype=np.float32)].astype(np.float32)
    Y = random_labels(rng, n, K)
    Zo = oracle.embed(n, src, dst, w, Y, K, False)
    csr = gee.csr_build(gee.to_device(n, src, dst, w, device=DEV))
    labels = dev(Y)
    Z1 = gee.embed(labels, K, csr=csr, seg_len=seg_len).cpu().numpy()
    assert_parity(Z1, Zo, what=f"negative weights, seg_len={seg_len}")
    Z2 = gee.embed(labels, K, csr=csr, seg_len=seg_len).cpu().numpy()
    assert np.array_equal(Z1.view(np.uint32), Z2.view(np.uint32))


def test_big_star_exact():
    """m = 2^20 + 3 unit leaves of class 2 around a class-1 centre: Z[centre] = [0, 1] exactly."""
    m = (1 << 20) + 3
    src = np.zeros(m, np.int32)
    dst = np.arange(1, m + 1, dtype=np.int32)
    Y = np.full(m + 1, 2, np.int32)
    Y[0] = 1
    for name, Z in run_both_forms(m + 1, src, dst, None, Y, 2, False, seg_lens=(0, 256)):
        assert Z[0, 0] == 0.0 and Z[0, 1] == 1.0, name
        assert np.all(Z[1:, 0] == 1.0) and np.all(Z[1:, 1] == 0.0), name
    for name, Z in run_both_forms(m + 1, src, dst, None, Y, 2, True, seg_lens=(0, 256)):
        assert abs(Z[0, 1] * math.sqrt(m) - 1.0) < 1e-6, name
        np.testing.assert_allclose(Z[1:, 0], 1 / math.sqrt(m), rtol=1e-6)


def test_power_of_two_classes_bit_equal():
    rng = np.random.default_rng(9)
    n, K = 1 << 14, 4
    Y = np.repeat(np.arange(1, K + 1, dtype=np.int32), n // K)  # n_k = 2^12
    rng.shuffle(Y)
    src, dst, _ = random_multigraph(rng, n, 400_000, False)
    Zo = oracle.embed(n, src, dst, None, Y, K).astype(np.float32)
    for name, Z in run_both_forms(n, src, dst, None, Y, K, False, seg_lens=(0, 128)):
        assert np.array_equal(Z.view(np.uint32), Zo.view(np.uint32)), name


def test_sbm_small_workload():
    wl = gen.sbm_small()
    g = wl.graph
    Zo = oracle.embed(g.n, g.src, g.dst, None, wl.labels, wl.K)
    for name, Z in run_both_forms(g.n, g.src, g.dst, None, wl.labels, wl.K, False):
        assert_parity(Z, Zo, what=name)
        # block structure: a labelled vertex's largest column is its own block (p_in = 10 p_out)
        kept = wl.labels > 0
        assert np.mean(Z[kept].argmax(1) + 1 == wl.labels[kept]) > 0.99


# --------------------------------------------------------------- determinism --

def test_pull_is_bit_reproducible_and_order_independent():
    rng = np.random.default_rng(12)
    wl = gen.er_weighted(seed=12, log2n=16, log2s=21, K=50)
    g = wl.graph
    labels = dev(wl.labels)
    for lap in (False, True):
        csr = gee.csr_build(gee.to_device(g.n, g.src, g.dst, g.w, device=DEV))
        Zs = [gee.embed(labels, 50, csr=csr, laplacian=lap, seg_len=512).cpu().numpy() for _ in range(3)]
        for Z in Zs[1:]:
            assert np.array_equal(Z.view(np.uint32), Zs[0].view(np.uint32))
        sh = gen.shuffle_records(g, seed=99)
        flip = rng.random(sh.s) < 0.5
        s2 = np.where(flip, sh.dst, sh.src).astype(np.int32)
        d2 = np.where(flip, sh.src, sh.dst).astype(np.int32)
        csr2 = gee.csr_build(gee.to_device(g.n, s2, d2, sh.w, device=DEV))
        assert torch.equal(csr2.col, csr.col) and torch.equal(csr2.row_ptr, csr.row_ptr)
        assert torch.equal(csr2.val.view(torch.int32), csr.val.view(torch.int32))
        Z2 = gee.embed(labels, 50, csr=csr2, laplacian=lap, seg_len=512).cpu().numpy()
        assert np.array_equal(Z2.view(np.uint32), Zs[0].view(np.uint32))


def test_push_unit_adjacency_is_reproducible():
    g = gen.rmat(15, 10 << 15, seed=13)
    Y = random_labels(np.random.default_rng(13), g.n, 20)
    coo = gee.to_device(g.n, g.src, g.dst, device=DEV)
    labels = dev(Y)
    Z1 = gee.embed(labels, 20, coo=coo)
    Z2 = gee.embed(labels, 20, coo=coo)
    assert torch.equal(Z1.view(torch.int32), Z2.view(torch.int32))


# ---------------------------------------------------------------- errors --

def _err_code(fn):
    with pytest.raises(gee.GeeError) as e:
        fn()
    return e.value.code


def test_data_errors_are_reported():
    n = 100
    src = np.arange(0, 99, dtype=np.int32)
    dst = np.arange(1, 100, dtype=np.int32)
    Y = np.ones(n, np.int32)
    coo = gee.to_device(n, src, dst, device=DEV)
    bad_labels = Y.copy()
    bad_labels[7] = 6
    assert _err_code(lambda: gee.embed(dev(bad_labels), 5, coo=coo)) == gee.GEE_ELABEL
    bad_labels[7] = -1
    assert _err_code(lambda: gee.counts(dev(bad_labels), 5)) == gee.GEE_ELABEL
    bad = gee.to_device(n, np.r_[src, 100], np.r_[dst, 0], device=DEV)
    assert _err_code(lambda: gee.embed(dev(Y), 5, coo=bad)) == gee.GEE_EVERTEX
    assert _err_code(lambda: gee.csr_build(bad)) == gee.GEE_EVERTEX
    neg = gee.to_device(n, src, dst, np.r_[np.ones(98, np.float32), -1.0], device=DEV)
    assert _err_code(lambda: gee.embed(dev(Y), 5, coo=neg, laplacian=True)) == gee.GEE_ENEGW
    csr = gee.csr_build(neg)
    assert _err_code(lambda: gee.embed(dev(Y), 5, csr=csr, laplacian=True)) == gee.GEE_ENEGW
    gee.embed(dev(Y), 5, csr=csr, laplacian=False)  # negative weights are fine for adjacency
    # a CSR column outside [0, n) is reported by the pull kernel
    col = csr.col.clone()
    col[3] = n + 5
    bad_csr = gee.DeviceCsr(n, csr.row_ptr, col, csr.val)
    assert _err_code(lambda: gee.embed(dev(Y), 5, csr=bad_csr)) == gee.GEE_EVERTEX


# ------------------------------------------------------------------ plumbing --

def test_hot_kernel_events_and_streams():
    wl = gen.er_weighted(seed=14, log2n=15, log2s=19, K=16)
    g = wl.graph
    coo = gee.to_device(g.n, g.src, g.dst, g.w, device=DEV)
    csr = gee.csr_build(coo)
    labels = dev(wl.labels)
    ev = (gee.HipEvent(), gee.HipEvent())
    Z = gee.embed(labels, 16, csr=csr, events=ev)
    ev[1].synchronize()
    assert ev[0].elapsed_ms(ev[1]) > 0.0
    ref = Z.clone()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s1):
        Za = gee.embed(labels, 16, csr=csr, check=False)
    with torch.cuda.stream(s2):
        Zb = gee.embed(labels, 16, coo=coo, check=False)
    torch.cuda.synchronize()
    assert torch.equal(Za, ref)
    Zo = oracle.embed(g.n, g.src, g.dst, g.w, wl.labels, 16)
    assert row_rel_err(Zb.cpu().numpy(), Zo) <= 1e-5


def test_copy_probe():
    a = torch.arange(1 << 20, dtype=torch.float32, device=DEV)
    b = torch.empty_like(a)
    gee.copy(b, a)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
