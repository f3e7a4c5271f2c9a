"""Batched GEE on the GPU: every vector's block equals the single-vector call and the
FP64 oracle; groups, layouts, split rows and errors."""
import numpy as np
import pytest
import torch

import gen
import oracle
import paper_2402_04403_amd as gee
from gpu_util import announce, assert_parity, random_labels

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]
DEV = torch.device("cuda:0")


@pytest.fixture(autouse=True)
def _announce(request):
    announce(request.node.nodeid)
    yield
    torch.cuda.synchronize()


def _graph(weighted, seed=51, scale=13, ef=10, hub=3000):
    rng = np.random.default_rng(seed)
    g = gen.rmat(scale, ef << scale, seed=seed)
    src = np.r_[g.src, np.zeros(hub, np.int32)].astype(np.int32)  # a hub that spans many segments
    dst = np.r_[g.dst, rng.integers(0, g.n, hub).astype(np.int32)]
    w = ((rng.integers(0, 1 << 24, src.size) + 1) * 2.0 ** -24).astype(np.float32) if weighted else None
    return g.n, src, dst, w


def _labels(rng, n, Ks):
    return np.stack([random_labels(rng, n, k, unknown=rng.uniform(0, 0.5)) for k in Ks]).astype(np.int32)


@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("seg_len", [0, 256])
def test_batch_blocks_match_single_calls_and_oracle(weighted, seg_len):
    n, src, dst, w = _graph(weighted)
    rng = np.random.default_rng(7)
    Ks = [1, 2, 3, 7, 50, 100, 255, 256, 300, 1000, 5, 64]
    laps = [b % 3 == 1 for b in range(len(Ks))]
    Y = _labels(rng, n, Ks)
    coo = gee.to_device(n, src, dst, w, device=DEV)
    csr = gee.csr_build(coo)
    Z, zoff = gee.embed_batch(torch.as_tensor(Y).to(DEV), Ks, laps, csr, seg_len=seg_len)
    Zh = Z.cpu().numpy()
    for b, (K, lap) in enumerate(zip(Ks, laps)):
        blk = Zh[:, zoff[b]:zoff[b] + K]
        Zs = gee.embed(torch.as_tensor(Y[b]).to(DEV), K, csr=csr, laplacian=lap, seg_len=seg_len).cpu().numpy()
        if not lap and not weighted:  # exact integer sums: identical bits
            assert np.array_equal(blk.view(np.uint32), Zs.view(np.uint32)), b
        Zo = oracle.embed(n, src, dst, w, Y[b], K, lap)
        assert_parity(blk, Zo, what=f"vector {b} K={K} lap={lap}")


def test_many_groups_interleaved_layout_and_gaps():
    """100 vectors alternating versions (groups of one), blocks in reverse order with gaps:
    gap columns stay untouched."""
    n, src, dst, w = _graph(False, seed=52, scale=12, ef=8)
    rng = np.random.default_rng(8)
    B = 100
    Ks = [int(k) for k in rng.integers(2, 40, B)]
    laps = [b % 2 == 1 for b in range(B)]
    zoff, acc = [0] * B, 0
    for b in reversed(range(B)):  # reverse column order, one spare column after each block
        zoff[b] = acc
        acc += Ks[b] + 1
    Y = _labels(rng, n, Ks)
    csr = gee.csr_build(gee.to_device(n, src, dst, w, device=DEV))
    Z = torch.full((n, acc), float("nan"), dtype=torch.float32, device=DEV)
    gee.embed_batch(torch.as_tensor(Y).to(DEV), Ks, laps, csr, Z=Z, zoff=zoff)
    Zh = Z.cpu().numpy()
    gaps = np.array([zoff[b] + Ks[b] for b in range(B)])
    assert np.all(np.isnan(Zh[:, gaps]))
    for b in range(0, B, 9):
        Zo = oracle.embed(n, src, dst, w, Y[b], Ks[b], laps[b])
        assert_parity(Zh[:, zoff[b]:zoff[b] + Ks[b]], Zo, what=f"vector {b}")


def test_large_group_of_64_and_hot_slot_csr():
    n, src, dst, w = _graph(False, seed=53, scale=14, ef=12)
    rng = np.random.default_rng(9)
    Ks = [int(np.floor(np.exp(rng.uniform(np.log(2), np.log(257))))) for _ in range(70)]
    laps = [False] * 70
    Y = _labels(rng, n, Ks)
    coo = gee.to_device(n, src, dst, w, device=DEV)
    plain = gee.csr_build(coo)
    hot = gee.csr_build(coo, hot_budget=2000)
    Zp, zoff = gee.embed_batch(torch.as_tensor(Y).to(DEV), Ks, laps, plain)
    Zh, _ = gee.embed_batch(torch.as_tensor(Y).to(DEV), Ks, laps, hot)
    assert torch.equal(Zp.view(torch.int32), Zh.view(torch.int32))
    Zn = Zp.cpu().numpy()
    for b in (0, 31, 63, 64, 69):
        Zo = oracle.embed(n, src, dst, w, Y[b], Ks[b], False)
        assert_parity(Zn[:, zoff[b]:zoff[b] + Ks[b]], Zo, what=f"vector {b}")


def test_label_rows_beyond_4gib():
    """64 vectors with 16-bit labels on 2^25 vertices: the label rows span (2^25 + 1) x 128
    bytes, past 4 GiB, so the pass addresses them by 64-bit pointers instead of 32-bit
    buffer offsets. Adjacency vectors equal their single calls bit for bit, a Laplacian one
    matches the oracle on sampled rows."""
    n = 1 << 25
    g = gen.er(n, 1 << 25, seed=57, weighted=False)
    Ks = [2] * 62 + [256, 3]
    laps = [False] * 63 + [True]
    coo = gee.to_device(n, g.src, g.dst, None, device=DEV)
    csr = gee.csr_build(coo, hot_budget=1000)
    v = torch.arange(n, device=DEV, dtype=torch.int64)
    Y = torch.stack([((v * (2 * b + 1) + b) % (k + 1)).to(torch.int32) for b, k in enumerate(Ks)])
    Z, zoff = gee.embed_batch(Y, Ks, laps, csr)
    sample = torch.randint(0, n, (1 << 20,), device=DEV, generator=torch.Generator(device=DEV).manual_seed(4))
    for b in (0, 61, 62):  # on 2^20 sampled rows (vector 62's whole block would be 34 GB)
        Zs = gee.embed(Y[b], Ks[b], csr=csr)
        got = Z[sample, zoff[b]:zoff[b] + Ks[b]]
        assert torch.equal(got.view(torch.int32), Zs[sample].view(torch.int32)), b
        del Zs
    rows = np.unique(np.random.default_rng(3).choice(n, 2000, replace=False)).astype(np.int64)
    Zo = oracle.embed_rows(n, g.src, g.dst, None, Y[63].cpu().numpy(), 3, True, rows)
    got = Z[torch.as_tensor(rows, device=DEV), zoff[63]:zoff[63] + 3].cpu().numpy()
    assert_parity(got, Zo, what="Laplacian vector beside 16-bit label rows past 4 GiB")


def test_batch_is_bit_reproducible():
    n, src, dst, w = _graph(True, seed=54)
    rng = np.random.default_rng(10)
    Ks = [5, 17, 50, 3]
    laps = [False, True, False, True]
    Y = torch.as_tensor(_labels(rng, n, Ks)).to(DEV)
    csr = gee.csr_build(gee.to_device(n, src, dst, w, device=DEV))
    Z1, _ = gee.embed_batch(Y, Ks, laps, csr, seg_len=512)
    Z2, _ = gee.embed_batch(Y, Ks, laps, csr, seg_len=512)
    assert torch.equal(Z1.view(torch.int32), Z2.view(torch.int32))


def test_batch_errors():
    n, src, dst, w = _graph(False, seed=55, scale=10, ef=4, hub=10)
    csr = gee.csr_build(gee.to_device(n, src, dst, w, device=DEV))
    Y = np.ones((2, n), np.int32)
    Y[1, 5] = 9  # K = 4
    with pytest.raises(gee.GeeError) as e:
        gee.embed_batch(torch.as_tensor(Y).to(DEV), [4, 4], [False, False], csr)
    assert e.value.code == gee.GEE_ELABEL
    with pytest.raises(gee.GeeError) as e:
        gee.embed_batch(torch.as_tensor(Y).to(DEV), [4, 4], [False, False], csr, zoff=[0, 2],
                        Z=torch.empty((n, 8), device=DEV))
    assert e.value.code == gee.GEE_EINVAL


def test_group_at_the_class_limit():
    """4096 classes in one group (the LDS limit of a group): two mixed-version vectors,
    then one vector alone; blocks equal the single calls / oracle."""
    n, src, dst, w = _graph(False, seed=56, scale=12, ef=6, hub=500)
    rng = np.random.default_rng(11)
    csr = gee.csr_build(gee.to_device(n, src, dst, w, device=DEV), hot_budget=300)
    for Ks, laps in (([2000, 2096], [True, False]), ([4096], [False])):
        Y = _labels(rng, n, Ks)
        Z, zoff = gee.embed_batch(torch.as_tensor(Y).to(DEV), Ks, laps, csr, seg_len=512)
        Zh = Z.cpu().numpy()
        for b, (K, lap) in enumerate(zip(Ks, laps)):
            blk = Zh[:, zoff[b]:zoff[b] + K]
            if not lap:
                Zs = gee.embed(torch.as_tensor(Y[b]).to(DEV), K, csr=csr, seg_len=512).cpu().numpy()
                assert np.array_equal(blk.view(np.uint32), Zs.view(np.uint32)), b
            assert_parity(blk, oracle.embed(n, src, dst, w, Y[b], K, lap), what=f"K={K} lap={lap}")


@pytest.mark.parametrize("Ks", [[255, 255, 3, 40], [255, 256, 3]])
def test_label_width_boundary(Ks):
    """Groups whose classes all fit 8 bits (K <= 255) gather 8-bit label rows, others
    16-bit: labels up to 255 (and 256) survive either width. Adjacency blocks equal the
    single-vector calls bit for bit; every block matches the oracle."""
    n, src, dst, w = _graph(False, seed=57, scale=12, ef=8, hub=500)
    rng = np.random.default_rng(9)
    Y = _labels(rng, n, Ks)
    for b, K in enumerate(Ks):
        Y[b, rng.choice(n, 64, replace=False)] = K  # the largest class is well populated
    laps = [False, True] + [False] * (len(Ks) - 2)
    csr = gee.csr_build(gee.to_device(n, src, dst, w, device=DEV))
    Z, zoff = gee.embed_batch(torch.as_tensor(Y).to(DEV), Ks, laps, csr)
    Zh = Z.cpu().numpy()
    for b, K in enumerate(Ks):
        blk = Zh[:, zoff[b]:zoff[b] + K]
        if not laps[b]:
            Zs = gee.embed(torch.as_tensor(Y[b]).to(DEV), K, csr=csr).cpu().numpy()
            assert np.array_equal(blk.view(np.uint32), Zs.view(np.uint32)), f"vector {b} K={K}"
        assert_parity(blk, oracle.embed(n, src, dst, w, Y[b], K, laps[b]), what=f"vector {b} K={K} lap={laps[b]}")


@pytest.mark.parametrize("weighted", [False, True])
def test_group_size_does_not_change_bits(weighted):
    """Vectors per group (the label tile) only changes how the vectors share passes: every
    vector's block has the same bits with groups of 1, 3 and 64, Laplacian ones included."""
    n, src, dst, w = _graph(weighted, seed=58, scale=12, ef=8, hub=800)
    rng = np.random.default_rng(10)
    Ks = [int(k) for k in rng.integers(2, 70, 11)]
    laps = [b % 3 == 1 for b in range(len(Ks))]
    Y = torch.as_tensor(_labels(rng, n, Ks)).to(DEV)
    csr = gee.csr_build(gee.to_device(n, src, dst, w, device=DEV))
    ref, zoff = gee.embed_batch(Y, Ks, laps, csr, seg_len=512)
    for gv in (1, 3):
        Z, _ = gee.embed_batch(Y, Ks, laps, csr, seg_len=512, group_vectors=gv)
        assert torch.equal(Z.view(torch.int32), ref.view(torch.int32)), gv
