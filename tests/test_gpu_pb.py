"""Propagation-blocked pull (unit-weight adjacency): the layout holds exactly the CSR's
entries, and Z is bit-identical to the pull form (integer counts) on every shape."""
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


def _same_bits(a, b):
    assert torch.equal(a.view(torch.int32), b.view(torch.int32))


def _check_layout(csr, pb):
    """Every (row, column) entry of the CSR appears once in the layout, cells ordered by
    column block; the tier slices hold exactly the entries of the first n_lds hot slots."""
    rp = csr.row_ptr.cpu().numpy()
    cols = csr.plain_col().cpu().numpy()
    raw = csr.col.cpu().numpy()
    rows = np.repeat(np.arange(csr.n, dtype=np.int64), np.diff(rp))
    start = pb.cell_start.cpu().numpy().reshape(pb.n_rb, pb.n_cb)
    count = pb.cell_count.cpu().numpy().reshape(pb.n_rb, pb.n_cb).astype(np.int64)
    assert count.sum() == csr.nnz
    n_vcb = (csr.n + (1 << 21) - 1) // (1 << 21)
    assert pb.n_cb == n_vcb + (pb.n_lds + (1 << 17) - 1) // (1 << 17)
    if pb.n_lds:
        assert torch.equal(pb.lds_ids.cpu(), csr.hot_ids[: pb.n_lds].cpu())
    # column-block-major order: cells (cb, rb) are consecutive, except the gap of fewer
    # than 16 entries before the first tier cell, which starts on a multiple of 16
    order = np.argsort(start.T.reshape(-1), kind="stable")
    flat_start, flat_count = start.T.reshape(-1)[order], count.T.reshape(-1)[order]
    flat_cb = np.repeat(np.arange(pb.n_cb), pb.n_rb)[order]
    gaps = flat_start[1:] - (flat_start + flat_count)[:-1]
    boundary = (flat_cb[1:] >= n_vcb) & (flat_cb[:-1] < n_vcb)
    assert np.all(gaps[~boundary] == 0)
    assert np.all((gaps[boundary] >= 0) & (gaps[boundary] < 16) & (flat_start[1:][boundary] % 16 == 0))
    colbytes = pb.col.cpu().numpy().view(np.uint8)
    pcol = pb.col.cpu().numpy().astype(np.int64)
    pul = pb.ul.cpu().numpy().astype(np.int64)
    rb_of = np.repeat(np.repeat(np.arange(pb.n_rb), pb.n_cb), count.reshape(-1))
    cb_of = np.repeat(np.tile(np.arange(pb.n_cb), pb.n_rb), count.reshape(-1))
    idx = np.concatenate([np.arange(a, a + c) for a, c in zip(start.reshape(-1), count.reshape(-1)) if c]) \
        if csr.nnz else np.zeros(0, np.int64)
    prow = rb_of * 256 + pul[idx]
    vcol = pcol[idx].copy()
    tier = cb_of >= n_vcb
    assert np.all(vcol[~tier] >> 21 == cb_of[~tier])
    if tier.any():  # tier slots: low 16 bits from byte 4 H0, then the 17th bits (H0 a multiple of 16)
        ti = idx[tier]
        H0 = int(ti.min())
        assert H0 % 16 == 0 and int(idx[~tier].max(initial=-1)) < H0
        r = ti - H0
        NT = int(tier.sum())
        assert int(r.max()) == NT - 1  # the tier's entries are contiguous from H0
        off = 4 * H0 + 2 * r
        hb = 4 * H0 + 2 * ((NT + 63) // 64 * 64)
        vcol[tier] = (colbytes[off].astype(np.int64) | (colbytes[off + 1].astype(np.int64) << 8)
                      | (((colbytes[hb + r // 8] >> (r % 8)) & 1).astype(np.int64) << 16))
    slots = vcol[tier] + ((cb_of[tier] - n_vcb) << 17)  # slot within the slice -> tier slot
    assert np.all((vcol[tier] >= 0) & (vcol[tier] < (1 << 17)) & (slots < max(pb.n_lds, 1)))
    if pb.n_lds:
        vcol[tier] = pb.lds_ids.cpu().numpy()[slots]
    in_tier = (raw < 0) & ((raw & 0x7FFFFFFF) < pb.n_lds)
    assert int(tier.sum()) == int(in_tier.sum())
    a = np.lexsort((cols, rows))
    b = np.lexsort((vcol, prow))
    assert np.array_equal(rows[a], prow[b]) and np.array_equal(cols[a], vcol[b])
    # word prefix of each row block's cells
    words = np.where(count > 0, ((start & 3) + count + 3) >> 2, 0)
    want = np.cumsum(words, axis=1) - words
    assert np.array_equal(pb.cell_word.cpu().numpy().astype(np.int64).reshape(pb.n_rb, pb.n_cb), want)


def test_small_graph_matches_pull_and_oracle():
    wl = gen.sbm_small()
    g = wl.graph
    coo = gee.to_device(g.n, g.src, g.dst, None, device=DEV)
    csr = gee.csr_build(coo)
    pb = gee.pb_build(csr)
    _check_layout(csr, pb)
    Y = torch.as_tensor(wl.labels).to(DEV)
    Zb = gee.embed_pb(Y, wl.K, pb)
    _same_bits(Zb, gee.embed(Y, wl.K, csr=csr))
    assert_parity(Zb.cpu().numpy(), oracle.embed(g.n, g.src, g.dst, None, wl.labels, wl.K, False), what="sbm")


@pytest.mark.parametrize("hot,tier", [(0, 0), (5000, 5000), (200_000, 200_000), (200_000, 1 << 17), (300_000, 0)])
@pytest.mark.parametrize("K", [1, 7, 50, 128])
def test_several_column_blocks(hot, tier, K):
    """n = 2^21 + 1000 vertices: two column blocks and a partial last row block; R-MAT hubs.
    Tiers of one slice, of two slices (the second partial), of exactly one full slice with
    hot slots decoded beyond it, and hot slots without a tier."""
    n = (1 << 21) + 1000
    rng = np.random.default_rng(K + hot)
    g = gen.rmat(21, 6 << 21, seed=5)
    src = np.r_[g.src, rng.integers(0, n, 200_000).astype(np.int32), np.full(50_000, n - 1, np.int32)]
    dst = np.r_[g.dst, rng.integers(0, n, 200_000).astype(np.int32), rng.integers(0, n, 50_000).astype(np.int32)]
    coo = gee.to_device(n, src, dst, None, device=DEV)
    csr = gee.csr_build(coo, hot_budget=hot)
    pb = gee.pb_build(csr, tier_slots=tier)
    assert pb.n_lds == tier and pb.n_cb == 2 + (tier + (1 << 17) - 1) // (1 << 17)
    if K == 50:
        _check_layout(csr, pb)
    Y = torch.as_tensor(random_labels(rng, n, K, unknown=0.3)).to(DEV)
    _same_bits(gee.embed_pb(Y, K, pb), gee.embed(Y, K, csr=csr))


@pytest.mark.parametrize("K", [7, 50])
def test_tier_beyond_64_slices(K):
    """Every vertex of an Erdős–Rényi graph on 2^24 - 1000 vertices in the tier: 128 slices,
    the last one partial (more slices than the scale-27 R-MAT's 64), bit-identical to
    the pull form."""
    n = (1 << 24) - 1000
    g = gen.er(n, 4 * n, seed=11, weighted=False)
    csr = gee.csr_build(gee.to_device(n, g.src, g.dst, None, device=DEV), hot_budget=n)
    pb = gee.pb_build(csr, tier_slots=n)
    assert pb.n_lds == n and pb.n_cb == 8 + 128
    Y = torch.as_tensor(random_labels(np.random.default_rng(K), n, K, unknown=0.2)).to(DEV)
    _same_bits(gee.embed_pb(Y, K, pb), gee.embed(Y, K, csr=csr))


@pytest.mark.parametrize("K", [7, 50])
def test_cells_beyond_one_per_thread(K):
    """Every vertex of a sparse Erdős–Rényi graph on 2^26 vertices in the tier: 512 slices
    and 32 vertex blocks, 544 cells per row block, more than the rows pass's 512 threads
    (each thread takes a second cell), bit-identical to the pull form."""
    n = 1 << 26
    g = gen.er(n, 2 * n, seed=5, weighted=False)
    csr = gee.csr_build(gee.to_device(n, g.src, g.dst, None, device=DEV), hot_budget=n)
    pb = gee.pb_build(csr, tier_slots=n)
    assert pb.n_lds == n and pb.n_cb == 32 + 512
    Y = torch.as_tensor(random_labels(np.random.default_rng(K + 1), n, K, unknown=0.2)).to(DEV)
    _same_bits(gee.embed_pb(Y, K, pb), gee.embed(Y, K, csr=csr))


@pytest.mark.parametrize("hot", [0, 1000, 150_000])
def test_layout_of_two_column_blocks(hot):
    n = (1 << 21) + 300
    rng = np.random.default_rng(2)
    src = rng.integers(0, n, 400_000).astype(np.int32)
    dst = rng.integers(0, n, 400_000).astype(np.int32)
    csr = gee.csr_build(gee.to_device(n, src, dst, None, device=DEV), hot_budget=hot)
    _check_layout(csr, gee.pb_build(csr, tier_slots=hot))


def test_tier_planner():
    """Slices are kept while their entries average at least min_per_row_block per
    256-row block: counted here from the CSR on the host."""
    g = gen.rmat(20, 16 << 20, seed=9)
    csr = gee.csr_build(gee.to_device(g.n, g.src, g.dst, None, device=DEV), hot_budget=600_000)
    rp = csr.row_ptr.cpu().numpy()
    hot = csr.hot_ids.cpu().numpy().astype(np.int64)
    deg = rp[hot + 1] - rp[hot]
    per_slice = [int(deg[j:j + (1 << 17)].sum()) for j in range(0, len(hot), 1 << 17)]
    n_rb = (g.n + 255) // 256
    for m in (0, 1, 4, 16, 64, 1 << 30):
        k = 0
        while k < len(per_slice) and per_slice[k] >= m * n_rb:
            k += 1
        want = len(hot) if k == len(per_slice) else k << 17
        assert gee.pb_tier_slots(csr, m) == want
    none = gee.csr_build(gee.to_device(g.n, g.src, g.dst, None, device=DEV), hot_budget=0)
    assert gee.pb_tier_slots(none) == 0
    pb = gee.pb_build(csr)  # the planner's tier
    Y = torch.as_tensor(random_labels(np.random.default_rng(1), g.n, 20, unknown=0.1)).to(DEV)
    _same_bits(gee.embed_pb(Y, 20, pb), gee.embed(Y, 20, csr=csr))


def test_unaligned_z_and_ragged_entries():
    """Z at an offset of one float (the rows kernel's scalar stores) and entry counts that
    are not a multiple of 4 or 16 (the gathers' head and tail, the last word's mask)."""
    rng = np.random.default_rng(11)
    for s_extra in (1, 3, 13):
        g = gen.rmat(14, 60_000 + s_extra, seed=s_extra)
        csr = gee.csr_build(gee.to_device(g.n, g.src, g.dst, None, device=DEV), hot_budget=777)
        pb = gee.pb_build(csr)
        for K in (3, 50):
            Y = torch.as_tensor(random_labels(rng, g.n, K, unknown=0.2)).to(DEV)
            buf = torch.full((g.n * K + 1,), -1.0, dtype=torch.float32, device=DEV)
            Zu = gee.embed_pb(Y, K, pb, Z=buf[1:].view(g.n, K))
            _same_bits(Zu, gee.embed(Y, K, csr=csr))
            assert buf[0].item() == -1.0


@pytest.mark.parametrize("K", [65, 66, 100, 127, 128, 129, 200, 255])
def test_large_K(K):
    """Above 64 classes a row block's bins take more than 64 KB of LDS (above 128, 16-bit
    counts or two passes of 128 rows, one workgroup per CU): class counts that
    are not a multiple of 4, with Z aligned (four-float stores when K is a multiple of 4)
    and at an offset of one float (scalar stores), nothing written outside Z."""
    rng = np.random.default_rng(K)
    g = gen.rmat(16, 400_000, seed=K)
    csr = gee.csr_build(gee.to_device(g.n, g.src, g.dst, None, device=DEV), hot_budget=5000)
    pb = gee.pb_build(csr)
    labels = random_labels(rng, g.n, K, unknown=0.2)
    Y = torch.as_tensor(labels).to(DEV)
    ref = gee.embed(Y, K, csr=csr)
    Zb = gee.embed_pb(Y, K, pb)
    _same_bits(Zb, ref)
    buf = torch.full((g.n * K + 2,), -1.0, dtype=torch.float32, device=DEV)
    _same_bits(gee.embed_pb(Y, K, pb, Z=buf[1:-1].view(g.n, K)), ref)
    assert buf[0].item() == -1.0 and buf[-1].item() == -1.0
    if K == 100:
        assert_parity(Zb.cpu().numpy(), oracle.embed(g.n, g.src, g.dst, None, labels, K, False), what="K100")


@pytest.mark.parametrize("tier", [0, 500])
@pytest.mark.parametrize("K", [3, 50, 100, 128, 255])
def test_hub_row_blocks(tier, K):
    """Row blocks with 2^16 entries or more take two passes (one per half of their rows,
    32-bit bins): hubs in the first half, the second half, and in a partial last block
    of 112 rows, next to ordinary blocks."""
    n = 70_000
    rng = np.random.default_rng(K + tier)
    hubs = [(300, 70_000), (256 * 5 + 200, 80_000), (n - 1, 66_000), (256 * 9 + 255, 30_000)]
    src = [rng.integers(0, n, 100_000)] + [np.full(d, h) for h, d in hubs]
    dst = [rng.integers(0, n, 100_000)] + [rng.integers(0, n, d) for _, d in hubs]
    src = np.concatenate(src).astype(np.int32)
    dst = np.concatenate(dst).astype(np.int32)
    csr = gee.csr_build(gee.to_device(n, src, dst, None, device=DEV), hot_budget=1000)
    pb = gee.pb_build(csr, tier_slots=tier)
    Y = torch.as_tensor(random_labels(rng, n, K, unknown=0.25)).to(DEV)
    _same_bits(gee.embed_pb(Y, K, pb), gee.embed(Y, K, csr=csr))


def test_all_unknown_and_empty_graph():
    rng = np.random.default_rng(3)
    n = 5000
    g = gen.rmat(12, 20_000, seed=3)
    csr = gee.csr_build(gee.to_device(g.n, g.src, g.dst, None, device=DEV))
    pb = gee.pb_build(csr)
    Z = gee.embed_pb(torch.zeros(g.n, dtype=torch.int32, device=DEV), 4, pb)
    assert torch.count_nonzero(Z) == 0
    empty = gee.csr_build(gee.to_device(n, np.zeros(0, np.int32), np.zeros(0, np.int32), None, device=DEV))
    pe = gee.pb_build(empty)
    Z = gee.embed_pb(torch.as_tensor(random_labels(rng, n, 3)).to(DEV), 3, pe)
    assert torch.count_nonzero(Z) == 0


def test_errors():
    g = gen.rmat(10, 4000, seed=4)
    csr = gee.csr_build(gee.to_device(g.n, g.src, g.dst, None, device=DEV))
    pb = gee.pb_build(csr)
    Y = torch.ones(g.n, dtype=torch.int32, device=DEV)
    Y[7] = 6
    with pytest.raises(gee.GeeError) as e:
        gee.embed_pb(Y, 5, pb)
    assert e.value.code == gee.GEE_ELABEL
    # a weighted layout with unit weights: the same counts as the unit-weight layout (sums
    # of ones are exact in FP32 and FP64 alike), and the same label error
    w = np.ones(g.s, np.float32)
    wcsr = gee.csr_build(gee.to_device(g.n, g.src, g.dst, w, device=DEV))
    wpb = gee.pb_build(wcsr)
    with pytest.raises(gee.GeeError) as e:
        gee.embed_pb(Y, 5, wpb)
    assert e.value.code == gee.GEE_ELABEL
    Y[7] = 2
    _same_bits(gee.embed_pb(Y, 5, wpb), gee.embed_pb(Y, 5, pb))
    # a layout struct whose weights do not match its fingerprint is skipped with an error
    mixed = gee.DevicePb(g.n, pb.col, pb.ul, pb.cell_start, pb.cell_count, pb.lds_ids, pb.cell_word, pb.nnz,
                         wpb.meta)
    with pytest.raises(gee.GeeError) as e:
        gee.embed_pb(Y, 5, mixed)
    assert e.value.code == gee.GEE_EVERTEX


def test_layout_of_another_graph_raises_vertex_error():
    """A layout used with labels of a smaller graph (its n says 2,000, its entries and tier
    name vertices up to 4,999) is caught by the fingerprint its build wrote: the passes
    read nothing of it and the call raises GEE_EVERTEX (the layout's arrays are those of
    the larger graph, so every table the smaller n implies lies inside them anyway)."""
    rng = np.random.default_rng(41)
    n_big, s = 5000, 60_000
    src = rng.integers(0, n_big, s).astype(np.int32)
    dst = rng.integers(0, n_big, s).astype(np.int32)
    csr = gee.csr_build(gee.to_device(n_big, src, dst, None, device=DEV), hot_budget=600)
    pb = gee.pb_build(csr, tier_slots=512)
    assert pb.n_lds == 512 and int(pb.lds_ids.max()) >= 2000
    stale = gee.DevicePb(2000, pb.col, pb.ul, pb.cell_start, pb.cell_count, pb.lds_ids, pb.cell_word, pb.nnz,
                         pb.meta)
    assert stale.n_cb == pb.n_cb and stale.n_rb < pb.n_rb
    labels = torch.as_tensor(random_labels(rng, 2000, 5)).to(DEV)
    with pytest.raises(gee.GeeError) as e:
        gee.embed_pb(labels, 5, stale)
    assert e.value.code == gee.GEE_EVERTEX
    # the layout itself, with labels of its own graph, is fine
    Yb = torch.as_tensor(random_labels(rng, n_big, 5)).to(DEV)
    _same_bits(gee.embed_pb(Yb, 5, pb), gee.embed(Yb, 5, csr=csr))


def _flags_host(n, src, dst, w):
    """Row-block flags of a weighted layout, from the records: a row of more than 128
    entries (of A + A^T) or a weight that is not >= 0 in one of the block's rows."""
    deg = np.bincount(src, minlength=n) + np.bincount(dst, minlength=n)
    bad = np.zeros(n, bool)
    neg = ~(w >= 0)
    bad[src[neg]] = True
    bad[dst[neg]] = True
    rows = (deg > 128) | bad
    n_rb = (n + 255) // 256
    return np.array([rows[256 * b: 256 * b + 256].any() for b in range(n_rb)], np.uint8)


@pytest.mark.parametrize("K", [5, 50, 100, 128, 255])
@pytest.mark.parametrize("tier", ["none", "all"])
def test_weighted_layout_matches_oracle(K, tier):
    """Weighted propagation-blocked pass: grid weights in (0, 1], plus a star of 400
    leaves (a row of more than 128 entries) and a few negative weights, so that row blocks
    take exact 32-bit integer sums, FP64 sums and, for K = 100, passes over half or a quarter of their
    rows. Within the bar of the oracle, flags as the records imply, and the same with Z
    at an offset of one float. The weights lie on the 2^-24 grid, so unflagged blocks add
    them exactly in 32-bit integers and every call gives the same bits."""
    rng = np.random.default_rng(K + (tier == "all"))
    n, s = 40_000, 500_000
    src = rng.integers(0, n, s).astype(np.int32)
    dst = rng.integers(0, n, s).astype(np.int32)
    hub = np.arange(1, 401, dtype=np.int32) * 37
    src = np.r_[src, np.full(hub.size, 5000, np.int32)].astype(np.int32)
    dst = np.r_[dst, hub].astype(np.int32)
    w = ((rng.integers(0, 1 << 24, src.size) + 1) * 2.0 ** -24).astype(np.float32)
    w[rng.choice(src.size, 50, replace=False)] *= -1
    Y = random_labels(rng, n, K, unknown=0.1)
    coo = gee.to_device(n, src, dst, w, device=DEV)
    csr = gee.csr_build(coo, hot_budget=n if tier == "all" else 0)
    pb = gee.pb_build(csr, tier_slots=None if tier == "all" else 0)
    assert pb.val is not None and (pb.n_lds > 0) == (tier == "all")
    assert np.array_equal(pb.rb_flag.cpu().numpy(), _flags_host(n, src, dst, w))
    meta = pb.meta.cpu().tolist()
    assert meta[:4] == [n, csr.nnz, pb.n_lds, 1]
    assert meta[4] == 24  # weights (r + 1) 2^-24 up to 1: exact 32-bit sums of 2^24 w
    labels = torch.as_tensor(Y).to(DEV)
    Z = gee.embed_pb(labels, K, pb)
    _same_bits(gee.embed_pb(labels, K, pb), Z)  # integer sums: the same bits on every call
    Zo = oracle.embed(n, src, dst, w, Y, K, False)
    Zn = Z.cpu().numpy()
    assert_parity(Zn, Zo, what=f"weighted layout K={K} tier={tier}")
    assert_parity(gee.embed_pb(labels, K, pb).cpu().numpy(), Zn.astype(np.float64), what="second call")
    buf = torch.full((n * K + 2,), -1.0, dtype=torch.float32, device=DEV)
    Zu = gee.embed_pb(labels, K, pb, Z=buf[1:-1].view(n, K))
    assert_parity(Zu.cpu().numpy(), Zo, what="Z at an offset of one float")
    assert buf[0].item() == -1.0 and buf[-1].item() == -1.0
    assert_parity(Z.cpu().numpy(), gee.embed(labels, K, csr=csr).cpu().numpy().astype(np.float64),
                  what="weighted layout vs pull")


def test_weighted_layout_er_workload_shape():
    """The weighted Erdos-Renyi workload's shape at 2^20 records (every vertex in the tier)
    against the oracle."""
    wl = gen.er_weighted(seed=7, log2n=16, log2s=20, K=50)
    g = wl.graph
    csr = gee.csr_build(gee.to_device(g.n, g.src, g.dst, g.w, device=DEV), hot_budget=g.n)
    pb = gee.pb_build(csr)
    assert pb.n_lds == g.n
    Z = gee.embed_pb(torch.as_tensor(wl.labels).to(DEV), wl.K, pb).cpu().numpy()
    assert_parity(Z, oracle.embed(g.n, g.src, g.dst, g.w, wl.labels, wl.K, False), what="weighted ER layout")


def test_weighted_layout_off_grid():
    """Weights with no common grid (significands down to 2^-70 and below):
    the build records no grid, every block sums in FP64 (shared bins, so two calls
    agree within rounding), and the result is within the bar of the oracle."""
    rng = np.random.default_rng(77)
    n, s, K = 30_000, 400_000, 20
    src = rng.integers(0, n, s).astype(np.int32)
    dst = rng.integers(0, n, s).astype(np.int32)
    # cubes of uniform doubles, rounded to FP32: exponents down to 2^-50 and beyond with full
    # significands (uniform FP32 draws would all be multiples of 2^-24)
    w = (rng.random(s) ** 3).astype(np.float32)
    w[w == 0] = 0.5
    Y = random_labels(rng, n, K)
    csr = gee.csr_build(gee.to_device(n, src, dst, w, device=DEV), hot_budget=n)
    pb = gee.pb_build(csr)
    assert pb.meta.cpu().tolist()[4] == -(1 << 62)
    labels = torch.as_tensor(Y).to(DEV)
    Z = gee.embed_pb(labels, K, pb).cpu().numpy()
    assert_parity(Z, oracle.embed(n, src, dst, w, Y, K, False), what="weights off any grid")
    assert_parity(gee.embed_pb(labels, K, pb).cpu().numpy(), Z.astype(np.float64), what="second call")


@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("K", [7, 100, 255])
def test_laplacian_layout_matches_oracle(weighted, K):
    """Laplacian layout: the degrees and each entry's w d_u^-1/2 d_v^-1/2 taken at the build,
    summed as a weighted layout's terms. Unit and grid weights, a hub row (FP64 blocks),
    isolated vertices (zero rows), with and without the tier; within the bar of the oracle
    and of the CSR pull form, d^-1/2 as the CSR's degrees give it."""
    rng = np.random.default_rng(K + 10 * weighted)
    n, s = 30_000, 300_000
    src = rng.integers(0, n - 500, s).astype(np.int32)  # the last 500 vertices isolated
    dst = rng.integers(0, n - 500, s).astype(np.int32)
    hub = np.arange(1, 301, dtype=np.int32) * 41
    src = np.r_[src, np.full(hub.size, 777, np.int32)].astype(np.int32)
    dst = np.r_[dst, hub].astype(np.int32)
    w = ((rng.integers(0, 1 << 24, src.size) + 1) * 2.0 ** -24).astype(np.float32) if weighted else None
    Y = random_labels(rng, n, K, unknown=0.2)
    Zo = oracle.embed(n, src, dst, w, Y, K, True)
    coo = gee.to_device(n, src, dst, w, device=DEV)
    labels = torch.as_tensor(Y).to(DEV)
    for hot in (0, n):
        csr = gee.csr_build(coo, hot_budget=hot)
        pb = gee.pb_build(csr, tier_slots=None if hot else 0, laplacian=True)
        assert pb.laplacian and pb.meta.cpu().tolist()[3] == 2
        d = oracle.degrees(n, src, dst, w)
        r = np.where(d > 0, 1.0 / np.sqrt(np.where(d > 0, d, 1.0)), 0.0).astype(np.float32)
        assert np.array_equal(pb.rsd.cpu().numpy(), r)
        Z = gee.embed_pb(labels, K, pb).cpu().numpy()
        assert_parity(Z, Zo, what=f"Laplacian layout K={K} weighted={weighted} hot={hot}")
        assert not Z[n - 500:].any()
        Zp = gee.embed(labels, K, csr=csr, laplacian=True).cpu().numpy()
        assert_parity(Z, Zp.astype(np.float64), what="Laplacian layout vs pull")


def test_laplacian_layout_negative_weight_and_mismatch():
    """A negative weight raises GEE_ENEGW at the Laplacian build; a Laplacian layout struct
    handed over without its d^-1/2 (read as adjacency) is refused by the fingerprint."""
    rng = np.random.default_rng(3)
    n, s = 2000, 10_000
    src = rng.integers(0, n, s).astype(np.int32)
    dst = rng.integers(0, n, s).astype(np.int32)
    w = np.ones(s, np.float32)
    w[17] = -0.5
    csr = gee.csr_build(gee.to_device(n, src, dst, w, device=DEV))
    with pytest.raises(gee.GeeError) as e:
        gee.pb_build(csr, laplacian=True)
    assert e.value.code == gee.GEE_ENEGW
    w[17] = 0.5
    csr = gee.csr_build(gee.to_device(n, src, dst, w, device=DEV))
    pb = gee.pb_build(csr, laplacian=True)
    as_adj = gee.DevicePb(n, pb.col, pb.ul, pb.cell_start, pb.cell_count, pb.lds_ids, pb.cell_word, pb.nnz, pb.meta,
                          pb.val, pb.rb_flag, None)
    labels = torch.as_tensor(random_labels(rng, n, 5)).to(DEV)
    with pytest.raises(gee.GeeError) as e:
        gee.embed_pb(labels, 5, as_adj)
    assert e.value.code == gee.GEE_EVERTEX
    assert_parity(gee.embed_pb(labels, 5, pb).cpu().numpy(),
                  oracle.embed(n, src, dst, w, labels.cpu().numpy(), 5, True), what="Laplacian layout")
