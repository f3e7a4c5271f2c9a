"""Parity at the workload sizes: the Erdős–Rényi weighted graph (n = 2^22, s = 2^26,
K = 50) in full against the oracle, the paper-scale R-MAT (scale 27, edge factor
14, 1,879,048,192 records) on sampled rows, in the launch configuration the
benchmark times (default segment length and window), with the propagation-blocked
pass compared in full against the pull pass, the batched workload (R-MAT scale 24,
64 vectors) on sampled rows of every vector, and the serving pool's first 60 jobs through
the serving loop. At the paper scale every row and every column of the push and pull
forms is also checked against sums taken on the host from the records."""
import time

import numpy as np
import pytest
import torch

import gen
import oracle
import paper_2402_04403_amd as gee
from gpu_util import announce, assert_parity

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]
DEV = torch.device("cuda:0")


@pytest.fixture(autouse=True)
def _announce(request):
    announce(request.node.nodeid)
    yield
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


@pytest.mark.timeout(900)
def test_er_weighted_full_parity():
    t0 = time.time()
    wl = gen.er_weighted()  # n = 2^22, s = 2^26, K = 50, 5% unknown
    g = wl.graph
    coo = gee.to_device(g.n, g.src, g.dst, g.w, device=DEV)
    labels = torch.as_tensor(wl.labels).to(DEV)
    csr = gee.csr_build(coo)
    assert np.array_equal(gee.counts(labels, wl.K).cpu().numpy(), oracle.counts(wl.labels, wl.K))
    d = gee.degrees(csr=csr).cpu().numpy()
    assert np.array_equal(d, oracle.degrees(g.n, g.src, g.dst, g.w))
    announce(f"  inputs ready {time.time() - t0:.1f}s")
    for lap in (False, True):
        Zo = oracle.embed(g.n, g.src, g.dst, g.w, wl.labels, wl.K, lap)
        announce(f"  oracle lap={lap} {time.time() - t0:.1f}s")
        Zp = gee.embed(labels, wl.K, csr=csr, laplacian=lap).cpu().numpy()
        e_pull = assert_parity(Zp, Zo, what=f"pull lap={lap}")
        Za = gee.embed(labels, wl.K, coo=coo, laplacian=lap).cpu().numpy()
        e_push = assert_parity(Za, Zo, what=f"push lap={lap}")
        announce(f"  lap={lap}: pull {e_pull:.2e} push {e_push:.2e}")
        del Zo, Zp, Za


def labelled_neighbour_sums(n, src, dst, Y, K, chunk=1 << 28):
    """Host sums over the records, for unit weights (Algorithm 1 with every W factor taken
    out): rows[u] = the labelled entries of row u of A + A^T (its records' other endpoints
    with a class), cols[k - 1] = the sum of the degrees of the class-k vertices (every
    entry (u, v) with Y(v) = k counted once); int64, exact."""
    rows = np.zeros(n, np.int64)
    deg = np.zeros(n, np.int64)
    for a in range(0, len(src), chunk):
        s_, d_ = src[a:a + chunk], dst[a:a + chunk]
        rows += np.bincount(s_[Y[d_] > 0], minlength=n)
        rows += np.bincount(d_[Y[s_] > 0], minlength=n)
        deg += np.bincount(s_, minlength=n)
        deg += np.bincount(d_, minlength=n)
    cols = np.bincount(Y, weights=deg, minlength=K + 1)  # FP64 sums of integers below 2^53: exact
    return rows, cols[1:].astype(np.int64)


def check_all_rows(Z, counts, want_rows, want_cols, what, chunk=1 << 22):
    """For unit weights Z[u, k-1] is count(u, k) / n_k rounded once to FP32, with count(u, k)
    the number of row u's entries of class k (below 2^23 here), so Z * n_k rounds back to
    that integer. Every row's recovered counts must add up to its labelled entries and
    every column's to its class's degree sum, exactly. The FP64 sums of Z * n_k must
    also meet the row bar (1e-5 relative) and, per column, the bound of one FP32
    rounding per element (2^-23 relative covers the 2^-24 rounding of every term; the
    roundings of equal counts do not cancel, so a column cannot be held much tighter)."""
    n, K = Z.shape
    nk = counts[1:].to(torch.float64)
    wr = torch.as_tensor(want_rows, device=Z.device)
    col_int = torch.zeros(K, dtype=torch.int64, device=Z.device)
    col_fp = torch.zeros(K, dtype=torch.float64, device=Z.device)
    worst = 0.0
    for a in range(0, n, chunk):
        x = Z[a:a + chunk].to(torch.float64) * nk
        c = torch.round(x)
        assert bool((c >= 0).all()), f"{what}: negative entry in rows {a}.."
        row_int = c.to(torch.int64).sum(1)
        bad = torch.nonzero(row_int != wr[a:a + chunk])
        assert bad.numel() == 0, f"{what}: row {a + int(bad[0, 0])} counts {int(row_int[bad[0, 0]])} " \
                                 f"labelled entries, the records give {int(wr[a + int(bad[0, 0])])}"
        row_fp = x.sum(1)
        ref = wr[a:a + chunk].to(torch.float64)
        e = ((row_fp - ref).abs() / ref.clamp(min=1)).max().item()
        worst = max(worst, e)
        col_int += c.to(torch.int64).sum(0)
        col_fp += x.sum(0)
    assert worst <= 1e-5, f"{what}: row sum relative error {worst:.3e}"
    wc = torch.as_tensor(want_cols, device=Z.device)
    assert torch.equal(col_int, wc), f"{what}: column counts differ from the class degree sums"
    ce = ((col_fp - wc.to(torch.float64)).abs() / wc.to(torch.float64).clamp(min=1)).max().item()
    assert ce <= 2.0 ** -23, f"{what}: column sum relative error {ce:.3e}"
    announce(f"  {what}: all {n} rows and {K} columns agree (row sums {worst:.1e}, columns {ce:.1e})")


@pytest.mark.slow
@pytest.mark.timeout(1200)
def test_rmat_paper_scale_sampled_rows():
    t0 = time.time()
    wl = gen.rmat_paper_scale()  # scale 27, edge factor 14, K = 50, 1% unknown
    g = wl.graph
    announce(f"  generated s={g.s} {time.time() - t0:.1f}s")
    coo = gee.to_device(g.n, g.src, g.dst, device=DEV)
    labels = torch.as_tensor(wl.labels).to(DEV)
    csr = gee.csr_build(coo, hot_budget=gee.PB_HOT_BUDGET)  # the configuration the benchmark times
    torch.cuda.synchronize()
    announce(f"  csr built nnz={csr.nnz} {time.time() - t0:.1f}s")
    assert csr.nnz == 2 * g.s
    assert np.array_equal(gee.counts(labels, wl.K).cpu().numpy(), oracle.counts(wl.labels, wl.K))
    # rows to compare: uniform rows, the highest-degree rows (split across many
    # segments), and isolated rows (must be exactly zero)
    rng = np.random.default_rng(27)
    deg = (csr.row_ptr[1:] - csr.row_ptr[:-1])
    top = torch.topk(deg, 64).indices.cpu().numpy()
    iso = torch.nonzero(deg == 0)[:64, 0].cpu().numpy()
    rows = np.unique(np.r_[rng.choice(g.n, 3000, replace=False), top, iso]).astype(np.int64)
    idx = torch.as_tensor(rows, device=DEV)
    Zp = gee.embed(labels, wl.K, csr=csr)
    pull_rows = Zp[idx].cpu().numpy()
    announce(f"  pull done {time.time() - t0:.1f}s")
    # propagation-blocked layout of the same CSR: all of Z, bit for bit
    pb = gee.pb_build(csr)
    Zb = gee.embed_pb(labels, wl.K, pb)
    assert torch.equal(Zb.view(torch.int32), Zp.view(torch.int32))
    del Zp, Zb, pb
    torch.cuda.empty_cache()
    announce(f"  propagation-blocked pass equal in full {time.time() - t0:.1f}s")
    Za = gee.embed(labels, wl.K, coo=coo)
    push_rows = Za[idx].cpu().numpy()
    announce(f"  push done {time.time() - t0:.1f}s")
    # every row and every column of both forms against sums taken on the host from the
    # records (the propagation-blocked Z equals the pull form's bit for bit)
    want_rows, want_cols = labelled_neighbour_sums(g.n, g.src, g.dst, wl.labels, wl.K)
    announce(f"  host invariants {time.time() - t0:.1f}s")
    cnt = torch.as_tensor(oracle.counts(wl.labels, wl.K), device=DEV)
    for name, Zf in (("push", Za), ("pull", gee.embed(labels, wl.K, csr=csr))):
        check_all_rows(Zf, cnt, want_rows, want_cols, name)
        del Zf
        torch.cuda.empty_cache()
    del Za
    announce(f"  all-row invariants {time.time() - t0:.1f}s")
    Zo = oracle.embed_rows(g.n, g.src, g.dst, None, wl.labels, wl.K, False, rows)
    announce(f"  oracle rows {time.time() - t0:.1f}s")
    assert_parity(pull_rows, Zo, what="pull, sampled rows")
    assert_parity(push_rows, Zo, what="push, sampled rows")
    # unit weights: both forms hold exact integer sums, so they agree bit for bit
    assert np.array_equal(pull_rows.view(np.uint32), push_rows.view(np.uint32))
    assert not pull_rows[np.isin(rows, iso)].any()


@pytest.mark.timeout(900)
def test_batched_full_size_sampled_rows():
    """The batched benchmark's workload (R-MAT scale 24, edge factor 16, 64 vectors, K
    log-uniform on [2, 256], even vectors adjacency and odd Laplacian) in the launch
    configuration it times (default segment length, 64 vectors per group): sampled rows
    of every vector against the oracle, and adjacency vector 0 bit for bit against a
    single pull call."""
    t0 = time.time()
    wl = gen.rmat_batched()
    g = wl.graph
    announce(f"  generated s={g.s} B={len(wl.Ks)} {time.time() - t0:.1f}s")
    coo = gee.to_device(g.n, g.src, g.dst, device=DEV)
    labels = torch.as_tensor(wl.labels).to(DEV)
    csr = gee.csr_build(coo, hot_budget=gee.DEFAULT_HOT_BUDGET)
    del coo
    torch.cuda.empty_cache()
    Z, zoff = gee.embed_batch(labels.view(-1), wl.Ks, wl.laps, csr)
    torch.cuda.synchronize()
    announce(f"  batched pass done {time.time() - t0:.1f}s")
    rng = np.random.default_rng(24)
    deg = csr.row_ptr[1:] - csr.row_ptr[:-1]
    top = torch.topk(deg, 32).indices.cpu().numpy()
    iso = torch.nonzero(deg == 0)[:32, 0].cpu().numpy()
    rows = np.unique(np.r_[rng.choice(g.n, 2000, replace=False), top, iso]).astype(np.int64)
    idx = torch.as_tensor(rows, device=DEV)
    picked = {b: Z[idx, zoff[b]:zoff[b] + wl.Ks[b]].cpu().numpy() for b in range(len(wl.Ks))}
    del Z
    torch.cuda.empty_cache()
    Zs = gee.embed(labels[0], wl.Ks[0], csr=csr)
    assert np.array_equal(Zs[idx].cpu().numpy().view(np.uint32), picked[0].view(np.uint32))
    del Zs
    for b, blk in picked.items():
        assert wl.laps[b] == (b % 2 == 1)
        Zo = oracle.embed_rows(g.n, g.src, g.dst, None, wl.labels[b], wl.Ks[b], wl.laps[b], rows)
        assert_parity(blk, Zo, what=f"vector {b} (K={wl.Ks[b]}, laplacian={wl.laps[b]}), sampled rows")
        assert not blk[np.isin(rows, iso)].any()
    announce(f"  oracle rows checked {time.time() - t0:.1f}s")


@pytest.mark.timeout(900)
def test_serving_pool_sampled_jobs():
    """The serving benchmark's pool (100 graphs, log-normal sizes up to 5*10^7 records) and
    the first 60 jobs of its mix, through the batched serving loop: every vector of every
    job checked against the oracle on sampled rows."""
    from paper_2402_04403_amd.serve import Request, Server

    t0 = time.time()
    pool = gen.serve_pool()
    jobs = gen.serve_jobs(pool)[:60]
    gids = sorted({j.gid for j in jobs})
    graphs = {}
    for gid in gids:
        g = pool[gid].make()
        graphs[gid] = (pool[gid].n, g.src, g.dst)
    announce(f"  {len(gids)} graphs generated {time.time() - t0:.1f}s")
    srv = Server(graphs, int(200e9), keep_results=True)
    for j in jobs:
        srv.submit(Request(j.jid, j.gid, j.Ks, [j.laplacian] * len(j.Ks),
                           torch.from_numpy(j.labels(graphs[j.gid][0])).pin_memory(), time.perf_counter()))
    done = {d.jid: d for d in srv.drain()}
    assert len(done) == len(jobs) and all(d.error == 0 for d in done.values())
    announce(f"  served {time.time() - t0:.1f}s")
    rng = np.random.default_rng(5)
    nvec = 0
    for j in jobs:
        n, src, dst = graphs[j.gid]
        Y = j.labels(n)
        Zj = done[j.jid].Z
        col = 0
        for b, K in enumerate(j.Ks):
            rows = np.unique(rng.choice(n, min(n, 200), replace=False)).astype(np.int64)
            Zo = oracle.embed_rows(n, src, dst, None, Y[b], K, j.laplacian, rows)
            got = Zj[torch.as_tensor(rows, device=DEV), col:col + K].cpu().numpy()
            assert_parity(got, Zo, what=f"job {j.jid} vector {b} on graph {j.gid} (n={n}, s={len(src)})")
            col += K
            nvec += 1
    announce(f"  {len(jobs)} jobs, {nvec} vectors checked {time.time() - t0:.1f}s")
