"""Recorded calls (hipGraph) and the batched form's segment-length tuner.

Every replay of a recorded sequence must give the bits an eager call gives on the same
labels; the test changes the labels between replays, with eager work and host
synchronisation in between, and checks every replay."""
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
    assert torch.equal(a.contiguous().view(torch.int32), b.contiguous().view(torch.int32))


def test_recorded_calls_replay_like_eager_calls():
    g = gen.rmat(15, 300_000, seed=21)
    n = g.n
    csr = gee.csr_build(gee.to_device(n, g.src, g.dst, None, device=DEV), hot_budget=3000)
    pb = gee.pb_build(csr, tier_slots=3000)
    Ks, laps = [5, 7, 3], [False, True, False]
    B = len(Ks)
    lab = torch.zeros(B * n, dtype=torch.int32, device=DEV)
    Zb = torch.empty((n, sum(Ks)), dtype=torch.float32, device=DEV)
    wsb = torch.empty(gee.embed_batch_workspace_bytes(n, Ks, laps, csr), dtype=torch.uint8, device=DEV)
    Zp = torch.empty((n, 5), dtype=torch.float32, device=DEV)
    wsp = torch.empty(gee.embed_workspace_bytes(5, csr=csr), dtype=torch.uint8, device=DEV)
    Zq = torch.empty((n, 5), dtype=torch.float32, device=DEV)
    wsq = torch.empty(gee.embed_pb_workspace_bytes(pb, 5), dtype=torch.uint8, device=DEV)
    err = torch.zeros(1, dtype=torch.int32, device=DEV)
    s = torch.cuda.Stream()

    def calls():
        gee.embed_batch(lab, Ks, laps, csr, Z=Zb, ws=wsb, err=err, stream=s, check=False)
        gee.embed(lab[:n], 5, csr=csr, Z=Zp, ws=wsp, err=err, stream=s, check=False)
        gee.embed_pb(lab[:n], 5, pb, Z=Zq, ws=wsq, err=err, stream=s, check=False)

    graph = gee.capture(calls, s)
    rng = np.random.default_rng(3)
    for rep in range(4):
        host = np.concatenate([random_labels(rng, n, k, unknown=0.2) for k in Ks]).astype(np.int32)
        lab.copy_(torch.as_tensor(host))
        torch.cuda.synchronize()
        graph.replay(s)
        s.synchronize()
        ref_b, _ = gee.embed_batch(lab, Ks, laps, csr)
        _same_bits(Zb, ref_b)
        _same_bits(Zp, gee.embed(lab[:n], 5, csr=csr))
        _same_bits(Zq, gee.embed_pb(lab[:n], 5, pb))
        assert int(err.item()) == 0
    graph.close()


def test_batch_tuner_returns_a_candidate():
    wl = gen.sbm_small(seed=4)
    g = wl.graph
    csr = gee.csr_build(gee.to_device(g.n, g.src, g.dst, None, device=DEV))
    rng = np.random.default_rng(5)
    Ks, laps = [wl.K, 3, wl.K], [False, False, True]
    host = [wl.labels, random_labels(rng, g.n, 3, unknown=0.1), wl.labels]
    lab = torch.as_tensor(np.concatenate(host).astype(np.int32)).to(DEV)
    cands, gcands = (1024, 0, 4096), (0, 2, 1)
    best, group, ms = gee.embed_batch_tune(lab, Ks, laps, csr, seg_lens=cands, group_vectors=gcands, reps=2)
    assert best in cands and group in gcands and ms > 0
    Z, zoff = gee.embed_batch(lab, Ks, laps, csr, seg_len=best, group_vectors=group)
    for b in range(len(Ks)):
        Zo = oracle.embed(g.n, g.src, g.dst, None, host[b], Ks[b], laps[b])
        assert_parity(Z[:, zoff[b]:zoff[b] + Ks[b]].cpu().numpy(), Zo, what=f"vector {b}")
