"""Labels from an embedding on the GPU (gee_argmax) and the refinement loop, against the
oracle: the argmax sees the same FP32 values on both sides, so labels are compared exactly."""
import numpy as np
import pytest
import torch

import gen
import oracle
import paper_2402_04403_amd as gee
from gpu_util import announce, random_labels

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]
DEV = torch.device("cuda:0")


@pytest.fixture(autouse=True)
def _announce(request):
    announce(request.node.nodeid)
    yield
    torch.cuda.synchronize()


@pytest.mark.parametrize("K,pad", [(5, 0), (50, 0), (50, 3), (300, 0)])
def test_argmax_matches_oracle(K, pad):
    g = gen.rmat(14, 120_000, seed=K)
    rng = np.random.default_rng(K + pad)
    csr = gee.csr_build(gee.to_device(g.n, g.src, g.dst, None, device=DEV))
    Y = random_labels(rng, g.n, K, unknown=0.3)
    Yd = torch.as_tensor(Y).to(DEV)
    Z = gee.embed(Yd, K, csr=csr)
    if pad:  # a wider Z with the block in its first K columns (rows read in place)
        Zw = torch.full((g.n, K + pad), -1.0, dtype=torch.float32, device=DEV)
        Zw[:, :K] = Z
        Z = Zw
    changed = torch.zeros(1, dtype=torch.int64, device=DEV)
    lab = gee.argmax(Z, K, prev=Yd, changed=changed)
    want, ch = oracle.argmax_labels(Z[:, :K].cpu().numpy(), prev=Y)
    assert np.array_equal(lab.cpu().numpy(), want)
    assert int(changed.item()) == ch


@pytest.mark.parametrize("form", ["pull", "pb"])
@pytest.mark.parametrize("record", [True, False])
def test_refine_recovers_blocks_like_the_oracle(form, record):
    wl = gen.sbm_small(seed=2)
    g = wl.graph
    truth = wl.labels.copy()
    known = truth > 0
    rng = np.random.default_rng(9)
    Y0 = truth.copy()
    noisy = rng.random(g.n) < 0.3
    Y0[noisy] = rng.integers(1, wl.K + 1, int(noisy.sum()))
    csr = gee.csr_build(gee.to_device(g.n, g.src, g.dst, None, device=DEV), hot_budget=256)
    args = dict(csr=csr) if form == "pull" else dict(pb=gee.pb_build(csr, tier_slots=256))
    Y, rounds, hist = gee.refine(torch.as_tensor(Y0).to(DEV), wl.K, record=record, **args)
    Yo, rounds_o, hist_o = oracle.refine(g.n, g.src, g.dst, Y0, wl.K)
    assert np.array_equal(Y.cpu().numpy(), Yo) and hist == hist_o and rounds == rounds_o
    assert hist[-1] == 0
    # the planted blocks come back (block ids are the class labels of the generator)
    assert np.mean(Yo[known] == truth[known]) > 0.99
