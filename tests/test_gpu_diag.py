"""The atomics-off diagnostic of the push form (the paper's unsafe-update run, Section IV):
exact where no two records update one element, never above the true value otherwise."""
import numpy as np
import pytest
import torch

import gen
import paper_2402_04403_amd as gee
from gpu_util import announce, random_labels

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]
DEV = torch.device("cuda:0")


@pytest.fixture(autouse=True)
def _announce(request):
    announce(request.node.nodeid)
    yield
    torch.cuda.synchronize()


@pytest.mark.parametrize("laplacian", [False, True])
def test_matching_has_no_races(laplacian):
    rng = np.random.default_rng(3)
    m = 200_000
    perm = rng.permutation(2 * m).astype(np.int32)
    src, dst = perm[:m].copy(), perm[m:].copy()  # every vertex in exactly one record
    w = ((rng.integers(0, 1 << 24, m) + 1) * 2.0 ** -24).astype(np.float32)
    Y = torch.as_tensor(random_labels(rng, 2 * m, 9, unknown=0.2)).to(DEV)
    coo = gee.to_device(2 * m, src, dst, w, device=DEV)
    Za = gee.embed(Y, 9, coo=coo, laplacian=laplacian)
    Zp = gee.embed_push_nonatomic(Y, 9, coo, laplacian=laplacian)
    assert torch.equal(Za.view(torch.int32), Zp.view(torch.int32))


def test_lost_updates_only_lower_the_result():
    g = gen.rmat(14, 16 << 14, seed=9)
    rng = np.random.default_rng(4)
    Y = torch.as_tensor(random_labels(rng, g.n, 5, unknown=0.1)).to(DEV)
    coo = gee.to_device(g.n, g.src, g.dst, None, device=DEV)
    Za = gee.embed(Y, 5, coo=coo).cpu().numpy()
    Zp = gee.embed_push_nonatomic(Y, 5, coo).cpu().numpy()
    assert np.all(np.isfinite(Zp))
    assert np.all(Zp <= Za)  # unit weights: integer partial sums, each a subset of the true one
