"""gee_embed_noalloc (the library's static scratch in place of a workspace) against
gee_embed on the same inputs, through the C ABI.

Two calls in a row per form and version, the second on a smaller graph, so the second
call runs over the scratch the first one left behind. The pull form and unit-weight
sums are deterministic, so those results are compared bit for bit; the push form's
weighted FP32 atomics add in an unspecified order and are compared at the 1e-5
per-row bar (and both against the FP64 oracle).
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_2402_04403_amd as gee
from gpu_util import announce, assert_parity, random_labels, random_multigraph

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]
DEV = torch.device("cuda:0")

# (n, s) of the first call, then of the second, smaller one
SIZES = [(200_003, 1_500_007), (10_007, 50_021)]


def _inputs(seed, n, s, weighted, K):
    rng = np.random.default_rng(seed)
    src, dst, w = random_multigraph(rng, n, s, weighted)
    Y = random_labels(rng, n, K)
    return src, dst, w, Y


@pytest.mark.parametrize("form", ["pull", "push"])
@pytest.mark.parametrize("weighted,lap", [(False, False), (True, False), (True, True)])
def test_noalloc_matches_embed_two_calls(form, weighted, lap):
    K = 50
    for i, (n, s) in enumerate(SIZES):
        announce(f"noalloc form={form} weighted={weighted} lap={lap} call={i} n={n} s={s}")
        src, dst, w, Y = _inputs(100 + i, n, s, weighted, K)
        coo = gee.to_device(n, src, dst, w, device=DEV)
        csr = gee.csr_build(coo, hot_budget=n // 20) if form == "pull" else None
        labels = torch.as_tensor(Y).to(DEV)
        want = gee.embed(labels, K, coo=coo, csr=csr, laplacian=lap).cpu().numpy()
        Z = torch.full((n, K), float("nan"), dtype=torch.float32, device=DEV)
        err = torch.zeros(1, dtype=torch.int32, device=DEV)
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated(DEV)
        gee.embed_noalloc(labels, K, Z, err, coo=coo, csr=csr, laplacian=lap, check=False)
        assert torch.cuda.memory_allocated(DEV) == before  # the binding allocates nothing either
        assert int(err.item()) == 0
        got = Z.cpu().numpy()
        if form == "pull" or not weighted:
            assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), "not bit-identical to gee_embed"
        else:
            assert_parity(got, want.astype(np.float64), what="noalloc vs gee_embed")
        Zo = oracle.embed(n, src, dst, w, Y, K, laplacian=lap)
        assert_parity(got, Zo, what="noalloc vs oracle")


def test_noalloc_data_error_and_refusal():
    n, s, K = 1000, 5000, 5
    rng = np.random.default_rng(7)
    src, dst, _ = random_multigraph(rng, n, s, False)
    coo = gee.to_device(n, src, dst, None, device=DEV)
    Y = random_labels(rng, n, K)
    Y[17] = K + 1  # a label outside [0, K]
    labels = torch.as_tensor(Y).to(DEV)
    Z = torch.empty((n, K), dtype=torch.float32, device=DEV)
    err = torch.zeros(1, dtype=torch.int32, device=DEV)
    gee.embed_noalloc(labels, K, Z, err, coo=coo, check=False)
    assert int(err.item()) == gee.GEE_ELABEL
    # a call whose workspace exceeds the static scratch is refused before any launch
    big_n = (gee.NOALLOC_SCRATCH_BYTES // 8) + 1  # Laplacian records alone take 8 bytes a vertex
    big = gee.Coo(big_n, 0, None, None, None)
    lib = gee.load()
    assert lib.gee_embed_noalloc(ctypes.byref(big), None, Z.data_ptr(), K, 1, Z.data_ptr(), err.data_ptr(), None,
                                 torch.cuda.current_stream().cuda_stream) == gee.GEE_EWORKSPACE
