"""The C ABI library loads, exports what include/gee.h declares, and rejects bad host
arguments before launching anything (CPU only: no call here reaches a kernel)."""
import ctypes
import os
import re

import pytest
import torch  # noqa: F401  (the HIP runtime libgee.so links against)

import paper_2402_04403_amd as gee
from paper_2402_04403_amd import build as hipbuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gee.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(gee.LIB_PATH):
        hipbuild.build(force=True)
    return gee.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w \*]*?\b(gee_\w+)\s*\(", text, flags=re.M)))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert {"gee_counts", "gee_weights", "gee_degrees", "gee_embed", "gee_embed_workspace", "gee_csr_build",
            "gee_csr_workspace", "gee_copy", "gee_strerror"} <= set(names)
    for name in names:
        assert hasattr(lib, name), f"{name} declared in gee.h but not exported"


def declared_arity():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    out = {}
    for m in re.finditer(r"\b(gee_\w+)\s*\(([^;{()]*)\)\s*;", text, flags=re.S):
        params = m.group(2).strip()
        out[m.group(1)] = 0 if params in ("", "void") else len(params.split(","))
    return out


def test_binding_arity_matches_header(lib):
    """Every ctypes prototype has exactly the header's parameter count. A short list lets
    ctypes pass the trailing arguments by default conversion (a Python int becomes a 32-bit
    int whose upper half in a 64-bit slot is undefined), which corrupts a stream handle."""
    arity = declared_arity()
    assert set(arity) == set(declared_functions())
    for name, n in arity.items():
        at = getattr(lib, name).argtypes
        assert at is not None, f"{name} has no argtypes"
        assert len(at) == n, f"{name}: {len(at)} argtypes, {n} parameters in gee.h"


def test_strerror(lib):
    for code in range(-7, 1):
        assert lib.gee_strerror(code)
    assert lib.gee_strerror(-99) == b"unknown status"


FAKE = 1 << 20  # an aligned non-null address; never dereferenced by these calls


def test_host_argument_errors(lib):
    assert lib.gee_counts(None, 10, 5, FAKE, FAKE, None) == gee.GEE_EINVAL
    assert lib.gee_counts(FAKE, 0, 5, FAKE, FAKE, None) == gee.GEE_EINVAL
    assert lib.gee_counts(FAKE, 10, 0, FAKE, FAKE, None) == gee.GEE_EINVAL
    assert lib.gee_counts(FAKE, 10, 65536, FAKE, FAKE, None) == gee.GEE_EINVAL
    assert lib.gee_weights(FAKE, 0, FAKE, None) == gee.GEE_EINVAL
    assert lib.gee_degrees(None, None, FAKE, FAKE, None) == gee.GEE_EINVAL
    assert lib.gee_copy(FAKE, FAKE + 4, 64, None) == gee.GEE_EINVAL
    assert lib.gee_copy(FAKE, FAKE, 60, None) == gee.GEE_EINVAL


def test_embed_argument_errors(lib):
    coo = gee.Coo(100, 1000, FAKE, FAKE, None)
    csr = gee.Csr(100, 2000, FAKE, FAKE, None, 0, None)
    o = gee.EmbedOpts(0, 0, None, None)
    ws = lambda c, r, K, lap=0, opt=o: lib.gee_embed_workspace(c, r, K, lap, ctypes.byref(opt))
    assert ws(ctypes.byref(coo), None, 5) > 0
    assert ws(None, ctypes.byref(csr), 5) > 0
    assert ws(None, None, 5) == 0
    assert ws(ctypes.byref(coo), None, 0) == 0
    assert ws(None, ctypes.byref(csr), 4097) == 0  # pull form: K <= 4096
    assert ws(ctypes.byref(coo), None, 65535) > 0  # push form: up to 65535 (16-bit labels)
    assert ws(None, ctypes.byref(csr), 5, 0, gee.EmbedOpts(10, 0, None, None)) == 0  # seg_len < 64
    assert ws(None, ctypes.byref(csr), 5, 0, gee.EmbedOpts(65536, 0, None, None)) == 0  # 16-bit counters
    assert ws(None, ctypes.byref(csr), 5, 0, gee.EmbedOpts(0, 65, None, None)) == 0
    bad_n = gee.Coo(0, 10, FAKE, FAKE, None)
    assert ws(ctypes.byref(bad_n), None, 5) == 0
    mismatch = gee.Coo(99, 10, FAKE, FAKE, None)
    assert ws(ctypes.byref(mismatch), ctypes.byref(csr), 5) == 0
    # workspace too small / misaligned / missing: rejected before any launch
    need = ws(None, ctypes.byref(csr), 5)
    call = lambda wsp, wsb: lib.gee_embed(None, ctypes.byref(csr), FAKE, 5, 0, FAKE, wsp, wsb, FAKE,
                                          ctypes.byref(o), None)
    assert call(FAKE, need - 1) == gee.GEE_EWORKSPACE
    assert call(FAKE + 8, need) == gee.GEE_EWORKSPACE
    assert call(None, need) == gee.GEE_EWORKSPACE
    assert lib.gee_embed(None, ctypes.byref(csr), None, 5, 0, FAKE, FAKE, need, FAKE, ctypes.byref(o),
                         None) == gee.GEE_EINVAL
    big = gee.Coo(100, (1 << 40) + 1, FAKE, FAKE, None)
    assert lib.gee_embed(ctypes.byref(big), None, FAKE, 5, 0, FAKE, FAKE, 1 << 30, FAKE, None,
                         None) == gee.GEE_EOVERFLOW


def test_workspace_sizes_scale(lib):
    o = gee.EmbedOpts(0, 0, None, None)
    small = gee.Csr(1000, 10_000, FAKE, FAKE, None, 0, None)
    large = gee.Csr(1000, 1_000_000, FAKE, FAKE, None, 0, None)
    a = lib.gee_embed_workspace(None, ctypes.byref(small), 50, 0, ctypes.byref(o))
    b = lib.gee_embed_workspace(None, ctypes.byref(large), 50, 0, ctypes.byref(o))
    assert b > a > 0 and a % 256 == 0 and b % 256 == 0
    lap = lib.gee_embed_workspace(None, ctypes.byref(small), 50, 1, ctypes.byref(o))
    assert lap > a  # 8-byte label records and FP64 degrees
    assert lib.gee_csr_workspace(1000, 5000, 1, 0) > lib.gee_csr_workspace(1000, 5000, 0, 0) > 0
    assert lib.gee_csr_workspace(1000, 5000, 0, 100) > lib.gee_csr_workspace(1000, 5000, 0, 0)
    assert lib.gee_csr_workspace(0, 5000, 0, 0) == 0
    assert lib.gee_csr_workspace(10, 5000, 0, -1) == 0
    hot = gee.Csr(1000, 10_000, FAKE, FAKE, None, 50, FAKE)
    assert lib.gee_embed_workspace(None, ctypes.byref(hot), 50, 0, ctypes.byref(o)) > a  # hot label table
    bad_hot = gee.Csr(1000, 10_000, FAKE, FAKE, None, 50, None)
    assert lib.gee_embed_workspace(None, ctypes.byref(bad_hot), 50, 0, ctypes.byref(o)) == 0
    too_many = gee.Csr(1000, 10_000, FAKE, FAKE, None, 1001, FAKE)
    assert lib.gee_embed_workspace(None, ctypes.byref(too_many), 50, 0, ctypes.byref(o)) == 0


def test_csr_build_argument_errors(lib):
    coo = gee.Coo(100, 1000, FAKE, FAKE, FAKE)
    need = lib.gee_csr_workspace(100, 1000, 1, 0)
    build = lambda c, hb, val, hot, wsb: lib.gee_csr_build(c, hb, FAKE, FAKE, val, hot, FAKE, wsb, FAKE, None)
    assert build(ctypes.byref(coo), 0, None, None, need) == gee.GEE_EINVAL  # weighted needs val
    assert build(ctypes.byref(coo), 0, FAKE, None, need - 1) == gee.GEE_EWORKSPACE
    assert build(None, 0, FAKE, None, need) == gee.GEE_EINVAL
    assert build(ctypes.byref(coo), -1, FAKE, None, need) == gee.GEE_EINVAL
    assert build(ctypes.byref(coo), 10, FAKE, None, need) == gee.GEE_EINVAL  # hot slots need hot_ids
    assert build(ctypes.byref(coo), 10, FAKE, FAKE, need) == gee.GEE_EWORKSPACE  # hot selection scratch


def test_python_binding_refuses_host_tensors(lib):
    with pytest.raises(ValueError):
        gee.counts(torch.zeros(4, dtype=torch.int32), 2)


def test_batch_argument_errors(lib):
    csr = gee.Csr(1000, 10_000, FAKE, FAKE, None, 0, None)
    o = gee.EmbedOpts(0, 0, None, None, 0)

    def ws(Ks, laps, zoff, ldz):
        st, keep = gee._batch_struct(None, Ks, laps, zoff, ldz, None)
        return lib.gee_embed_batch_workspace(ctypes.byref(csr), ctypes.byref(st), ctypes.byref(o))

    assert ws([5, 7, 3], [0, 1, 0], [0, 5, 12], 15) > 0
    assert ws([5, 7], [0, 0], [0, 5], 11) == 0  # block past ldz
    assert ws([5, 7], [0, 0], [0, 4], 20) == 0  # overlapping blocks
    assert ws([0, 7], [0, 0], [0, 5], 20) == 0  # K < 1
    assert ws([4097], [0], [0], 5000) == 0  # K above the batched limit (one group's classes)
    assert ws([4096], [1], [0], 4096) > 0
    assert ws([5], [0], [0], 1 << 31) == 0  # Z column ids must fit 32 bits
    assert ws([5, 7], [0, 0], [7, 0], 20) > 0  # any column order
    big = ws([50] * 64, [0] * 64, [50 * i for i in range(64)], 3200)
    lap = ws([50] * 64, [1] * 64, [50 * i for i in range(64)], 3200)
    assert big > 0 and lap > big  # degrees and d^-1/2 for the Laplacian vectors
    for g, ok in ((0, True), (1, True), (64, True), (-1, False), (65, False)):
        o.group_vectors = g
        assert (ws([5, 7, 3], [0, 1, 0], [0, 5, 12], 15) > 0) == ok, g
    o.group_vectors = 16  # four groups of 16: smaller label matrices than one group of 64
    assert 0 < ws([50] * 64, [0] * 64, [50 * i for i in range(64)], 3200) < big
    o.group_vectors = 0
    st, keep = gee._batch_struct(None, [5], [0], [0], 5, None)
    assert lib.gee_embed_batch(ctypes.byref(csr), ctypes.byref(st), FAKE, 1 << 30, FAKE, None, None) == gee.GEE_EINVAL


def test_noalloc_argument_errors(lib):
    """The static-scratch entry point checks its arguments as gee_embed does and refuses a
    call whose workspace exceeds the scratch before touching the GPU."""
    m = re.search(r"#define GEE_NOALLOC_SCRATCH_BYTES \((\d+)u << (\d+)\)", open(HEADER).read())
    assert m and int(m.group(1)) << int(m.group(2)) == gee.NOALLOC_SCRATCH_BYTES
    o = gee.EmbedOpts(0, 0, None, None)
    assert lib.gee_embed_noalloc(None, None, FAKE, 5, 0, FAKE, FAKE, ctypes.byref(o), None) == gee.GEE_EINVAL
    assert lib.gee_embed_noalloc(None, None, FAKE, 0, 0, FAKE, FAKE, ctypes.byref(o), None) == gee.GEE_EINVAL
    big_n = gee.NOALLOC_SCRATCH_BYTES // 8 + 1  # Laplacian records alone: 8 bytes a vertex
    big = gee.Coo(big_n, 0, None, None, None)
    assert lib.gee_embed_workspace(ctypes.byref(big), None, 5, 1, ctypes.byref(o)) > gee.NOALLOC_SCRATCH_BYTES
    assert lib.gee_embed_noalloc(ctypes.byref(big), None, FAKE, 5, 1, FAKE, FAKE, ctypes.byref(o), None) == \
        gee.GEE_EWORKSPACE
    rp = gee.Csr(big_n, 0, FAKE, None, None, 0, None)
    assert lib.gee_embed_noalloc(None, ctypes.byref(rp), FAKE, 5, 1, FAKE, FAKE, ctypes.byref(o), None) == \
        gee.GEE_EWORKSPACE


def test_push_nonatomic_argument_errors(lib):
    """The atomics-off diagnostic needs the edge list (its push form has no CSR input)."""
    o = gee.EmbedOpts(0, 0, None, None)
    assert lib.gee_embed_push_nonatomic(None, FAKE, 5, 0, FAKE, FAKE, 1 << 30, FAKE, ctypes.byref(o), None) == \
        gee.GEE_EINVAL


def test_pb_argument_errors(lib):
    """Layout sizes and the checks done before anything launches."""
    assert lib.gee_pb_cells(0, 0) == 0
    assert lib.gee_pb_cells(256, 0) == 1
    assert lib.gee_pb_cells(257, 0) == 2
    assert lib.gee_pb_cells(256, 1) == 2  # one vertex column block + one tier slice
    assert lib.gee_pb_cells(256, 1 << 17) == 2
    assert lib.gee_pb_cells(256, (1 << 17) + 1) == 3
    assert lib.gee_pb_cells(256, 1 << 23) == 65
    assert lib.gee_pb_cells(256, 1 << 26) == 513  # 512 slices, the most
    assert lib.gee_pb_cells(256, (1 << 26) + 1) == 0
    assert lib.gee_pb_cells(256, -1) == 0
    assert lib.gee_pb_cells((1 << 21) + 1, 0) == 2 * ((((1 << 21) + 1) + 255) // 256)
    plain = gee.Csr(1000, 10_000, FAKE, FAKE, None, 0, None)
    hot = gee.Csr(1000, 10_000, FAKE, FAKE, None, 700, FAKE)
    weighted = gee.Csr(1000, 10_000, FAKE, FAKE, FAKE, 0, None)
    huge = gee.Csr(1000, (1 << 32) - 64, FAKE, FAKE, None, 0, None)
    bw = lambda c, tier, lap=0: lib.gee_pb_build_workspace(ctypes.byref(c), tier, lap)
    assert bw(plain, 0) > 10_000 * 16
    assert bw(plain, 1) == 0    # no hot slots to put in the tier
    assert bw(hot, 700) > 10_000 * 16
    assert bw(hot, 701) == 0
    assert bw(weighted, 0) > bw(plain, 0)
    assert bw(plain, 0, 1) > bw(weighted, 0)  # the terms and the degrees
    assert bw(huge, 0) == 0      # 32-bit cell lengths
    def build(c, tier, col=FAKE, ul=FAKE, word=FAKE, ids=FAKE, val=None, flag=None, meta=FAKE, wsb=1 << 40,
              lap=0, rsd=None):
        return lib.gee_pb_build(ctypes.byref(c), tier, lap, col, ul, FAKE, FAKE, word, ids, val, flag, rsd, meta,
                                FAKE, wsb, FAKE, None)

    assert build(huge, 0) == gee.GEE_EOVERFLOW
    assert build(hot, 700, ids=None) == gee.GEE_EINVAL  # lds_ids needed
    assert build(hot, 701) == gee.GEE_EINVAL  # more tier slots than hot slots
    assert build(plain, 0, ul=FAKE + 4) == gee.GEE_EINVAL  # ul 16-byte aligned
    assert build(plain, 0, word=None) == gee.GEE_EINVAL  # cell_word needed
    assert build(plain, 0, meta=None) == gee.GEE_EINVAL  # the fingerprint is written by every build
    assert build(plain, 0, val=FAKE, flag=FAKE) == gee.GEE_EINVAL  # no weights to lay out
    assert build(weighted, 0, val=FAKE, flag=None) == gee.GEE_EINVAL  # row-block flags needed
    assert build(weighted, 0, val=None, flag=FAKE) == gee.GEE_EINVAL  # weights needed
    assert build(weighted, 0, val=FAKE + 4, flag=FAKE) == gee.GEE_EINVAL  # weights 16-byte aligned
    assert build(weighted, 0, val=FAKE, flag=FAKE, wsb=bw(weighted, 0) - 1) == gee.GEE_EWORKSPACE
    assert build(plain, 0, lap=1, val=FAKE, flag=FAKE) == gee.GEE_EINVAL  # d^-1/2 output needed
    assert build(plain, 0, lap=1, rsd=FAKE) == gee.GEE_EINVAL  # Laplacian terms and flags needed
    assert build(plain, 0, rsd=FAKE) == gee.GEE_EINVAL  # d^-1/2 only for a Laplacian layout
    assert build(plain, 0, lap=1, val=FAKE, flag=FAKE, rsd=FAKE, wsb=bw(plain, 0, 1) - 1) == gee.GEE_EWORKSPACE
    # the tier planner: nothing to plan without hot slots; checks before any launch
    assert lib.gee_pb_tier_slots(ctypes.byref(plain), 4, None, 0, None) == 0
    assert lib.gee_pb_tier_slots(ctypes.byref(hot), 4, None, 0, None) == gee.GEE_EWORKSPACE
    assert lib.gee_pb_tier_slots(ctypes.byref(hot), -1, FAKE, 512, None) == gee.GEE_EINVAL
    assert lib.gee_pb_tier_slots(ctypes.byref(hot), 4, FAKE, 256, None) == gee.GEE_EWORKSPACE
    assert lib.gee_pb_tier_slots(None, 4, FAKE, 256, None) == gee.GEE_EINVAL
    pb = gee.Pb(1000, 10_000, 4, 1, FAKE, FAKE, FAKE, FAKE, 0, None, FAKE, None, None, FAKE)
    assert lib.gee_embed_pb_workspace(ctypes.byref(pb), 255) > 10_000
    assert lib.gee_embed_pb_workspace(ctypes.byref(pb), 256) == 0
    assert lib.gee_embed_pb_workspace(ctypes.byref(pb), 0) == 0
    tiered = gee.Pb(1000, 10_000, 4, 2, FAKE, FAKE, FAKE, FAKE, 5, FAKE, FAKE, None, None, FAKE)
    assert lib.gee_embed_pb_workspace(ctypes.byref(tiered), 8) > 10_000
    weighted_pb = gee.Pb(1000, 10_000, 4, 1, FAKE, FAKE, FAKE, FAKE, 0, None, FAKE, FAKE, FAKE, FAKE)
    assert lib.gee_embed_pb_workspace(ctypes.byref(weighted_pb), 8) > 10_000
    assert lib.gee_embed_pb_workspace(ctypes.byref(tiered), 8) > 10_000
    o = gee.EmbedOpts(0, 0, None, None)
    def P(n_rb=4, n_cb=1, col=FAKE, ul=FAKE, n_lds=0, ids=None, word=FAKE, val=None, flag=None, meta=FAKE, rsd=None):
        return gee.Pb(1000, 10_000, n_rb, n_cb, col, ul, FAKE, FAKE, n_lds, ids, word, val, flag, meta, rsd)

    for bad in (P(n_rb=5),  # n_rb does not match n
                P(n_lds=5, ids=FAKE),  # n_cb without the tier slice
                P(n_cb=2, n_lds=5),  # tier slots without ids
                P(n_cb=514, n_lds=(1 << 26) + 1, ids=FAKE),  # tier above 2^26
                P(col=FAKE + 4),  # col unaligned
                P(ul=FAKE + 8),  # ul unaligned
                P(word=None),  # no word prefix
                P(meta=None),  # no fingerprint
                P(val=FAKE),  # weights without row-block flags
                P(flag=FAKE),  # row-block flags without weights
                P(val=FAKE + 4, flag=FAKE),  # weights unaligned
                P(rsd=FAKE)):  # d^-1/2 without terms
        assert lib.gee_embed_pb_workspace(ctypes.byref(bad), 8) == 0
        assert lib.gee_embed_pb(ctypes.byref(bad), FAKE, 8, FAKE, FAKE, 1 << 30, FAKE, ctypes.byref(o), None) == \
            gee.GEE_EINVAL


def test_capture_and_tune_argument_errors(lib):
    """Recording needs a real stream and a handle; the tuner checks its candidates first."""
    h = ctypes.c_void_p()
    assert lib.gee_capture_begin(None) == gee.GEE_EINVAL
    assert lib.gee_capture_end(None, ctypes.byref(h)) == gee.GEE_EINVAL
    assert lib.gee_capture_end(FAKE, None) == gee.GEE_EINVAL
    assert lib.gee_graph_launch(None, None) == gee.GEE_EINVAL
    lib.gee_graph_destroy(None)  # ignored
    best, group, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_float()
    c = (ctypes.c_int32 * 2)(4096, 8192)
    bad = (ctypes.c_int32 * 2)(4096, 100)  # not a multiple of 64
    g = (ctypes.c_int32 * 2)(64, 32)
    gbad = (ctypes.c_int32 * 2)(64, 65)  # more than 64 vectors per group
    csr = gee.Csr(1000, 10_000, FAKE, FAKE, None, 0, None)
    st = gee.Batch(1, FAKE, None, None, None, 8, FAKE)
    for args in ((c, 0, g, 2, 3), (c, 2, g, 2, 0), (bad, 2, g, 2, 3), (c, 2, gbad, 2, 3), (c, 2, None, 2, 3),
                 (c, 2, g, -1, 3)):
        assert lib.gee_embed_batch_tune(ctypes.byref(csr), ctypes.byref(st), args[0], args[1], args[2], args[3],
                                        args[4], FAKE, 1 << 30, FAKE, None, ctypes.byref(best), ctypes.byref(group),
                                        ctypes.byref(ms)) == gee.GEE_EINVAL
    assert lib.gee_embed_batch_tune(ctypes.byref(csr), ctypes.byref(st), c, 2, g, 2, 3, FAKE, 1 << 30, FAKE, None, None,
                                    ctypes.byref(group), ctypes.byref(ms)) == gee.GEE_EINVAL


def test_argmax_argument_errors(lib):
    """Checks done before anything launches: buffers, sizes, K within ldz, distinct labels and prev."""
    E = gee.GEE_EINVAL
    assert lib.gee_argmax(None, 10, 5, 5, None, FAKE, None, None) == E
    assert lib.gee_argmax(FAKE, 10, 5, 5, None, None, None, None) == E
    assert lib.gee_argmax(FAKE, 0, 5, 5, None, FAKE, None, None) == E
    assert lib.gee_argmax(FAKE, 10, 0, 5, None, FAKE, None, None) == E
    assert lib.gee_argmax(FAKE, 10, 6, 5, None, FAKE, None, None) == E  # K above ldz
    assert lib.gee_argmax(FAKE, 10, 5, 5, FAKE, FAKE, None, None) == E  # labels overwrite prev
