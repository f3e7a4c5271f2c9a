"""MI355X-native one-hot graph encoder embedding (GEE).

A thin ctypes binding over ``libgee.so`` (hand-written HIP for gfx950; C ABI in
``include/gee.h``). PyTorch supplies device memory and the current stream; every step
of the computation runs in the library's kernels. There is no CPU fallback: without a
built library or a GPU every compute call raises.

Functions mirror the C entry points:

* :func:`counts`   — ``gee_counts``: class counts n_k (Algorithm 1's count(Y = k)).
* :func:`weights`  — ``gee_weights``: inv[k] = 1 / n_k, the nonzeros of W.
* :func:`degrees`  — ``gee_degrees``: weighted degree d = (A + A^T) 1.
* :func:`csr_build` — ``gee_csr_build``: canonical symmetric CSR of A + A^T.
* :func:`embed`    — ``gee_embed``: Z by the edge-parallel push form (COO) or the
  deterministic CSR-pull form (CSR), adjacency or Laplacian version.
* :func:`embed_noalloc` — ``gee_embed_noalloc``: the same with the library's static
  scratch instead of a workspace, for callers that cannot allocate.
* :func:`embed_batch` — ``gee_embed_batch``: many label vectors over one graph, one CSR
  pass per group of up to 64 vectors.
* :func:`copy`     — ``gee_copy``: the streaming copy probe used for measurement.
"""
from __future__ import annotations

import ctypes
import time
import os
from dataclasses import dataclass

import torch  # loads the HIP runtime libgee.so must share: import before the library

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgee.so")

GEE_OK, GEE_EINVAL, GEE_ELABEL, GEE_EVERTEX, GEE_ENEGW, GEE_EOVERFLOW, GEE_EWORKSPACE, GEE_EHIP = 0, -1, -2, -3, -4, -5, -6, -7

# Hot-vertex slots the benchmark configuration gives a CSR: a 4 MiB table of 1-byte
# label records in degree-rank order, so the hottest labels share the lines that stay
# in one XCD's 4 MiB L2 beside the streaming traffic.
DEFAULT_HOT_BUDGET = 1 << 22
# Hot slots for a graph embedded through its propagation-blocked layout: the entries of
# the 2^23 highest-degree vertices read their labels from LDS (64 tier slices).
PB_HOT_BUDGET = 1 << 23


class GeeError(RuntimeError):
    def __init__(self, code: int, where: str = ""):
        self.code = int(code)
        msg = _lib_or_none().gee_strerror(self.code).decode() if _lib_or_none() else str(code)
        super().__init__(f"{where}: {msg} ({self.code})" if where else f"{msg} ({self.code})")


class Coo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("s", ctypes.c_int64), ("src", ctypes.c_void_p),
                ("dst", ctypes.c_void_p), ("w", ctypes.c_void_p)]


class Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("val", ctypes.c_void_p), ("n_hot", ctypes.c_int64),
                ("hot_ids", ctypes.c_void_p)]


class Pb(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("n_rb", ctypes.c_int64), ("n_cb", ctypes.c_int32),
                ("col", ctypes.c_void_p), ("ul", ctypes.c_void_p), ("cell_start", ctypes.c_void_p),
                ("cell_count", ctypes.c_void_p), ("n_lds", ctypes.c_int64), ("lds_ids", ctypes.c_void_p),
                ("cell_word", ctypes.c_void_p), ("val", ctypes.c_void_p), ("rb_flag", ctypes.c_void_p),
                ("meta", ctypes.c_void_p), ("rsd", ctypes.c_void_p)]


class Batch(ctypes.Structure):
    _fields_ = [("B", ctypes.c_int32), ("labels", ctypes.c_void_p), ("K", ctypes.POINTER(ctypes.c_int32)),
                ("laplacian", ctypes.POINTER(ctypes.c_int32)), ("zoff", ctypes.POINTER(ctypes.c_int64)),
                ("ldz", ctypes.c_int64), ("Z", ctypes.c_void_p)]


class EmbedOpts(ctypes.Structure):
    _fields_ = [("seg_len", ctypes.c_int32), ("rows_per_window", ctypes.c_int32),
                ("hot_begin", ctypes.c_void_p), ("hot_end", ctypes.c_void_p), ("group_vectors", ctypes.c_int32)]


_lib = None


def _lib_or_none():
    return _lib


def load():
    """Load libgee.so (built in-tree by ``build.py``); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libgee.so not built at {LIB_PATH}; run paper_2402_04403_amd/build.py")
        lib = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, sz, ci = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_int
        CooP, CsrP, OptP = ctypes.POINTER(Coo), ctypes.POINTER(Csr), ctypes.POINTER(EmbedOpts)
        lib.gee_strerror.restype = ctypes.c_char_p
        lib.gee_strerror.argtypes = [ci]
        lib.gee_counts.restype = ci
        lib.gee_counts.argtypes = [vp, i64, i32, vp, vp, vp]
        lib.gee_weights.restype = ci
        lib.gee_weights.argtypes = [vp, i32, vp, vp]
        lib.gee_degrees.restype = ci
        lib.gee_degrees.argtypes = [CooP, CsrP, vp, vp, vp]
        lib.gee_embed_workspace.restype = sz
        lib.gee_embed_workspace.argtypes = [CooP, CsrP, i32, ci, OptP]
        lib.gee_embed.restype = ci
        lib.gee_embed.argtypes = [CooP, CsrP, vp, i32, ci, vp, vp, sz, vp, OptP, vp]
        lib.gee_embed_noalloc.restype = ci
        lib.gee_embed_noalloc.argtypes = [CooP, CsrP, vp, i32, ci, vp, vp, OptP, vp]
        PbP = ctypes.POINTER(Pb)
        lib.gee_pb_cells.restype = i64
        lib.gee_pb_cells.argtypes = [i64, i64]
        lib.gee_pb_tier_slots.restype = i64
        lib.gee_pb_tier_slots.argtypes = [CsrP, i64, vp, sz, vp]
        lib.gee_pb_build_workspace.restype = sz
        lib.gee_pb_build_workspace.argtypes = [CsrP, i64, ci]
        lib.gee_pb_build.restype = ci
        # csr, n_lds, laplacian, col, ul, cell_start, cell_count, cell_word, lds_ids, val, rb_flag, rsd,
        # meta, ws, ws_bytes, err, stream
        lib.gee_pb_build.argtypes = [CsrP, i64, ci] + [vp] * 11 + [sz, vp, vp]
        lib.gee_embed_pb_workspace.restype = sz
        lib.gee_embed_pb_workspace.argtypes = [PbP, i32]
        lib.gee_embed_pb.restype = ci
        lib.gee_embed_pb.argtypes = [PbP, vp, i32, vp, vp, sz, vp, OptP, vp]
        lib.gee_embed_push_nonatomic.restype = ci
        lib.gee_embed_push_nonatomic.argtypes = [CooP, vp, i32, ci, vp, vp, sz, vp, OptP, vp]
        lib.gee_csr_workspace.restype = sz
        lib.gee_csr_workspace.argtypes = [i64, i64, ci, i64]
        lib.gee_csr_build.restype = ci
        lib.gee_csr_build.argtypes = [CooP, i64, vp, vp, vp, vp, vp, sz, vp, vp]
        BatchP = ctypes.POINTER(Batch)
        lib.gee_embed_batch_workspace.restype = sz
        lib.gee_embed_batch_workspace.argtypes = [CsrP, BatchP, OptP]
        lib.gee_embed_batch.restype = ci
        lib.gee_embed_batch.argtypes = [CsrP, BatchP, vp, sz, vp, OptP, vp]
        lib.gee_embed_batch_tune.restype = ci
        lib.gee_embed_batch_tune.argtypes = [CsrP, BatchP, ctypes.POINTER(ctypes.c_int32), ci,
                                             ctypes.POINTER(ctypes.c_int32), ci, ci, vp, sz, vp, vp,
                                             ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                             ctypes.POINTER(ctypes.c_float)]
        lib.gee_argmax.restype = ci
        lib.gee_argmax.argtypes = [vp, i64, i32, i64, vp, vp, vp, vp]
        lib.gee_capture_begin.restype = ci
        lib.gee_capture_begin.argtypes = [vp]
        lib.gee_capture_end.restype = ci
        lib.gee_capture_end.argtypes = [vp, ctypes.POINTER(vp)]
        lib.gee_graph_launch.restype = ci
        lib.gee_graph_launch.argtypes = [vp, vp]
        lib.gee_graph_destroy.restype = None
        lib.gee_graph_destroy.argtypes = [vp]
        lib.gee_copy.restype = ci
        lib.gee_copy.argtypes = [vp, vp, sz, vp]
        _lib = lib
    return _lib


# ------------------------------------------------------------------ helpers --

def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _ptr(t):
    return None if t is None else t.data_ptr()


def _need(t, dtype, numel, name, device):
    if t is None:
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous {dtype} tensor")
    if t.device.type != "cuda" or (device is not None and t.device != device):
        raise ValueError(f"{name}: expected a tensor on {device or 'a GPU'}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name}: expected {numel} elements, got {t.numel()}")


def _rc(code, where):
    if code != GEE_OK:
        raise GeeError(code, where)


def _check_err(err: torch.Tensor, where: str):
    code = int(err.item())  # synchronises the stream the call ran on
    if code != GEE_OK:
        raise GeeError(code, where)


class HipEvent:
    """A HIP event created through the HIP runtime torch uses (plumbing for timing)."""

    _hip = None

    def __init__(self):
        if HipEvent._hip is None:
            load()
            hip = ctypes.CDLL("libamdhip64.so.7")  # resolves to the runtime already loaded
            hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
            hip.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
            hip.hipEventSynchronize.argtypes = [ctypes.c_void_p]
            hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
            hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
            hip.hipEventQuery.argtypes = [ctypes.c_void_p]
            HipEvent._hip = hip
        self.handle = ctypes.c_void_p()
        if HipEvent._hip.hipEventCreate(ctypes.byref(self.handle)) != 0:
            raise RuntimeError("hipEventCreate failed")

    def record(self, stream=None):
        if HipEvent._hip.hipEventRecord(self.handle, ctypes.c_void_p(_stream(stream))) != 0:
            raise RuntimeError("hipEventRecord failed")

    def synchronize(self):
        HipEvent._hip.hipEventSynchronize(self.handle)

    def done(self) -> bool:
        """True once the work recorded before the event has completed (hipEventQuery)."""
        rc = HipEvent._hip.hipEventQuery(self.handle)
        if rc not in (0, 600):  # hipSuccess, hipErrorNotReady
            raise RuntimeError(f"hipEventQuery failed ({rc})")
        return rc == 0

    def elapsed_ms(self, end: "HipEvent") -> float:
        ms = ctypes.c_float()
        if HipEvent._hip.hipEventElapsedTime(ctypes.byref(ms), self.handle, end.handle) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return float(ms.value)

    def __del__(self):
        try:
            if self.handle and HipEvent._hip is not None:
                HipEvent._hip.hipEventDestroy(self.handle)
        except Exception:
            pass


# ------------------------------------------------------------------ graphs --

@dataclass
class DeviceCoo:
    n: int
    src: torch.Tensor
    dst: torch.Tensor
    w: torch.Tensor | None = None

    @property
    def s(self) -> int:
        return int(self.src.numel())

    def struct(self) -> Coo:
        dev = self.src.device
        _need(self.src, torch.int32, None, "src", dev)
        _need(self.dst, torch.int32, self.s, "dst", dev)
        if self.w is not None:
            _need(self.w, torch.float32, self.s, "w", dev)
        return Coo(self.n, self.s, _ptr(self.src), _ptr(self.dst), _ptr(self.w))


@dataclass
class DeviceCsr:
    """Symmetric CSR on the GPU. With ``hot_ids`` set, a column with bit 31 set names
    slot ``col & 0x7fffffff`` of ``hot_ids`` instead of a vertex."""

    n: int
    row_ptr: torch.Tensor
    col: torch.Tensor
    val: torch.Tensor | None = None
    hot_ids: torch.Tensor | None = None

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    @property
    def n_hot(self) -> int:
        return 0 if self.hot_ids is None else int(self.hot_ids.numel())

    def struct(self) -> Csr:
        # the checked struct is kept while the fields name the same buffers (serving loops
        # call this once per launch)
        key = (self.n, _ptr(self.row_ptr), _ptr(self.col), self.nnz, _ptr(self.val), _ptr(self.hot_ids), self.n_hot)
        got = self.__dict__.get("_struct")
        if got is not None and got[0] == key:
            return got[1]
        dev = self.row_ptr.device
        _need(self.row_ptr, torch.int64, self.n + 1, "row_ptr", dev)
        _need(self.col, torch.int32, None, "col", dev)
        if self.val is not None:
            _need(self.val, torch.float32, self.nnz, "val", dev)
        if self.hot_ids is not None:
            _need(self.hot_ids, torch.int32, None, "hot_ids", dev)
        st = Csr(self.n, self.nnz, _ptr(self.row_ptr), _ptr(self.col), _ptr(self.val), self.n_hot,
                 _ptr(self.hot_ids))
        self.__dict__["_struct"] = (key, st)
        return st

    def plain_col(self) -> torch.Tensor:
        """Columns as vertex ids (hot slots resolved)."""
        if self.hot_ids is None:
            return self.col
        hot = self.col < 0
        slot = (self.col & 0x7FFFFFFF).long()
        return torch.where(hot, self.hot_ids[slot.clamp(max=max(self.n_hot - 1, 0))], self.col)


def to_device(n: int, src, dst, w=None, device="cuda") -> DeviceCoo:
    """Copy a host edge list (NumPy or tensors) to the GPU as int32 / float32."""
    def t(a, dt):
        if a is None:
            return None
        a = torch.as_tensor(a)
        return a.to(device=device, dtype=dt).contiguous()
    return DeviceCoo(n, t(src, torch.int32), t(dst, torch.int32), t(w, torch.float32))


# --------------------------------------------------------------- entry points --

def counts(labels: torch.Tensor, K: int, stream=None, check: bool = True) -> torch.Tensor:
    lib = load()
    _need(labels, torch.int32, None, "labels", None)
    out = torch.empty(K + 1, dtype=torch.int64, device=labels.device)
    err = torch.zeros(1, dtype=torch.int32, device=labels.device)
    _rc(lib.gee_counts(_ptr(labels), labels.numel(), K, _ptr(out), _ptr(err), _stream(stream)), "gee_counts")
    if check:
        _check_err(err, "gee_counts")
    return out


def weights(cnt: torch.Tensor, K: int, stream=None) -> torch.Tensor:
    lib = load()
    _need(cnt, torch.int64, K + 1, "counts", None)
    inv = torch.empty(K + 1, dtype=torch.float64, device=cnt.device)
    _rc(lib.gee_weights(_ptr(cnt), K, _ptr(inv), _stream(stream)), "gee_weights")
    return inv


def degrees(coo: DeviceCoo | None = None, csr: DeviceCsr | None = None, stream=None, check: bool = True):
    lib = load()
    g = coo if coo is not None else csr
    if g is None:
        raise ValueError("degrees: give coo or csr")
    dev = (coo.src if coo is not None else csr.row_ptr).device
    deg = torch.empty(g.n, dtype=torch.float64, device=dev)
    err = torch.zeros(1, dtype=torch.int32, device=dev)
    cs = ctypes.byref(coo.struct()) if coo is not None else None
    rs = ctypes.byref(csr.struct()) if csr is not None else None
    _rc(lib.gee_degrees(cs, rs, _ptr(deg), _ptr(err), _stream(stream)), "gee_degrees")
    if check:
        _check_err(err, "gee_degrees")
    return deg


def csr_build(coo: DeviceCoo, hot_budget: int = 0, stream=None, check: bool = True) -> DeviceCsr:
    """Canonical symmetric CSR; ``hot_budget > 0`` gives the highest-degree vertices hot slots."""
    lib = load()
    st = coo.struct()
    dev = coo.src.device
    nnz = 2 * coo.s
    n_hot = min(int(hot_budget), coo.n)
    row_ptr = torch.empty(coo.n + 1, dtype=torch.int64, device=dev)
    col = torch.empty(nnz, dtype=torch.int32, device=dev)
    val = torch.empty(nnz, dtype=torch.float32, device=dev) if coo.w is not None else None
    hot_ids = torch.empty(n_hot, dtype=torch.int32, device=dev) if n_hot > 0 else None
    wsb = lib.gee_csr_workspace(coo.n, coo.s, 1 if coo.w is not None else 0, n_hot)
    if wsb == 0:
        raise GeeError(GEE_EINVAL, "gee_csr_workspace")
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    err = torch.zeros(1, dtype=torch.int32, device=dev)
    _rc(lib.gee_csr_build(ctypes.byref(st), n_hot, _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(hot_ids), _ptr(ws),
                          wsb, _ptr(err), _stream(stream)), "gee_csr_build")
    if check:
        _check_err(err, "gee_csr_build")
    del ws
    return DeviceCsr(coo.n, row_ptr, col, val, hot_ids)


PB_ROWS = 256
PB_COLS = 1 << 21
PB_SLICE = 1 << 17
PB_MAX_TIER = 1 << 26


@dataclass
class DevicePb:
    """Propagation-blocked layout of a CSR (entries by 2^21-vertex column block, then by
    tier slice of 2^17 hot slots; cells of 256-row blocks), with the entries' weights in
    layout order for a weighted CSR."""

    n: int
    col: torch.Tensor         # [nnz + 64] int32; tier slots (17 bits) packed from byte 4 H0
    ul: torch.Tensor          # [nnz + 32 rounded up to 16]
    cell_start: torch.Tensor
    cell_count: torch.Tensor
    lds_ids: torch.Tensor     # [n_lds]
    cell_word: torch.Tensor   # [n_rb * n_cb]
    nnz: int = 0
    meta: torch.Tensor | None = None     # [8] int64 fingerprint (and weight grid) written by the build
    val: torch.Tensor | None = None      # [nnz + 32 rounded up to 16] float32: w, or w d_u^-1/2 d_v^-1/2 (Laplacian)
    rb_flag: torch.Tensor | None = None  # [n_rb] uint8, weighted and Laplacian layouts
    rsd: torch.Tensor | None = None      # [n] float32 d^-1/2, Laplacian layouts

    @property
    def laplacian(self) -> bool:
        return self.rsd is not None

    @property
    def n_rb(self) -> int:
        return (self.n + PB_ROWS - 1) // PB_ROWS

    @property
    def n_cb(self) -> int:
        return (self.n + PB_COLS - 1) // PB_COLS + (self.n_lds + PB_SLICE - 1) // PB_SLICE

    @property
    def n_lds(self) -> int:
        return int(self.lds_ids.numel())

    def struct(self) -> Pb:
        return Pb(self.n, self.nnz, self.n_rb, self.n_cb, _ptr(self.col), _ptr(self.ul), _ptr(self.cell_start),
                  _ptr(self.cell_count), self.n_lds, _ptr(self.lds_ids) if self.n_lds else None,
                  _ptr(self.cell_word), _ptr(self.val), _ptr(self.rb_flag), _ptr(self.meta), _ptr(self.rsd))


def pb_tier_slots(csr: DeviceCsr, min_per_row_block: int = 4, stream=None) -> int:
    """Tier size for pb_build: leading slices of 2^17 hot slots whose entries average at
    least ``min_per_row_block`` per 256-row block (gee_pb_tier_slots; synchronizes)."""
    lib = load()
    ws = torch.empty(8 * 512, dtype=torch.uint8, device=csr.row_ptr.device)  # one count per slice
    r = int(lib.gee_pb_tier_slots(ctypes.byref(csr.struct()), min_per_row_block, _ptr(ws), ws.numel(),
                                  _stream(stream)))
    if r < 0:
        raise GeeError(r, "gee_pb_tier_slots")
    return r


def pb_build(csr: DeviceCsr, tier_slots: int | None = None, laplacian: bool = False, stream=None,
             check: bool = True) -> DevicePb:
    """Layout for gee_embed_pb from a CSR (per-graph preprocessing; a weighted CSR gives a
    weighted layout; ``laplacian`` a layout of the Laplacian version, with the degrees taken
    once here). The first ``tier_slots`` hot slots are read from LDS; None takes
    pb_tier_slots(csr)."""
    lib = load()
    rs = csr.struct()
    dev = csr.row_ptr.device
    n_lds = pb_tier_slots(csr, stream=stream) if tier_slots is None else int(tier_slots)
    cells = int(lib.gee_pb_cells(csr.n, n_lds))
    wsb = int(lib.gee_pb_build_workspace(ctypes.byref(rs), n_lds, 1 if laplacian else 0))
    if wsb == 0 or cells == 0:
        raise GeeError(GEE_EINVAL, "gee_pb_build_workspace")
    col = torch.empty(csr.nnz + 64, dtype=torch.int32, device=dev)
    ul = torch.empty((csr.nnz + 32 + 15) // 16 * 16, dtype=torch.uint8, device=dev)
    cell_start = torch.empty(cells, dtype=torch.int64, device=dev)
    cell_count = torch.empty(cells, dtype=torch.int32, device=dev)
    cell_word = torch.empty(cells, dtype=torch.int32, device=dev)
    lds_ids = torch.empty(n_lds, dtype=torch.int32, device=dev)
    meta = torch.empty(8, dtype=torch.int64, device=dev)
    carried = csr.val is not None or laplacian
    val = torch.empty((csr.nnz + 32 + 15) // 16 * 16, dtype=torch.float32, device=dev) if carried else None
    rb_flag = torch.empty((csr.n + PB_ROWS - 1) // PB_ROWS, dtype=torch.uint8, device=dev) if carried else None
    rsd = torch.empty(csr.n, dtype=torch.float32, device=dev) if laplacian else None
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    err = torch.zeros(1, dtype=torch.int32, device=dev)
    _rc(lib.gee_pb_build(ctypes.byref(rs), n_lds, 1 if laplacian else 0, _ptr(col), _ptr(ul), _ptr(cell_start),
                         _ptr(cell_count), _ptr(cell_word), _ptr(lds_ids) if n_lds else None, _ptr(val),
                         _ptr(rb_flag), _ptr(rsd), _ptr(meta), _ptr(ws), wsb, _ptr(err), _stream(stream)),
        "gee_pb_build")
    if check:
        _check_err(err, "gee_pb_build")
    del ws
    return DevicePb(csr.n, col, ul, cell_start, cell_count, lds_ids, cell_word, csr.nnz, meta, val, rb_flag, rsd)


def embed_pb_workspace_bytes(pb: DevicePb, K: int) -> int:
    return int(load().gee_embed_pb_workspace(ctypes.byref(pb.struct()), K))


def embed_pb(labels: torch.Tensor, K: int, pb: DevicePb, Z: torch.Tensor | None = None, ws: torch.Tensor | None = None,
             err: torch.Tensor | None = None, events=None, stream=None, check: bool = True) -> torch.Tensor:
    """Z [n, K] of a graph from its propagation-blocked layout, in the version the layout was
    built for (adjacency, or Laplacian for a layout built with ``laplacian``)."""
    lib = load()
    dev = pb.cell_start.device
    _need(labels, torch.int32, pb.n, "labels", dev)
    st = pb.struct()
    wsb = int(lib.gee_embed_pb_workspace(ctypes.byref(st), K))
    if wsb == 0:
        raise GeeError(GEE_EINVAL, "gee_embed_pb_workspace")
    if Z is None:
        Z = torch.empty((pb.n, K), dtype=torch.float32, device=dev)
    _need(Z, torch.float32, pb.n * K, "Z", dev)
    if ws is None or ws.numel() < wsb:
        ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    if err is None:
        err = torch.zeros(1, dtype=torch.int32, device=dev)
    o = _opts(0, 0, events)
    _rc(lib.gee_embed_pb(ctypes.byref(st), _ptr(labels), K, _ptr(Z), _ptr(ws), ws.numel(), _ptr(err),
                         ctypes.byref(o), _stream(stream)), "gee_embed_pb")
    if check:
        _check_err(err, "gee_embed_pb")
    return Z


def _opts(seg_len=0, rows_per_window=0, events=None, group_vectors=0):
    o = EmbedOpts(seg_len, rows_per_window, None, None, group_vectors)
    if events is not None:
        o.hot_begin, o.hot_end = events[0].handle, events[1].handle
    return o


def embed_workspace_bytes(K: int, coo: DeviceCoo | None = None, csr: DeviceCsr | None = None,
                          laplacian: bool = False, seg_len: int = 0, rows_per_window: int = 0) -> int:
    lib = load()
    cs = ctypes.byref(coo.struct()) if coo is not None else None
    rs = ctypes.byref(csr.struct()) if csr is not None else None
    o = _opts(seg_len, rows_per_window)
    return int(lib.gee_embed_workspace(cs, rs, K, 1 if laplacian else 0, ctypes.byref(o)))


def embed(labels: torch.Tensor, K: int, coo: DeviceCoo | None = None, csr: DeviceCsr | None = None,
          laplacian: bool = False, Z: torch.Tensor | None = None, ws: torch.Tensor | None = None,
          err: torch.Tensor | None = None, seg_len: int = 0, rows_per_window: int = 0, events=None,
          stream=None, check: bool = True) -> torch.Tensor:
    """GEE embedding Z [n, K] (FP32). ``csr`` selects the CSR-pull form, else the push form on ``coo``."""
    lib = load()
    g = csr if csr is not None else coo
    if g is None:
        raise ValueError("embed: give coo (push form) or csr (pull form)")
    dev = (csr.row_ptr if csr is not None else coo.src).device
    _need(labels, torch.int32, g.n, "labels", dev)
    cs = ctypes.byref(coo.struct()) if (coo is not None and csr is None) else None
    rs = ctypes.byref(csr.struct()) if csr is not None else None
    o = _opts(seg_len, rows_per_window, events)
    wsb = int(lib.gee_embed_workspace(cs, rs, K, 1 if laplacian else 0, ctypes.byref(o)))
    if wsb == 0:
        raise GeeError(GEE_EINVAL, "gee_embed_workspace")
    if Z is None:
        Z = torch.empty((g.n, K), dtype=torch.float32, device=dev)
    _need(Z, torch.float32, g.n * K, "Z", dev)
    if ws is None or ws.numel() < wsb:
        ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    if err is None:
        err = torch.zeros(1, dtype=torch.int32, device=dev)
    _rc(lib.gee_embed(cs, rs, _ptr(labels), K, 1 if laplacian else 0, _ptr(Z), _ptr(ws), ws.numel(), _ptr(err),
                      ctypes.byref(o), _stream(stream)), "gee_embed")
    if check:
        _check_err(err, "gee_embed")
    return Z


# Bytes of the library's static scratch used by gee_embed_noalloc (GEE_NOALLOC_SCRATCH_BYTES).
NOALLOC_SCRATCH_BYTES = 64 << 20


def embed_noalloc(labels: torch.Tensor, K: int, Z: torch.Tensor, err: torch.Tensor, coo: DeviceCoo | None = None,
                  csr: DeviceCsr | None = None, laplacian: bool = False, seg_len: int = 0, rows_per_window: int = 0,
                  stream=None, check: bool = True) -> torch.Tensor:
    """``gee_embed_noalloc``: the embedding with the library's static scratch in place of a
    workspace, for callers that cannot allocate. The caller passes Z and the error word;
    the library allocates nothing. Calls that overlap on one GPU race on the scratch."""
    lib = load()
    g = csr if csr is not None else coo
    if g is None:
        raise ValueError("embed_noalloc: give coo (push form) or csr (pull form)")
    dev = (csr.row_ptr if csr is not None else coo.src).device
    _need(labels, torch.int32, g.n, "labels", dev)
    _need(Z, torch.float32, g.n * K, "Z", dev)
    _need(err, torch.int32, 1, "err", dev)
    cs = ctypes.byref(coo.struct()) if (coo is not None and csr is None) else None
    rs = ctypes.byref(csr.struct()) if csr is not None else None
    o = _opts(seg_len, rows_per_window)
    _rc(lib.gee_embed_noalloc(cs, rs, _ptr(labels), K, 1 if laplacian else 0, _ptr(Z), _ptr(err), ctypes.byref(o),
                              _stream(stream)), "gee_embed_noalloc")
    if check:
        _check_err(err, "gee_embed_noalloc")
    return Z


def embed_push_nonatomic(labels: torch.Tensor, K: int, coo: DeviceCoo, laplacian: bool = False,
                         Z: torch.Tensor | None = None, ws: torch.Tensor | None = None,
                         err: torch.Tensor | None = None, events=None, stream=None, check: bool = True) -> torch.Tensor:
    """Diagnostic only, not the embedding: the push form with plain (racing) updates of Z,
    the paper's atomics-off measurement. Z is wrong wherever two records update one element."""
    lib = load()
    dev = coo.src.device
    _need(labels, torch.int32, coo.n, "labels", dev)
    cs = ctypes.byref(coo.struct())
    o = _opts(0, 0, events)
    wsb = int(lib.gee_embed_workspace(cs, None, K, 1 if laplacian else 0, ctypes.byref(o)))
    if wsb == 0:
        raise GeeError(GEE_EINVAL, "gee_embed_workspace")
    if Z is None:
        Z = torch.empty((coo.n, K), dtype=torch.float32, device=dev)
    _need(Z, torch.float32, coo.n * K, "Z", dev)
    if ws is None or ws.numel() < wsb:
        ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    if err is None:
        err = torch.zeros(1, dtype=torch.int32, device=dev)
    _rc(lib.gee_embed_push_nonatomic(cs, _ptr(labels), K, 1 if laplacian else 0, _ptr(Z), _ptr(ws), ws.numel(),
                                     _ptr(err), ctypes.byref(o), _stream(stream)), "gee_embed_push_nonatomic")
    if check:
        _check_err(err, "gee_embed_push_nonatomic")
    return Z


def _batch_struct(labels, Ks, laps, zoff, ldz, Z):
    B = len(Ks)
    K_arr = (ctypes.c_int32 * B)(*[int(k) for k in Ks])
    L_arr = (ctypes.c_int32 * B)(*[1 if x else 0 for x in laps])
    Z_arr = (ctypes.c_int64 * B)(*[int(z) for z in zoff])
    st = Batch(B, _ptr(labels), ctypes.cast(K_arr, ctypes.POINTER(ctypes.c_int32)),
               ctypes.cast(L_arr, ctypes.POINTER(ctypes.c_int32)), ctypes.cast(Z_arr, ctypes.POINTER(ctypes.c_int64)),
               int(ldz), _ptr(Z))
    return st, (K_arr, L_arr, Z_arr)


def embed_batch(labels: torch.Tensor, Ks, laplacian, csr: DeviceCsr, Z: torch.Tensor | None = None, zoff=None,
                ws: torch.Tensor | None = None, err: torch.Tensor | None = None, seg_len: int = 0, events=None,
                stream=None, check: bool = True, group_vectors: int = 0):
    """Embed B label vectors (``labels`` [B, n] int32) over one graph in one pass per group
    (at most ``group_vectors`` vectors per group; 0 is the library's 64).

    ``Ks[b]`` and ``laplacian[b]`` give each vector's classes and version. By default the blocks
    are packed side by side: Z is [n, sum(Ks)] and vector b owns columns zoff[b] .. zoff[b]+Ks[b].
    A given ``ws`` must hold ``embed_batch_workspace_bytes`` (else GeeError GEE_EWORKSPACE).
    Returns (Z, zoff)."""
    lib = load()
    B = len(Ks)
    dev = csr.row_ptr.device
    _need(labels, torch.int32, B * csr.n, "labels", dev)
    if zoff is None:
        zoff, acc = [], 0
        for k in Ks:
            zoff.append(acc)
            acc += int(k)
    if Z is None:
        Z = torch.empty((csr.n, int(max(z + k for z, k in zip(zoff, Ks)))), dtype=torch.float32, device=dev)
    if Z.dim() != 2 or Z.shape[0] != csr.n or not Z.is_contiguous() or Z.dtype != torch.float32:
        raise ValueError("Z: expected a contiguous float32 [n, ldz] tensor")
    st, keep = _batch_struct(labels, Ks, laplacian, zoff, Z.shape[1], Z)
    rs = csr.struct()
    o = _opts(seg_len, 0, events, group_vectors)
    if ws is None:  # a given workspace is checked by the library (GEE_EWORKSPACE when short)
        wsb = int(lib.gee_embed_batch_workspace(ctypes.byref(rs), ctypes.byref(st), ctypes.byref(o)))
        if wsb == 0:
            raise GeeError(GEE_EINVAL, "gee_embed_batch_workspace")
        ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    if err is None:
        err = torch.zeros(1, dtype=torch.int32, device=dev)
    _rc(lib.gee_embed_batch(ctypes.byref(rs), ctypes.byref(st), _ptr(ws), ws.numel(), _ptr(err), ctypes.byref(o),
                            _stream(stream)), "gee_embed_batch")
    del keep
    if check:
        _check_err(err, "gee_embed_batch")
    return Z, list(zoff)


def embed_batch_tune(labels: torch.Tensor, Ks, laplacian, csr: DeviceCsr, seg_lens=(2048, 4096, 8192, 16384, 32768),
                     group_vectors=(0,), reps: int = 3, Z: torch.Tensor | None = None, zoff=None, stream=None):
    """Segment length and group size for embed_batch on this graph and batch
    (``gee_embed_batch_tune``): times every pair of candidates and returns (best seg_len,
    best group_vectors, mean ms per call). group_vectors 0 is the library's 64. Synchronizes."""
    lib = load()
    B = len(Ks)
    dev = csr.row_ptr.device
    _need(labels, torch.int32, B * csr.n, "labels", dev)
    if zoff is None:
        zoff, acc = [], 0
        for k in Ks:
            zoff.append(acc)
            acc += int(k)
    if Z is None:
        Z = torch.empty((csr.n, int(max(z + k for z, k in zip(zoff, Ks)))), dtype=torch.float32, device=dev)
    st, keep = _batch_struct(labels, Ks, laplacian, zoff, Z.shape[1], Z)
    rs = csr.struct()
    sizes = [int(lib.gee_embed_batch_workspace(ctypes.byref(rs), ctypes.byref(st), ctypes.byref(_opts(L, 0, None, G))))
             for L in seg_lens for G in group_vectors]
    wsb = max(sizes) if min(sizes) > 0 else 0
    if wsb == 0:
        raise GeeError(GEE_EINVAL, "gee_embed_batch_workspace")
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    err = torch.zeros(1, dtype=torch.int32, device=dev)
    cands = (ctypes.c_int32 * len(seg_lens))(*[int(x) for x in seg_lens])
    gcands = (ctypes.c_int32 * len(group_vectors))(*[int(x) for x in group_vectors])
    best, bestg, ms = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_float(0.0)
    _rc(lib.gee_embed_batch_tune(ctypes.byref(rs), ctypes.byref(st), cands, len(seg_lens), gcands, len(group_vectors),
                                 int(reps), _ptr(ws), wsb, _ptr(err), _stream(stream), ctypes.byref(best),
                                 ctypes.byref(bestg), ctypes.byref(ms)),
        "gee_embed_batch_tune")
    del keep
    _check_err(err, "gee_embed_batch_tune")
    return int(best.value), int(bestg.value), float(ms.value)


class Graph:
    """Library calls recorded once (``gee_capture_begin`` / ``gee_capture_end``) and replayed
    with one launch each time; every replay reads what the recorded buffers hold then."""

    def __init__(self, handle: int, stream):
        self._h = handle
        self.stream = stream

    def replay(self, stream=None):
        if not self._h:
            raise RuntimeError("graph destroyed")
        _rc(load().gee_graph_launch(self._h, _stream(stream if stream is not None else self.stream)),
            "gee_graph_launch")

    def close(self):
        if self._h:
            load().gee_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def capture(fn, stream) -> Graph:
    """Record the library calls ``fn()`` makes on ``stream`` (a non-default torch stream) as
    a graph. ``fn`` must pass every buffer (Z, ws, err) and ``check=False``: nothing may be
    allocated or synchronized while recording."""
    lib = load()
    s = _stream(stream)
    _rc(lib.gee_capture_begin(s), "gee_capture_begin")
    h = ctypes.c_void_p()
    try:
        with torch.cuda.stream(stream):
            fn()
    except BaseException:
        lib.gee_capture_end(s, ctypes.byref(h))
        if h.value:
            lib.gee_graph_destroy(h)
        raise
    _rc(lib.gee_capture_end(s, ctypes.byref(h)), "gee_capture_end")
    return Graph(h.value, stream)


def argmax(Z: torch.Tensor, K: int | None = None, prev: torch.Tensor | None = None, out: torch.Tensor | None = None,
           changed: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Labels from an embedding (``gee_argmax``): 1 + the first column of each row's largest
    positive entry, 0 for a row without one. With ``prev``, ``changed`` (int64 [1]) gets the
    number of labels that differ from it."""
    lib = load()
    if Z.dim() != 2 or Z.dtype != torch.float32 or not Z.is_contiguous():
        raise ValueError("Z: expected a contiguous float32 [n, ldz] tensor")
    n, ldz = Z.shape
    K = ldz if K is None else int(K)
    dev = Z.device
    if out is None:
        out = torch.empty(n, dtype=torch.int32, device=dev)
    _need(out, torch.int32, n, "out", dev)
    if prev is not None:
        _need(prev, torch.int32, n, "prev", dev)
    _rc(lib.gee_argmax(_ptr(Z), n, K, ldz, _ptr(prev), _ptr(out), _ptr(changed), _stream(stream)), "gee_argmax")
    return out


def refine(labels: torch.Tensor, K: int, csr: DeviceCsr | None = None, pb: DevicePb | None = None,
           max_iter: int = 50, record: bool = True, stats: dict | None = None):
    """Refine a labelling by GEE: embed with the current labels, give every vertex the class
    of its largest entry of Z (``argmax``), repeat until no label changes, until a round
    changes no fewer labels than the round two before it (the synchronous updates have
    settled into a cycle), or ``max_iter`` rounds. Runs over the CSR (pull form) or the
    propagation-blocked layout. With ``record`` the two alternating rounds (labels A -> B
    and B -> A) are recorded once as graphs and replayed. Returns (labels, rounds run,
    changes per round); ``stats`` (if given) receives the recording and loop times in ms."""
    if (csr is None) == (pb is None):
        raise ValueError("refine: give csr or pb")
    n = (csr or pb).n
    dev = labels.device
    _need(labels, torch.int32, n, "labels", dev)
    bufs = [labels.clone(), torch.empty_like(labels)]
    Z = torch.empty((n, K), dtype=torch.float32, device=dev)
    wsb = embed_workspace_bytes(K, csr=csr) if csr is not None else embed_pb_workspace_bytes(pb, K)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    err = torch.zeros(1, dtype=torch.int32, device=dev)
    changed = torch.zeros(1, dtype=torch.int64, device=dev)
    stream = torch.cuda.Stream(device=dev)

    def round_(src, dst):
        if csr is not None:
            embed(src, K, csr=csr, Z=Z, ws=ws, err=err, stream=stream, check=False)
        else:
            embed_pb(src, K, pb, Z=Z, ws=ws, err=err, stream=stream, check=False)
        argmax(Z, K, prev=src, out=dst, changed=changed, stream=stream)

    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    graphs = None
    if record:
        graphs = [capture(lambda: round_(bufs[0], bufs[1]), stream), capture(lambda: round_(bufs[1], bufs[0]), stream)]
    t1 = time.perf_counter()
    history = []
    cur = 0
    for _ in range(max_iter):
        if graphs is not None:
            graphs[cur].replay(stream)
        else:
            round_(bufs[cur], bufs[1 - cur])
        stream.synchronize()
        cur = 1 - cur
        history.append(int(changed.item()))
        if history[-1] == 0 or (len(history) >= 3 and history[-1] >= history[-3]):
            break
    t2 = time.perf_counter()
    if stats is not None:
        stats["record_ms"] = (t1 - t0) * 1e3
        stats["loop_ms"] = (t2 - t1) * 1e3
    _check_err(err, "refine")
    if graphs is not None:
        for g in graphs:
            g.close()
    return bufs[cur], len(history), history


def embed_batch_workspace_bytes(n: int, Ks, laplacian, csr: DeviceCsr, seg_len: int = 0, zoff=None, ldz=None,
                                group_vectors: int = 0) -> int:
    lib = load()
    if zoff is None:
        zoff, acc = [], 0
        for k in Ks:
            zoff.append(acc)
            acc += int(k)
    ldz = ldz or int(max(z + k for z, k in zip(zoff, Ks)))
    st, keep = _batch_struct(None, Ks, laplacian, zoff, ldz, None)
    o = _opts(seg_len, 0, None, group_vectors)
    return int(lib.gee_embed_batch_workspace(ctypes.byref(csr.struct()), ctypes.byref(st), ctypes.byref(o)))


def copy(dst: torch.Tensor, src: torch.Tensor, stream=None) -> None:
    lib = load()
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nbytes:
        raise ValueError("copy: destination too small")
    _rc(lib.gee_copy(_ptr(dst), _ptr(src), nbytes, _stream(stream)), "gee_copy")
