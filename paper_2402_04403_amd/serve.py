"""A serving loop for GEE jobs on many graphs, on one GPU.

A job is a set of label vectors (each with its K and version) on one graph of a
pool. Jobs arrive over time. The server keeps graphs resident in HBM (the canonical
CSR is built on first use and reused by later jobs; least recently used graphs are
evicted when memory is needed), admits arrived jobs in arrival order while their
output and scratch fit an HBM budget, and at every poll launches all admitted jobs:
the jobs on one graph are fused into one ``gee_embed_batch`` call (continuous
batching: a job that arrives while others run joins the next launch), and calls on
different graphs go to different HIP streams so their work overlaps on the device; each
launch takes the stream with the least estimated work in flight.

A job's result does not depend on which other jobs share its launch: the batched
pass gives every vector its own bins, filled in CSR order, and the segmentation
depends only on the graph and the segment length. Optionally a job of few vectors on
a large graph (at most ``route_vectors`` vectors, default 0: none; at least
``route_items`` rows + entries) runs as one ``gee_embed`` call per vector instead,
inside the same launch: the batched pass gives its lanes to vectors, so a call with few
vectors leaves most lanes idle, while the plain pull gives them to entries. The choice
depends only on the job and its graph. It shortens such jobs but costs throughput when
jobs on one graph could have shared a batched call. Unit-weight adjacency vectors get the
same bits from either pass, so on a graph of at least ``route_items`` they follow the
load instead: a launch with no batched Laplacian work and at most ``route_adjacency``
adjacency vectors (default 0: off) runs them as plain calls.
Small graphs can be packed (``pack_items`` > 0): the graphs whose rows + entries are at
most ``pack_items`` are grouped, in id order, into disjoint-union CSRs of at most
``pack_limit`` rows + entries, and the jobs on all members of a pack run in one launch
over their union (each job's label rows hold zeros, unknown, outside its graph, and its
result is its graph's rows of Z). A member is always served through its pack, alone or
in a mix, so packing keeps every job's result independent of the mix; each vector then
writes the union's rows of Z, which costs little for small graphs.
``plain`` mode is the comparison: one job at a time, one ``gee_embed`` call per vector,
in arrival order.

Latency of a job = device completion of its launch minus its arrival, both on the
host clock (the completion is read from HIP events against a reference event).

A job that cannot be served comes back from ``poll`` as a ``Done`` with a nonzero
``error`` and no result, and the loop keeps serving: ``ERR_BUDGET`` when its launch can
never fit the HBM budget beside its graph, or the library's status code when the library
refuses the launch it is in (it checks arguments before queuing work).
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import (DEFAULT_HOT_BUDGET, DeviceCsr, GeeError, HipEvent, csr_build, embed, embed_batch,
               embed_workspace_bytes, to_device)

# Done.error of a job whose launch can never fit the HBM budget beside its graph (the
# library's own status codes are 0 and negative numbers above -100).
ERR_BUDGET = -100


@dataclass
class Request:
    jid: int
    gid: int
    Ks: list
    laplacian: list
    labels: torch.Tensor  # host int32 [B, n] (pinned for asynchronous upload)
    arrival: float        # host clock (time.perf_counter)


@dataclass
class Done:
    jid: int
    gid: int
    arrival: float
    finish: float
    records: int         # edge records of the graph
    vectors: int
    error: int = 0
    Z: torch.Tensor | None = None  # [n, sum K] when results are kept

    @property
    def latency(self) -> float:
        return self.finish - self.arrival


@dataclass
class _Graph:
    gid: int
    csr: DeviceCsr
    s: int
    bytes: int
    last_use: float = 0.0
    busy: int = 0


@dataclass
class _Launch:
    event: HipEvent
    reqs: list
    graph: _Graph
    bytes: int
    slot: int  # this launch's word of the error mirrors
    stream: int = 0
    work: float = 0.0  # estimated device bytes (Z written, entries read per vector)
    keep: list = field(default_factory=list)
    Z: torch.Tensor | None = None
    zoff: list | None = None


def batch_workspace_bound(n: int, nnz: int, n_hot: int, Ks, laps, seg_len: int = 0) -> int:
    """An upper bound, in closed form, on gee_embed_batch's workspace for one graph and
    batch (admission needs a bound per job, and the library's exact query costs a few
    ctypes objects per call). It takes the widest label row (min(64, B + 1 rounded up to
    8) bytes: a group of fewer than 64 vectors keeps a zero padding column) and the most classes of a group (min(sum K, 4096)) for every group-sized
    table, and the library's default segment length (the power of two at or above
    (n + nnz) / 32768 within [512, 16384]) when seg_len is 0."""
    if seg_len:
        L = seg_len
    else:
        want, L = (n + nnz) // 32768, 512
        while L < want and L < 16384:
            L *= 2
    nseg = (n + nnz + L - 1) // L
    B, S = len(Ks), int(sum(Ks))
    gs = min(64, (B + 1 + 7) // 8 * 8)
    kt = min(S, 4096)
    parts = [8 * (S + B), 2 * (n + 1) * gs, 2 * n_hot * gs, 8 * kt, 4 * 64, 4 * (nseg + 1), 8 * (nseg + 1),
             16 * nseg * kt]
    if any(laps):
        parts += [8 * n, 4 * n, 4 * n_hot]
    return sum(p + 256 for p in parts) + 256  # each table starts 256-byte aligned


def plan_packs(graphs: dict, pack_items: int, pack_limit: int):
    """Packs of small graphs. Graphs whose rows + entries (n + 2s) are at most pack_items
    go, in id order, into packs of at most pack_limit rows + entries; the others stand
    alone. Returns (unit, members): unit[gid] = (key of the CSR that serves the graph,
    first row of the graph in it), with key = gid for a graph on its own and a negative
    key for a pack; members[key] = the pack's graph ids in order."""
    unit: dict[int, tuple[int, int]] = {}
    members: dict[int, list[int]] = {}
    fill = 0
    for gid in sorted(graphs):
        n, src = graphs[gid][0], graphs[gid][1]
        items = n + 2 * len(src)
        if pack_items <= 0 or items > pack_items:
            unit[gid] = (gid, 0)
            continue
        if not members or fill + items > pack_limit:
            members[-1 - len(members)] = []
            fill = 0
        key = -len(members)
        unit[gid] = (key, sum(graphs[m][0] for m in members[key]))
        members[key].append(gid)
        fill += items
    return unit, members


class Server:
    """Continuous-batching GEE server over a pool of graphs (``graphs[gid] = (n, src, dst)``
    host arrays). ``hbm_budget`` bounds resident graphs plus in-flight outputs and scratch."""

    MAX_INFLIGHT = 1024  # launches in flight at once
    MAX_LAUNCH_VECTORS = 4096  # label vectors in one launch (one gee_embed_batch call)

    def __init__(self, graphs: dict, hbm_budget: int, streams: int = 4, mode: str = "batched",
                 seg_len: int = 0, hot_budget: int = DEFAULT_HOT_BUDGET, keep_results: bool = False,
                 device: str = "cuda:0", route_vectors: int = 0, route_items: int = 1 << 22,
                 pack_items: int = 0, pack_limit: int = 1 << 22, route_adjacency: int = 0):
        if mode not in ("batched", "plain"):
            raise ValueError("mode: batched or plain")
        self.pool = graphs
        self.budget = int(hbm_budget)
        self.mode = mode
        self.seg_len = seg_len
        self.route_vectors = route_vectors
        self.route_items = route_items
        self.route_adjacency = route_adjacency
        self.hot_budget = hot_budget
        self.keep = keep_results
        self.dev = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(max(1, streams if mode == "batched" else 1))]
        self._next_stream = 0
        self.resident: dict[int, _Graph] = {}
        self.pending: collections.deque[Request] = collections.deque()
        self.inflight: list[_Launch] = []
        self.used = 0  # bytes: resident graphs + in-flight launches
        self.evictions = 0
        # Small graphs (rows + entries <= pack_items) are served in packs: the members of
        # a pack, in id order, form one disjoint-union CSR of at most pack_limit rows +
        # entries, and all jobs on any member run in one launch over it. A member is
        # always served through its pack, so its jobs' results do not depend on the mix.
        # unit[gid] = (key of the resident CSR, first row of the graph in it); packs have
        # negative keys.
        self.unit, self.members = plan_packs(graphs, pack_items, pack_limit)
        self._ws_plain = {}  # (gid, K, laplacian) -> gee_embed workspace bytes
        # one error word per in-flight launch, copied back to pinned host memory behind the
        # launch on its stream: a finished launch's word is read without a device sync
        self._err_dev = torch.zeros(self.MAX_INFLIGHT, dtype=torch.int32, device=self.dev)
        self._err_host = torch.zeros(self.MAX_INFLIGHT, dtype=torch.int32, pin_memory=True)
        self._free_slots = list(range(self.MAX_INFLIGHT - 1, -1, -1))
        # slots of refused launches, each freed once an event recorded behind the work
        # queued before the refusal has completed
        self._slot_wait: list[tuple[HipEvent, int]] = []
        # jobs finished or refused but not yet returned (a poll that raised keeps them)
        self._ready: list[Done] = []
        self._admitted_last = 0
        self._last_stream = 0
        # one small launch on every stream, so that the first jobs do not wait while the
        # runtime sets up the streams' queues
        for st in self.streams:
            with torch.cuda.stream(st):
                self._err_dev.zero_()
        torch.cuda.synchronize(self.dev)
        self.ref = HipEvent()
        self.ref.record(torch.cuda.current_stream(self.dev))
        self.ref.synchronize()
        self.ref_host = time.perf_counter()

    # ------------------------------------------------------------ memory ----
    def _graph_bytes(self, n: int, s: int) -> int:
        hot = min(self.hot_budget, n)
        return 8 * (n + 1) + 4 * 2 * s + 4 * hot

    def _routes_plain(self, g: _Graph, Ks) -> bool:
        """The job runs as one gee_embed call per vector (plain mode, or few vectors on a
        large graph)."""
        return self.mode == "plain" or (len(Ks) <= self.route_vectors and g.csr.n + g.csr.nnz >= self.route_items)

    def _launch_bytes(self, g: _Graph, Ks, laps) -> int:
        n = g.csr.n

        def plain():
            ws = max(self._plain_ws(g, k, l) for k, l in zip(Ks, laps))
            return ws + 4 * n * int(sum(Ks)) + 4 * n * len(Ks) + 4 * n * max(Ks)

        if self._routes_plain(g, Ks):
            return plain()
        # the job's share of a fused launch is at most what it would need alone
        ws = batch_workspace_bound(n, g.csr.nnz, g.csr.n_hot, Ks, laps, self.seg_len)
        fused = ws + 4 * n * int(sum(Ks)) + 4 * n * len(Ks)
        if self.route_adjacency > 0 and n + g.csr.nnz >= self.route_items and not any(laps):
            return max(fused, plain())  # the launch may run it either way
        return fused

    def _plain_ws(self, g: _Graph, k: int, lap: bool) -> int:
        key = (g.gid, int(k), bool(lap))
        b = self._ws_plain.get(key)
        if b is None:
            b = self._ws_plain[key] = embed_workspace_bytes(k, csr=g.csr, laplacian=lap, seg_len=self.seg_len)
        return b

    def _evict_for(self, need: int, keep_gid: int) -> bool:
        while self.used + need > self.budget:
            idle = [g for g in self.resident.values() if g.busy == 0 and g.gid != keep_gid]
            if not idle:
                return False
            victim = min(idle, key=lambda g: g.last_use)
            self.used -= victim.bytes
            del self.resident[victim.gid]
            self._ws_plain = {k: b for k, b in self._ws_plain.items() if k[0] != victim.gid}
            self.evictions += 1
        return True

    def _unit_bytes(self, gid: int) -> int:
        """Resident bytes of the CSR that serves unit gid (a graph, or a pack of graphs)."""
        parts = [self.pool[m] for m in self.members[gid]] if gid < 0 else [self.pool[gid]]
        return self._graph_bytes(sum(p[0] for p in parts), sum(len(p[1]) for p in parts))

    def _resident(self, gid: int) -> _Graph | None:
        g = self.resident.get(gid)
        if g is not None:
            return g
        if gid < 0:  # a pack: members side by side, each shifted to its first row
            parts = [self.pool[m] for m in self.members[gid]]
            offs = np.cumsum([0] + [p[0] for p in parts])
            n = int(offs[-1])
            src = np.concatenate([np.asarray(p[1], np.int64) + o for p, o in zip(parts, offs)]).astype(np.int32)
            dst = np.concatenate([np.asarray(p[2], np.int64) + o for p, o in zip(parts, offs)]).astype(np.int32)
        else:
            n, src, dst = self.pool[gid]
        need = self._graph_bytes(n, len(src))
        if not self._evict_for(need, gid):
            return None
        coo = to_device(n, src, dst, None, device=self.dev)
        csr = csr_build(coo, hot_budget=min(self.hot_budget, n), check=True)
        del coo
        g = _Graph(gid, csr, len(src), need)
        self.resident[gid] = g
        self.used += need
        return g

    def warm(self, gids) -> int:
        """Make graphs resident ahead of their first job (while the budget allows); returns how many are."""
        for gid in gids:
            if self._resident(self.unit[gid][0]) is None:
                break
        return len(self.resident)

    SMALL_RESERVE = 512  # 1 MiB blocks kept for small buffers (torch serves those from a separate pool)

    def reserve(self) -> int:
        """Allocate and free one block of the budget not held by resident graphs, so that
        torch's caching allocator keeps it as one segment and later launches are carved
        from it instead of calling the device allocator while jobs wait; likewise
        SMALL_RESERVE blocks of 1 MiB for the pool torch keeps for buffers of at most
        1 MiB. Returns the bytes set aside."""
        free = self.budget - self.used
        if free <= 0:
            return 0
        small = min(self.SMALL_RESERVE, free // (4 << 20))
        blocks = [torch.empty(1 << 20, dtype=torch.uint8, device=self.dev) for _ in range(small)]
        big = free - small * (1 << 20)  # two 1 MiB blocks share a 2 MiB segment
        block = torch.empty(big, dtype=torch.uint8, device=self.dev) if big > 0 else None
        del blocks, block
        return free

    # ------------------------------------------------------------ serving ----
    def submit(self, req: Request):
        if len(req.Ks) > self.MAX_LAUNCH_VECTORS:
            raise ValueError(f"job {req.jid} has {len(req.Ks)} vectors; a launch holds {self.MAX_LAUNCH_VECTORS}")
        self.pending.append(req)

    def idle(self) -> bool:
        return not self.pending and not self.inflight and not self._ready

    def _host_time(self, ev: HipEvent) -> float:
        return self.ref_host + self.ref.elapsed_ms(ev) * 1e-3

    def _admit(self) -> list:
        """Pending requests admitted in arrival order while their graph and launch fit."""
        out = []
        limit = 1 if self.mode == "plain" else len(self.pending)
        if self.mode == "plain" and self.inflight:
            return out
        gids = {}  # unit -> vectors admitted: one launch per unit, each holding an error slot
        while self.pending and len(out) < limit:
            r = self.pending[0]
            u = self.unit[r.gid][0]
            if u not in gids and len(gids) >= len(self._free_slots):
                break
            if gids.get(u, 0) + len(r.Ks) > self.MAX_LAUNCH_VECTORS:
                break  # the launch is full; the job waits for the next poll
            g = self._resident(u)
            if g is None:
                if self._unit_bytes(u) > self.budget:  # the graph alone can never fit
                    self.pending.popleft()
                    self._ready.append(self._refused(r, ERR_BUDGET))
                    continue
                break
            need = self._launch_bytes(g, r.Ks, r.laplacian)
            if need > self.budget - g.bytes:
                # the job can never run: it is finished with an error and the loop goes on
                self.pending.popleft()
                self._ready.append(self._refused(r, ERR_BUDGET))
                continue
            if self.used + need > self.budget and not self._evict_for(need, u):
                break
            self.pending.popleft()
            self.used += need
            g.busy += 1
            gids[u] = gids.get(u, 0) + len(r.Ks)
            out.append((r, g, need))
        return out

    def _hold_slot(self, slot: int):
        """Keep a refused launch's error slot out of use until the work queued before the
        refusal on its stream has completed (if even the event cannot be recorded, the slot
        stays out of use)."""
        try:
            ev = HipEvent()
            ev.record(self.streams[self._last_stream])
        except Exception:
            return
        self._slot_wait.append((ev, slot))

    def _refused(self, r: Request, code: int) -> Done:
        n, src, _ = self.pool[r.gid]
        return Done(r.jid, r.gid, r.arrival, time.perf_counter(), len(src), len(r.Ks), int(code), None)

    def _launch(self, group: list, slot: int):
        g = group[0][1]
        reqs = [r for r, _, _ in group]
        nbytes = sum(b for _, _, b in group)
        Ks = [k for r in reqs for k in r.Ks]
        # the stream with the least estimated work in flight, so that a short launch does
        # not queue behind a long one while another stream is idle
        work = 4.0 * g.csr.n * sum(Ks) + 4.0 * (g.csr.n + g.csr.nnz) * len(Ks)
        load = [0.0] * len(self.streams)
        for L in self.inflight:
            load[L.stream] += L.work
        si = min(range(len(self.streams)), key=lambda i: (load[i], (i - self._next_stream) % len(self.streams)))
        self._next_stream = (si + 1) % len(self.streams)
        self._last_stream = si
        stream = self.streams[si]
        laps = [l for r in reqs for l in r.laplacian]
        zoff, acc = [], 0
        for k in Ks:
            zoff.append(acc)
            acc += k
        # vector index of each job's first vector in the launch
        first, b0 = [], 0
        for r in reqs:
            first.append(b0)
            b0 += len(r.Ks)
        n = g.csr.n
        plain = [self._routes_plain(g, r.Ks) for r in reqs]
        if self.route_adjacency > 0 and g.csr.n + g.csr.nnz >= self.route_items:
            # adjacency vectors take the same bits in either pass, so they may follow the
            # load: when nothing else in this launch needs the batched pass and they are
            # few, one plain call each is shorter than the batched walk
            lap_batched = any(not plain[i] and any(r.laplacian) for i, r in enumerate(reqs))
            adj = [i for i, r in enumerate(reqs) if not plain[i] and not any(r.laplacian)]
            if not lap_batched and 0 < sum(len(reqs[i].Ks) for i in adj) <= self.route_adjacency:
                for i in adj:
                    plain[i] = True
        fused = [i for i, r in enumerate(reqs) if not plain[i]]
        fset = set(fused)
        vs = [first[i] + b for i in fused for b in range(len(reqs[i].Ks))]  # fused vectors
        pv = [first[i] + b for i, r in enumerate(reqs) if i not in fset for b in range(len(r.Ks))]
        # Device buffers come from the pool of torch's current stream, which reserve()
        # fills, and are marked as used by the launch's stream: torch keeps free blocks per
        # stream, so buffers allocated on the launch's stream would bypass the reservation
        # and reach the device allocator while jobs wait. Label rows: the fused jobs'
        # vectors first (one contiguous block for the batched call), then the others.
        labels = torch.empty((len(Ks), n), dtype=torch.int32, device=self.dev)
        Z = torch.empty((n, int(sum(Ks))), dtype=torch.float32, device=self.dev)
        bufs = [labels, Z]
        pack = g.gid < 0  # labels go to the member's rows of the union, zeros elsewhere
        if pack:
            r0s = [self.unit[r.gid][1] for r in reqs]
            ns = [self.pool[r.gid][0] for r in reqs]
            stage = torch.empty(sum(len(r.Ks) * m for r, m in zip(reqs, ns)), dtype=torch.int32, device=self.dev)
            bufs.append(stage)
        if vs:
            fK, fl, fz = [Ks[v] for v in vs], [laps[v] for v in vs], [zoff[v] for v in vs]
            ws_b = torch.empty(batch_workspace_bound(n, g.csr.nnz, g.csr.n_hot, fK, fl, self.seg_len),
                               dtype=torch.uint8, device=self.dev)
            bufs.append(ws_b)
        if pv:
            ws_p = torch.empty(max(self._plain_ws(g, Ks[v], laps[v]) for v in pv), dtype=torch.uint8, device=self.dev)
            zb = torch.empty(n * max(Ks[v] for v in pv), dtype=torch.float32, device=self.dev)
            bufs += [ws_p, zb]
        for t in bufs:
            t.record_stream(stream)
        with torch.cuda.stream(stream):
            err = self._err_dev[slot:slot + 1]
            err.zero_()
            row, rows, at = [0, len(vs)], [], 0
            if pack:
                labels.zero_()
            for i, r in enumerate(reqs):
                side = 0 if i in fset else 1
                rows.append(row[side])
                B = len(r.Ks)
                if pack:
                    st = stage[at:at + B * ns[i]].view(B, ns[i])
                    at += B * ns[i]
                    st.copy_(r.labels, non_blocking=True)
                    labels[row[side]:row[side] + B, r0s[i]:r0s[i] + ns[i]].copy_(st)
                else:
                    labels[row[side]:row[side] + B].copy_(r.labels, non_blocking=True)
                row[side] += B
            if vs:  # one batched call over the fused jobs' vectors, their blocks of Z in place
                embed_batch(labels[:len(vs)].reshape(-1), fK, fl, g.csr, Z=Z, zoff=fz, ws=ws_b, err=err,
                            seg_len=self.seg_len, stream=stream, check=False)
            for i, r in enumerate(reqs):
                if i in fset:
                    continue
                for b, (k, lap) in enumerate(zip(r.Ks, r.laplacian)):
                    v = first[i] + b
                    Zb = zb[:n * k].view(n, k)
                    embed(labels[rows[i] + b], k, csr=g.csr, laplacian=lap, Z=Zb, ws=ws_p, err=err,
                          seg_len=self.seg_len, stream=stream, check=False)
                    if self.keep:  # results side by side, as a batched launch returns them
                        Z[:, zoff[v]:zoff[v] + k].copy_(Zb)
            self._err_host[slot:slot + 1].copy_(err, non_blocking=True)
            ev = HipEvent()
            ev.record(stream)
        self.inflight.append(_Launch(ev, reqs, g, nbytes, slot, si, work, keep=bufs + [r.labels for r in reqs],
                                     Z=Z if self.keep else None, zoff=zoff))

    def poll(self) -> list:
        """Retire finished launches, admit and launch pending jobs; returns the jobs finished
        (those refused included, with their error code)."""
        finished, self._ready = self._ready, []
        try:
            self._poll(finished)
        except BaseException:
            self._ready = finished + self._ready  # returned by the next poll
            raise
        finished += self._ready
        self._ready = []
        return finished

    def _poll(self, finished: list):
        waiting = []
        for ev, slot in self._slot_wait:
            if ev.done():
                self._free_slots.append(slot)
            else:
                waiting.append((ev, slot))
        self._slot_wait = waiting
        still = []
        for L in self.inflight:
            if not L.event.done():
                still.append(L)
                continue
            t = self._host_time(L.event)
            e = int(self._err_host[L.slot])
            self._free_slots.append(L.slot)
            col = 0
            for r in L.reqs:
                kz = int(sum(r.Ks))
                n, src, _ = self.pool[r.gid]
                r0 = self.unit[r.gid][1]
                Zr = L.Z[r0:r0 + n, col:col + kz] if L.Z is not None else None
                col += kz
                finished.append(Done(r.jid, r.gid, r.arrival, t, len(src), len(r.Ks), e, Zr))
            self.used -= L.bytes
            L.graph.busy -= len(L.reqs)
            L.graph.last_use = t
        self.inflight = still
        admitted = self._admit()
        self._admitted_last = len(admitted)
        by_graph = collections.OrderedDict()
        for item in admitted:
            by_graph.setdefault(item[1].gid, []).append(item)
        groups = list(by_graph.values())
        for gi, group in enumerate(groups):
            slot = self._free_slots.pop()
            try:
                self._launch(group, slot)
            except GeeError as exc:
                # the library refused a call of this launch (it checks its arguments before
                # queuing work): its jobs finish with the library's code, their memory and
                # graph claim are given back, and the other launches go ahead. The error
                # slot returns to use once the work queued on the stream before the refusal
                # (which may write it) has completed; buffers that work uses are held by
                # torch's allocator until the stream passes them.
                self.used -= sum(b for _, _, b in group)
                group[0][1].busy -= len(group)
                self._hold_slot(slot)
                self._ready += [self._refused(r, exc.code) for r, _, _ in group]
            except BaseException as exc:
                # anything else ends the poll: the memory and graph claims of this launch and
                # of those not yet made are given back, their jobs wait again at the head of
                # the queue in arrival order, and the exception names this launch's jobs
                for grp in groups[gi:]:
                    self.used -= sum(b for _, _, b in grp)
                    grp[0][1].busy -= len(grp)
                self.pending.extendleft(reversed([item[0] for grp in groups[gi:] for item in grp]))
                self._hold_slot(slot)
                exc.refused_jobs = [r.jid for r, _, _ in group]
                raise

    def drain(self) -> list:
        """Poll until every submitted job has come back. Raises RuntimeError if jobs are
        pending that no poll can ever admit (nothing in flight, no slot coming free, and
        the last poll admitted and returned nothing)."""
        out = []
        while not self.idle():
            got = self.poll()
            out += got
            if (not got and not self._admitted_last and self.pending and not self.inflight
                    and not self._slot_wait):
                raise RuntimeError(f"{len(self.pending)} pending jobs cannot be admitted "
                                   f"({len(self._free_slots)} free launch slots, {self.used} of "
                                   f"{self.budget} bytes in use)")
        return out
