"""A serving loop for GEE jobs on many graphs, on one GPU.

A job is a set of label vectors (each with its K and version) on one graph of a
pool. Jobs arrive over time. The server keeps graphs resident in HBM (the canonical
CSR is built on first use and reused by later jobs; least recently used graphs are
evicted when memory is needed), admits arrived jobs in arrival order while their
output and scratch fit an HBM budget, and at every poll launches all admitted jobs:
the jobs on one graph are fused into one ``gee_embed_batch`` call (continuous
batching: a job that arrives while others run joins the next launch), and calls on
different graphs go to different HIP streams so their work overlaps on the device.

A job's result does not depend on which other jobs share its launch: the batched
pass gives every vector its own bins, filled in CSR order, and the segmentation
depends only on the graph and the segment length. ``plain`` mode is the comparison:
one job at a time, one ``gee_embed`` call per vector, in arrival order.

Latency of a job = device completion of its launch minus its arrival, both on the
host clock (the completion is read from HIP events against a reference event).
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import torch

from . import (DEFAULT_HOT_BUDGET, DeviceCsr, HipEvent, csr_build, embed, embed_batch,
               embed_batch_workspace_bytes, embed_workspace_bytes, to_device)


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
    keep: list = field(default_factory=list)
    Z: torch.Tensor | None = None
    zoff: list | None = None


class Server:
    """Continuous-batching GEE server over a pool of graphs (``graphs[gid] = (n, src, dst)``
    host arrays). ``hbm_budget`` bounds resident graphs plus in-flight outputs and scratch."""

    MAX_INFLIGHT = 1024  # launches in flight at once

    def __init__(self, graphs: dict, hbm_budget: int, streams: int = 4, mode: str = "batched",
                 seg_len: int = 0, hot_budget: int = DEFAULT_HOT_BUDGET, keep_results: bool = False,
                 device: str = "cuda:0"):
        if mode not in ("batched", "plain"):
            raise ValueError("mode: batched or plain")
        self.pool = graphs
        self.budget = int(hbm_budget)
        self.mode = mode
        self.seg_len = seg_len
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
        # one error word per in-flight launch, copied back to pinned host memory behind the
        # launch on its stream: a finished launch's word is read without a device sync
        self._err_dev = torch.zeros(self.MAX_INFLIGHT, dtype=torch.int32, device=self.dev)
        self._err_host = torch.zeros(self.MAX_INFLIGHT, dtype=torch.int32, pin_memory=True)
        self._free_slots = list(range(self.MAX_INFLIGHT - 1, -1, -1))
        self.ref = HipEvent()
        self.ref.record(torch.cuda.current_stream(self.dev))
        self.ref.synchronize()
        self.ref_host = time.perf_counter()

    # ------------------------------------------------------------ memory ----
    def _graph_bytes(self, n: int, s: int) -> int:
        hot = min(self.hot_budget, n)
        return 8 * (n + 1) + 4 * 2 * s + 4 * hot

    def _launch_bytes(self, g: _Graph, Ks, laps) -> int:
        n = g.csr.n
        if self.mode == "batched":
            ws = embed_batch_workspace_bytes(n, Ks, laps, g.csr, seg_len=self.seg_len)
            return ws + 4 * n * int(sum(Ks)) + 4 * n * len(Ks) * 2
        ws = max(embed_workspace_bytes(k, csr=g.csr, laplacian=l, seg_len=self.seg_len) for k, l in zip(Ks, laps))
        return ws + 4 * n * int(sum(Ks)) + 4 * n * len(Ks)

    def _evict_for(self, need: int, keep_gid: int) -> bool:
        while self.used + need > self.budget:
            idle = [g for g in self.resident.values() if g.busy == 0 and g.gid != keep_gid]
            if not idle:
                return False
            victim = min(idle, key=lambda g: g.last_use)
            self.used -= victim.bytes
            del self.resident[victim.gid]
            self.evictions += 1
        return True

    def _resident(self, gid: int) -> _Graph | None:
        g = self.resident.get(gid)
        if g is not None:
            return g
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
            if self._resident(gid) is None:
                break
        return len(self.resident)

    # ------------------------------------------------------------ serving ----
    def submit(self, req: Request):
        self.pending.append(req)

    def idle(self) -> bool:
        return not self.pending and not self.inflight

    def _host_time(self, ev: HipEvent) -> float:
        return self.ref_host + self.ref.elapsed_ms(ev) * 1e-3

    def _admit(self) -> list:
        """Pending requests admitted in arrival order while their graph and launch fit."""
        out = []
        limit = 1 if self.mode == "plain" else len(self.pending)
        if self.mode == "plain" and self.inflight:
            return out
        gids = set()  # one launch per graph, each holding an error slot
        while self.pending and len(out) < limit:
            r = self.pending[0]
            if r.gid not in gids and len(gids) >= len(self._free_slots):
                break
            g = self._resident(r.gid)
            if g is None:
                break
            need = self._launch_bytes(g, r.Ks, r.laplacian)
            if need > self.budget - g.bytes:
                raise ValueError(f"job {r.jid} needs {need} bytes beside its graph; the budget is {self.budget}")
            if self.used + need > self.budget and not self._evict_for(need, r.gid):
                break
            self.pending.popleft()
            self.used += need
            g.busy += 1
            gids.add(r.gid)
            out.append((r, g, need))
        return out

    def _launch(self, group: list, slot: int):
        g = group[0][1]
        reqs = [r for r, _, _ in group]
        nbytes = sum(b for _, _, b in group)
        stream = self.streams[self._next_stream]
        self._next_stream = (self._next_stream + 1) % len(self.streams)
        Ks = [k for r in reqs for k in r.Ks]
        laps = [l for r in reqs for l in r.laplacian]
        n = g.csr.n
        with torch.cuda.stream(stream):
            err = self._err_dev[slot:slot + 1]
            err.zero_()
            labels = torch.cat([r.labels.to(self.dev, non_blocking=True) for r in reqs]) if len(reqs) > 1 else \
                reqs[0].labels.to(self.dev, non_blocking=True)
            Z = torch.empty((n, int(sum(Ks))), dtype=torch.float32, device=self.dev)
            zoff, acc = [], 0
            for k in Ks:
                zoff.append(acc)
                acc += k
            if self.mode == "batched":
                embed_batch(labels.view(-1), Ks, laps, g.csr, Z=Z, zoff=zoff, err=err, seg_len=self.seg_len,
                            stream=stream, check=False)
            else:
                for b, (k, lap) in enumerate(zip(Ks, laps)):
                    Zb = torch.empty((n, k), dtype=torch.float32, device=self.dev)
                    embed(labels[b], k, csr=g.csr, laplacian=lap, Z=Zb, err=err, seg_len=self.seg_len,
                          stream=stream, check=False)
                    if self.keep:  # results side by side, as the batched launch returns them
                        Z[:, zoff[b]:zoff[b] + k].copy_(Zb)
            self._err_host[slot:slot + 1].copy_(err, non_blocking=True)
            ev = HipEvent()
            ev.record(stream)
        self.inflight.append(_Launch(ev, reqs, g, nbytes, slot, keep=[labels, Z] + [r.labels for r in reqs],
                                     Z=Z if self.keep else None, zoff=zoff))

    def poll(self) -> list:
        """Retire finished launches, admit and launch pending jobs; returns the jobs finished."""
        finished = []
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
                Zr = L.Z[:, col:col + kz] if L.Z is not None else None
                col += kz
                finished.append(Done(r.jid, r.gid, r.arrival, t, L.graph.s, len(r.Ks), e, Zr))
            self.used -= L.bytes
            L.graph.busy -= len(L.reqs)
            L.graph.last_use = t
        self.inflight = still
        admitted = self._admit()
        by_graph = collections.OrderedDict()
        for item in admitted:
            by_graph.setdefault(item[0].gid, []).append(item)
        for group in by_graph.values():
            self._launch(group, self._free_slots.pop())
        return finished

    def drain(self) -> list:
        out = []
        while not self.idle():
            out += self.poll()
        return out
