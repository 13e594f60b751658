"""Continuous-batching J/K server on one GPU.

Every molecule of the stream stays resident as a library handle (shell
pairs, Schwarz factors, quartet lists and cached launch plans), so requests
on the same molecule reuse them -- the analogue of the paper's
geometry-frozen caches reused across many densities at one geometry
(Sect. 3, metric-cache paragraph).

Work runs on a pool of "slots": one stream each (default priority) plus a
fixed device arena carved out of the memory budget.  A free slot takes the
oldest waiting requests whose combined workspace fits its arena (admission by
device memory) and launches them as one batched build (`jk_build_batch`), so
requests that arrive while others run are folded into the next launch and
overlap on the device with the other slots.  A lone request replays a HIP
graph of its build (captured per slot, molecule and density-group count:
8, 16, 32, 48 or 64 densities) from fixed slot buffers, so zero padding
adds no digestion work.

Latency of a request = completion (a HIP event on its slot's stream, read
against an event recorded at the start of the run) minus its scheduled
arrival time.  Only argument marshalling and scheduling happen here; all
arithmetic runs in libjk.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import jk


class _Shape:
    """Stands in for a density tensor where only its count is needed."""

    def __init__(self, nd):
        self.shape = (nd,)


@dataclass
class Request:
    index: int
    arrival: float          # seconds after the start of the run
    mol: int
    D: torch.Tensor         # [nd, n, n] float64 on the device
    J: torch.Tensor | None = None
    K: torch.Tensor | None = None
    done_ms: float = -1.0   # completion, ms after the start event
    slot: int = -1
    batch: int = 0          # size of the launch it ran in
    graph: bool = False

    @property
    def nd(self):
        return int(self.D.shape[0])


def _bucket(nd):
    """Density count a graph is captured for: the digestion works in groups
    of 8 (up to 8 densities) or 16, so a request runs on the graph of its
    group count and the zero padding adds no digestion work."""
    return 8 if nd <= 8 else (nd + 15) // 16 * 16


def _buckets(max_nd):
    out, b = [], 8
    while b <= max(8, max_nd):
        out.append(b)
        b = 16 if b == 8 else b + 16
    return out


@dataclass
class _Slot:
    stream: torch.cuda.Stream
    arena: torch.Tensor
    busy: list = field(default_factory=list)
    event: torch.cuda.Event | None = None
    stage: dict = field(default_factory=dict)     # mol -> (D, J, K) staging for graphs
    graphs: dict = field(default_factory=dict)    # (mol, nd_bucket) -> graph


class JKServer:
    """Serve J/K requests over resident molecules."""

    def __init__(self, bases, n_slots: int = 4, mem_budget: int | None = None, precision: int = jk.JK_MIXED,
                 max_batch: int = 16, use_graphs: bool = True, graph_max_nd: int = 64, batch_nbf_max: int | None = None,
                 device="cuda:0"):
        self.dev = torch.device(device)
        self.handles = [jk.JKBasis(b) for b in bases]
        self.nbf = [h.nbf for h in self.handles]
        self.opts = jk.jk_default_opts(precision=precision)
        self.max_batch = max_batch
        # requests on molecules above this size always launch alone (their
        # builds fill the GPU by themselves; batching would only hold back the
        # earlier requests of a batch until its end)
        self.batch_nbf_max = batch_nbf_max
        self.use_graphs = use_graphs
        self.graph_max_nd = graph_max_nd
        if mem_budget is None:
            free, _ = torch.cuda.mem_get_info(self.dev)
            mem_budget = int(free * 0.5)
        self.mem_budget = mem_budget
        per_slot = mem_budget // n_slots
        self.slots = [_Slot(torch.cuda.Stream(device=self.dev),
                            torch.empty(per_slot, dtype=torch.uint8, device=self.dev)) for _ in range(n_slots)]
        self.slot_bytes = per_slot
        self.peak_admitted = 0
        self._single = {}           # (mol, nd) -> workspace of that request alone
        self.sched_s = 0.0          # host time spent choosing and sizing launches

    # ------------------------------------------------------------- sizes --
    def workspace_bytes(self, reqs) -> int:
        """Exact workspace of one batched launch of `reqs` (plans the batch)."""
        hs = [self.handles[r.mol].h for r in reqs]
        return jk.jk_batch_workspace_bytes(hs, [r.nd for r in reqs], self.opts)

    def single_bytes(self, mol, nd) -> int:
        """Workspace of one request alone, cached per (molecule, nd)."""
        key = (mol, nd)
        if key not in self._single:
            self._single[key] = self.workspace_bytes([Request(-1, 0.0, mol, _Shape(nd))])
        return self._single[key]

    def graph_bytes(self, mol, nd_bucket) -> int:
        n = self.nbf[mol]
        return jk.jk_workspace_bytes(self.handles[mol].h, nd_bucket, self.opts) + 3 * nd_bucket * n * n * 8

    def _batchable(self, req) -> bool:
        return self.batch_nbf_max is None or self.nbf[req.mol] <= self.batch_nbf_max

    def fits_alone(self, req) -> bool:
        return self.single_bytes(req.mol, req.nd) <= self.slot_bytes

    # ------------------------------------------------------------ graphs --
    def _graph(self, slot: _Slot, mol: int, ndb: int):
        key = (mol, ndb)
        if key in slot.graphs:
            return slot.graphs[key]
        n = self.nbf[mol]
        ws_bytes = jk.jk_workspace_bytes(self.handles[mol].h, ndb, self.opts)
        need = ws_bytes + 3 * ndb * n * n * 8
        if need > self.slot_bytes:
            return None
        # arena layout for a graph: [workspace | D | J | K]; every graph of the
        # slot starts at the arena base, so graphs of one slot never run together
        base = slot.arena
        o = jk.jk_default_opts(precision=self.opts.precision)
        o.workspace = base.data_ptr()
        o.workspace_bytes = ws_bytes
        mats = base[ws_bytes:ws_bytes + 3 * ndb * n * n * 8].view(torch.float64).view(3, ndb, n, n)
        D, J, K = mats[0], mats[1], mats[2]
        g = jk.jk_graph_create(self.handles[mol].h, D, J, K, o)
        slot.graphs[key] = (g, D, J, K)
        return slot.graphs[key]

    def warm_graphs(self, mols=None, max_nd=None, on_progress=None):
        """Capture the graphs of every (slot, molecule, density bucket)."""
        mols = range(len(self.handles)) if mols is None else mols
        max_nd = max_nd or self.graph_max_nd
        for si, slot in enumerate(self.slots):
            for m in mols:
                for ndb in _buckets(max_nd):
                    self._graph(slot, m, ndb)
                if on_progress:
                    on_progress(si, m)
        torch.cuda.synchronize(self.dev)

    # ------------------------------------------------------------ launch --
    def _launch(self, slot: _Slot, reqs):
        s = slot.stream
        for r in reqs:
            r.J = torch.empty_like(r.D)
            r.K = torch.empty_like(r.D)
            r.batch = len(reqs)
        with torch.cuda.stream(s):
            if len(reqs) == 1 and self.use_graphs and reqs[0].nd <= self.graph_max_nd:
                r = reqs[0]
                ndb = _bucket(r.nd)
                gr = self._graph(slot, r.mol, ndb)
                if gr is not None:
                    g, D, J, K = gr
                    D[:r.nd].copy_(r.D)
                    if ndb > r.nd:
                        D[r.nd:].zero_()
                    jk.jk_graph_launch(g, s)
                    r.J.copy_(J[:r.nd])
                    r.K.copy_(K[:r.nd])
                    r.graph = True
                    self._done(slot, reqs)
                    return
            o = jk.jk_default_opts(precision=self.opts.precision)
            o.workspace = slot.arena.data_ptr()
            o.workspace_bytes = self.slot_bytes
            jk.jk_build_batch([self.handles[r.mol].h for r in reqs], [r.D for r in reqs],
                              [r.J for r in reqs], [r.K for r in reqs], o, s)
        self._done(slot, reqs)

    def _done(self, slot, reqs):
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(slot.stream)
        slot.event = ev
        slot.busy = list(reqs)

    # --------------------------------------------------------------- run --
    def run(self, requests, on_progress=None, on_launch=None):
        """Serve `requests` (sorted by arrival).  Returns summary statistics;
        each request gets J, K, done_ms and its slot.  on_launch(slot, reqs)
        is called for every launch, on_progress(done, total) on every
        completion."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        for r in reqs:
            if not self.fits_alone(r):
                raise MemoryError(f"request {r.index} needs more than a slot's {self.slot_bytes} bytes")
        torch.cuda.synchronize(self.dev)
        start = torch.cuda.Event(enable_timing=True)
        start.record(self.slots[0].stream)
        t0 = time.perf_counter()
        queue = []
        nxt = 0
        done = 0
        n = len(reqs)
        while done < n:
            now = time.perf_counter() - t0
            while nxt < n and reqs[nxt].arrival <= now:
                queue.append(reqs[nxt])
                nxt += 1
            progressed = False
            for si, slot in enumerate(self.slots):
                if slot.busy and slot.event.query():
                    for r in slot.busy:
                        r.done_ms = start.elapsed_time(slot.event)
                    done += len(slot.busy)
                    slot.busy = []
                    progressed = True
                    if on_progress:
                        on_progress(done, n)
                if not slot.busy and queue:
                    # admission in arrival order: requests join while the sum of
                    # their alone-workspaces fits the slot (cached per molecule
                    # and density count); one exact sizing of the launch, which
                    # sheds the newest requests in the rare case it does not fit
                    ts = time.perf_counter()
                    batch = [queue[0]]
                    est = self.single_bytes(queue[0].mol, queue[0].nd)
                    for r in queue[1:]:
                        if len(batch) >= self.max_batch or not self._batchable(batch[0]) or not self._batchable(r):
                            break
                        e = self.single_bytes(r.mol, r.nd)
                        if est + e > self.slot_bytes:
                            break
                        batch.append(r)
                        est += e
                    ws = self.workspace_bytes(batch)
                    while ws > self.slot_bytes and len(batch) > 1:
                        batch.pop()
                        ws = self.workspace_bytes(batch)
                    self.sched_s += time.perf_counter() - ts
                    self.peak_admitted = max(self.peak_admitted, ws)
                    for r in batch:
                        queue.remove(r)
                        r.slot = si
                    if on_launch:
                        on_launch(si, batch)
                    self._launch(slot, batch)
                    progressed = True
            if not progressed:
                time.sleep(5e-5)
        torch.cuda.synchronize(self.dev)
        out = summarize(reqs)
        out["host_sched_ms"] = self.sched_s * 1e3
        return out

    def close(self):
        for slot in self.slots:
            for g, *_ in slot.graphs.values():
                jk.jk_graph_destroy(g)
            slot.graphs.clear()
        for h in self.handles:
            h.close()


def summarize(reqs):
    lat = np.array([r.done_ms / 1e3 - r.arrival for r in reqs])
    first = min(r.arrival for r in reqs)
    last = max(r.done_ms / 1e3 for r in reqs)
    builds = sum(r.nd for r in reqs)
    return dict(requests=len(reqs), builds=builds, makespan_s=last - first, builds_per_s=builds / (last - first),
                p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
                mean_batch=float(np.mean([r.batch for r in reqs])),
                graph_fraction=float(np.mean([r.graph for r in reqs])))


def one_at_a_time(handles, reqs, opts, device="cuda:0", on_progress=None):
    """The plain form: one request after the other on one stream, each a
    separate jk_build as soon as it has arrived and the previous one is done."""
    dev = torch.device(device)
    reqs = sorted(reqs, key=lambda r: r.arrival)
    s = torch.cuda.Stream(device=dev)
    torch.cuda.synchronize(dev)
    start = torch.cuda.Event(enable_timing=True)
    start.record(s)
    t0 = time.perf_counter()
    for r in reqs:
        while time.perf_counter() - t0 < r.arrival:
            time.sleep(5e-5)
        r.J = torch.empty_like(r.D)
        r.K = torch.empty_like(r.D)
        with torch.cuda.stream(s):
            jk.jk_build(handles[r.mol].h, r.D, r.J, r.K, opts, s)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(s)
        ev.synchronize()
        r.done_ms = start.elapsed_time(ev)
        r.batch = 1
        if on_progress:
            on_progress(r.index + 1, len(reqs))
    return summarize(reqs)
