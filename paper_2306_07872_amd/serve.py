"""Continuous-batching SSSP server on resident graphs.

Queries (graph id, source) are served from per-graph tile sessions
(``dawn_tile_*``): a tile holds the distance state of up to `tile_k` queries
of one graph as the columns of an [n x K] tile in HBM.  The scheduler works in
ticks:

1. collect: tiles whose last run has finished report their done columns; each
   finished column is copied out (device -> pinned host) and the column is
   freed as soon as the copy is enqueued;
2. admit: waiting queries (FIFO per graph) take free columns of a tile of
   their graph; a graph without a free column gets a new tile if the HBM
   budget still holds it, otherwise its queries wait;
3. run: every tile with live columns that is not already running gets
   `steps_per_tick` GOVM steps enqueued on its own stream (by default as one
   replay of a HIP graph captured at the tile's first run), followed by an
   asynchronous copy of its done bits and an event.

A tile takes new columns also while a run of it is in flight: the admission
is enqueued on the tile's stream behind that run and joins the next run.  The
done bits of a run are taken only for columns admitted before the run was
launched (a column's previous query stays live on the device until the column
is reused, so the bits of a run launched before a reuse speak for that
previous query).

Columns join and leave a running tile between step chunks; the arithmetic of
a column does not depend on the other columns (different sources never update
the same path, Section 3.5), so each answer is the same alone and in the mix.
The host never waits on the device: it polls events.

A query that finds its graph idle -- no live tile column, no lone run in
flight, no other query of the graph waiting -- runs alone as a plain
single-source run (``dawn_sssp_ws``) on the graph's own stream: one column of
a tile pays for the whole tile's row width on every distance it touches,
about twice the time of the single-source kernels on the largest graphs.
Queries of that graph arriving meanwhile go to tiles as usual.  The
distances are the same either way (they are unique).

The executor is pluggable (``tile_factory``) so the scheduling logic can be
exercised without a GPU; the default executor is the HIP tile session.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

from . import (INFO_BYTES, Csr, Tile, dist_dtype, done_columns, get_tuning, info_tensor,
               read_info, set_tuning, sssp, sssp_workspace_bytes, tgraph, tile_bytes, workspace)


@dataclass
class Query:
    qid: int
    gid: int
    source: int
    t_arrive: float
    t_admit: float | None = None
    t_done: float | None = None
    state: str = "waiting"        # waiting | running | reading | done | cancelled | failed
    result: object = None         # host numpy array once done
    steps: int | None = None
    status: int | None = None     # run status of a failed lone run (dawn_run_info.converged)
    _col: int | None = None
    _tile: object = None
    _read: object = None
    _admit_run: int = 0           # runs of its tile launched before its admission

    @property
    def latency(self) -> float | None:
        return None if self.t_done is None else self.t_done - self.t_arrive


class GpuTileExecutor:
    """One HIP tile session with its own stream, pinned host buffers and events."""

    def __init__(self, csr: Csr, k: int, device="cuda", tgraph=None, graphs: bool = True):
        import torch
        self.torch = torch
        self.csr = csr
        self.k = k
        self.stream = torch.cuda.Stream(device=device)   # default priority
        with torch.cuda.stream(self.stream):
            self.tile = Tile(csr, k, stream=self.stream)
        if tgraph is not None:
            self.tile.set_tgraph(tgraph)
        self.done_host = torch.zeros((k + 31) // 32, dtype=torch.int32, pin_memory=True)
        self.nbytes = tile_bytes(csr.n, csr.m, k)
        self._run_event = None
        # graphs: a run of s steps is captured once as a HIP graph and
        # replayed (one launch per tick instead of 3 s + 1)
        self.graphs = graphs
        self._captured = None

    # -- steps ---------------------------------------------------------------
    def admit(self, col: int, source: int):
        self.tile.admit(col, source, stream=self.stream)

    def evict(self, col: int):
        self.tile.evict(col, stream=self.stream)

    def launch(self, steps: int):
        torch = self.torch
        if self.graphs:
            if self._captured != steps:
                self.tile.capture(steps)
                self._captured = steps
            done = self.tile.replay(stream=self.stream)
        else:
            done = self.tile.run(steps, stream=self.stream)
        with torch.cuda.stream(self.stream):
            self.done_host.copy_(done, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.stream)
        self._run_event = ev

    def running(self) -> bool:
        return self._run_event is not None and not self._run_event.query()

    def finished_run(self) -> bool:
        return self._run_event is not None and self._run_event.query()

    def idle(self) -> bool:
        """No run in flight and none waiting to be collected."""
        return self._run_event is None

    def done_cols(self) -> list[int]:
        self._run_event = None
        return done_columns(self.done_host.numpy(), self.k)

    # -- results ---------------------------------------------------------------
    def read(self, col: int):
        """Enqueue the copy of column col to pinned host memory; returns a
        handle with ready() / value()."""
        torch = self.torch
        with torch.cuda.stream(self.stream):
            dev = self.tile.read(col, stream=self.stream)
            host = torch.empty(self.csr.n, dtype=dist_dtype(self.csr.wtype), pin_memory=True)
            host.copy_(dev, non_blocking=True)
            steps = self.tile.steps(stream=self.stream)
            steps_host = torch.empty_like(steps, device="cpu", pin_memory=True)
            steps_host.copy_(steps, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.stream)
        return _ReadHandle(ev, host, steps_host, col, keep=(dev, steps))

    def close(self):
        self.stream.synchronize()
        self.tile.close()


class GpuSoloExecutor:
    """Lone queries of one graph as plain single-source runs on the graph's
    own stream, one at a time, with the result copied to pinned host memory."""

    def __init__(self, csr: Csr, device="cuda"):
        import torch
        self.torch = torch
        self.csr = csr
        self.stream = torch.cuda.Stream(device=device)   # default priority
        nws = sssp_workspace_bytes(csr.n, csr.m)
        # allocated (and the run info zeroed) on the executor's own stream, so
        # the zeroing is ordered before the first run on that stream
        with torch.cuda.stream(self.stream):
            self.ws = workspace(nws, device)
            self.out = torch.empty(csr.n, dtype=dist_dtype(csr.wtype), device=device)
            self.info = info_tensor(device)
        self.nbytes = nws + 4 * csr.n + INFO_BYTES
        self._pending = None

    def launch(self, source: int):
        torch = self.torch
        # Kernels of other streams (tiles, other lone runs) share the compute
        # units, so the run must not wait at a grid barrier for workgroups
        # that cannot start: past the one-workgroup size it takes step
        # launches and, for the steps after them, a one-workgroup persistent
        # launch.
        prev = None
        if self.csr.m > get_tuning()["small_m"]:
            prev = set_tuning(mode=1, ss_tail_grid=1)
        try:
            with torch.cuda.stream(self.stream):
                sssp(self.csr, source, out=self.out, ws=self.ws, info=self.info,
                     stream=self.stream, check=False)
        finally:
            if prev is not None:
                set_tuning(**prev)
        with torch.cuda.stream(self.stream):
            host = torch.empty(self.csr.n, dtype=self.out.dtype, pin_memory=True)
            host.copy_(self.out, non_blocking=True)
            info_host = torch.empty(INFO_BYTES, dtype=torch.uint8, pin_memory=True)
            info_host.copy_(self.info, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.stream)
        self._pending = (ev, host, info_host)

    def busy(self) -> bool:
        return self._pending is not None

    def finished(self) -> bool:
        return self._pending is not None and self._pending[0].query()

    def value(self):
        """(distances, steps, converged) of the finished run."""
        _, host, info_host = self._pending
        self._pending = None
        inf = read_info(info_host)
        return host.numpy(), inf["steps"], inf["converged"]

    def close(self):
        self.stream.synchronize()


class _ReadHandle:
    def __init__(self, ev, host, steps_host, col, keep):
        self.ev, self.host, self.steps_host, self.col, self._keep = ev, host, steps_host, col, keep

    def ready(self) -> bool:
        return self.ev.query()

    def value(self):
        return self.host.numpy(), int(self.steps_host.numpy()[self.col])


class _TileSlot:
    def __init__(self, gid: int, ex):
        self.gid = gid
        self.ex = ex
        self.free = list(range(ex.k))
        self.live: dict[int, Query] = {}
        self.runs = 0                 # runs launched so far


class Server:
    """Continuous-batching SSSP over resident graphs (see module docstring)."""

    def __init__(self, hbm_budget: int | None = None, tile_k: int = 64, steps_per_tick: int = 4,
                 max_tiles_per_graph: int = 4, tile_factory=None, clock=time.perf_counter,
                 device="cuda", pull: bool = True, graphs: bool = True, solo: bool = True,
                 solo_factory=None):
        self.graphs: dict[int, Csr] = {}
        # pull steps need each graph's reverse graph, built when the graph is
        # added and resident with it (like the CSR, outside the tile budget);
        # only the HIP executor uses them
        self.pull = pull and tile_factory is None
        self.tile_k = tile_k
        self.steps_per_tick = steps_per_tick
        self.max_tiles_per_graph = max_tiles_per_graph
        self.device = device
        self.clock = clock
        self.tile_factory = tile_factory or (
            lambda csr, k: GpuTileExecutor(csr, k, device,
                                           getattr(csr, "_tgraph", None) if self.pull else None,
                                           graphs))
        # lone queries as plain single-source runs (with a custom tile executor
        # only when a matching solo executor is given too)
        self.solo = solo and (tile_factory is None or solo_factory is not None)
        self.solo_factory = solo_factory or (lambda csr: GpuSoloExecutor(csr, device))
        self.solos: dict[int, object] = {}
        self.solo_query: dict[int, Query] = {}
        if hbm_budget is None:
            import torch
            free, _ = torch.cuda.mem_get_info()
            hbm_budget = int(free * 0.8)
        self.hbm_budget = int(hbm_budget)
        self.hbm_used = 0
        self.tiles: dict[int, list[_TileSlot]] = collections.defaultdict(list)
        self.waiting: collections.deque[Query] = collections.deque()
        self.reading: list[Query] = []
        self.done: list[Query] = []
        self._next_qid = 0
        self.refused_tiles = 0

    # -- graphs and queries -------------------------------------------------
    def add_graph(self, gid: int, csr: Csr):
        self.graphs[gid] = csr
        if self.pull:
            tgraph(csr)

    def tile_cost(self, gid: int) -> int:
        c = self.graphs[gid]
        return tile_bytes(c.n, c.m, self.tile_k)

    def solo_cost(self, gid: int) -> int:
        c = self.graphs[gid]
        return sssp_workspace_bytes(c.n, c.m) + 4 * c.n + INFO_BYTES

    def submit(self, gid: int, source: int, t_arrive: float | None = None) -> Query:
        if gid not in self.graphs:
            raise KeyError(f"graph {gid} is not resident")
        if not 0 <= source < self.graphs[gid].n:
            raise ValueError("source out of range")
        q = Query(self._next_qid, gid, int(source), self.clock() if t_arrive is None else t_arrive)
        self._next_qid += 1
        self.waiting.append(q)
        return q

    def cancel(self, q: Query):
        if q.state == "waiting":
            self.waiting.remove(q)
            q.state = "cancelled"
        elif q.state == "running" and q._tile is None:
            q.state = "cancelled"     # a lone run: its result is dropped when it ends
        elif q.state == "running":
            slot = q._tile
            slot.ex.evict(q._col)
            del slot.live[q._col]
            slot.free.append(q._col)
            q.state = "cancelled"

    # -- scheduling -----------------------------------------------------------
    def _collect(self):
        now = None
        for gid in list(self.solo_query):
            ex = self.solos[gid]
            if not ex.finished():
                continue
            q = self.solo_query.pop(gid)
            d, steps, conv = ex.value()
            if q.state == "cancelled":
                continue
            now = self.clock() if now is None else now
            q.t_done = now
            if conv != 1:
                q.state, q.status = "failed", conv
                continue
            q.result, q.steps = d, steps
            q.state = "done"
            self.done.append(q)
        for gid, slots in self.tiles.items():
            for slot in slots:
                if not slot.ex.finished_run():
                    continue
                for col in slot.ex.done_cols():
                    q = slot.live.get(col)
                    if q is None or q._admit_run >= slot.runs:
                        continue    # free, or admitted after this run was launched
                    del slot.live[col]
                    q._read = slot.ex.read(col)
                    q.state = "reading"
                    slot.free.append(col)   # the read is enqueued before any later admit
                    self.reading.append(q)
        still = []
        for q in self.reading:
            if q._read.ready():
                now = self.clock() if now is None else now
                q.result, q.steps = q._read.value()
                q._read = None
                q.t_done = now
                q.state = "done"
                self.done.append(q)
            else:
                still.append(q)
        self.reading = still

    def _slot_for(self, gid: int):
        for slot in self.tiles[gid]:
            if slot.free:
                return slot
        if len(self.tiles[gid]) >= self.max_tiles_per_graph:
            return None
        cost = self.tile_cost(gid)
        if self.hbm_used + cost > self.hbm_budget:
            self._reclaim(cost)
        if self.hbm_used + cost > self.hbm_budget:
            self.refused_tiles += 1
            return None
        slot = _TileSlot(gid, self.tile_factory(self.graphs[gid], self.tile_k))
        self.hbm_used += cost
        self.tiles[gid].append(slot)
        return slot

    def _solo_for(self, gid: int):
        """The graph's lone-query executor (created within the HBM budget), or None."""
        ex = self.solos.get(gid)
        if ex is not None:
            return ex
        cost = self.solo_cost(gid)
        if self.hbm_used + cost > self.hbm_budget:
            self._reclaim(cost)
        if self.hbm_used + cost > self.hbm_budget:
            return None
        ex = self.solo_factory(self.graphs[gid])
        self.solos[gid] = ex
        self.hbm_used += cost
        return ex

    def _reclaim(self, need: int):
        """Destroy idle tiles (no live columns, not running) and idle lone-query
        executors until `need` fits."""
        for gid in list(self.solos):
            if self.hbm_used + need <= self.hbm_budget:
                return
            if gid not in self.solo_query:
                self.solos.pop(gid).close()
                self.hbm_used -= self.solo_cost(gid)
        for gid, slots in self.tiles.items():
            for slot in list(slots):
                if self.hbm_used + need <= self.hbm_budget:
                    return
                if not slot.live and slot.ex.idle() and len(slot.free) == slot.ex.k:
                    slot.ex.close()
                    slots.remove(slot)
                    self.hbm_used -= self.tile_cost(gid)

    def _admit(self):
        now = self.clock()
        blocked = set()
        keep = collections.deque()
        waiting_per_graph = collections.Counter(q.gid for q in self.waiting)
        while self.waiting:
            q = self.waiting.popleft()
            if q.gid in blocked:
                keep.append(q)
                continue
            if (self.solo and waiting_per_graph[q.gid] == 1 and q.gid not in self.solo_query
                    and not any(s.live for s in self.tiles[q.gid])):
                ex = self._solo_for(q.gid)
                if ex is not None:
                    ex.launch(q.source)
                    self.solo_query[q.gid] = q
                    q._tile, q._col = None, None
                    q.state, q.t_admit = "running", now
                    waiting_per_graph[q.gid] -= 1
                    continue
            waiting_per_graph[q.gid] -= 1
            slot = self._slot_for(q.gid)
            if slot is None:
                blocked.add(q.gid)
                keep.append(q)
                continue
            col = slot.free.pop(0)
            slot.ex.admit(col, q.source)
            slot.live[col] = q
            q._col, q._tile, q._admit_run = col, slot, slot.runs
            q.state, q.t_admit = "running", now
        self.waiting = keep

    def _run(self):
        # a tile is launched again only after its previous run was collected
        for slots in self.tiles.values():
            for slot in slots:
                if slot.live and slot.ex.idle():
                    slot.ex.launch(self.steps_per_tick)
                    slot.runs += 1

    def tick(self) -> int:
        """One scheduling round; returns how many queries finished in it."""
        before = len(self.done)
        self._collect()
        self._admit()
        self._run()
        return len(self.done) - before

    def busy(self) -> bool:
        return bool(self.waiting or self.reading or self.solo_query or
                    any(s.live for slots in self.tiles.values() for s in slots))

    def run_until_idle(self, max_ticks: int = 10_000_000):
        for _ in range(max_ticks):
            if not self.busy():
                return
            self.tick()
        raise RuntimeError("server did not drain")

    def close(self):
        for slots in self.tiles.values():
            for slot in slots:
                slot.ex.close()
        for ex in self.solos.values():
            ex.close()
        self.tiles.clear()
        self.solos.clear()
        self.solo_query.clear()
        self.hbm_used = 0


def poisson_arrivals(rate_per_s: float, count: int, uniforms: np.ndarray) -> np.ndarray:
    """Arrival times (s) of a Poisson process from `count` uniforms in [0,1)."""
    gaps = -np.log1p(-uniforms[:count]) / rate_per_s
    return np.cumsum(gaps)


def percentiles(lat_s) -> dict:
    a = np.asarray(lat_s, dtype=np.float64) * 1e3
    if a.size == 0:
        return {"p50_ms": None, "p99_ms": None, "mean_ms": None}
    return {"p50_ms": float(np.percentile(a, 50)), "p99_ms": float(np.percentile(a, 99)),
            "mean_ms": float(a.mean())}


def serve_open_loop(server: Server, arrivals, requests, clock=time.perf_counter) -> dict:
    """Replay (time, gid, source) requests against `server` in real time:
    each request is submitted when its arrival time has passed.  Returns
    latency percentiles and throughput."""
    order = np.argsort(arrivals, kind="stable")
    t0 = clock()
    i = 0
    qs = []
    while i < len(order) or server.busy():
        now = clock() - t0
        while i < len(order) and arrivals[order[i]] <= now:
            gid, src = requests[order[i]]
            qs.append(server.submit(gid, src, t_arrive=t0 + arrivals[order[i]]))
            i += 1
        server.tick()
    t1 = clock()
    lat = [q.latency for q in qs if q.state == "done"]
    out = percentiles(lat)
    out["completed"] = len(lat)
    out["queries_per_s"] = len(lat) / (t1 - t0) if t1 > t0 else None
    out["wall_s"] = t1 - t0
    return out
