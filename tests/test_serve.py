"""Serving scheduler logic on the CPU, with an oracle-backed fake executor.

The fake stands in for a HIP tile session: a column admitted with source s
finishes after a number of step launches and then reads back the oracle's
distances.  Like the device, a run reports as done every column that is live
and no longer active when the run ends, including a finished column whose
query was already collected and which has not been reused yet.  The tests
check admission by HBM budget, FIFO service, column reuse, cancellation, and
that admissions while a run is in flight are never answered from that run's
done bits.
"""
import numpy as np
import pytest

import graphgen
import oracle
from paper_2306_07872_amd import serve


class FakeCsr:
    def __init__(self, g):
        self.g = g
        self.n, self.m, self.wtype = g.n, g.m, g.wtype


class FakeRead:
    def __init__(self, value, steps):
        self._v, self._s, self.polls = value, steps, 0

    def ready(self):
        self.polls += 1
        return self.polls >= 2

    def value(self):
        return self._v, self._s


class FakeExecutor:
    created = 0

    def __init__(self, csr, k, lag=1):
        FakeExecutor.created += 1
        self.csr, self.k, self.lag = csr, k, lag
        self.nbytes = 1
        self.cols = {}          # col -> [source, steps left, steps taken]; stays after done
        self.run_polls = None
        self.run_done = []
        self.admit_while_running = 0
        self.closed = False

    def admit(self, col, source):
        if self.run_polls is not None:
            self.admit_while_running += 1
        need = 1 + (source % 5)
        self.cols[col] = [source, need, 0]

    def evict(self, col):
        self.cols.pop(col, None)

    def launch(self, steps):
        for c in self.cols.values():
            take = min(steps, c[1])
            c[1] -= take
            c[2] += take
        # done bits as the device computes them when the run ends: live and idle
        self.run_done = [col for col, c in self.cols.items() if c[1] == 0]
        self.run_polls = 0

    def running(self):
        if self.run_polls is None:
            return False
        self.run_polls += 1
        return self.run_polls <= self.lag

    def finished_run(self):
        if self.run_polls is None:
            return False
        self.run_polls += 1
        return self.run_polls > self.lag

    def idle(self):
        return self.run_polls is None

    def done_cols(self):
        self.run_polls = None
        return list(self.run_done)

    def read(self, col):
        src, left, taken = self.cols[col]
        d, _ = oracle.sssp(self.csr.g, src)
        return FakeRead(d, taken)

    def close(self):
        self.closed = True


def make_server(budget, tile_k=4, steps=2, max_tiles=3, lag=1):
    import itertools
    ticks = itertools.count()
    clock = lambda: next(ticks) * 1e-3
    return serve.Server(hbm_budget=budget, tile_k=tile_k, steps_per_tick=steps,
                        max_tiles_per_graph=max_tiles,
                        tile_factory=lambda csr, k: FakeExecutor(csr, k, lag), clock=clock)


@pytest.fixture
def graphs():
    return [graphgen.er(60, 300, 1 + i, weights="u32" if i % 2 == 0 else "f32lognormal")
            for i in range(3)]


def _patch_cost(srv, cost):
    srv.tile_cost = lambda gid: cost


def test_all_queries_complete_with_oracle_answers(graphs):
    srv = make_server(budget=10)
    _patch_cost(srv, 1)
    for i, g in enumerate(graphs):
        srv.add_graph(i, FakeCsr(g))
    rng = np.random.default_rng(0)
    qs = [srv.submit(int(rng.integers(0, 3)), int(rng.integers(0, 60))) for _ in range(40)]
    srv.run_until_idle()
    for q in qs:
        assert q.state == "done"
        ref, _ = oracle.sssp(graphs[q.gid], q.source)
        assert np.array_equal(q.result, ref)
        assert q.steps == 1 + (q.source % 5)
        assert q.t_done >= q.t_admit >= q.t_arrive


def test_budget_limits_tiles_and_idle_tiles_are_reclaimed(graphs):
    srv = make_server(budget=1)   # room for one tile at a time
    _patch_cost(srv, 1)
    for i, g in enumerate(graphs):
        srv.add_graph(i, FakeCsr(g))
    qs = [srv.submit(i % 3, i) for i in range(12)]
    peak = 0
    while srv.busy():
        srv.tick()
        peak = max(peak, srv.hbm_used)
        assert srv.hbm_used <= srv.hbm_budget
    assert peak == 1
    assert all(q.state == "done" for q in qs)
    assert srv.refused_tiles > 0


def test_fifo_within_a_graph(graphs):
    srv = make_server(budget=1, tile_k=2, max_tiles=1)
    _patch_cost(srv, 1)
    srv.add_graph(0, FakeCsr(graphs[0]))
    qs = [srv.submit(0, 5 * i) for i in range(8)]   # equal step counts
    srv.run_until_idle()
    admit_order = sorted(qs, key=lambda q: (q.t_admit, q.qid))
    assert [q.qid for q in admit_order] == [q.qid for q in qs]


def test_cancel_waiting_and_running(graphs):
    srv = make_server(budget=1, tile_k=2, max_tiles=1, steps=1)
    _patch_cost(srv, 1)
    srv.add_graph(0, FakeCsr(graphs[0]))
    a = srv.submit(0, 4)    # 5 steps
    b = srv.submit(0, 9)
    c = srv.submit(0, 3)    # waits: no free column
    srv.tick()
    assert a.state == b.state == "running" and c.state == "waiting"
    srv.cancel(c)
    assert c.state == "cancelled"
    srv.tick()
    srv.tick()
    assert a.state == "running"
    srv.cancel(a)
    assert a.state == "cancelled"
    srv.run_until_idle()
    assert b.state == "done" and a.result is None and c.result is None


def test_admission_while_running_never_reads_an_early_answer(graphs):
    """A finished column is collected and freed; the next run is launched while
    it is still live on the device (so that run reports it done); a new query
    then takes the column while the run is in flight.  The run's done bit
    speaks for the old query and must not answer the new one."""
    srv = make_server(budget=5, tile_k=2, max_tiles=1, steps=2, lag=2)
    _patch_cost(srv, 1)
    srv.add_graph(0, FakeCsr(graphs[0]))
    q1 = srv.submit(0, 5)           # needs 1 step
    q2 = srv.submit(0, 4)           # needs 5 steps
    srv.tick()                      # admit q1 -> col 0, q2 -> col 1; run 1
    while q1.state != "done":
        srv.tick()                  # run 1 collected: q1 read, col 0 freed; run 2 launched
    slot = srv.tiles[0][0]
    assert not slot.ex.idle() and 0 in slot.ex.run_done
    q3 = srv.submit(0, 3)           # needs 4 steps; reuses col 0 while run 2 is in flight
    srv.tick()
    assert q3.state == "running" and q3._col == 0 and slot.ex.admit_while_running == 1
    srv.run_until_idle()
    for q in (q1, q2, q3):
        assert q.state == "done"
        assert q.steps == 1 + (q.source % 5)    # read only once its own steps were done
        ref, _ = oracle.sssp(graphs[0], q.source)
        assert np.array_equal(q.result, ref)


def test_poisson_arrivals_and_percentiles():
    u = np.linspace(0.01, 0.99, 1000)
    t = serve.poisson_arrivals(100.0, 1000, u)
    assert np.all(np.diff(t) > 0)
    assert abs(t[-1] / 1000 - 1 / 100.0) < 0.005
    p = serve.percentiles([0.001, 0.002, 0.003])
    assert abs(p["p50_ms"] - 2.0) < 1e-9


class FakeSolo:
    """Stands in for a lone single-source run: done after `lag` polls."""
    created = 0

    def __init__(self, csr, lag=2):
        FakeSolo.created += 1
        self.csr, self.lag = csr, lag
        self.src, self.polls, self.launches = None, 0, 0
        self.closed = False

    def launch(self, source):
        assert self.src is None
        self.src, self.polls = source, 0
        self.launches += 1

    def finished(self):
        if self.src is None:
            return False
        self.polls += 1
        return self.polls > self.lag

    def value(self):
        d, _ = oracle.sssp(self.csr.g, self.src)
        steps = 1 + (self.src % 5)
        self.src = None
        return d, steps, 1

    def close(self):
        self.closed = True


def make_solo_server(budget, tile_k=4, steps=2, max_tiles=3):
    import itertools
    ticks = itertools.count()
    clock = lambda: next(ticks) * 1e-3
    srv = serve.Server(hbm_budget=budget, tile_k=tile_k, steps_per_tick=steps,
                       max_tiles_per_graph=max_tiles,
                       tile_factory=lambda csr, k: FakeExecutor(csr, k, 1),
                       solo_factory=lambda csr: FakeSolo(csr), clock=clock)
    srv.tile_cost = lambda gid: 1
    srv.solo_cost = lambda gid: 1
    return srv


def test_lone_query_runs_alone_and_later_ones_join_tiles(graphs):
    srv = make_solo_server(budget=10)
    for i, g in enumerate(graphs):
        srv.add_graph(i, FakeCsr(g))
    a = srv.submit(0, 7)
    srv.tick()
    assert a.state == "running" and a._tile is None and 0 in srv.solo_query
    b = srv.submit(0, 3)             # arrives while the lone run is in flight
    c = srv.submit(1, 4)             # another graph, idle: runs alone too
    srv.tick()
    assert b.state == "running" and b._tile is not None
    assert c.state == "running" and c._tile is None
    srv.run_until_idle()
    for q in (a, b, c):
        assert q.state == "done"
        ref, _ = oracle.sssp(graphs[q.gid], q.source)
        assert np.array_equal(q.result, ref)
        assert q.steps == 1 + (q.source % 5)


def test_queries_arriving_together_share_a_tile(graphs):
    srv = make_solo_server(budget=10)
    srv.add_graph(0, FakeCsr(graphs[0]))
    qs = [srv.submit(0, s) for s in (1, 2, 3)]
    srv.tick()
    assert not srv.solo_query and all(q._tile is not None for q in qs)
    srv.run_until_idle()
    assert all(q.state == "done" for q in qs)


def test_lone_runs_count_against_the_budget_and_are_reclaimed(graphs):
    srv = make_solo_server(budget=1)
    for i, g in enumerate(graphs):
        srv.add_graph(i, FakeCsr(g))
    qs = []
    for i in range(9):
        qs.append(srv.submit(i % 3, i))
        srv.tick()
        assert srv.hbm_used <= srv.hbm_budget
    srv.run_until_idle()
    assert all(q.state == "done" for q in qs)
    for q in qs:
        ref, _ = oracle.sssp(graphs[q.gid], q.source)
        assert np.array_equal(q.result, ref)


def test_cancel_a_lone_run(graphs):
    srv = make_solo_server(budget=10)
    srv.add_graph(0, FakeCsr(graphs[0]))
    a = srv.submit(0, 2)
    srv.tick()
    assert a._tile is None
    srv.cancel(a)
    srv.run_until_idle()
    assert a.state == "cancelled" and a.result is None and not srv.solo_query
