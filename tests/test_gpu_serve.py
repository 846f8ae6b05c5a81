"""Serving on the GPU: queries of several resident graphs, arriving while others
run, are answered exactly as the same query run alone."""
import numpy as np
import pytest

import graphgen
import oracle
from gpu_helpers import announce, assert_sssp_matches, to_np

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("pull,graphs,solo", [(False, False, True), (False, True, False),
                                              (True, True, True)])
def test_server_mix_equals_alone(dawn, pull, graphs, solo):
    """pull=True: the tiles take pull steps (from 5 % of the edges in the
    frontier) while queries join and leave them.  graphs=True: each tick's
    steps are a replay of the tile's captured run."""
    prev = dawn.set_tuning(tile_pull=50, tile_pull_src=0) if pull else None
    try:
        _mix_equals_alone(dawn, pull, graphs, solo)
    finally:
        if prev is not None:
            dawn.set_tuning(**prev)


def _mix_equals_alone(dawn, pull, graphs, solo):
    import torch
    from paper_2306_07872_amd import serve
    gs = [graphgen.rmat(12, 8, 40, weights="u32"),
          graphgen.rmat(13, 16, 41, weights="f32lognormal"),
          graphgen.grid(48, 40, 0.01, 42, weights="f32unit")]
    csrs = [dawn.Csr.from_graph(g) for g in gs]
    srv = serve.Server(tile_k=64, steps_per_tick=3, max_tiles_per_graph=2, pull=pull,
                       graphs=graphs, solo=solo)
    for i, c in enumerate(csrs):
        srv.add_graph(i, c)
    rng = np.random.default_rng(7)
    qs = []
    announce("server mix: 3 graphs, 90 queries, pull", pull, "graphs", graphs)
    for t in range(90):
        gi = int(rng.integers(0, 3))
        src = int(graphgen.pick_sources(gs[gi], 1, 1000 + t)[0])
        qs.append(srv.submit(gi, src))
        srv.tick()                    # arrivals interleave with running work
    srv.run_until_idle()
    torch.cuda.synchronize()
    for q in qs:
        assert q.state == "done"
        alone = to_np(dawn.sssp(csrs[q.gid], q.source))
        torch.cuda.synchronize()
        assert np.array_equal(np.asarray(q.result).view(np.uint32), alone.view(np.uint32)), q.qid
    for q in qs[::15]:
        assert_sssp_matches(gs[q.gid], q.source, q.result, tag=f"served q{q.qid}")
    srv.close()


def test_server_tiny_budget_still_serves_everything(dawn):
    import torch
    from paper_2306_07872_amd import serve
    gs = [graphgen.er(2000, 16000, 50 + i, weights="u32") for i in range(3)]
    csrs = [dawn.Csr.from_graph(g) for g in gs]
    one_tile = dawn.tile_bytes(2000, 16000, 64)
    srv = serve.Server(hbm_budget=one_tile, tile_k=64, steps_per_tick=2)
    for i, c in enumerate(csrs):
        srv.add_graph(i, c)
    qs = [srv.submit(i % 3, (37 * i) % 2000) for i in range(30)]
    announce("server tiny budget")
    peak = 0
    while srv.busy():
        srv.tick()
        peak = max(peak, srv.hbm_used)
    assert peak <= one_tile
    torch.cuda.synchronize()
    for q in qs:
        ref, _ = oracle.sssp(gs[q.gid], q.source)
        assert np.array_equal(np.asarray(q.result).view(np.uint32), ref)
    srv.close()


def test_server_cancel_running_query(dawn):
    import torch
    from paper_2306_07872_amd import serve
    g = graphgen.grid(64, 64, 0.0, 3, weights="f32unit")
    csr = dawn.Csr.from_graph(g)
    srv = serve.Server(tile_k=64, steps_per_tick=1, max_tiles_per_graph=1)
    srv.add_graph(0, csr)
    a = srv.submit(0, 0)
    b = srv.submit(0, 4095)
    srv.tick()
    srv.tick()
    srv.cancel(a)
    c = srv.submit(0, 2080)
    srv.run_until_idle()
    torch.cuda.synchronize()
    assert a.state == "cancelled" and b.state == "done" and c.state == "done"
    for q in (b, c):
        assert_sssp_matches(g, q.source, q.result, tag=f"cancel-mix q{q.qid}")
    srv.close()


@pytest.mark.parametrize("pull", [False, True])
def test_tile_replay_equals_run(dawn, pull):
    """A captured run replayed tick after tick, with admissions, reads and
    eager work on the stream between replays, does what dawn_tile_run does:
    after every replay, each column it reports done holds the lone query's
    distances, as in an eagerly run twin tile.  (The step at which a column
    finishes may differ between the two: a step relaxes in place, so a
    distance lowered earlier in the same step can carry further.)"""
    import torch
    g = graphgen.rmat(12, 16, 61, weights="u32")
    csr = dawn.Csr.from_graph(g)
    srcs = [int(s) for s in graphgen.pick_sources(g, 6, 62)]
    alone = {c: None for c in range(len(srcs))}
    prev = dawn.set_tuning(tile_pull=50, tile_pull_src=0) if pull else None
    try:
        tg = dawn.tgraph(csr) if pull else None
        tiles = {"replay": dawn.Tile(csr, 64), "run": dawn.Tile(csr, 64)}
        if pull:
            for t in tiles.values():
                t.set_tgraph(tg)
        tiles["replay"].capture(2)
        announce("tile replay vs run, pull", pull)
        done = {name: set() for name in tiles}
        for tick in range(40):
            if tick < len(srcs):            # one admission per tick, into both tiles
                for t in tiles.values():
                    t.admit(tick, srcs[tick])
            bits = {"replay": to_np(tiles["replay"].replay()).copy(),
                    "run": to_np(tiles["run"].run(2)).copy()}
            torch.cuda.synchronize()
            for name, t in tiles.items():
                for c in range(min(tick + 1, len(srcs))):
                    if c in done[name] or not (int(bits[name][c // 32]) >> (c % 32)) & 1:
                        continue
                    done[name].add(c)
                    if alone[c] is None:
                        alone[c] = to_np(dawn.sssp(csr, srcs[c]))
                    x = to_np(t.read(c))
                    torch.cuda.synchronize()
                    assert np.array_equal(x, alone[c]), (name, tick, c)
            if all(len(d) == len(srcs) for d in done.values()):
                break
        assert all(len(d) == len(srcs) for d in done.values()), done
        for t in tiles.values():
            t.close()
    finally:
        if prev is not None:
            dawn.set_tuning(**prev)


def test_tile_replay_without_capture_is_rejected(dawn):
    g = graphgen.rmat(8, 8, 63, weights="u32")
    t = dawn.Tile(dawn.Csr.from_graph(g), 64)
    try:
        with pytest.raises(dawn.DawnError):
            t.replay()
        with pytest.raises(dawn.DawnError):
            t.capture(0)
    finally:
        t.close()


def test_lone_queries_run_alone_and_match_the_oracle(dawn):
    """Queries that find their graph idle run as plain single-source runs; one
    arriving while such a run is in flight joins a tile; all are exact."""
    import torch
    from paper_2306_07872_amd import serve
    gs = [graphgen.rmat(14, 16, 60, weights="u32"), graphgen.rmat(13, 8, 61, weights="f32lognormal")]
    csrs = [dawn.Csr.from_graph(g) for g in gs]
    srv = serve.Server(tile_k=64, steps_per_tick=2, max_tiles_per_graph=1)
    for i, c in enumerate(csrs):
        srv.add_graph(i, c)
    announce("server lone queries")
    s0 = graphgen.pick_sources(gs[0], 3, 5)
    a = srv.submit(0, int(s0[0]))
    srv.tick()
    assert a.state == "running" and a._tile is None
    b = srv.submit(0, int(s0[1]))
    c = srv.submit(1, int(graphgen.pick_sources(gs[1], 1, 6)[0]))
    srv.tick()
    assert b._tile is not None and c._tile is None
    srv.run_until_idle()
    torch.cuda.synchronize()
    srv.close()
    for q in (a, b, c):
        assert q.state == "done" and q.steps > 0
        assert_sssp_matches(gs[q.gid], q.source, q.result, tag=f"lone q{q.qid}")
