"""Serving on the GPU: queries of several resident graphs, arriving while others
run, are answered exactly as the same query run alone."""
import numpy as np
import pytest

import graphgen
import oracle
from gpu_helpers import announce, assert_sssp_matches, to_np

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("pull", [False, True])
def test_server_mix_equals_alone(dawn, pull):
    """pull=True: the tiles take pull steps (from 5 % of the edges in the
    frontier) while queries join and leave them."""
    prev = dawn.set_tuning(tile_pull=50, tile_pull_src=0) if pull else None
    try:
        _mix_equals_alone(dawn, pull)
    finally:
        if prev is not None:
            dawn.set_tuning(**prev)


def _mix_equals_alone(dawn, pull):
    import torch
    from paper_2306_07872_amd import serve
    gs = [graphgen.rmat(12, 8, 40, weights="u32"),
          graphgen.rmat(13, 16, 41, weights="f32lognormal"),
          graphgen.grid(48, 40, 0.01, 42, weights="f32unit")]
    csrs = [dawn.Csr.from_graph(g) for g in gs]
    srv = serve.Server(tile_k=64, steps_per_tick=3, max_tiles_per_graph=2, pull=pull)
    for i, c in enumerate(csrs):
        srv.add_graph(i, c)
    rng = np.random.default_rng(7)
    qs = []
    announce("server mix: 3 graphs, 90 queries, pull", pull)
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
