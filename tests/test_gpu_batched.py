"""GPU parity of the batched paths: multi-source tiles, all pairs, the
many-graph launch, and tile sessions."""
import numpy as np
import pytest

import graphgen
import oracle
from graphgen import workloads
from gpu_helpers import announce, assert_sssp_matches, to_np

pytestmark = pytest.mark.gpu


def _msssp(dawn, g, sources, **tune):
    import torch
    prev = dawn.set_tuning(**tune) if tune else None
    try:
        csr = dawn.Csr.from_graph(g)
        info = dawn.info_tensor()
        out = dawn.msssp(csr, sources, info=info)
        torch.cuda.synchronize()
        return to_np(out), dawn.read_info(info)
    finally:
        if prev is not None:
            dawn.set_tuning(**prev)


@pytest.mark.parametrize("wk", ["u32", "f32lognormal"])
@pytest.mark.parametrize("k", [1, 37, 64, 130])
def test_msssp_columns_match_oracle(dawn, wk, k):
    g = graphgen.rmat(13, 16, 3, weights=wk)
    srcs = graphgen.pick_sources(g, k, 11)
    announce("msssp", wk, "k", k)
    D, info = _msssp(dawn, g, srcs)
    assert D.shape == (k, g.n)
    for j in range(0, k, max(1, k // 6)):
        assert_sssp_matches(g, int(srcs[j]), D[j], tag=f"msssp k={k} col {j}")
    assert info["converged"] == 1


TILE_TUNINGS = [
    dict(),
    dict(tile_k=64, tile_t_wave=32, tile_t_chunk=64),
    dict(tile_k=128, tile_t_wave=65536, wg_threads=1024),
    dict(tile_k=512, tile_t_wave=40, tile_t_chunk=100, wg_threads=512, grid=5),
    dict(mode=1, tile_step_launches=3, tile_t_wave=32, tile_t_chunk=64),
    dict(tile_step_launches=4096),          # every step a step launch
    dict(tile_step_launches=1, tile_t_wave=32, tile_t_chunk=64),
    dict(tile_t_group=0, tile_skip=0),
    dict(tile_t_group=31, tile_t_wave=32, tile_t_chunk=64, wg_threads=512),
    dict(mode=2, tile_skip=0),
    dict(mode=2, tile_t_group=64, tile_t_wave=100, wg_threads=1024),
    dict(tile_sparse=0),                    # segment mapping everywhere
    dict(tile_sparse=512, tile_skip=1),     # one edge per lane everywhere
    dict(tile_sparse=3, tile_t_wave=32, tile_t_chunk=64, tile_skip=1, wg_threads=512),
]


# One-segment tiles (K <= 64): group-tier rows with at most tile_sparse active
# sources are relaxed one edge per lane.
ONE_SEG_TUNINGS = [
    dict(),
    dict(tile_sparse=64, tile_t_group=64, tile_t_wave=128),  # every group-tier row, up to 64 edges
    dict(tile_sparse=0),                     # never
    dict(tile_sparse=64, tile_t_group=64, tile_t_wave=128, mode=2),
    dict(tile_sparse=2, tile_t_group=16, tile_step_launches=4096, tile_skip=1),
]


@pytest.mark.parametrize("wk", ["u32", "f32lognormal"])
@pytest.mark.parametrize("ti", range(len(ONE_SEG_TUNINGS)))
def test_one_segment_tile_rows_one_edge_per_lane(dawn, wk, ti):
    """Every column of a one-segment tile matches the oracle whichever rows
    take the lane-per-edge path, on R-MAT and on a many-step grid."""
    for g in (graphgen.rmat(12, 16, 31, weights=wk), graphgen.grid(40, 30, 0.02, 32)):
        srcs = graphgen.pick_sources(g, 50, 7 + ti)
        announce("one-segment tile", g.name, g.wtype, ONE_SEG_TUNINGS[ti])
        D, info = _msssp(dawn, g, srcs, **ONE_SEG_TUNINGS[ti])
        for j in range(len(srcs)):
            assert_sssp_matches(g, int(srcs[j]), D[j], tag=f"{g.name} col {j}")
        assert info["converged"] == 1


@pytest.mark.parametrize("ti", range(len(TILE_TUNINGS)))
def test_msssp_tuning_invariance_and_sssp_identity(dawn, ti):
    """Column j of a tile equals a lone single-source run from sources[j]
    bit for bit, whatever the tile width, tiers or launch geometry."""
    import torch
    g = graphgen.rmat(14, 16, 9, weights="u32")
    srcs = graphgen.pick_sources(g, 150, ti)
    srcs = np.concatenate([srcs, srcs[:3]])  # duplicate sources are allowed
    announce("msssp tuning", TILE_TUNINGS[ti])
    D, info = _msssp(dawn, g, srcs, **TILE_TUNINGS[ti])
    csr = dawn.Csr.from_graph(g)
    for j in (0, 1, 77, 149, 150, 152):
        lone = to_np(dawn.sssp(csr, int(srcs[j])))
        torch.cuda.synchronize()
        assert np.array_equal(D[j].view(np.uint32), lone.view(np.uint32))
    ref, _ = oracle.sssp(g, int(srcs[5]), "u32")
    assert np.array_equal(D[5].view(np.uint32), ref)


def test_msssp_grid_f32(dawn):
    g = graphgen.grid(64, 48, 0.01, 3, weights="f32unit")
    srcs = graphgen.pick_sources(g, 70, 1)
    announce("msssp grid f32")
    D, info = _msssp(dawn, g, srcs)
    for j in (0, 33, 69):
        assert_sssp_matches(g, int(srcs[j]), D[j], tag=f"grid col {j}")


def test_msssp_unit_weight_counters(dawn):
    """Unit weights: per-source counters are the sums of the per-source exact
    values (mu = 1 for every source)."""
    g = graphgen.rmat(12, 8, 4, weights="u32one")
    srcs = graphgen.pick_sources(g, 40, 2)
    D, info = _msssp(dawn, g, srcs)
    exp_edges = sum(oracle.m_reach(g, int(s)) for s in srcs)
    exp_impr = sum(int((oracle.bfs(g, int(s)) >= 0).sum()) - 1 for s in srcs)
    exp_steps = max(int(oracle.bfs(g, int(s)).max()) + 1 for s in srcs)
    assert info["edges_scanned"] == exp_edges
    assert info["improvements"] == exp_impr
    assert info["steps"] == exp_steps
    assert info["union_edges"] <= info["edges_scanned"]


def test_apsp_er_small_equals_floyd_warshall(dawn):
    import torch
    g, _ = workloads.er_small()
    csr = dawn.Csr.from_graph(g)
    announce("apsp er_small")
    A = to_np(dawn.apsp(csr))
    torch.cuda.synchronize()
    F = oracle.fw(g)
    exp = np.where(F == np.iinfo(np.uint64).max, 0xFFFFFFFF, F).astype(np.uint32)
    assert np.array_equal(A.view(np.uint32), exp)
    assert np.all(np.diag(A) == 0)


def test_apsp_f32_small(dawn):
    import torch
    g = graphgen.er(300, 1500, 8, weights="f32lognormal")
    csr = dawn.Csr.from_graph(g)
    A = to_np(dawn.apsp(csr))
    torch.cuda.synchronize()
    for s in (0, 150, 299):
        assert_sssp_matches(g, s, A[s], tag=f"apsp row {s}")


def _batch_graphs(count=9, seed=7):
    return workloads.er_batch(seed=seed, count=count, lo=2.0, hi=3.7)


def test_batch_union_matches_each_graph(dawn):
    import torch
    gs = _batch_graphs()
    csrs = [dawn.Csr.from_graph(g) for g, _ in gs]
    b = dawn.Batch(csrs)
    srcs = torch.tensor([s for _, s in gs], dtype=torch.int32, device="cuda")
    info = dawn.info_tensor()
    announce("batch", len(gs), "graphs, total_n", b.total_n)
    out = b.run(srcs, info=info)
    torch.cuda.synchronize()
    parts = b.split(out)
    for (g, s), d in zip(gs, parts):
        assert_sssp_matches(g, s, to_np(d), tag=f"batch {g.name}")
    assert dawn.read_info(info)["converged"] == 1
    b.close()


def test_batch_union_held_in_lds(dawn):
    """A union small enough to sit whole in LDS (n <= 6144, m <= 16384) runs in
    the one-workgroup edge-parallel kernel with one seed per graph (vertex
    offsets); each graph's distances equal the oracle's."""
    import torch
    gs = workloads.er_batch(seed=9, count=4, lo=2.0, hi=2.6)
    assert sum(g.n for g, _ in gs) <= 6144 and sum(g.m for g, _ in gs) <= 16384
    csrs = [dawn.Csr.from_graph(g) for g, _ in gs]
    b = dawn.Batch(csrs)
    srcs = torch.tensor([s for _, s in gs], dtype=torch.int32, device="cuda")
    info = dawn.info_tensor()
    announce("batch in LDS", len(gs), "graphs, total_n", b.total_n)
    out = b.run(srcs, info=info)
    torch.cuda.synchronize()
    for (g, s), d in zip(gs, b.split(out)):
        assert_sssp_matches(g, s, to_np(d), tag=f"lds batch {g.name}")
    assert dawn.read_info(info)["converged"] == 1
    b.close()


# captured: the persistent launch alone; step launches then the persistent
# launch for the rest (3 step launches); step launches covering every step, the
# persistent launch returning at once (64 step launches); mode 1 explicitly
CAPTURE_TUNINGS = [dict(), dict(small_m=0, step_min_m=0, step_launches=3),
                   dict(small_m=0, step_min_m=0, step_launches=64),
                   dict(small_m=0, mode=1, step_launches=5)]


@pytest.mark.parametrize("ti", range(len(CAPTURE_TUNINGS)))
def test_batch_graph_capture_replay(dawn, ti):
    """Captured once, replayed with new sources written into the same buffer;
    every replay (with eager work in between) matches a fresh eager run."""
    prev = dawn.set_tuning(**CAPTURE_TUNINGS[ti]) if CAPTURE_TUNINGS[ti] else None
    try:
        _capture_replay(dawn, ti)
    finally:
        if prev is not None:
            dawn.set_tuning(**prev)


def _capture_replay(dawn, ti):
    import torch
    gs = _batch_graphs(count=6, seed=9)
    csrs = [dawn.Csr.from_graph(g) for g, _ in gs]
    b = dawn.Batch(csrs)
    srcs = torch.tensor([s for _, s in gs], dtype=torch.int32, device="cuda")
    out = torch.empty(b.total_n, dtype=torch.float32, device="cuda")
    info = dawn.info_tensor()
    announce("batch capture", CAPTURE_TUNINGS[ti])
    b.capture(srcs, out, info=info)
    rng = np.random.default_rng(1)
    for rep in range(4):
        new = [int(graphgen.pick_sources(g, 1, 100 + rep * 10 + i)[0]) for i, (g, _) in enumerate(gs)]
        srcs.copy_(torch.tensor(new, dtype=torch.int32))
        b.replay()
        torch.cuda.synchronize()
        eager = b.run(srcs.clone())
        junk = torch.randn(1000, device="cuda").sum()   # unrelated eager work between replays
        torch.cuda.synchronize()
        assert np.array_equal(to_np(out).view(np.uint32), to_np(eager).view(np.uint32))
        for (g, _), s, d in zip(gs, new, b.split(out)):
            assert_sssp_matches(g, s, to_np(d), tag=f"replay {rep}", check_invariants=False)
        del junk, rng
        rng = None
    b.close()


def test_batch_rejects_mixed_weight_types(dawn):
    g1 = graphgen.er(100, 400, 1, weights="u32")
    g2 = graphgen.er(100, 400, 2, weights="f32lognormal")
    with pytest.raises(dawn.DawnError):
        dawn.Batch([dawn.Csr.from_graph(g1), dawn.Csr.from_graph(g2)])


def _drain(dawn, tile, steps=4, limit=100000):
    import torch
    for _ in range(limit):
        done = tile.run(steps)
        torch.cuda.synchronize()
        if tile_all_done(dawn, tile, done):
            return
    raise AssertionError("tile did not finish")


def tile_all_done(dawn, tile, done):
    live = getattr(tile, "_live", set())
    cols = set(dawn.done_columns(done.cpu().numpy(), tile.k))
    return live <= cols


@pytest.mark.parametrize("wk", ["u32", "f32lognormal"])
def test_tile_session_mix_equals_alone(dawn, wk):
    """Queries admitted at different times into a shared tile give exactly
    the distances of the same query run alone."""
    import torch
    g = graphgen.rmat(13, 16, 12, weights=wk)
    csr = dawn.Csr.from_graph(g)
    srcs = graphgen.pick_sources(g, 12, 5)
    tile = dawn.Tile(csr, 8)
    tile._live = set()
    results = {}
    pending = list(enumerate(srcs))
    free = list(range(8))
    inflight = {}
    announce("tile session", wk)
    step = 0
    while pending or inflight:
        while pending and free and (step % 3 == 0 or not inflight):
            qi, s = pending.pop(0)
            col = free.pop(0)
            tile.admit(col, int(s))
            tile._live.add(col)
            inflight[col] = (qi, int(s))
        done = tile.run(2)
        torch.cuda.synchronize()
        for col in dawn.done_columns(done.cpu().numpy(), tile.k):
            if col in inflight:
                qi, s = inflight.pop(col)
                results[qi] = to_np(tile.read(col))
                tile._live.discard(col)
                free.append(col)
        step += 1
        assert step < 100000
    torch.cuda.synchronize()
    for qi, s in enumerate(srcs):
        alone = to_np(dawn.sssp(csr, int(s)))
        torch.cuda.synchronize()
        assert np.array_equal(results[qi].view(np.uint32), alone.view(np.uint32)), qi
        assert_sssp_matches(g, int(s), results[qi], tag=f"tile q{qi}", check_invariants=False)
    tile.close()


def test_tile_evict_and_reuse(dawn):
    import torch
    g = graphgen.grid(40, 40, 0.0, 1, weights="f32unit")
    csr = dawn.Csr.from_graph(g)
    tile = dawn.Tile(csr, 64)
    tile._live = {0, 1}
    tile.admit(0, 0)
    tile.admit(1, 1599)
    tile.run(5)
    tile.evict(1)           # cancel a running query
    tile._live = {0}
    _drain(dawn, tile)
    tile.admit(1, 820)      # reuse the freed column
    tile._live = {0, 1}
    _drain(dawn, tile)
    torch.cuda.synchronize()
    for col, s in ((0, 0), (1, 820)):
        assert_sssp_matches(g, s, to_np(tile.read(col)), tag=f"evict col {col}")
    steps = tile.steps().cpu().numpy()
    assert steps[0] > 40 and steps[1] > 20
    tile.close()


@pytest.mark.slow
def test_full_size_tile_rmat20_sampled(dawn):
    """R-MAT scale 20, k = 256, launched as the benchmark launches it: sampled
    columns against Dijkstra element by element, invariants on more."""
    import torch
    g, srcs = workloads.rmat20_tile()
    csr = dawn.Csr.from_graph(g)
    tg = dawn.tgraph(csr)
    for use_tg in (True, False):  # the benchmark's configuration, then push steps only
        announce("rmat20 tile k=256 full, reverse graph", use_tg)
        info = dawn.info_tensor()
        D = dawn.msssp(csr, srcs, info=info, tgraph=tg if use_tg else None)
        torch.cuda.synchronize()
        inf = dawn.read_info(info)
        assert inf["converged"] == 1
        for j in (0, 255):
            assert_sssp_matches(g, int(srcs[j]), to_np(D[j]), tag=f"rmat20 col {j}")
        for j in (17, 128):
            rc, v = oracle.check(g, int(srcs[j]), to_np(D[j]))
            assert rc == 0, f"col {j}: invariant V{rc} at {v}"


# ---------------------------------------------------------------------------
# pull steps (reverse graph): same relaxations, so results are identical
# ---------------------------------------------------------------------------
PULL_TUNINGS = [
    dict(tile_pull=0, tile_pull_src=0),               # every step a pull step
    dict(tile_pull=1001),                             # never
    dict(),                                           # by frontier size and density
    dict(tile_pull=0, tile_pull_src=0, tile_k=512),   # two 4-segment quads per target
    dict(tile_pull=50, tile_pull_src=0, tile_t_wave=32, tile_t_chunk=64, tile_sparse=0,
         tile_t_group=0),
    dict(tile_pull=0, tile_pull_src=0, tile_k=64),    # one segment: four in-edges at a time
    dict(tile_pull=0, tile_pull_src=0, tile_k=128),   # two segments: two in-edges at a time
    dict(tile_pull=0, tile_pull_src=0, tile_k=192),   # three segments: one group idle
    dict(tile_pull=0, tile_pull_src=64),              # only steps with many active sources
]


def _msssp_tg(dawn, csr, sources, tg, **tune):
    import torch
    prev = dawn.set_tuning(**tune) if tune else None
    try:
        info = dawn.info_tensor()
        out = dawn.msssp(csr, sources, info=info, tgraph=tg)
        torch.cuda.synchronize()
        return to_np(out), dawn.read_info(info)
    finally:
        if prev is not None:
            dawn.set_tuning(**prev)


@pytest.mark.parametrize("ti", range(len(PULL_TUNINGS)))
@pytest.mark.parametrize("wk", ["u32", "f32lognormal"])
def test_msssp_pull_steps_match_push_and_oracle(dawn, wk, ti):
    g = graphgen.rmat(13, 16, 21, weights=wk)   # hubs: targets with several in-edge chunks
    csr = dawn.Csr.from_graph(g)
    tg = dawn.tgraph(csr)
    srcs = graphgen.pick_sources(g, 150, 4 + ti)
    srcs = np.concatenate([srcs, srcs[:2]])      # duplicate sources
    announce("msssp pull", wk, PULL_TUNINGS[ti])
    D, info = _msssp_tg(dawn, csr, srcs, tg, **PULL_TUNINGS[ti])
    P, pinfo = _msssp(dawn, g, srcs)             # push steps only
    assert np.array_equal(D.view(np.uint32), P.view(np.uint32))
    for j in (0, 75, 149, 151):
        assert_sssp_matches(g, int(srcs[j]), D[j], tag=f"pull col {j}")
    assert info["converged"] == 1
    # both directions relax the same (edge, source) pairs; only the order of
    # updates within a step (and so the step count) may differ
    assert info["union_edges"] > 0 and info["edges_scanned"] > 0


@pytest.mark.parametrize("wk", ["u32", "f32lognormal"])
def test_msssp_pull_quads_of_four_and_one_segment(dawn, wk):
    """k = 300 sources in one 320-column tile: a pull task covers four
    segments (one in-edge at a time) or the fifth alone (four at a time)."""
    g = graphgen.rmat(11, 16, 23, weights=wk)
    csr = dawn.Csr.from_graph(g)
    tg = dawn.tgraph(csr)
    srcs = graphgen.pick_sources(g, 300, 9)
    announce("msssp pull k=300", wk)
    D, info = _msssp_tg(dawn, csr, srcs, tg, tile_pull=0, tile_pull_src=0, tile_k=320)
    P, _ = _msssp(dawn, g, srcs, tile_k=320)
    assert np.array_equal(D.view(np.uint32), P.view(np.uint32))
    for j in (0, 255, 256, 299):
        assert_sssp_matches(g, int(srcs[j]), D[j], tag=f"pull col {j}")
    assert info["converged"] == 1


def test_msssp_pull_hub_target_with_many_chunks(dawn):
    """A star whose centre has 100000 in-edges (about a hundred in-edge chunks,
    combined with atomics) and out-edges to every leaf."""
    n = 100001
    leaves = np.arange(1, n)
    src = np.concatenate([leaves, np.zeros(n - 1, np.int64), leaves[:-1]])
    dst = np.concatenate([np.zeros(n - 1, np.int64), leaves, leaves[1:]])
    rng = np.random.default_rng(11)
    w = rng.integers(1, 1000, size=src.size).astype(np.uint32)
    g = graphgen.from_edges(n, src, dst, w, "u32")
    csr = dawn.Csr.from_graph(g)
    tg = dawn.tgraph(csr)
    srcs = np.array([0, 5, 77777, 100000, 3], dtype=np.int32)
    announce("msssp pull star")
    D, info = _msssp_tg(dawn, csr, srcs, tg, tile_pull=0, tile_pull_src=0)
    for j, s in enumerate(srcs):
        assert_sssp_matches(g, int(s), D[j], tag=f"star pull source {s}")


def test_msssp_pull_grid_f32_many_steps(dawn):
    g = graphgen.grid(64, 48, 0.01, 3, weights="f32unit")
    csr = dawn.Csr.from_graph(g)
    tg = dawn.tgraph(csr)
    srcs = graphgen.pick_sources(g, 70, 1)
    announce("msssp pull grid f32")
    D, info = _msssp_tg(dawn, csr, srcs, tg, tile_pull=0, tile_pull_src=0)
    for j in (0, 33, 69):
        assert_sssp_matches(g, int(srcs[j]), D[j], tag=f"pull grid col {j}")
