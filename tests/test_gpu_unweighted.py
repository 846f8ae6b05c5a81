"""GPU parity of the hop-count tiles (every edge weight 1, ``dawn_umsssp_ws``)
against BFS levels from the oracle, against the weighted tile run with unit
weights, and between push-only and pull runs."""
import numpy as np
import pytest

import graphgen
import oracle
from gpu_helpers import INF32, announce, to_np

pytestmark = pytest.mark.gpu


def _levels(g, s):
    lvl = oracle.bfs(g, int(s))
    return np.where(lvl >= 0, lvl, -1).astype(np.int64).astype(np.uint32)  # -1 -> INF


def _umsssp(dawn, csr, sources, tg=None, **tune):
    import torch
    prev = dawn.set_tuning(**tune) if tune else None
    try:
        info = dawn.info_tensor()
        out = dawn.umsssp(csr, sources, info=info, tgraph=tg, check=False)
        torch.cuda.synchronize()
        return to_np(out), dawn.read_info(info)
    finally:
        if prev is not None:
            dawn.set_tuning(**prev)


def _assert_levels(g, srcs, D, cols, tag):
    for j in cols:
        ref = _levels(g, srcs[j])
        got = D[j].view(np.uint32)
        bad = np.nonzero(got != ref)[0]
        assert bad.size == 0, (f"{tag} col {j} source {srcs[j]}: {bad.size} mismatches, "
                               f"first v={bad[0]} gpu={got[bad[0]]} ref={ref[bad[0]]}")


PULL = [dict(tile_pull=1001), dict(tile_pull=0, tile_pull_src=0), dict(), dict(tile_pull=0, tile_pull_src=0, tile_k=64),
        dict(tile_pull=0, tile_pull_src=0, tile_k=128), dict(tile_pull=0, tile_pull_src=0, tile_k=192),
        dict(tile_pull=50, tile_pull_src=0, tile_t_wave=32, tile_t_chunk=64, tile_t_group=0)]


@pytest.mark.parametrize("ti", range(len(PULL)))
def test_umsssp_rmat_matches_bfs_and_weighted_unit(dawn, ti):
    # random weights that the hop-count path must ignore
    g = graphgen.rmat(13, 16, 31, weights="u32")
    csr = dawn.Csr.from_graph(g)
    tg = dawn.tgraph(csr)
    srcs = graphgen.pick_sources(g, 150, 40 + ti)
    srcs = np.concatenate([srcs, srcs[:2]])  # duplicate sources
    announce("umsssp rmat13", PULL[ti])
    D, info = _umsssp(dawn, csr, srcs, tg, **PULL[ti])
    assert info["converged"] == 1
    _assert_levels(g, srcs, D, range(len(srcs)), "umsssp")
    # the weighted tile with every weight 1 gives the same matrix
    g1 = graphgen.from_edges(g.n, *_edges(g), np.ones(g.m, np.uint32), "u32")
    P = to_np(dawn.msssp(dawn.Csr.from_graph(g1), srcs))
    assert np.array_equal(D.view(np.uint32), P.view(np.uint32))


def _edges(g):
    rp = np.asarray(g.rowptr, dtype=np.int64)
    src = np.repeat(np.arange(g.n), np.diff(rp))
    return src, np.asarray(g.colidx, dtype=np.int64)


def test_umsssp_counters_are_the_bfs_ones(dawn):
    """Unit weights make every step exact (mu = 1): per source, the edges
    scanned are m_reach(s), the improvements are the reached vertices minus
    the source, and the step count is its eccentricity + 1."""
    g = graphgen.rmat(12, 8, 4, weights="u32")
    csr = dawn.Csr.from_graph(g)
    tg = dawn.tgraph(csr)
    srcs = graphgen.pick_sources(g, 40, 2)
    for tune in (dict(tile_pull=1001), dict(tile_pull=0, tile_pull_src=0), dict()):
        announce("umsssp counters", tune)
        D, info = _umsssp(dawn, csr, srcs, tg, **tune)
        _assert_levels(g, srcs, D, range(len(srcs)), f"counters {tune}")
        lv = [oracle.bfs(g, int(s)) for s in srcs]
        assert info["edges_scanned"] == sum(oracle.m_reach(g, int(s)) for s in srcs)
        assert info["improvements"] == sum(int((x >= 0).sum()) - 1 for x in lv)
        assert info["steps"] == max(int(x.max()) + 1 for x in lv)
        assert info["frontier_entries"] == sum(
            int(((x >= 0) & (g.outdeg() > 0)).sum()) for x in lv)


def test_umsssp_five_segments(dawn):
    g = graphgen.rmat(11, 16, 23, weights="u32")
    csr = dawn.Csr.from_graph(g)
    tg = dawn.tgraph(csr)
    srcs = graphgen.pick_sources(g, 300, 9)
    for tune in (dict(tile_pull=0, tile_pull_src=0, tile_k=320), dict(tile_pull=1001, tile_k=320)):
        announce("umsssp k=300", tune)
        D, info = _umsssp(dawn, csr, srcs, tg, **tune)
        _assert_levels(g, srcs, D, (0, 63, 64, 255, 256, 299), f"k300 {tune}")


def test_umsssp_hub_target_with_many_chunks(dawn):
    """A star whose centre has 100000 in-edges (split pull chunks, combined
    with atomics) and out-edges to every leaf, plus a path among the leaves."""
    n = 100001
    leaves = np.arange(1, n)
    src = np.concatenate([leaves, np.zeros(n - 1, np.int64), leaves[:-1]])
    dst = np.concatenate([np.zeros(n - 1, np.int64), leaves, leaves[1:]])
    g = graphgen.from_edges(n, src, dst, np.ones(src.size, np.uint32), "u32")
    csr = dawn.Csr.from_graph(g)
    tg = dawn.tgraph(csr)
    srcs = np.array([0, 5, 77777, 100000, 3], dtype=np.int32)
    announce("umsssp star")
    for tune in (dict(tile_pull=0, tile_pull_src=0), dict()):
        D, info = _umsssp(dawn, csr, srcs, tg, **tune)
        _assert_levels(g, srcs, D, range(len(srcs)), f"star {tune}")


def test_umsssp_grid_many_steps(dawn):
    g = graphgen.grid(64, 48, 0.01, 3, weights="f32unit")
    csr = dawn.Csr.from_graph(g)
    tg = dawn.tgraph(csr)
    srcs = graphgen.pick_sources(g, 70, 1)
    announce("umsssp grid")
    D, info = _umsssp(dawn, csr, srcs, tg, tile_pull=100, tile_pull_src=0)
    _assert_levels(g, srcs, D, (0, 33, 69), "grid")
    assert info["converged"] == 1


def test_umsssp_chain_and_tiny_graphs(dawn):
    L = 300
    src = np.arange(L - 1)
    g = graphgen.from_edges(L, src, src + 1, np.full(L - 1, 7, np.uint32), "u32")
    csr = dawn.Csr.from_graph(g)
    announce("umsssp chain")
    D, info = _umsssp(dawn, csr, np.array([0, 150, L - 1], np.int32), dawn.tgraph(csr))
    assert np.array_equal(D[0].view(np.uint32), np.arange(L, dtype=np.uint32))
    assert np.all(D[1][:150].view(np.uint32) == INF32)
    assert np.array_equal(D[1][150:].view(np.uint32), np.arange(L - 150, dtype=np.uint32))
    assert D[2].view(np.uint32)[L - 1] == 0 and np.all(D[2][:L - 1].view(np.uint32) == INF32)
    assert info["steps"] == L  # L - 1 hops, plus the step that finds nothing
    # n = 1, m = 0
    g1 = graphgen.from_edges(1, np.zeros(0, np.int64), np.zeros(0, np.int64),
                             np.zeros(0, np.uint32), "u32")
    D1, info1 = _umsssp(dawn, dawn.Csr.from_graph(g1), np.array([0], np.int32))
    assert D1.view(np.uint32).tolist() == [[0]] and info1["converged"] == 1


def test_umsssp_source_out_of_range_is_reported(dawn):
    g = graphgen.rmat(8, 8, 5, weights="u32")
    csr = dawn.Csr.from_graph(g)
    for bad in (g.n, -1):
        announce("umsssp bad source", bad)
        D, info = _umsssp(dawn, csr, np.array([0, bad, 3], np.int32))
        assert info["converged"] == -1


def test_umsssp_eight_segments(dawn):
    """k = 500 in one 512-column tile: mask rows of 8 words (16-byte loads)."""
    g = graphgen.rmat(11, 16, 29, weights="u32")
    csr = dawn.Csr.from_graph(g)
    tg = dawn.tgraph(csr)
    srcs = graphgen.pick_sources(g, 500, 12)
    for tune in (dict(tile_pull=0, tile_pull_src=0, tile_k=512), dict(tile_pull=1001, tile_k=512), dict(tile_k=512)):
        announce("umsssp k=500", tune)
        D, info = _umsssp(dawn, csr, srcs, tg, **tune)
        _assert_levels(g, srcs, D, (0, 127, 128, 383, 448, 499), f"k500 {tune}")
        assert info["converged"] == 1


@pytest.mark.slow
def test_umsssp_full_size_rmat20_sampled(dawn):
    """The benchmark-suite configuration (R-MAT scale 20, 256 sources, reverse
    graph resident): sampled columns against BFS element by element."""
    from graphgen import workloads
    g, srcs = workloads.rmat20_tile()
    csr = dawn.Csr.from_graph(g)
    announce("umsssp rmat20 k=256 full")
    D, info = _umsssp(dawn, csr, srcs, dawn.tgraph(csr))
    assert info["converged"] == 1
    _assert_levels(g, srcs, D, (0, 77, 255), "rmat20")


# --- the unit weight type (DAWN_W_UNIT): weights never read ------------------

UNIT_SSSP_TUNINGS = [dict(), dict(small_m=0, mode=2), dict(small_m=0, mode=1, step_launches=3),
                     dict(small_m=0, step_min_m=0, step_launches=2), dict(small_m=0, ss_skip=0),
                     dict(small_m=0, mode=1, step_launches=4096)]


@pytest.mark.parametrize("ti", range(len(UNIT_SSSP_TUNINGS)))
def test_unit_weight_type_sssp_is_bfs(dawn, ti):
    import torch
    for g in (graphgen.rmat(11, 8, 61, weights="u32"), graphgen.rmat(14, 8, 62, weights="f32unit"),
              graphgen.grid(40, 30, 0.02, 63, weights="f32unit")):
        csr = dawn.Csr.from_graph(g, wtype="unit")
        prev = dawn.set_tuning(**UNIT_SSSP_TUNINGS[ti]) if UNIT_SSSP_TUNINGS[ti] else None
        try:
            for s in graphgen.pick_sources(g, 2, 70 + ti):
                announce("sssp unit", g.name, UNIT_SSSP_TUNINGS[ti], int(s))
                info = dawn.info_tensor()
                ws = dawn.workspace(dawn.sssp_workspace_bytes(g.n, g.m))
                d = dawn.sssp(csr, int(s), ws=ws, info=info)
                torch.cuda.synchronize()
                assert np.array_equal(to_np(d).view(np.uint32), _levels(g, s))
                lv = oracle.bfs(g, int(s))
                i = dawn.read_info(info)
                assert i["steps"] == int(lv.max()) + 1 and i["improvements"] == int((lv >= 0).sum()) - 1
        finally:
            if prev is not None:
                dawn.set_tuning(**prev)


def test_unit_weight_type_batched_calls_are_hop_counts(dawn):
    import torch
    g = graphgen.rmat(10, 8, 64, weights="u32")
    csr = dawn.Csr.from_graph(g, wtype="unit")
    srcs = graphgen.pick_sources(g, 70, 3)
    announce("msssp / apsp unit")
    D = to_np(dawn.msssp(csr, srcs))
    Dt = to_np(dawn.msssp(csr, srcs, tgraph=dawn.tgraph(csr)))  # reverse graph without weights
    torch.cuda.synchronize()
    for j in (0, 33, 69):
        assert np.array_equal(D[j].view(np.uint32), _levels(g, srcs[j]))
    assert np.array_equal(D.view(np.uint32), Dt.view(np.uint32))
    A = to_np(dawn.apsp(csr))
    for s in (0, 511, g.n - 1):
        assert np.array_equal(A[s].view(np.uint32), _levels(g, s))
