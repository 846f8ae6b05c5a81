"""GPU parity of single-source GOVM (dawn_sssp / dawn_sssp_ws) against the oracle."""
import numpy as np
import pytest

import graphgen
import oracle
from graphgen import workloads
from gpu_helpers import INF32, announce, assert_sssp_matches, to_np

pytestmark = pytest.mark.gpu


def _run(dawn, g, s, **tune):
    import torch
    prev = dawn.set_tuning(**tune) if tune else None
    try:
        csr = dawn.Csr.from_graph(g)
        info = dawn.info_tensor()
        out = dawn.sssp(csr, int(s), info=info)
        torch.cuda.synchronize()
        return to_np(out), dawn.read_info(info)
    finally:
        if prev is not None:
            dawn.set_tuning(**prev)


def test_er_small_bitexact(dawn):
    g, src = workloads.er_small()
    for s in [0, 1, 17, 999]:
        announce("er_small u32 source", s)
        d, info = _run(dawn, g, s)
        assert_sssp_matches(g, s, d, tag="er_small")
        assert info["converged"] == 1


@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("wk", ["u32", "f32lognormal", "f32range02", "f32unit"])
def test_rmat_weight_kinds(dawn, wk, mode):
    g = graphgen.rmat(14, 16, 5, weights=wk)
    for s in graphgen.pick_sources(g, 3, 9):
        announce("rmat14", wk, "mode", mode, "source", s)
        d, info = _run(dawn, g, s, mode=mode)
        assert_sssp_matches(g, s, d, tag=f"rmat14-{wk}-m{mode}")
        assert info["converged"] == 1


# Thresholds small enough that every tier (lane, wave, chunked workgroup) runs,
# and geometries that change the work split; results must not change.
TUNINGS = [
    dict(),
    dict(t_lane=1, t_wave=64, t_chunk=256),
    dict(t_lane=64, t_wave=65536, t_chunk=1 << 20),
    dict(t_lane=4, t_wave=100, t_chunk=300, wg_threads=1024),
    dict(t_lane=8, t_wave=64, t_chunk=256, wg_threads=512, grid=7),
    dict(mode=1, grid=3, step_launches=1),
    dict(mode=1, grid=3, step_launches=4096),  # every step a step launch
    dict(mode=1, t_lane=2, t_wave=64, t_chunk=256, step_launches=5),
    dict(small_m=1 << 30),                    # one workgroup for the whole graph
    dict(small_m=1 << 30, wg_threads=256),
    dict(step_min_m=0, step_launches=2),      # step launches, then a persistent launch
    dict(mode=1, step_launches=2, ss_tail_grid=1),  # ... of one workgroup
    dict(mode=2, ss_tail_grid=3),             # a persistent launch of three workgroups
    dict(step_min_m=0, step_launches=1, wg_threads=1024, t_lane=2, t_wave=64, t_chunk=256),
    dict(step_min_m=0),
    dict(ss_skip=0, small_m=0),                # every frontier row expanded in its step
    dict(ss_skip=0, small_m=0, mode=1, t_lane=2, t_wave=64, t_chunk=256, step_launches=3),
]


@pytest.mark.parametrize("ti", range(len(TUNINGS)))
def test_tiers_and_geometry_do_not_change_results(dawn, ti):
    g = graphgen.rmat(15, 16, 7, weights="u32")
    gf = graphgen.rmat(13, 24, 8, weights="f32lognormal")
    for gg in (g, gf):
        for s in graphgen.pick_sources(gg, 2, ti + 1):
            announce("tuning", TUNINGS[ti], gg.name, "source", s)
            d, info = _run(dawn, gg, s, **TUNINGS[ti])
            assert_sssp_matches(gg, s, d, tag=f"tuning{ti}")


# Rows of at most t_lane edges are taken from a scan of the step's frontier
# bitmap, not from a queue.  Vertex counts that leave a partial last word and
# block, grids of one to a few workgroups (many bitmap blocks per wavefront),
# t_lane at both ends of its range, and the last vertex as a source.
SCAN_GRAPHS = [(31, 3), (33, 3), (2047, 4), (2049, 4), (65537, 6), (200003, 8)]
SCAN_TUNINGS = [
    dict(small_m=0, mode=2, ss_tail_grid=1),
    dict(small_m=0, mode=2, ss_tail_grid=3),
    dict(small_m=0, mode=1, grid=5, step_launches=4096),
    dict(small_m=0, t_lane=1),
    dict(small_m=0, t_lane=4096, t_wave=4096),
]


@pytest.mark.parametrize("ti", range(len(SCAN_TUNINGS)))
def test_short_rows_from_the_frontier_bitmap(dawn, ti):
    for n, deg in SCAN_GRAPHS:
        g = graphgen.er(n, n * deg, 300 + n, weights="u32")
        for s in list(graphgen.pick_sources(g, 2, ti + 1)) + [n - 1]:
            announce("bitmap scan", SCAN_TUNINGS[ti], "n", n, "source", s)
            d, info = _run(dawn, g, s, **SCAN_TUNINGS[ti])
            assert info["converged"] == 1
            assert_sssp_matches(g, int(s), d, tag=f"scan{ti}-n{n}")
        gu = graphgen.er(n, n * deg, 300 + n, weights="u32one")
        announce("bitmap scan, unit weights", SCAN_TUNINGS[ti], "n", n)
        d, info = _run(dawn, gu, n - 1, **SCAN_TUNINGS[ti])
        lvl = oracle.bfs(gu, n - 1)
        assert np.array_equal(to_np_u32(d), np.where(lvl < 0, INF32, lvl).astype(np.uint32))
        _, c = oracle.govm(gu, n - 1)
        for key in ("steps", "edges_scanned", "improvements", "frontier_entries"):
            assert info[key] == c[key], key


def test_grid_f32_small(dawn):
    g = graphgen.grid(96, 80, 0.01, 31, weights="f32unit")
    for s in graphgen.pick_sources(g, 3, 2):
        announce("grid96x80 f32 source", s)
        d, info = _run(dawn, g, s)
        assert_sssp_matches(g, s, d, tag="grid")
        assert info["steps"] > 96   # a high-step-count case


def test_grid_f32_tiny_and_small_paths(dawn):
    """n <= 6144 runs in one workgroup with its state in LDS (with m <= 16384
    the whole graph, edge-parallel steps; 70x70 has more edges and takes the
    queue kernel), larger small graphs in one workgroup over global memory;
    every many-step fp32 case matches the oracle."""
    for rows, cols in ((40, 40), (60, 60), (70, 70), (90, 90)):
        g = graphgen.grid(rows, cols, 0.02, 5, weights="f32unit")
        for s in graphgen.pick_sources(g, 2, 3):
            announce("grid", rows, cols, "f32 source", s)
            d, info = _run(dawn, g, s)
            assert_sssp_matches(g, s, d, tag=f"grid{rows}")
            assert info["steps"] > rows


@pytest.mark.parametrize("small_m", [None, 0, 1 << 30])
def test_edge_cases(dawn, small_m):
    tune = {} if small_m is None else dict(small_m=small_m)
    cases = []
    cases.append(("n1", graphgen.from_edges(1, [], [], np.zeros(0, np.uint32), "u32"), 0))
    cases.append(("m0", graphgen.from_edges(7, [], [], np.zeros(0, np.uint32), "u32"), 3))
    cases.append(("isolated", graphgen.from_edges(4, [0, 1], [1, 2], np.array([3, 4], np.uint32),
                                                  "u32"), 3))
    cases.append(("selfloop-parallel",
                  graphgen.from_edges(3, [0, 0, 0, 1, 1], [0, 1, 1, 1, 2],
                                      np.array([1, 9, 4, 0, 2], np.uint32), "u32"), 0))
    cases.append(("zero-weights", graphgen.from_edges(4, [0, 1, 2, 0], [1, 2, 3, 3],
                                                      np.array([0, 0, 0, 1], np.uint32), "u32"), 0))
    cases.append(("zero-weights-f32",
                  graphgen.from_edges(4, [0, 1, 2, 0], [1, 2, 3, 3],
                                      np.array([0, 0, 0, 1], np.float32), "f32"), 0))
    big = 0xFFFFFFFF - 5
    cases.append(("saturate", graphgen.from_edges(3, [0, 1], [1, 2], np.array([big, 10], np.uint32),
                                                  "u32"), 0))
    # star: one hub with a long row (chunked workgroup tier), leaves point back
    n = 200001
    src = np.concatenate([np.zeros(n - 1, np.int64), np.arange(1, n)])
    dst = np.concatenate([np.arange(1, n), np.zeros(n - 1, np.int64)])
    rng = np.random.default_rng(3)
    w = rng.integers(1, 1000, size=src.size).astype(np.uint32)
    cases.append(("star", graphgen.from_edges(n, src, dst, w, "u32"), 0))
    cases.append(("star-leaf", graphgen.from_edges(n, src, dst, w, "u32"), 12345))
    # ragged tail: sizes not multiples of 64 / 32
    cases.append(("ragged", graphgen.er(1001, 7003, 4, weights="u32", wlo=0, whi=3), 1000))
    for name, g, s in cases:
        announce("edge case", name, "n", g.n, "m", g.m, "source", s, tune)
        d, info = _run(dawn, g, s, **tune)
        assert_sssp_matches(g, s, d, tag=name)
        assert info["converged"] == 1


def test_chain_step_count(dawn):
    L = 3000
    rng = np.random.default_rng(5)
    w = rng.integers(1, 100, size=L).astype(np.uint32)
    g = graphgen.from_edges(L + 1, np.arange(L), np.arange(1, L + 1), w, "u32")
    announce("chain", L)
    for mode in (1, 2):
        d, info = _run(dawn, g, 0, mode=mode)
        assert to_np_u32(d).tolist() == np.concatenate([[0], np.cumsum(w)]).tolist()
        assert info["steps"] == L + 1            # Algorithm 2: L updating steps + 1
        assert info["edges_scanned"] == L and info["improvements"] == L


def to_np_u32(d):
    return np.asarray(d).view(np.uint32)


def _lds_cases():
    """Graphs at and around the whole-graph-in-LDS limits (n <= 6144, m <= 16384)."""
    rng = np.random.default_rng(11)
    cases = [("er-m16384", graphgen.er(6144, 16384, 12, weights="u32", wlo=1, whi=100), 5),
             ("er-m16385", graphgen.er(6144, 16385, 12, weights="u32", wlo=1, whi=100), 5),
             ("er-zero-weights", graphgen.er(2000, 12000, 13, weights="u32", wlo=0, whi=2), 7),
             ("grid60-f32", graphgen.grid(60, 60, 0.02, 14, weights="f32unit"), 100)]
    # a hub row of 5999 edges (one thread writes its edges' source ids) and a
    # ring of leaf edges back into the graph
    n = 6000
    src = np.concatenate([np.zeros(n - 1, np.int64), np.arange(1, n)])
    dst = np.concatenate([np.arange(1, n), (np.arange(1, n) * 7) % n])
    w = rng.integers(1, 1000, size=src.size).astype(np.uint32)
    cases.append(("hub", graphgen.from_edges(n, src, dst, w, "u32"), 0))
    cases.append(("hub-leaf", graphgen.from_edges(n, src, dst, w, "u32"), 4321))
    return cases


@pytest.mark.parametrize("wg", [0, 256, 512])
def test_lds_graph_limits_and_shapes(dawn, wg):
    """One-workgroup runs of graphs held whole in LDS: at the edge limit and one
    edge past it (the queue kernel), zero weights, fp32, a hub row; every
    workgroup size gives the oracle's distances."""
    for name, g, s in _lds_cases():
        announce("lds case", name, "n", g.n, "m", g.m, "source", s, "wg", wg)
        d, info = _run(dawn, g, s, small_m=1 << 30, wg_threads=wg)
        assert_sssp_matches(g, s, d, tag=name)
        assert info["converged"] == 1


def test_lds_graph_counters_are_algorithm2s(dawn):
    """Edge-parallel steps count what Algorithm 2 counts: at unit weights the
    counters of sequential Algorithm 2 exactly, and on a chain L + 1 steps
    with L edges scanned and L improvements."""
    g = graphgen.rmat(12, 3, 22, weights="u32one")
    assert g.n <= 6144 and g.m <= 16384
    for s in graphgen.pick_sources(g, 3, 5):
        announce("lds unit weights source", s)
        d, info = _run(dawn, g, s, small_m=1 << 30)
        lvl = oracle.bfs(g, s)
        assert np.array_equal(to_np_u32(d), np.where(lvl < 0, INF32, lvl).astype(np.uint32))
        _, c = oracle.govm(g, s)
        for key in ("steps", "edges_scanned", "improvements", "frontier_entries"):
            assert info[key] == c[key], key
    L = 3000
    rng = np.random.default_rng(6)
    w = rng.integers(1, 100, size=L).astype(np.uint32)
    g = graphgen.from_edges(L + 1, np.arange(L), np.arange(1, L + 1), w, "u32")
    announce("lds chain", L)
    d, info = _run(dawn, g, 0, small_m=1 << 30)
    assert to_np_u32(d).tolist() == np.concatenate([[0], np.cumsum(w)]).tolist()
    assert info["steps"] == L + 1
    assert info["edges_scanned"] == L and info["improvements"] == L
    assert info["frontier_entries"] == L


def test_unit_weights_are_bfs_with_mu_one(dawn):
    """Unit weights: each vertex is finalised in the step it is first reached,
    so the counters are exact (Section 1, contribution 3: mu = 1)."""
    g = graphgen.rmat(15, 8, 21, weights="u32one")
    for s in graphgen.pick_sources(g, 3, 4):
        announce("unit weights source", s)
        for mode in (1, 2):
            d, info = _run(dawn, g, s, mode=mode)
            lvl = oracle.bfs(g, s)
            exp = np.where(lvl < 0, INF32, lvl).astype(np.uint32)
            assert np.array_equal(to_np_u32(d), exp)
            reach = lvl >= 0
            assert info["steps"] == lvl.max() + 1
            assert info["edges_scanned"] == oracle.m_reach(g, s)
            assert info["improvements"] == int(reach.sum()) - 1
            assert info["frontier_entries"] == int((reach & (g.outdeg() > 0)).sum())
            _, c = oracle.govm(g, s)
            for key in ("steps", "edges_scanned", "improvements", "frontier_entries"):
                assert info[key] == c[key]


def test_ws_entry_point_and_workspace_reuse(dawn):
    import torch
    g = graphgen.rmat(13, 16, 2, weights="u32")
    csr = dawn.Csr.from_graph(g)
    ws = dawn.workspace(dawn.sssp_workspace_bytes(g.n, g.m))
    info = dawn.info_tensor()
    for s in graphgen.pick_sources(g, 4, 3):
        announce("ws reuse source", s)
        out = dawn.sssp(csr, int(s), ws=ws, info=info)
        torch.cuda.synchronize()
        assert_sssp_matches(g, s, to_np(out), tag="ws")
        assert dawn.read_info(info)["converged"] == 1


def test_host_validation_errors(dawn):
    import torch
    g = graphgen.er(100, 400, 1)
    csr = dawn.Csr.from_graph(g)
    with pytest.raises(dawn.DawnError) as e:
        dawn.sssp(csr, 100)
    assert e.value.status == 1
    with pytest.raises(dawn.DawnError) as e:
        dawn.sssp(csr, -1)
    assert e.value.status == 1
    small = dawn.workspace(64)
    with pytest.raises(dawn.DawnError) as e:
        dawn.sssp(csr, 0, ws=small[:128])
    assert e.value.status in (1, 3)
    with pytest.raises(dawn.DawnError):
        dawn.set_tuning(t_lane=0)
    torch.cuda.synchronize()


def test_device_validation_flags_bad_csr(dawn):
    """validate=1 checks the CSR on the device and reports converged = -1."""
    import torch
    g = graphgen.er(50, 200, 2, weights="f32lognormal")
    bad_w = g.w.copy()
    bad_w[7] = -1.0
    bad = g.with_weights(bad_w, "f32")
    prev = dawn.set_tuning(validate=1)
    try:
        for gg, exp in ((g, 1), (bad, -1)):
            csr = dawn.Csr.from_graph(gg)
            info = dawn.info_tensor()
            out = dawn.sssp(csr, 0, info=info, check=False)
            torch.cuda.synchronize()
            assert dawn.read_info(info)["converged"] == exp
            if exp == -1:
                assert np.all(np.isinf(to_np(out)))
    finally:
        dawn.set_tuning(**prev)


@pytest.mark.slow
def test_full_size_rmat22_sampled(dawn):
    """The scale-22 R-MAT at full size, launched as the benchmark launches it:
    one source compared element by element with Dijkstra, the invariants on
    two more."""
    import torch
    g, srcs = workloads.rmat22(nsrc=3)
    csr = dawn.Csr.from_graph(g)
    for i, s in enumerate(srcs):
        announce("rmat22 full source", s)
        out = dawn.sssp(csr, int(s))
        torch.cuda.synchronize()
        d = to_np(out)
        if i == 0:
            assert_sssp_matches(g, s, d, tag="rmat22")
        else:
            rc, v = oracle.check(g, int(s), d)
            assert rc == 0, f"invariant V{rc} at {v}"


@pytest.mark.slow
def test_full_size_grid_sampled(dawn):
    import torch
    g, srcs = workloads.grid2048(nsrc=1)
    csr = dawn.Csr.from_graph(g)
    s = int(srcs[0])
    announce("grid2048 full source", s)
    info = dawn.info_tensor()
    out = dawn.sssp(csr, s, info=info)
    torch.cuda.synchronize()
    assert_sssp_matches(g, s, to_np(out), tag="grid2048")
    assert dawn.read_info(info)["steps"] > 2000


# --- pull steps on the single-source path (dawn_sssp_tg_ws) -------------------

PULL_SS = [dict(small_m=0, mode=1, ss_pull=0, step_launches=4096),    # every step a pull step
           dict(small_m=0, mode=1, ss_pull=200, step_launches=3),    # by frontier size
           dict(small_m=0, step_min_m=0, ss_pull=0, step_launches=2),  # steps, then persistent
           dict(small_m=0, mode=2, ss_pull=0),                 # persistent: never pulls
           dict(small_m=0, mode=1, ss_pull=0, ss_skip=0, t_lane=2, t_wave=64, t_chunk=256,
                step_launches=4096)]


def _sssp_tg(dawn, csr, s, tg, **tune):
    import torch
    prev = dawn.set_tuning(**tune)
    try:
        info = dawn.info_tensor()
        d = dawn.sssp(csr, int(s), info=info, tgraph=tg)
        torch.cuda.synchronize()
        return to_np(d), dawn.read_info(info)
    finally:
        dawn.set_tuning(**prev)


@pytest.mark.parametrize("ti", range(len(PULL_SS)))
@pytest.mark.parametrize("wk", ["u32", "f32lognormal", "grid"])
def test_sssp_pull_steps_match_oracle(dawn, wk, ti):
    if wk == "grid":
        g = graphgen.grid(60, 50, 0.01, 81, weights="f32unit")
    else:
        g = graphgen.rmat(13, 16, 80, weights=wk)   # hubs: targets with several in-edge chunks
    csr = dawn.Csr.from_graph(g)
    tg = dawn.tgraph(csr)
    for s in graphgen.pick_sources(g, 3, 90 + ti):
        announce("sssp pull", wk, PULL_SS[ti], int(s))
        d, info = _sssp_tg(dawn, csr, s, tg, **PULL_SS[ti])
        assert info["converged"] == 1
        assert_sssp_matches(g, int(s), d, tag=f"pull {PULL_SS[ti]}")


def test_sssp_pull_signed_and_unit_weights(dawn):
    g0 = graphgen.rmat(12, 16, 82, weights="u32", wlo=1, whi=100)
    gi, p = graphgen.potential_shift(g0, 2000, 5)
    csr = dawn.Csr.from_graph(gi)
    tg = dawn.tgraph(csr)
    for s in graphgen.pick_sources(g0, 2, 6):
        announce("sssp pull i32", int(s))
        d, info = _sssp_tg(dawn, csr, s, tg, **PULL_SS[0])
        ref, ok = oracle.bellman_ford(gi, int(s))
        assert ok and info["converged"] == 1
        ref = np.where(ref == np.iinfo(np.int64).max, np.iinfo(np.int32).max, ref)
        assert np.array_equal(d.view(np.int32).astype(np.int64), ref)
    cu = dawn.Csr.from_graph(g0, wtype="unit")
    tgu = dawn.tgraph(cu)
    for s in graphgen.pick_sources(g0, 2, 7):
        announce("sssp pull unit", int(s))
        d, info = _sssp_tg(dawn, cu, s, tgu, **PULL_SS[0])
        lv = oracle.bfs(g0, int(s))
        ref = np.where(lv >= 0, lv, -1).astype(np.int64).astype(np.uint32)
        assert np.array_equal(d.view(np.uint32), ref)
        # every step exact at unit weights: the counters are the BFS ones
        assert info["edges_scanned"] == oracle.m_reach(g0, int(s))
        assert info["improvements"] == int((lv >= 0).sum()) - 1
        assert info["frontier_entries"] == int(((lv >= 0) & (g0.outdeg() > 0)).sum())
        assert info["steps"] == int(lv.max()) + 1
