"""Pins for the CPU oracle (no GPU).

The oracle's Dijkstra is pinned to things other than itself: brute-force path
enumeration, Floyd-Warshall, closed forms, a hand-worked fixture, the
unit-weight special case (the paper's mu = 1 claim, Section 1), and planted
mistakes the invariant checker must reject.
"""
import os

import numpy as np
import pytest

import graphgen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
INF = 0xFFFFFFFF


def load_golden(name):
    edges, out = [], {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            if key == "edge":
                edges.append(tuple(int(x) for x in vals))
            else:
                out[key] = vals
    return edges, out


def tiny_graph(rng, n, p, wmode):
    """Random directed graph on n vertices: each ordered pair (self-loops
    included) present with prob p, plus a few parallel edges."""
    src, dst = [], []
    for u in range(n):
        for v in range(n):
            if rng.random() < p:
                src.append(u); dst.append(v)
    for _ in range(rng.integers(0, 3)):
        if src:
            i = rng.integers(0, len(src))
            src.append(src[i]); dst.append(dst[i])
    m = len(src)
    if wmode == "u32":
        w = rng.integers(0, 20, size=m).astype(np.uint32)     # zero weights included
    elif wmode == "dyadic":
        w = (rng.integers(0, 64, size=m) / 16.0).astype(np.float32)  # exact sums
    else:  # general fp32, rounding in play
        w = rng.lognormal(0.0, 1.5, size=m).astype(np.float32)
    return graphgen.from_edges(n, src, dst, w, "u32" if wmode == "u32" else "f32")


# ---------------------------------------------------------------------------
# hand-worked fixture
# ---------------------------------------------------------------------------

def _golden_graph(weights_unit=False, as_f32=False):
    edges, meta = load_golden("handworked_small.txt")
    n = int(meta["n"][0])
    src = [e[0] for e in edges]
    dst = [e[1] for e in edges]
    w = [1 if weights_unit else e[2] for e in edges]
    w = np.array(w, dtype=np.float32 if as_f32 else np.uint32)
    return graphgen.from_edges(n, src, dst, w, "f32" if as_f32 else "u32"), meta


def test_golden_u32_distances_and_hops():
    g, meta = _golden_graph()
    d, h = oracle.sssp(g, int(meta["source"][0]), "u32")
    exp = [INF if x == "INF" else int(x) for x in meta["dist"]]
    assert d.tolist() == exp
    assert h.tolist() == [int(x) for x in meta["hops"]]


def test_golden_f32_modes_agree_exactly():
    g, meta = _golden_graph(as_f32=True)
    exp = [np.inf if x == "INF" else float(x) for x in meta["dist"]]
    d64, h64 = oracle.sssp(g, 0, "f64")
    d32, h32 = oracle.sssp(g, 0, "f32fold")
    assert d64.tolist() == exp
    assert d32.astype(np.float64).tolist() == exp
    assert h64.tolist() == h32.tolist() == [int(x) for x in meta["hops"]]


def test_golden_unit_weights_mu_one():
    g, meta = _golden_graph(weights_unit=True)
    lvl = oracle.bfs(g, 0)
    exp = [-1 if x == "INF" else int(x) for x in meta["unit_levels"]]
    assert lvl.tolist() == exp
    d, _ = oracle.sssp(g, 0, "u32")
    assert [(-1 if x == INF else int(x)) for x in d] == exp
    for order in (0, 1, 2):
        dg, c = oracle.govm(g, 0, order=order, seed=3)
        assert [(-1 if x == INF else int(x)) for x in dg] == exp
        assert c["steps"] == int(meta["unit_steps"][0])
        assert c["edges_scanned"] == int(meta["unit_edges_scanned"][0])
        assert c["improvements"] == int(meta["unit_improvements"][0])
        assert c["converged"] == 1


# ---------------------------------------------------------------------------
# brute force and Floyd-Warshall
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(40))
def test_dijkstra_matches_brute_force_u32(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 9))
    g = tiny_graph(rng, n, float(rng.uniform(0.1, 0.6)), "u32")
    s = int(rng.integers(0, n))
    d, h = oracle.sssp(g, s, "u32")
    bd, bh = oracle.brute(g, s, "u32")
    exp = np.where(bd == np.iinfo(np.uint64).max, INF, bd).astype(np.uint64)
    assert d.astype(np.uint64).tolist() == exp.tolist()
    assert h.tolist() == bh.tolist()


@pytest.mark.parametrize("seed", range(40))
def test_dijkstra_matches_brute_force_f32(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(1, 9))
    g = tiny_graph(rng, n, float(rng.uniform(0.1, 0.6)), "general")
    s = int(rng.integers(0, n))
    d64, h64 = oracle.sssp(g, s, "f64")
    b64, bh64 = oracle.brute(g, s, "f64")
    assert d64.tolist() == b64.tolist()
    assert h64.tolist() == bh64.tolist()
    d32, h32 = oracle.sssp(g, s, "f32fold")
    b32, bh32 = oracle.brute(g, s, "f32fold")
    assert d32.astype(np.float64).tolist() == b32.tolist()
    assert h32.tolist() == bh32.tolist()


@pytest.mark.parametrize("seed", range(6))
def test_floyd_warshall_rows_match_dijkstra(seed):
    rng = np.random.default_rng(2000 + seed)
    n = int(rng.integers(20, 64))
    g = tiny_graph(rng, n, 4.0 / n, "u32")
    D = oracle.fw(g)
    for s in range(n):
        d, _ = oracle.sssp(g, s, "u32")
        exp = np.where(D[s] == np.iinfo(np.uint64).max, INF, D[s]).astype(np.uint64)
        assert d.astype(np.uint64).tolist() == exp.tolist()
    gf = tiny_graph(rng, n, 4.0 / n, "dyadic")   # dyadic weights: every sum exact
    Df = oracle.fw(gf)
    for s in range(n):
        d64, _ = oracle.sssp(gf, s, "f64")
        d32, _ = oracle.sssp(gf, s, "f32fold")
        assert d64.tolist() == Df[s].tolist()
        assert d32.astype(np.float64).tolist() == Df[s].tolist()


def test_floyd_warshall_brute_tiny():
    rng = np.random.default_rng(77)
    for _ in range(10):
        n = int(rng.integers(2, 8))
        g = tiny_graph(rng, n, 0.4, "u32")
        D = oracle.fw(g)
        for s in range(n):
            bd, _ = oracle.brute(g, s, "u32")
            assert D[s].tolist() == bd.tolist()


# ---------------------------------------------------------------------------
# closed forms and special cases
# ---------------------------------------------------------------------------

def test_unit_grid_is_manhattan():
    g = graphgen.grid(13, 17, 0.0, 5, weights="f32unit")
    g = g.with_weights(np.ones(g.m, dtype=np.uint32), "u32")
    s = 3 * 17 + 5
    d, h = oracle.sssp(g, s, "u32")
    r, c = np.divmod(np.arange(g.n), 17)
    man = np.abs(r - 3) + np.abs(c - 5)
    assert d.tolist() == man.tolist()
    assert h.tolist() == man.tolist()


def test_chain_prefix_sums_and_steps():
    L = 50
    rng = np.random.default_rng(5)
    w = rng.integers(1, 100, size=L).astype(np.uint32)
    g = graphgen.from_edges(L + 1, np.arange(L), np.arange(1, L + 1), w, "u32")
    d, h = oracle.sssp(g, 0, "u32")
    assert d.tolist() == np.concatenate([[0], np.cumsum(w)]).tolist()
    assert h.tolist() == list(range(L + 1))
    _, c = oracle.govm(g, 0)
    assert c["steps"] == L + 1   # L updating steps + one with no update


def test_arborescence_unique_path_sums():
    rng = np.random.default_rng(9)
    n = 300
    parent = np.array([rng.integers(0, v) for v in range(1, n)])
    w = rng.integers(0, 1000, size=n - 1).astype(np.uint32)
    g = graphgen.from_edges(n, parent, np.arange(1, n), w, "u32")
    exp = np.zeros(n, dtype=np.int64)
    for v in range(1, n):
        exp[v] = exp[parent[v - 1]] + int(w[v - 1])
    d, _ = oracle.sssp(g, 0, "u32")
    assert d.astype(np.int64).tolist() == exp.tolist()


def test_degenerate_graphs():
    g = graphgen.from_edges(1, [], [], np.zeros(0, np.uint32), "u32")
    assert oracle.sssp(g, 0, "u32")[0].tolist() == [0]
    g = graphgen.from_edges(5, [], [], np.zeros(0, np.uint32), "u32")
    assert oracle.sssp(g, 2, "u32")[0].tolist() == [INF, INF, 0, INF, INF]
    # isolated source with edges elsewhere
    g = graphgen.from_edges(4, [0, 1], [1, 2], np.array([3, 4], np.uint32), "u32")
    assert oracle.sssp(g, 3, "u32")[0].tolist() == [INF, INF, INF, 0]
    # self-loops and parallel edges: the cheapest parallel edge wins
    g = graphgen.from_edges(3, [0, 0, 0, 1, 1], [0, 1, 1, 1, 2],
                            np.array([1, 9, 4, 0, 2], np.uint32), "u32")
    assert oracle.sssp(g, 0, "u32")[0].tolist() == [0, 4, 6]


def test_u32_saturation_reads_as_inf():
    big = 0xFFFFFFFF - 5
    g = graphgen.from_edges(3, [0, 1], [1, 2], np.array([big, 10], np.uint32), "u32")
    d, h = oracle.sssp(g, 0, "u32")
    assert d.tolist() == [0, big, INF]
    rc, _ = oracle.check(g, 0, d)
    assert rc == 0


def test_unit_weights_equal_bfs_levels_rmat():
    g = graphgen.rmat(12, 8, 3, weights="u32one")
    for s in graphgen.pick_sources(g, 4, 1):
        lvl = oracle.bfs(g, s)
        d, h = oracle.sssp(g, s, "u32")
        assert np.array_equal(np.where(lvl < 0, INF, lvl).astype(np.uint32), d)
        _, c = oracle.govm(g, s)
        reach = lvl >= 0
        assert c["steps"] == lvl.max() + 1
        assert c["edges_scanned"] == oracle.m_reach(g, s)
        assert c["improvements"] == int(reach.sum()) - 1
        assert c["frontier_entries"] == int((reach & (g.outdeg() > 0)).sum())


def test_f32_fold_equals_f64_on_dyadic_weights():
    # weights j/16 with j in [0,64]: every path sum on this graph stays below
    # 2^20 and is a multiple of 2^-4, so fp32 holds it exactly and the fold
    # and the fp64 sum must agree bit for bit
    g = graphgen.rmat(11, 8, 4, weights="u32", wlo=0, whi=64)
    g = g.with_weights((g.w.astype(np.float64) / 16.0).astype(np.float32), "f32")
    for s in graphgen.pick_sources(g, 3, 2):
        d64, h64 = oracle.sssp(g, s, "f64")
        d32, h32 = oracle.sssp(g, s, "f32fold")
        assert np.array_equal(d32.astype(np.float64), d64)
        assert np.array_equal(h32, h64)


# ---------------------------------------------------------------------------
# the Algorithm 2 restatement reaches the definition, in any order
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("wk", ["u32", "f32lognormal", "f32range02"])
def test_govm_restatement_equals_dijkstra(wk):
    g = graphgen.rmat(10, 8, 11, weights=wk)
    for s in graphgen.pick_sources(g, 3, 5):
        mode = "u32" if g.wtype == "u32" else "f32fold"
        ref, _ = oracle.sssp(g, s, mode)
        for order in (0, 1, 2):
            d, c = oracle.govm(g, s, order=order, seed=int(s))
            assert c["converged"] == 1
            assert np.array_equal(d.view(np.uint32), ref.view(np.uint32))


def test_govm_per_vertex_updates():
    """Path-update counts (Section 4.2): hand-worked on a triangle (the direct
    edge 0 -> 1 is found first and replaced a step later by 0 -> 2 -> 1), one
    update per reached vertex at unit weights (a shortest path found is never
    updated again), and the counts sum to the improvements."""
    g = graphgen.from_edges(3, [0, 0, 2], [1, 2, 1], np.array([5, 1, 1], np.uint32), "u32")
    d, c = oracle.govm(g, 0, per_vertex=True)
    assert d.tolist() == [0, 2, 1]
    assert c["updates"].tolist() == [0, 2, 1]
    assert c["improvements"] == 3 and c["steps"] == 3
    gu = graphgen.rmat(11, 8, 13, weights="u32one")
    for s in graphgen.pick_sources(gu, 3, 2):
        _, c = oracle.govm(gu, int(s), per_vertex=True)
        reach = oracle.bfs(gu, int(s)) >= 0
        exp = reach.astype(np.int32)
        exp[int(s)] = 0
        assert np.array_equal(c["updates"], exp)
    gw = graphgen.rmat(11, 8, 13, weights="u32")
    s = int(graphgen.pick_sources(gw, 1, 4)[0])
    for order in (0, 1, 2):
        _, c = oracle.govm(gw, s, order=order, seed=1, per_vertex=True)
        assert int(c["updates"].sum()) == c["improvements"]
        assert int(c["updates"].max()) >= 2   # weighted: some paths are updated again


# ---------------------------------------------------------------------------
# invariant checker: accepts the truth, rejects planted mistakes
# ---------------------------------------------------------------------------

def _reachable_finite(d, s):
    idx = [v for v in range(len(d)) if v != s and d[v] != INF]
    return idx


def test_checker_accepts_oracle_results():
    g = graphgen.rmat(11, 8, 8, weights="u32")
    for s in graphgen.pick_sources(g, 3, 1):
        d, _ = oracle.sssp(g, s, "u32")
        assert oracle.check(g, s, d) == (0, -1)
    gf = graphgen.rmat(11, 8, 8, weights="f32lognormal")
    for s in graphgen.pick_sources(gf, 3, 1):
        d32, _ = oracle.sssp(gf, s, "f32fold")
        assert oracle.check(gf, s, d32) == (0, -1)


def test_checker_rejects_planted_mistakes():
    g = graphgen.rmat(10, 8, 9, weights="u32")
    s = int(graphgen.pick_sources(g, 1, 3)[0])
    d, _ = oracle.sssp(g, s, "u32")
    fin = _reachable_finite(d, s)
    unreach = np.nonzero(d == INF)[0]
    assert fin and unreach.size
    v = fin[len(fin) // 2]
    # V1: wrong source value
    bad = d.copy(); bad[s] = 1
    assert oracle.check(g, s, bad)[0] == 1
    # too low: no tight chain reaches v any more
    bad = d.copy(); bad[v] -= 1
    assert oracle.check(g, s, bad)[0] in (2, 3)
    # too high: some in-edge can still be relaxed
    bad = d.copy(); bad[v] += 1
    assert oracle.check(g, s, bad)[0] == 2
    # reachable vertex reported INF
    bad = d.copy(); bad[v] = INF
    assert oracle.check(g, s, bad)[0] == 2
    # unreachable vertex given a finite value
    bad = d.copy(); bad[unreach[0]] = 5
    assert oracle.check(g, s, bad)[0] in (2, 3, 4)
    # ... and one with no out-edges, so only the tight-chain rule can object
    sink = [int(v) for v in unreach if g.outdeg()[v] == 0]
    if sink:
        bad = d.copy(); bad[sink[0]] = 5
        assert oracle.check(g, s, bad)[0] in (3, 4)


def test_checker_rejects_f32_mistakes():
    g = graphgen.rmat(10, 8, 10, weights="f32lognormal")
    s = int(graphgen.pick_sources(g, 1, 3)[0])
    d, _ = oracle.sssp(g, s, "f32fold")
    fin = [v for v in range(g.n) if v != s and np.isfinite(d[v])]
    v = fin[len(fin) // 3]
    bad = d.copy(); bad[s] = -0.0
    assert oracle.check(g, s, bad)[0] == 1
    bad = d.copy(); bad[v] = np.nextafter(d[v], np.float32(0))
    assert oracle.check(g, s, bad)[0] in (2, 3)
    bad = d.copy(); bad[v] = np.nextafter(d[v], np.float32(np.inf))
    assert oracle.check(g, s, bad)[0] == 2


def test_f32_tolerance_gate():
    g = graphgen.rmat(11, 8, 12, weights="f32lognormal")
    s = int(graphgen.pick_sources(g, 1, 4)[0])
    d32, _ = oracle.sssp(g, s, "f32fold")
    assert oracle.f32_tolerance_violations(g, s, d32).size == 0
    d64, h64 = oracle.sssp(g, s, "f64")
    # an error of 1e-4 relative is far outside 2^-22 * hops
    v = int(np.nonzero(np.isfinite(d64) & (h64 > 1))[0][0])
    bad = d32.copy(); bad[v] = np.float32(d64[v] * (1 + 1e-4))
    assert v in oracle.f32_tolerance_violations(g, s, bad)
    bad = d32.copy(); bad[v] = np.inf
    assert v in oracle.f32_tolerance_violations(g, s, bad)


# --- signed int32 weights: Bellman-Ford with the source guard ---------------

I64MAX = np.iinfo(np.int64).max


@pytest.mark.parametrize("seed", range(4))
def test_bellman_ford_equals_dijkstra_on_nonnegative_weights(seed):
    g = graphgen.rmat(9, 8, 300 + seed, weights="u32")
    gi = graphgen.from_edges(g.n, np.repeat(np.arange(g.n), g.outdeg()), g.colidx,
                             g.w.astype(np.int64), "i32")
    for s in graphgen.pick_sources(g, 3, seed):
        d, ok = oracle.bellman_ford(gi, int(s))
        ref, _ = oracle.sssp(g, int(s), "u32")
        assert ok
        assert np.array_equal(np.where(d == I64MAX, 0xFFFFFFFF, d), ref.astype(np.int64))


@pytest.mark.parametrize("seed", range(4))
def test_bellman_ford_potential_shift_identity(seed):
    """w'(u,v) = w(u,v) + p(u) - p(v) keeps every cycle's weight, so the
    shortest paths are those of w and d'(v) = d(v) + p(s) - p(v)."""
    g = graphgen.er(300, 2400, 400 + seed, weights="u32", wlo=1, whi=50)
    gs, p = graphgen.potential_shift(g, 500, seed)
    assert (gs.w < 0).mean() > 0.2
    for s in graphgen.pick_sources(g, 3, seed):
        d, ok = oracle.bellman_ford(gs, int(s))
        ref, _ = oracle.sssp(g, int(s), "u32")
        assert ok
        reach = ref != 0xFFFFFFFF
        assert np.array_equal(d == I64MAX, ~reach)
        assert np.array_equal(d[reach], ref[reach].astype(np.int64) + p[s] - p[reach])


def _g(n, edges):
    e = np.array(edges, dtype=np.int64).reshape(-1, 3)
    return graphgen.from_edges(n, e[:, 0], e[:, 1], e[:, 2], "i32")


def test_bellman_ford_worked_examples():
    # 0->1 (4), 0->2 (5), 2->1 (-3), 1->3 (2), 3->2 (1): the cycle 2-1-3 weighs 0
    g = _g(4, [(0, 1, 4), (0, 2, 5), (2, 1, -3), (1, 3, 2), (3, 2, 1)])
    d, ok = oracle.bellman_ford(g, 0)
    assert ok and d.tolist() == [0, 2, 5, 4]
    # the same cycle at weight -1 is reachable: no shortest paths
    g = _g(4, [(0, 1, 4), (0, 2, 5), (2, 1, -3), (1, 3, 2), (3, 2, 0)])
    assert not oracle.bellman_ford(g, 0)[1]
    # a negative cycle that the source cannot reach changes nothing
    g = _g(4, [(0, 1, 3), (2, 3, -5), (3, 2, 1)])
    d, ok = oracle.bellman_ford(g, 0)
    assert ok and d.tolist() == [0, 3, I64MAX, I64MAX]
    # a negative cycle through the source only: its edge back into the source
    # is never relaxed (the source keeps 0), so the distances exist
    g = _g(2, [(0, 1, -2), (1, 0, 1)])
    d, ok = oracle.bellman_ford(g, 0)
    assert ok and d.tolist() == [0, -2]
    # from the other end the guard drops 0->1 instead
    d1, ok1 = oracle.bellman_ford(g, 1)
    assert ok1 and d1.tolist() == [1, 0]
