"""Generator tests: determinism, sizes, structure and weight ranges (no GPU)."""
import numpy as np

import graphgen
from graphgen import workloads


def test_er_sizes_no_self_loops_deterministic():
    g = graphgen.er(1000, 8000, 1)
    assert g.n == 1000 and g.m == 8000
    src = np.repeat(np.arange(g.n), g.outdeg())
    assert not np.any(src == g.colidx)
    assert g.w.dtype == np.uint32 and g.w.min() >= 1 and g.w.max() <= 100
    assert g.sha256() == graphgen.er(1000, 8000, 1).sha256()
    assert g.sha256() != graphgen.er(1000, 8000, 2).sha256()


def test_rmat_counts_and_determinism():
    g = graphgen.rmat(14, 16, 3)
    assert g.n == 1 << 14
    assert 0.99 * 16 * g.n < g.m <= 16 * g.n     # only self-loops dropped
    src = np.repeat(np.arange(g.n), g.outdeg())
    assert not np.any(src == g.colidx)
    # rows sorted by column
    for u in range(0, g.n, 97):
        row = g.colidx[g.rowptr[u]:g.rowptr[u + 1]]
        assert np.all(np.diff(row) >= 0)
    assert g.w.min() >= 1 and g.w.max() <= 255
    assert g.sha256() == graphgen.rmat(14, 16, 3).sha256()
    # skew: the hub is far above the mean degree
    assert g.outdeg().max() > 20 * (g.m / g.n)


def test_grid_structure():
    rows, cols = 31, 47
    g = graphgen.grid(rows, cols, 0.01, 9)
    pairs = rows * (cols - 1) + (rows - 1) * cols
    ndel = int(0.01 * pairs)
    assert g.m == 2 * (pairs - ndel)
    src = np.repeat(np.arange(g.n), g.outdeg())
    dr = np.abs(src // cols - g.colidx // cols)
    dc = np.abs(src % cols - g.colidx % cols)
    assert np.all(dr + dc == 1)
    fwd = set(zip(src.tolist(), g.colidx.tolist()))
    assert all((b, a) in fwd for a, b in fwd)   # both directions stored
    assert g.w.dtype == np.float32 and g.w.min() > 0 and g.w.max() <= 1.0


def test_grid_full_size_counts():
    g = graphgen.grid(2048, 2048, 0.01, 2048)
    assert g.n == 4194304 and g.m == 16601334


def test_weight_samplers():
    w = graphgen.weights_f32_unit(100000, 3)
    q = w.astype(np.float64) * 2 ** 24
    assert w.min() > 0 and w.max() <= 1 and np.all(q == np.round(q))
    w = graphgen.weights_f32_range02(100000, 3)
    assert w.min() >= 0 and w.max() <= 2 and (w == 0).any() is not None
    w = graphgen.weights_f32_lognormal(200000, 4)
    lw = np.log(w.astype(np.float64))
    assert abs(lw.mean()) < 0.02 and abs(lw.std() - 1) < 0.02
    assert np.all(np.isfinite(w)) and np.all(w > 0)
    wu = graphgen.weights_u32(100000, 1, 255, 5)
    assert wu.min() == 1 and wu.max() == 255


def test_sources_distinct_with_out_edges():
    g = graphgen.rmat(12, 8, 1)
    s = graphgen.pick_sources(g, 256, 7)
    assert len(set(s.tolist())) == 256
    assert np.all(g.outdeg()[s] >= 1)
    assert np.array_equal(s, graphgen.pick_sources(g, 256, 7))


def test_workload_recipes_small():
    g, s = workloads.er_small()
    assert g.n == 1000 and g.m == 8000 and s.tolist() == [0]
    batch = workloads.er_batch(count=4, lo=2.0, hi=3.0)
    assert len(batch) == 4
    for gi, si in batch:
        assert gi.m == 8 * gi.n and gi.wtype == "f32" and gi.outdeg()[si] >= 1
    spec = [workloads.serving_graph_spec(i) for i in range(32)]
    assert min(x["scale"] for x in spec) == 14 and max(x["scale"] for x in spec) == 22
    assert {x["edge_factor"] for x in spec} == {8, 16, 32}
