"""GPU parity of single-source runs with signed int32 weights: bit-exact
against the Bellman-Ford oracle (with Algorithm 2's source guard) and against
Dijkstra through the potential-shift identity, on every kernel family; a
reachable negative cycle reports converged = 0."""
import numpy as np
import pytest

import graphgen
import oracle
from gpu_helpers import announce, to_np

pytestmark = pytest.mark.gpu

I32MAX = np.iinfo(np.int32).max
I64MAX = np.iinfo(np.int64).max

# tiny (n <= 6144, one workgroup in LDS), small (one workgroup), persistent,
# step launches, and step launches then persistent
TUNINGS = [dict(), dict(small_m=0, mode=2), dict(small_m=0, mode=1),
           dict(small_m=0, step_min_m=0, step_launches=2),
           dict(small_m=0, mode=1, step_launches=4096)]


def _sssp(dawn, csr, s, **tune):
    import torch
    prev = dawn.set_tuning(**tune) if tune else None
    try:
        info = dawn.info_tensor()
        ws = dawn.workspace(dawn.sssp_workspace_bytes(csr.n, csr.m))
        out = dawn.sssp(csr, int(s), ws=ws, info=info, check=False)
        torch.cuda.synchronize()
        return to_np(out).view(np.int32), dawn.read_info(info)
    finally:
        if prev is not None:
            dawn.set_tuning(**prev)


def _ref(g, s):
    d, ok = oracle.bellman_ford(g, int(s))
    assert ok
    return np.where(d == I64MAX, I32MAX, d).astype(np.int64)


@pytest.mark.parametrize("ti", range(len(TUNINGS)))
@pytest.mark.parametrize("kind", ["rmat_lds", "rmat", "er", "rmat_big"])
def test_signed_weights_match_bellman_ford_and_potentials(dawn, kind, ti):
    if kind == "rmat_lds":  # m <= 16384: the whole graph in LDS, edge-parallel steps
        g0 = graphgen.rmat(10, 8, 50, weights="u32", wlo=1, whi=100)
        assert g0.m <= 16384
    elif kind == "rmat":
        g0 = graphgen.rmat(11, 8, 51, weights="u32", wlo=1, whi=100)
    elif kind == "er":
        g0 = graphgen.er(3000, 24000, 52, weights="u32", wlo=1, whi=100)
    else:  # n > 6144: the multi-workgroup and single-workgroup global-memory kernels
        g0 = graphgen.rmat(14, 8, 53, weights="u32", wlo=1, whi=100)
    g, p = graphgen.potential_shift(g0, 3000, 7 + ti)
    assert (g.w < 0).mean() > 0.2
    csr = dawn.Csr.from_graph(g)
    for s in graphgen.pick_sources(g, 3, 60 + ti):
        announce("sssp i32", kind, TUNINGS[ti], int(s))
        d, info = _sssp(dawn, csr, s, **TUNINGS[ti])
        assert info["converged"] == 1
        ref = _ref(g, s)
        bad = np.nonzero(d.astype(np.int64) != ref)[0]
        assert bad.size == 0, f"source {s}: {bad.size} mismatches, v={bad[0]} {d[bad[0]]} {ref[bad[0]]}"
        # Dijkstra on the unshifted weights, shifted back: d'(v) = d(v) + p(s) - p(v)
        d0, _ = oracle.sssp(g0, int(s), "u32")
        reach = d0 != 0xFFFFFFFF
        assert np.array_equal(d[reach].astype(np.int64), d0[reach].astype(np.int64) + p[s] - p[reach])
        assert np.all(d[~reach] == I32MAX)


def _g(n, edges):
    e = np.array(edges, dtype=np.int64).reshape(-1, 3)
    return graphgen.from_edges(n, e[:, 0], e[:, 1], e[:, 2], "i32")


@pytest.mark.parametrize("ti", range(len(TUNINGS)))
def test_negative_cycle_reaches_the_step_cap(dawn, ti):
    # a ring of 500 vertices (weights 1) with one edge of -600 closing it: the
    # cycle weighs -101 and is reachable from 0
    n = 500
    edges = [(i, i + 1, 1) for i in range(n - 1)] + [(n - 1, 1, -600)]
    g = _g(n, edges)
    assert not oracle.bellman_ford(g, 0)[1]
    announce("sssp i32 negative cycle", TUNINGS[ti])
    d, info = _sssp(dawn, dawn.Csr.from_graph(g), 0, **TUNINGS[ti])
    assert info["converged"] == 0


@pytest.mark.parametrize("ti", range(len(TUNINGS)))
def test_negative_cycle_through_the_source_is_cut_by_the_guard(dawn, ti):
    g = _g(4, [(0, 1, -2), (1, 0, 1), (1, 2, 5), (2, 3, -7), (3, 1, 3)])
    d, info = _sssp(dawn, dawn.Csr.from_graph(g), 0, **TUNINGS[ti])
    assert info["converged"] == 1
    assert d.tolist() == _ref(g, 0).tolist() == [0, -2, 3, -4]


def test_sums_outside_int32(dawn):
    big = 1 << 30
    # above: 2^30 + 2^30 >= INT32_MAX reads as unreachable
    g = _g(3, [(0, 1, big), (1, 2, big)])
    d, info = _sssp(dawn, dawn.Csr.from_graph(g), 0)
    assert d.tolist() == [0, big, I32MAX] and info["converged"] == 1
    # below: -2^30 - 2^30 = INT32_MIN leaves the range: not converged
    g = _g(3, [(0, 1, -big), (1, 2, -big)])
    for tune in TUNINGS:
        d, info = _sssp(dawn, dawn.Csr.from_graph(g), 0, **tune)
        assert info["converged"] == 0, tune
    # and the flag does not outlive its run
    g = _g(3, [(0, 1, -5), (1, 2, 7)])
    d, info = _sssp(dawn, dawn.Csr.from_graph(g), 0)
    assert d.tolist() == [0, -5, 2] and info["converged"] == 1
