"""Seeded random parity sweep of the HIP path against the oracle.

Graphs of several families and sizes (so that the one-workgroup LDS, tiny,
small, persistent and step-launch paths and the tile tiers are all reached),
uint32 weights (zero weights included) and fp32 weights of three
distributions, single-source and batched calls under launch tunings drawn
from fixed lists.  Every single-source result and a sample of every batch's
columns is compared with the oracle: uint32 bit for bit, fp32 bit for bit
against the fp32-fold oracle and within the fp64 tolerance.  The same
families also run with signed int32 weights (potential-shifted, so no cycle
is negative: Bellman-Ford and Dijkstra shifted back) and as hop counts (BFS
levels).  The draws are seeded, so every run checks the same cases.
"""
import numpy as np
import pytest

import graphgen
import oracle
from gpu_helpers import INF32, announce, assert_sssp_matches, to_np

pytestmark = pytest.mark.gpu

SS_TUNINGS = [
    dict(),
    dict(small_m=0),                                   # multi-workgroup paths
    dict(small_m=0, mode=1, step_launches=3),          # step launches, then persistent
    dict(small_m=0, mode=2),                           # persistent only
    dict(small_m=0, t_lane=4, t_wave=64, t_chunk=256), # every tier on small rows
    dict(small_m=1 << 30),                             # one workgroup whatever the size
]
TILE_TUNINGS = [
    dict(),
    dict(tile_sparse=64, tile_t_group=64, tile_t_wave=128),
    dict(tile_step_launches=2),
    dict(mode=2),
    dict(tile_skip=1, tile_t_wave=32, tile_t_chunk=64),
    dict(tile_sparse=0, tile_t_group=0),
]
WEIGHTS = ["u32", "u32zero", "f32unit", "f32lognormal", "f32range02"]
CASES = 64


def _weights(kind):
    if kind == "u32zero":
        return dict(weights="u32", wlo=0, whi=3)
    return dict(weights=kind)


def _graph(rng, i, wk=None):
    fam = int(rng.integers(0, 5))
    drawn = WEIGHTS[int(rng.integers(0, len(WEIGHTS)))]
    wk = wk or drawn
    seed = 9000 + i
    if fam == 0:
        n = int(rng.integers(2, 9000))
        m = int(rng.integers(0, 10 * n))
        return graphgen.er(n, m, seed, **_weights(wk))
    if fam == 1:
        scale = int(rng.integers(3, 15))
        ef = int(rng.integers(1, 17))
        kw = _weights(wk)
        if wk == "u32zero":
            return graphgen.rmat(scale, ef, seed, weights="u32", wlo=0, whi=3)
        return graphgen.rmat(scale, ef, seed, **kw)
    if fam == 2:
        rows, cols = int(rng.integers(1, 90)), int(rng.integers(1, 90))
        return graphgen.grid(rows, cols, 0.02, seed,
                             weights="u32" if wk.startswith("u32") else wk)
    w = graphgen.make_weights
    if fam == 3:  # star: a hub row, leaves pointing back
        n = int(rng.integers(2, 20000))
        src = np.concatenate([np.zeros(n - 1, np.int64), np.arange(1, n)])
        dst = np.concatenate([np.arange(1, n), np.zeros(n - 1, np.int64)])
    else:         # chain with a few shortcuts
        n = int(rng.integers(2, 3000))
        extra = int(rng.integers(0, 20))
        src = np.concatenate([np.arange(n - 1), rng.integers(0, n, extra)])
        dst = np.concatenate([np.arange(1, n), rng.integers(0, n, extra)])
    kind = "u32" if wk == "u32zero" else wk
    ww, wt = w(src.size, kind, seed, 0 if wk == "u32zero" else 1, 3 if wk == "u32zero" else 255)
    return graphgen.from_edges(n, src, dst, ww, wt, name=f"fam{fam}")


def _sources(g, k, seed):
    s = graphgen.pick_sources(g, k, seed)
    return s if s.size else np.zeros(1, np.int32)


@pytest.mark.parametrize("i", range(CASES))
def test_random_graph_sssp_and_msssp(dawn, i):
    import torch
    rng = np.random.default_rng(424242 + i)
    g = _graph(rng, i)
    csr = dawn.Csr.from_graph(g)
    ti = int(rng.integers(0, len(SS_TUNINGS)))
    srcs = _sources(g, 2, 77 + i)
    announce("random sssp", i, g.name, "n", g.n, "m", g.m, g.wtype, SS_TUNINGS[ti])
    prev = dawn.set_tuning(**SS_TUNINGS[ti]) if SS_TUNINGS[ti] else None
    try:
        for s in srcs:
            info = dawn.info_tensor()
            d = dawn.sssp(csr, int(s), info=info)
            torch.cuda.synchronize()
            assert dawn.read_info(info)["converged"] == 1
            assert_sssp_matches(g, int(s), to_np(d), tag=f"case {i} sssp")
    finally:
        if prev is not None:
            dawn.set_tuning(**prev)
    k = int(rng.integers(1, 300))
    tj = int(rng.integers(0, len(TILE_TUNINGS)))
    ks = _sources(g, k, 177 + i)
    announce("random msssp", i, g.name, "k", ks.size, TILE_TUNINGS[tj])
    prev = dawn.set_tuning(**TILE_TUNINGS[tj]) if TILE_TUNINGS[tj] else None
    try:
        info = dawn.info_tensor()
        D = to_np(dawn.msssp(csr, ks, info=info))
        torch.cuda.synchronize()
        assert dawn.read_info(info)["converged"] == 1
    finally:
        if prev is not None:
            dawn.set_tuning(**prev)
    cols = sorted(set(np.linspace(0, ks.size - 1, min(ks.size, 6)).astype(int).tolist()))
    for j in cols:
        assert_sssp_matches(g, int(ks[j]), D[j], tag=f"case {i} msssp col {j}")


I32MAX = np.iinfo(np.int32).max
I64MAX = np.iinfo(np.int64).max


@pytest.mark.parametrize("i", range(24))
def test_random_graph_signed_weights(dawn, i):
    import torch
    rng = np.random.default_rng(515151 + i)
    g0 = _graph(rng, i, wk="u32")
    g, p = graphgen.potential_shift(g0, 3000, 31 + i)
    csr = dawn.Csr.from_graph(g)
    ti = int(rng.integers(0, len(SS_TUNINGS)))
    announce("random i32 sssp", i, g.name, "n", g.n, "m", g.m, SS_TUNINGS[ti])
    prev = dawn.set_tuning(**SS_TUNINGS[ti]) if SS_TUNINGS[ti] else None
    try:
        for s in _sources(g, 2, 277 + i):
            info = dawn.info_tensor()
            d = to_np(dawn.sssp(csr, int(s), info=info)).view(np.int32).astype(np.int64)
            torch.cuda.synchronize()
            assert dawn.read_info(info)["converged"] == 1
            ref, ok = oracle.bellman_ford(g, int(s))
            assert ok
            ref = np.where(ref == I64MAX, I32MAX, ref)
            bad = np.nonzero(d != ref)[0]
            assert bad.size == 0, f"case {i} source {s}: {bad.size} mismatches at {bad[:5]}"
            d0, _ = oracle.sssp(g0, int(s), "u32")
            reach = d0 != INF32
            assert np.array_equal(d[reach], d0[reach].astype(np.int64) + p[s] - p[reach])
    finally:
        if prev is not None:
            dawn.set_tuning(**prev)


UNIT_TILE_TUNINGS = [dict(), dict(tile_step_launches=2), dict(mode=2)]


@pytest.mark.parametrize("i", range(24))
def test_random_graph_hop_counts(dawn, i):
    import torch
    rng = np.random.default_rng(616161 + i)
    g = _graph(rng, i)
    csr = dawn.Csr.from_graph(g, wtype="unit")
    ti = int(rng.integers(0, len(SS_TUNINGS)))
    announce("random unit sssp", i, g.name, "n", g.n, "m", g.m, SS_TUNINGS[ti])

    def levels(s):
        lv = oracle.bfs(g, int(s))
        return np.where(lv >= 0, lv, -1).astype(np.int64).astype(np.uint32)

    prev = dawn.set_tuning(**SS_TUNINGS[ti]) if SS_TUNINGS[ti] else None
    try:
        for s in _sources(g, 2, 377 + i):
            info = dawn.info_tensor()
            d = to_np(dawn.sssp(csr, int(s), info=info)).view(np.uint32)
            torch.cuda.synchronize()
            assert dawn.read_info(info)["converged"] == 1
            assert np.array_equal(d, levels(s)), f"case {i} source {s}"
    finally:
        if prev is not None:
            dawn.set_tuning(**prev)
    tj = int(rng.integers(0, len(UNIT_TILE_TUNINGS)))
    ks = _sources(g, int(rng.integers(1, 300)), 477 + i)
    announce("random unit msssp", i, g.name, "k", ks.size, UNIT_TILE_TUNINGS[tj])
    prev = dawn.set_tuning(**UNIT_TILE_TUNINGS[tj]) if UNIT_TILE_TUNINGS[tj] else None
    try:
        D = to_np(dawn.msssp(csr, ks)).view(np.uint32)
        torch.cuda.synchronize()
    finally:
        if prev is not None:
            dawn.set_tuning(**prev)
    for j in sorted(set(np.linspace(0, ks.size - 1, min(ks.size, 6)).astype(int).tolist())):
        assert np.array_equal(D[j], levels(ks[j])), f"case {i} column {j}"
