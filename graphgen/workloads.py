"""Workload recipes: the synthetic graphs that stand in for the paper's SNAP and
SuiteSparse inputs (Section 4.1, Table 2), sized to the paper's modal buckets.

Every recipe is seeded; the same call gives byte-identical arrays.
"""
from __future__ import annotations

import numpy as np

from . import Graph, er, grid, pick_sources, rmat, uniform

# Plain SSSP, one source (vertex 0): directed ER n=1000, m=8000, u32 weights in [1,100].
def er_small(seed: int = 1) -> tuple[Graph, np.ndarray]:
    g = er(1000, 8000, seed, weights="u32", wlo=1, whi=100)
    return g, np.array([0], dtype=np.int32)


# Plain single-source at scale: R-MAT scale 22, edge factor 16, u32 weights [1,255];
# 16 sources.
def rmat22(seed: int = 22, nsrc: int = 16, scale: int = 22) -> tuple[Graph, np.ndarray]:
    g = rmat(scale, 16, seed, weights="u32", wlo=1, whi=255)
    return g, pick_sources(g, nsrc, seed + 100)


# High step count: 2048x2048 grid, 1 % of pairs deleted, fp32 weights U(0,1]; 8 sources.
def grid2048(seed: int = 2048, nsrc: int = 8, side: int = 2048) -> tuple[Graph, np.ndarray]:
    g = grid(side, side, 0.01, seed, weights="f32unit")
    return g, pick_sources(g, nsrc, seed + 1)


# Batching: R-MAT scale 20, edge factor 16, u32 weights [1,255]; 256 distinct sources.
def rmat20_tile(seed: int = 20, k: int = 256, scale: int = 20) -> tuple[Graph, np.ndarray]:
    g = rmat(scale, 16, seed, weights="u32", wlo=1, whi=255)
    return g, pick_sources(g, k, seed + 100)


# Batching across graphs: 64 uneven directed ER graphs, n = round(10^U(lo,hi)),
# m = 8n, fp32 lognormal(0,1) weights, one source each.
def er_batch(seed: int = 64, count: int = 64, lo: float = 4.0, hi: float = 6.0
             ) -> list[tuple[Graph, int]]:
    u = uniform(count, seed)
    out = []
    for i in range(count):
        n = int(round(10 ** (lo + (hi - lo) * u[i])))
        g = er(n, 8 * n, seed * 1000 + i, weights="f32lognormal")
        src = int(pick_sources(g, 1, seed * 1000 + i + 500)[0])
        out.append((g, src))
    return out


# Serving: 32 resident R-MAT graphs; graph i has scale 14 + (i mod 9), edge factor
# (8,16,32)[(i div 9) mod 3]; u32 [1,255] if i is even, else fp32 lognormal(0,1).
def serving_graph_spec(i: int, max_scale: int = 22) -> dict:
    scale = min(14 + (i % 9), max_scale)
    ef = (8, 16, 32)[(i // 9) % 3]
    weights = "u32" if i % 2 == 0 else "f32lognormal"
    return {"scale": scale, "edge_factor": ef, "weights": weights, "seed": 500 + i}


def serving_graph(i: int, max_scale: int = 22) -> Graph:
    s = serving_graph_spec(i, max_scale)
    return rmat(s["scale"], s["edge_factor"], s["seed"], weights=s["weights"])
