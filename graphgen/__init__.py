"""Seeded synthetic graph inputs, shared by the oracle and the GPU path.

This module only produces inputs (edge lists, CSR arrays, weights, source
lists).  It holds none of the shortest-path arithmetic; the oracle and the HIP
library each implement that on their own.

The C generator (``graphgen.c``) is compiled with gcc into ``libgraphgen.so``
next to this file; ``build()`` does that, and importing builds it once if it is
missing.
"""
from __future__ import annotations

import ctypes
import hashlib
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")

_i32p = ctypes.POINTER(ctypes.c_int32)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_f32p = ctypes.POINTER(ctypes.c_float)
_f64p = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64


def build(force: bool = True) -> str:
    """Compile graphgen.c into libgraphgen.so (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.gg_er_edges.argtypes = [_i64, _i64, _u64, _i32p, _i32p]
        lib.gg_er_edges.restype = _i64
        lib.gg_rmat_edges.argtypes = [ctypes.c_int32, _i64, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, _u64, ctypes.c_int32, _i32p, _i32p]
        lib.gg_rmat_edges.restype = _i64
        lib.gg_grid_pairs.argtypes = [ctypes.c_int32, ctypes.c_int32]
        lib.gg_grid_pairs.restype = _i64
        lib.gg_grid_edges.argtypes = [ctypes.c_int32, ctypes.c_int32, _i64, _u64, _i32p, _i32p]
        lib.gg_grid_edges.restype = _i64
        lib.gg_csr_build.argtypes = [_i64, _i64, _i32p, _i32p, _i32p, _i32p]
        lib.gg_csr_build.restype = ctypes.c_int32
        lib.gg_weights_u32.argtypes = [_i64, ctypes.c_uint32, ctypes.c_uint32, _u64, _u32p]
        lib.gg_weights_f32_unit.argtypes = [_i64, _u64, _f32p]
        lib.gg_weights_f32_range02.argtypes = [_i64, _u64, _f32p]
        lib.gg_weights_f32_lognormal.argtypes = [_i64, _u64, _f32p]
        lib.gg_pick_sources.argtypes = [_i64, _i32p, _i64, _u64, _i32p]
        lib.gg_pick_sources.restype = _i64
        lib.gg_uniform.argtypes = [_i64, _u64, _f64p]
        _lib = lib
    return _lib


def _p(a: np.ndarray, t):
    return a.ctypes.data_as(t)


@dataclass
class Graph:
    """Directed graph in CSR form (int32 rowptr/colidx) with per-edge weights.

    ``wtype`` is ``"u32"`` (uint32 weights), ``"f32"`` (float32 weights, all
    finite, sign bit clear) or ``"i32"`` (int32 weights of either sign).
    """
    n: int
    rowptr: np.ndarray
    colidx: np.ndarray
    w: np.ndarray
    wtype: str
    name: str = "graph"
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.colidx.shape[0])

    def outdeg(self) -> np.ndarray:
        return np.diff(self.rowptr.astype(np.int64))

    def sha256(self) -> str:
        h = hashlib.sha256()
        for a in (self.rowptr, self.colidx, self.w):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()

    def with_weights(self, w: np.ndarray, wtype: str) -> "Graph":
        return Graph(self.n, self.rowptr, self.colidx, np.ascontiguousarray(w), wtype,
                     self.name, dict(self.meta))


# ---------------------------------------------------------------------------
# weights
# ---------------------------------------------------------------------------

def weights_u32(m: int, lo: int, hi: int, seed: int) -> np.ndarray:
    w = np.empty(m, dtype=np.uint32)
    if m:
        _L().gg_weights_u32(m, lo, hi, seed, _p(w, _u32p))
    return w


def weights_f32_unit(m: int, seed: int) -> np.ndarray:
    """fp32 uniform on (0,1], multiples of 2^-24."""
    w = np.empty(m, dtype=np.float32)
    if m:
        _L().gg_weights_f32_unit(m, seed, _p(w, _f32p))
    return w


def weights_f32_range02(m: int, seed: int) -> np.ndarray:
    """fp32 uniform on [0,2], multiples of 2^-23 (zero included)."""
    w = np.empty(m, dtype=np.float32)
    if m:
        _L().gg_weights_f32_range02(m, seed, _p(w, _f32p))
    return w


def weights_f32_lognormal(m: int, seed: int) -> np.ndarray:
    w = np.empty(m, dtype=np.float32)
    if m:
        _L().gg_weights_f32_lognormal(m, seed, _p(w, _f32p))
    return w


def make_weights(m: int, kind: str, seed: int, lo: int = 1, hi: int = 255):
    """kind: 'u32' (uniform [lo,hi]), 'f32unit' ((0,1]), 'f32range02' ([0,2]),
    'f32lognormal', 'f32one' (all 1.0), 'u32one' (all 1)."""
    if kind == "u32":
        return weights_u32(m, lo, hi, seed), "u32"
    if kind == "u32one":
        return np.ones(m, dtype=np.uint32), "u32"
    if kind == "f32unit":
        return weights_f32_unit(m, seed), "f32"
    if kind == "f32range02":
        return weights_f32_range02(m, seed), "f32"
    if kind == "f32lognormal":
        return weights_f32_lognormal(m, seed), "f32"
    if kind == "f32one":
        return np.ones(m, dtype=np.float32), "f32"
    raise ValueError(f"unknown weight kind {kind!r}")


# ---------------------------------------------------------------------------
# graphs
# ---------------------------------------------------------------------------

def csr_from_edges(n: int, src: np.ndarray, dst: np.ndarray):
    """Edge list -> (rowptr, colidx), rows sorted by column, duplicates kept."""
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    m = int(src.shape[0])
    rowptr = np.empty(n + 1, dtype=np.int32)
    colidx = np.empty(m, dtype=np.int32)
    rc = _L().gg_csr_build(n, m, _p(src, _i32p), _p(dst, _i32p), _p(rowptr, _i32p),
                           _p(colidx, _i32p))
    if rc != 0:
        raise ValueError(f"gg_csr_build failed ({rc})")
    return rowptr, colidx


def from_edges(n: int, src, dst, w, wtype: str | None = None, name: str = "custom") -> Graph:
    """Build a graph from an explicit edge list (weights follow the edge order).

    The rows are sorted by column with a stable key so each weight stays with
    its edge."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    w = np.asarray(w)
    if wtype is None:
        wtype = "f32" if np.issubdtype(w.dtype, np.floating) else "u32"
    w = w.astype({"f32": np.float32, "u32": np.uint32, "i32": np.int32}[wtype])
    order = np.lexsort((dst, src)) if src.size else np.zeros(0, dtype=np.int64)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    if src.size:
        np.add.at(rowptr, src + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int32)
    return Graph(n, rowptr, dst[order].astype(np.int32), np.ascontiguousarray(w[order]), wtype,
                 name)


def er(n: int, m: int, seed: int, weights: str = "u32", wlo: int = 1, whi: int = 100,
       wseed: int | None = None) -> Graph:
    """Directed Erdos-Renyi, uniform endpoints, self-loops redrawn (m exact)."""
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    if m:
        rc = _L().gg_er_edges(n, m, seed, _p(src, _i32p), _p(dst, _i32p))
        if rc < 0:
            raise ValueError("gg_er_edges failed")
    rowptr, colidx = csr_from_edges(n, src, dst)
    del src, dst
    w, wt = make_weights(m, weights, seed * 7919 + 1 if wseed is None else wseed, wlo, whi)
    return Graph(n, rowptr, colidx, w, wt, f"er_n{n}_m{m}",
                 {"kind": "er", "seed": seed, "weights": weights})


def rmat(scale: int, edge_factor: int, seed: int, weights: str = "u32", wlo: int = 1,
         whi: int = 255, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         permute: bool = True, wseed: int | None = None) -> Graph:
    """R-MAT with 2^scale vertices and edge_factor*2^scale edge draws; self-loops
    dropped, duplicates kept, seeded vertex relabelling."""
    n = 1 << scale
    mdraw = edge_factor * n
    src = np.empty(mdraw, dtype=np.int32)
    dst = np.empty(mdraw, dtype=np.int32)
    k = _L().gg_rmat_edges(scale, mdraw, a, b, c, seed, 1 if permute else 0,
                           _p(src, _i32p), _p(dst, _i32p))
    if k < 0:
        raise ValueError("gg_rmat_edges failed")
    rowptr, colidx = csr_from_edges(n, src[:k], dst[:k])
    del src, dst
    w, wt = make_weights(int(k), weights, seed * 7919 + 1 if wseed is None else wseed, wlo, whi)
    return Graph(n, rowptr, colidx, w, wt, f"rmat_s{scale}_ef{edge_factor}",
                 {"kind": "rmat", "seed": seed, "weights": weights, "draws": mdraw})


def grid(rows: int, cols: int, del_frac: float, seed: int, weights: str = "f32unit",
         wseed: int | None = None) -> Graph:
    """4-neighbour grid; floor(del_frac * pairs) undirected pairs deleted at
    random; both directions of the rest stored; weight per directed edge."""
    npairs = int(_L().gg_grid_pairs(rows, cols))
    ndel = int(del_frac * npairs)
    cap = 2 * npairs
    src = np.empty(max(cap, 1), dtype=np.int32)
    dst = np.empty(max(cap, 1), dtype=np.int32)
    k = _L().gg_grid_edges(rows, cols, ndel, seed, _p(src, _i32p), _p(dst, _i32p))
    if k < 0:
        raise ValueError("gg_grid_edges failed")
    n = rows * cols
    rowptr, colidx = csr_from_edges(n, src[:k], dst[:k])
    del src, dst
    w, wt = make_weights(int(k), weights, seed * 7919 + 1 if wseed is None else wseed)
    return Graph(n, rowptr, colidx, w, wt, f"grid_{rows}x{cols}",
                 {"kind": "grid", "seed": seed, "weights": weights, "deleted_pairs": ndel})


def potential_shift(g: Graph, pmax: int, seed: int) -> tuple[Graph, np.ndarray]:
    """Signed weights without negative cycles: w'(u,v) = w(u,v) + p(u) - p(v)
    for a uint32 graph g and integer potentials p uniform in [0, pmax] (every
    cycle keeps its weight, so none becomes negative; many edges do).
    Returns the int32-weighted graph and p."""
    assert g.wtype == "u32"
    rng = np.random.default_rng(seed)
    p = rng.integers(0, pmax + 1, size=g.n).astype(np.int64)
    src = np.repeat(np.arange(g.n, dtype=np.int64), g.outdeg())
    w = g.w.astype(np.int64) + p[src] - p[g.colidx.astype(np.int64)]
    assert w.min() >= -(1 << 31) and w.max() < (1 << 31)
    return Graph(g.n, g.rowptr, g.colidx, np.ascontiguousarray(w.astype(np.int32)), "i32",
                 g.name + f"_shift{pmax}"), p


def pick_sources(g: Graph, k: int, seed: int) -> np.ndarray:
    """k distinct sources, uniform among vertices with out-degree >= 1."""
    out = np.empty(max(k, 1), dtype=np.int32)
    got = _L().gg_pick_sources(g.n, _p(g.rowptr, _i32p), k, seed, _p(out, _i32p))
    if got < 0:
        raise MemoryError("gg_pick_sources failed")
    return out[:got].copy()


def uniform(count: int, seed: int) -> np.ndarray:
    out = np.empty(max(count, 1), dtype=np.float64)
    if count:
        _L().gg_uniform(count, seed, _p(out, _f64p))
    return out[:count]
