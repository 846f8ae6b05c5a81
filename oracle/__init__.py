"""TEST INFRASTRUCTURE ONLY -- the CPU oracle for the GOVM hot path.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The HIP library never calls it and it
never calls the HIP library; the two share no code.  What the oracle computes,
and which part of the paper each function follows, is stated in ``oracle.c``:

* ``sssp``   -- Dijkstra (Section 2.1), lexicographic (distance, hops) keys, in
  three modes: ``u32`` (exact 64-bit sums, clipped to the uint32 INF), ``f64``
  (fp64 sums of the fp32 weights) and ``f32fold`` (fp32 left fold, RNE).
* ``fw``     -- Floyd-Warshall (Section 2.3), the recurrence Section 3.1 says the
  method's fixed point shares.
* ``brute``  -- every simple path from the source (n <= 12).
* ``bfs``    -- hop levels; the unit-weight special case of Section 1 (mu = 1).
* ``check``  -- invariants V1..V4 of any candidate distance vector.
* ``govm``   -- Algorithm 2 restated sequentially; step and work counters only.

Pins: ``tests/test_oracle.py`` checks each of these against brute force, closed
forms and planted mistakes.  The paper's own mu figures (Section 4.2) need its
datasets: parity unpinned for those numbers.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

U32_INF = np.uint32(0xFFFFFFFF)

_i32p = ctypes.POINTER(ctypes.c_int32)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_f32p = ctypes.POINTER(ctypes.c_float)
_f64p = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (plain IEEE arithmetic: no fast-math, no FMA
    contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-Wall",
                               "-fno-strict-aliasing", "-ffp-contract=off", "-fno-fast-math",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        L.oracle_sssp_u32.argtypes = [_i32, _i32p, _i32p, _u32p, _i32, _u32p, _i32p]
        L.oracle_sssp_u32.restype = _i32
        L.oracle_sssp_f64.argtypes = [_i32, _i32p, _i32p, _f32p, _i32, _f64p, _i32p]
        L.oracle_sssp_f64.restype = _i32
        L.oracle_sssp_f32fold.argtypes = [_i32, _i32p, _i32p, _f32p, _i32, _f32p, _i32p]
        L.oracle_sssp_f32fold.restype = _i32
        L.oracle_fw_u64.argtypes = [_i32, _i32p, _i32p, _u32p, _u64p]
        L.oracle_fw_f64.argtypes = [_i32, _i32p, _i32p, _f32p, _f64p]
        L.oracle_brute.argtypes = [_i32, _i32p, _i32p, _vp, _i32, _i32, _u64p, _f64p, _i32p]
        L.oracle_brute.restype = _i32
        L.oracle_bellman_ford_i32.argtypes = [_i32, _i32p, _i32p, _i32p, _i32, _i64p]
        L.oracle_bellman_ford_i32.restype = _i32
        L.oracle_bfs.argtypes = [_i32, _i32p, _i32p, _i32, _i32p]
        L.oracle_bfs.restype = _i32
        L.oracle_check_u32.argtypes = [_i32, _i32p, _i32p, _u32p, _i32, _u32p, _i32p]
        L.oracle_check_u32.restype = _i32
        L.oracle_check_f32.argtypes = [_i32, _i32p, _i32p, _f32p, _i32, _f32p, _i32p]
        L.oracle_check_f32.restype = _i32
        L.oracle_govm.argtypes = [_i32, _i32p, _i32p, _vp, _i32, _i32, _i32, ctypes.c_uint64,
                                  _vp, _i64p, _i32p]
        L.oracle_govm.restype = _i32
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def _csr(g):
    return (int(g.n), _p(g.rowptr, _i32p), _p(g.colidx, _i32p))


def default_mode(g) -> str:
    return "u32" if g.wtype == "u32" else "f64"


def sssp(g, s: int, mode: str | None = None):
    """Dijkstra distances and min-hop counts from s.  Returns (dist, hops).

    u32 mode: uint32 array, 0xFFFFFFFF = unreachable (or a sum >= 2^32-1).
    f64 mode: float64 array; f32fold mode: float32 array; +inf = unreachable.
    hops: int32, -1 = unreachable."""
    mode = mode or default_mode(g)
    n, rp, ci = _csr(g)
    hops = np.empty(n, dtype=np.int32)
    if mode == "u32":
        assert g.wtype == "u32"
        d = np.empty(n, dtype=np.uint32)
        rc = _L().oracle_sssp_u32(n, rp, ci, _p(g.w, _u32p), int(s), _p(d, _u32p), _p(hops, _i32p))
    elif mode == "f64":
        assert g.wtype == "f32"
        d = np.empty(n, dtype=np.float64)
        rc = _L().oracle_sssp_f64(n, rp, ci, _p(g.w, _f32p), int(s), _p(d, _f64p), _p(hops, _i32p))
    elif mode == "f32fold":
        assert g.wtype == "f32"
        d = np.empty(n, dtype=np.float32)
        rc = _L().oracle_sssp_f32fold(n, rp, ci, _p(g.w, _f32p), int(s), _p(d, _f32p),
                                      _p(hops, _i32p))
    else:
        raise ValueError(mode)
    if rc != 0:
        raise MemoryError("oracle sssp failed")
    return d, hops


def fw(g):
    """Floyd-Warshall all pairs; u32 graphs -> uint64 matrix (UINT64_MAX = none),
    f32 graphs -> float64 matrix (+inf = none)."""
    n, rp, ci = _csr(g)
    if g.wtype == "u32":
        D = np.empty((n, n), dtype=np.uint64)
        _L().oracle_fw_u64(n, rp, ci, _p(g.w, _u32p), _p(D, _u64p))
    else:
        D = np.empty((n, n), dtype=np.float64)
        _L().oracle_fw_f64(n, rp, ci, _p(g.w, _f32p), _p(D, _f64p))
    return D


def brute(g, s: int, mode: str | None = None):
    """Min over all simple paths.  mode 'u32' -> uint64 dists, 'f64' -> float64
    exact sums, 'f32fold' -> fp32 left folds (as float64).  Returns (dist, hops)."""
    mode = mode or default_mode(g)
    n, rp, ci = _csr(g)
    hops = np.empty(n, dtype=np.int32)
    du = np.empty(n, dtype=np.uint64)
    df = np.empty(n, dtype=np.float64)
    code = {"u32": 0, "f64": 1, "f32fold": 2}[mode]
    rc = _L().oracle_brute(n, rp, ci, g.w.ctypes.data_as(_vp), int(s), code, _p(du, _u64p),
                           _p(df, _f64p), _p(hops, _i32p))
    if rc != 0:
        raise ValueError("brute force needs n <= 12")
    return (du if code == 0 else df), hops


def bellman_ford(g, s: int):
    """Signed int32 weights: (dist, ok).  dist: int64, INT64_MAX where
    unreachable; shortest paths of the graph without the edges into s (the
    source's distance is never lowered, as in Algorithm 2).  ok = False when
    a negative cycle is reachable (dist is then meaningless)."""
    assert g.wtype == "i32"
    n, rp, ci = _csr(g)
    d = np.empty(n, dtype=np.int64)
    ok = _L().oracle_bellman_ford_i32(n, rp, ci, _p(g.w, _i32p), int(s), _p(d, _i64p))
    return d, bool(ok)


def bfs(g, s: int):
    n, rp, ci = _csr(g)
    lvl = np.empty(n, dtype=np.int32)
    _L().oracle_bfs(n, rp, ci, int(s), _p(lvl, _i32p))
    return lvl


def check(g, s: int, d) -> tuple[int, int]:
    """Invariants V1..V4 on a candidate distance vector (uint32 for u32 graphs,
    float32 for f32 graphs).  Returns (code, vertex); code 0 = all hold."""
    n, rp, ci = _csr(g)
    bad = ctypes.c_int32(-1)
    if g.wtype == "u32":
        d = np.ascontiguousarray(d, dtype=np.uint32)
        rc = _L().oracle_check_u32(n, rp, ci, _p(g.w, _u32p), int(s), _p(d, _u32p),
                                   ctypes.byref(bad))
    else:
        d = np.ascontiguousarray(d, dtype=np.float32)
        rc = _L().oracle_check_f32(n, rp, ci, _p(g.w, _f32p), int(s), _p(d, _f32p),
                                   ctypes.byref(bad))
    if rc < 0:
        raise MemoryError("oracle check failed")
    return int(rc), int(bad.value)


def govm(g, s: int, order: int = 0, seed: int = 0, per_vertex: bool = False):
    """Algorithm 2 restated (see oracle.c).  Returns (dist, counters dict); with
    per_vertex=True the dict also holds ``updates``, the number of times each
    vertex's distance was lowered (int32[n])."""
    n, rp, ci = _csr(g)
    is_f32 = 1 if g.wtype == "f32" else 0
    d = np.empty(n, dtype=np.float32 if is_f32 else np.uint32)
    c = np.zeros(5, dtype=np.int64)
    upd = np.zeros(n, dtype=np.int32) if per_vertex else None
    rc = _L().oracle_govm(n, rp, ci, g.w.ctypes.data_as(_vp), is_f32, int(s), int(order),
                          int(seed), d.ctypes.data_as(_vp), _p(c, _i64p),
                          _p(upd, _i32p) if per_vertex else None)
    if rc != 0:
        raise MemoryError("oracle govm failed")
    res = {"steps": int(c[0]), "converged": int(c[1]), "frontier_entries": int(c[2]),
           "edges_scanned": int(c[3]), "improvements": int(c[4])}
    if per_vertex:
        res["updates"] = upd
    return d, res


# ---------------------------------------------------------------------------
# comparison helpers used by the parity tests
# ---------------------------------------------------------------------------

def f32_tolerance_violations(g, s: int, d_gpu: np.ndarray, d64=None, h64=None, d32=None,
                             h32=None) -> np.ndarray:
    """Vertices where |d_gpu - d64| > 2^-22 * hops(v) * d64(v), with
    hops(v) = max(h64(v), h32(v)); INF must match exactly and d[s] must be 0."""
    if d64 is None:
        d64, h64 = sssp(g, s, "f64")
    if d32 is None:
        d32, h32 = sssp(g, s, "f32fold")
    d_gpu = np.asarray(d_gpu, dtype=np.float32).astype(np.float64)
    hops = np.maximum(h64, h32).astype(np.float64)
    inf_ref = ~np.isfinite(d64)
    inf_gpu = ~np.isfinite(d_gpu)
    bad = inf_ref != inf_gpu
    fin = ~inf_ref & ~inf_gpu
    tol = np.ldexp(1.0, -22) * hops * d64
    with np.errstate(invalid="ignore"):
        err = np.where(fin, np.abs(d_gpu - np.where(fin, d64, 0.0)), 0.0)
    bad |= fin & (err > tol)
    if d_gpu[s] != 0.0:
        bad[s] = True
    return np.nonzero(bad)[0]


def m_reach(g, s: int) -> int:
    """Sum of out-degrees over vertices reachable from s (the directed analogue
    of E_wcc(s), Table 1 / Section 3.4)."""
    lvl = bfs(g, s)
    return int(g.outdeg()[lvl >= 0].sum())


def time_sources(g, sources, threads: int, mode: str | None = None, keep: bool = False) -> dict:
    """Run Dijkstra from each source on `threads` host threads (ctypes releases
    the GIL).  Returns the wall time (and, with keep=True, the distance array
    of each source, in the order given)."""
    sources = list(int(x) for x in sources)
    idx = [0]
    lock = threading.Lock()
    dist = [None] * len(sources)

    def worker():
        while True:
            with lock:
                if idx[0] >= len(sources):
                    return
                i = idx[0]
                idx[0] += 1
            d, _ = sssp(g, sources[i], mode)
            if keep:
                dist[i] = d

    ts = [threading.Thread(target=worker) for _ in range(max(1, threads))]
    t0 = time.perf_counter()
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    res = {"seconds": time.perf_counter() - t0, "sources": len(sources), "threads": len(ts)}
    if keep:
        res["dist"] = dist
    return res
