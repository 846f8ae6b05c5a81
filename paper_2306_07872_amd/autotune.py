"""Project autotuner for the GOVM launch parameters.

Picks the tile width, degree-tier thresholds, the pull-step rule (frontier
share and source density), the sparse and group tiers, workgroup shape, grid
size, step launches and step-loop mode that maximise sources/s on a
calibration graph of the same class as the target, by coordinate descent from
the library defaults: each parameter in turn is swept over a short candidate
list (which always holds the current value) with the others held, and the best
value is kept.  Every candidate runs the real HIP path (with the reverse graph
when one is given, so pull steps are part of the search); since the distances
are unique (the fixed point of Algorithm 2 does not depend on how the work is
split), tuning never changes results, only time.

Results are cached as JSON keyed by (GPU architecture, compute units, graph
class, weight type, call kind) in $DAWN_TUNE_CACHE (default
~/.cache/paper_2306_07872_amd/tune.json).
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np

from . import Csr, DawnError, check_runs, get_tuning, msssp, set_tuning, sssp, workspace
from . import sssp_workspace_bytes, tile_bytes

SSSP_SPACE = {
    "wg_threads": [256, 512, 1024],
    "mode": [1, 2],
    "t_lane": [16, 64, 256, 1024],
    "t_wave": [256, 1024, 2048, 8192],
    "t_chunk": [1024, 4096, 8192, 32768],
}

MSSSP_SPACE = {
    "tile_k": [64, 128, 256, 512],
    "tile_pull": [200, 300, 400, 600],
    "tile_pull_src": [4, 8, 16, 32],
    "tile_sparse": [0, 4, 8, 16],
    "tile_t_group": [0, 8, 16],
    "tile_t_wave": [32, 64, 256],
    "tile_t_chunk": [128, 256, 1024],
    "tile_step_launches": [12, 16, 24],
    "wg_threads": [256, 512],
    "grid_per_cu": [2, 4, 8],
}


def cache_path() -> str:
    return os.environ.get("DAWN_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_2306_07872_amd",
                                       "tune.json"))


def graph_class(csr: Csr) -> str:
    """Coarse class of a graph: size, mean degree and degree skew buckets."""
    import torch
    deg = torch.diff(csr.rowptr.to(torch.int64))
    mean = max(csr.m / max(csr.n, 1), 1e-9)
    mx = float(deg.max().item()) if csr.n else 0.0
    skew = mx / mean
    return (f"n2^{int(math.log2(max(csr.n, 1)))}-d{int(round(math.log2(mean + 1)))}"
            f"-skew{'hi' if skew > 64 else 'lo'}")


def device_key() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(p, "gcnArchName", p.name).split(":")[0]
    return f"{arch}-cu{p.multi_processor_count}"


def _load_cache() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(cache: dict):
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + f".tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _to_tuning(params: dict, cus: int) -> dict:
    t = dict(params)
    gpc = t.pop("grid_per_cu", None)
    if gpc is not None:
        t["grid"] = int(gpc) * cus
    return t


def _time_calls(fn, reps: int) -> float:
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def descend(space: dict, base: dict, cus: int, t_default: float, time_trial,
            rounds: int = 1, min_gain: float = 0.03):
    """Coordinate descent over `space` (field -> candidate values), starting
    from the tuning `base` whose calls take `t_default`.  time_trial(trial)
    sets the fields of `trial` over the defaults and returns the time of the
    calls, or None for a combination the library rejects.  A candidate
    replaces the value held only when it is faster by more than `min_gain` (a
    fraction).  Returns (the chosen fields, their time)."""
    best = {}
    best_t = t_default
    for _ in range(rounds):
        for key, cands in space.items():
            cur = best.get(key, base.get(key, base["grid"] // cus if key == "grid_per_cu"
                                     else None))
            cands = list(cands)
            if cur is not None and cur not in cands:
                cands.append(cur)   # the value held now is always a candidate
            results = []
            for c in cands:
                trial = dict(best)
                trial[key] = c
                t = time_trial(trial)
                if t is not None:
                    results.append((t, c))
            if not results:
                continue
            held = [t for t, c in results if c == cur]
            t_held = held[0] if held else best_t
            t, c = min(results)
            if t < t_held * (1.0 - min_gain):
                best[key] = c
                best_t = t
            else:
                best_t = min(best_t, t_held)
    return best, best_t


def tune(csr: Csr, sources, kind: str = "msssp", reps: int = 2, rounds: int = 1,
         space: dict | None = None, verbose: bool = False, tgraph=None,
         min_gain: float = 0.03) -> dict:
    """Coordinate-descent search; returns {'tuning': ..., 'sources_per_s': ...,
    'default_sources_per_s': ...}.  A candidate replaces the value held only
    when it is faster by more than `min_gain` (a fraction), so timing noise does
    not move the result.  The library tuning is restored to what it was before
    the call."""
    import torch
    cus = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
    sources = np.asarray(sources, dtype=np.int32)
    dev = csr.rowptr.device
    space = dict(space or (MSSSP_SPACE if kind == "msssp" else SSSP_SPACE))
    saved = get_tuning()
    try:
        if kind == "msssp":
            src_t = torch.as_tensor(sources, device=dev)
            kmax = max(space.get("tile_k", [saved["tile_k"]]))
            ws = workspace(tile_bytes(csr.n, csr.m, min(len(sources), kmax)), dev)
            out = torch.empty((len(sources), csr.n), dtype=torch.uint32 if csr.wtype == "u32"
                              else torch.float32, device=dev)

            def call():
                msssp(csr, src_t, out=out, ws=ws, tgraph=tgraph, check=False)
            units = len(sources)
        else:
            ws = workspace(sssp_workspace_bytes(csr.n, csr.m), dev)
            out = torch.empty(csr.n, dtype=torch.uint32 if csr.wtype == "u32" else torch.float32,
                              device=dev)

            def call():
                for s in sources:
                    sssp(csr, int(s), out=out, ws=ws, tgraph=tgraph, check=False)
            units = len(sources)

        set_tuning(reset=True)
        base = get_tuning()
        t_default = _time_calls(call, reps)

        def time_trial(trial):
            set_tuning(reset=True)
            try:
                set_tuning(**_to_tuning(trial, cus))
            except DawnError:
                return None  # a combination the library rejects (t_wave below t_lane)
            t = _time_calls(call, reps)
            if verbose:
                print(f"  {kind} {trial}: {units / t:.1f} sources/s", flush=True)
            return t

        best, best_t = descend(space, base, cus, t_default, time_trial, rounds, min_gain)
        check_runs()
        return {"tuning": _to_tuning(best, cus), "sources_per_s": units / best_t,
                "default_sources_per_s": units / t_default, "kind": kind}
    finally:
        set_tuning(reset=True)
        set_tuning(**saved)


def tune_cached(csr: Csr, sources, kind: str = "msssp", calibration: Csr | None = None,
                force: bool = False, **kw) -> dict:
    """Tuning for `csr` from the cache, or found on `calibration` (a smaller
    graph of the same class, with `sources` valid on it; default: `csr`
    itself) and stored under `csr`'s key."""
    key = f"{device_key()}|{graph_class(csr)}|{csr.wtype}|{kind}"
    cache = _load_cache()
    if key in cache and not force:
        return cache[key]
    target = calibration if calibration is not None else csr
    res = tune(target, sources, kind, **kw)
    res["key"] = key
    res["calibration"] = {"n": target.n, "m": target.m, "class": graph_class(target)}
    cache[key] = res
    _store_cache(cache)
    return res


def apply(result: dict):
    """Set the library tuning to a result of tune()/tune_cached()."""
    set_tuning(reset=True)
    set_tuning(**result["tuning"])
