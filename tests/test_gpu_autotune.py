"""The autotuner runs the real HIP path, never changes results, and caches."""
import json
import os

import numpy as np
import pytest

import graphgen
from gpu_helpers import announce, to_np

pytestmark = pytest.mark.gpu


def test_autotune_keeps_results_and_caches(dawn, tmp_path, monkeypatch):
    import torch
    from paper_2306_07872_amd import autotune
    monkeypatch.setenv("DAWN_TUNE_CACHE", str(tmp_path / "tune.json"))
    g = graphgen.rmat(13, 16, 77, weights="u32")
    csr = dawn.Csr.from_graph(g)
    srcs = graphgen.pick_sources(g, 96, 1)
    base = to_np(dawn.msssp(csr, srcs))
    base1 = to_np(dawn.sssp(csr, int(srcs[0])))
    torch.cuda.synchronize()
    announce("autotune msssp")
    small = {"tile_k": [64, 128], "grid_per_cu": [8, 16], "tile_t_wave": [32, 256]}
    r = autotune.tune_cached(csr, srcs, "msssp", space=small, reps=1)
    assert r["sources_per_s"] > 0 and "tile_k" in r["tuning"]
    assert json.load(open(tmp_path / "tune.json"))[r["key"]]["tuning"] == r["tuning"]
    prev = dawn.get_tuning()
    autotune.apply(r)
    tuned = to_np(dawn.msssp(csr, srcs))
    torch.cuda.synchronize()
    assert np.array_equal(tuned.view(np.uint32), base.view(np.uint32))
    announce("autotune sssp")
    r1 = autotune.tune_cached(csr, srcs[:4], "sssp", space={"wg_threads": [256, 1024], "mode": [1, 2]},
                              reps=1)
    autotune.apply(r1)
    d1 = to_np(dawn.sssp(csr, int(srcs[0])))
    torch.cuda.synchronize()
    assert np.array_equal(d1.view(np.uint32), base1.view(np.uint32))
    # a second call is served from the cache
    again = autotune.tune_cached(csr, srcs, "msssp", space=small, reps=1)
    assert again == json.load(open(tmp_path / "tune.json"))[r["key"]]
    dawn.set_tuning(reset=True)
    dawn.set_tuning(**prev)
