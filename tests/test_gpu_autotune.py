"""The autotuner runs the real HIP path, never changes results (checked
against the oracle), and caches."""
import json

import numpy as np
import pytest

import graphgen
import oracle
from gpu_helpers import announce, assert_sssp_matches, to_np

pytestmark = pytest.mark.gpu


def test_autotune_keeps_results_and_caches(dawn, tmp_path, monkeypatch):
    import torch
    from paper_2306_07872_amd import autotune
    monkeypatch.setenv("DAWN_TUNE_CACHE", str(tmp_path / "tune.json"))
    g = graphgen.rmat(13, 16, 77, weights="u32")
    csr = dawn.Csr.from_graph(g)
    srcs = graphgen.pick_sources(g, 96, 1)
    prev = dawn.get_tuning()
    try:
        announce("autotune msssp")
        small = {"tile_k": [64, 128], "grid_per_cu": [8, 16], "tile_t_wave": [32, 256],
                 "tile_pull": [0, 1001]}
        # min_gain = -1: every field takes its fastest candidate, so the tuning
        # checked below is one the search chose, not the defaults
        r = autotune.tune_cached(csr, srcs, "msssp", space=small, reps=1, min_gain=-1.0,
                                 tgraph=dawn.tgraph(csr))
        assert r["sources_per_s"] > 0
        assert {"tile_k", "grid", "tile_t_wave", "tile_pull"} == set(r["tuning"])
        assert json.load(open(tmp_path / "tune.json"))[r["key"]]["tuning"] == r["tuning"]
        autotune.apply(r)
        tuned = to_np(dawn.msssp(csr, srcs, tgraph=dawn.tgraph(csr)))
        torch.cuda.synchronize()
        for j in range(0, len(srcs), 7):
            assert_sssp_matches(g, int(srcs[j]), tuned[j], tag=f"tuned msssp col {j}")
        announce("autotune sssp")
        r1 = autotune.tune_cached(csr, srcs[:4], "sssp",
                                  space={"wg_threads": [256, 1024], "mode": [1, 2]}, reps=1,
                                  min_gain=-1.0)
        assert {"wg_threads", "mode"} == set(r1["tuning"])
        autotune.apply(r1)
        for s in srcs[:3]:
            d1 = to_np(dawn.sssp(csr, int(s)))
            ref, _ = oracle.sssp(g, int(s), "u32")
            assert np.array_equal(d1.view(np.uint32), ref)
        # a second call is served from the cache
        again = autotune.tune_cached(csr, srcs, "msssp", space=small, reps=1, min_gain=-1.0)
        assert again == json.load(open(tmp_path / "tune.json"))[r["key"]]
    finally:
        dawn.set_tuning(reset=True)
        dawn.set_tuning(**prev)
