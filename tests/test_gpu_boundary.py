"""The C ABI's run contract on the GPU: calls enqueue work and return without
waiting on the host, multi-source runs can be captured into a HIP graph and
replayed, runs that end without converging are reported (never returned as
ordinary distances), persistent grids fit what the compute units hold, and
tile sessions live in caller-owned memory."""
import time

import numpy as np
import pytest

import graphgen
import oracle
from gpu_helpers import announce, assert_sssp_matches, to_np

pytestmark = pytest.mark.gpu


_CYCLES_PER_MS = []


def _sleep_stream(torch, ms):
    """Occupy the current stream for about `ms` milliseconds (a bounded spin
    kernel, calibrated once), so that a call that waited for the device would
    be seen waiting."""
    if not _CYCLES_PER_MS:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        torch.cuda._sleep(50_000_000)
        torch.cuda.synchronize()
        dt = max(time.perf_counter() - t0, 1e-4)
        _CYCLES_PER_MS.append(50_000_000 / (dt * 1e3))
    torch.cuda._sleep(int(min(ms * _CYCLES_PER_MS[0], 4e10)))


@pytest.mark.parametrize("what", ["msssp", "msssp_tg", "sssp_steps", "umsssp", "apsp"])
def test_calls_do_not_wait_on_the_host(dawn, what):
    import torch
    if not hasattr(torch.cuda, "_sleep"):
        pytest.skip("torch.cuda._sleep unavailable")
    g = graphgen.rmat(14, 16, 41, weights="u32")
    csr = dawn.Csr.from_graph(g)
    tg = dawn.tgraph(csr)
    srcs = graphgen.pick_sources(g, 100, 2)
    src_t = torch.as_tensor(srcs, dtype=torch.int32, device="cuda")
    prev = dawn.set_tuning(small_m=0, step_min_m=0)   # single source: step launches first
    try:
        # warm everything up (allocator, module load, reverse graph)
        dawn.msssp(csr, src_t, tgraph=tg)
        dawn.sssp(csr, int(srcs[0]))
        dawn.umsssp(csr, src_t)
        csr_small = dawn.Csr.from_graph(graphgen.er(300, 2000, 4, weights="u32"))
        dawn.apsp(csr_small)
        torch.cuda.synchronize()
        announce("no host wait", what)
        _sleep_stream(torch, 400)
        t0 = time.perf_counter()
        if what == "msssp":
            out = dawn.msssp(csr, src_t, check=False)
        elif what == "msssp_tg":
            out = dawn.msssp(csr, src_t, tgraph=tg, check=False)
        elif what == "sssp_steps":
            out = dawn.sssp(csr, int(srcs[3]), check=False)
        elif what == "umsssp":
            out = dawn.umsssp(csr, src_t, check=False)
        else:
            out = dawn.apsp(csr_small, check=False)
        t_call = time.perf_counter() - t0
        torch.cuda.synchronize()
        t_all = time.perf_counter() - t0
        assert t_all > 0.3, "the spin kernel did not hold the stream"
        assert t_call < 0.1 * t_all, f"call took {t_call:.3f}s of {t_all:.3f}s: it waited"
        dawn.check_runs()
        if what in ("msssp", "msssp_tg"):
            assert_sssp_matches(g, int(srcs[7]), to_np(out)[7], tag=what)
    finally:
        dawn.set_tuning(**prev)


@pytest.mark.parametrize("use_tg", [False, True])
@pytest.mark.parametrize("wk", ["u32", "f32lognormal"])
def test_msssp_capture_replay_with_new_sources(dawn, wk, use_tg):
    """dawn_msssp_ws / dawn_msssp_tg_ws captured once into a HIP graph; each
    replay reads new source ids from the captured buffer and matches a fresh
    eager run and the oracle, with unrelated eager work between replays."""
    import torch
    g = graphgen.rmat(13, 16, 52, weights=wk)
    csr = dawn.Csr.from_graph(g)
    tg = dawn.tgraph(csr) if use_tg else None
    k = 96
    src_t = torch.as_tensor(graphgen.pick_sources(g, k, 1), dtype=torch.int32, device="cuda")
    out = torch.empty((k, g.n), dtype=dawn.dist_dtype(g.wtype), device="cuda")
    ws = dawn.workspace(dawn.msssp_workspace_bytes(g.n, g.m, k))
    info = dawn.info_tensor()
    dawn.msssp(csr, src_t, out=out, ws=ws, info=info, tgraph=tg)   # eager warm-up
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    announce("msssp capture", wk, "tgraph", use_tg)
    with torch.cuda.graph(graph, stream=s):
        dawn.msssp(csr, src_t, out=out, ws=ws, info=info, tgraph=tg, check=False)
    for rep in range(4):
        new = graphgen.pick_sources(g, k, 10 + rep)
        src_t.copy_(torch.as_tensor(new, dtype=torch.int32))
        graph.replay()
        torch.cuda.synchronize()
        got = to_np(out).copy()
        assert dawn.read_info(info)["converged"] == 1
        eager = to_np(dawn.msssp(csr, new, tgraph=tg))
        junk = torch.randn(4096, device="cuda").sum()   # unrelated eager work
        torch.cuda.synchronize()
        del junk
        assert np.array_equal(got.view(np.uint32), eager.view(np.uint32)), f"replay {rep}"
        for j in (0, 41, k - 1):
            assert_sssp_matches(g, int(new[j]), got[j], tag=f"replay {rep} col {j}",
                                check_invariants=False)


# persistent launches whose grid barriers give up at the first wait
# (barrier_ms = 0): every kernel still exits, and the run is reported
ABORT_CASES = ["sssp", "msssp", "umsssp", "batch"]


@pytest.mark.parametrize("what", ABORT_CASES)
def test_barrier_give_up_is_reported_not_returned(dawn, what):
    import torch
    g = graphgen.rmat(12, 16, 61, weights="u32")
    csr = dawn.Csr.from_graph(g)
    srcs = graphgen.pick_sources(g, 64, 3)

    def run(info=None, check=True):
        if what == "sssp":
            return dawn.sssp(csr, int(srcs[0]), info=info, check=check)
        if what == "msssp":
            return dawn.msssp(csr, srcs, info=info, check=check)
        if what == "umsssp":
            return dawn.umsssp(csr, srcs, info=info, check=check)
        b = dawn.Batch([csr, dawn.Csr.from_graph(graphgen.er(3000, 24000, 2, weights="u32"))])
        o = b.run(torch.tensor([int(srcs[0]), 5], dtype=torch.int32, device="cuda"), info=info)
        if check:
            if info is None:
                dawn.check_runs()
            else:
                dawn._check_info(info)
        b.close()
        return o

    tune = dict(small_m=0, mode=2, barrier_ms=0)
    if what == "umsssp":
        tune = dict(tile_step_launches=0, barrier_ms=0)
    prev = dawn.set_tuning(**tune)
    try:
        announce("barrier give-up", what)
        with pytest.raises(dawn.DawnError) as e:
            run()
        assert e.value.status == dawn.E_INCOMPLETE and "-2" in str(e.value)
        info = dawn.info_tensor()
        run(info=info, check=False)
        torch.cuda.synchronize()
        assert dawn.read_info(info)["converged"] == -2
    finally:
        dawn.set_tuning(**prev)
    # every kernel exited: the same run with the normal bound converges
    prev = dawn.set_tuning(**{k: v for k, v in tune.items() if k != "barrier_ms"})
    try:
        info = dawn.info_tensor()
        out = run(info=info)
        torch.cuda.synchronize()
        assert dawn.read_info(info)["converged"] == 1
        if what == "sssp":
            assert_sssp_matches(g, int(srcs[0]), to_np(out), tag="after give-up")
    finally:
        dawn.set_tuning(**prev)


def residency_rule(vgprs: int, lds: int, threads: int) -> int:
    """Workgroups per gfx950 CU (restated from dawn_api.hip's rule)."""
    if vgprs <= 0:
        return 0
    waves = (threads + 63) // 64
    per_simd = (waves + 3) // 4
    alloc = max(8, (vgprs + 7) // 8 * 8)
    by_regs = min(8, 512 // alloc) // per_simd
    by_lds = 160 * 1024 // lds if lds > 0 else 16
    return max(0, min(by_regs, by_lds, 16))


@pytest.mark.parametrize("threads", [0, 256, 512, 1024])
def test_persistent_grids_follow_the_residency_rule(dawn, threads):
    prev = dawn.set_tuning(wg_threads=threads)
    try:
        q = dawn.device_query()
    finally:
        dawn.set_tuning(**prev)
    assert q["cus"] >= 1
    ss_t = threads or 1024
    tile_t = threads or 1024
    for key, vg, lds, api, t in (("ss", q["ss_vgprs"], q["ss_lds"], q["ss_api_blocks_per_cu"], ss_t),
                                 ("tile", q["tile_vgprs"], q["tile_lds"],
                                  q["tile_api_blocks_per_cu"], tile_t)):
        rule = residency_rule(vg, lds, t)
        exp = max(1, min(rule, api) if api > 0 else rule)
        assert q[f"{key}_blocks_per_cu"] == exp, (key, q)
        assert q[f"{key}_grid"] == exp * q["cus"]
        assert 0 < vg <= 512 and lds > 0


def test_tile_session_in_caller_memory(dawn):
    """A tile session runs in a workspace the caller owns; destroying the
    session leaves the buffer to the caller."""
    import torch
    g = graphgen.rmat(11, 16, 71, weights="u32")
    csr = dawn.Csr.from_graph(g)
    buf = dawn.workspace(dawn.tile_bytes(g.n, g.m, 64))
    tile = dawn.Tile(csr, 64, ws=buf)
    srcs = graphgen.pick_sources(g, 3, 2)
    for c, s in enumerate(srcs):
        tile.admit(c, int(s))
    for _ in range(200):
        done = tile.run(8)
        torch.cuda.synchronize()
        if set(range(3)) <= set(dawn.done_columns(done.cpu().numpy(), tile.k)):
            break
    for c, s in enumerate(srcs):
        ref, _ = oracle.sssp(g, int(s), "u32")
        assert np.array_equal(to_np(tile.read(c)).view(np.uint32), ref)
    tile.close()
    buf.fill_(7)   # still the caller's memory
    torch.cuda.synchronize()
    assert int(buf[0].item()) == 7
    with pytest.raises(dawn.DawnError):
        dawn.Tile(csr, 64, ws=dawn.workspace(1000))
