"""GPU parity of the multi-source tile path (dawn_msssp, dawn_msssp_ws,
dawn_msssp_tg_ws) on the cases Algorithm 2's strict comparison and source
guard must survive: n = 1, m = 0, isolated sources and sources without
out-edges, self-loops with parallel edges, zero-weight edges and zero-weight
cycles (also through the source), uint32 sums at 2^32 - 1 (saturation), fp32
weights with zeros and with increments below half an ulp, ragged n and k,
duplicate sources.  Every column is compared element by element with the
oracle, on every launch path: push steps only, pull steps on every step, the
default density rule, the persistent launch alone, and a mix of one step
launch with the persistent launch."""
import numpy as np
import pytest

import graphgen
from gpu_helpers import announce, assert_sssp_matches, to_np

pytestmark = pytest.mark.gpu

BIG = 0xFFFFFFFF


def _cases(wt):
    """(name, graph, sources) for weight type wt ("u32" or "f32")."""
    dt = np.uint32 if wt == "u32" else np.float32
    E = lambda n, es, name: graphgen.from_edges(  # noqa: E731
        n, [e[0] for e in es], [e[1] for e in es], np.array([e[2] for e in es], dt), wt, name)
    cases = []
    cases.append(("n1", graphgen.from_edges(1, [], [], np.zeros(0, dt), wt), [0, 0, 0]))
    cases.append(("m0", graphgen.from_edges(7, [], [], np.zeros(0, dt), wt), [3, 0, 6, 3]))
    # 3 isolated, 2 has no out-edges
    cases.append(("isolated", E(4, [(0, 1, 3), (1, 2, 4)], "isolated"), [3, 2, 0, 1, 3]))
    cases.append(("selfloop-parallel",
                  E(3, [(0, 0, 1), (0, 1, 9), (0, 1, 4), (1, 1, 0), (1, 2, 2), (2, 2, 5)], "sp"),
                  [0, 1, 2]))
    # zero weights, a zero-weight cycle 1 -> 2 -> 1, and a zero-weight edge
    # back into the source (the candidate 0 is not below the source's 0)
    cases.append(("zero-cycle",
                  E(5, [(0, 1, 0), (1, 2, 0), (2, 1, 0), (2, 3, 0), (0, 3, 1), (3, 0, 0),
                        (3, 4, 2), (4, 4, 0)], "zc"), [0, 1, 3, 4, 2]))
    if wt == "u32":
        # 0 -> 2 sums to 2^32 - 2 (finite); one more unit saturates to INF;
        # 0 -> 1 -> 4 overflows 32 bits and must read INF, not wrap
        cases.append(("saturate",
                      E(5, [(0, 1, BIG - 5), (1, 4, 10), (0, 2, BIG - 1), (2, 3, 1), (1, 2, 7)],
                        "sat"), [0, 1, 2]))
    else:
        # increments below half an ulp of the distance are absorbed by the
        # fp32 add: 1 + 2^-30 == 1, so the longer path never improves
        tiny = np.float32(2.0 ** -30)
        cases.append(("absorbed",
                      graphgen.from_edges(4, [0, 1, 0, 2], [1, 2, 2, 3],
                                          np.array([1.0, tiny, 1.0, tiny], np.float32), "f32",
                                          "abs"), [0, 1]))
    kind = "u32" if wt == "u32" else "f32range02"   # f32: U[0,2] including zeros
    g = graphgen.er(1001, 7003, 4, weights=kind, wlo=0, whi=3) if wt == "u32" else \
        graphgen.er(1001, 7003, 4, weights=kind)
    cases.append(("ragged-er", g, list(graphgen.pick_sources(g, 37, 5)) + [1000, 0, 0]))
    # hubs with more than 1024 in-edges (pull chunks of one target combined
    # with atomics) and many zero-weight ties
    g = graphgen.rmat(12, 16, 31, weights="u32", wlo=0, whi=2) if wt == "u32" else \
        graphgen.rmat(12, 16, 31, weights="f32range02")
    cases.append(("rmat12-ties", g, list(graphgen.pick_sources(g, 130, 6))))
    return cases


# launch paths of the tile: (name, tuning, use the reverse graph, use _ws with info)
PATHS = [
    ("push", dict(), False, False),
    ("push-ws", dict(), False, True),
    ("pull-every-step", dict(tile_pull=0, tile_pull_src=0, tile_step_launches=4096), True, True),
    ("pull-default", dict(), True, False),
    ("persistent", dict(mode=2), False, True),
    ("pull-then-persistent", dict(tile_pull=0, tile_pull_src=0, tile_step_launches=1), True, True),
    ("tile64-sparse", dict(tile_k=64, tile_sparse=512, tile_t_wave=32, tile_t_chunk=64), True,
     True),
]


@pytest.mark.parametrize("pi", range(len(PATHS)))
@pytest.mark.parametrize("wt", ["u32", "f32"])
def test_tile_edge_cases_match_oracle(dawn, wt, pi):
    import torch
    name_p, tune, use_tg, use_ws = PATHS[pi]
    prev = dawn.set_tuning(**tune) if tune else None
    try:
        for name, g, srcs in _cases(wt):
            srcs = np.asarray(srcs, dtype=np.int32)
            announce("tile edge", wt, name_p, name, "n", g.n, "m", g.m, "k", len(srcs))
            csr = dawn.Csr.from_graph(g)
            tg = dawn.tgraph(csr) if use_tg else None
            info = dawn.info_tensor() if use_ws else None
            D = dawn.msssp(csr, srcs, info=info, tgraph=tg)   # raises unless converged
            torch.cuda.synchronize()
            D = to_np(D)
            assert D.shape == (len(srcs), g.n)
            for j, s in enumerate(srcs):
                assert_sssp_matches(g, int(s), D[j], tag=f"{name_p} {name} col {j}")
            if info is not None:
                assert dawn.read_info(info)["converged"] == 1
    finally:
        if prev is not None:
            dawn.set_tuning(**prev)


def test_apsp_edge_graphs(dawn):
    import torch
    for wt in ("u32", "f32"):
        for name, g, _ in _cases(wt)[:6]:
            announce("apsp edge", wt, name)
            A = to_np(dawn.apsp(dawn.Csr.from_graph(g)))
            torch.cuda.synchronize()
            for s in range(g.n):
                assert_sssp_matches(g, s, A[s], tag=f"apsp {name} row {s}")


@pytest.mark.parametrize("bad", ["n", "neg"])
def test_msssp_bad_device_source_is_reported(dawn, bad):
    """A source id outside [0, n) can only be seen on the device: the tile
    ends before its first step and the call reports it (converged = -1 in the
    run info; a plain call raises through the run-status record)."""
    import torch
    g = graphgen.rmat(9, 8, 3, weights="u32")
    csr = dawn.Csr.from_graph(g)
    b = g.n if bad == "n" else -1
    srcs = np.array([0, 5, b, 7], np.int32)
    announce("msssp bad source", b)
    with pytest.raises(dawn.DawnError) as e:
        dawn.msssp(csr, srcs)
    assert e.value.status == dawn.E_INCOMPLETE
    info = dawn.info_tensor()
    dawn.msssp(csr, srcs, info=info, check=False)
    torch.cuda.synchronize()
    assert dawn.read_info(info)["converged"] == -1
    assert dawn.run_status() == (0, 1)   # runs with run info leave the record alone
    # the record does not outlive the failure: a good call passes
    D = to_np(dawn.msssp(csr, np.array([0, 5], np.int32)))
    assert_sssp_matches(g, 5, D[1], tag="after bad source")
