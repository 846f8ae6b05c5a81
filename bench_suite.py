#!/usr/bin/env python3
"""Measurements of the workloads other than bench.py's headline one.

    python bench_suite.py [--only c1,c2,c3,c4b,c5,hop,mu] [--out results.jsonl]

c1   plain SSSP latency: directed ER n=1000 m=8000, uint32 weights [1,100],
     source 0; per-call latency percentiles (host-observed, with a device
     synchronisation after every call) and steps.
c2   plain single-source GOVM at scale: R-MAT scale 22, edge factor 16, uint32
     weights [1,255], 16 sources one per launch; GTEPS per source, p50/p99,
     the single-source kernel's HBM roofline (algorithmic bytes / kernel time).
c3   high step count: 2048x2048 grid, 1 % of pairs deleted, fp32 weights
     U(0,1], 8 sources; ms per call, steps, ms per step.
c4b  64 uneven ER graphs (n = 10^U(4,6), m = 8n, fp32 lognormal), one source
     each: one persistent launch over the disjoint union, also replayed from a
     captured HIP graph, against 64 plain calls.
c5   serving: Poisson arrivals over 32 resident R-MAT graphs (scales 14 + i%9
     capped at --c5-max-scale, edge factors 8/16/32, half uint32 half fp32
     lognormal); p50/p99 latency and completed queries/s per offered rate.
hop  hop counts (every weight 1, the unweighted case): the C4a graph (R-MAT
     scale 20, edge factor 16) with its 256 sources as one hop-count tile with
     the reverse graph resident; ms per call, GTEPS (reachable edges per
     second, mu = 1), sources/s, two columns checked against BFS, and the
     weighted tile on the same graph and sources for comparison.
mu   the validation experiment of Section 4.2 on synthetic graphs: the same
     topology with fp32 weights all 1.0 and uniform on [0,2]; per graph, the
     share of distance updates beyond the first per reached vertex
     (improvements / reached - 1; 0 at unit weights), mu_e (edges scanned /
     edges reachable), mu_v (rows expanded / vertices reached with out-edges),
     steps, and the time ratio of the two weightings.

Every input is synthetic and seeded (graphgen.workloads).  Each section prints
one JSON line; --out appends them to a file.  Every line carries the SHA-256
of the graph arrays (rowptr, colidx, weights; for several graphs, of their
hashes in order).  Sections c1, c2, c3 and c4b also run a CPU-baseline leg: the
oracle (binary-heap Dijkstra) timed on the host's cores (threads = the CPU
affinity count, one source per thread; the CPU model is printed) over the same
sources, whose distances are then compared element by element with the GPU's
(uint32 bit for bit; fp32 bit for bit against the fp32-fold mode and within
2^-22 * hops * d against the fp64 mode).  c5 compares a sample of the served
queries the same way.  A section whose results differ from the oracle exits
non-zero after printing its line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


FAILURES = []


def threads() -> int:
    return max(1, len(os.sched_getaffinity(0)))


def graphs_sha256(gs) -> str:
    import hashlib
    if len(gs) == 1:
        return gs[0].sha256()
    h = hashlib.sha256()
    for g in gs:
        h.update(g.sha256().encode())
    return h.hexdigest()


def cpu_baseline(g, sources, mode, work_edges=None, what=""):
    """CPU-baseline leg: the oracle's Dijkstra from each source on the host's
    cores (timed), returning the baseline record and the distance arrays."""
    import oracle
    from bench import cpu_model
    r = oracle.time_sources(g, [int(s) for s in sources], threads(), mode, keep=True)
    rec = {"kind": "oracle", "mode": mode, "cores": r["threads"], "cpu_model": cpu_model(),
           "sources": len(sources), "seconds": round(r["seconds"], 3),
           "sources_per_s": round(len(sources) / r["seconds"], 2),
           "sample": f"binary-heap Dijkstra ({mode}) from each of the {len(sources)} sources{what}, "
                     "one source per thread"}
    if work_edges is not None:
        rec["gteps"] = round(work_edges / r["seconds"] / 1e9, 4)
        rec["unit"] = "GTEPS"
    return rec, r["dist"]


def parity(g, s, got, ref_mode_dist=None):
    """Mismatch count of one GPU result against the oracle: uint32 bit for bit;
    fp32 bit for bit against the fp32-fold oracle and within the fp64 tolerance."""
    import numpy as np
    import oracle
    got = np.asarray(got)
    if g.wtype == "u32":
        ref = ref_mode_dist if ref_mode_dist is not None else oracle.sssp(g, s, "u32")[0]
        return int((got.view(np.uint32) != ref).sum())
    d32, _ = oracle.sssp(g, s, "f32fold")
    bad = int((got.view(np.uint32) != d32.view(np.uint32)).sum())
    return bad + int(oracle.f32_tolerance_violations(g, s, got.view(np.float32)).size)


def note_parity(section, bad, checked):
    if bad:
        FAILURES.append(f"{section}: {bad} mismatches over {checked} checked results")
    return {"checked": checked, "mismatched": bad}


def emit(rec, out):
    line = json.dumps(rec)
    print(line, flush=True)
    if out:
        with open(out, "a") as f:
            f.write(line + "\n")


def reach_edges(torch, d, outdeg, inf):
    fin = d != inf
    return int((fin.to(torch.int64) * outdeg).sum().item())


def ss_bytes(info, n):
    """Algorithmic bytes of a single-source run: per edge scanned 8 (column +
    weight) + 4 (target distance); per improvement 4; per frontier row 16
    (queue id, row bounds, own distance); 8 per vertex (init + result)."""
    return (12 * info["edges_scanned"] + 4 * info["improvements"] + 16 * info["frontier_entries"]
            + 8 * n)


def percentile_ms(xs):
    import numpy as np
    a = np.asarray(xs) * 1e3
    return {"p50_ms": float(np.percentile(a, 50)), "p99_ms": float(np.percentile(a, 99)),
            "mean_ms": float(a.mean())}


def c1(args, dawn, torch, np):
    from graphgen import workloads
    g, srcs = workloads.er_small()
    csr = dawn.Csr.from_graph(g)
    out = torch.empty(g.n, dtype=torch.uint32, device="cuda")
    ws = dawn.workspace(dawn.sssp_workspace_bytes(g.n, g.m))
    info = dawn.info_tensor()
    for _ in range(50):
        dawn.sssp(csr, 0, out=out, ws=ws, info=info, check=False)
    torch.cuda.synchronize()
    lat = []
    for _ in range(args.c1_reps):
        t0 = time.perf_counter()
        dawn.sssp(csr, 0, out=out, ws=ws, info=info, check=False)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
    i = dawn.read_info(info)
    got = out.cpu().numpy()
    # CPU-baseline leg: per-call latency of the oracle on one host thread
    import oracle
    clat = []
    for _ in range(args.c1_reps):
        t0 = time.perf_counter()
        ref, _ = oracle.sssp(g, 0, "u32")
        clat.append(time.perf_counter() - t0)
    from bench import cpu_model
    cpu = {"kind": "oracle", "mode": "u32", "cores": 1, "cpu_model": cpu_model(),
           "sample": f"binary-heap Dijkstra from source 0, {args.c1_reps} calls",
           **{k.replace("_ms", "_us"): v * 1e3 for k, v in percentile_ms(clat).items()}}
    rec = {"config": "c1_er_n1000_m8000_u32", "graph_sha256": g.sha256(), "reps": args.c1_reps,
           "steps": i["steps"], "converged": i["converged"],
           "parity": note_parity("c1", int((got != ref).sum()) + (i["converged"] != 1), 1),
           "cpu_baseline": cpu}
    rec.update({k.replace("_ms", "_us"): v * 1e3 for k, v in percentile_ms(lat).items()})
    return rec


def c2(args, dawn, torch, np):
    from graphgen import workloads
    t = time.perf_counter()
    g, srcs = workloads.rmat22(nsrc=args.c2_sources, scale=args.c2_scale)
    log(f"c2 graph n={g.n} m={g.m} ({time.perf_counter() - t:.1f}s)")
    csr = dawn.Csr.from_graph(g)
    tg = dawn.tgraph(csr) if args.c2_tgraph else None
    out = torch.empty(g.n, dtype=torch.uint32, device="cuda")
    ws = dawn.workspace(dawn.sssp_workspace_bytes(g.n, g.m))
    info = dawn.info_tensor()
    outdeg = torch.as_tensor(np.diff(g.rowptr.astype(np.int64)), device="cuda")
    dawn.sssp(csr, int(srcs[0]), out=out, ws=ws, info=info, tgraph=tg, check=False)
    torch.cuda.synchronize()
    per, gteps, mu, steps, kb, kms, reach, got, conv = [], [], [], [], 0, 0.0, [], [], []
    for s in srcs:
        dawn.kernel_timer(True)
        t0 = time.perf_counter()
        dawn.sssp(csr, int(s), out=out, ws=ws, info=info, tgraph=tg, check=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        dawn.kernel_timer(False)
        ms, _ = dawn.kernel_time()
        i = dawn.read_info(info)
        r = reach_edges(torch, out, outdeg, 0xFFFFFFFF)
        per.append(dt)
        reach.append(r)
        gteps.append(r / dt / 1e9)
        mu.append(i["edges_scanned"] / max(r, 1))
        steps.append(i["steps"])
        conv.append(i["converged"])
        kb += ss_bytes(i, g.n)
        kms += ms
        got.append(out.cpu().numpy())
    cpu, dist = cpu_baseline(g, srcs, "u32", sum(reach), " on the same graph")
    bad = sum(int((a != b).sum()) for a, b in zip(got, dist)) + sum(c != 1 for c in conv)
    rec = {"config": f"c2_rmat{args.c2_scale}_ef16_u32_plain", "n": g.n, "m": g.m,
           "graph_sha256": g.sha256(), "reverse_graph": tg is not None,
           "sources": len(srcs), "gteps_per_source_mean": float(np.mean(gteps)),
           "gteps_per_source_min": float(np.min(gteps)), "mu_e_mean": float(np.mean(mu)),
           "steps_mean": float(np.mean(steps)),
           "roofline": {"bound": "hbm",
                        "kernel": ("ss_step_kernel<0, false> (uint32 weights) + "
                                   "ss_persistent_kernel<0> (the steps after the step launches)"
                                   if g.m >= dawn.get_tuning()["step_min_m"]
                                   else "ss_persistent_kernel<0> (uint32 weights)"),
                        "achieved": kb / (kms * 1e-3) / 1e9, "peak": 8000.0, "unit": "GB/s",
                        "frac": kb / (kms * 1e-3) / 1e9 / 8000.0},
           "parity": note_parity("c2", bad, len(srcs)), "cpu_baseline": cpu}
    rec.update(percentile_ms(per))
    return rec


def c3(args, dawn, torch, np):
    from graphgen import workloads
    g, srcs = workloads.grid2048(nsrc=args.c3_sources, side=args.c3_side)
    csr = dawn.Csr.from_graph(g)
    out = torch.empty(g.n, dtype=torch.float32, device="cuda")
    ws = dawn.workspace(dawn.sssp_workspace_bytes(g.n, g.m))
    info = dawn.info_tensor()
    outdeg = torch.as_tensor(np.diff(g.rowptr.astype(np.int64)), device="cuda")
    dawn.sssp(csr, int(srcs[0]), out=out, ws=ws, info=info, check=False)
    torch.cuda.synchronize()
    per, steps, gteps, reach, got, conv = [], [], [], [], [], []
    for s in srcs:
        t0 = time.perf_counter()
        dawn.sssp(csr, int(s), out=out, ws=ws, info=info, check=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        i = dawn.read_info(info)
        fin = torch.isfinite(out)
        r = int((fin.to(torch.int64) * outdeg).sum().item())
        per.append(dt)
        reach.append(r)
        steps.append(i["steps"])
        conv.append(i["converged"])
        gteps.append(r / dt / 1e9)
        got.append(out.cpu().numpy())
    cpu, _ = cpu_baseline(g, srcs, "f64", sum(reach), " (fp64 sums of the fp32 weights)")
    bad = sum(parity(g, int(s), d) for s, d in zip(srcs, got)) + sum(c != 1 for c in conv)
    rec = {"config": f"c3_grid{args.c3_side}_f32", "n": g.n, "m": g.m,
           "graph_sha256": g.sha256(), "sources": len(srcs),
           "steps_mean": float(np.mean(steps)),
           "ms_per_step": float(np.mean([p * 1e3 / s for p, s in zip(per, steps)])),
           "gteps_mean": float(np.mean(gteps)),
           "parity": note_parity("c3", bad, len(srcs)), "cpu_baseline": cpu}
    rec.update(percentile_ms(per))
    # The same sources as one batched call (a tile with one column per
    # source): the sources/s the library gives on this graph.  Every column is
    # compared bit for bit with its source's single-source result (checked
    # against the oracle above).
    src_t = torch.as_tensor(np.asarray(srcs, dtype=np.int32), device="cuda")
    tinfo = dawn.info_tensor()
    tout = dawn.msssp(csr, src_t, info=tinfo, check=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dawn.msssp(csr, src_t, out=tout, info=tinfo, check=False)
    torch.cuda.synchronize()
    t_tile = time.perf_counter() - t0
    ti = dawn.read_info(tinfo)
    tb = tout.cpu().numpy()
    tile_bad = sum(int((tb[j].view(np.uint32) != got[j].view(np.uint32)).sum())
                   for j in range(len(srcs))) + int(ti["converged"] != 1)
    rec["batched"] = {"sources": len(srcs), "ms": t_tile * 1e3, "steps": ti["steps"],
                      "sources_per_s": len(srcs) / t_tile, "gteps": sum(reach) / t_tile / 1e9,
                      "vs_single_source_sources_per_s": (len(srcs) / t_tile) / (len(srcs) / sum(per)),
                      "parity": note_parity("c3 batched", tile_bad, len(srcs))}
    return rec


def c4b(args, dawn, torch, np):
    from graphgen import workloads
    t = time.perf_counter()
    gs = workloads.er_batch(count=args.c4b_graphs)
    log(f"c4b {len(gs)} graphs generated ({time.perf_counter() - t:.1f}s)")
    csrs = [dawn.Csr.from_graph(g) for g, _ in gs]
    b = dawn.Batch(csrs)
    srcs = torch.tensor([s for _, s in gs], dtype=torch.int32, device="cuda")
    out = torch.empty(b.total_n, dtype=torch.float32, device="cuda")
    info = dawn.info_tensor()
    b.run(srcs, out=out, info=info)
    torch.cuda.synchronize()
    reps = args.c4b_reps
    t0 = time.perf_counter()
    for _ in range(reps):
        b.run(srcs, out=out, info=info)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / reps
    i = dawn.read_info(info)
    b.capture(srcs, out, info=info)
    b.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.replay()
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t0) / reps
    # reachable edges per graph, from the batched result
    work = 0
    for (g, _), d in zip(gs, b.split(out)):
        od = torch.as_tensor(np.diff(g.rowptr.astype(np.int64)), device="cuda")
        work += int((torch.isfinite(d).to(torch.int64) * od).sum().item())
    # plain: one call per graph
    wss = [dawn.workspace(dawn.sssp_workspace_bytes(c.n, c.m)) for c in csrs]
    outs = [torch.empty(c.n, dtype=torch.float32, device="cuda") for c in csrs]
    for c, (_, s), w, o in zip(csrs, gs, wss, outs):
        dawn.sssp(c, s, out=o, ws=w, check=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        for c, (_, s), w, o in zip(csrs, gs, wss, outs):
            dawn.sssp(c, s, out=o, ws=w, check=False)
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / reps
    # CPU-baseline leg: the oracle on every graph from its source (fp64 sums);
    # parity of every graph's distances (batched run) with the oracle
    import oracle
    from bench import cpu_model
    got = [d.cpu().numpy() for d in b.split(out)]
    import threading
    lock, nxt, bad = threading.Lock(), [0], [0]

    def worker():
        while True:
            with lock:
                if nxt[0] >= len(gs):
                    return
                j = nxt[0]
                nxt[0] += 1
            oracle.sssp(gs[j][0], gs[j][1], "f64")

    ts = [threading.Thread(target=worker) for _ in range(threads())]
    t0 = time.perf_counter()
    for th in ts:
        th.start()
    for th in ts:
        th.join()
    t_cpu = time.perf_counter() - t0
    for (g, s), d in zip(gs, got):
        bad[0] += parity(g, s, d)
    cpu = {"kind": "oracle", "mode": "f64", "cores": len(ts), "cpu_model": cpu_model(),
           "sample": f"binary-heap Dijkstra (fp64) on each of the {len(gs)} graphs from its source",
           "seconds": round(t_cpu, 3), "graphs_per_s": round(len(gs) / t_cpu, 2),
           "gteps": round(work / t_cpu / 1e9, 4), "unit": "GTEPS"}
    b.close()
    return {"config": f"c4b_er_batch{len(gs)}_f32lognormal", "total_n": b.total_n,
            "graph_sha256": graphs_sha256([g for g, _ in gs]),
            "parity": note_parity("c4b", bad[0] + (i["converged"] != 1), len(gs)),
            "cpu_baseline": cpu,
            "total_m": b.total_m, "steps": i["steps"],
            "batch_ms": t_batch * 1e3, "graph_replay_ms": t_graph * 1e3, "plain_ms": t_plain * 1e3,
            "graphs_per_s_batch": len(gs) / t_batch, "graphs_per_s_replay": len(gs) / t_graph,
            "graphs_per_s_plain": len(gs) / t_plain,
            "aggregate_gteps_batch": work / t_batch / 1e9,
            "aggregate_gteps_plain": work / t_plain / 1e9,
            "edges_scanned": i["edges_scanned"], "mu_e": i["edges_scanned"] / max(work, 1),
            "frontier_entries": i["frontier_entries"], "improvements": i["improvements"]}


def c5(args, dawn, torch, np):
    import graphgen
    from graphgen import workloads
    from paper_2306_07872_amd import serve
    t = time.perf_counter()
    graphs = [workloads.serving_graph(i, args.c5_max_scale) for i in range(args.c5_graphs)]
    log(f"c5 {len(graphs)} graphs ({sum(g.m for g in graphs) / 1e6:.0f}M edges, "
        f"{time.perf_counter() - t:.1f}s)")
    csrs = [dawn.Csr.from_graph(g) for g in graphs]
    src_pool = [graphgen.pick_sources(g, 64, 900 + i) for i, g in enumerate(graphs)]

    def requests(nq, seed):
        u = graphgen.uniform(2 * nq, seed)
        out = []
        for j in range(nq):
            gi = min(int(u[2 * j] * len(graphs)), len(graphs) - 1)
            pool = src_pool[gi]
            out.append((gi, int(pool[min(int(u[2 * j + 1] * len(pool)), len(pool) - 1)])))
        return out

    if args.c5_pull_src is not None:
        dawn.set_tuning(tile_pull_src=args.c5_pull_src)

    def new_server():
        srv = serve.Server(tile_k=args.c5_tile_k, steps_per_tick=args.c5_steps_per_tick,
                           max_tiles_per_graph=2, pull=not args.c5_no_pull,
                           graphs=not args.c5_no_graphs, solo=not args.c5_no_solo)
        for i, c in enumerate(csrs):
            srv.add_graph(i, c)
        return srv

    # closed loop: everything submitted at once -> capacity
    srv = new_server()
    reqs = requests(args.c5_queries, 5)
    warm = [srv.submit(gi, s) for gi, s in reqs[:len(graphs)]]
    srv.run_until_idle()
    t0 = time.perf_counter()
    qs = [srv.submit(gi, s) for gi, s in reqs]
    srv.run_until_idle()
    cap = len(qs) / (time.perf_counter() - t0)
    closed = serve.percentiles([q.latency for q in qs])
    # parity of served queries: every query of the largest graph (scale 22,
    # edge factor 32 when all 32 graphs are served) and of three more graphs,
    # at most args.c5_check in all, against the oracle
    big = max(range(len(graphs)), key=lambda i: graphs[i].m)
    picks = [q for q in qs if q.gid == big][:args.c5_check // 2]
    for gi in (0, len(graphs) // 3, 2 * len(graphs) // 3):
        picks += [q for q in qs if q.gid == gi][:max(1, args.c5_check // 6)]
    bad = sum(parity(graphs[q.gid], q.source, q.result) for q in picks)
    bad += sum(q.state != "done" for q in qs)
    recs = [{"config": "c5_serving_closed_loop", "graphs": len(graphs), "queries": len(qs),
             "graph_sha256": graphs_sha256(graphs),
             "pull": not args.c5_no_pull, "captured_runs": not args.c5_no_graphs,
             "lone_runs": not args.c5_no_solo,
             "capacity_qps": cap, **closed,
             "parity": {**note_parity("c5", bad, len(picks)),
                        "largest_graph": {"id": big, "n": graphs[big].n, "m": graphs[big].m}}}]
    log(f"c5 closed-loop capacity {cap:.1f} queries/s")
    for frac in args.c5_rates:
        rate = frac * cap
        u = graphgen.uniform(args.c5_queries, 17 + int(frac * 100))
        arr = serve.poisson_arrivals(rate, args.c5_queries, u)
        res = serve.serve_open_loop(srv, arr, requests(args.c5_queries, 31 + int(frac * 100)))
        rec = {"config": "c5_serving_poisson", "offered_fraction": frac, "offered_qps": rate, **res}
        log(f"c5 rate {frac:.2f}x: {rec}")
        recs.append(rec)
    srv.close()
    return recs


def hop(args, dawn, torch, np):
    import oracle
    from graphgen import workloads
    g, srcs = workloads.rmat20_tile()
    csr = dawn.Csr.from_graph(g)
    tg = dawn.tgraph(csr)
    k = len(srcs)
    src_t = torch.as_tensor(srcs, dtype=torch.int32, device="cuda")
    out = torch.empty((k, g.n), dtype=torch.uint32, device="cuda")
    ws = dawn.workspace(dawn.umsssp_workspace_bytes(g.n, g.m, k))
    info = dawn.info_tensor()
    dawn.umsssp(csr, src_t, out=out, ws=ws, info=info, tgraph=tg, check=False)
    torch.cuda.synchronize()
    ok = True
    for j in (0, k - 1):
        lv = oracle.bfs(g, int(srcs[j]))
        ref = np.where(lv >= 0, lv, -1).astype(np.int64).astype(np.uint32)
        ok &= bool(np.array_equal(out[j].cpu().numpy(), ref))
    ts = []
    for _ in range(args.hop_reps):
        t0 = time.perf_counter()
        dawn.umsssp(csr, src_t, out=out, ws=ws, info=info, tgraph=tg, check=False)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    i = dawn.read_info(info)
    t = float(np.median(ts))
    wout = torch.empty((k, g.n), dtype=torch.uint32, device="cuda")
    wws = dawn.workspace(dawn.msssp_workspace_bytes(g.n, g.m, k))
    dawn.msssp(csr, src_t, out=wout, ws=wws, tgraph=tg, check=False)
    torch.cuda.synchronize()
    wts = []
    for _ in range(args.hop_reps):
        t0 = time.perf_counter()
        dawn.msssp(csr, src_t, out=wout, ws=wws, tgraph=tg, check=False)
        torch.cuda.synchronize()
        wts.append(time.perf_counter() - t0)
    # mu = 1: the edges scanned are exactly the reachable edges of the sources
    return {"config": "hop_rmat20_ef16_k256", "n": g.n, "m": g.m, "k": k,
            "ms_per_call": t * 1e3, "sources_per_s": k / t, "gteps": i["edges_scanned"] / t / 1e9,
            "steps": i["steps"], "bfs_exact_cols_0_last": ok,
            "weighted_tile_ms_same_sources": float(np.median(wts)) * 1e3}


def seq_alg2(g, srcs, np, order=0):
    """Sequential Algorithm 2 (the oracle's restatement, CPU): mu_e, mu_v, the
    extra updates per reached vertex, and the share of reached vertices whose
    distance was lowered more than once (the paper's re-updated paths)."""
    import oracle
    od = g.outdeg()
    es = rows = mr = rr = reached = imp = multi = steps = 0
    for s in srcs:
        _, c = oracle.govm(g, int(s), order=order, seed=int(s), per_vertex=True)
        reach = oracle.bfs(g, int(s)) >= 0
        es += c["edges_scanned"]
        rows += c["frontier_entries"]
        mr += int(od[reach].sum())
        rr += int((reach & (od > 0)).sum())
        reached += int(reach.sum()) - 1
        imp += c["improvements"]
        multi += int((c["updates"] >= 2).sum())
        steps += c["steps"]
    k = len(srcs)
    return {"order": ["in place, index order", "Jacobi", "in place, random order"][order],
            "mu_e": es / max(mr, 1), "mu_v": rows / max(rr, 1),
            "extra_updates_per_reached": imp / max(reached, 1) - 1.0,
            "share_reached_updated_more_than_once": multi / max(reached, 1),
            "steps_mean": steps / k}


def mu(args, dawn, torch, np):
    """Section 4.2's experiment on synthetic graphs (GPU single-source runs),
    each beside sequential Algorithm 2 on the same sources (CPU), plus the C4a
    tile's mu beside sequential Algorithm 2 for its sources."""
    import graphgen
    from graphgen import workloads
    graphs = [("rmat18_ef16", lambda wk: graphgen.rmat(18, 16, 180, weights=wk)),
              ("er_n262144_m16n", lambda wk: graphgen.er(1 << 18, 16 << 18, 181, weights=wk)),
              ("grid512_1pct", lambda wk: graphgen.grid(512, 512, 0.01, 182, weights=wk))]
    recs = []
    for name, make in graphs:
        row = {"config": f"mu_{name}"}
        for wk in ("f32one", "f32range02"):
            g = make(wk)
            csr = dawn.Csr.from_graph(g)
            out = torch.empty(g.n, dtype=torch.float32, device="cuda")
            ws = dawn.workspace(dawn.sssp_workspace_bytes(g.n, g.m))
            info = dawn.info_tensor()
            outdeg = torch.as_tensor(np.diff(g.rowptr.astype(np.int64)), device="cuda")
            srcs = graphgen.pick_sources(g, args.mu_sources, 7)
            dawn.sssp(csr, int(srcs[0]), out=out, ws=ws, info=info, check=False)
            torch.cuda.synchronize()
            tot = dict(t=0.0, reached=0, reached_rows=0, reach_edges=0, imp=0, rows=0, es=0, steps=0)
            for s in srcs:
                t0 = time.perf_counter()
                dawn.sssp(csr, int(s), out=out, ws=ws, info=info, check=False)
                torch.cuda.synchronize()
                tot["t"] += time.perf_counter() - t0
                i = dawn.read_info(info)
                fin = torch.isfinite(out)
                tot["reached"] += int(fin.sum().item()) - 1
                tot["reached_rows"] += int((fin & (outdeg > 0)).sum().item())
                tot["reach_edges"] += int((fin.to(torch.int64) * outdeg).sum().item())
                tot["imp"] += i["improvements"]
                tot["rows"] += i["frontier_entries"]
                tot["es"] += i["edges_scanned"]
                tot["steps"] += i["steps"]
            k = len(srcs)
            row[wk] = {"graph_sha256": g.sha256(),
                       "gpu": {"extra_updates_per_reached": tot["imp"] / max(tot["reached"], 1) - 1.0,
                               "mu_e": tot["es"] / max(tot["reach_edges"], 1),
                               "mu_v": tot["rows"] / max(tot["reached_rows"], 1),
                               "steps_mean": tot["steps"] / k, "ms_mean": tot["t"] * 1e3 / k},
                       "sequential_alg2": seq_alg2(g, srcs, np)}
        row["time_ratio_range02_over_one"] = (row["f32range02"]["gpu"]["ms_mean"]
                                              / row["f32one"]["gpu"]["ms_mean"])
        log(f"mu {name}: {row}")
        recs.append(row)
    # the C4a tile (R-MAT scale 20, uint32 [1,255]) against sequential Algorithm 2
    g, srcs = workloads.rmat20_tile()
    csr = dawn.Csr.from_graph(g)
    tg = dawn.tgraph(csr)
    info = dawn.info_tensor()
    out = dawn.msssp(csr, srcs, info=info, tgraph=tg)
    i = dawn.read_info(info)
    outdeg = torch.as_tensor(np.diff(g.rowptr.astype(np.int64)), device="cuda")
    work = sum(reach_edges(torch, out[j], outdeg, 0xFFFFFFFF) for j in range(out.shape[0]))
    sub = srcs[:args.mu_sources * 2]
    recs.append({"config": "mu_c4a_rmat20_u32_k256", "graph_sha256": g.sha256(),
                 "gpu_tile": {"mu_e": i["edges_scanned"] / max(work, 1),
                              "extra_updates_per_reached":
                                  i["improvements"] / max(int((out != 0xFFFFFFFF).sum().item())
                                                          - len(srcs), 1) - 1.0,
                              "steps": i["steps"]},
                 "sequential_alg2": [seq_alg2(g, sub, np, order) for order in (0, 1)],
                 "sequential_sources": len(sub)})
    return recs


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--only", default="c1,c2,c3,c4b,c5,hop")
    ap.add_argument("--out", default=None)
    ap.add_argument("--c1-reps", type=int, default=1000)
    ap.add_argument("--c2-scale", type=int, default=22)
    ap.add_argument("--c2-sources", type=int, default=16)
    ap.add_argument("--c2-tgraph", action="store_true",
                    help="keep the reverse graph resident (pull steps per tuning ss_pull)")
    ap.add_argument("--c3-side", type=int, default=2048)
    ap.add_argument("--c3-sources", type=int, default=8)
    ap.add_argument("--c4b-graphs", type=int, default=64)
    ap.add_argument("--c4b-reps", type=int, default=3)
    ap.add_argument("--c5-graphs", type=int, default=32)
    ap.add_argument("--c5-max-scale", type=int, default=22)
    ap.add_argument("--c5-queries", type=int, default=2000)
    ap.add_argument("--c5-tile-k", type=int, default=64)
    ap.add_argument("--c5-no-pull", action="store_true", help="serve with push steps only")
    ap.add_argument("--c5-no-graphs", action="store_true",
                    help="launch each tick's steps one by one instead of replaying a captured run")
    ap.add_argument("--c5-no-solo", action="store_true",
                    help="serve every query from tiles (no lone single-source runs)")
    ap.add_argument("--c5-pull-src", type=int, default=None,
                    help="tuning tile_pull_src while serving (default: the library's)")
    ap.add_argument("--c5-steps-per-tick", type=int, default=4)
    ap.add_argument("--c5-check", type=int, default=24,
                    help="served queries compared with the oracle")
    ap.add_argument("--c5-rates", default="0.1,0.25,0.5,0.7,0.8,0.9,1.0,1.2")
    ap.add_argument("--mu-sources", type=int, default=8)
    ap.add_argument("--hop-reps", type=int, default=5)
    ap.add_argument("--tuning", default=None,
                    help="JSON object of tuning fields applied before every section")
    args = ap.parse_args()
    args.c5_rates = [float(x) for x in args.c5_rates.split(",")]
    import numpy as np
    import torch

    import paper_2306_07872_amd as dawn
    torch.cuda.set_device(0)
    dawn.load()
    if args.tuning:
        dawn.set_tuning(**json.loads(args.tuning))
    for name in args.only.split(","):
        fn = {"c1": c1, "c2": c2, "c3": c3, "c4b": c4b, "c5": c5, "hop": hop, "mu": mu}[name]
        log(f"== {name}")
        t = time.perf_counter()
        recs = fn(args, dawn, torch, np)
        for r in (recs if isinstance(recs, list) else [recs]):
            r["section_s"] = round(time.perf_counter() - t, 1)
            emit(r, args.out)
    if FAILURES:
        log("results differ from the oracle: " + "; ".join(FAILURES))
        return 1
    return 0


if __name__ == "__main__":
    sys.exit(main())
