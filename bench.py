#!/usr/bin/env python3
"""Benchmark of batched multi-source GOVM against plain single-source GOVM.

Workload (default): directed R-MAT, scale 20 (1,048,576 vertices), edge
factor 16, a=0.57 b=0.19 c=0.19, uint32 weights uniform in [1,255]; 256
distinct sources run as one [n x 256] distance tile per step.

One "step" = one dawn_msssp call over the 256 sources: tile reset, seeding,
every GOVM step until no source changes, and the transposed store of the
[256 x n] result.  The graph and sources are resident in HBM before timing.

Printed: ONE JSON line.  value = aggregate GTEPS of the batched call
(sum over sources of the edges reachable from the source, divided by the
wall time of a step).  Also: sources/s batched and plain, their ratio, the
roofline of the dominant kernel (the tile's relaxation kernel, timed with HIP
events on its launch stream) and the CPU oracle's rate on a bounded sample of
the same sources.

roofline.traffic is the relaxation kernel's measured HBM bytes per launch
(rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by what the counters read for a
copy of known size), read from the committed counter summary under
profiles/; it is reported only while the kernel sources, the tuning and the
workload are the ones the counters were taken with, and is null otherwise.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "tile_step_kernel_rmat20_k256_traffic.md")
# every source that shapes the relaxation kernels or their launches (grids,
# launch sequence, tile layout)
KERNEL_SOURCES = ("paper_2306_07872_amd/csrc/govm_tile.hip",
                  "paper_2306_07872_amd/csrc/govm_device.hpp",
                  "paper_2306_07872_amd/csrc/govm_host.hpp",
                  "paper_2306_07872_amd/csrc/dawn_api.hip")


def kernel_sources_sha256() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


# tuning fields that shape the tile's launches (the others only concern
# single-source runs)
TILE_TUNING_KEYS = ("wg_threads", "grid", "mode", "tile_step_launches", "tile_k", "tile_t_wave",
                    "tile_t_chunk", "tile_t_group", "tile_skip", "tile_sparse")


def measured_traffic(tuning: dict, workload: str):
    """HBM bytes per relaxation launch from the committed counter summary, or
    None when it was taken with other kernel sources, tile tuning or workload."""
    try:
        with open(TRAFFIC_SUMMARY) as f:
            text = f.read()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            fields[k.strip("`")] = v.strip().strip("`")
    try:
        taken = json.loads(fields["tuning"])
        if (fields["kernel_sources_sha256"] != kernel_sources_sha256()
                or any(taken.get(k) != tuning.get(k) for k in TILE_TUNING_KEYS)
                or fields["workload"] != workload):
            return None
        return int(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model() -> str:
    """The host CPU's model name (lscpu, else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def reach_edges(torch, dist, outdeg, inf):
    """Sum of out-degrees over vertices each row of `dist` reaches (finite)."""
    tot = []
    for r0 in range(0, dist.shape[0], 32):
        blk = dist[r0:r0 + 32]
        fin = blk != inf
        tot.append((fin.to(torch.int64) * outdeg).sum(dim=1))
    return torch.cat(tot).cpu().tolist()


def tile_kernel_bytes(info: dict, nseg: int, skip: bool) -> int:
    """Algorithmic bytes of the tile's relaxation kernel over one call.

    per union-frontier row: row bounds 8 B + queue id 4 B + its mask words read
      and cleared, 2 * 8 B per 64-source segment (3 * 8 B when the next-step
      mask is read to skip pairs already lowered again);
    per active (row, source): the source's distance at the row, 4 B;
    per union edge: column id + weight, 8 B;
    per active (edge, source): the target's distance, 4 B;
    per improvement: the new distance, 4 B."""
    per_row = 12 + (24 if skip else 16) * nseg
    return (info["union_rows"] * per_row + 4 * info["frontier_entries"]
            + 8 * info["union_edges"] + 4 * info["edges_scanned"] + 4 * info["improvements"])


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=int, default=20)
    ap.add_argument("--k", type=int, default=256)
    ap.add_argument("--plain", type=int, default=256, help="sources timed one per launch")
    ap.add_argument("--cpu-sample", type=int, default=256, help="sources timed on the oracle")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-pull", action="store_true",
                    help="no reverse graph: every tile step pushes")
    ap.add_argument("--tune", action="append", default=[], metavar="KEY=VALUE",
                    help="library tuning field (see dawn_tuning), repeatable; implies "
                         "--no-autotune")
    ap.add_argument("--no-autotune", action="store_true",
                    help="run the library's default tuning only (no autotuner)")
    ap.add_argument("--calibration-scale", type=int, default=18,
                    help="R-MAT scale of the autotuner's calibration graph (same generator, "
                         "edge factor and weights as the workload)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run a plain device-to-device copy of this many MiB (a kernel "
                         "of known traffic, to scale profiler byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "design (sources sharded across GPUs) is not part of this build.", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2306_07872_amd as dawn
    from graphgen import workloads

    torch.cuda.set_device(0)
    dawn.load()
    if args.tune:
        dawn.set_tuning(**{k: int(v) for k, v in (t.split("=", 1) for t in args.tune)})
    if args.copy_calibration > 0:
        nel = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(nel, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_calibration} MiB read + {args.copy_calibration} MiB written")
        del a, b
        # a gather of known bytes, shaped like the tile's pull steps: distinct
        # random 1 KiB rows (256 uint32) of a table of `copy_calibration` MiB
        rows = args.copy_calibration * 1024
        src = torch.ones((rows, 256), dtype=torch.int32, device="cuda")
        g = torch.Generator(device="cuda")
        g.manual_seed(7)
        idx = torch.randperm(rows, device="cuda", generator=g)[:rows // 4]
        torch.cuda.synchronize()
        dst = torch.index_select(src, 0, idx)
        torch.cuda.synchronize()
        log(f"gather calibration: {rows // 4} distinct random 1 KiB rows: "
            f"{rows // 4 / 1024:.0f} MiB of rows + {idx.numel() * 8 / 2**20:.1f} MiB of indices "
            f"read, {rows // 4 / 1024:.0f} MiB written")
        del src, idx, dst
    t_gen = time.perf_counter()
    g, srcs = workloads.rmat20_tile(k=args.k, scale=args.scale)
    log(f"graph {g.name}: n={g.n} m={g.m} k={len(srcs)} ({time.perf_counter() - t_gen:.1f}s)")
    csr = dawn.Csr.from_graph(g)
    # the reverse graph for pull steps: built once per graph, like the CSR
    tg = None
    t_tg = 0.0
    if not args.no_pull:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tg = dawn.tgraph(csr)
        torch.cuda.synchronize()
        t_tg = time.perf_counter() - t0
        log(f"reverse graph built in {t_tg * 1e3:.1f} ms")
    src_t = torch.as_tensor(srcs, dtype=torch.int32, device="cuda")
    k = int(src_t.numel())
    out = torch.empty((k, g.n), dtype=torch.uint32, device="cuda")
    info = dawn.info_tensor()

    # ---- autotuner: launch parameters found on a calibration graph of the same
    # class (R-MAT, edge factor 16, uint32 [1,255], a smaller scale), applied
    # to the workload; the default tuning is timed beside it
    autotuned = None
    if not args.no_autotune and not args.tune:
        import tempfile

        from paper_2306_07872_amd import autotune
        cache_dir = tempfile.mkdtemp(prefix="dawn_tune_")
        os.environ.setdefault("DAWN_TUNE_CACHE", os.path.join(cache_dir, "tune.json"))
        gc, sc = workloads.rmat20_tile(seed=18, k=args.k, scale=args.calibration_scale)
        cal = dawn.Csr.from_graph(gc)
        tgc = dawn.tgraph(cal) if tg is not None else None
        t_tune = time.perf_counter()
        autotuned = autotune.tune_cached(csr, sc, "msssp", calibration=cal, tgraph=tgc, reps=3)
        t_tune = time.perf_counter() - t_tune
        log(f"autotune ({t_tune:.1f}s) key {autotuned['key']}: {autotuned['tuning']} "
            f"({autotuned['sources_per_s']:.0f} vs default "
            f"{autotuned['default_sources_per_s']:.0f} sources/s on the calibration graph)")
        del cal, tgc

    def timed(label):
        """Warmup, then the timed steps of the batched call; kernel events on."""
        for _ in range(args.warmup):
            dawn.msssp(csr, src_t, out=out, ws=ws, info=info, tgraph=tg, check=False)
        torch.cuda.synchronize()
        dawn.kernel_timer(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            dawn.msssp(csr, src_t, out=out, ws=ws, info=info, tgraph=tg, check=False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        dawn.kernel_timer(False)
        k_ms, k_launches = dawn.kernel_time()
        inf = dawn.read_info(info)
        ms = (t1 - t0) * 1e3 / args.steps
        log(f"batched ({label}): {ms:.3f} ms/step, kernel {k_ms / max(k_launches, 1):.3f} "
            f"ms/launch, info {inf}")
        return ms, k_ms, k_launches, inf

    default_ms = None
    if autotuned is not None:
        dawn.set_tuning(reset=True)
        ws = dawn.workspace(dawn.msssp_workspace_bytes(g.n, g.m, k))
        default_ms, _, _, dinf = timed("default tuning")
        if dinf["converged"] != 1:
            log(f"batched run did not converge (status {dinf['converged']})")
            return 1
        autotune.apply(autotuned)
    tune = dawn.get_tuning()
    ws = dawn.workspace(dawn.msssp_workspace_bytes(g.n, g.m, k))
    ms_step, k_ms, k_launches, inf = timed("autotuned" if autotuned is not None else "as set")
    if inf["converged"] != 1:
        log(f"batched run did not converge (status {inf['converged']}): no figure is reported")
        return 1
    log(f"batched: {ms_step:.3f} ms/step, kernel {k_ms / max(k_launches, 1):.3f} ms/launch, "
        f"info {inf}")

    outdeg = torch.as_tensor(np.diff(g.rowptr.astype(np.int64)), device="cuda")
    reach = reach_edges(torch, out, outdeg, 0xFFFFFFFF)
    work = float(sum(reach))
    gteps = work / (ms_step * 1e-3) / 1e9
    srcs_per_s = k / (ms_step * 1e-3)

    # ---- plain single-source on the same sources ------------------------------
    nplain = min(args.plain, k)
    plain_s, plain_gteps = float("nan"), float("nan")
    if nplain > 0:
        out1 = torch.empty(g.n, dtype=torch.uint32, device="cuda")
        ws1 = dawn.workspace(dawn.sssp_workspace_bytes(g.n, g.m))
        for s in srcs[:3]:
            dawn.sssp(csr, int(s), out=out1, ws=ws1, check=False)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for s in srcs[:nplain]:
            dawn.sssp(csr, int(s), out=out1, ws=ws1, check=False)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        dawn.check_runs()   # every plain run converged
        plain_s = (t3 - t2) / nplain
        plain_gteps = float(sum(reach[:nplain])) / (t3 - t2) / 1e9
        log(f"plain: {plain_s * 1e3:.3f} ms/source ({nplain} sources)")

    # ---- roofline of the dominant kernel -------------------------------------
    # The tile's GOVM step kernel: every launch the kernel timer recorded during
    # the K timed calls (events on the launch stream).  Algorithmic bytes come
    # from the device counters of the last call; every call does the same work
    # up to the order of updates inside a step.
    nseg = (min(k, tune["tile_k"]) + 63) // 64
    kbytes_call = tile_kernel_bytes(inf, nseg, bool(tune["tile_skip"]))
    avg_kms = k_ms / max(k_launches, 1)
    per_launch_bytes = kbytes_call * args.steps / max(k_launches, 1)
    achieved = per_launch_bytes / (avg_kms * 1e-3) / 1e9
    if tune["mode"] == 2:
        kname = "tile_persistent_kernel<false>"
    elif tg is not None:
        kname = "tile relaxation: tile_step_kernel<false> (push steps) + tile_pull_kernel<false> (pull steps)"
    else:
        kname = "tile_step_kernel<false>"
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(tune, f"rmat{args.scale}_ef16_u32_k{k}"),
                "kernel": kname, "kernel_ms": round(avg_kms, 5),
                "launches_per_step": round(k_launches / args.steps, 2),
                "algorithmic_bytes": int(per_launch_bytes),
                "algorithmic_bytes_per_call": int(kbytes_call)}

    # ---- CPU oracle on a bounded sample ---------------------------------------
    # The oracle (binary-heap Dijkstra) is timed on the first cpu_sample sources;
    # its distances are then compared with the GPU's columns of those sources,
    # element by element, after the timed region.
    cpu = None
    if not args.no_cpu:
        import oracle
        threads = max(1, len(os.sched_getaffinity(0)))
        sample = [int(s) for s in srcs[:args.cpu_sample]]
        r = oracle.time_sources(g, sample, threads, "u32", keep=True)
        sw = float(sum(reach[:len(sample)]))
        host = out[:len(sample)].cpu().numpy()
        bad = [j for j, d in enumerate(r["dist"]) if not np.array_equal(host[j], d)]
        cpu = {"value": round(sw / r["seconds"] / 1e9, 4), "unit": "GTEPS", "cores": r["threads"],
               "kind": "oracle",
               "sample": f"binary-heap Dijkstra (uint64 sums) from the first {len(sample)} of the "
                         f"{k} sources on the same graph, one source per thread",
               "cpu_model": cpu_model(),
               "sources_per_s": round(len(sample) / r["seconds"], 2),
               "seconds": round(r["seconds"], 2),
               "columns_checked": len(sample), "columns_mismatched": len(bad)}
        log(f"cpu oracle: {cpu}")
        if bad:
            log(f"GPU columns {bad[:8]} differ from the oracle: no figure is reported")
            return 1

    res = {
        "metric": "GTEPS & sources/s, batched k-source GOVM vs plain 1-source GOVM; p50/p99 query ms",
        "value": round(gteps, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"rmat{args.scale}_ef16_u32_k{k}", "n": g.n, "m": g.m, "k": k,
                   "weights": "uint32 uniform [1,255]", "sources": "uniform among out-degree>=1",
                   "graph_sha256": g.sha256(), "sources_sha256": hashlib.sha256(
                       np.ascontiguousarray(srcs, dtype=np.int32).tobytes()).hexdigest(),
                   "reverse_graph": tg is not None,
                   "reverse_graph_build_ms": round(t_tg * 1e3, 2) if tg is not None else None},
        "sources_per_s": round(srcs_per_s, 1),
        "plain_sources_per_s": round(1.0 / plain_s, 1) if nplain else None,
        "plain_gteps": round(plain_gteps, 3) if nplain else None,
        "batched_vs_plain_sources_per_s": round(srcs_per_s * plain_s, 2) if nplain else None,
        "steps_max": inf["steps"],
        "mu_e": round(inf["edges_scanned"] / max(work, 1.0), 4),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "tuning": tune,
        "autotune": None if autotuned is None else {
            "key": autotuned["key"], "calibration": autotuned.get("calibration"),
            "tuned_fields": autotuned["tuning"],
            "default_tuning_ms_per_step": round(default_ms, 4),
            "tuned_vs_default": round(default_ms / ms_step, 3)},
    }
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
