"""Benchmark: kNN (k = 20) + covariance query points/s on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload batched|scan|map|tiny|served|...]

Default workload ``batched``, the largest single-GPU configuration: 48
uneven LiDAR scans (16 frames x 3 sensors, 20k-131k points each, 3,757,703
queries) against the resident 2,000,000-point voxelised track map, k = 20,
r = 2 m; cell size and launch shape from the autotuner.  One step is one
``lkc_knn_cov_batched`` call over all 48 scans: the query key and radix
sort launches, the group search (``k_group``) and the wavefront-per-query
search of the queries it hands over (``k_fallback``).  The plain
one-call-per-scan loop is timed beside it, the same call replayed from a
captured HIP graph is timed as an extra, and a short served stream (3
sensors at 20 Hz, real time) reports p50/p99 per-scan latency for the
served and the plain loop (``--served-seconds``, 0 = off).

Other workloads: ``scan`` (one spinning-LiDAR scan, ~118k points, sensor
frame, self-query, k = 20, r = 2 m, 1 m cells; a step is rebuild + fused
search), ``map`` (65,536-point scan against the resident map; a step is one
fused call), ``tiny`` (2,048-point plane + wall, k = 10, no cap),
``served`` (the served stream alone), ``weighted``, ``gicp``, ``voxel``,
``submap``, ``walls``.

Prints ONE JSON line.  ``value`` = queries/s over the timed steps (inputs
resident in HBM).  ``roofline`` is for the search kernel: algorithmic bytes
per query ``20 k + 100`` (query read, k neighbour gathers of 12 B, idx + d2 +
count, mean + cov + reg_cov writes) times the queries of one launch, divided
by the launch's mean duration from HIP events on the stream the kernel runs
on.  ``traffic`` comes from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
summary for the same kernel source, else null.  ``cpu_baseline`` is the FP64
oracle (brute force) on the host's cores over a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "kNN(k=20)+covariance query points/s and % HBM roofline; p99 scan latency"


def b_alg(k: int) -> int:
    return 20 * k + 100


def b_floor(k: int) -> int:
    """Algorithmic bytes without the neighbour gather (query, idx, d2,
    count, mean, cov, reg_cov): 8k + 100."""
    return 8 * k + 100


# VALU lane operations per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# (one wave64 instruction occupies a SIMD for four cycles; packed FP32 not
# counted)
VALU_LANE_OPS_PEAK = 256 * 4 * 16 * 2.4e9


# GICP reduction: source point (12) + its covariance (36) + correspondence
# (4) + the target point (16, float4 record) + its covariance (36)
B_GICP_REDUCE = 104


def b_knn(k: int) -> int:
    """kNN without covariance: query read, k gathers, idx + d2, count."""
    return 12 + 12 * k + 8 * k + 4


def kernel_src_sha() -> str:
    h = hashlib.sha256()
    for f in ("search.hip", "lkc_device.h"):
        with open(os.path.join(ROOT, "paper_2308_07173_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def committed_traffic(workload: str):
    """HBM bytes per launch from the committed PMC summary, if the search
    kernel source is unchanged since it was taken."""
    path = os.path.join(ROOT, "profiles", f"pmc_search_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_src_sha") != kernel_src_sha():
        return None
    return d.get("traffic_bytes")


def committed_valu(workload: str):
    """VALU instructions (wavefront level) per search-kernel launch from the
    committed PMC summary, under the same source check as the traffic, with
    the cell size and launch configuration they were counted at ({} = the
    default configuration)."""
    path = os.path.join(ROOT, "profiles", f"pmc_search_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_src_sha") != kernel_src_sha():
        return None
    if d.get("valu_insts_per_dispatch") is None:
        return None
    return d["valu_insts_per_dispatch"], {"cell_m": d.get("valu_cell_m"),
                                          "launch_cfg": d.get("valu_launch_cfg", {})}


def copy_bandwidth(torch, dev, mib: int = 1024, reps: int = 10) -> float:
    """Achievable HBM bandwidth, GB/s: a streaming elementwise kernel that
    reads and writes `mib` MiB each, timed with events."""
    src = torch.ones((mib << 20) // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.add(src, 1.0, out=dst)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        torch.add(src, 1.0, out=dst)
    b.record()
    b.synchronize()
    gbs = 2 * (mib << 20) * reps / (a.elapsed_time(b) * 1e-3) / 1e9
    del src, dst
    return gbs


def group_counts(torch, dev, ctx, step, n_queries: int):
    """Candidates tested and insertion steps of the group search, summed over
    its groups, from one profiled run of `step` (outside the timed region)."""
    groups = (n_queries + 63) // 64
    buf = torch.zeros((groups, 25), dtype=torch.int32, device=dev)
    ctx.set_profile(buf)
    step()
    torch.cuda.synchronize()
    ctx.set_profile(None)
    P = buf.cpu().numpy().view(np.uint32).astype(np.int64)
    return {"chunk_candidates": int(P[:, 4].sum()), "pops": int(P[:, 5].sum()),
            "lane_inserts": int(P[:, 8].sum())}


def cpu_threads() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def oracle_baseline(target, queries, k, radius, sample_rows, label, weight=None):
    from oracle import oracle
    q = queries[sample_rows]
    th = cpu_threads()
    t0 = time.perf_counter()
    idx, d2, cnt = oracle.knn(target, q, k, radius, threads=th)
    if weight is None:
        oracle.covariances(target, idx, cnt, eps=1e-3, threads=th)
    else:
        oracle.covariances_weighted(target, idx, cnt, weight[0], weight[1], queries=q, eps=1e-3)
    dt = time.perf_counter() - t0
    return {"value": q.shape[0] / dt, "unit": "queries/s", "cores": th, "kind": "oracle",
            "sample": f"{q.shape[0]} of {queries.shape[0]} queries ({label}); "
                      f"{dt:.2f} s FP64 brute-force kNN + covariance"}


def pct(xs, p):
    return float(np.percentile(np.asarray(xs), p)) if len(xs) else float("nan")


def served_stream(args, lkc, workloads, torch, duration, time_scale, saturated=True):
    """Served stream: 3 sensors x 20 Hz Poisson arrivals, scans of 10k-131k
    points against 4 resident maps (0.5, 1, 2, 4 M points), continuous
    batching in two slots, beside the plain one-call-per-scan loop under the
    same arrivals.  ``saturated`` also replays the same requests released all
    at once (the loops' capacity)."""
    from paper_2308_07173_amd import serve
    k, radius, cell = 20, 2.0, 1.0
    maps = workloads.served_maps()
    pool = workloads.served_scan_pool()
    sched = workloads.served_schedule(duration=duration, seed=5)
    reqs = [serve.ServeRequest(i, r.t_arrival, r.map_id,
                               np.ascontiguousarray(pool[i % len(pool)][:r.n_points]), r.sensor)
            for i, r in enumerate(sched)]
    budget = None if args.hbm_budget_gb <= 0 else int(args.hbm_budget_gb * 2**30)
    ex = serve.GpuExecutor(maps, cell=cell, k=k, radius=radius, hbm_budget_bytes=budget,
                           use_graphs=True)
    # buffer sets and graphs of every bucket a single request or a batch of
    # the stream can take, captured before the timed streams
    ex.warm([r.points.shape[0] for r in reqs])
    warm = reqs[: min(12, len(reqs))]
    serve.serve_loop(warm, ex, time_scale=math.inf)
    serve.serve_loop(reqs, ex, time_scale=math.inf)
    # batches of a bucket met for the first time inside the timed streams
    # run eagerly rather than pay a capture
    ex.capture_new = False
    res = serve.summarize(serve.serve_loop(reqs, ex, time_scale=time_scale))
    plain = serve.summarize(serve.plain_loop(reqs, ex, time_scale=time_scale))
    out = {"requests": res["requests"], "duration_s": duration, "time_scale": time_scale,
           "k": k, "radius_m": radius, "cell_m": cell, "hbm_budget_bytes": ex.budget,
           "resident_map_bytes": ex.resident_bytes, "served": res, "plain_per_scan": plain}
    if saturated:
        sat = serve.summarize(serve.serve_loop(reqs, ex, time_scale=math.inf))
        sat_plain = serve.summarize(serve.plain_loop(reqs, ex, time_scale=math.inf))
        out["saturated"] = {"served_queries_per_s": sat["queries_per_s"],
                            "plain_queries_per_s": sat_plain["queries_per_s"],
                            "served_mean_batch_requests": sat["mean_batch_requests"],
                            "served_wall_s": sat["wall_s"], "plain_wall_s": sat_plain["wall_s"]}
    ex.close()
    return out


def served(args, lkc, workloads, torch):
    r = served_stream(args, lkc, workloads, torch, args.duration, args.time_scale)
    res = r["served"]
    out = {
        "metric": METRIC, "value": res["queries_per_s"], "unit": "queries/s", "n_gpus": 1,
        "steps": res["batches"], "warmup": 12,
        "ms_per_step": res["wall_s"] / max(1, res["batches"]) * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded ray-cast race-track LiDAR)",
        "config": {"workload": "served stream: 3 LiDARs x 20 Hz Poisson, 10k-131k-point scans, "
                               "4 resident maps (0.5/1/2/4 M points)",
                   **{key: r[key] for key in ("requests", "duration_s", "time_scale", "k",
                                              "radius_m", "cell_m", "hbm_budget_bytes",
                                              "resident_map_bytes")}},
        "served": res, "plain_per_scan": r["plain_per_scan"], "saturated": r["saturated"],
        "latency_ms": {"p50": res["p50_ms"], "p99": res["p99_ms"]},
    }
    print(json.dumps(out))


def gicp(args, lkc, workloads, torch, ctx, cfg):
    """GICP linearisation of a 65,536-point scan against the resident
    2,000,000-point map: float32 transform, k = 1 correspondence search
    (1 m radius), FP64 per-point system and fixed-order reduction.  One step
    is one lkc_gicp_linearize; the covariances of both clouds are computed
    once beforehand (lkc_knn_cov_self, k = 20, r = 2 m)."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    m, _ = workloads.build_map(2_000_000, seed=2)
    s = workloads.source_scan(65_536, seed=3)
    cell, max_d = 1.0, 1.0
    mp, sp = torch.from_numpy(m).to(dev), torch.from_numpy(s).to(dev)
    tgt = lkc.lkc_build_target(ctx, mp, cell)
    src_t = lkc.lkc_build_target(ctx, sp, cell)
    tcov = lkc.lkc_knn_cov_self(ctx, tgt, 20, 2.0, 1e-3)["reg"]
    scov = lkc.lkc_knn_cov_self(ctx, src_t, 20, 2.0, 1e-3)["reg"]
    src_t.free()
    th = 0.002
    T = np.eye(4)
    T[:3, :3] = [[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]]
    T[:3, 3] = [0.05, -0.03, 0.01]
    system, corr = lkc.lkc_gicp_linearize(ctx, tgt, tcov, sp, scov, T, max_d, cfg=cfg)
    K, W = args.steps, args.warmup
    for _ in range(W):
        lkc.lkc_gicp_linearize(ctx, tgt, tcov, sp, scov, T, max_d, corr=corr, system=system,
                               cfg=cfg)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(K)]
    phases = []
    t0 = time.perf_counter()
    for i in range(K):
        evs[i][0].record(stream)
        lkc.lkc_gicp_linearize(ctx, tgt, tcov, sp, scov, T, max_d, corr=corr, system=system,
                               cfg=cfg)
        evs[i][1].record(stream)
        torch.cuda.synchronize()
        st = ctx.search_stats()
        phases.append((st["sort_ms"], st["group_ms"], st["fallback_ms"], st["reduce_ms"],
                       st["fallback_queries"]))
    total = time.perf_counter() - t0
    n = s.shape[0]
    call_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    ph = np.array(phases)
    sort_ms, group_ms, fb_ms, red_ms = (float(ph[:, i].mean()) for i in range(4))
    fb_q = int(ph[-1, 4])
    sysd = lkc.split_system(system)
    red_gbs = n * B_GICP_REDUCE / (red_ms * 1e-3) / 1e9
    grp_gbs = (n - fb_q) * b_knn(1) / (group_ms * 1e-3) / 1e9
    if red_ms >= group_ms:
        roof = {"kernel": "k_gicp_reduce", "achieved": red_gbs, "bytes_per_query": B_GICP_REDUCE,
                "queries_per_launch": n, "kernel_ms": red_ms}
    else:
        roof = {"kernel": "k_group (k=1)", "achieved": grp_gbs, "bytes_per_query": b_knn(1),
                "queries_per_launch": n - fb_q, "kernel_ms": group_ms}
    roof.update(bound="hbm", peak=HBM_PEAK_GBS, unit="GB/s",
                frac=roof["achieved"] / HBM_PEAK_GBS, traffic=None)
    res = {
        "metric": "GICP linearisation source points/s (correspondence + FP64 system)",
        "value": n * K / total, "unit": "points/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": total / K * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 search, f64 system",
        "data": "synthetic (seeded ray-cast race-track LiDAR)",
        "config": {"workload": "GICP step: 65,536-point scan vs 2,000,000-point voxelised map",
                   "n_points": n, "map_points": int(m.shape[0]), "max_corr_dist_m": max_d,
                   "cell_m": cell, "step": "transform + k=1 search + FP64 system reduction"},
        "roofline": roof,
        "phases_ms": {"query_sort": sort_ms, "k_group": group_ms, "k_fallback": fb_ms,
                      "reduce": red_ms, "call": call_ms},
        "fallback_queries": fb_q,
        "system": {"correspondences": sysd["count"], "rejected": sysd["rejected"],
                   "error": sysd["E"]},
        "other_kernel_GBs": {"k_gicp_reduce": red_gbs, "k_group": grp_gbs},
    }
    if not args.no_cpu_baseline:
        from oracle import oracle
        rows = np.sort(np.random.default_rng(0).choice(n, 1024, replace=False))
        tc, sc = tcov.cpu().numpy(), scov.cpu().numpy()
        c0 = time.perf_counter()
        oc, _ = oracle.gicp_correspond(s[rows], m, T, max_d, threads=cpu_threads())
        oracle.gicp_linearize(s[rows], sc[rows], m, tc, T, oc)
        dt = time.perf_counter() - c0
        res["cpu_baseline"] = {"value": len(rows) / dt, "unit": "points/s",
                               "cores": cpu_threads(), "kind": "oracle",
                               "sample": f"{len(rows)} of {n} source points; {dt:.2f} s FP64 "
                                         "brute-force correspondences + system"}
    tgt.free()
    print(json.dumps(res))
    ctx.synchronize()


def timed_calls(torch, fn, K, W):
    """Run fn W times untimed, then K times between HIP events on torch's
    current stream; returns (mean event ms, wall seconds of the K calls)."""
    stream = torch.cuda.current_stream()
    for _ in range(W):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(K)]
    t0 = time.perf_counter()
    for i in range(K):
        evs[i][0].record(stream)
        fn()
        evs[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return float(np.mean([a.elapsed_time(b) for a, b in evs])), wall


def voxel_and_submap(args, lkc, workloads, torch, ctx):
    """The steps before the path.  voxel: the 48 uneven scans of the batched
    workload (3,757,703 points, world frame) voxel-filtered at 0.2 m in one
    call.  submap: the map points within 50 m of a pose near the track, from
    the resident 2,000,000-point map, through its race-line index (only the
    pose's bin of map points is read), in one call."""
    dev = torch.device("cuda:0")
    K, W = args.steps, args.warmup
    if args.workload == "voxel":
        pts = np.concatenate(workloads.batched_scans(16, seed=4))
        n = pts.shape[0]
        p = torch.from_numpy(pts).to(dev)
        leaf = 0.2
        out = lkc.lkc_voxel_filter(ctx, p, leaf)
        m = int(out["count"].shape[0])
        ms, wall = timed_calls(torch, lambda: lkc.lkc_voxel_filter(ctx, p, leaf), K, W)
        alg = 12 * n + 28 * m      # points in; centroid + count + voxel out
        config = {"workload": "voxel filter of 48 uneven LiDAR scans (16 frames x 3 sensors)",
                  "n_points": n, "leaf_m": leaf, "voxels": m,
                  "step": "one lkc_voxel_filter call (bounds, key sort, runs, FP64 means)"}
        metric = "voxel filter input points/s"
        if not args.no_cpu_baseline:
            from oracle import oracle
            c0 = time.perf_counter()
            oracle.voxel_filter(pts, leaf)
            dt = time.perf_counter() - c0
            cpu = {"value": n / dt, "unit": "points/s", "cores": 1, "kind": "oracle",
                   "sample": f"all {n} points; {dt:.2f} s (qsort + FP64 sums, one thread)"}
    else:
        m_pts, _ = workloads.build_map(2_000_000, seed=2)
        n = m_pts.shape[0]
        t = lkc.lkc_build_target(ctx, torch.from_numpy(m_pts).to(dev), 1.0)
        s_line = np.arange(0.0, workloads.PERIMETER, 1.0)
        lx, ly, _ = workloads.centreline_pose(s_line)
        line = np.stack([lx, ly, np.zeros_like(lx)], axis=1).astype(np.float32)
        radius = 50.0
        c0 = time.perf_counter()
        rl = lkc.lkc_raceline_build(ctx, t, line, 2.0, radius, 8.0)
        build_s = time.perf_counter() - c0
        info = rl.info()
        _, bin_pts = rl.bins()
        px, py, _ = workloads.track_pose(123.4, 2.5)
        center = np.array([px, py, 0.5], np.float32)
        pose = torch.from_numpy(center).to(dev)
        cap = info["max_bin_points"]
        out = (torch.empty(cap, dtype=torch.int32, device=dev), None,
               torch.empty(3, dtype=torch.int64, device=dev))
        lkc.lkc_submap_window(ctx, rl, pose, radius, out=out)
        w_info = out[2].cpu().numpy()
        if w_info[2] != lkc.LKC_WINDOW_OK:
            raise RuntimeError(f"window status {w_info}")
        m, b = int(w_info[0]), int(w_info[1])
        touched = int(bin_pts[b])
        ms, wall = timed_calls(torch, lambda: lkc.lkc_submap_window(ctx, rl, pose, radius,
                                                                      out=out), K, W)
        full_ms, _ = timed_calls(torch, lambda: lkc.lkc_submap_extract(ctx, t, center, radius),
                                 max(2, K // 10), 1)
        words = (n + 31) // 32
        # the bin's points in (float4), the window's indices out, the bitmap
        # read by the count and the emit passes
        alg = 16 * touched + 4 * m + 8 * words
        config = {"workload": "race-line keyed sliding window: points within 50 m of a pose "
                              "2.5 m off the centreline, 2,000,000-point map",
                  "map_points": n, "radius_m": radius, "window_points": m,
                  "bin_points_read": touched, "bins": info["n_bins"],
                  "bin_length_m": info["bin_length"], "cover_radius_m": info["cover_radius"],
                  "index_build_s": build_s, "full_map_scan_ms": full_ms,
                  "step": "one lkc_submap_window call (pose hash, the bin's point ranges, "
                          "window bitmap, ascending compaction), pose on the device"}
        metric = "submap windows/s"
        if not args.no_cpu_baseline:
            from oracle import oracle
            c0 = time.perf_counter()
            oracle.submap(m_pts, center, radius)
            dt = time.perf_counter() - c0
            cpu = {"value": 1.0 / dt, "unit": "windows/s", "cores": 1, "kind": "oracle",
                   "sample": f"one window by the definition over all {n} map points; "
                             f"{dt:.3f} s (one thread)"}
        rl.free()
        t.free()
    achieved = alg / (ms * 1e-3) / 1e9
    value, unit = (n * K / wall, "points/s") if args.workload == "voxel" else \
        (K / wall, "windows/s")
    res = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": K,
           "warmup": W, "ms_per_step": wall / K * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic (seeded ray-cast race-track LiDAR)", "config": config,
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                        "kernel": "whole call", "bytes_per_call": alg, "call_ms": ms}}
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu
    print(json.dumps(res))
    ctx.synchronize()


def walls(args, lkc, workloads, torch, ctx):
    """Wall-detection front end on one 118k-point scan (sensor frame): voxel
    filter (0.2 m), z-vote (0.2 m cells, 3 votes), clustering of the kept
    voxels (0.5 m).  One step is the three calls."""
    dev = torch.device("cuda:0")
    K, W = args.steps, args.warmup
    pts = workloads.single_scan(seed=1)
    n = pts.shape[0]
    p = torch.from_numpy(pts).to(dev)
    state = {}

    def step():
        vox = lkc.lkc_voxel_filter(ctx, p, 0.2)["centroid"]
        keep, _ = lkc.lkc_zvote(ctx, vox, 0.2, 3, with_votes=False)
        labels, k = lkc.lkc_euclid_cluster(ctx, vox, 0.5, mask=keep)
        state.update(voxels=int(vox.shape[0]), kept=int(keep.sum().item()), clusters=k)

    ms, wall = timed_calls(torch, step, K, W)
    res = {"metric": "wall-detection front end: scan points/s (voxel filter + z-vote + "
                     "clustering)",
           "value": n * K / wall, "unit": "points/s", "n_gpus": 1, "steps": K, "warmup": W,
           "ms_per_step": wall / K * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32",
           "data": "synthetic (seeded ray-cast race-track LiDAR)",
           "config": {"workload": "one 128x1024 spinning-LiDAR scan, sensor frame",
                      "n_points": n, "leaf_m": 0.2, "vote_cell_m": 0.2, "tau": 3,
                      "eps_m": 0.5, **state,
                      "step": "lkc_voxel_filter + lkc_zvote + lkc_euclid_cluster (masked)"},
           "step_event_ms": ms,
           "roofline": None}
    if not args.no_cpu_baseline:
        from oracle import oracle
        c0 = time.perf_counter()
        v = oracle.voxel_filter(pts, 0.2)["centroid"].astype(np.float32)
        keep, _ = oracle.zvote(v, 0.2, 3)
        oracle.euclid_cluster(v[keep == 1], 0.5)
        dt = time.perf_counter() - c0
        res["cpu_baseline"] = {"value": n / dt, "unit": "points/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"the whole scan; {dt:.2f} s (sort-based voxel filter "
                                         "and vote, all-pairs clustering, one thread)"}
    print(json.dumps(res))
    ctx.synchronize()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="batched",
                    choices=["scan", "map", "weighted", "gicp", "batched", "tiny", "served",
                             "voxel", "submap", "walls"])
    ap.add_argument("--sigma", type=float, default=0.2,
                    help="weighted: Laplacian kernel width in metres")
    ap.add_argument("--time-scale", type=float, default=1.0,
                    help="served: schedule compression (1 = real time, inf = open loop)")
    ap.add_argument("--served-seconds", type=float, default=20.0,
                    help="batched: seconds of served stream (real time) whose p50/p99 "
                         "latency are reported beside the batched line (0 = off)")
    ap.add_argument("--duration", type=float, default=60.0, help="served: stream seconds")
    ap.add_argument("--hbm-budget-gb", type=float, default=0.0,
                    help="served: device memory budget (0 = 80 %% of free)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batched and tiny: skip the autotuner (default launch shape; "
                         "batched also 1 m cells)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cfg", default="", help="launch cfg, e.g. tile_queries=32,merge_min=8")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the run, launch one plain device copy of this many MiB "
                         "(reference dispatch for HBM byte counters)")
    ap.add_argument("--calib-gather-mib", type=int, default=0,
                    help="after the run, launch one float4 row gather of this many MiB "
                         "(rows read through a permutation inside every 64-row block): "
                         "a second reference dispatch, for reads shaped like the searches'")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: this path has no multi-GPU mode "
              "(queries are independent and would shard across GPUs with no exchange).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2308_07173_amd import lkc, workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    cfg = None
    if args.cfg:
        cfg = {kv.split("=")[0]: int(kv.split("=")[1]) for kv in args.cfg.split(",")}
    ctx = lkc.Context()
    ctx.set_timing(True)
    stream = torch.cuda.current_stream()
    phases = []   # per timed step: the library's phase times of the search call

    def record_phases():
        st = ctx.search_stats()
        phases.append((st["sort_ms"], st["group_ms"], st["fallback_ms"], st["fallback_queries"]))
    K, W = args.steps, args.warmup
    extra = {}

    def ev():
        return torch.cuda.Event(enable_timing=True)

    if args.workload == "served":
        return served(args, lkc, workloads, torch)
    if args.workload == "gicp":
        return gicp(args, lkc, workloads, torch, ctx, cfg)
    if args.workload in ("voxel", "submap"):
        return voxel_and_submap(args, lkc, workloads, torch, ctx)
    if args.workload == "walls":
        return walls(args, lkc, workloads, torch, ctx)
    if args.workload in ("scan", "tiny"):
        if args.workload == "scan":
            pts = workloads.single_scan(seed=1)
            k, radius, cell = 20, 2.0, 1.0
            config = {"workload": "one 128x1024 spinning-LiDAR scan, self-query",
                      "n_points": int(pts.shape[0]), "k": k, "radius_m": radius,
                      "cell_m": cell,
                      "step": "grid rebuild (asynchronous) + fused kNN+covariance"}
        else:
            pts = workloads.plane_wall(2048, seed=0)
            k, radius, cell = 10, math.inf, 1.0
            config = {"workload": "2048-point plane + wall, self-query", "n_points": 2048,
                      "k": k, "radius_m": None, "cell_m": cell,
                      "step": "grid rebuild (asynchronous) + fused kNN+covariance"}
            if not args.no_autotune and not args.cfg:
                # the launch shape only (the cell is the configuration's)
                from paper_2308_07173_amd import autotune
                tune = autotune.autotune(pts, pts, k, radius, cells=(cell,),
                                         sample=pts.shape[0], ctx=ctx)
                cfg = tune["cfg"] or None
                config["autotune"] = {"cfg": tune["cfg"], "candidates": len(tune["table"])}
        p = torch.from_numpy(pts).to(dev)
        Q = p.shape[0]
        tgt = lkc.lkc_build_target(ctx, p, cell)
        out = lkc.lkc_knn_cov_self(ctx, tgt, k, radius, 1e-3, cfg=cfg)

        def step(kstart=None, kend=None):
            tgt.rebuild(p, sync=False)
            if kstart is not None:
                kstart.record(stream)
            lkc.lkc_knn_cov_self(ctx, tgt, k, radius, 1e-3, out=out, cfg=cfg)
            if kend is not None:
                kend.record(stream)

        for _ in range(W):
            step()
        torch.cuda.synchronize()
        ks = [(ev(), ev()) for _ in range(K)]
        lat = []
        t0 = time.perf_counter()
        for i in range(K):
            s0 = time.perf_counter()
            step(*ks[i])
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - s0)
            record_phases()
        t1 = time.perf_counter()
        kern_ms = float(np.mean([a.elapsed_time(b) for a, b in ks]))
        total = t1 - t0
        queries_per_launch = Q
        extra["latency_ms"] = {"p50": pct(lat, 50) * 1e3, "p99": pct(lat, 99) * 1e3,
                               "max": max(lat) * 1e3}
        extra["search_kernel_ms"] = kern_ms
        # the rest of a step with a host wait after it: the rebuild's GPU time
        # plus the host's launch overhead and the wait (the rebuild's own GPU
        # time is pipelined.build_ms and graph_replay.build_ms below)
        extra["rebuild_host_and_wait_ms_mean"] = total / K * 1e3 - kern_ms
        info = tgt.info()
        extra["grid"] = {"cells": info["n_cells"], "hash_capacity": info["hash_capacity"],
                         "sort_passes": info["sort_passes"]}
        # steps back to back without a host wait between them (the build of
        # one scan overlaps nothing, but its launches no longer trail a sync):
        # the GPU time of a step, and of the search alone
        def search_only():
            lkc.lkc_knn_cov_self(ctx, tgt, k, radius, 1e-3, out=out, cfg=cfg)
        ctx.set_timing(False)
        pms, _ = timed_calls(torch, step, K, 2)
        sms, _ = timed_calls(torch, search_only, K, 2)
        ctx.set_timing(True)
        extra["pipelined"] = {"ms_per_step": pms, "search_ms": sms, "build_ms": pms - sms}
        # the same step (rebuild + fused search, nothing synchronised in
        # between) captured once as a HIP graph and replayed: the launches of
        # the build no longer wait on the host
        ref = {key: v.clone() for key, v in out.items()}
        ctx.set_timing(False)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            step()
        ctx.set_timing(True)
        g.replay()
        torch.cuda.synchronize()
        same = all(torch.equal(ref[key], out[key]) for key in ref)
        glat = []
        for _ in range(max(K, 20)):
            s0 = time.perf_counter()
            g.replay()
            torch.cuda.synchronize()
            glat.append(time.perf_counter() - s0)
        gms, _ = timed_calls(torch, g.replay, K, 2)
        extra["graph_replay"] = {"ms_per_step": gms, "build_ms": gms - kern_ms,
                                 "latency_ms": {"p50": pct(glat, 50) * 1e3,
                                                "p99": pct(glat, 99) * 1e3},
                                 "equal_to_eager": bool(same)}
        del g
        baseline_args = (pts, pts, k, radius, np.arange(Q), "the whole scan")
    elif args.workload in ("map", "weighted"):
        m, _ = workloads.build_map(2_000_000, seed=2)
        s = workloads.source_scan(65_536, seed=3)
        k, radius, cell = 20, 2.0, 1.0
        config = {"workload": "65,536-point scan vs 2,000,000-point voxelised map",
                  "n_points": 65536, "map_points": 2_000_000, "k": k, "radius_m": radius,
                  "cell_m": cell, "step": "fused kNN+covariance (map resident)"}
        weighted = args.workload == "weighted"
        if weighted:
            config["step"] = "fused kNN + Laplacian-weighted covariance (map resident)"
            config["kernel"] = {"kind": "laplacian", "sigma_m": args.sigma}
        mp = torch.from_numpy(m).to(dev)
        sq = torch.from_numpy(s).to(dev)
        torch.cuda.synchronize()
        b0 = time.perf_counter()
        tgt = lkc.lkc_build_target(ctx, mp, cell)
        torch.cuda.synchronize()
        extra["map_build_ms"] = (time.perf_counter() - b0) * 1e3
        if weighted:
            out = lkc.lkc_knn_cov_weighted(ctx, tgt, sq, k, "laplacian", args.sigma, radius,
                                           1e-3, cfg=cfg)
        else:
            out = lkc.lkc_knn_cov(ctx, tgt, sq, k, radius, 1e-3, cfg=cfg)
        Q = sq.shape[0]

        def step(kstart=None, kend=None):
            if kstart is not None:
                kstart.record(stream)
            if weighted:
                lkc.lkc_knn_cov_weighted(ctx, tgt, sq, k, "laplacian", args.sigma, radius,
                                         1e-3, out=out, cfg=cfg)
            else:
                lkc.lkc_knn_cov(ctx, tgt, sq, k, radius, 1e-3, out=out, cfg=cfg)
            if kend is not None:
                kend.record(stream)

        for _ in range(W):
            step()
        torch.cuda.synchronize()
        ks = [(ev(), ev()) for _ in range(K)]
        lat = []
        t0 = time.perf_counter()
        for i in range(K):
            s0 = time.perf_counter()
            step(*ks[i])
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - s0)
            record_phases()
        t1 = time.perf_counter()
        kern_ms = float(np.mean([a.elapsed_time(b) for a, b in ks]))
        total = t1 - t0
        queries_per_launch = Q
        extra["latency_ms"] = {"p50": pct(lat, 50) * 1e3, "p99": pct(lat, 99) * 1e3}
        extra["search_kernel_ms"] = kern_ms
        rows = np.sort(np.random.default_rng(0).choice(Q, 4096, replace=False))
        baseline_args = (m, s, k, radius, rows, "seeded subsample")
        if weighted:
            baseline_args = baseline_args + (("laplacian", args.sigma),)
    else:  # batched
        m, _ = workloads.build_map(2_000_000, seed=2)
        scans = workloads.batched_scans(16, seed=4)
        k, radius, cell = 20, 2.0, 1.0
        allq = np.concatenate(scans)
        offs = np.cumsum([0] + [sc.shape[0] for sc in scans])
        Q = allq.shape[0]
        config = {"workload": "48 uneven scans (16 frames x 3 LiDARs) vs 2,000,000-point map",
                  "n_points": int(Q), "scans": len(scans), "map_points": 2_000_000, "k": k,
                  "radius_m": radius, "cell_m": cell,
                  "step": "one lkc_knn_cov_batched call over all scans: query keys + radix "
                          "sort, group search (k_group), wavefront search of the queries "
                          "it hands over (k_fallback)"}
        if not args.no_autotune and not args.cfg:
            from paper_2308_07173_amd import autotune
            tune = autotune.autotune(m, allq, k, radius, sample=allq.shape[0], reps=5, ctx=ctx)
            cell, cfg = tune["cell"], (tune["cfg"] or None)
            config["autotune"] = {"cell_m": cell, "cfg": tune["cfg"], "sample": tune["sample"],
                                  "candidates": len(tune["table"])}
            # Shapes within 2 % of the best are the autotuner's own noise band
            # (it keeps an earlier candidate unless a later one is 2 % faster):
            # among them, take the one the committed counter summary was taken
            # at, so that the VALU rate below belongs to the shape timed here.
            cv = committed_valu(args.workload)
            if cv is not None:
                at = cv[1]
                for c_, g_, ms_ in tune["table"]:
                    if (c_ == at["cell_m"] and dict(g_) == at["launch_cfg"]
                            and ms_ <= 1.02 * tune["ms"]):
                        cell, cfg = c_, (dict(g_) or None)
                        config["autotune"]["profiled_shape_within_2pct"] = True
            config["cell_m"] = cell
        mp = torch.from_numpy(m).to(dev)
        aq = torch.from_numpy(allq).to(dev)
        tgt = lkc.lkc_build_target(ctx, mp, cell)
        ctx.reserve(Q)
        tset = lkc.TargetSet(ctx, [tgt], max_scans=len(scans))
        tset.stage([(int(offs[i]), int(scans[i].shape[0]), 0) for i in range(len(scans))])
        out = lkc.lkc_knn_cov_batched(ctx, tset, aq, k, radius, 1e-3, cfg=cfg)

        def step(kstart=None, kend=None):
            if kstart is not None:
                kstart.record(stream)
            lkc.lkc_knn_cov_batched(ctx, tset, aq, k, radius, 1e-3, out=out, cfg=cfg)
            if kend is not None:
                kend.record(stream)

        for _ in range(W):
            step()
        torch.cuda.synchronize()
        ks = [(ev(), ev()) for _ in range(K)]
        t0 = time.perf_counter()
        for i in range(K):
            step(*ks[i])
            torch.cuda.synchronize()
            record_phases()
        t1 = time.perf_counter()
        kern_ms = float(np.mean([a.elapsed_time(b) for a, b in ks]))
        total = t1 - t0
        queries_per_launch = Q
        extra["search_kernel_ms"] = kern_ms
        # the plain path: one fused launch per scan, same stream
        views = [aq[offs[i]:offs[i + 1]] for i in range(len(scans))]
        outs = [lkc.lkc_knn_cov(ctx, tgt, v, k, radius, 1e-3) for v in views]
        torch.cuda.synchronize()
        pe = (ev(), ev())
        pe[0].record(stream)
        for v, o in zip(views, outs):
            lkc.lkc_knn_cov(ctx, tgt, v, k, radius, 1e-3, out=o)
        pe[1].record(stream)
        torch.cuda.synchronize()
        plain_ms = pe[0].elapsed_time(pe[1])
        extra["plain_per_scan_loop_ms"] = plain_ms
        extra["plain_per_scan_loop_qps"] = Q / (plain_ms * 1e-3)
        # the same call replayed from a captured HIP graph (bitwise equal to
        # the eager call)
        ref = {key: v.clone() for key, v in out.items()}
        ctx.set_timing(False)     # no phase events inside the capture
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            lkc.lkc_knn_cov_batched(ctx, tset, aq, k, radius, 1e-3, out=out, cfg=cfg)
        ctx.set_timing(True)
        g.replay()
        torch.cuda.synchronize()
        same = all(torch.equal(ref[key], out[key]) for key in ref)
        gms, _ = timed_calls(torch, g.replay, K, 2)
        extra["graph_replay"] = {"ms": gms, "queries_per_s": Q / (gms * 1e-3),
                                 "bitwise_equal_to_eager": bool(same)}
        del g
        rows = np.sort(np.random.default_rng(0).choice(Q, Q // 64, replace=False))
        baseline_args = (m, allq, k, radius, rows, "seeded 1/64 subsample")

    value = queries_per_launch * K / total
    ph = np.array(phases, dtype=np.float64)
    sort_ms, group_ms, fb_ms = (float(ph[:, i].mean()) for i in range(3))
    fb_q = int(ph[-1, 3])
    extra["fallback_queries"] = fb_q
    # dominant kernel: the group search, its algorithmic bytes those of the
    # queries it answers (the rest go to the wavefront search); or the
    # wavefront search when it takes longer (one wavefront per query)
    group_q = queries_per_launch - fb_q
    dom = ("k_group", group_q, group_ms) if group_ms >= fb_ms else ("k_fallback", fb_q, fb_ms)
    achieved = dom[1] * b_alg(k) / (dom[2] * 1e-3) / 1e9
    path_achieved = queries_per_launch * b_alg(k) / (kern_ms * 1e-3) / 1e9
    extra["phases_ms"] = {"query_sort": sort_ms, "k_group": group_ms, "k_fallback": fb_ms}
    extra["search_call"] = {"ms": kern_ms, "achieved_GBs": path_achieved,
                            "frac": path_achieved / HBM_PEAK_GBS}
    traffic = committed_traffic(args.workload) if dom[0] == "k_group" else None
    hbm_meas = copy_bandwidth(torch, dev)
    floor_achieved = dom[1] * b_floor(k) / (dom[2] * 1e-3) / 1e9
    if dom[0] == "k_group":
        # the group search is bound by VALU issue, not HBM: every query
        # examines hundreds of candidates for its 20k + 100 bytes
        gc = group_counts(torch, dev, ctx, step, queries_per_launch)
        pairs = 64 * gc["chunk_candidates"]    # each broadcast candidate meets 64 lanes
        cand = {"pairs_tested": pairs, "pairs_per_s": pairs / (group_ms * 1e-3),
                "insertion_steps": gc["pops"], "lane_insertions": gc["lane_inserts"]}
        cv = committed_valu(args.workload)
        if cv is not None:
            vi, counted_at = cv
            cand["valu"] = {"insts_per_launch": vi, "counted_at": counted_at,
                            "peak": VALU_LANE_OPS_PEAK}
            # the count depends on the launch shape (reach and cell size change
            # the walk), so a rate is given only for the shape it was counted at
            if counted_at == {"cell_m": config.get("cell_m"), "launch_cfg": cfg or {}}:
                lane_ops = 64 * vi / (group_ms * 1e-3)
                cand["valu"].update(lane_ops_per_s=lane_ops, frac=lane_ops / VALU_LANE_OPS_PEAK)
            else:
                cand["valu"].update(lane_ops_per_s=None, frac=None)
        extra["group_search_work"] = cand
    if args.workload == "weighted":
        config["note"] = "roofline bytes as the plain path: the weights add no HBM traffic"
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": total / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded ray-cast race-track LiDAR)",
        "config": config,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_counted_at": ((committed_valu(args.workload) or (None, None))[1]
                                            if traffic is not None else None),
                     "kernel": dom[0], "bytes_per_query": b_alg(k),
                     "queries_per_launch": int(dom[1]), "kernel_ms": dom[2],
                     "measured_peak": hbm_meas, "frac_of_measured": achieved / hbm_meas,
                     "floor_bytes_per_query": b_floor(k), "floor_achieved": floor_achieved,
                     "floor_frac": floor_achieved / HBM_PEAK_GBS},
    }
    res.update(extra)
    if cfg:
        res["launch_cfg"] = cfg
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = oracle_baseline(*baseline_args)
    if args.workload == "batched" and args.served_seconds > 0:
        # the served stream in real time: per-scan latency of the served and
        # the plain one-call-per-scan loop under the same arrivals
        sv = served_stream(args, lkc, workloads, torch, args.served_seconds, 1.0,
                           saturated=False)
        res["served_stream"] = {
            "workload": "3 LiDARs x 20 Hz Poisson, 10k-131k-point scans, 4 resident maps "
                        "(0.5/1/2/4 M points), real time",
            "seconds": args.served_seconds, "requests": sv["requests"],
            "served": {key: sv["served"][key] for key in ("p50_ms", "p99_ms", "max_ms",
                                                          "queries_per_s",
                                                          "mean_batch_requests")},
            "plain_per_scan": {key: sv["plain_per_scan"][key]
                               for key in ("p50_ms", "p99_ms", "max_ms", "queries_per_s")}}
        res["latency_ms"] = {"p50": sv["served"]["p50_ms"], "p99": sv["served"]["p99_ms"],
                             "source": "served stream (real time), arrival to results"}
    if args.calib_copy_mib > 0:
        # a plain streaming kernel of known size: reads nb bytes, writes nb
        # bytes (an elementwise add; a device copy may go to the DMA engine)
        nb = args.calib_copy_mib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.add(src, 1.0, out=dst)
        torch.cuda.synchronize()
        res["calib_copy_bytes"] = nb
    if args.calib_gather_mib > 0:
        # 16-byte rows gathered by the library's lkc_calib_gather through a
        # uint32 index: each 64-row block is read in a shuffled order (one
        # wavefront's rows, as the searches read a chunk's points), so
        # every line fetched is used whole
        rows = (args.calib_gather_mib << 20) // 16 // 64 * 64
        g = torch.Generator().manual_seed(7)
        blk = torch.arange(rows, dtype=torch.int64).view(-1, 64)
        shuf = torch.argsort(torch.rand(blk.shape, generator=g), dim=1)
        idx = torch.gather(blk, 1, shuf).reshape(-1).to(torch.int32).to(dev)
        src4 = torch.ones(rows, 4, dtype=torch.float32, device=dev)
        out4 = torch.empty_like(src4)
        torch.cuda.synchronize()
        ctx.calib_gather(src4, idx, out4)
        ctx.synchronize()
        assert bool((out4 == 1.0).all())
        res["calib_gather"] = {"rows": rows, "bytes_read": rows * (16 + 4),
                               "bytes_written": rows * 16}
    print(json.dumps(res))
    ctx.synchronize()


if __name__ == "__main__":
    main()
