#!/usr/bin/env python3
"""Throughput of the raycast-and-policy query on one MI355X.

One step is one blocking ``rmpc_query``: cast 65536 Halton rays from one robot state through
the resident 400^3 paper-shaped map, evaluate one obstacle policy per ray, metric-sum, resolve
in float64 and read the 144-byte result back to the host (the paper's frame: load, execute,
block-reduce, read back).  ``value`` is rays per second over the timed steps.

Printed as one JSON line with a ``roofline`` entry for the dominant kernel (algorithmic bytes
per launch over the dispatch-timed kernel duration) and a ``cpu_baseline`` entry (the float64
oracle on the host cores, bounded sample).
"""
import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "rays/sec (raycast+RMP+resolve) at 65536 rays/query; served p50/p99 query latency"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_2301_08068_amd/csrc/raycast.hip", "paper_2301_08068_amd/csrc/rmpc_device.h",
                  "paper_2301_08068_amd/csrc/rmpc_kernels.h", "paper_2301_08068_amd/csrc/rmpc_walk.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "raycast_rmp_paper400_f32_traffic.txt")
L2_FILE = os.path.join(ROOT, "profiles", "raycast_rmp_paper400_f32_instmix_l2.txt")
L2_LINE_BYTES = 128

CONFIGS = {
    # name: (map builder, encoding, state seed, rays, max range[, subvoxel])
    "paper": ("paper", "f32", 200, 65536, 10.0),
    "paper_f16": ("paper", "f16", 200, 65536, 10.0),
    "paper_u8": ("paper", "u8", 200, 65536, 10.0),
    # the paper shape with sub-voxel hit distances (the TSDF's zero crossing)
    "paper_subvoxel": ("paper", "f32", 200, 65536, 10.0, 1),
    "tiny": ("tiny", "f32", 100, 1024, 5.0),
}
ELEM_BYTES = {"f32": 4, "f16": 2, "u8": 1}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _profile_values(path):
    """key: value lines of a committed profile summary, or None when the file is missing or was
    taken on other kernel sources than the current ones."""
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        line = line.lstrip("# ")
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return vals


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken on
    the current kernel sources; None otherwise."""
    vals = _profile_values(TRAFFIC_FILE)
    try:
        return float(vals["fetch_bytes_per_launch"]) + float(vals["write_bytes_per_launch"])
    except (TypeError, KeyError, ValueError):
        return None


def measured_l2():
    """L2 requests (TCC_HIT + TCC_MISS) and hit rate per launch from the committed rocprofv3
    counter summary, if it was taken on the current kernel sources; None otherwise."""
    vals = _profile_values(L2_FILE)
    try:
        return float(vals["l2_hits_per_launch"]) + float(vals["l2_misses_per_launch"]), float(vals["l2_hit_rate"])
    except (TypeError, KeyError, ValueError):
        return None


def build_map(kind: str, enc: str):
    from paper_2301_08068_amd import workloads as W
    vm = W.paper_map(2) if kind == "paper" else W.tiny_map(1)
    data = {"f32": vm.tsdf, "f16": W.encode_f16(vm.tsdf), "u8": W.encode_u8(vm.tsdf)}[enc]
    return vm, data


def cpu_model() -> str:
    """The host CPU's model name (lscpu's "Model name", else /proc/cpuinfo's "model name")."""
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(vm, data, enc, x, v, n_rays, params, budget_s):
    """The float64 oracle as it stands, on every core of this process's affinity set and on one
    core: each figure is the median of 5 runs (each run: full queries for about budget_s / 10 s
    of wall time) after one warm-up query."""
    import oracle
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    om = oracle.OracleMap(data, vm.voxel_m, vm.origin_m, enc)
    dirs = oracle.directions(n_rays)
    run_s = budget_s / 10.0

    def one_run(threads):
        done, t0 = 0, time.perf_counter()
        while True:
            oracle.query(om, x, v, n_rays, params, nthreads=threads, dirs=dirs)
            done += 1
            el = time.perf_counter() - t0
            if el >= run_s:
                return done, done * n_rays / el

    rates = {}
    for threads in (cores, 1):
        oracle.query(om, x, v, n_rays, params, nthreads=threads, dirs=dirs)   # warm-up
        runs = [one_run(threads) for _ in range(5)]
        rates[threads] = (statistics.median(r for _, r in runs), sum(d for d, _ in runs))
    return {"value": rates[cores][0], "unit": "rays/s", "cores": cores, "kind": "oracle",
            "value_1_core": rates[1][0], "nproc": os.cpu_count(), "cpu_model": cpu_model(),
            "sample": f"full queries of {n_rays} rays on the same map and state, float64 C oracle, OpenMP "
                      f"over rays; median of 5 runs of ~{run_s:.1f} s after a warm-up query, on {cores} "
                      f"cores ({rates[cores][1]} queries) and on 1 core ({rates[1][1]} queries)"}


def batch_compare(steps, warmup, plain_repeats=1):
    """Batched form (512 states along 8 trajectories, ray counts log-uniform in [4096, 65536]):
    one tuned persistent launch per step replayed from a hipGraph, against the same 512 states
    as blocking single queries (the plain path).  Returns rays/s of both and the tuned launch."""
    import torch
    from paper_2301_08068_amd import binding
    from paper_2301_08068_amd import workloads as W
    vm = W.paper_map(2)
    xs, vs = W.trajectory_states(vm, 8, 64, seed0=300)
    counts = W.ray_counts(len(xs), seed=399)
    params = W.params("static", max_range=10.0)
    ctx = binding.Context(0, arena_bytes=1 << 30)
    try:
        mid = ctx.upload(vm.tsdf, vm.voxel_m, vm.origin_m, "f32")
        qs = [dict(kind="map", map_id=mid, n=int(n), x=x, v=v) for x, v, n in zip(xs, vs, counts)]
        descs = binding.query_descs(qs)
        tuned = binding.rmpc_tune_batch(ctx.ptr, descs, params, None)
        ctx.config(binding.CONFIG_BATCH, use_graph=1)
        total = int(counts.sum())
        for _ in range(warmup):
            binding.rmpc_query_batch(ctx.ptr, descs, params, None, stream=ctx.stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            binding.rmpc_query_batch(ctx.ptr, descs, params, None, stream=ctx.stream)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        # the plain path: one blocking query per state
        preps = [binding.PreparedQuery(ctx.ptr, mid, q["x"], q["v"], q["n"], params, stream=ctx.stream)
                 for q in qs]
        for pq in preps[:16]:
            pq()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(plain_repeats):
            for pq in preps:
                pq()
        plain = (time.perf_counter() - t1) / plain_repeats
    finally:
        ctx.close()
    return {"rays_per_step": total, "states": len(qs), "batch_ms": 1e3 * el / steps,
            "batch_rays_per_s": total * steps / el, "plain_ms": 1e3 * plain, "plain_rays_per_s": total / plain,
            "tuned": tuned}


def batch_bench(args):
    """The batched form as its own bench line."""
    r = batch_compare(args.steps, args.warmup, plain_repeats=3)
    out = {"metric": "rays/sec (raycast+RMP+resolve), 512 states of uneven ray counts per launch",
           "value": r["batch_rays_per_s"], "unit": "rays/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": r["batch_ms"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "512 states on 8 seeded trajectories through the 400^3 f32 map; "
                                  "ray counts log-uniform in [4096, 65536]; one persistent launch per "
                                  "step replayed from a hipGraph",
                      "rays_per_step": r["rays_per_step"], "tuned": r["tuned"],
                      "plain_rays_per_s": r["plain_rays_per_s"], "plain_ms": r["plain_ms"]}}
    print(json.dumps(out), flush=True)


SERVE_RATES = (2000, 5000, 10000, 20000)


def _serve_open_loop(binding, ctx, reqs, arrivals):
    """Submit each request at its arrival time (s from now) and collect results as they
    complete; returns submit times and latencies from the scheduled arrival (s)."""
    import numpy as np
    n = len(reqs)
    idx_of = {}
    sub = np.zeros(n)
    lat = np.full(n, np.nan)
    done_t = 0.0
    i = done = 0
    t0 = time.perf_counter()
    last_progress = t0
    while done < n:
        now = time.perf_counter() - t0
        while i < n and arrivals[i] <= now:
            idx_of[binding.rmpc_submit(ctx.ptr, reqs[i])] = i
            sub[i] = time.perf_counter() - t0
            i += 1
        tks, lats, _, k = binding.rmpc_poll_completed(ctx.ptr, 1024, raw=True)
        if k:
            tnow = time.perf_counter()
            done_t = tnow - t0
            last_progress = tnow
            for t, l in zip(tks, lats):
                j = idx_of.pop(t)
                lat[j] = (sub[j] - arrivals[j]) + l     # arrival -> result on the host
            done += k
        elif time.perf_counter() - last_progress > 60.0:
            raise RuntimeError("serving run made no progress for 60 s")
    return sub, lat, done_t


def _serve_rate(binding, ctx, reqs, n_units, is_grid, arrivals, server_kw, n_warm):
    """One open-loop Poisson run: after an untimed paced pass over the first n_warm requests
    at the same rate (the GPU's clocks ramp up under load within tens of milliseconds; a run
    that starts from a lightly loaded GPU would measure that ramp), submit each request at its
    arrival time, collect results as they complete, and return per-request latency from the
    scheduled arrival (s) and counters."""
    import numpy as np
    binding.rmpc_server_start(ctx.ptr, **server_kw)
    try:
        _serve_open_loop(binding, ctx, reqs[:n_warm], arrivals[:n_warm])
        base = binding.rmpc_server_stats(ctx.ptr)
        n = len(reqs)
        sub, lat, done_t = _serve_open_loop(binding, ctx, reqs, arrivals)
        st = binding.rmpc_server_stats(ctx.ptr)
    finally:
        binding.rmpc_server_stop(ctx.ptr)
    units = float(np.sum(n_units))
    lag = sub - arrivals[:n]
    return {
        "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 3),
        "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 3),
        "p50_grid_ms": round(1e3 * float(np.percentile(lat[is_grid], 50)), 3),
        "p99_grid_ms": round(1e3 * float(np.percentile(lat[is_grid], 99)), 3),
        "p50_scan_ms": round(1e3 * float(np.percentile(lat[~is_grid], 50)), 3),
        "p99_scan_ms": round(1e3 * float(np.percentile(lat[~is_grid], 99)), 3),
        "evals_per_s": units / done_t,
        "offered_evals_per_s": units / float(arrivals[n - 1]),
        "launches": st["launches"] - base["launches"],
        "mean_batch": round(n / max(1, st["launches"] - base["launches"]), 2),
        "batch_max_since_start": st["batch_max"],
        "staging_waits": st["staging_waits"] - base["staging_waits"],
        "refused": st["refused"] - base["refused"],
        "staging_peak_bytes": st["staging_peak"],
        "submit_lag_p99_ms": round(1e3 * float(np.percentile(lag, 99)), 3),
        "wall_s": round(done_t, 3),
    }


def scan_bench(args):
    """LiDAR scan policy (Sec. III-G) on a 128 x 2048 beam frame over a 90-degree vertical field
    of view (262,144 points, device-resident): blocking rmpc_scan_query steps, points/s."""
    import numpy as np
    import torch
    import oracle
    from paper_2301_08068_amd import binding
    from paper_2301_08068_amd import workloads as W
    vm = W.paper_map(2)
    x, v = W.free_state(vm, 610)
    pts = W.synth_scan(vm, x, 610, n_elev=128, n_azim=2048, fov_deg=90.0)
    n = pts.shape[0]
    params = W.params("lidar")
    ctx = binding.Context(0, arena_bytes=1 << 28)
    dev = torch.from_numpy(pts).to("cuda:0")
    ptr = dev.data_ptr()
    # the timed steps: blocking scan queries through a prepared C call, as a control loop makes them
    step = binding.PreparedScan(ctx.ptr, ptr, n, v, params, stream=ctx.stream)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    binding.rmpc_set_profiling(ctx.ptr, True)
    for _ in range(min(args.steps, 100)):
        step()
    kms, nl = binding.rmpc_get_profile(ctx.ptr)
    binding.rmpc_set_profiling(ctx.ptr, False)
    kern_s = kms / 1e3 / max(nl, 1)
    alg_bytes = 12 * n
    out = {"metric": "scan points/sec (LiDAR policy + resolve), 262,144-point frame", "value": n * args.steps / elapsed,
           "unit": "points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "128 x 2048 beams over +-45 degrees elevation, ranges to the analytic first "
                                  "surface of the 400^3 paper-shaped map + N(0, 0.02^2) m, 10 % dropouts; "
                                  "LiDAR policy parameters; blocking query with result readback",
                      "points": n, "kernel_us": round(kern_s * 1e6, 2)},
           "roofline": {"bound": "hbm", "achieved": round(alg_bytes / kern_s / 1e9, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(alg_bytes / kern_s / 1e9 / HBM_PEAK_GBS, 4), "traffic": None,
                        "kernel": "scan_rmp_kernel", "algorithmic_bytes_per_launch": alg_bytes}}
    if not args.no_cpu_baseline:
        oracle.scan(pts, v, params)
        done, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < min(args.cpu_seconds, 5.0):
            oracle.scan(pts, v, params)
            done += 1
        el = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": done * n / el, "unit": "points/s", "cores": 1, "kind": "oracle",
                               "sample": f"{done} full frames ({el:.1f} s wall, float64 C oracle, one thread)"}
    ctx.close()
    print(json.dumps(out), flush=True)


def sparse_bench(args):
    """A sparse block map of an outdoor-sized world (160 m x 160 m of ground with 1,500 random
    obstacles at 0.05 m: ~0.48 M stored 8^3 blocks, where the dense grid would hold 2.6e9
    voxels): blocking 65,536-ray queries through the block hash, rays/s."""
    import numpy as np
    import torch
    import oracle
    from paper_2301_08068_amd import binding
    from paper_2301_08068_amd import workloads as W
    sm = W.sparse_world(20)
    x, v = W.sparse_free_state(sm, 700)
    n_rays, rmax = 65536, 10.0
    params = W.params("static", max_range=rmax)
    ctx = binding.Context(0, arena_bytes=(3 << 30) // 2)
    mid = ctx.upload_sparse(sm.coords, sm.values, sm.voxel_m, sm.origin_m, "f32", sm.trunc_m)
    over = {k: v for k, v in (("lookahead", args.lookahead), ("lane_target_log2", args.lane_target)) if v}
    launch = ctx.config(binding.CONFIG_SPARSE, **over)
    step = binding.PreparedQuery(ctx.ptr, mid, x, v, n_rays, params, stream=ctx.stream)
    for _ in range(args.warmup):
        step()
    visits = step().visits
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    binding.rmpc_set_profiling(ctx.ptr, True)
    for _ in range(max(args.steps, 100)):
        step()
    kms, nl = binding.rmpc_get_profile(ctx.ptr)
    binding.rmpc_set_profiling(ctx.ptr, False)
    ctx.close()
    kern_s = kms / 1e3 / max(nl, 1)
    alg_bytes = visits * 4 + 12 * n_rays
    out = {"metric": "rays/sec (raycast+RMP+resolve) at 65536 rays/query on a sparse block map",
           "value": n_rays * args.steps / el, "unit": "rays/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "160 m x 160 m world, 0.05 m voxels, ground + 1500 obstacles, sparse 8^3 blocks; "
                                  "65536 rays, 10 m",
                      "blocks": sm.n_blocks, "stored_voxels_occupied": round(sm.occupied_fraction(), 4),
                      "mean_visits_per_ray": round(visits / n_rays, 2), "kernel_us": round(kern_s * 1e6, 2),
                      "launch_lookahead": launch["lookahead"], "launch_lane_target_log2": launch["lane_target_log2"]},
           "roofline": {"bound": "hbm", "achieved": round(alg_bytes / kern_s / 1e9, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(alg_bytes / kern_s / 1e9 / HBM_PEAK_GBS, 4), "traffic": None,
                        "kernel": "sparse_rmp_kernel", "algorithmic_bytes_per_launch": alg_bytes}}
    if not args.no_cpu_baseline:
        # the oracle walks the same voxels expanded into a dense crop around the robot
        g = ((x - sm.origin_m) / sm.voxel_m).astype(np.float32)
        reach = int(np.ceil(rmax / sm.voxel_m)) + 16
        lo = (np.floor((g.astype(np.float64) - reach) / 8) * 8).astype(np.int64)
        hi = (np.ceil((g.astype(np.float64) + reach) / 8) * 8).astype(np.int64)
        dense, o_dense = sm.dense_crop(lo, hi)
        om = oracle.OracleMap(dense, sm.voxel_m, o_dense, "f32")
        dirs = oracle.directions(n_rays)
        gd = (g.astype(np.float64) - lo).astype(np.float32)
        cores = len(os.sched_getaffinity(0))
        oracle.trace(om, gd, dirs, rmax, nthreads=cores)
        done, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < min(args.cpu_seconds, 5.0):
            o = oracle.trace(om, gd, dirs, rmax, nthreads=cores)
            oracle.combine(params, dirs, o["d"], o["hit"], v)
            done += 1
        elc = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": done * n_rays / elc, "unit": "rays/s", "cores": cores, "kind": "oracle",
                               "sample": f"{done} full queries ({elc:.1f} s wall) of the float64 oracle on a dense "
                                         f"{dense.shape[2]}x{dense.shape[1]}x{dense.shape[0]} crop holding every "
                                         "voxel the rays can reach"}
    print(json.dumps(out), flush=True)


def edt_bench(args):
    """Exact distance transform of the 400^3 paper-shaped map's occupancy (rmpc_edt): the
    distance field of the ESDF policy, rebuilt after a map update."""
    import torch
    from paper_2301_08068_amd import binding
    from paper_2301_08068_amd import workloads as W
    vm = W.paper_map(2)
    ctx = binding.Context(0, arena_bytes=1 << 30)
    mid = ctx.upload(vm.tsdf, vm.voxel_m, vm.origin_m, "f32")
    out = torch.empty(vm.tsdf.shape, dtype=torch.int32, device="cuda:0")
    args_c = (binding.C.c_void_p(ctx.ptr), mid, binding.C.c_void_p(out.data_ptr()), binding.C.c_void_p(ctx.stream))
    for _ in range(min(args.warmup, 3)):
        binding._check(binding._lib.rmpc_edt(*args_c), "rmpc_edt")
    steps = min(args.steps, 20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        binding._check(binding._lib.rmpc_edt(*args_c), "rmpc_edt")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    n = vm.tsdf.size
    print(json.dumps({"metric": "distance-transform voxels/sec (exact squared EDT of the occupancy)",
                      "value": n * steps / el, "unit": "voxels/s", "n_gpus": 1, "steps": steps,
                      "warmup": min(args.warmup, 3), "ms_per_step": 1e3 * el / steps, "higher_is_better": True,
                      "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
                      "config": {"workload": "400^3 paper-shaped f32 map (0.05 m, map seed 2), 10.6 % occupied"}}),
          flush=True)
    ctx.close()


def serve_compare(n_requests, rates, slots, check_alone=True):
    """Serving: an open-loop Poisson stream of half grid-raycast requests (ray counts
    log-uniform in [4096, 65536]) and half 64 x 1024 LiDAR-scan requests (points staged from
    pinned host memory) over four resident maps (two 400^3 fp16 TSDF, two 256^3 u8
    occupancy), continuous batching over several launch slots against a one-request-per-launch
    server.  Returns one row per rate, the resident map bytes, the launch configuration and how
    many sampled results equal the result of the same request alone."""
    import numpy as np
    import torch
    from paper_2301_08068_amd import binding
    from paper_2301_08068_amd import workloads as W
    vms = [("f16", W.paper_map(10)), ("f16", W.paper_map(11)), ("u8", W.occ_source_map(12)),
           ("u8", W.occ_source_map(13))]
    ctx = binding.Context(0, arena_bytes=2 << 30)
    try:
        mids, resident = [], 0
        for enc, vm in vms:
            data = W.encode_f16(vm.tsdf) if enc == "f16" else W.encode_u8(vm.tsdf)
            resident += data.nbytes
            mids.append(ctx.upload(data, vm.voxel_m, vm.origin_m, enc))
        n_states, n_scans = 64, 2
        states = [[W.free_state(vm, 1000 * m + k) for k in range(n_states)] for m, (_, vm) in enumerate(vms)]
        scans = [[torch.from_numpy(W.synth_scan(vm, states[m][k][0], 600 + 10 * m + k)).pin_memory()
                  for k in range(n_scans)] for m, (_, vm) in enumerate(vms)]
        mp, sp = W.params("static", max_range=10.0), W.params("lidar")
        n = n_requests
        rng = np.random.default_rng(501)
        is_grid = rng.uniform(size=n) < 0.5
        m_idx = rng.integers(0, len(vms), size=n)
        s_idx = rng.integers(0, n_states, size=n)
        c_idx = rng.integers(0, n_scans, size=n)
        counts = W.ray_counts(n, seed=399)
        reqs, units = [], np.zeros(n)
        for j in range(n):
            m, (x, v) = int(m_idx[j]), states[int(m_idx[j])][int(s_idx[j])]
            if is_grid[j]:
                q = dict(kind="map", map_id=mids[m], n=int(counts[j]), x=x, v=v)
                reqs.append(binding.request(q))
                units[j] = counts[j]
            else:
                pts = scans[m][int(c_idx[j])]
                reqs.append(binding.request(dict(kind="scan", n=pts.shape[0], v=states[m][int(c_idx[j])][1]),
                                            pts.data_ptr()))
                units[j] = pts.shape[0]
        launch = ctx.config(binding.CONFIG_BATCH)
        scan_bytes = 12 * 65536
        modes = {
            "continuous": dict(n_slots=slots, max_batch=256, map_params=mp, scan_params=sp,
                               launch=launch, staging_bytes=64 * scan_bytes),
            "one_per_launch": dict(n_slots=1, max_batch=1, map_params=mp, scan_params=sp, launch=launch,
                                   staging_bytes=2 * scan_bytes),
        }
        rows = []
        for rate in rates:
            arrivals = W.poisson_arrivals(rate, n, seed=500)
            row = {"rate_req_s": rate}
            for name, kw in modes.items():
                row[name] = _serve_rate(binding, ctx, reqs, units, is_grid, arrivals, kw, max(64, min(n, rate // 20)))
                print(json.dumps({"progress": f"rate {rate} {name}", **row[name]}), file=sys.stderr, flush=True)
            rows.append(row)
        equal, sample = 0, []
        if check_alone:
            # equality with the alone result on a sample of the mix
            sample = list(range(0, n, max(1, n // 48)))[:48]
            binding.rmpc_server_start(ctx.ptr, **modes["continuous"])
            try:
                tks = [binding.rmpc_submit(ctx.ptr, reqs[j]) for j in sample]
                got = {}
                while len(got) < len(tks):
                    for t, r, _ in binding.rmpc_poll_completed(ctx.ptr, 64):
                        got[t] = r
            finally:
                binding.rmpc_server_stop(ctx.ptr)
            for t, j in zip(tks, sample):
                q = reqs[j].q
                if q.kind == binding.KIND_MAP:
                    alone = ctx.query_batch([dict(kind="map", map_id=q.map_id, n=q.n, x=list(q.x), v=list(q.v))],
                                            map_params=mp)[0]
                else:
                    m = int(m_idx[j])
                    alone = ctx.query_batch([dict(kind="scan", points=scans[m][int(c_idx[j])].cuda(), v=list(q.v))],
                                            scan_params=sp)[0]
                equal += int(np.array_equal(got[t]["f"], alone["f"]) and np.array_equal(got[t]["S"], alone["S"]))
    finally:
        ctx.close()
    return {"rows": rows, "resident_map_bytes": resident, "launch": launch,
            "sample_equal_alone": f"{equal}/{len(sample)}"}


def serve_bench(args):
    """The serving loop as its own bench line (four rates, args.serve_requests each)."""
    r = serve_compare(args.serve_requests, SERVE_RATES, args.serve_slots)
    rows = r["rows"]
    top = rows[-1]["continuous"]
    n = args.serve_requests
    out = {"metric": METRIC, "value": top["evals_per_s"], "unit": "ray-policy evaluations/s (grid rays + scan points)",
           "n_gpus": 1, "steps": n, "warmup": 64, "ms_per_step": None, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f16/u8 maps, f32 sums, f64 resolve",
           "data": "synthetic",
           "config": {"workload": f"Poisson arrivals at {list(SERVE_RATES)} req/s, {n} requests each; 50 % grid "
                                  "queries (rays log-uniform in [4096, 65536]) and 50 % 64x1024 LiDAR scans "
                                  "(pinned host points, staged by the server); 4 resident maps (two 400^3 fp16 "
                                  "TSDF, two 256^3 u8 occupancy)",
                      "resident_map_bytes": r["resident_map_bytes"], "launch": r["launch"], "slots": args.serve_slots,
                      "rates": rows, "sample_equal_alone": r["sample_equal_alone"]}}
    print(json.dumps(out), flush=True)


def rollout_bench(args):
    """Closed-loop flights (ray policy + goal attractor, 1 kHz policy steps) across 10 m cubes
    of random obstacles at three clutter levels (after Sec. IV-A), for ray counts 4^2 .. 64^2,
    every flight of a clutter level advanced together by rmpc_rollout_batch (one launch per
    step): success rate (goal reached without collision), smoothness of the successful paths
    sampled at 100 Hz, and time per batched step."""
    import numpy as np
    from paper_2301_08068_amd import binding
    from paper_2301_08068_amd import workloads as W
    params = W.params("static")
    alpha, beta, dt, horizon_s, tol, every = 10.0, 15.0, 0.001, args.rollout_horizon, 0.2, 10
    n_ref = 4.0     # averaged reading: ray sums times n_ref / N
    max_steps = int(round(horizon_s / dt))
    rays = [int(r) for r in args.rollout_rays.split(",")]
    n_maps = max(1, args.rollouts // 4)
    per_map = max(1, args.rollouts // n_maps)
    ctx = binding.Context(0, arena_bytes=1 << 30)
    rows = []
    for n_prims in (50, 100, 200):
        maps, occ = [], []
        for j in range(n_maps):
            vm = W.eval_map(7000 + 100 * n_prims + j, n_prims)
            maps.append((ctx.upload(vm.tsdf, vm.voxel_m, vm.origin_m, "f32"),
                         [W.eval_pair(vm, 50 * j + k) for k in range(per_map)]))
            occ.append(vm.occupied_fraction())
        # the ray sums as the paper writes them (weight 1), and averaged over the rays with
        # n_ref times the attractor's weight (weight n_ref / N)
        cases = [("as_written", n, 1.0) for n in rays] + [("averaged", n, n_ref / n) for n in rays]
        flights, tags = [], []
        for weighting, n, w in cases:
            for mid, pairs in maps:
                for x0, goal in pairs:
                    flights.append(dict(map_id=mid, n_rays=n, x0=x0, v0=np.zeros(3), goal=goal, alpha=alpha,
                                        beta=beta, dt=dt, max_steps=max_steps, goal_tol=tol, ray_weight=w,
                                        smooth_every=every))
                    tags.append((weighting, n))
        # launch configuration of the per-step batches, tuned on the batch of the start states
        tuned = binding.rmpc_tune_batch(ctx.ptr, binding.query_descs(
            [dict(kind="map", map_id=f["map_id"], n=f["n_rays"], x=f["x0"], v=f["v0"]) for f in flights]),
            params, None, stream=ctx.stream)
        t0 = time.perf_counter()
        res = ctx.rollout_batch(flights, params)
        el = time.perf_counter() - t0
        launches = max(r["n_steps"] for r in res) + 1
        for weighting, n, _ in cases:
            rs = [r for r, t in zip(res, tags) if t == (weighting, n)]
            ok = [r for r in rs if r["status"] == binding.ROLLOUT_GOAL]
            row = {"obstacles": n_prims, "ray_weighting": weighting, "rays": n, "flights": len(rs),
                   "success_rate": len(ok) / len(rs),
                   "collisions": sum(r["status"] == binding.ROLLOUT_COLLISION for r in rs),
                   "left_grid": sum(r["status"] == binding.ROLLOUT_LEFT_GRID for r in rs),
                   "timeouts": sum(r["status"] == binding.ROLLOUT_TIMEOUT for r in rs),
                   "smoothness_mean": float(np.mean([r["smoothness"] for r in ok])) if ok else None,
                   "smoothness_p10": float(np.percentile([r["smoothness"] for r in ok], 10)) if ok else None,
                   "flight_time_s_mean": float(np.mean([r["n_steps"] * dt for r in ok])) if ok else None}
            rows.append(row)
            print(json.dumps({"progress": row}), file=sys.stderr, flush=True)
        level = {"obstacles": n_prims, "occupied_fraction_mean": float(np.mean(occ)), "flights": len(flights),
                 "batch_config": tuned,
                 "batched_steps": launches, "ms_per_batched_step": 1e3 * el / launches,
                 "flight_steps_per_s": sum(r["n_steps"] for r in res) / el}
        rows.append(level)
        print(json.dumps({"progress": level}), file=sys.stderr, flush=True)
        for mid, _ in maps:
            ctx.release(mid)
    ctx.close()
    head = [r for r in rows if r.get("rays") == 1024 and r.get("ray_weighting") == "averaged"]
    lv = [r for r in rows if "batched_steps" in r]
    out = {"metric": "closed-loop rollout success rate (1024 rays per query, averaged ray sums, "
                     "mean over 50/100/200 obstacles)",
           "value": float(np.mean([r["success_rate"] for r in head])) if head else None,
           "unit": "fraction of flights reaching the goal",
           "n_gpus": 1, "steps": int(sum(r["batched_steps"] for r in lv)), "warmup": 0,
           "ms_per_step": float(np.mean([r["ms_per_batched_step"] for r in lv])),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"{n_maps} seeded 10 m cubes (200^3 f32 voxels of 0.05 m) per clutter level of "
                                  f"50/100/200 random spheres and boxes, {per_map} start/goal pairs per map on "
                                  "opposite faces with 0.3 m clearance; static-map policy parameters, attractor "
                                  f"alpha {alpha}, beta {beta}; dt {dt} s, at most {horizon_s} s of flight, goal "
                                  f"radius {tol} m, smoothness on states every {every} steps; ray sums as written "
                                  f"and averaged (weight {n_ref:g}/N); one batched launch per step for all flights "
                                  "of a clutter level", "per_ray_count": rows}}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--config", default="paper", choices=sorted(CONFIGS) + ["batch", "serve", "rollout", "scan_os0", "edt", "sparse"])
    ap.add_argument("--rollouts", type=int, default=32,
                    help="rollout config: flights per clutter level and ray count")
    ap.add_argument("--rollout-horizon", type=float, default=90.0,
                    help="rollout config: seconds of flight before a timeout")
    ap.add_argument("--rollout-rays", default="16,64,256,1024,4096",
                    help="rollout config: comma-separated rays per query")
    ap.add_argument("--serve-requests", type=int, default=20000)
    ap.add_argument("--serve-slots", type=int, default=3)
    ap.add_argument("--lookahead", type=int, default=0, help="query launch: steps planned per round (4, 8, 16)")
    ap.add_argument("--lane-target", type=int, default=0, help="query launch: log2 of the lanes a query aims for")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="paper config: skip the batched-vs-plain and served-latency passes")
    ap.add_argument("--extras-requests", type=int, default=2000,
                    help="paper config: requests per rate of the served-latency pass")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device copy of this many bytes 20 times (counter "
                         "calibration for HBM traffic) and exit")
    args = ap.parse_args()
    if args.copy_bytes:
        import torch
        a = torch.ones(args.copy_bytes // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(20):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_bytes, "launches": 20}), flush=True)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the query path runs on a single MI355X and has no "
              "multi-GPU form (queries shard by state; see the design notes).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2301_08068_amd import build as lib_build
    if not os.path.exists(lib_build.LIB):
        lib_build.build()
    from paper_2301_08068_amd import binding
    from paper_2301_08068_amd import workloads as W
    if args.config == "batch":
        batch_bench(args)
        return
    if args.config == "serve":
        serve_bench(args)
        return
    if args.config == "edt":
        edt_bench(args)
        return
    if args.config == "sparse":
        sparse_bench(args)
        return
    if args.config == "scan_os0":
        scan_bench(args)
        return
    if args.config == "rollout":
        rollout_bench(args)
        return

    kind, enc, seed, n_rays, rmax, *rest = CONFIGS[args.config]
    subvoxel = rest[0] if rest else 0
    vm, data = build_map(kind, enc)
    x, v = W.free_state(vm, seed)
    params = W.params("static", max_range=rmax, subvoxel=subvoxel)

    ctx = binding.Context(0, arena_bytes=1 << 30)
    mid = ctx.upload(data, vm.voxel_m, vm.origin_m, enc)
    over = {k: v for k, v in (("lookahead", args.lookahead), ("lane_target_log2", args.lane_target)) if v}
    launch = ctx.config(binding.CONFIG_QUERY, **over)
    step = binding.PreparedQuery(ctx.ptr, mid, x, v, n_rays, params, stream=ctx.stream)
    for _ in range(args.warmup):
        step()
    visits = step().visits

    # the timed steps: blocking queries as a caller makes them (no profiling events)
    lat = [0.0] * args.steps
    clock = time.perf_counter
    torch.cuda.synchronize()
    t0 = clock()
    for k in range(args.steps):
        ts = clock()
        step()
        lat[k] = clock() - ts
    torch.cuda.synchronize()
    elapsed = clock() - t0
    # kernel duration: a separate pass with each dispatch's own start/stop events
    binding.rmpc_set_profiling(ctx.ptr, True)
    for _ in range(max(args.steps, 100)):
        step()
    kms, nl = binding.rmpc_get_profile(ctx.ptr)
    binding.rmpc_set_profiling(ctx.ptr, False)
    ctx.close()

    kern_s = kms / 1e3 / max(nl, 1)
    alg_bytes = visits * ELEM_BYTES[enc] + 12 * n_rays
    achieved = alg_bytes / kern_s / 1e9
    traffic = measured_traffic() if args.config == "paper" else None
    l2 = measured_l2() if args.config == "paper" else None
    lat_us = sorted(1e6 * t for t in lat)
    shape = "400^3 0.05 m, 200 primitives + walls, seed 2" if kind == "paper" else "64^3 0.1 m, 20 spheres + floor, seed 1"
    config = {
        "workload": f"{shape}; {enc} map; 1 state (seed {seed}); {n_rays} Halton rays, {rmax:g} m; blocking query",
        "rays_per_query": n_rays,
        "map_storage": enc,
        "subvoxel_distances": bool(subvoxel),
        "occupied_fraction": round(vm.occupied_fraction(), 4),
        "mean_visits_per_ray": round(visits / n_rays, 2),
        "latency_p50_us": round(lat_us[len(lat_us) // 2], 1),
        "latency_p99_us": round(lat_us[min(len(lat_us) - 1, int(0.99 * len(lat_us)))], 1),
        "kernel_us": round(kern_s * 1e6, 2),
        "kernel_launches_timed": nl,
        "launch_lookahead": launch["lookahead"],
        "launch_lane_target_log2": launch["lane_target_log2"],
    }
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "kernel": "raycast_rmp_kernel",
                "algorithmic_bytes_per_launch": alg_bytes,
                "limiter": "latency: the dependent round chain of the slowest waves, then the reduction tail"}
    if l2 is not None:
        req, hit_rate = l2
        roofline["l2_bytes_per_launch"] = int(req * L2_LINE_BYTES)
        roofline["l2_gbs"] = round(req * L2_LINE_BYTES / kern_s / 1e9, 1)
        roofline["l2_hit_rate"] = hit_rate
    if args.config == "paper" and not args.no_extras:
        # the metric's second half: the batched form against the plain path, and served p50/p99
        b = batch_compare(steps=5, warmup=2)
        config["batch_states"] = b["states"]
        config["batch_rays_per_s"] = round(b["batch_rays_per_s"])
        config["plain_rays_per_s"] = round(b["plain_rays_per_s"])
        config["batch_over_plain"] = round(b["batch_rays_per_s"] / b["plain_rays_per_s"], 2)
        sv = serve_compare(args.extras_requests, (2000, 20000, 40000), args.serve_slots, check_alone=True)
        for row in sv["rows"]:
            r = row["rate_req_s"]
            for mode, tag in (("continuous", "served"), ("one_per_launch", "one_per_launch")):
                m = row[mode]
                config[f"{tag}_{r}_p50_ms"] = m["p50_ms"]
                config[f"{tag}_{r}_p99_ms"] = m["p99_ms"]
                if mode == "continuous":
                    config[f"{tag}_{r}_mean_batch"] = m["mean_batch"]
                    config[f"{tag}_{r}_evals_per_s"] = round(m["evals_per_s"])
        config["served_requests_per_rate"] = args.extras_requests
        config["served_equal_alone"] = sv["sample_equal_alone"]
    out = {
        "metric": METRIC,
        "value": n_rays * args.steps / elapsed,
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": config,
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(vm, data, enc, x, v, n_rays, params, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
