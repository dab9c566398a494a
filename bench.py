"""Benchmark: P-NDF queries/s on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload powerlaw2048]
                    [--algo plain|brute] [--no-cpu-baseline] [--no-octaves]

A step is one pndf_eval_batch over the whole query batch (queries and the mesh /
hierarchy already resident in HBM).  Prints one JSON line.

Roofline: the dominant (and only) kernel of a step is the evaluation kernel.  Its
work is counted per query by an instrumented launch (nodes, leaf cells, clusters,
hits) and priced two ways:
    bytes it must read   B = 28 + (16 + 4 [tau > 0]) nodes + 9 cells + 41 clusters + 4 hits
    vector ALU lane-ops  F = 12 nodes + 40 cells + 40 clusters + 30 hits
The kernel's counters show it issue-bound on the vector ALU (about 90 % VALU busy),
so `roofline` is the ALU one: F per launch over the launch time, against 256 CUs x
64 lanes x 2.4 GHz = 39.3 T lane-ops/s (one 32-bit operation per lane per clock,
no packed-FP32 or FMA double counting); `roofline_hbm` gives B against 8 TB/s.
The duration is measured with HIP events on the stream the kernel runs on.  HBM
traffic comes from rocprofv3 FETCH_SIZE / WRITE_SIZE runs recorded under profiles/
(null when the kernel source changed since they were taken).
"""
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

METRIC = "P-NDF queries/sec at 1 MI355X vs footprint size; p99 tile latency (serving)"
HBM_PEAK_GBS = 8000.0
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12   # 32-bit lane operations per second, in T
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_eval_plain_powerlaw2048.json")
EVAL_SRC = ("eval.hip", "pndf_internal.h")
SAMPLE_SRC = ("sample.hip", "pndf_internal.h")
SAMPLE_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_sample_powerlaw2048.json")


def kernel_hash(files=EVAL_SRC):
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_2505_08985_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def algorithmic_ops(counts):
    c = counts.astype(np.float64)
    return float(np.sum(12.0 * c[:, 0] + 40.0 * c[:, 1] + 40.0 * c[:, 2] + 30.0 * c[:, 3]))


def algorithmic_bytes(counts, tau):
    c = counts.astype(np.float64)
    per_node = 16.0 + (4.0 if tau > 0 else 0.0)
    return float(np.sum(28.0 + per_node * c[:, 0] + 9.0 * c[:, 1] + 41.0 * c[:, 2] + 4.0 * c[:, 3]))


def load_traffic(workload, algo, kernel="gaussian", sigma_to_r=3.0, queries=None):
    """The measured HBM bytes per launch, if the committed counters were taken on this
    source and this exact launch: the workload's own batch at the default support."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    try:
        t = json.load(open(TRAFFIC_FILE))
    except Exception:
        return None
    import workloads
    if (t.get("kernel_hash") != kernel_hash() or t.get("workload") != workload or t.get("algo") != algo
            or t.get("kernel", "gaussian") != kernel or sigma_to_r != 3.0
            or queries != workloads.CONFIGS[workload]["queries"]["count"]):
        return None
    return float(t["hbm_bytes_per_launch"])


def cpu_baseline(nrm, q, tau, budget_s=15.0, kernel="gaussian", sigma_to_r=3.0):
    """The FP64 oracle, as it stands, on a bounded prefix of the same (randomly
    ordered) query stream, all host threads."""
    import oracle
    oracle.load()
    threads = oracle.num_threads()
    k = 256
    t0 = time.perf_counter()
    oracle.evaluate(nrm, q[:k], tau=tau, kernel=kernel, sigma_to_r=sigma_to_r)
    dt = time.perf_counter() - t0
    k2 = int(min(len(q), max(k, budget_s / max(dt, 1e-6) * k)))
    t0 = time.perf_counter()
    oracle.evaluate(nrm, q[:k2], tau=tau, kernel=kernel, sigma_to_r=sigma_to_r)
    dt2 = time.perf_counter() - t0
    return {"value": k2 / dt2, "unit": "queries/s", "cores": threads, "kind": "oracle",
            "sample": "first %d queries of the same seeded stream (%.1f s, FP64 brute force over "
                      "every included cell)" % (k2, dt2)}


SERVE_MAPS = (dict(kind="bumps", n=1024, seed=411, count=8192),
              dict(kind="scratched", n=4096, seed=301),
              dict(kind="powerlaw", n=8192, seed=501, rms_slope=0.15))


def serve_bench(args):
    """Serving workload: Poisson arrivals of render tiles (64 x 64 px x 4 spp) over three
    resident maps, footprints from synthetic ray differentials; continuous batching
    (per-batch launches or persistent plans on concurrent streams) against FIFO per-tile plain evaluation,
    at fractions of the plain per-tile throughput."""
    import torch
    import paper_2505_08985_amd as P
    import workloads
    tau = args.serve_tau
    hiers, ns = [], []
    t0 = time.perf_counter()
    for mc in SERVE_MAPS:
        nrm = workloads.make_map(**mc)
        mesh = P.build_mesh(torch.from_numpy(nrm).cuda())
        hiers.append(P.build_hierarchy(mesh, cluster=True))
        ns.append(mc["n"])
        del nrm
        torch.cuda.synchronize()
        print("[serve] map %s %d^2 resident (%.1f s)" % (mc["kind"], mc["n"], time.perf_counter() - t0),
              file=sys.stderr, flush=True)
    rng = np.random.default_rng(401)
    ntiles = args.serve_tiles
    mids = rng.integers(0, len(SERVE_MAPS), ntiles)
    smax = args.serve_sigma_max
    tiles = [workloads.tile_request(ns[m], int(rng.integers(1 << 30)), sigma_range=(0.5, smax)) for m in mids]
    # plain per-tile cost (each tile alone, synchronised)
    dq = [torch.from_numpy(t).cuda() for t in tiles]
    for m, q in zip(mids[:4], dq[:4]):
        P.eval_batch(hiers[m], q, tau=tau)
    torch.cuda.synchronize()
    cost = []
    for k, (m, q) in enumerate(zip(mids, dq)):
        a = time.perf_counter()
        P.eval_batch(hiers[m], q, tau=tau)
        torch.cuda.synchronize()
        cost.append(time.perf_counter() - a)
        if k % 10 == 9:
            print("[serve] plain per-tile: %d tiles timed" % (k + 1), file=sys.stderr, flush=True)
    cost = np.array(cost)
    plain_tiles_per_s = ntiles / cost.sum()
    print("[serve] plain per-tile: %.2f tiles/s (median tile %.2f ms, max %.1f ms)"
          % (plain_tiles_per_s, 1e3 * np.median(cost), 1e3 * cost.max()), file=sys.stderr, flush=True)
    qpt = tiles[0].shape[0]
    # persistent per-tile cost (one plan per map, default tuning), each tile alone
    plans = [P.Plan(h, qpt, tau=tau) for h in hiers]
    for m, q in zip(mids[:4], dq[:4]):
        plans[m].eval(q)
    torch.cuda.synchronize()
    cost_p = []
    for m, q in zip(mids, dq):
        a = time.perf_counter()
        plans[m].eval(q)
        torch.cuda.synchronize()
        cost_p.append(time.perf_counter() - a)
    cost_p = np.array(cost_p)
    del plans
    print("[serve] persistent per-tile: %.2f tiles/s (median tile %.2f ms, max %.1f ms)"
          % (ntiles / cost_p.sum(), 1e3 * np.median(cost_p), 1e3 * cost_p.max()), file=sys.stderr, flush=True)
    results = []
    srv = P.Server(hiers, slots=args.serve_slots, max_batch_queries=qpt * args.serve_batch_tiles,
                   max_pending=4 * ntiles, tau=tau, algo=args.serve_algo)
    srv.replay(mids[:4], np.zeros(4), tiles[:4])  # warm-up
    for frac in [float(f) for f in args.serve_rates.split(",")]:
        rate = frac * plain_tiles_per_s
        arr = np.cumsum(rng.exponential(1.0 / rate, ntiles))
        arr -= arr[0]
        # FIFO per-tile plain / persistent evaluation at the same arrivals (simulated
        # from the measured costs)
        def fifo(cst):
            free, lat_f = 0.0, []
            for a, c in zip(arr, cst):
                start = max(a, free)
                free = start + c
                lat_f.append(1e3 * (free - a))
            return lat_f, free
        lat_fifo, free = fifo(cost)
        lat_fifo_p, _ = fifo(cost_p)
        srv.reset_stats()
        a = time.perf_counter()
        outs, lat = srv.replay(mids, arr, tiles)
        wall = time.perf_counter() - a
        st = srv.stats()
        results.append({"rate_frac": frac, "tiles_per_s_offered": rate,
                        "served_queries_per_s": ntiles * qpt / wall,
                        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                        "mean_batch_tiles": st["mean_batch_requests"],
                        "fifo_plain_p50_ms": float(np.percentile(lat_fifo, 50)),
                        "fifo_plain_p99_ms": float(np.percentile(lat_fifo, 99)),
                        "fifo_plain_queries_per_s": ntiles * qpt / max(free, arr[-1]),
                        "fifo_persistent_p50_ms": float(np.percentile(lat_fifo_p, 50)),
                        "fifo_persistent_p99_ms": float(np.percentile(lat_fifo_p, 99))})
        print("[serve] %s" % json.dumps(results[-1]), file=sys.stderr, flush=True)
    # saturation throughput: everything arrives at once
    srv.reset_stats()
    a = time.perf_counter()
    srv.replay(mids, np.zeros(ntiles), tiles)
    sat = ntiles * qpt / (time.perf_counter() - a)
    srv.close()
    line = {"metric": METRIC, "value": sat, "unit": "queries/s", "n_gpus": 1, "steps": ntiles,
            "warmup": 4, "ms_per_step": 1e3 * qpt / sat, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "serving: Poisson 64x64x4 tiles over bumps1024 / scratched4096 / "
                                   "powerlaw8192", "tau": tau, "sigma_range": [0.5, smax],
                       "slots": args.serve_slots, "batch_tiles": args.serve_batch_tiles,
                       "batch_algo": args.serve_algo},
            "plain_per_tile_queries_per_s": plain_tiles_per_s * qpt,
            "persistent_per_tile_queries_per_s": ntiles * qpt / cost_p.sum(),
            "per_tile_ms": {"plain_median": 1e3 * float(np.median(cost)), "plain_max": 1e3 * float(cost.max()),
                            "persistent_median": 1e3 * float(np.median(cost_p)),
                            "persistent_max": 1e3 * float(cost_p.max())},
            "by_rate": results}
    print(json.dumps(line), flush=True)


def sample_bench(args):
    """Sampling throughput: one P-NDF sample per query of the workload's query
    stream (pndf_sample_batch), uniforms drawn on the device beforehand."""
    import torch
    import paper_2505_08985_amd as P
    import workloads
    cfg = workloads.CONFIGS[args.workload]
    mc, qc = cfg["map"], cfg["queries"]
    tau = args.sample_tau
    n = mc["n"]
    kern = args.kernel
    s2r = args.sigma_to_r if args.sigma_to_r is not None else (3.0 if kern == "gaussian" else 1.5)
    count = args.queries or (1 << 24)
    nrm = workloads.make_map(**mc)
    q = workloads.uniform_queries(n, count, qc["seed"], qc["sigma"], qc["radius"])
    print("[bench] sampling on %s: map %d^2, %d samples, tau %g, %s" % (args.workload, n, count, tau, kern),
          file=sys.stderr, flush=True)
    torch.cuda.set_device(0)
    mesh = P.build_mesh(torch.from_numpy(nrm).cuda())
    hier = P.build_hierarchy(mesh, cluster=tau > 0)
    tq = torch.from_numpy(q).cuda()
    g = torch.Generator(device="cuda")
    g.manual_seed(1)
    attempts = 2 if tau > 0 else 1
    xi = torch.rand((attempts, count, 2), dtype=torch.float64, device="cuda", generator=g)
    m = torch.empty((count, 2), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        P.sample_batch(hier, tq, xi, tau=tau, sigma_to_r=s2r, kernel=kern, tri=False, m=m)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = ev0.elapsed_time(ev1) / args.steps
    mm = m.cpu().numpy()
    assert np.isfinite(mm).mean() > 0.999
    # algorithmic bytes per sample: query 24, one uniform pair 16, the sample 8, the
    # unit's four corner normals 32 and clamp byte 1; with the cut, 4 per residual read
    # (entry level down to the unit) and 1 for the cluster clamp byte instead
    _, tri, _ = P.sample_batch(hier, tq, xi, tau=tau, sigma_to_r=s2r, kernel=kern)
    lev = (tri.cpu().numpy().view(np.uint64) >> np.uint64(58)).astype(np.int64)
    per = 81.0
    if tau > 0:
        rmax = np.maximum(q[:, 2], q[:, 3]).astype(np.float64) * s2r
        l0 = np.minimum(np.ceil(np.log2(np.maximum(rmax, 1.0))), int(np.log2(n)))
        valid = lev >= 0
        per += float(4.0 * np.mean(np.where(lev > 0, l0 - lev + 1, l0)[valid]))
    abytes = per * count
    achieved = abytes / (kernel_ms * 1e-3) / 1e9
    traffic = None
    try:
        t = json.load(open(SAMPLE_TRAFFIC_FILE))
        if (t.get("kernel_hash") == kernel_hash(SAMPLE_SRC) and t.get("samples") == count and tau == 0
                and kern == "gaussian" and args.workload == "powerlaw2048"):
            traffic = float(t["hbm_bytes_per_launch"])
    except (OSError, ValueError, KeyError):
        pass
    line = {"metric": "P-NDF samples/sec at 1 MI355X", "value": count * args.steps / wall, "unit": "samples/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": args.workload + " sampling", "map": "%s %dx%d" % (mc["kind"], n, n),
                       "samples": count, "tau": tau, "kernel": kern, "sigma_to_r": s2r, "attempts": attempts},
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
            "kernel_ms": kernel_ms, "algorithmic_bytes_per_sample": per,
            "cluster_share": float((lev > 0).mean())}
    print(json.dumps(line), flush=True)


FP64_PEAK_TFLOPS = 78.6
# FP64 operations per triangle of the projected area's fast path (triangle inside
# the visible region): rotation 12, visibility tests 24, three boundary segments of
# ~40 each (asin and sqrt counted as one operation), kernel weight 20, sum 4
PROJ_OPS_PER_TRIANGLE = 180.0


def projarea_bench(args):
    """Projected area P(w) (pndf_projected_area, brute force): footprints
    log-uniform in [1, 8] texels on the workload's map, directions uniform on the
    hemisphere."""
    import torch
    import paper_2505_08985_amd as P
    import workloads
    cfg = workloads.CONFIGS[args.workload]
    mc, qc = cfg["map"], cfg["queries"]
    n = mc["n"]
    kern = args.kernel
    s2r = args.sigma_to_r if args.sigma_to_r is not None else (3.0 if kern == "gaussian" else 1.5)
    count = args.queries or (1 << 16)
    nrm = workloads.make_map(**mc)
    q = workloads.uniform_queries(n, count, qc["seed"], (1.0, 8.0), qc["radius"])
    rng = np.random.default_rng(7)
    z = rng.uniform(0, 1, count)
    ph = rng.uniform(0, 2 * np.pi, count)
    r = np.sqrt(1 - z * z)
    q[:, 4] = (r * np.cos(ph)).astype(np.float32)
    q[:, 5] = (r * np.sin(ph)).astype(np.float32)
    # keep |w_xy| <= 1 after rounding to float32 (|w_xy| > 1 is an invalid direction)
    over = (q[:, 4].astype(np.float64) ** 2 + q[:, 5].astype(np.float64) ** 2) > 1.0
    q[over, 4:6] *= np.float32(1.0 - 2.0 ** -22)
    print("[bench] projected area on %s: map %d^2, %d queries, sigma 1-8, %s" % (args.workload, n, count, kern),
          file=sys.stderr, flush=True)
    torch.cuda.set_device(0)
    mesh = P.build_mesh(torch.from_numpy(nrm).cuda())
    hier = P.build_hierarchy(mesh, cluster=False)
    tq = torch.from_numpy(q).cuda()
    stream = torch.cuda.current_stream()

    def step():
        return P.projected_area(hier, tq, sigma_to_r=s2r, kernel=kern)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        out = step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = ev0.elapsed_time(ev1) / args.steps
    assert np.isfinite(out.cpu().numpy()).all()
    # triangles per query: two per included cell
    rx = np.float32(s2r) * q[:, 2]
    ry = np.float32(s2r) * q[:, 3]
    nx = np.floor(q[:, 0] + rx) - (np.ceil(q[:, 0] - rx) - 1) + 1
    ny = np.floor(q[:, 1] + ry) - (np.ceil(q[:, 1] - ry) - 1) + 1
    tris = float((2.0 * nx * ny).sum())
    achieved = tris * PROJ_OPS_PER_TRIANGLE / (kernel_ms * 1e-3) / 1e12
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        k = 256
        t1 = time.perf_counter()
        oracle.projected_area(nrm, q[:k], sigma_to_r=s2r, kernel=kern)
        dt = time.perf_counter() - t1
        k2 = int(min(count, max(k, 10.0 / max(dt, 1e-6) * k)))
        t1 = time.perf_counter()
        oracle.projected_area(nrm, q[:k2], sigma_to_r=s2r, kernel=kern)
        dt2 = time.perf_counter() - t1
        cpu = {"value": k2 / dt2, "unit": "queries/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": "first %d queries (%.1f s, FP64 brute force)" % (k2, dt2)}
    line = {"metric": "P-NDF projected areas/sec at 1 MI355X", "value": count * args.steps / wall,
            "unit": "queries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": 1e3 * wall / args.steps, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": args.workload + " projected area", "map": "%s %dx%d" % (mc["kind"], n, n),
                       "queries": count, "sigma": [1.0, 8.0], "kernel": kern, "sigma_to_r": s2r},
            "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None},
            "cpu_baseline": cpu, "kernel_ms": kernel_ms, "triangles_per_query": tris / count}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="powerlaw2048")
    ap.add_argument("--algo", default="plain")
    ap.add_argument("--queries", type=int, default=0, help="override the batch size")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-octaves", action="store_true")
    ap.add_argument("--input-order", action="store_true", help="keep the query order (no spatial ordering)")
    ap.add_argument("--tuning", default=None, metavar="BPC,SPLIT",
                    help="persistent tuning (blocks per CU, split level) instead of autotuning")
    ap.add_argument("--autotune", action="store_true",
                    help="autotune the persistent plan (default: the plan's default tuning)")
    ap.add_argument("--autotune-queries", type=int, default=1 << 14,
                    help="size of the autotuning sample (a prefix of the batch); a sample much smaller "
                         "than the batch is dominated by its slowest queries and favours fewer workers")
    ap.add_argument("--kernel", default="gaussian", choices=["gaussian", "disk", "box"],
                    help="footprint kernel")
    ap.add_argument("--sigma-to-r", type=float, default=None,
                    help="support half-width in sigma (default 3 for gaussian, 1.5 for disk and box)")
    ap.add_argument("--serve", action="store_true", help="serving benchmark (continuous batching)")
    ap.add_argument("--sample", action="store_true", help="sampling benchmark (pndf_sample_batch)")
    ap.add_argument("--sample-tau", type=float, default=0.0)
    ap.add_argument("--projarea", action="store_true", help="projected-area benchmark (pndf_projected_area)")
    ap.add_argument("--serve-tau", type=float, default=1e-3)
    ap.add_argument("--serve-tiles", type=int, default=200)
    ap.add_argument("--serve-sigma-max", type=float, default=4096.0)
    ap.add_argument("--serve-rates", default="0.5,0.8,0.95")
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-batch-tiles", type=int, default=4)
    ap.add_argument("--serve-algo", default="plain", choices=["plain", "persistent"],
                    help="how the server evaluates a batch")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB (3 times), to scale the "
                         "FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (queries are "
              "independent and would shard by batch, each GPU holding the whole map and hierarchy)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calibrate_copy:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": nbytes, "copies": 3}), flush=True)
        return
    if args.serve:
        serve_bench(args)
        return
    if args.sample:
        sample_bench(args)
        return
    if args.projarea:
        projarea_bench(args)
        return
    import paper_2505_08985_amd as P
    import workloads

    kern = args.kernel
    s2r = args.sigma_to_r if args.sigma_to_r is not None else (3.0 if kern == "gaussian" else 1.5)
    kw = dict(kernel=kern, sigma_to_r=s2r)
    cfg = workloads.CONFIGS[args.workload]
    mc, qc, tau = cfg["map"], cfg["queries"], float(cfg["tau"])
    n = mc["n"]
    t0 = time.perf_counter()
    nrm = workloads.make_map(**mc)
    count = args.queries or qc["count"]
    q = workloads.uniform_queries(n, count, qc["seed"], qc["sigma"], qc["radius"])
    gen_s = time.perf_counter() - t0
    print("[bench] workload %s: map %d^2, %d queries (generated in %.1f s)" % (args.workload, n, count, gen_s),
          file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    dev_map = torch.from_numpy(nrm).cuda()
    t0 = time.perf_counter()
    mesh = P.build_mesh(dev_map)
    hier = P.build_hierarchy(mesh, cluster=True)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    del dev_map
    tq = torch.from_numpy(q).cuda()
    out = torch.empty(count, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    tuning = None
    if args.algo == "persistent":
        if args.tuning:
            bpc, split = (int(v) for v in args.tuning.split(","))
            tuning = dict(blocks_per_cu=bpc, split_level=split, queue_factor=16, use_graph=1)
        elif args.autotune:
            sample = tq[:min(count, args.autotune_queries)]
            print("[bench] autotuning on %d queries ..." % sample.shape[0], file=sys.stderr, flush=True)
            tuning, tms = P.autotune(hier, sample, tau=tau, **kw)
            print("[bench] autotuned %s (%.3f ms on %d queries)" % (tuning, tms, sample.shape[0]),
                  file=sys.stderr, flush=True)
        plan = P.Plan(hier, count, tau=tau, tuning=tuning, **kw)
        tuning = plan.tuning()
        print("[bench] plan tuning %s" % tuning, file=sys.stderr, flush=True)

        def step():
            plan.eval(tq, out=out)
    else:
        def step():
            P.eval_batch(hier, tq, tau=tau, algo=args.algo, out=out, input_order=args.input_order, **kw)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = ev0.elapsed_time(ev1) / args.steps
    print("[bench] timed %d steps: %.3f ms/step (events %.3f ms)" % (args.steps, 1e3 * wall / args.steps,
                                                                     kernel_ms), file=sys.stderr, flush=True)
    value = count * args.steps / wall
    d = out.cpu().numpy()
    assert np.isfinite(d).all() and (d >= 0).all()

    if args.algo == "persistent":
        st = plan.stats()
        assert st["error"] == 0, st
        ref = P.eval_batch(hier, tq, tau=tau, **kw)
        assert torch.equal(ref.view(torch.int32), out.view(torch.int32)), "persistent != plain"
    # instrumented launch: work units for the algorithmic byte count
    _, counts = P.eval_counts(hier, tq, tau=tau, algo="brute" if args.algo == "brute" else "plain", **kw)
    counts = counts.cpu().numpy()
    abytes = algorithmic_bytes(counts, tau)
    achieved = abytes / (kernel_ms * 1e-3) / 1e9
    aops = algorithmic_ops(counts)
    achieved_ops = aops / (kernel_ms * 1e-3) / 1e12
    traffic = load_traffic(args.workload, args.algo, kern, s2r, count)
    work = {"nodes_per_query": float(counts[:, 0].mean()), "cells_per_query": float(counts[:, 1].mean()),
            "clusters_per_query": float(counts[:, 2].mean()), "hits_per_query": float(counts[:, 3].mean()),
            "algorithmic_bytes_per_launch": abytes, "algorithmic_alu_ops_per_launch": aops}

    octaves = None
    if not args.no_octaves and isinstance(qc["sigma"], tuple):
        octaves = {}
        lo, hi = qc["sigma"]
        o = 0
        while lo * 2 ** o < hi:
            a, b = lo * 2 ** o, min(hi, lo * 2 ** (o + 1))
            sel = np.where((q[:, 2] >= a) & (q[:, 2] < b))[0]
            if len(sel):
                sq = tq[torch.from_numpy(sel).cuda()]
                so = torch.empty(len(sel), dtype=torch.float32, device="cuda")
                oalgo = "plain" if args.algo == "persistent" else args.algo
                P.eval_batch(hier, sq, tau=tau, algo=oalgo, out=so, **kw)
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                reps = 3
                for _ in range(reps):
                    P.eval_batch(hier, sq, tau=tau, algo=oalgo, out=so, **kw)
                e1.record(stream)
                torch.cuda.synchronize()
                octaves["sigma %g-%g" % (a, b)] = len(sel) * reps / (e0.elapsed_time(e1) * 1e-3)
            o += 1

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(nrm, q, tau, **kw)

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "map": "%s %dx%d" % (mc["kind"], n, n), "queries": count,
                   "sigma": list(qc["sigma"]) if isinstance(qc["sigma"], tuple) else qc["sigma"],
                   "h_radius": qc["radius"], "tau": tau, "algo": args.algo, "kernel": kern, "sigma_to_r": s2r,
                   "tuning": tuning},
        "roofline": {"bound": "alu", "achieved": achieved_ops, "peak": ALU_PEAK_TOPS, "unit": "Tops/s",
                     "frac": achieved_ops / ALU_PEAK_TOPS, "traffic": traffic},
        "roofline_hbm": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
        "cpu_baseline": cpu,
        "kernel_ms": kernel_ms,
        "build_s": build_s,
        "work": work,
        "queries_per_s_by_sigma_octave": octaves,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
