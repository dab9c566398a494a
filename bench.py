"""Benchmark: P-NDF queries/s on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload powerlaw8192]
                    [--algo plain|brute|persistent] [--no-cpu-baseline] [--no-octaves]
                    [--no-extras]

A step is one pndf_eval_batch over the whole query batch (queries and the mesh /
hierarchy already resident in HBM).  Prints one JSON line.  The default workload
is the largest configuration that fits one GPU: the 8192^2 power-law map, 2^24
queries with footprints log-uniform in [1, 8192] texels, cluster cut tau = 1e-3.
Extra keys: the 2048^2 power-law workload (tau = 0), a short serving run (p50/p99
tile latency), queries/s per footprint-size octave.

Roofline: the dominant kernel of a step is the evaluation kernel.  The work it
must do is counted by a CPU pass (bench_workcount.c) that applies the descent's
rules from the entry level -- nodes box-tested, leaf cells tested, cluster nodes
used -- on a stratified sample (512 queries per footprint-size octave,
extrapolated by each octave's share of the batch), with the hits of the same
sample from the GPU (the hit set is fixed by the definition), and priced as
    bytes  B = 24 (query) + 4 (D) + 16 nodes + 8 cells + 36 clusters
    ops    F = 12 nodes + 40 cells + 40 clusters + 30 hits   (32-bit lane operations)
against 8 TB/s and 256 CUs x 64 lanes x 2.4 GHz = 39.3 T lane-ops/s.  The
duration is measured with HIP events on the stream the kernel runs on.  HBM
traffic comes from rocprofv3 FETCH_SIZE / WRITE_SIZE runs recorded under
profiles/ (null when the kernel source changed since they were taken).
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
EVAL_SRC = ("eval.hip", "pndf_internal.h")
SAMPLE_SRC = ("sample.hip", "pndf_internal.h")
SAMPLE_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_sample_powerlaw2048.json")
WORKCOUNT_SRC = os.path.join(ROOT, "bench_workcount.c")
WORKCOUNT_LIB = os.path.join(ROOT, "bench_workcount.so")


def kernel_hash(files=EVAL_SRC):
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_2505_08985_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_file(workload, algo):
    return os.path.join(ROOT, "profiles", "traffic_eval_%s_%s.json" % (algo, workload))


def load_traffic(workload, algo, kernel="gaussian", sigma_to_r=3.0, queries=None):
    """The measured HBM bytes per launch, if the committed counters were taken on this
    source and this exact launch: the workload's own batch at the default support."""
    path = traffic_file(workload, algo)
    if not os.path.exists(path):
        return None
    try:
        t = json.load(open(path))
    except (OSError, ValueError):
        return None
    import workloads
    if (t.get("kernel_hash") != kernel_hash() or t.get("workload") != workload or t.get("algo") != algo
            or t.get("kernel", "gaussian") != kernel or sigma_to_r != 3.0
            or queries != workloads.CONFIGS[workload]["queries"]["count"] or t.get("queries") != queries):
        return None
    return float(t["hbm_bytes_per_launch"])


def build_workcount(force=False):
    if force or not os.path.exists(WORKCOUNT_LIB) or os.path.getmtime(WORKCOUNT_LIB) < os.path.getmtime(WORKCOUNT_SRC):
        import subprocess
        tmp = WORKCOUNT_LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-fopenmp", "-fno-fast-math",
                               WORKCOUNT_SRC, "-o", tmp, "-lm"])
        os.replace(tmp, WORKCOUNT_LIB)
    return WORKCOUNT_LIB


def count_work(n, boxes, own, es, q, tau, s2r):
    """CPU counting pass: (nodes, cells, clusters) per query by the descent's rules."""
    import ctypes
    lib = ctypes.CDLL(build_workcount())
    fp = ctypes.POINTER(ctypes.c_float)
    lib.wc_count.argtypes = [ctypes.c_int, fp, fp, fp, fp, ctypes.c_int64, ctypes.c_float, ctypes.c_float,
                             ctypes.POINTER(ctypes.c_uint64)]
    lib.wc_count.restype = ctypes.c_int
    q = np.ascontiguousarray(q, dtype=np.float32)
    out = np.zeros((len(q), 3), dtype=np.uint64)
    rc = lib.wc_count(n, boxes.ctypes.data_as(fp), own.ctypes.data_as(fp) if own is not None else None,
                      es.ctypes.data_as(fp) if es is not None else None,
                      q.ctypes.data_as(fp), len(q), tau, s2r, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    if rc:
        raise RuntimeError("wc_count failed (%d)" % rc)
    return out.astype(np.float64)


def sigma_octave(q):
    return np.floor(np.log2(np.maximum(q[:, 2], q[:, 3]))).astype(np.int64)


def algorithmic_work(P, hier, q, tq, n, tau, s2r, kw, per_octave=512, seed=3):
    """Algorithmic work of one launch over the batch: the CPU counting pass on a
    sample of per_octave queries per footprint-size octave, extrapolated by each
    octave's population; hits of the same sample from the GPU (eval_counts, which
    also gives the kernel's own instrumented counts for comparison)."""
    import torch
    L = int(np.log2(n))
    boxes, own, es = [], [], []
    for level in range(1, L + 1):
        ex = P.hier_export_level(hier, level)
        boxes.append(ex["bbox_all" if tau > 0 else "bbox"].cpu().numpy().reshape(-1))
        if tau > 0:
            own.append(ex["bbox_clu"].cpu().numpy().reshape(-1))
            es.append(ex["clu_e"].cpu().numpy().reshape(-1))
    boxes = np.ascontiguousarray(np.concatenate(boxes))
    own = np.ascontiguousarray(np.concatenate(own)) if tau > 0 else None
    es = np.ascontiguousarray(np.concatenate(es)) if tau > 0 else None
    oq = sigma_octave(q)
    rng = np.random.default_rng(seed)
    tot = np.zeros(4)      # nodes, cells, clusters, hits (extrapolated to the batch)
    ktot = np.zeros(3)     # the kernel's own counts (nodes, cells, clusters), extrapolated
    by_oct = {}
    for o in np.unique(oq):
        pool = np.where(oq == o)[0]
        pick = np.sort(rng.choice(pool, min(per_octave, len(pool)), replace=False))
        w = count_work(n, boxes, own, es, q[pick], tau, s2r)
        _, c = P.eval_counts(hier, tq[torch.from_numpy(pick).cuda()], tau=tau, **kw)
        c = c.cpu().numpy().astype(np.float64)
        mean = np.concatenate([w.mean(axis=0), [c[:, 3].mean()]])
        tot += mean * len(pool)
        ktot += c[:, :3].mean(axis=0) * len(pool)
        by_oct["sigma %d-%d" % (2 ** o, 2 ** (o + 1))] = {
            "queries": int(len(pool)), "sampled": int(len(pick)), "nodes": mean[0], "cells": mean[1],
            "clusters": mean[2], "hits": mean[3]}
    nodes, cells, clus, hits = tot
    abytes = 28.0 * len(q) + 16.0 * nodes + 8.0 * cells + 36.0 * clus
    abytes_iso = 28.0 * len(q) + 16.0 * nodes + 32.0 * cells + 36.0 * clus   # every cell's 4 corners on their own
    aops = 12.0 * nodes + 40.0 * cells + 40.0 * clus + 30.0 * hits
    nq = float(len(q))
    return {"nodes_per_query": nodes / nq, "cells_per_query": cells / nq, "clusters_per_query": clus / nq,
            "hits_per_query": hits / nq, "algorithmic_bytes_per_launch": abytes,
            "algorithmic_bytes_per_launch_isolated_cells": abytes_iso,
            "algorithmic_alu_ops_per_launch": aops,
            "kernel_counts_per_query": {"nodes": ktot[0] / nq, "cells": ktot[1] / nq, "clusters": ktot[2] / nq},
            "sample": "CPU counting pass on %d queries per sigma octave, extrapolated by octave population; "
                      "hits from the GPU on the same sample" % per_octave,
            "by_sigma_octave": by_oct}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_rates(oracle, nrm, q, oq, tau, clusters, kw, budget_s, seed):
    """Queries/s of the oracle per footprint-size octave: each octave timed on
    random queries of its own until budget_s / octaves seconds have passed."""
    rng = np.random.default_rng(seed)
    octs = np.unique(oq)
    per = budget_s / len(octs)
    rates, used = {}, 0
    for o in octs:
        pool = rng.permutation(np.where(oq == o)[0])
        k, done, t = 4, 0, 0.0
        while done < len(pool) and t < per:
            sel = pool[done:done + k]
            a = time.perf_counter()
            oracle.evaluate(nrm, q[sel], tau=tau, clusters=clusters, **kw)
            t += time.perf_counter() - a
            done += len(sel)
            k *= 2
        rates[int(o)] = done / t
        used += done
    return rates, used


def cpu_baseline(nrm, q, tau, budget_s=20.0, one_core_s=8.0, kernel="gaussian", sigma_to_r=3.0):
    """The FP64 oracle as it stands, on the machine's host threads and on one core: each
    footprint-size octave timed on random queries of its own (bounded time per
    octave), the whole batch's time extrapolated from the octaves' populations."""
    import oracle
    oracle.load()
    kw = dict(kernel=kernel, sigma_to_r=sigma_to_r)
    clusters, fit_s = None, 0.0
    if tau > 0:
        a = time.perf_counter()
        clusters = oracle.cluster_all(nrm)
        fit_s = time.perf_counter() - a
    oq = sigma_octave(q)
    pop = {int(o): int((oq == o).sum()) for o in np.unique(oq)}
    threads = oracle.num_threads()
    rates, used = oracle_rates(oracle, nrm, q, oq, tau, clusters, kw, budget_s, 11)
    total_s = sum(pop[o] / rates[o] for o in pop)
    oracle.set_threads(1)
    try:
        rates1, used1 = oracle_rates(oracle, nrm, q, oq, tau, clusters, kw, one_core_s, 12)
    finally:
        oracle.set_threads(threads)
    total1_s = sum(pop[o] / rates1[o] for o in pop)
    return {"value": len(q) / total_s, "unit": "queries/s", "cores": threads, "kind": "oracle",
            "sample": "%d random queries of the batch, each sigma octave timed for %.1f s, the batch's time "
                      "extrapolated from the octave populations (FP64 brute force over the cut's triangles%s)"
                      % (used, budget_s / len(pop), "; cluster fit %.1f s not included" % fit_s if tau > 0 else ""),
            "cpu_model": cpu_model(), "one_core": len(q) / total1_s, "one_core_sample": used1,
            "by_sigma_octave": {"sigma %d-%d" % (2 ** o, 2 ** (o + 1)): rates[o] for o in sorted(rates)},
            "oracle_cluster_fit_s": fit_s if tau > 0 else None}


SERVE_MAPS = (dict(kind="bumps", n=1024, seed=411, count=8192),
              dict(kind="scratched", n=4096, seed=301),
              dict(kind="powerlaw", n=8192, seed=501, rms_slope=0.15))


def serve_run(P, hiers, ns, ntiles, rates, tau, slots, batch_tiles, algo, sigma_max, seed, chunk,
              persistent_costs=False, log=True):
    """Poisson arrivals of render tiles (64 x 64 px x 4 spp) over resident maps at
    fractions of the baseline's capacity.  The baseline is the same C++ runtime
    evaluating one whole tile per plain launch, back to back on one stream (FIFO);
    the served configuration uses `slots` streams, batches of up to batch_tiles
    tiles of one map and pieces of at most `chunk` queries per request.  Every
    served result is checked bit for bit against pndf_eval_batch on the tile."""
    import torch
    import workloads
    rng = np.random.default_rng(seed)
    mids = rng.integers(0, len(hiers), ntiles)
    tiles = [workloads.tile_request(ns[m], int(rng.integers(1 << 30)), sigma_range=(0.5, sigma_max)) for m in mids]
    qpt = tiles[0].shape[0]

    def say(msg):
        if log:
            print("[serve] " + msg, file=sys.stderr, flush=True)

    # each tile alone (plain launch, host-synchronised), and its reference result
    dq = [torch.from_numpy(t).cuda() for t in tiles]
    for m, q in zip(mids[:4], dq[:4]):
        P.eval_batch(hiers[m], q, tau=tau)
    torch.cuda.synchronize()
    cost, ref = [], []
    for m, q in zip(mids, dq):
        a = time.perf_counter()
        r = P.eval_batch(hiers[m], q, tau=tau)
        torch.cuda.synchronize()
        cost.append(time.perf_counter() - a)
        ref.append(r.cpu().numpy())
    cost = np.array(cost)
    say("tiles alone: median %.2f ms, max %.1f ms" % (1e3 * np.median(cost), 1e3 * cost.max()))
    # one plain launch per map over all of its tiles' queries (throughput reference)
    a = time.perf_counter()
    for m in range(len(hiers)):
        sel = [k for k in range(ntiles) if mids[k] == m]
        if sel:
            P.eval_batch(hiers[m], torch.cat([dq[k] for k in sel]), tau=tau)
    torch.cuda.synchronize()
    one_launch_qps = ntiles * qpt / (time.perf_counter() - a)
    cost_p = None
    if persistent_costs:
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
        for pl in plans:
            pl.close()
    del dq

    def check(outs):
        for k in range(ntiles):
            assert np.array_equal(outs[k].view(np.uint32), ref[k].view(np.uint32)), "served tile %d differs" % k

    fifo = P.Server(hiers, slots=1, max_batch_queries=qpt, max_pending=4 * ntiles, tau=tau, algo="plain")
    srv = P.Server(hiers, slots=slots, max_batch_queries=qpt * batch_tiles, max_pending=4 * ntiles, tau=tau,
                   algo=algo, chunk_queries=chunk)
    for x in (fifo, srv):
        x.replay(mids[:4], np.zeros(4), tiles[:4])  # warm-up
    # saturation: everything arrives at once
    a = time.perf_counter()
    outs, _ = fifo.replay(mids, np.zeros(ntiles), tiles)
    fifo_cap = ntiles / (time.perf_counter() - a)
    check(outs)
    a = time.perf_counter()
    outs, _ = srv.replay(mids, np.zeros(ntiles), tiles)
    sat = ntiles * qpt / (time.perf_counter() - a)
    check(outs)
    say("saturation: baseline %.0f tiles/s, served %.0f tiles/s" % (fifo_cap, sat / qpt))
    results = []
    for frac in rates:
        rate = frac * fifo_cap
        arr = np.cumsum(rng.exponential(1.0 / rate, ntiles))
        arr -= arr[0]
        a = time.perf_counter()
        _, lat_f = fifo.replay(mids, arr, tiles)
        wall_f = time.perf_counter() - a
        srv.reset_stats()
        a = time.perf_counter()
        outs, lat = srv.replay(mids, arr, tiles)
        wall = time.perf_counter() - a
        check(outs)
        st = srv.stats()
        results.append({"rate_frac": frac, "tiles_per_s_offered": rate,
                        "served_queries_per_s": ntiles * qpt / wall,
                        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                        "max_ms": float(lat.max()), "mean_batch_pieces": st["mean_batch_requests"],
                        "baseline_queries_per_s": ntiles * qpt / wall_f,
                        "baseline_p50_ms": float(np.percentile(lat_f, 50)),
                        "baseline_p99_ms": float(np.percentile(lat_f, 99))})
        say(json.dumps(results[-1]))
    fifo.close()
    srv.close()
    out = {"queries_per_tile": qpt, "tiles": ntiles,
           "baseline_per_tile_queries_per_s": fifo_cap * qpt, "saturation_queries_per_s": sat,
           "one_launch_per_map_queries_per_s": one_launch_qps,
           "tile_alone_ms": {"median": 1e3 * float(np.median(cost)), "p99": 1e3 * float(np.percentile(cost, 99)),
                             "max": 1e3 * float(cost.max())},
           "by_rate": results}
    if cost_p is not None:
        out["persistent_tile_alone_ms"] = {"median": 1e3 * float(np.median(cost_p)), "max": 1e3 * float(cost_p.max())}
    return out


def serve_bench(args):
    """Serving workload: Poisson arrivals of render tiles (64 x 64 px x 4 spp) over three
    resident maps, footprints from synthetic ray differentials; continuous batching
    with pieces against the FIFO plain per-tile baseline of the same runtime, at
    fractions of the baseline's capacity."""
    import torch
    import paper_2505_08985_amd as P
    import workloads
    hiers, ns, keep = [], [], []
    t0 = time.perf_counter()
    for mc in SERVE_MAPS:
        nrm = workloads.make_map(**mc)
        mesh = P.build_mesh(torch.from_numpy(nrm).cuda())
        h = P.build_hierarchy(mesh, cluster=True)
        keep.append(mesh)
        hiers.append(h)
        ns.append(mc["n"])
        del nrm
        torch.cuda.synchronize()
        print("[serve] map %s %d^2 resident (%.1f s)" % (mc["kind"], mc["n"], time.perf_counter() - t0),
              file=sys.stderr, flush=True)
    res = serve_run(P, hiers, ns, args.serve_tiles, [float(f) for f in args.serve_rates.split(",")], args.serve_tau,
                    args.serve_slots, args.serve_batch_tiles, args.serve_algo, args.serve_sigma_max, 401,
                    args.serve_chunk, persistent_costs=True)
    qpt = res["queries_per_tile"]
    sat = res["saturation_queries_per_s"]
    line = {"metric": METRIC, "value": sat, "unit": "queries/s", "n_gpus": 1, "steps": args.serve_tiles,
            "warmup": 4, "ms_per_step": 1e3 * qpt / sat, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "serving: Poisson 64x64x4 tiles over bumps1024 / scratched4096 / "
                                   "powerlaw8192", "tau": args.serve_tau, "sigma_range": [0.5, args.serve_sigma_max],
                       "slots": args.serve_slots, "batch_tiles": args.serve_batch_tiles,
                       "chunk_queries": args.serve_chunk, "batch_algo": args.serve_algo}}
    line.update(res)
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
    if args.sample_presorted:
        # the stream as a renderer issues it, tile by tile: neighbouring samples have
        # neighbouring footprint centres (sorted by a 64 x 64 Morton bucket, host-side,
        # before the timed region)
        b = np.clip((q[:, :2] / n * 64).astype(np.int64), 0, 63)
        code = np.zeros(len(q), dtype=np.int64)
        for bit in range(6):
            code |= ((b[:, 0] >> bit) & 1) << (2 * bit) | ((b[:, 1] >> bit) & 1) << (2 * bit + 1)
        q = np.ascontiguousarray(q[np.argsort(code, kind="stable")])
    print("[bench] sampling on %s: map %d^2, %d samples, tau %g, %s%s" % (args.workload, n, count, tau, kern,
          ", footprint centres in Morton order" if args.sample_presorted else ""), file=sys.stderr, flush=True)
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
    # unit's four corner normals 32 and its clamp bits 1 (a byte, for a cell or a
    # cluster node alike); with the cut, 4 per residual read (entry level down to the unit)
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
                and kern == "gaussian" and args.workload == "powerlaw2048" and not args.sample_presorted):
            traffic = float(t["hbm_bytes_per_launch"])
    except (OSError, ValueError, KeyError):
        pass
    line = {"metric": "P-NDF samples/sec at 1 MI355X", "value": count * args.steps / wall, "unit": "samples/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": args.workload + " sampling", "map": "%s %dx%d" % (mc["kind"], n, n),
                       "samples": count, "tau": tau, "kernel": kern, "sigma_to_r": s2r, "attempts": attempts,
                       "sample_order": "morton" if args.sample_presorted else "random"},
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
    ap.add_argument("--no-extras", action="store_true",
                    help="headline workload only (no powerlaw2048 line, no serving summary)")
    ap.add_argument("--summary-tiles", type=int, default=64, help="tiles of the headline's serving summary")
    ap.add_argument("--workload", default="powerlaw8192")
    ap.add_argument("--algo", default="plain")
    ap.add_argument("--queries", type=int, default=0, help="override the batch size")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-octaves", action="store_true")
    ap.add_argument("--input-order", action="store_true", help="keep the query order (no spatial ordering)")
    ap.add_argument("--tuning", default=None, metavar="BPC,SPLIT",
                    help="persistent tuning (blocks per CU, split level) instead of autotuning")
    ap.add_argument("--autotune", action="store_true",
                    help="autotune the persistent plan (default: the plan's default tuning)")
    ap.add_argument("--autotune-queries", type=int, default=1 << 18,
                    help="size of the autotuning sample (every footprint-size octave in proportion to the "
                         "batch); a sample much smaller than the batch is dominated by its slowest queries "
                         "and favours fewer workers")
    ap.add_argument("--kernel", default="gaussian", choices=["gaussian", "disk", "box"],
                    help="footprint kernel")
    ap.add_argument("--sigma-to-r", type=float, default=None,
                    help="support half-width in sigma (default 3 for gaussian, 1.5 for disk and box)")
    ap.add_argument("--serve", action="store_true", help="serving benchmark (continuous batching)")
    ap.add_argument("--sample", action="store_true", help="sampling benchmark (pndf_sample_batch)")
    ap.add_argument("--sample-tau", type=float, default=0.0)
    ap.add_argument("--sample-presorted", action="store_true",
                    help="sampling: footprint centres in Morton order (as a renderer's tiles issue them)")
    ap.add_argument("--projarea", action="store_true", help="projected-area benchmark (pndf_projected_area)")
    ap.add_argument("--serve-tau", type=float, default=1e-3)
    ap.add_argument("--serve-tiles", type=int, default=200)
    ap.add_argument("--serve-sigma-max", type=float, default=4096.0)
    ap.add_argument("--serve-rates", default="0.5,0.8,0.95")
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-batch-tiles", type=int, default=1,
                    help="batch size in tiles (a batch ends with its slowest query, so tiles of very "
                         "different cost are better not batched together)")
    ap.add_argument("--serve-algo", default="plain", choices=["plain", "persistent"],
                    help="how the server evaluates a batch")
    ap.add_argument("--serve-chunk", type=int, default=0,
                    help="largest piece of one request in one batch (0: whole requests)")
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

    torch.cuda.set_device(0)
    head = measure(P, args.workload, args, args.steps, args.warmup, algo=args.algo, octaves=not args.no_octaves)
    extras = {}
    if not args.no_extras and args.workload != "powerlaw2048":
        r = measure(P, "powerlaw2048", args, 20, 5, algo="plain", octaves=not args.no_octaves)
        extras["powerlaw2048"] = {k: r["line"][k] for k in ("value", "ms_per_step", "config", "roofline",
                                                           "roofline_alt", "work", "queries_per_s_by_sigma_octave")}
        del r
    serving = None
    if not args.no_extras:
        serving = serving_summary(P, head, args)
    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(head["nrm"], head["q"], head["tau"], kernel=head["kernel"], sigma_to_r=head["s2r"])
    line = head["line"]
    line["cpu_baseline"] = cpu
    line["serving"] = serving
    line["other_workloads"] = extras or None
    line["hbm_achievable"] = stream_bandwidth()
    print(json.dumps(line), flush=True)


def stream_bandwidth(mib=2048, reps=5):
    """Achievable HBM bandwidth on this machine, as context for the 8 TB/s peak: a
    device-to-device copy of 2 GiB (read + write bytes) and a read-only reduction of
    the same buffer, best of a few runs, timed with HIP events."""
    import torch
    n = (mib << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def best(fn, nbytes):
        fn()
        torch.cuda.synchronize()
        t = 1e30
        for _ in range(reps):
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            t = min(t, e0.elapsed_time(e1))
        return nbytes / (t * 1e-3) / 1e9

    copy = best(lambda: dst.copy_(src), 2 * 4 * n)
    read = best(lambda: src.sum(), 4 * n)
    del src, dst
    return {"copy_gbs": copy, "read_gbs": read, "peak_gbs": HBM_PEAK_GBS,
            "method": "2 GiB float32: copy_ (read + write bytes) and sum (read bytes), best of %d, HIP events" % reps}


def measure(P, workload, args, steps, warmup, algo="plain", octaves=True):
    """Build one workload, time `steps` evaluations of the whole batch after `warmup`,
    and price the launch by the counting pass.  Returns the JSON line's fields and
    the resident objects."""
    import torch
    import workloads
    kern = args.kernel
    s2r = args.sigma_to_r if args.sigma_to_r is not None else (3.0 if kern == "gaussian" else 1.5)
    kw = dict(kernel=kern, sigma_to_r=s2r)
    cfg = workloads.CONFIGS[workload]
    mc, qc, tau = cfg["map"], cfg["queries"], float(cfg["tau"])
    n = mc["n"]
    t0 = time.perf_counter()
    nrm = workloads.make_map(**mc)
    count = (args.queries or qc["count"]) if workload == args.workload else qc["count"]
    q = workloads.uniform_queries(n, count, qc["seed"], qc["sigma"], qc["radius"])
    gen_s = time.perf_counter() - t0
    print("[bench] workload %s: map %d^2, %d queries, tau %g (generated in %.1f s)" % (workload, n, count, tau, gen_s),
          file=sys.stderr, flush=True)
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
    if algo == "persistent":
        if args.tuning:
            bpc, split = (int(v) for v in args.tuning.split(","))
            tuning = dict(blocks_per_cu=bpc, split_level=split, queue_factor=16, use_graph=1)
        elif args.autotune:
            sample = autotune_sample(q, tq, args.autotune_queries)
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
            P.eval_batch(hier, tq, tau=tau, algo=algo, out=out, input_order=args.input_order, **kw)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = ev0.elapsed_time(ev1) / steps
    print("[bench] %s: timed %d steps: %.3f ms/step (events %.3f ms)" % (workload, steps, 1e3 * wall / steps,
                                                                        kernel_ms), file=sys.stderr, flush=True)
    value = count * steps / wall
    d = out.cpu().numpy()
    assert np.isfinite(d).all() and (d >= 0).all()
    if algo == "persistent":
        st = plan.stats()
        assert st["error"] == 0, st
        ref = P.eval_batch(hier, tq, tau=tau, **kw)
        assert torch.equal(ref.view(torch.int32), out.view(torch.int32)), "persistent != plain"
        plan.close()

    work = algorithmic_work(P, hier, q, tq, n, tau, s2r, kw)
    abytes, aops = work["algorithmic_bytes_per_launch"], work["algorithmic_alu_ops_per_launch"]
    achieved = abytes / (kernel_ms * 1e-3) / 1e9
    achieved_ops = aops / (kernel_ms * 1e-3) / 1e12
    traffic = load_traffic(workload, algo, kern, s2r, count)
    hbm = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS, "traffic": traffic}
    alu = {"bound": "alu", "achieved": achieved_ops, "peak": ALU_PEAK_TOPS, "unit": "Tops/s",
           "frac": achieved_ops / ALU_PEAK_TOPS, "traffic": traffic}
    # the binding roofline is the one the launch comes closer to
    roof, alt = (hbm, alu) if hbm["frac"] >= alu["frac"] else (alu, hbm)

    oct_rates = None
    if octaves:
        oct_rates = {}
        oq = sigma_octave(q)
        oalgo = "plain" if algo == "persistent" else algo
        for o in np.unique(oq):
            sel = np.where(oq == o)[0]
            sq = tq[torch.from_numpy(sel).cuda()]
            so = torch.empty(len(sel), dtype=torch.float32, device="cuda")
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
            oct_rates["sigma %d-%d" % (2 ** o, 2 ** (o + 1))] = len(sel) * reps / (e0.elapsed_time(e1) * 1e-3)
        print("[bench] %s: per-octave rates measured" % workload, file=sys.stderr, flush=True)

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": 1e3 * wall / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload, "map": "%s %dx%d" % (mc["kind"], n, n), "queries": count,
                   "sigma": list(qc["sigma"]) if isinstance(qc["sigma"], tuple) else qc["sigma"],
                   "h_radius": qc["radius"], "tau": tau, "algo": algo, "kernel": kern, "sigma_to_r": s2r,
                   "tuning": tuning},
        "roofline": roof,
        "roofline_alt": alt,
        "kernel_ms": kernel_ms,
        "build_s": build_s,
        "work": work,
        "queries_per_s_by_sigma_octave": oct_rates,
    }
    return {"line": line, "nrm": nrm, "q": q, "tq": tq, "hier": hier, "mesh": mesh, "tau": tau, "n": n,
            "kernel": kern, "s2r": s2r}


def autotune_sample(q, tq, size, seed=5):
    """A sample that loads the GPU like the batch: every footprint-size octave in
    proportion to its share of the batch (at least one query each)."""
    import torch
    oq = sigma_octave(q)
    rng = np.random.default_rng(seed)
    frac = min(1.0, size / float(len(q)))
    pick = []
    for o in np.unique(oq):
        pool = np.where(oq == o)[0]
        pick.append(rng.choice(pool, max(1, int(round(frac * len(pool)))), replace=False))
    pick = np.sort(np.concatenate(pick))
    return tq[torch.from_numpy(pick).cuda()]


def serving_summary(P, head, args):
    """A short serving run for the headline line: Poisson arrivals of 64 x 64 x 4
    render tiles over the three serving maps at 0.95 of the baseline's capacity."""
    import torch
    import workloads
    hiers, ns = [], []
    keep = []
    for mc in SERVE_MAPS:
        if mc["kind"] == "powerlaw" and mc["n"] == head["n"] and head["line"]["config"]["workload"] == "powerlaw8192":
            hiers.append(head["hier"])
        else:
            nrm = workloads.make_map(**mc)
            mesh = P.build_mesh(torch.from_numpy(nrm).cuda())
            h = P.build_hierarchy(mesh, cluster=True)
            keep.append((mesh, h))
            hiers.append(h)
        ns.append(mc["n"])
    torch.cuda.synchronize()
    res = serve_run(P, hiers, ns, ntiles=args.summary_tiles, rates=[0.95], tau=args.serve_tau,
                    slots=args.serve_slots, batch_tiles=args.serve_batch_tiles, algo=args.serve_algo,
                    sigma_max=args.serve_sigma_max, seed=401, chunk=args.serve_chunk)
    r = res["by_rate"][0]
    return {"tiles": args.summary_tiles, "queries_per_tile": res["queries_per_tile"],
            "offered_load": "0.95 of the baseline's capacity (FIFO, one whole tile per plain launch, same runtime)",
            "served_queries_per_s": r["served_queries_per_s"], "p50_ms": r["p50_ms"], "p99_ms": r["p99_ms"],
            "baseline_p50_ms": r["baseline_p50_ms"], "baseline_p99_ms": r["baseline_p99_ms"],
            "baseline_per_tile_queries_per_s": res["baseline_per_tile_queries_per_s"],
            "saturation_queries_per_s": res["saturation_queries_per_s"],
            "one_launch_per_map_queries_per_s": res["one_launch_per_map_queries_per_s"],
            "tile_alone_ms": res["tile_alone_ms"],
            "tau": args.serve_tau, "slots": args.serve_slots, "batch_tiles": args.serve_batch_tiles,
            "chunk_queries": args.serve_chunk, "maps": "bumps1024 / scratched4096 / powerlaw8192"}


if __name__ == "__main__":
    main()
