"""Serving runtime: continuous batching over resident maps.  Every request's result
equals its evaluation alone (bit for bit: terms are summed exactly), whatever the
batch it lands in; admission refuses work beyond the memory budget."""
import sys

import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a HIP device")]


def announce(msg):
    print("[gpu-case] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def maps():
    import torch
    import paper_2505_08985_amd as P
    import workloads
    out = []
    for kind, n, seed in (("bumps", 128, 401), ("powerlaw", 256, 402), ("scratched", 256, 403)):
        kw = dict(scratches=200, flakes=500) if kind == "scratched" else {}
        nrm = workloads.make_map(kind, n, seed, **kw)
        mesh = P.build_mesh(torch.from_numpy(nrm).cuda())
        out.append((nrm, P.build_hierarchy(mesh, cluster=True)))
    torch.cuda.synchronize()
    return out


def tiles(maps, count, seed, tile=16):
    import workloads
    rng = np.random.default_rng(seed)
    mids, qs = [], []
    for k in range(count):
        m = int(rng.integers(0, len(maps)))
        n = maps[m][0].shape[0]
        qs.append(workloads.tile_request(n, int(rng.integers(1 << 30)), tile=tile, spp=4,
                                         sigma_range=(0.5, 2.0 * n)))
        mids.append(m)
    return mids, qs


@pytest.mark.parametrize("chunk", [0, 100])
@pytest.mark.parametrize("algo", ["plain", "persistent"])
@pytest.mark.parametrize("tau", [0.0, 1e-3])
def test_served_results_equal_alone(maps, tau, algo, chunk):
    """Whole requests, or pieces of at most 100 queries (a 1024-query tile is
    spread over up to 11 batches, between the pieces of other tiles)."""
    import torch
    import paper_2505_08985_amd as P
    announce("serving: mixed tiles over 3 maps, tau=%g, %s batches, chunk %d" % (tau, algo, chunk))
    mids, qs = tiles(maps, 40, 7)
    srv = P.Server([h for _, h in maps], slots=3, max_batch_queries=4096, max_pending=64, tau=tau, algo=algo,
                   chunk_queries=chunk)
    arrivals = np.cumsum(np.random.default_rng(1).exponential(0.002, len(qs)))
    outs, lat = srv.replay(mids, arrivals, qs)
    st = srv.stats()
    assert st["completed"] == len(qs) and (lat > 0).all()
    for m, q, o in zip(mids, qs, outs):
        alone = P.eval_batch(maps[m][1], torch.from_numpy(q).cuda(), tau=tau).cpu().numpy()
        np.testing.assert_array_equal(o.view(np.uint32), alone.view(np.uint32))
    srv.close()


@pytest.mark.parametrize("algo", ["plain", "persistent"])
def test_batches_mix_requests(maps, algo):
    import paper_2505_08985_amd as P
    announce("serving: burst arrivals share batches (%s)" % algo)
    mids, qs = tiles(maps, 30, 11, tile=8)
    srv = P.Server([h for _, h in maps], slots=1, max_batch_queries=8192, max_pending=64, algo=algo)
    outs, lat = srv.replay(mids, np.zeros(len(qs)), qs)
    st = srv.stats()
    assert st["completed"] == 30 and st["mean_batch_requests"] > 1.5, st
    assert st["p99_ms"] >= st["p50_ms"] > 0
    srv.close()


def test_admission_by_memory(maps):
    import paper_2505_08985_amd as P
    announce("serving: admission refuses beyond the memory budget")
    mids, qs = tiles(maps, 12, 13, tile=16)   # 1024 queries each
    srv = P.Server([h for _, h in maps], slots=1, max_batch_queries=1024,
                   memory_budget=28 * 1024 * 2 + 2048, max_pending=64)
    tickets, refused = [], 0
    for m, q in zip(mids, qs):
        try:
            tickets.append(srv.submit(m, q)[0])
        except P.PndfError as e:
            assert e.status == 6  # PNDF_EAGAIN
            refused += 1
    assert refused > 0
    for t in tickets:
        assert srv.wait(t) > 0
    srv.drain()
    assert srv.stats()["refused"] == refused
    # once drained, the budget is free again
    t, out = srv.submit(mids[0], qs[0])
    srv.wait(t)
    srv.close()


def test_submit_validation(maps):
    import paper_2505_08985_amd as P
    announce("serving: argument validation")
    srv = P.Server([h for _, h in maps], slots=1, max_batch_queries=256)
    q = np.zeros((300, 6), dtype=np.float32)
    with pytest.raises(P.PndfError):
        srv.submit(0, q)              # larger than a batch
    with pytest.raises(P.PndfError):
        srv.submit(5, q[:10])         # no such map
    with pytest.raises(P.PndfError):
        srv.wait(12345)
    srv.close()
    with pytest.raises(P.PndfError):
        P.Server([h for _, h in maps], slots=1, max_batch_queries=256, algo="brute")
    with pytest.raises(P.PndfError):
        P.Server([h for _, h in maps], slots=1, max_batch_queries=256, kernel=7)


@pytest.mark.parametrize("algo", ["plain", "persistent"])
def test_served_box_kernel_equals_alone(maps, algo):
    import torch
    import paper_2505_08985_amd as P
    announce("serving: box footprints, %s batches" % algo)
    mids, qs = tiles(maps, 16, 17, tile=8)
    srv = P.Server([h for _, h in maps], slots=2, max_batch_queries=2048, max_pending=64, algo=algo,
                   kernel="box", sigma_to_r=1.5)
    outs, lat = srv.replay(mids, np.zeros(len(qs)), qs)
    for m, q, o in zip(mids, qs, outs):
        alone = P.eval_batch(maps[m][1], torch.from_numpy(q).cuda(), kernel="box", sigma_to_r=1.5).cpu().numpy()
        np.testing.assert_array_equal(o.view(np.uint32), alone.view(np.uint32))
    srv.close()


def test_pieces_interleave(maps):
    """With pieces, a burst of requests of one map shares batches piece by piece:
    more pieces than requests, several requests per batch, results as alone."""
    import torch
    import paper_2505_08985_amd as P
    announce("serving: pieces of large requests interleave")
    mids, qs = tiles(maps, 12, 23, tile=16)      # 1024 queries each
    mids = [1] * len(qs)
    qs = [q * np.array([0.5, 0.5, 1, 1, 1, 1], dtype=np.float32) for q in qs]   # all on the 256^2 map
    srv = P.Server([h for _, h in maps], slots=1, max_batch_queries=1024, max_pending=64, chunk_queries=256)
    outs, lat = srv.replay(mids, np.zeros(len(qs)), qs)
    st = srv.stats()
    assert st["completed"] == len(qs)
    assert st["batches"] >= len(qs) and st["mean_batch_requests"] > 1.5, st   # 4 pieces of 256 per batch
    for m, q, o in zip(mids, qs, outs):
        alone = P.eval_batch(maps[m][1], torch.from_numpy(q).cuda()).cpu().numpy()
        np.testing.assert_array_equal(o.view(np.uint32), alone.view(np.uint32))
    srv.close()


def test_replay_validates_before_submitting(maps):
    """A trace with decreasing arrival times, an unknown map or an oversized request
    is refused as a whole before anything is submitted; the server stays usable."""
    import torch
    import paper_2505_08985_amd as P
    announce("serving: replay validation")
    mids, qs = tiles(maps, 6, 29, tile=8)        # 256 queries each
    srv = P.Server([h for _, h in maps], slots=2, max_batch_queries=256, max_pending=64)
    arr = np.array([0.0, 0.001, 0.002, 0.001, 0.003, 0.004])
    with pytest.raises(P.PndfError):
        srv.replay(mids, arr, qs)                # decreasing arrivals
    big = qs[:5] + [np.zeros((300, 6), dtype=np.float32)]
    with pytest.raises(P.PndfError):
        srv.replay(mids, np.zeros(6), big)       # oversized request
    with pytest.raises(P.PndfError):
        srv.replay([0, 1, 2, 9, 0, 1], np.zeros(6), qs)   # no such map
    assert srv.stats()["completed"] == 0         # nothing ran
    outs, lat = srv.replay(mids, np.zeros(6), qs)
    assert srv.stats()["completed"] == 6
    for m, q, o in zip(mids, qs, outs):
        alone = P.eval_batch(maps[m][1], torch.from_numpy(q).cuda()).cpu().numpy()
        np.testing.assert_array_equal(o.view(np.uint32), alone.view(np.uint32))
    srv.close()


def test_serving_maps_alone_and_in_the_mix():
    """The serving configuration itself: 1024^2 bumps, 4096^2 scratched metal and the
    8192^2 power-law map resident together, 64 render tiles (64 x 64 px x 4 spp)
    with footprints from synthetic ray differentials (sigma 0.5-4096), tau = 1e-3,
    Poisson arrivals, 4 slots, batches of up to 4 tiles in pieces of 1024 queries:
    every tile's result equals its evaluation alone, bit for bit."""
    import torch
    import paper_2505_08985_amd as P
    import workloads
    announce("serving: 64 tiles over bumps1024 / scratched4096 / powerlaw8192, pieces of 1024")
    recipes = (dict(kind="bumps", n=1024, seed=411, count=8192), dict(kind="scratched", n=4096, seed=301),
               dict(kind="powerlaw", n=8192, seed=501, rms_slope=0.15))
    hiers, ns, meshes = [], [], []
    for mc in recipes:
        nrm = workloads.make_map(**mc)
        mesh = P.build_mesh(torch.from_numpy(nrm).cuda())
        meshes.append(mesh)
        hiers.append(P.build_hierarchy(mesh, cluster=True))
        ns.append(mc["n"])
        del nrm
    torch.cuda.synchronize()
    rng = np.random.default_rng(401)
    mids = rng.integers(0, 3, 64)
    qs = [workloads.tile_request(ns[m], int(rng.integers(1 << 30)), sigma_range=(0.5, 4096.0)) for m in mids]
    qpt = qs[0].shape[0]
    srv = P.Server(hiers, slots=4, max_batch_queries=4 * qpt, max_pending=256, tau=1e-3, chunk_queries=1024)
    arr = np.cumsum(rng.exponential(0.01, len(qs)))
    outs, lat = srv.replay(mids, arr - arr[0], qs)
    assert srv.stats()["completed"] == len(qs)
    for k, (m, q, o) in enumerate(zip(mids, qs, outs)):
        alone = P.eval_batch(hiers[m], torch.from_numpy(q).cuda(), tau=1e-3).cpu().numpy()
        assert np.isfinite(alone).all()
        np.testing.assert_array_equal(o.view(np.uint32), alone.view(np.uint32), err_msg="tile %d" % k)
    srv.close()
