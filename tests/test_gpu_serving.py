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


@pytest.mark.parametrize("algo", ["plain", "persistent"])
@pytest.mark.parametrize("tau", [0.0, 1e-3])
def test_served_results_equal_alone(maps, tau, algo):
    import torch
    import paper_2505_08985_amd as P
    announce("serving: mixed tiles over 3 maps, tau=%g, %s batches" % (tau, algo))
    mids, qs = tiles(maps, 40, 7)
    srv = P.Server([h for _, h in maps], slots=3, max_batch_queries=4096, max_pending=64, tau=tau, algo=algo)
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
