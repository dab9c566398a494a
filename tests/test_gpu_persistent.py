"""The persistent work-stealing traversal (plans, graph replay, autotuner):
bit-identical to the plain per-batch kernel, and therefore to the oracle
within the parity bar, for any tuning and batch composition."""
import sys

import numpy as np
import pytest

from conftest import gpu_available
from parity import compare

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a HIP device")]


def announce(msg):
    print("[gpu-case] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import paper_2505_08985_amd as P
    return P


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def mixed(n, count, seed, smin, smax, radius):
    rng = np.random.default_rng(seed)
    q = np.zeros((count, 6), dtype=np.float32)
    q[:, 0:2] = rng.uniform(-n, 2 * n, (count, 2))
    q[:, 2] = np.exp(rng.uniform(np.log(smin), np.log(smax), count))
    q[:, 3] = q[:, 2] * np.exp(rng.uniform(-0.5, 0.5, count))
    r = radius * np.sqrt(rng.uniform(size=count))
    t = rng.uniform(0, 2 * np.pi, count)
    q[:, 4], q[:, 5] = r * np.cos(t), r * np.sin(t)
    return q


@pytest.fixture(scope="module")
def setup(P):
    import torch
    import workloads
    nrm = workloads.make_map("powerlaw", 256, 17)
    mesh = P.build_mesh(to_dev(nrm))
    hier = P.build_hierarchy(mesh, cluster=True)
    torch.cuda.synchronize()
    return nrm, hier


@pytest.mark.parametrize("tau", [0.0, 1e-3])
@pytest.mark.parametrize("tuning", [
    dict(blocks_per_cu=1, split_level=1, queue_factor=64, use_graph=1),
    dict(blocks_per_cu=2, split_level=3, queue_factor=16, use_graph=0),
    dict(blocks_per_cu=4, split_level=5, queue_factor=1, use_graph=1),
    dict(blocks_per_cu=8, split_level=1, queue_factor=1, use_graph=0),
])
@pytest.mark.parametrize("input_order", [False, True])
def test_persistent_equals_plain_bitwise(P, setup, tau, tuning, input_order):
    import torch
    nrm, hier = setup
    announce("persistent %s tau=%g input_order=%s" % (tuning, tau, input_order))
    q = mixed(256, 3001, 3, 0.05, 120.0, 0.4)
    tq = to_dev(q)
    plain = P.eval_batch(hier, tq, tau=tau)
    plan = P.Plan(hier, 4096, tau=tau, tuning=tuning, input_order=input_order)
    for rep in range(3):
        got = plan.eval(tq)
        torch.cuda.synchronize()
        st = plan.stats()
        assert st["error"] == 0, st
        assert torch.equal(got.view(torch.int32), plain.view(torch.int32)), (rep, st)
    # a few footprints cover the whole map: once the small ones are done, the idle
    # workers must have been fed with pieces of the big ones
    assert st["spawned"] > 0, st
    plan.close()


@pytest.mark.parametrize("split_level", [1, 3])
def test_persistent_queue_full(P, setup, split_level):
    """Eight whole-map footprints and a queue of eight slots: the queue fills at once
    and later offers are refused (the nodes stay with their wave); the result is
    still the plain kernel's, bit for bit."""
    import torch
    nrm, hier = setup
    announce("persistent queue full, split_level=%d" % split_level)
    q = mixed(256, 8, 31, 100.0, 120.0, 0.3)
    tq = to_dev(q)
    plain = P.eval_batch(hier, tq, tau=0.0)
    plan = P.Plan(hier, 8, tuning=dict(blocks_per_cu=2, split_level=split_level, queue_factor=1, use_graph=1))
    for rep in range(2):
        got = plan.eval(tq)
        st = plan.stats()
        assert st["error"] == 0, st
        assert torch.equal(got.view(torch.int32), plain.view(torch.int32)), (rep, st)
    assert st["spawned"] > 0 and st["refused"] > 0, st
    plan.close()


def test_persistent_matches_oracle(P, oracle_mod, setup):
    nrm, hier = setup
    announce("persistent vs oracle")
    q = mixed(256, 700, 5, 0.3, 60.0, 0.35)
    plan = P.Plan(hier, 1000, tuning=dict(blocks_per_cu=2, split_level=2, queue_factor=32, use_graph=1))
    d = plan.eval(to_dev(q)).cpu().numpy()
    assert plan.stats()["spawned"] > 0
    ref = oracle_mod.evaluate(nrm, q, records=True)
    compare(ref, d)


def test_persistent_batch_sizes_and_mix(P, setup):
    import torch
    nrm, hier = setup
    announce("persistent: varying batch sizes on one plan, alone vs in the mix")
    q = mixed(256, 5000, 9, 0.05, 150.0, 0.4)
    tq = to_dev(q)
    plain = P.eval_batch(hier, tq)
    plan = P.Plan(hier, 5000, tuning=dict(blocks_per_cu=2, split_level=3, queue_factor=8, use_graph=1))
    for a, b in ((0, 5000), (17, 18), (100, 1333), (4000, 5000), (0, 1)):
        got = plan.eval(tq[a:b])
        assert torch.equal(got.view(torch.int32), plain[a:b].view(torch.int32)), (a, b)
    perm = torch.from_numpy(np.random.default_rng(0).permutation(5000)).cuda()
    got = plan.eval(tq[perm])
    assert torch.equal(got.view(torch.int32), plain[perm].view(torch.int32))
    # empty batch and bounds
    assert plan.eval(tq[:0]).numel() == 0
    with pytest.raises(P.PndfError):
        plan.eval(torch.cat([tq, tq[:1]]))


def test_brute_plain_persistent_identical(P, setup):
    import torch
    nrm, hier = setup
    announce("brute == plain == persistent, bit for bit")
    q = mixed(256, 800, 13, 0.05, 40.0, 0.35)
    tq = to_dev(q)
    a = P.eval_batch(hier, tq, algo="brute")
    b = P.eval_batch(hier, tq, algo="plain")
    c = P.Plan(hier, 800, tuning=dict(blocks_per_cu=1, split_level=2, queue_factor=16, use_graph=1)).eval(tq)
    assert torch.equal(a.view(torch.int32), b.view(torch.int32))
    assert torch.equal(b.view(torch.int32), c.view(torch.int32))


def test_autotuner(P, setup):
    import torch
    nrm, hier = setup
    announce("autotuner")
    q = mixed(256, 4096, 21, 0.5, 100.0, 0.4)
    tq = to_dev(q)
    best, ms = P.autotune(hier, tq)
    assert 1 <= best["blocks_per_cu"] <= 8 and 2 <= best["split_level"] <= 8 and ms > 0
    plan = P.Plan(hier, 4096, tuning=best)
    got = plan.eval(tq)
    assert torch.equal(got.view(torch.int32), P.eval_batch(hier, tq).view(torch.int32))


def test_blocks_beyond_resident_are_clamped(P, setup):
    """A grid larger than what fits on the GPU at once runs as the resident grid:
    the plan reports the effective count, and the result is unchanged."""
    import torch
    nrm, hier = setup
    announce("persistent blocks_per_cu 64 -> resident")
    q = mixed(256, 1500, 23, 0.5, 100.0, 0.4)
    tq = to_dev(q)
    plan = P.Plan(hier, 2048, tuning=dict(blocks_per_cu=64, split_level=4, queue_factor=16, use_graph=1))
    eff = plan.tuning()
    assert 1 <= eff["blocks_per_cu"] <= 10 and eff["split_level"] == 4, eff
    got = plan.eval(tq)
    assert plan.stats()["error"] == 0
    assert torch.equal(got.view(torch.int32), P.eval_batch(hier, tq).view(torch.int32))
    small = P.Plan(hier, 2048, tuning=dict(blocks_per_cu=1, split_level=4, queue_factor=16, use_graph=1))
    assert small.tuning()["blocks_per_cu"] == 1
