"""pndf_eval_batch_noalloc: the entry point for callers that cannot allocate
device memory returns pndf_eval_batch's bits, on consecutive calls of decreasing
size (the static workspace keeps the previous call's contents), and refuses
batches beyond its workspace without launching anything."""
import sys

import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a HIP device")]


def announce(msg):
    print("[gpu-case] " + msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("tau", [0.0, 1e-3])
def test_noalloc_equals_eval_batch(tau):
    import torch
    import paper_2505_08985_amd as P
    import workloads
    announce("no-allocation entry point: 2 calls (60000 then 9000 queries), tau=%g" % tau)
    nrm = workloads.make_map("powerlaw", 512, 31)
    mesh = P.build_mesh(torch.from_numpy(nrm).cuda())
    hier = P.build_hierarchy(mesh, cluster=True)
    for count, seed in ((60000, 1), (9000, 2), (1000, 3)):
        q = workloads.uniform_queries(512, count, seed, (0.5, 40.0), 0.3)
        tq = torch.from_numpy(q).cuda()
        ref = P.eval_batch(hier, tq, tau=tau)
        got = P.eval_batch_noalloc(hier, tq, tau=tau)
        torch.cuda.synchronize()
        assert torch.equal(ref.view(torch.int32), got.view(torch.int32)), count
        assert torch.isfinite(got).all() and (got > 0).sum() > count // 20


def test_noalloc_limits():
    import torch
    import paper_2505_08985_amd as P
    announce("no-allocation entry point: batch beyond the workspace is refused")
    nrm = np.zeros((8, 8, 2), dtype=np.float32)
    nrm[..., 0] = 0.1
    mesh = P.build_mesh(torch.from_numpy(nrm).cuda())
    hier = P.build_hierarchy(mesh, cluster=False)
    big = torch.zeros(((1 << 22) + 1, 6), dtype=torch.float32, device="cuda")
    with pytest.raises(P.PndfError):
        P.eval_batch_noalloc(hier, big)
    out = P.eval_batch_noalloc(hier, torch.zeros((0, 6), device="cuda"))
    assert out.numel() == 0
