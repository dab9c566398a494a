"""GPU sampling of the P-NDF (pndf_sample_batch, through the C ABI) against the
FP64 oracle's sampler, and against the GPU's own evaluation (the histogram of
samples must follow D).

Parity protocol: both sides get the same uniforms.  Outside the oracle's flagged
samples (a cut decision within rounding of the threshold, or u within 1e-8 of a
unit edge or diagonal, where the triangle may differ under rounding) the
triangle id is identical, u agrees to 1e-9 relative and m to 2e-6 (float32 output;
cluster normals are fitted separately on each side and agree to 2e-6 of their
scale, so 2e-5 for cluster samples).
"""
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
def P():
    import paper_2505_08985_amd as P
    return P


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def random_disk_map(n, seed, radius=0.5):
    rng = np.random.default_rng(seed)
    r = radius * np.sqrt(rng.uniform(size=(n, n)))
    t = rng.uniform(0, 2 * np.pi, size=(n, n))
    return np.stack([r * np.cos(t), r * np.sin(t)], axis=-1).astype(np.float32)


def flat_patch_map(n, seed):
    """Random normals with flat 4 x 4 patches: their cells are clamped."""
    nrm = random_disk_map(n, seed, 0.45)
    for k in range(0, n - 4, 9):
        nrm[k:k + 4, k:k + 4] = nrm[k, k]
    return nrm


MAPS = {
    "bumps64": lambda: __import__("workloads").make_map("bumps", 64, 101, count=32),
    "powerlaw128": lambda: __import__("workloads").make_map("powerlaw", 128, 7),
    "scratched128": lambda: __import__("workloads").make_map(
        "scratched", 128, 9, scratches=120, flakes=300),
    "flatpatch32": lambda: flat_patch_map(32, 4),
}


def queries(n, count, seed, smin, smax):
    rng = np.random.default_rng(seed)
    q = np.zeros((count, 6), dtype=np.float32)
    q[:, 0:2] = rng.uniform(-n, 2 * n, (count, 2))
    q[:, 2] = np.exp(rng.uniform(np.log(smin), np.log(smax), count))
    q[:, 3] = q[:, 2] * np.exp(rng.uniform(-0.7, 0.7, count))
    return q


def build(P, nrm, cluster):
    import torch
    mesh = P.build_mesh(to_dev(nrm))
    hier = P.build_hierarchy(mesh, cluster=cluster)
    torch.cuda.synchronize()
    return mesh, hier


def oracle_xi(xi):
    """(attempts, Q, 2) attempt-major -> the oracle's (Q, 2 attempts) rows."""
    a, nq, _ = xi.shape
    return np.ascontiguousarray(xi.transpose(1, 0, 2).reshape(nq, 2 * a))


def compare(ref, m, tri, u):
    nan_ref = np.isnan(ref["m"][:, 0])
    assert np.array_equal(nan_ref, np.isnan(m[:, 0])), "NaN pattern differs"
    ok = ~nan_ref & (ref["flags"] == 0)
    assert np.array_equal(tri[ok], ref["tri"][ok].view(np.int64)), "triangle ids differ"
    assert (tri[nan_ref] == -1).all()
    np.testing.assert_allclose(u[ok], ref["u"][ok], rtol=1e-9, atol=1e-9)
    lev = (ref["tri"][ok] >> np.uint64(58)).astype(np.int64)
    tol = np.where(lev > 0, 2e-5, 2e-6)[:, None]
    err = np.abs(m[ok].astype(np.float64) - ref["m"][ok])
    assert (err <= tol).all(), "m differs by up to %g" % err.max()
    # flagged samples whose triangle agrees must agree in m too
    fl = ~nan_ref & (ref["flags"] != 0) & (tri == ref["tri"].view(np.int64))
    if fl.any():
        lev2 = (ref["tri"][fl] >> np.uint64(58)).astype(np.int64)
        tol2 = np.where(lev2 > 0, 2e-5, 2e-6)[:, None]
        assert (np.abs(m[fl].astype(np.float64) - ref["m"][fl]) <= tol2).all()
    return dict(flagged=int((ref["flags"] != 0).sum()), nan=int(nan_ref.sum()),
                clusters=int((lev > 0).sum()))


@pytest.mark.parametrize("tau", [0.0, 1e-3, 1e-2])
@pytest.mark.parametrize("kernel", ["gaussian", "disk", "box"])
@pytest.mark.parametrize("name", sorted(MAPS))
def test_sample_parity(P, oracle_mod, name, kernel, tau):
    """Footprints from 0.05 to 0.5 N texels (periodic images, anisotropic, centres
    outside the base period), a ragged batch, four uniform pairs per sample."""
    import torch
    announce("sample %s %s tau=%g" % (name, kernel, tau))
    nrm = MAPS[name]()
    n = nrm.shape[0]
    s2r = 3.0 if kernel == "gaussian" else 1.5
    q = queries(n, 3001, 41, 0.05, 0.5 * n)
    xi = np.random.default_rng(42).uniform(size=(4, len(q), 2))
    _, hier = build(P, nrm, cluster=tau > 0)
    m, tri, u = P.sample_batch(hier, to_dev(q), to_dev(xi), tau=tau, sigma_to_r=s2r, kernel=kernel, u=True)
    torch.cuda.synchronize()
    clusters = oracle_mod.cluster_all(nrm) if tau > 0 else None
    ref = oracle_mod.sample(nrm, q, oracle_xi(xi), tau=tau, sigma_to_r=s2r, kernel=kernel, clusters=clusters)
    st = compare(ref, m.cpu().numpy(), tri.cpu().numpy(), u.cpu().numpy())
    print(st)
    assert st["flagged"] <= 0.02 * len(q) and st["nan"] <= 0.001 * len(q)
    if tau >= 1e-2:
        assert st["clusters"] > 100
    # deterministic: a second call gives the same bits
    m2, tri2, _ = P.sample_batch(hier, to_dev(q), to_dev(xi), tau=tau, sigma_to_r=s2r, kernel=kernel)
    assert torch.equal(m2.view(torch.int32), m.view(torch.int32)) and torch.equal(tri2, tri)


def test_sample_edge_cases(P, oracle_mod):
    import torch
    announce("sample edge cases")
    nrm = random_disk_map(16, 5, 0.45)
    _, hier = build(P, nrm, cluster=True)
    q = np.array([
        [3.5, 4.5, 0.01, 0.01, 0, 0],          # tiny footprint
        [3.5, 4.5, 1e-3, 5.0, 0, 0],           # extreme anisotropy
        [-100.25, 700.5, 2.0, 2.0, 0, 0],      # far outside the base period
        [7.0, 7.0, 200.0, 200.0, 0, 0],        # many periods wide
        [np.nan, 1, 1, 1, 0, 0],               # invalid
        [1, 1, 0.0, 1, 0, 0],
        [1, 1, 1, 2e7, 0, 0],                  # r beyond 2^24 (for sigma_to_r 1.5 and 3)
        [8.0, 8.0, 1.0 / 3.0, 1.0 / 3.0, 0, 0],
        [5.0, 5.0, 1.0, 1.0, 0, 0],            # uniform 1.0: invalid
        [5.0, 5.0, 1.0, 1.0, 0, 0],            # uniform < 0: invalid
        [5.0, 5.0, 1.0, 1.0, 0, 0],            # NaN uniform in an unused pair: fine
        [5.0, 5.0, 1.0, 1.0, 0, 0],            # uniform 0 exactly
    ], dtype=np.float32)
    xi = np.random.default_rng(3).uniform(size=(2, len(q), 2))
    xi[0, 8, 0] = 1.0
    xi[0, 9, 1] = -0.25
    xi[1, 10, :] = np.nan
    xi[0, 11, :] = 0.0
    for tau in (0.0, 1e-3):
        for kernel in ("gaussian", "box"):
            m, tri, u = P.sample_batch(hier, to_dev(q), to_dev(xi), tau=tau, kernel=kernel,
                                       sigma_to_r=3.0 if kernel == "gaussian" else 1.5, u=True)
            m = m.cpu().numpy()
            ref = oracle_mod.sample(nrm, q, oracle_xi(xi), tau=tau, kernel=kernel,
                                    sigma_to_r=3.0 if kernel == "gaussian" else 1.5)
            compare(ref, m, tri.cpu().numpy(), u.cpu().numpy())
            assert np.isnan(m[4:7]).all() and np.isnan(m[8:10]).all()
            assert not np.isnan(m[[0, 1, 2, 3, 7, 10, 11]]).any()
    # empty batch, argument validation
    e = torch.zeros((0, 6), device="cuda")
    P.sample_batch(hier, e, torch.zeros((1, 0, 2), dtype=torch.float64, device="cuda"))
    qd, xd = to_dev(q), to_dev(xi)
    with pytest.raises(P.PndfError):
        P.sample_batch(hier, qd, torch.zeros((0, len(q), 2), dtype=torch.float64, device="cuda"))
    with pytest.raises(P.PndfError):
        P.sample_batch(hier, qd, xd, kernel=5)
    with pytest.raises(P.PndfError):
        P.sample_batch(hier, qd, xd, sigma_to_r=-1.0)
    _, hier0 = build(P, nrm, cluster=False)
    with pytest.raises(P.PndfError):
        P.sample_batch(hier0, qd, xd, tau=1e-3)
    # uniforms not 16-byte aligned (one double into an allocation)
    base = torch.zeros(2 * len(q) + 1, dtype=torch.float64, device="cuda")
    with pytest.raises(P.PndfError):
        P.sample_batch(hier, qd, base[1:].view(1, len(q), 2))


@pytest.mark.parametrize("kernel,tau", [("gaussian", 0.0), ("gaussian", 1e-2), ("disk", 1e-2), ("box", 0.0)])
def test_sample_histogram_matches_gpu_evaluation(P, kernel, tau):
    """The GPU's samples follow the GPU's own D: the histogram of 2^23 sampled
    normals against the integral of D (pndf_eval_batch on a sub-grid) over each bin,
    normalised (the same check as the oracle's pin, at GPU sample counts)."""
    import torch
    import workloads
    announce("sample histogram vs evaluation %s tau=%g" % (kernel, tau))
    nrm = workloads.make_map("powerlaw", 128, 7)
    _, hier = build(P, nrm, cluster=tau > 0)
    s2r = 3.0 if kernel == "gaussian" else 1.5
    x, y, s = 61.3, 40.7, (3.0 if kernel == "gaussian" else 6.0)
    ns = 1 << 23
    qd = torch.tensor([[x, y, s, s, 0, 0]], dtype=torch.float32, device="cuda").repeat(ns, 1)
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    xi = torch.rand((4, ns, 2), dtype=torch.float64, device="cuda", generator=g)
    m, tri, _ = P.sample_batch(hier, qd, xi, tau=tau, sigma_to_r=s2r, kernel=kernel)
    m = m.cpu().numpy().astype(np.float64)
    good = ~np.isnan(m[:, 0])
    assert good.mean() > 0.9999
    lim = float(np.abs(m[good]).max()) * 1.02
    nb = 16
    edges = np.linspace(-lim, lim, nb + 1)
    hist, _, _ = np.histogram2d(m[good, 0], m[good, 1], bins=[edges, edges])
    freq = hist / good.sum()
    sub = 48 if kernel == "gaussian" else 96
    w = edges[1] - edges[0]
    cx = (edges[:-1, None] + (np.arange(sub)[None, :] + 0.5) * w / sub).ravel()
    mx, my = np.meshgrid(cx, cx, indexing="ij")
    qs = np.zeros((mx.size, 6), dtype=np.float32)
    qs[:, 0], qs[:, 1], qs[:, 2], qs[:, 3] = x, y, s, s
    qs[:, 4], qs[:, 5] = mx.ravel(), my.ravel()
    D = P.eval_batch(hier, to_dev(qs), tau=tau, sigma_to_r=s2r, kernel=kernel).cpu().numpy().astype(np.float64)
    binint = D.reshape(nb, sub, nb, sub).sum(axis=(1, 3))
    p = binint / binint.sum()
    big = p > 5e-3
    assert big.sum() >= 10
    rel = np.abs(freq[big] - p[big]) / p[big]
    print("bins %d, median rel %.4f, max rel %.4f" % (big.sum(), np.median(rel), rel.max()))
    assert np.median(rel) < 0.02
    assert rel.max() < 0.08


def test_sample_full_size_sampled(P, oracle_mod):
    """The bench launch: 2^24 samples on the 2048^2 power-law map (sigma in [1, 64],
    tau = 0 and 1e-3), checked against the oracle on 4096 samples drawn from the
    launch's output."""
    import torch
    import workloads
    announce("sample full size powerlaw2048 2^24")
    cfg = workloads.CONFIGS["powerlaw2048"]
    mc, qc = cfg["map"], cfg["queries"]
    n = mc["n"]
    count = 1 << 24
    nrm = workloads.make_map(**mc)
    q = workloads.uniform_queries(n, count, qc["seed"], qc["sigma"], qc["radius"])
    _, hier = build(P, nrm, cluster=True)
    tq = to_dev(q)
    g = torch.Generator(device="cuda")
    g.manual_seed(1)
    xi = torch.rand((2, count, 2), dtype=torch.float64, device="cuda", generator=g)
    pick = np.sort(np.random.default_rng(9).choice(count, 4096, replace=False))
    for tau in (0.0, 1e-3):
        m, tri, u = P.sample_batch(hier, tq, xi, tau=tau, u=True)
        torch.cuda.synchronize()
        sel = torch.from_numpy(pick).cuda()
        ms, ts, us = m[sel].cpu().numpy(), tri[sel].cpu().numpy(), u[sel].cpu().numpy()
        xs = xi[:, sel, :].cpu().numpy()
        clusters = oracle_mod.cluster_all(nrm) if tau > 0 else None
        ref = oracle_mod.sample(nrm, q[pick], oracle_xi(xs), tau=tau, clusters=clusters)
        st = compare(ref, ms, ts, us)
        print(tau, st)
        assert st["flagged"] <= 0.02 * len(pick)
        if tau > 0:
            assert st["clusters"] > 500
