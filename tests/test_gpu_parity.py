"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Every case prints what it runs before touching the device.
"""
import math
import sys

import numpy as np
import pytest

from conftest import gpu_available
from parity import check_cluster_fit, compare

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a HIP device")]

EPS32 = float(np.float32(1e-6))


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


def gpu_build(P, nrm, cluster=True):
    import torch
    mesh = P.build_mesh(to_dev(nrm))
    hier = P.build_hierarchy(mesh, cluster=cluster)
    torch.cuda.synchronize()
    return mesh, hier


def gpu_hits(P, hier, q, tau=0.0, algo="auto", kernel="gaussian", sigma_to_r=3.0):
    import torch
    d, off, ids, terms = P.eval_hits(hier, to_dev(q), tau=tau, algo=algo, kernel=kernel, sigma_to_r=sigma_to_r)
    torch.cuda.synchronize()
    return d.cpu().numpy(), off.cpu().numpy(), ids.cpu().numpy().view(np.uint64), terms.cpu().numpy()


def normal_radius(nrm, scale=1.1):
    """Query-normal disk radius covering the map's own normals."""
    return scale * float(np.sqrt((nrm.astype(np.float64) ** 2).sum(-1)).max())


def random_disk_map(n, seed, radius=0.5):
    rng = np.random.default_rng(seed)
    r = radius * np.sqrt(rng.uniform(size=(n, n)))
    t = rng.uniform(0, 2 * np.pi, size=(n, n))
    return np.stack([r * np.cos(t), r * np.sin(t)], axis=-1).astype(np.float32)


def mixed_queries(n, count, seed, smin, smax, radius, aniso=True, spread=1.0):
    rng = np.random.default_rng(seed)
    q = np.zeros((count, 6), dtype=np.float32)
    q[:, 0:2] = rng.uniform(-spread * n, (1 + spread) * n, (count, 2)) if spread > 0 else rng.uniform(0, n, (count, 2))
    q[:, 2] = np.exp(rng.uniform(np.log(smin), np.log(smax), count))
    q[:, 3] = q[:, 2] * (np.exp(rng.uniform(-0.7, 0.7, count)) if aniso else 1.0)
    r = radius * np.sqrt(rng.uniform(size=count))
    t = rng.uniform(0, 2 * np.pi, count)
    q[:, 4] = r * np.cos(t)
    q[:, 5] = r * np.sin(t)
    return q


MAPS = {
    "bumps64": lambda: __import__("workloads").make_map("bumps", 64, 101, count=32),
    "powerlaw128": lambda: __import__("workloads").make_map("powerlaw", 128, 7),
    "disk32": lambda: random_disk_map(32, 3, 0.45),
    "scratched128": lambda: __import__("workloads").make_map(
        "scratched", 128, 9, scratches=60, flakes=150),
}


# --------------------------------------------------------------- mesh build
@pytest.mark.parametrize("name", sorted(MAPS))
def test_mesh_build_bit_exact(P, oracle_mod, name):
    announce("mesh build %s" % name)
    nrm = MAPS[name]()
    mesh, hier = gpu_build(P, nrm, cluster=False)
    deg, det = P.mesh_export(mesh)
    odet, odeg = oracle_mod.mesh(nrm)
    np.testing.assert_array_equal(deg.cpu().numpy(), odeg)
    want = np.where(odet < EPS32, np.float32(EPS32), odet.astype(np.float32)).astype(np.float32)
    np.testing.assert_array_equal(det.cpu().numpy(), want)


def test_mesh_rejects_bad_maps(P):
    import torch
    announce("mesh validation")
    bad = np.zeros((8, 8, 2), dtype=np.float32)
    bad[3, 4] = (0.8, 0.7)                     # |n| >= 1
    with pytest.raises(P.PndfError):
        P.build_mesh(to_dev(bad))
    bad[3, 4] = (np.nan, 0)
    with pytest.raises(P.PndfError):
        P.build_mesh(to_dev(bad))
    with pytest.raises(P.PndfError):
        P.build_mesh(torch.zeros((6, 6, 2), device="cuda"))   # not a power of two
    with pytest.raises(P.PndfError):
        P.build_mesh(torch.zeros((8, 8, 2), device="cuda"), eps=0.0)


# ----------------------------------------------------------- hierarchy build
def triangle_boxes(nrm, deg, rho):
    """Per-cell box over both triangles (clamped ones by their replacement disk)."""
    n = nrm.shape[0]
    f = nrm.astype(np.float64)
    n0 = f
    n1 = np.roll(f, -1, axis=1)
    n2 = np.roll(f, -1, axis=0)
    n3 = np.roll(n1, -1, axis=0)
    c = 0.5 * (n1 + n2)
    lo = np.full((n, n, 2), np.inf)
    hi = np.full((n, n, 2), -np.inf)
    for bit, verts in ((1, (n0, n1, n2)), (2, (n3, n2, n1))):
        dg = (deg & bit) != 0
        vmin = np.minimum(np.minimum(verts[0], verts[1]), verts[2])
        vmax = np.maximum(np.maximum(verts[0], verts[1]), verts[2])
        vmin = np.where(dg[..., None], c - rho, vmin)
        vmax = np.where(dg[..., None], c + rho, vmax)
        lo = np.minimum(lo, vmin)
        hi = np.maximum(hi, vmax)
    return lo, hi


@pytest.mark.parametrize("name", sorted(MAPS))
def test_hierarchy_boxes_and_clusters(P, oracle_mod, name):
    announce("hierarchy build %s" % name)
    nrm = MAPS[name]()
    n = nrm.shape[0]
    L = int(math.log2(n))
    mesh, hier = gpu_build(P, nrm, cluster=True)
    _, odeg = oracle_mod.mesh(nrm)
    rho = math.sqrt(2 * EPS32 / (3 * math.sqrt(3)))
    clo, chi = triangle_boxes(nrm, odeg, rho)
    for level in range(1, L + 1):
        ex = P.hier_export_level(hier, level)
        m = n >> level
        s = 1 << level
        box = ex["bbox"].cpu().numpy().astype(np.float64)
        lo = clo.reshape(m, s, m, s, 2).min(axis=(1, 3))
        hi = chi.reshape(m, s, m, s, 2).max(axis=(1, 3))
        # conservative and tight: contains every triangle, within 2e-6 of the true extent
        assert (box[..., 0] <= lo[..., 0]).all() and (box[..., 1] <= lo[..., 1]).all()
        assert (box[..., 2] >= hi[..., 0]).all() and (box[..., 3] >= hi[..., 1]).all()
        assert (box[..., 0] >= lo[..., 0] - 2e-6).all() and (box[..., 2] <= hi[..., 0] + 2e-6).all()
        ns, e = oracle_mod.cluster_level(nrm, level)
        check_cluster_fit(ex, ns, e, m, level)
        # cluster boxes cover the cluster triangles
        ball = ex["bbox_all"].cpu().numpy()
        assert (ball[..., 0] <= box[..., 0]).all() and (ball[..., 2] >= box[..., 2]).all()
        cn = ex["clu_n"].cpu().numpy()
        cdet = ex["clu_det"].cpu().numpy()
        # the node's own cluster box: inside the subtree's, covering its two cluster
        # triangles (a clamped one by its replacement's square), and tight
        bclu = ex["bbox_clu"].cpu().numpy().astype(np.float64)
        assert (ball[..., :2] <= bclu[..., :2]).all() and (ball[..., 2:] >= bclu[..., 2:]).all()
        cc = 0.5 * (cn[:, :, 1, :] + cn[:, :, 2, :])          # float32, as the kernels form it
        rl = np.float32(rho) * np.float32(s)
        own_lo = np.full((m, m, 2), np.inf)
        own_hi = np.full((m, m, 2), -np.inf)
        for half, idx in ((0, (0, 1, 2)), (1, (3, 2, 1))):
            v = cn[:, :, list(idx), :].astype(np.float64)
            dv = np.abs((v[:, :, 2, 0] - v[:, :, 0, 0]) * (v[:, :, 1, 1] - v[:, :, 0, 1])
                        - (v[:, :, 2, 1] - v[:, :, 0, 1]) * (v[:, :, 1, 0] - v[:, :, 0, 0])) / (s * s)
            cl = (dv < EPS32)[..., None]
            own_lo = np.minimum(own_lo, np.where(cl, cc - rl, v.min(axis=2)))
            own_hi = np.maximum(own_hi, np.where(cl, cc + rl, v.max(axis=2)))
        assert (bclu[..., :2] <= own_lo).all() and (bclu[..., 2:] >= own_hi).all()
        slack = 2e-6 + 2e-6 * float(rl)
        assert (bclu[..., :2] >= own_lo - slack).all() and (bclu[..., 2:] <= own_hi + slack).all()
        for half, idx in ((0, (0, 1, 2)), (1, (3, 2, 1))):
            v = cn[:, :, list(idx), :]
            d = np.abs((v[:, :, 2, 0].astype(np.float64) - v[:, :, 0, 0]) * (v[:, :, 1, 1].astype(np.float64) - v[:, :, 0, 1])
                       - (v[:, :, 2, 1].astype(np.float64) - v[:, :, 0, 1]) * (v[:, :, 1, 0].astype(np.float64) - v[:, :, 0, 0])) / (s * s)
            clamped = d < EPS32
            want = np.where(clamped, np.float32(EPS32), d.astype(np.float32))
            np.testing.assert_allclose(cdet[..., half], want, rtol=1e-6)
            nc = ~clamped
            assert (ball[..., 0][nc] <= v[..., 0].min(axis=2)[nc]).all()
            assert (ball[..., 2][nc] >= v[..., 0].max(axis=2)[nc]).all()


# ------------------------------------------------------------- evaluation
def run_parity(P, oracle_mod, nrm, q, tau=0.0, algo="auto", clusters=None, hier=None):
    if hier is None:
        _, hier = gpu_build(P, nrm, cluster=tau > 0)
    d, off, ids, terms = gpu_hits(P, hier, q, tau=tau, algo=algo)
    ref = oracle_mod.evaluate(nrm, q, tau=tau, clusters=clusters, records=True)
    st = compare(ref, d, off, ids)
    # the plain output equals the hit-record pass bit for bit
    import torch
    d2 = P.eval_batch(hier, to_dev(q), tau=tau, algo=algo).cpu().numpy()
    np.testing.assert_array_equal(d2.view(np.uint32), d.view(np.uint32))
    return st


def test_brute_bumps64_all_queries(P, oracle_mod):
    """The small configuration: 64^2 bumps, 4096 queries, sigma = 2, |h| < 0.3."""
    import workloads
    announce("eval brute bumps64 4096 queries")
    nrm = workloads.make_map("bumps", 64, 101, count=32)
    q = workloads.uniform_queries(64, 4096, 102, 2.0, 0.3)
    st = run_parity(P, oracle_mod, nrm, q, algo="brute")
    assert st["nonzero"] > 100


@pytest.mark.parametrize("algo", ["plain", "brute"])
def test_plain_bumps64_all_queries(P, oracle_mod, algo):
    import workloads
    announce("eval %s bumps64 4096 queries, query normals inside the map's range" % algo)
    nrm = workloads.make_map("bumps", 64, 101, count=32)
    q = workloads.uniform_queries(64, 4096, 102, 2.0, 0.1)
    st = run_parity(P, oracle_mod, nrm, q, algo=algo)
    assert st["nonzero"] > 1000


@pytest.mark.parametrize("name", sorted(MAPS))
def test_plain_mixed_footprints(P, oracle_mod, name):
    """Footprints from 0.05 to ~2N texels (periodic images), anisotropic, centres
    outside the base period; a ragged batch size."""
    announce("eval plain mixed %s" % name)
    nrm = MAPS[name]()
    n = nrm.shape[0]
    q = mixed_queries(n, 1499, 11, 0.05, 0.7 * n, normal_radius(nrm))
    st = run_parity(P, oracle_mod, nrm, q)
    print(st)
    assert st["nonzero"] > 200


@pytest.mark.parametrize("tau", [1e-4, 1e-3, 1e-2])
@pytest.mark.parametrize("name", ["bumps64", "powerlaw128", "scratched128"])
def test_cluster_cut(P, oracle_mod, name, tau):
    announce("eval cut tau=%g %s" % (tau, name))
    nrm = MAPS[name]()
    n = nrm.shape[0]
    clusters = oracle_mod.cluster_all(nrm)
    q = mixed_queries(n, 1003, 21, 0.3, 0.5 * n, normal_radius(nrm))
    st = run_parity(P, oracle_mod, nrm, q, tau=tau, clusters=clusters)
    print(st)
    assert st["nonzero"] > 200
    assert st["cut_ambiguous"] <= 20


def flat_patch_map(n, seed, patches):
    """A random-disk map with square flat patches (texels [a, a + w) on both axes, one
    normal v each): every cell inside a patch, and every node whose cluster fit covers
    only patch texels (an exact fit, e^l = 0), has zero-area normal triangles."""
    nrm = random_disk_map(n, seed, 0.45)
    for a, w, v in patches:
        nrm[a:a + w, a:a + w] = v
    return nrm


@pytest.mark.parametrize("tau", [1e-4, 1e-2])
def test_cluster_cut_on_clamped_cluster_triangles(P, oracle_mod, tau):
    """Nodes inside a flat patch are under the cut for any tau > 0 (e^l = 0) and both
    of their cluster triangles have zero area, so both are replaced by the small
    equilateral triangle about the shared edge's midpoint (section on preventing the
    Jacobian singularity).  Query normals at the patch normal lie inside those
    replacements: the cut evaluation must hit them (a zero-area triangle tested as
    stored would miss) and agree with the oracle."""
    announce("eval cut tau=%g on clamped cluster triangles (flat patches, 32^2)" % tau)
    patches = [(8, 6, (0.2, -0.1)), (20, 6, (-0.15, 0.25))]
    nrm = flat_patch_map(32, 5, patches)
    rng = np.random.default_rng(17)
    nq = 301
    q = np.zeros((nq, 6), dtype=np.float32)
    which = rng.integers(0, len(patches), nq)
    for j, (a, w, v) in enumerate(patches):
        sel = which == j
        q[sel, 0:2] = a + 0.5 * w + rng.uniform(-1.0, 1.0, (int(sel.sum()), 2))
        q[sel, 4:6] = np.asarray(v, dtype=np.float32) + rng.uniform(-2e-5, 2e-5, (int(sel.sum()), 2))
    q[:, 2] = rng.uniform(0.8, 3.0, nq)
    q[:, 3] = q[:, 2] * np.exp(rng.uniform(-0.3, 0.3, nq))
    _, hier = gpu_build(P, nrm, cluster=True)
    st = run_parity(P, oracle_mod, nrm, q, tau=tau, hier=hier)
    print(st)
    assert st["nonzero"] >= 0.9 * nq and st["cut_ambiguous"] == 0, st
    # some hits are cluster triangles of flat nodes (four equal fitted normals)
    _, _, ids, _ = gpu_hits(P, hier, q, tau=tau)
    lev, I, J, _ = oracle_mod.decode_id(ids)
    flat_hits = 0
    for level in sorted(set(lev[lev > 0].tolist())):
        cn = P.hier_export_level(hier, level)["clu_n"].cpu().numpy()
        assert np.isfinite(cn).all()      # the export holds the fitted normals themselves
        sel = lev == level
        v = cn[J[sel], I[sel]]            # (hits, 4, 2); patches are symmetric in I, J
        flat_hits += int((v == v[:, :1]).all(axis=(1, 2)).sum())
    print("cluster hits on flat nodes:", flat_hits)
    assert flat_hits > 0


def test_edge_cases(P, oracle_mod):
    import torch
    announce("eval edge cases")
    nrm = random_disk_map(16, 5, 0.45)
    _, hier = gpu_build(P, nrm, cluster=True)
    # empty batch
    out = P.eval_batch(hier, torch.zeros((0, 6), device="cuda"))
    assert out.numel() == 0
    q = np.array([
        [3.5, 4.5, 0.01, 0.01, 0.1, 0.1],       # tiny footprint: entry level 0
        [3.5, 4.5, 1e-3, 5.0, 0.1, 0.1],        # extreme anisotropy
        [-100.25, 700.5, 2.0, 2.0, 0.0, 0.0],   # far outside the base period
        [7.0, 7.0, 200.0, 200.0, 0.05, -0.1],   # many periods wide
        [7.0, 7.0, 2.0, 2.0, 1.5, 0.0],         # |h| > 1: zero
        [7.0, 7.0, 2.0, 2.0, 0.999, 0.0],
        [np.nan, 1, 1, 1, 0, 0],                 # invalid: NaN
        [1, 1, 0.0, 1, 0, 0],                   # sigma = 0
        [1, 1, 1, -2, 0, 0],                    # sigma < 0
        [1, 1, 1, 1, np.inf, 0],
        [3e7, 1, 1, 1, 0, 0],                   # beyond 2^24
        [1, 1, 1e7, 1, 0, 0],                   # r beyond 2^24
        [8.0, 8.0, 1.0 / 3.0, 1.0 / 3.0, 0.2, 0.1],  # box edges on cell boundaries
        [0.0, 0.0, 2.0 / 3.0, 2.0 / 3.0, -0.2, 0.1],
    ], dtype=np.float32)
    d, off, ids, terms = gpu_hits(P, hier, q)
    ref = oracle_mod.evaluate(nrm, q, records=True)
    compare(ref, d, off, ids)
    assert np.isnan(d[6:12]).all() and d[4] == 0.0
    clusters = oracle_mod.cluster_all(nrm)
    d, off, ids, terms = gpu_hits(P, hier, q, tau=1e-3)
    compare(oracle_mod.evaluate(nrm, q, tau=1e-3, clusters=clusters, records=True), d, off, ids)


def test_minimal_map(P, oracle_mod):
    announce("eval on a 2x2 map")
    nrm = random_disk_map(2, 8, 0.4)
    q = mixed_queries(2, 301, 3, 0.05, 6.0, 0.4)
    run_parity(P, oracle_mod, nrm, q)


def test_options_and_errors(P):
    import torch
    announce("eval option validation")
    nrm = random_disk_map(8, 2)
    _, hier = gpu_build(P, nrm, cluster=False)
    q = torch.zeros((4, 6), device="cuda")
    q[:, 2:4] = 1.0
    with pytest.raises(P.PndfError):
        P.eval_batch(hier, q, tau=1e-3)           # no clusters
    with pytest.raises(P.PndfError):
        P.eval_batch(hier, q, tau=-1.0)
    with pytest.raises(P.PndfError):
        P.eval_batch(hier, q, sigma_to_r=0.0)
    with pytest.raises(P.PndfError):
        P.eval_batch(hier, q, kernel=3)
    _, hier2 = gpu_build(P, nrm, cluster=True)
    with pytest.raises(P.PndfError):
        P.eval_batch(hier2, q, tau=1e-3, algo="brute")


def test_sigma_to_r(P, oracle_mod):
    announce("eval with a different support width")
    nrm = random_disk_map(32, 6, 0.4)
    q = mixed_queries(32, 500, 4, 0.3, 8.0, 0.35)
    _, hier = gpu_build(P, nrm, cluster=False)
    import torch
    d, off, ids, terms = P.eval_hits(hier, to_dev(q), sigma_to_r=2.0)
    ref = oracle_mod.evaluate(nrm, q, sigma_to_r=2.0, records=True)
    compare(ref, d.cpu().numpy(), off.cpu().numpy(), ids.cpu().numpy().view(np.uint64))


def test_counts_are_consistent(P, oracle_mod):
    import workloads
    announce("eval counters")
    nrm = workloads.make_map("powerlaw", 128, 7)
    q = mixed_queries(128, 700, 5, 0.3, 30.0, 0.3, spread=0)
    _, hier = gpu_build(P, nrm, cluster=True)
    import torch
    tq = to_dev(q)
    d, c = P.eval_counts(hier, tq)
    d0 = P.eval_batch(hier, tq)
    assert torch.equal(d.view(torch.int32), d0.view(torch.int32))
    dd, off, ids, terms = P.eval_hits(hier, tq)
    c = c.cpu().numpy()
    np.testing.assert_array_equal(c[:, 3], np.diff(off.cpu().numpy()))
    assert (c[:, 2] == 0).all()
    db, cb = P.eval_counts(hier, tq, algo="brute")
    cb = cb.cpu().numpy()
    for k in range(len(q)):
        sx = np.float32(3) * q[k, 2]
        sy = np.float32(3) * q[k, 3]
        nx = math.floor(np.float32(q[k, 0] + sx)) - (math.ceil(np.float32(q[k, 0] - sx)) - 1) + 1
        ny = math.floor(np.float32(q[k, 1] + sy)) - (math.ceil(np.float32(q[k, 1] - sy)) - 1) + 1
        assert cb[k, 1] == min(nx, 128) * min(ny, 128)
    # the hierarchy tests at most as many cells as brute force and finds the same hits
    assert (c[:, 1] <= cb[:, 1]).all()
    np.testing.assert_array_equal(c[:, 3], cb[:, 3])
    dt, ct = P.eval_counts(hier, tq, tau=1e-2)
    assert ct.cpu().numpy()[:, 2].sum() > 0


def lattice_map(n, seed, step, jitter):
    """Texel normals on the 1/128 lattice: a regular grid of the given step with a
    jitter of up to `jitter` lattice units.  Every offset v - h with h on the 1/256
    lattice and every edge function (products of such offsets) is exact in float32
    and FP64, so the inclusive triangle test has one right answer for every h,
    including h on an edge or at a vertex."""
    rng = np.random.default_rng(seed)
    i = np.arange(n) - n // 2
    gx = i[None, :] * step + rng.integers(-jitter, jitter + 1, (n, n))
    gy = i[:, None] * step + rng.integers(-jitter, jitter + 1, (n, n))
    return (np.stack([gx, gy], axis=-1) / 128.0).astype(np.float32)


@pytest.mark.parametrize("n,step,jitter", [(16, 8, 1), (32, 4, 2)])
def test_query_normals_on_edges_and_vertices(P, oracle_mod, n, step, jitter):
    """h at texel normals (the six triangles around the vertex contain it), at the
    midpoints of mesh edges (horizontal, vertical and cell diagonals: both triangles
    of the edge) and at other 1/256-lattice points, with the footprint around that
    vertex or edge.  On the 16^2 map (no clamped cell) every decision is exact, so
    the GPU hit sets equal the oracle's exactly; on the 32^2 map some cells are
    clamped (replacement triangles off the lattice) and the sets agree outside the
    oracle's ambiguity band.  Brute force, plain and persistent give the same bits."""
    import torch
    announce("eval lattice map %d step %d: h on edges and vertices" % (n, step))
    nrm = lattice_map(n, 21 + n, step, jitter)
    clamped = oracle_mod.mesh(nrm)[1] != 0
    rng = np.random.default_rng(n)
    count = 1500
    third = count // 3
    ci = rng.integers(0, n, count)
    cj = rng.integers(0, n, count)
    q = np.zeros((count, 6), dtype=np.float32)
    # footprint around cell (ci, cj): its neighbours' triangles are in the support
    q[:, 0] = ci + 0.5 + n * rng.integers(-1, 2, count)
    q[:, 1] = cj + 0.5 + n * rng.integers(-1, 2, count)
    q[:, 2] = np.exp(rng.uniform(np.log(0.3), np.log(2.0 * n), count))
    q[:, 3] = q[:, 2] * np.exp(rng.uniform(-0.5, 0.5, count))
    q[:, 2:4] = np.maximum(q[:, 2:4], 0.3)
    kind = rng.integers(0, 3, count)
    i1, j1 = (ci + 1) % n, (cj + 1) % n
    pa = np.where(kind[:, None] == 2, nrm[cj, i1], nrm[cj, ci])          # edge start
    pb = np.select([kind[:, None] == 0, kind[:, None] == 1], [nrm[cj, i1], nrm[j1, ci]], nrm[j1, ci])
    q[:third, 4:6] = nrm[cj[:third], ci[:third]]                          # vertex (ci, cj)
    q[third:2 * third, 4:6] = (0.5 * (pa + pb))[third:2 * third]          # edge midpoints
    q[2 * third:, 4:6] = rng.integers(-140, 141, (count - 2 * third, 2)) / 256.0
    assert np.array_equal(q[:, 4:6] * 256.0, np.round(q[:, 4:6] * 256.0))
    _, hier = gpu_build(P, nrm, cluster=False)
    ref = oracle_mod.evaluate(nrm, q, records=True)
    d, off, ids, _ = gpu_hits(P, hier, q, algo="plain")
    st = compare(ref, d, off, ids)
    nhit = ref["nhit"]
    if not clamped.any():
        hoff, hid = ref["hit_off"], ref["hit_id"]
        for k in range(count):
            assert set(ids[off[k]:off[k + 1]].tolist()) == set(hid[hoff[k]:hoff[k + 1]].tolist()), k
        assert np.array_equal(nhit, np.diff(off))
        assert (nhit[:third] >= 6).all()
        assert (nhit[third:2 * third] >= 2).all()
    else:
        assert (nhit[:third] >= 6).mean() > 0.8
    assert st["nonzero"] > count // 2
    tq = to_dev(q)
    bits = [P.eval_batch(hier, tq, algo=algo).view(torch.int32) for algo in ("plain", "brute")]
    plan = P.Plan(hier, count)
    bits.append(plan.eval(tq).view(torch.int32))
    plan.close()
    torch.cuda.synchronize()
    assert torch.equal(bits[0], bits[1]) and torch.equal(bits[0], bits[2])


def test_deterministic_alone_and_in_the_mix(P):
    import torch
    import workloads
    announce("determinism: repeat and batch composition")
    nrm = workloads.make_map("powerlaw", 256, 12)
    _, hier = gpu_build(P, nrm, cluster=True)
    q = mixed_queries(256, 4000, 6, 0.5, 40.0, 0.3, spread=0)
    tq = to_dev(q)
    for tau in (0.0, 1e-3):
        a = P.eval_batch(hier, tq, tau=tau)
        b = P.eval_batch(hier, tq, tau=tau)
        assert torch.equal(a.view(torch.int32), b.view(torch.int32))
        sub = np.arange(5, 4000, 37)
        alone = P.eval_batch(hier, to_dev(q[sub]), tau=tau)
        assert torch.equal(alone.view(torch.int32), a[torch.from_numpy(sub).cuda()].view(torch.int32))
        perm = np.random.default_rng(1).permutation(4000)
        c = P.eval_batch(hier, to_dev(q[perm]), tau=tau)
        inv = np.argsort(perm)
        assert torch.equal(c[torch.from_numpy(inv).cuda()].view(torch.int32), a.view(torch.int32))


# ------------------------------------------------------- footprint kernels
@pytest.mark.parametrize("tau", [0.0, 1e-3])
@pytest.mark.parametrize("kernel", ["disk", "box"])
@pytest.mark.parametrize("name", ["bumps64", "powerlaw128", "scratched128"])
def test_footprint_kernels(P, oracle_mod, name, kernel, tau):
    """Disk and box footprints (support half-axes 1.5 sigma, normalised over
    the support, truncated where the triangle is hit): plain against the
    oracle, and brute (tau = 0) and the persistent kernel bit-identical to
    plain."""
    import torch
    announce("eval %s kernel tau=%g %s" % (kernel, tau, name))
    nrm = MAPS[name]()
    n = nrm.shape[0]
    clusters = oracle_mod.cluster_all(nrm) if tau > 0 else None
    q = mixed_queries(n, 1201, 31, 0.05, 0.5 * n, normal_radius(nrm))
    _, hier = gpu_build(P, nrm, cluster=tau > 0)
    d, off, ids, terms = gpu_hits(P, hier, q, tau=tau, algo="plain", kernel=kernel, sigma_to_r=1.5)
    ref = oracle_mod.evaluate(nrm, q, tau=tau, clusters=clusters, records=True, kernel=kernel,
                              sigma_to_r=1.5)
    st = compare(ref, d, off, ids)
    print(st)
    assert st["nonzero"] > 50
    assert st["cut_ambiguous"] <= 20
    qd = to_dev(q)
    plain = P.eval_batch(hier, qd, tau=tau, algo="plain", kernel=kernel, sigma_to_r=1.5).cpu().numpy()
    np.testing.assert_array_equal(plain.view(np.uint32), d.view(np.uint32))
    if tau == 0:
        brute = P.eval_batch(hier, qd, algo="brute", kernel=kernel, sigma_to_r=1.5).cpu().numpy()
        np.testing.assert_array_equal(brute.view(np.uint32), d.view(np.uint32))
    plan = P.Plan(hier, len(q), tau=tau, sigma_to_r=1.5, kernel=kernel)
    pers = plan.eval(qd).cpu().numpy()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(pers.view(np.uint32), d.view(np.uint32))


def test_footprint_kernels_differ_from_gaussian(P, oracle_mod):
    """The three kernels weight the same hits differently: on a flat region the
    box and disk values are their constant densities."""
    announce("eval kernel comparison on a flat map")
    nrm = np.zeros((16, 16, 2), dtype=np.float32)
    nrm[..., 0] = 0.125
    nrm[..., 1] = -0.0625
    _, hier = gpu_build(P, nrm, cluster=False)
    q = np.array([[8.0, 8.0, 2.0, 3.0, 0.125, -0.0625]], dtype=np.float32)
    out = {}
    for k in ("gaussian", "disk", "box"):
        out[k] = float(P.eval_batch(hier, to_dev(q), kernel=k, sigma_to_r=1.5).cpu().numpy()[0])
        ref = oracle_mod.evaluate(nrm, q, kernel=k, sigma_to_r=1.5)["D"][0]
        assert abs(out[k] - ref) <= 1e-4 * ref, (k, out[k], ref)
    assert len({round(v, 3) for v in out.values()}) == 3


def test_launches_split_into_chunks(P, oracle_mod):
    """Calls whose batch exceeds a launch's query count run as several launches (each
    covering its own slots); with the launch size forced down to 1000 queries every
    entry point returns the bits of a single launch."""
    import os
    import torch
    import workloads
    announce("launch chunking: 5000 queries in launches of 1000")
    nrm = workloads.make_map("powerlaw", 128, 7)
    _, hier = gpu_build(P, nrm, cluster=True)
    q = mixed_queries(128, 5000, 41, 0.3, 30.0, normal_radius(nrm), spread=0)
    tq = to_dev(q)
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    xi = torch.rand((2, 5000, 2), dtype=torch.float64, device="cuda", generator=g)
    w = q.copy()
    w[:, 4:6] = 0.5 * w[:, 4:6]
    tw = to_dev(w)

    def run():
        out = {}
        for algo in ("plain", "brute"):
            out[algo] = P.eval_batch(hier, tq, algo=algo).cpu().numpy()
        out["cut"] = P.eval_batch(hier, tq, tau=1e-3).cpu().numpy()
        out["counts"] = P.eval_counts(hier, tq)[1].cpu().numpy()
        d, off, ids, terms = P.eval_hits(hier, tq, tau=1e-3)
        out["hits"] = (d.cpu().numpy(), off.cpu().numpy(), ids.cpu().numpy())
        m, tri, u = P.sample_batch(hier, tq, xi, tau=1e-3, u=True)
        out["sample"] = (m.cpu().numpy(), tri.cpu().numpy(), u.cpu().numpy())
        out["proj"] = P.projected_area(hier, tw).cpu().numpy()
        torch.cuda.synchronize()
        return out

    one = run()
    os.environ["PNDF_LAUNCH_CHUNK"] = "1000"
    try:
        many = run()
    finally:
        del os.environ["PNDF_LAUNCH_CHUNK"]
    for key in one:
        a, b = one[key], many[key]
        for x, y in (zip(a, b) if isinstance(a, tuple) else [(a, b)]):
            assert np.array_equal(x.view(np.uint8), y.view(np.uint8)), key
    assert np.isfinite(one["plain"]).all() and (one["plain"] > 0).sum() > 500


@pytest.mark.parametrize("nq", [4095, 4096, 40000])
def test_spatial_order_changes_no_bit(P, nq):
    """Batches from 4096 queries on run in spatial order, smaller ones in input order:
    either way every result equals the input-order evaluation bit for bit (the sums
    are exact), at and around the threshold, with and without the cut."""
    import torch
    import workloads
    announce("spatial order vs input order, %d queries" % nq)
    nrm = workloads.make_map("powerlaw", 256, 61)
    _, hier = gpu_build(P, nrm, cluster=True)
    q = torch.from_numpy(workloads.uniform_queries(256, nq, 62, (0.5, 64.0), 0.4)).cuda()
    for tau in (0.0, 1e-3):
        a = P.eval_batch(hier, q, tau=tau).cpu().numpy()
        b = P.eval_batch(hier, q, tau=tau, input_order=True).cpu().numpy()
        np.testing.assert_array_equal(a.view(np.uint32), b.view(np.uint32))
        assert np.isfinite(a).all() and (a > 0).mean() > 0.05
