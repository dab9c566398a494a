"""The benchmark's CPU counting pass (bench_workcount.c) against a direct Python walk
of the same rules on small random hierarchies: entry level and roots from the
support box, one box test per visited node, a node under the cut counted as a
cluster node when h lies in its box (from level 2 up the box of its own cluster
triangles), cells counted at level 1, and a non-root node of level 3 or more whose
children are all under the cut tested a second time, against the union of their
own boxes, and left unexpanded when it misses h.  CPU only."""
import math

import numpy as np
import pytest

import bench


def walk(n, box, own, e, q, tau, s2r, union_skip=True):
    L = int(math.log2(n))
    off = {}
    o = 0
    for l in range(1, L + 1):
        off[l] = o
        o += (n >> l) ** 2
    x, y, sx, sy, hx, hy = [float(v) for v in q]
    rx, ry = np.float32(s2r) * np.float32(sx), np.float32(s2r) * np.float32(sy)
    clo = [math.ceil(np.float32(x) - rx) - 1, math.ceil(np.float32(y) - ry) - 1]
    chi = [math.floor(np.float32(x) + rx), math.floor(np.float32(y) + ry)]
    t = np.float32(np.float32(rx * ry) * np.float32(tau))
    cut = tau > 0

    def meets(start, s, lo, hi):
        # some periodic image [start + p n, start + p n + s - 1] meets [lo, hi]
        return any(start + p * n <= hi and start + p * n + s - 1 >= lo for p in range(-3, 4))

    def inside(b, px, py):
        return b[0] <= px <= b[2] and b[1] <= py <= b[3]

    cnt = [0, 0, 0]

    def visit(l, I, J, root=False):
        m = n >> l
        k = off[l] + J * m + I
        cnt[0] += 1
        if cut and e[k] <= t:
            b = own[k] if l >= 2 else box[k]
            if inside(b, np.float32(hx), np.float32(hy)):
                cnt[2] += 1
            return
        if not inside(box[k], np.float32(hx), np.float32(hy)):
            return
        if union_skip and cut and not root and l >= 3:
            mc = n >> (l - 1)
            kids = [off[l - 1] + (2 * J + dj) * mc + 2 * I + di for dj in range(2) for di in range(2)]
            if all(e[kc] <= t for kc in kids):
                cnt[0] += 1   # the union box is a second box test
                if not any(inside(own[kc], np.float32(hx), np.float32(hy)) for kc in kids):
                    return
        s = 1 << (l - 1)
        for dj in range(2):
            for di in range(2):
                ci, cj = 2 * I + di, 2 * J + dj
                if not (meets(ci * s, s, clo[0], chi[0]) and meets(cj * s, s, clo[1], chi[1])):
                    continue
                if l == 1:
                    cnt[1] += 1
                else:
                    visit(l - 1, ci, cj)

    rmax = max(rx, ry)
    l0 = 0
    while l0 < L and (1 << l0) < rmax:
        l0 += 1
    m, s = n >> l0, 1 << l0
    a = [clo[0] // s, clo[1] // s]
    ln = [min(chi[0] // s - a[0] + 1, m), min(chi[1] // s - a[1] + 1, m)]
    for yy in range(ln[1]):
        J = (a[1] + yy) % m
        for xx in range(ln[0]):
            I = (a[0] + xx) % m
            if l0 == 0:
                cnt[1] += 1
            else:
                visit(l0, I, J, root=True)
    return cnt


@pytest.mark.parametrize("tau", [0.0, 0.005, 0.02])
def test_counting_pass_matches_a_direct_walk(tau):
    rng = np.random.default_rng(11)
    n = 32
    nodes = sum((n >> l) ** 2 for l in range(1, 6))
    c = rng.uniform(-0.5, 0.5, (nodes, 2)).astype(np.float32)
    w = rng.uniform(0.05, 0.6, (nodes, 2)).astype(np.float32)
    box = np.concatenate([c - w, c + w], axis=1).astype(np.float32)
    shrink = rng.uniform(0.0, 0.5, (nodes, 1)).astype(np.float32)
    own = np.concatenate([c - w * shrink, c + w * shrink], axis=1).astype(np.float32)
    # residuals grow about 4x per level, as fits of a rough map do
    lev = np.concatenate([np.full((n >> l) ** 2, l) for l in range(1, 6)])
    e = (rng.uniform(0.5, 2.0, nodes) * 0.01 * 4.0 ** lev).astype(np.float32)
    nq = 400
    q = np.stack([rng.uniform(0, n, nq), rng.uniform(0, n, nq), np.exp(rng.uniform(np.log(0.3), np.log(16.0), nq)),
                  np.exp(rng.uniform(np.log(0.3), np.log(16.0), nq)), rng.uniform(-0.6, 0.6, nq),
                  rng.uniform(-0.6, 0.6, nq)], axis=1).astype(np.float32)
    got = bench.count_work(n, np.ascontiguousarray(box.reshape(-1)), np.ascontiguousarray(own.reshape(-1)) if tau > 0 else None,
                           np.ascontiguousarray(e) if tau > 0 else None, q, tau, 3.0)
    want = np.array([walk(n, box, own, e, qq, tau, 3.0) for qq in q], dtype=np.float64)
    np.testing.assert_array_equal(got, want)
    assert want[:, 0].sum() > 0 and (tau == 0 or want[:, 2].sum() > 0)
    if tau > 0:
        # the union rule is exercised: without it more nodes would be visited
        full = np.array([walk(n, box, own, e, qq, tau, 3.0, union_skip=False) for qq in q], dtype=np.float64)
        assert (full[:, 0] != want[:, 0]).any() and (full[:, 1:] == want[:, 1:]).all()
