"""Parity checking of GPU results against the FP64 oracle.

Protocol: the oracle reports, per query, its hit triangles with their terms and
every triangle whose normal-space boundary lies within 1e-6 of the query normal
(ambiguous: hit or miss may flip under float32 rounding), with the term it would
contribute.  The GPU's hit-id set must equal the oracle's outside the ambiguous
set.  The reference value is then recomputed with the GPU's include/exclude
choice for each ambiguous triangle, and |D_gpu - D_ref| <= rtol * D_ref.
Queries with a cluster cut decision (oracle flag bit 0) or a cluster clamp
decision (bit 2) that an independent fit could take differently after float32
rounding, or with a triangle whose footprint-support test for the disk or box
kernel is within rounding of its edge (bit 1), are excluded from the strict
comparison and counted.
The GPU result is a float32: below float32's normal range (FLT_MIN = 2^-126) it
cannot carry relative precision, so the bound has an absolute floor of
rtol * FLT_MIN.
"""
import numpy as np

RTOL = 1e-4
FLT_MIN = float(np.finfo(np.float32).tiny)


def _split(off, vals):
    return [vals[off[k]:off[k + 1]] for k in range(len(off) - 1)]


def compare(ref, d_gpu, gpu_off=None, gpu_ids=None, rtol=RTOL, check_ids=True):
    """ref: oracle.evaluate(..., records=True) dict.  d_gpu: (Q,) float32.
    gpu_off / gpu_ids: CSR hit lists from the GPU (optional).
    Returns a dict of statistics; raises AssertionError on a mismatch."""
    d_gpu = np.asarray(d_gpu, dtype=np.float64)
    nq = len(d_gpu)
    D = ref["D"]
    flags = ref["flags"]
    nan_ref = np.isnan(D)
    assert np.array_equal(nan_ref, np.isnan(d_gpu)), "NaN pattern differs"
    skip = (flags & 7) != 0
    hoff, hid, hterm = ref["hit_off"], ref["hit_id"], ref["hit_term"]
    aoff, aid, aterm = ref["amb_off"], ref["amb_id"], ref["amb_term"]
    worst = 0.0
    n_amb_q = 0
    bad = []
    for k in range(nq):
        if nan_ref[k] or skip[k]:
            continue
        h_ids = hid[hoff[k]:hoff[k + 1]]
        h_terms = hterm[hoff[k]:hoff[k + 1]]
        a_ids = aid[aoff[k]:aoff[k + 1]]
        a_terms = aterm[aoff[k]:aoff[k + 1]]
        amb = set(a_ids.tolist())
        if amb:
            n_amb_q += 1
        if gpu_ids is not None:
            g = gpu_ids[gpu_off[k]:gpu_off[k + 1]].tolist()
            gset = set(g)
            if check_ids:
                assert len(gset) == len(g), "query %d: duplicate GPU hit ids" % k
                diff = gset.symmetric_difference(set(h_ids.tolist()))
                if not diff <= amb:
                    bad.append((k, sorted(diff - amb)[:4]))
                    continue
            # reference with the GPU's choice on ambiguous triangles
            dref = float(sum(t for i, t in zip(h_ids.tolist(), h_terms.tolist()) if i not in amb))
            dref += float(sum(t for i, t in zip(a_ids.tolist(), a_terms.tolist()) if i in gset))
        else:
            if amb:
                # without the GPU's ids, accept any choice on the ambiguous set
                base = float(sum(t for i, t in zip(h_ids.tolist(), h_terms.tolist()) if i not in amb))
                lo, hi = base, base + float(np.sum(a_terms))
                if lo * (1 - rtol) - rtol * FLT_MIN <= d_gpu[k] <= hi * (1 + rtol) + rtol * FLT_MIN:
                    continue
                bad.append((k, "value %r outside [%r, %r]" % (d_gpu[k], lo, hi)))
                continue
            dref = D[k]
        if dref == 0.0:
            if d_gpu[k] != 0.0:
                bad.append((k, "gpu %r ref 0" % d_gpu[k]))
            continue
        err = abs(d_gpu[k] - dref)
        if dref >= FLT_MIN:
            worst = max(worst, err / dref)
        if err > rtol * max(dref, FLT_MIN):
            bad.append((k, "rel err %.3g (gpu %r ref %r)" % (err / dref, d_gpu[k], dref)))
    assert not bad, "%d mismatching queries, first: %s" % (len(bad), bad[:5])
    return dict(worst_rel=worst, ambiguous_queries=n_amb_q, cut_ambiguous=int(skip.sum()),
                nonzero=int((np.nan_to_num(D) > 0).sum()))


FIT_E_REL, FIT_E_ABS, FIT_N_ABS = 1e-10, 1e-20, 1e-10   # the oracle's stated fit agreement


def rounded_interval(x, tol):
    """The float32 values an FP64 value within tol of x can round to: [fl32(x - tol),
    fl32(x + tol)] (rounding is monotone)."""
    return (x - tol).astype(np.float32), (x + tol).astype(np.float32)


def check_cluster_fit(ex, ns, e, m, level):
    """The GPU fit of one level against the oracle's FP64 fit (Eq. normal_optimization,
    e^l its minimised value).  The oracle flags the cut and clamp decisions that two
    FP64 fits agreeing to 1e-10 (e^l: relative, plus 1e-20 of the level's largest;
    normals: absolute) could take differently after float32 rounding; this checks
    that premise node by node: every stored float32 value is a rounding of a value
    within that bound of the oracle's."""
    gn = ex["clu_n"].cpu().numpy().reshape(m * m, 4, 2)
    ge = ex["clu_e"].cpu().numpy().reshape(m * m)
    lo, hi = rounded_interval(ns, FIT_N_ABS)
    bad_n = (gn < lo) | (gn > hi)
    assert not bad_n.any(), (level, int(bad_n.sum()), float(np.abs(gn.astype(np.float64) - ns).max()))
    lo, hi = rounded_interval(e, FIT_E_REL * np.abs(e) + FIT_E_ABS * float(e.max()))
    bad_e = (ge < lo) | (ge > hi)
    assert not bad_e.any(), (level, int(bad_e.sum()), float((np.abs(ge - e) / np.maximum(e, 1e-300)).max()))
    n32, e32 = ns.astype(np.float32), e.astype(np.float32)
    print("level %d: float32 N* differ from the oracle's rounding in %d of %d, e^l in %d of %d"
          % (level, int((gn != n32).sum()), gn.size, int((ge != e32).sum()), ge.size))
