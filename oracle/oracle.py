"""ctypes wrapper around the FP64 oracle (pndf_oracle.c).

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports this module.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pndf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def build(force=True):
    """Compile the oracle with gcc (OpenMP, no fast-math, no FMA contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
           "-ffp-contract=off", "-Wall", "-Wno-unknown-pragmas", _SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    lib.or_mesh.argtypes = [ctypes.c_int, _fp, ctypes.c_float, _dp, _u8p]
    lib.or_cluster_nodes.argtypes = [ctypes.c_int, _fp, ctypes.c_float, ctypes.c_int, _i64p,
                                     ctypes.c_int64, _dp, _dp]
    lib.or_fine_contrib.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    _dp, _dp, _dp, _dp]
    lib.or_eval.argtypes = [ctypes.c_int, _fp, ctypes.c_float, _dp, _dp, _fp, ctypes.c_int64,
                            ctypes.c_float, ctypes.c_float, ctypes.c_double,
                            _dp, _i64p, _i64p, _i32p,
                            _i64p, _u64p, _dp, _i64p, _u64p, _dp, _u8p]
    lib.or_eval_k.argtypes = [ctypes.c_int, _fp, ctypes.c_float, _dp, _dp, _fp, ctypes.c_int64,
                              ctypes.c_float, ctypes.c_float, ctypes.c_double, ctypes.c_int,
                              _dp, _i64p, _i64p, _i32p,
                              _i64p, _u64p, _dp, _i64p, _u64p, _dp, _u8p]
    lib.or_sample_normals.argtypes = [ctypes.c_int, _fp, ctypes.c_float, _dp, ctypes.c_int64, _dp]
    lib.or_sample_k.argtypes = [ctypes.c_int, _fp, ctypes.c_float, _dp, _dp, _fp, _dp, ctypes.c_int64,
                                ctypes.c_int, ctypes.c_float, ctypes.c_float, ctypes.c_double, ctypes.c_int,
                                _dp, _dp, _u64p, _i32p]
    lib.or_projected_area.argtypes = [ctypes.c_int, _fp, ctypes.c_float, _fp, ctypes.c_int64, ctypes.c_float,
                                      ctypes.c_int, _dp]
    lib.or_tri_projected.argtypes = [_dp, _dp]
    lib.or_tri_projected.restype = ctypes.c_double
    lib.or_num_threads.argtypes = []
    lib.or_set_threads.argtypes = [ctypes.c_int]
    lib.or_set_threads.restype = None
    for f in (lib.or_mesh, lib.or_cluster_nodes, lib.or_fine_contrib, lib.or_eval, lib.or_eval_k,
              lib.or_sample_normals, lib.or_sample_k, lib.or_projected_area, lib.or_num_threads):
        f.restype = ctypes.c_int
    _lib = lib
    return lib


def set_threads(n):
    """Run the oracle's parallel loops on n host threads from now on."""
    load().or_set_threads(int(n))


def num_threads():
    """OpenMP threads the oracle runs with."""
    return int(load().or_num_threads())


def _p(a, t):
    return None if a is None else a.ctypes.data_as(t)


def _map(nrm):
    nrm = np.ascontiguousarray(nrm, dtype=np.float32)
    if nrm.ndim != 3 or nrm.shape[0] != nrm.shape[1] or nrm.shape[2] != 2:
        raise ValueError("normal map must be (N, N, 2)")
    return nrm


def mesh(nrm, eps=1e-6):
    """Per-cell Jacobians (N, N, 2) [lower, upper] in FP64 and clamp bits (N, N)."""
    nrm = _map(nrm)
    n = nrm.shape[0]
    det = np.empty((n, n, 2), dtype=np.float64)
    deg = np.empty((n, n), dtype=np.uint8)
    rc = load().or_mesh(n, _p(nrm, _fp), eps, _p(det, _dp), _p(deg, _u8p))
    if rc:
        raise ValueError("or_mesh failed (%d)" % rc)
    return det, deg


def cluster_level(nrm, level, eps=1e-6, ids=None):
    """Cluster fit of the given node ids (row-major at that level; default all).
    Returns (nstar (k, 4, 2) FP64, e (k,) FP64)."""
    nrm = _map(nrm)
    n = nrm.shape[0]
    m = n >> level
    if ids is None:
        ids = np.arange(m * m, dtype=np.int64)
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    ns = np.empty((len(ids), 4, 2), dtype=np.float64)
    e = np.empty(len(ids), dtype=np.float64)
    rc = load().or_cluster_nodes(n, _p(nrm, _fp), eps, level, _p(ids, _i64p), len(ids),
                                 _p(ns, _dp), _p(e, _dp))
    if rc:
        raise ValueError("or_cluster_nodes failed (%d)" % rc)
    return ns, e


def cluster_all(nrm, eps=1e-6):
    """Every level's cluster fit.  Returns a dict: `levels` {l: (nstar (m*m, 4, 2),
    e (m*m,)) FP64, row-major nodes}, views into the packed FP64 arrays `clu_n64`
    (8 per node) and `clu_e64` (levels 1..L), which `evaluate` and `sample` take
    (they decide on the float32 roundings, as a stored hierarchy does), and those
    roundings `clu_n`, `clu_e` (float32)."""
    nrm = _map(nrm)
    n = nrm.shape[0]
    L = int(np.log2(n))
    total = sum((n >> l) ** 2 for l in range(1, L + 1))
    clu_n64 = np.empty(total * 8, dtype=np.float64)
    clu_e64 = np.empty(total, dtype=np.float64)
    levels = {}
    off = 0
    lib = load()
    for l in range(1, L + 1):
        m = (n >> l) ** 2
        ns = clu_n64[8 * off:8 * (off + m)].reshape(m, 4, 2)
        e = clu_e64[off:off + m]
        ids = np.arange(m, dtype=np.int64)
        rc = lib.or_cluster_nodes(n, _p(nrm, _fp), eps, l, _p(ids, _i64p), m, _p(ns, _dp), _p(e, _dp))
        if rc:
            raise ValueError("or_cluster_nodes failed (%d)" % rc)
        levels[l] = (ns, e)
        off += m
    return dict(levels=levels, clu_n64=clu_n64, clu_e64=clu_e64,
                clu_n=clu_n64.astype(np.float32), clu_e=clu_e64.astype(np.float32))


def fine_contrib(a, i, j, half, nv):
    """One fine triangle's (A, B, C) with unit weight; nv = (4, 2) corner normals.
    Returns (A (4,4), B (4,2), C, cluster_half)."""
    nv = np.ascontiguousarray(nv, dtype=np.float64).reshape(8)
    A = np.zeros(16)
    B = np.zeros(8)
    C = np.zeros(1)
    ch = load().or_fine_contrib(a, i, j, half, _p(nv, _dp), _p(A, _dp), _p(B, _dp), _p(C, _dp))
    return A.reshape(4, 4), B.reshape(4, 2), float(C[0]), ch


KERNELS = {"gaussian": 0, "disk": 1, "box": 2}


def evaluate(nrm, queries, tau=0.0, eps=1e-6, sigma_to_r=3.0, band=1e-6, clusters=None,
             records=False, kernel="gaussian"):
    """Evaluate queries (Q, 6) float32.  Returns dict with D (FP64), nhit, namb, flags
    and, with records=True, per-query hit and ambiguous-triangle lists as CSR:
    hit_off, hit_id, hit_term, amb_off, amb_id, amb_term, amb_hit.
    kernel: "gaussian" (sigma the standard deviation, support r = sigma_to_r sigma),
    "disk" or "box" (normalised over the ellipse / rectangle of half-axes
    r = sigma_to_r sigma, truncated at the hit point)."""
    kid = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    nrm = _map(nrm)
    n = nrm.shape[0]
    q = np.ascontiguousarray(queries, dtype=np.float32).reshape(-1, 6)
    nq = q.shape[0]
    if tau > 0 and clusters is None:
        clusters = cluster_all(nrm, eps)
    cn = clusters["clu_n64"] if clusters is not None else None
    ce = clusters["clu_e64"] if clusters is not None else None
    D = np.empty(nq, dtype=np.float64)
    nhit = np.empty(nq, dtype=np.int64)
    namb = np.empty(nq, dtype=np.int64)
    flags = np.empty(nq, dtype=np.int32)
    lib = load()
    args = [n, _p(nrm, _fp), eps, _p(cn, _dp), _p(ce, _dp), _p(q, _fp), nq, tau, sigma_to_r,
            band, kid, _p(D, _dp), _p(nhit, _i64p), _p(namb, _i64p), _p(flags, _i32p)]
    rc = lib.or_eval_k(*args, None, None, None, None, None, None, None)
    if rc:
        raise ValueError("or_eval failed (%d)" % rc)
    out = dict(D=D, nhit=nhit, namb=namb, flags=flags)
    if not records:
        return out
    hoff = np.zeros(nq + 1, dtype=np.int64)
    hoff[1:] = np.cumsum(nhit)
    aoff = np.zeros(nq + 1, dtype=np.int64)
    aoff[1:] = np.cumsum(namb)
    hid = np.zeros(max(1, hoff[-1]), dtype=np.uint64)
    hterm = np.zeros(max(1, hoff[-1]), dtype=np.float64)
    aid = np.zeros(max(1, aoff[-1]), dtype=np.uint64)
    aterm = np.zeros(max(1, aoff[-1]), dtype=np.float64)
    ahit = np.zeros(max(1, aoff[-1]), dtype=np.uint8)
    D2 = np.empty(nq, dtype=np.float64)
    rc = lib.or_eval_k(n, _p(nrm, _fp), eps, _p(cn, _dp), _p(ce, _dp), _p(q, _fp), nq, tau,
                     sigma_to_r, band, kid, _p(D2, _dp), _p(nhit, _i64p), _p(namb, _i64p),
                     _p(flags, _i32p), _p(hoff, _i64p), _p(hid, _u64p), _p(hterm, _dp),
                     _p(aoff, _i64p), _p(aid, _u64p), _p(aterm, _dp), _p(ahit, _u8p))
    if rc:
        raise ValueError("or_eval failed (%d)" % rc)
    out.update(hit_off=hoff, hit_id=hid[:hoff[-1]], hit_term=hterm[:hoff[-1]],
               amb_off=aoff, amb_id=aid[:aoff[-1]], amb_term=aterm[:aoff[-1]],
               amb_hit=ahit[:aoff[-1]].astype(bool))
    return out


def sample_normals(nrm, u, eps=1e-6):
    """n(u) of Eq. (interpolation) at points u (K, 2), with the clamp-consistent
    warp of Eq. (debias) inside clamped triangles."""
    nrm = _map(nrm)
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, 2)
    out = np.empty_like(u)
    rc = load().or_sample_normals(nrm.shape[0], _p(nrm, _fp), eps, _p(u, _dp), len(u),
                                  _p(out, _dp))
    if rc:
        raise ValueError("or_sample_normals failed")
    return out


def sample(nrm, queries, xi, tau=0.0, eps=1e-6, sigma_to_r=3.0, kernel="gaussian", clusters=None,
           band=1e-8):
    """Draw one sample of the P-NDF per query (Q, 6) float32 (x, y, sx, sy used)
    from the uniforms xi (Q, 2 * attempts) float64 in [0, 1).  Returns dict u (Q, 2)
    unrolled texture coordinates, m (Q, 2) sampled normals, tri (Q,) triangle ids,
    flags (Q,): bit0 a cut or cluster clamp decision that another FP64 fit could take
    differently after float32 rounding, bit1 u within
    `band` of a unit edge / diagonal, bit2 every attempt rejected."""
    kid = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    nrm = _map(nrm)
    q = np.ascontiguousarray(queries, dtype=np.float32).reshape(-1, 6)
    nq = q.shape[0]
    xi = np.ascontiguousarray(xi, dtype=np.float64).reshape(nq, -1)
    attempts = xi.shape[1] // 2
    assert xi.shape[1] == 2 * attempts and attempts >= 1
    if tau > 0 and clusters is None:
        clusters = cluster_all(nrm, eps)
    cn = clusters["clu_n64"] if clusters is not None else None
    ce = clusters["clu_e64"] if clusters is not None else None
    u = np.empty((nq, 2))
    m = np.empty((nq, 2))
    tri = np.empty(nq, dtype=np.uint64)
    flags = np.empty(nq, dtype=np.int32)
    rc = load().or_sample_k(nrm.shape[0], _p(nrm, _fp), eps, _p(cn, _dp), _p(ce, _dp), _p(q, _fp),
                            _p(xi, _dp), nq, attempts, tau, sigma_to_r, band, kid,
                            _p(u, _dp), _p(m, _dp), _p(tri, _u64p), _p(flags, _i32p))
    if rc:
        raise ValueError("or_sample_k failed (%d)" % rc)
    return dict(u=u, m=m, tri=tri, flags=flags)


def projected_area(nrm, queries, eps=1e-6, sigma_to_r=3.0, kernel="gaussian"):
    """P(w) per query (Q, 6) float32: x, y, sx, sy, w_x, w_y (w_z = sqrt(1 - w_x^2 - w_y^2)),
    with the footprint kernel constant over each triangle (its value at the uv
    centroid).  Brute force, FP64."""
    kid = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    nrm = _map(nrm)
    q = np.ascontiguousarray(queries, dtype=np.float32).reshape(-1, 6)
    out = np.empty(len(q))
    rc = load().or_projected_area(nrm.shape[0], _p(nrm, _fp), eps, _p(q, _fp), len(q), sigma_to_r, kid,
                                  _p(out, _dp))
    if rc:
        raise ValueError("or_projected_area failed (%d)" % rc)
    return out


def tri_projected(tri, w):
    """Integral of (w . m~) / m~_z over the part of the normal triangle tri (3, 2)
    where m~ . w >= 0 and |m| <= 1, for the unit direction w (3,), w_z >= 0."""
    tri = np.ascontiguousarray(tri, dtype=np.float64).reshape(3, 2)
    w = np.ascontiguousarray(w, dtype=np.float64).reshape(3)
    return float(load().or_tri_projected(_p(tri, _dp), _p(w, _dp)))


def triangle_id(level, I, J, half):
    """Triangle id encoding: level (6 bits) | J (29 bits) | I (28 bits) | half."""
    return (np.uint64(level) << np.uint64(58)) | (np.uint64(J) << np.uint64(29)) | \
        (np.uint64(I) << np.uint64(1)) | np.uint64(half)


def decode_id(ids):
    ids = np.asarray(ids, dtype=np.uint64)
    level = (ids >> np.uint64(58)).astype(np.int64)
    J = ((ids >> np.uint64(29)) & np.uint64((1 << 29) - 1)).astype(np.int64)
    I = ((ids >> np.uint64(1)) & np.uint64((1 << 28) - 1)).astype(np.int64)
    half = (ids & np.uint64(1)).astype(np.int64)
    return level, I, J, half
