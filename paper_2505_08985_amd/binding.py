"""Python binding of the C ABI in include/pndf.h (argument marshalling only).

Device memory and streams come from PyTorch-ROCm; every step of the evaluation
runs in the library's HIP kernels.  There is no CPU fallback: if the library is
not built this module raises on import.
"""
import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpndf.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libpndf.so is not built: run `python -m paper_2505_08985_amd.build` "
                      "(or __graft_entry__.build()) first")
_lib = ctypes.CDLL(LIB_PATH)

PNDF_OK, PNDF_EINVAL, PNDF_ENOMEM, PNDF_EDEVICE, PNDF_EOVERFLOW, PNDF_EUNSUPPORTED, PNDF_EAGAIN = range(7)
ALGOS = {"auto": 0, "brute": 1, "plain": 2, "persistent": 3}

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_f32 = ctypes.c_float


class EvalOpts(ctypes.Structure):
    _fields_ = [("kernel", _i32), ("tau", _f32), ("sigma_to_r", _f32), ("algo", _i32), ("flags", _i32)]


class HierOpts(ctypes.Structure):
    _fields_ = [("cluster", _i32)]


class Tuning(ctypes.Structure):
    _fields_ = [("blocks_per_cu", _i32), ("split_level", _i32), ("queue_factor", _i32), ("use_graph", _i32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class PlanStats(ctypes.Structure):
    _fields_ = [("spawned", _u64), ("refused", _u64), ("idle_spins", _u64), ("error", ctypes.c_uint32)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_build_mesh = _sig("pndf_build_mesh", _i32, [_vp, _i32, _f32, _vp, ctypes.POINTER(_vp)])
_build_hier = _sig("pndf_build_hierarchy", _i32, [_vp, ctypes.POINTER(HierOpts), _vp, ctypes.POINTER(_vp)])
_eval_batch = _sig("pndf_eval_batch", _i32, [_vp, _vp, _i64, ctypes.POINTER(EvalOpts), _vp, _vp])
_eval_batch_noalloc = _sig("pndf_eval_batch_noalloc", _i32, [_vp, _vp, _i64, ctypes.POINTER(EvalOpts), _vp, _vp])
_eval_counts = _sig("pndf_eval_counts", _i32, [_vp, _vp, _i64, ctypes.POINTER(EvalOpts), _vp, _vp, _vp])
_eval_hits = _sig("pndf_eval_hits", _i32, [_vp, _vp, _i64, ctypes.POINTER(EvalOpts), _vp, _vp, _vp, _vp,
                                           _u64, ctypes.POINTER(_u64), _vp])
_sample_batch = _sig("pndf_sample_batch", _i32, [_vp, _vp, _i64, _vp, _i32, ctypes.POINTER(EvalOpts), _vp, _vp,
                                                 _vp, _vp])
_projected_area = _sig("pndf_projected_area", _i32, [_vp, _vp, _i64, ctypes.POINTER(EvalOpts), _vp, _vp, _vp])
_destroy_mesh = _sig("pndf_destroy_mesh", None, [_vp])
_destroy_hier = _sig("pndf_destroy_hierarchy", None, [_vp])
_status_string = _sig("pndf_status_string", ctypes.c_char_p, [_i32])
_last_error = _sig("pndf_last_error", ctypes.c_char_p, [])
_mesh_info = _sig("pndf_mesh_info", _i32, [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_f32), ctypes.POINTER(_i64)])
_mesh_export = _sig("pndf_mesh_export", _i32, [_vp, _vp, _vp, _vp])
_hier_info = _sig("pndf_hier_info", _i32, [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i64)])
_hier_export = _sig("pndf_hier_export_level", _i32, [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp])

_default_tuning = _sig("pndf_default_tuning", _i32, [_vp, ctypes.POINTER(Tuning)])
_plan_create = _sig("pndf_plan_create", _i32, [_vp, _i64, ctypes.POINTER(EvalOpts), ctypes.POINTER(Tuning), _vp,
                                               ctypes.POINTER(_vp)])
_plan_eval = _sig("pndf_plan_eval", _i32, [_vp, _vp, _i64, _vp, _vp])
_plan_get_stats = _sig("pndf_plan_get_stats", _i32, [_vp, ctypes.POINTER(PlanStats), _vp])
_plan_get_tuning = _sig("pndf_plan_get_tuning", _i32, [_vp, ctypes.POINTER(Tuning)])
_plan_destroy = _sig("pndf_plan_destroy", None, [_vp])
_autotune = _sig("pndf_autotune", _i32, [_vp, _vp, _i64, ctypes.POINTER(EvalOpts), ctypes.POINTER(Tuning),
                                         ctypes.POINTER(ctypes.c_double), _vp])

EXPORTED = ["pndf_build_mesh", "pndf_build_hierarchy", "pndf_eval_batch", "pndf_eval_batch_noalloc", "pndf_eval_counts",
            "pndf_eval_hits", "pndf_sample_batch", "pndf_projected_area", "pndf_destroy_mesh", "pndf_destroy_hierarchy", "pndf_status_string",
            "pndf_last_error", "pndf_mesh_info", "pndf_mesh_export", "pndf_hier_info",
            "pndf_hier_export_level", "pndf_default_tuning", "pndf_plan_create", "pndf_plan_eval",
            "pndf_plan_get_stats", "pndf_plan_get_tuning", "pndf_plan_destroy", "pndf_autotune"]


class PndfError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _last_error().decode(errors="replace")
        super().__init__("%s: %s (%s)" % (where, _status_string(status).decode(), msg))


def _check(st, where):
    if st != PNDF_OK:
        raise PndfError(st, where)


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return _vp(stream.cuda_stream)


def _dev_ptr(t, dtype, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s" % (name, dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return _vp(t.data_ptr())


class Mesh:
    def __init__(self, handle, n, eps):
        self._h = handle
        self.n = n
        self.eps = eps

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            _destroy_mesh(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Hierarchy:
    def __init__(self, handle, mesh, cluster):
        self._h = handle
        self.mesh = mesh
        self.n = mesh.n
        self.cluster = cluster

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            _destroy_hier(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_mesh(normals, eps=1e-6, stream=None):
    """normals: (N, N, 2) float32 device tensor."""
    if normals.dim() != 3 or normals.shape[0] != normals.shape[1] or normals.shape[2] != 2:
        raise ValueError("normals must have shape (N, N, 2)")
    out = _vp()
    _check(_build_mesh(_dev_ptr(normals, torch.float32, "normals"), int(normals.shape[0]), float(eps),
                       _stream(stream), ctypes.byref(out)), "pndf_build_mesh")
    return Mesh(out, int(normals.shape[0]), float(eps))


def build_hierarchy(mesh, cluster=True, stream=None):
    out = _vp()
    opts = HierOpts(1 if cluster else 0)
    _check(_build_hier(mesh.handle, ctypes.byref(opts), _stream(stream), ctypes.byref(out)),
           "pndf_build_hierarchy")
    return Hierarchy(out, mesh, bool(cluster))


EVAL_INPUT_ORDER = 1


KERNELS = {"gaussian": 0, "disk": 1, "box": 2}


def _opts(tau, sigma_to_r, algo, kernel=0, flags=0):
    kernel = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    return EvalOpts(int(kernel), float(tau), float(sigma_to_r), ALGOS[algo] if isinstance(algo, str) else int(algo),
                    int(flags))


def _queries(q):
    if q.dim() != 2 or q.shape[1] != 6:
        raise ValueError("queries must have shape (Q, 6)")
    return _dev_ptr(q, torch.float32, "queries"), int(q.shape[0])


def eval_batch(hier, queries, tau=0.0, sigma_to_r=3.0, algo="auto", out=None, stream=None, kernel=0,
               input_order=False):
    qp, nq = _queries(queries)
    if out is None:
        out = torch.empty(nq, dtype=torch.float32, device=queries.device)
    o = _opts(tau, sigma_to_r, algo, kernel, EVAL_INPUT_ORDER if input_order else 0)
    _check(_eval_batch(hier.handle, qp, nq, ctypes.byref(o), _dev_ptr(out, torch.float32, "out"),
                       _stream(stream)), "pndf_eval_batch")
    return out


def eval_batch_noalloc(hier, queries, tau=0.0, sigma_to_r=3.0, algo="auto", out=None, stream=None, kernel=0,
                       input_order=False):
    """pndf_eval_batch_noalloc: as eval_batch, with the library's static workspace
    (at most 2^22 queries; calls on one GPU must not overlap)."""
    qp, nq = _queries(queries)
    if out is None:
        out = torch.empty(nq, dtype=torch.float32, device=queries.device)
    o = _opts(tau, sigma_to_r, algo, kernel, EVAL_INPUT_ORDER if input_order else 0)
    _check(_eval_batch_noalloc(hier.handle, qp, nq, ctypes.byref(o), _dev_ptr(out, torch.float32, "out"),
                               _stream(stream)), "pndf_eval_batch_noalloc")
    return out


def sample_batch(hier, queries, xi, tau=0.0, sigma_to_r=3.0, kernel=0, tri=True, u=False, m=None, stream=None):
    """One P-NDF sample per query.  xi: (attempts, Q, 2) float64 device tensor of
    uniforms in [0, 1).  Returns (m (Q, 2) float32, tri (Q,) int64 or None,
    u (Q, 2) float64 or None)."""
    qp, nq = _queries(queries)
    if xi.dim() != 3 or xi.shape[1] != nq or xi.shape[2] != 2:
        raise ValueError("xi must have shape (attempts, Q, 2)")
    dev = queries.device
    if m is None:
        m = torch.empty((nq, 2), dtype=torch.float32, device=dev)
    t = torch.empty(nq, dtype=torch.int64, device=dev) if tri else None
    uu = torch.empty((nq, 2), dtype=torch.float64, device=dev) if u else None
    o = _opts(tau, sigma_to_r, "auto", kernel)
    _check(_sample_batch(hier.handle, qp, nq, _dev_ptr(xi, torch.float64, "xi"), int(xi.shape[0]), ctypes.byref(o),
                         _dev_ptr(m, torch.float32, "m"), _vp(t.data_ptr()) if tri else None,
                         _vp(uu.data_ptr()) if u else None, _stream(stream)), "pndf_sample_batch")
    return m, t, uu


def projected_area(hier, queries, sigma_to_r=3.0, kernel=0, lam=False, stream=None):
    """P(w) per query (Q, 6): x, y, sx, sy, w_x, w_y.  Returns P (Q,) float32, and
    Lambda(w) = P / w_z - 1 too if lam."""
    qp, nq = _queries(queries)
    P = torch.empty(nq, dtype=torch.float32, device=queries.device)
    L = torch.empty(nq, dtype=torch.float32, device=queries.device) if lam else None
    o = _opts(0.0, sigma_to_r, "auto", kernel)
    _check(_projected_area(hier.handle, qp, nq, ctypes.byref(o), _dev_ptr(P, torch.float32, "P"),
                           _vp(L.data_ptr()) if lam else None, _stream(stream)), "pndf_projected_area")
    return (P, L) if lam else P


def eval_counts(hier, queries, tau=0.0, sigma_to_r=3.0, algo="auto", stream=None, kernel=0):
    """Returns (D, counts (Q, 4) int32: nodes, cells, clusters, hits)."""
    qp, nq = _queries(queries)
    out = torch.empty(nq, dtype=torch.float32, device=queries.device)
    counts = torch.zeros((nq, 4), dtype=torch.int32, device=queries.device)
    o = _opts(tau, sigma_to_r, algo, kernel)
    _check(_eval_counts(hier.handle, qp, nq, ctypes.byref(o), _dev_ptr(out, torch.float32, "out"),
                        _dev_ptr(counts, torch.int32, "counts"), _stream(stream)), "pndf_eval_counts")
    return out, counts


def eval_hits(hier, queries, tau=0.0, sigma_to_r=3.0, algo="auto", capacity=None, stream=None, kernel=0):
    """Returns (D, offsets (Q+1,) int64, ids (H,) int64, terms (H,) float32)."""
    qp, nq = _queries(queries)
    dev = queries.device
    out = torch.empty(nq, dtype=torch.float32, device=dev)
    offs = torch.zeros(nq + 1, dtype=torch.int64, device=dev)
    o = _opts(tau, sigma_to_r, algo, kernel)
    req = _u64(0)
    cap = 0 if capacity is None else int(capacity)
    ids = torch.empty(max(cap, 1), dtype=torch.int64, device=dev)
    terms = torch.empty(max(cap, 1), dtype=torch.float32, device=dev)
    st = _eval_hits(hier.handle, qp, nq, ctypes.byref(o), _dev_ptr(out, torch.float32, "out"),
                    _dev_ptr(offs, torch.int64, "offsets"), _vp(ids.data_ptr()), _vp(terms.data_ptr()),
                    cap, ctypes.byref(req), _stream(stream))
    if st == PNDF_EOVERFLOW and capacity is None:
        cap = int(req.value)
        ids = torch.empty(max(cap, 1), dtype=torch.int64, device=dev)
        terms = torch.empty(max(cap, 1), dtype=torch.float32, device=dev)
        st = _eval_hits(hier.handle, qp, nq, ctypes.byref(o), _dev_ptr(out, torch.float32, "out"),
                        _dev_ptr(offs, torch.int64, "offsets"), _vp(ids.data_ptr()), _vp(terms.data_ptr()),
                        cap, ctypes.byref(req), _stream(stream))
    _check(st, "pndf_eval_hits")
    total = int(req.value)
    return out, offs, ids[:total], terms[:total]


def mesh_info(mesh):
    n, eps, b = _i32(), _f32(), _i64()
    _check(_mesh_info(mesh.handle, ctypes.byref(n), ctypes.byref(eps), ctypes.byref(b)), "pndf_mesh_info")
    return dict(n=n.value, eps=eps.value, bytes=b.value)


def mesh_export(mesh, stream=None):
    n = mesh.n
    deg = torch.empty((n, n), dtype=torch.uint8, device="cuda")
    det = torch.empty((n, n, 2), dtype=torch.float32, device="cuda")
    _check(_mesh_export(mesh.handle, _vp(deg.data_ptr()), _vp(det.data_ptr()), _stream(stream)),
           "pndf_mesh_export")
    return deg, det


def hier_info(hier):
    lv, cl, b = _i32(), _i32(), _i64()
    _check(_hier_info(hier.handle, ctypes.byref(lv), ctypes.byref(cl), ctypes.byref(b)), "pndf_hier_info")
    return dict(levels=lv.value, cluster=bool(cl.value), bytes=b.value)


def hier_export_level(hier, level, stream=None):
    m = hier.n >> level
    bbox = torch.empty((m, m, 4), dtype=torch.float32, device="cuda")
    if hier.cluster:
        bbox_all = torch.empty((m, m, 4), dtype=torch.float32, device="cuda")
        bbox_clu = torch.empty((m, m, 4), dtype=torch.float32, device="cuda")
        clu_n = torch.empty((m, m, 4, 2), dtype=torch.float32, device="cuda")
        clu_e = torch.empty((m, m), dtype=torch.float32, device="cuda")
        clu_det = torch.empty((m, m, 2), dtype=torch.float32, device="cuda")
        ptrs = [_vp(t.data_ptr()) for t in (bbox_all, bbox_clu, clu_n, clu_e, clu_det)]
    else:
        bbox_all = bbox_clu = clu_n = clu_e = clu_det = None
        ptrs = [None] * 5
    _check(_hier_export(hier.handle, int(level), _vp(bbox.data_ptr()), *ptrs, _stream(stream)),
           "pndf_hier_export_level")
    return dict(bbox=bbox, bbox_all=bbox_all, bbox_clu=bbox_clu, clu_n=clu_n, clu_e=clu_e, clu_det=clu_det)


class Plan:
    """Persistent work-stealing evaluation plan (workspace + instantiated HIP graph)."""

    def __init__(self, hier, max_nq, tau=0.0, sigma_to_r=3.0, tuning=None, stream=None, input_order=False,
                 kernel=0):
        self.hier = hier  # the hierarchy must outlive the plan
        self.max_nq = int(max_nq)
        o = _opts(tau, sigma_to_r, "persistent", kernel, flags=EVAL_INPUT_ORDER if input_order else 0)
        t = None
        if tuning is not None:
            t = tuning if isinstance(tuning, Tuning) else Tuning(**tuning)
        h = _vp()
        _check(_plan_create(hier.handle, self.max_nq, ctypes.byref(o), ctypes.byref(t) if t is not None else None,
                            _stream(stream), ctypes.byref(h)), "pndf_plan_create")
        self._h = h

    def eval(self, queries, out=None, stream=None):
        qp, nq = _queries(queries)
        if out is None:
            out = torch.empty(nq, dtype=torch.float32, device=queries.device)
        _check(_plan_eval(self._h, qp, nq, _dev_ptr(out, torch.float32, "out"), _stream(stream)),
               "pndf_plan_eval")
        return out

    def tuning(self):
        t = Tuning()
        _check(_plan_get_tuning(self._h, ctypes.byref(t)), "pndf_plan_get_tuning")
        return t.as_dict()

    def stats(self, stream=None):
        st = PlanStats()
        _check(_plan_get_stats(self._h, ctypes.byref(st), _stream(stream)), "pndf_plan_get_stats")
        return dict(spawned=int(st.spawned), refused=int(st.refused), idle_spins=int(st.idle_spins),
                    error=int(st.error))

    def close(self):
        if getattr(self, "_h", None):
            _plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def default_tuning(hier):
    t = Tuning()
    _check(_default_tuning(hier.handle, ctypes.byref(t)), "pndf_default_tuning")
    return t.as_dict()


def autotune(hier, queries, tau=0.0, sigma_to_r=3.0, stream=None, kernel=0):
    """Returns (best tuning dict, ms per batch of `queries`)."""
    qp, nq = _queries(queries)
    o = _opts(tau, sigma_to_r, "persistent", kernel)
    t = Tuning()
    ms = ctypes.c_double(0)
    _check(_autotune(hier.handle, qp, nq, ctypes.byref(o), ctypes.byref(t), ctypes.byref(ms), _stream(stream)),
           "pndf_autotune")
    return t.as_dict(), float(ms.value)


class ServerOpts(ctypes.Structure):
    _fields_ = [("slots", _i32), ("max_batch_queries", _i64), ("memory_budget", _i64), ("max_pending", _i32),
                ("tau", _f32), ("sigma_to_r", _f32), ("tuning", Tuning), ("algo", _i32), ("kernel", _i32),
                ("chunk_queries", _i64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("completed", _u64), ("refused", _u64), ("queries", _u64), ("batches", _u64),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("max_ms", ctypes.c_double),
                ("mean_batch_requests", ctypes.c_double), ("busy_s", ctypes.c_double)]

    def as_dict(self):
        return {k: (float(getattr(self, k)) if t is ctypes.c_double else int(getattr(self, k)))
                for k, t in self._fields_}


_server_create = _sig("pndf_server_create", _i32, [ctypes.POINTER(_vp), _i32, ctypes.POINTER(ServerOpts),
                                                   ctypes.POINTER(_vp)])
_server_submit = _sig("pndf_server_submit", _i32, [_vp, _i32, _vp, _i64, _vp, ctypes.POINTER(_u64)])
_server_wait = _sig("pndf_server_wait", _i32, [_vp, _u64, ctypes.c_double, ctypes.POINTER(ctypes.c_double)])
_server_drain = _sig("pndf_server_drain", _i32, [_vp])
_server_get_stats = _sig("pndf_server_get_stats", _i32, [_vp, ctypes.POINTER(ServerStats)])
_server_reset_stats = _sig("pndf_server_reset_stats", _i32, [_vp])
_server_replay = _sig("pndf_server_replay", _i32, [_vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp])
_server_destroy = _sig("pndf_server_destroy", None, [_vp])
EXPORTED += ["pndf_server_create", "pndf_server_submit", "pndf_server_wait", "pndf_server_drain",
             "pndf_server_get_stats", "pndf_server_reset_stats", "pndf_server_replay", "pndf_server_destroy"]


class Server:
    """Continuous-batching server over resident hierarchies (host-side requests)."""

    def __init__(self, hiers, slots=2, max_batch_queries=1 << 16, memory_budget=None, max_pending=256,
                 tau=0.0, sigma_to_r=3.0, tuning=None, algo="plain", kernel=0, chunk_queries=0):
        import numpy as np
        self._np = np
        self.hiers = list(hiers)  # keep the hierarchies alive
        if memory_budget is None:
            memory_budget = 28 * max_batch_queries * max(4, 2 * slots) + 4096
        t = Tuning(0, 1, 16, 1) if tuning is None else (tuning if isinstance(tuning, Tuning) else Tuning(**tuning))
        o = ServerOpts(int(slots), int(max_batch_queries), int(memory_budget), int(max_pending), float(tau),
                       float(sigma_to_r), t, ALGOS[algo] if isinstance(algo, str) else int(algo),
                       KERNELS[kernel] if isinstance(kernel, str) else int(kernel), int(chunk_queries))
        arr = (_vp * len(self.hiers))(*[h.handle for h in self.hiers])
        h = _vp()
        _check(_server_create(arr, len(self.hiers), ctypes.byref(o), ctypes.byref(h)), "pndf_server_create")
        self._h = h
        self._keep = {}

    def submit(self, map_id, queries, out=None):
        """queries: (Q, 6) float32 numpy array.  Returns (ticket, out array) or raises PndfError
        (status PNDF_EAGAIN when not admitted)."""
        np = self._np
        q = np.ascontiguousarray(queries, dtype=np.float32)
        if out is None:
            out = np.empty(q.shape[0], dtype=np.float32)
        t = _u64(0)
        _check(_server_submit(self._h, int(map_id), q.ctypes.data_as(_vp), q.shape[0], out.ctypes.data_as(_vp),
                              ctypes.byref(t)), "pndf_server_submit")
        self._keep[int(t.value)] = (q, out)
        return int(t.value), out

    def wait(self, ticket, timeout=-1.0):
        ms = ctypes.c_double(0)
        _check(_server_wait(self._h, int(ticket), float(timeout), ctypes.byref(ms)), "pndf_server_wait")
        self._keep.pop(int(ticket), None)
        return float(ms.value)

    def drain(self):
        _check(_server_drain(self._h), "pndf_server_drain")

    def stats(self):
        st = ServerStats()
        _check(_server_get_stats(self._h, ctypes.byref(st)), "pndf_server_get_stats")
        return st.as_dict()

    def reset_stats(self):
        _check(_server_reset_stats(self._h), "pndf_server_reset_stats")

    def replay(self, map_ids, arrivals, queries):
        """Replay an arrival trace; returns (list of result arrays, latencies in ms)."""
        np = self._np
        n = len(queries)
        qs = [np.ascontiguousarray(q, dtype=np.float32) for q in queries]
        outs = [np.empty(q.shape[0], dtype=np.float32) for q in qs]
        mids = np.ascontiguousarray(map_ids, dtype=np.int32)
        arr = np.ascontiguousarray(arrivals, dtype=np.float64)
        qp = (_vp * n)(*[q.ctypes.data for q in qs])
        op = (_vp * n)(*[o.ctypes.data for o in outs])
        nq = np.ascontiguousarray([q.shape[0] for q in qs], dtype=np.int64)
        lat = np.zeros(n, dtype=np.float64)
        _check(_server_replay(self._h, n, mids.ctypes.data_as(_vp), arr.ctypes.data_as(_vp), ctypes.cast(qp, _vp),
                              nq.ctypes.data_as(_vp), ctypes.cast(op, _vp), lat.ctypes.data_as(_vp)),
               "pndf_server_replay")
        return outs, lat

    def close(self):
        if getattr(self, "_h", None):
            _server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
