// Host side of the C ABI declared in include/pndf.h: argument validation, handle
// ownership, device allocation and kernel dispatch.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "pndf_internal.h"

namespace pndf {

static thread_local std::string g_last_error;

// Batches from this size on are evaluated in spatial order (results do not depend on
// the order; only cache locality does).  A random batch of 16384 queries runs 7 %
// faster without the order passes, but render tiles served side by side need the
// order's locality: with 32768 as the threshold a served stream of 16384-query tiles
// lost a quarter of its throughput, though each tile alone ran faster.
constexpr int64_t kOrderMin = 4096;

void set_error(const std::string& msg) { g_last_error = msg; }

int64_t launch_chunk()
{
    const char* v = std::getenv("PNDF_LAUNCH_CHUNK");
    if (v) {
        const long long c = std::atoll(v);
        if (c > 0 && c < kLaunchChunk) return (int64_t)c;
    }
    return kLaunchChunk;
}

pndf_status hip_fail(hipError_t e, const char* what)
{
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? PNDF_ENOMEM : PNDF_EDEVICE;
}

static pndf_status invalid(const std::string& msg)
{
    set_error(msg);
    return PNDF_EINVAL;
}

// Surface an earlier asynchronous fault before starting new work.
static pndf_status check_sticky()
{
    hipError_t e = hipPeekAtLastError();
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return hip_fail(e, "earlier device error");
    }
    return PNDF_OK;
}

static int ilog2_exact(int n)
{
    int l = 0;
    while (l < 31 && (1 << l) < n) ++l;
    return (1 << l) == n ? l : -1;
}

static void fill_view(pndf_hier* h)
{
    HierDev& d = h->dev;
    const pndf_mesh* m = h->mesh;
    d.nrm = m->nrm;
    d.deg = m->deg;
    d.det = m->det;
    d.bbox = h->bbox;
    d.bbox_all = h->bbox_all;
    d.clu_t = h->clu_t;
    d.clu_e = h->clu_e;
    d.clu_det = h->clu_det;
    d.bbox_c = h->bbox_c;
    d.bbox_u = h->bbox_u;
    d.grp = h->grp;
    d.bbox_k = h->bbox_k;
    d.quad = h->quad;
    d.n = m->n;
    d.L = m->L;
    d.logn = m->L;
    d.eps = m->eps;
    d.rho = (float)std::sqrt(2.0 * (double)m->eps / (3.0 * std::sqrt(3.0)));
}

static void mesh_release(pndf_mesh* m)
{
    if (!m) return;
    if (m->refs.fetch_sub(1) == 1) {
        (void)hipFree(m->nrm);
        (void)hipFree(m->deg);
        (void)hipFree(m->det);
        delete m;
    }
}

static pndf_status resolve_opts(const pndf_hier* h, const pndf_eval_opts* o, pndf_eval_opts* out)
{
    pndf_eval_opts d;
    d.kernel = PNDF_KERNEL_GAUSSIAN;
    d.tau = 0.f;
    d.sigma_to_r = 3.f;
    d.algo = PNDF_ALGO_AUTO;
    d.flags = 0;
    if (o) d = *o;
    if (d.kernel != PNDF_KERNEL_GAUSSIAN && d.kernel != PNDF_KERNEL_DISK && d.kernel != PNDF_KERNEL_BOX)
        return invalid("unknown footprint kernel");
    if (!(std::isfinite(d.tau) && d.tau >= 0.f)) return invalid("tau must be finite and >= 0");
    if (!(std::isfinite(d.sigma_to_r) && d.sigma_to_r > 0.f))
        return invalid("sigma_to_r must be finite and > 0");
    if (d.flags & ~PNDF_EVAL_INPUT_ORDER) return invalid("unknown flags");
    if (d.algo < PNDF_ALGO_AUTO || d.algo > PNDF_ALGO_PERSISTENT) return invalid("unknown algo");
    if (d.algo == PNDF_ALGO_PERSISTENT) {
        set_error("the persistent traversal runs through a plan (pndf_plan_create, pndf_plan_eval)");
        return PNDF_EUNSUPPORTED;
    }
    if (d.tau > 0.f && !h->cluster) return invalid("tau > 0 needs a hierarchy built with clusters");
    if (d.tau > 0.f && d.algo == PNDF_ALGO_BRUTE) return invalid("brute force evaluates tau = 0 only");
    *out = d;
    return PNDF_OK;
}

}  // namespace pndf

using namespace pndf;

extern "C" {

const char* pndf_status_string(pndf_status s)
{
    switch (s) {
    case PNDF_OK: return "ok";
    case PNDF_EINVAL: return "invalid argument";
    case PNDF_ENOMEM: return "out of memory";
    case PNDF_EDEVICE: return "device error";
    case PNDF_EOVERFLOW: return "buffer too small";
    case PNDF_EUNSUPPORTED: return "unsupported";
    case PNDF_EAGAIN: return "try again";
    }
    return "unknown status";
}

const char* pndf_last_error(void) { return g_last_error.c_str(); }

pndf_status pndf_build_mesh(const float* normals, int32_t n, float eps, void* stream,
                            pndf_mesh** out)
{
    if (!out) return invalid("out is NULL");
    *out = nullptr;
    if (!normals) return invalid("normals is NULL");
    const int L = ilog2_exact(n);
    if (n < 2 || L < 0) return invalid("map side must be a power of two >= 2");
    if (n > 8192) {
        set_error("map side above 8192");
        return PNDF_EUNSUPPORTED;
    }
    if (!(std::isfinite(eps) && eps > 0.f)) return invalid("eps must be finite and > 0");
    pndf_status st = check_sticky();
    if (st != PNDF_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    pndf_mesh* m = new (std::nothrow) pndf_mesh;
    if (!m) return PNDF_ENOMEM;
    m->n = n;
    m->L = L;
    m->eps = eps;
    (void)hipGetDevice(&m->device);
    const size_t np = (size_t)(n + 1) * (n + 1), nc = (size_t)n * n;
    unsigned* d_flag = nullptr;
    hipError_t e = hipMalloc(&m->nrm, sizeof(float2) * np);
    if (e == hipSuccess) e = hipMalloc(&m->deg, nc);
    if (e == hipSuccess) e = hipMalloc(&m->det, sizeof(float2) * nc);
    if (e == hipSuccess) e = hipMalloc(&d_flag, sizeof(unsigned));
    if (e == hipSuccess) e = hipMemsetAsync(d_flag, 0, sizeof(unsigned), s);
    if (e == hipSuccess) e = launch_build_mesh(normals, n, eps, m->nrm, m->deg, m->det, d_flag, s);
    unsigned flag = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&flag, d_flag, sizeof(unsigned), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(d_flag);
    if (e != hipSuccess) {
        mesh_release(m);
        return hip_fail(e, "pndf_build_mesh");
    }
    if (flag) {
        mesh_release(m);
        return invalid("normal map has a non-finite value or |n| >= 1");
    }
    m->bytes = (int64_t)(sizeof(float2) * np + nc + sizeof(float2) * nc);
    *out = m;
    return PNDF_OK;
}

void pndf_destroy_mesh(pndf_mesh* mesh) { mesh_release(mesh); }

pndf_status pndf_mesh_info(const pndf_mesh* mesh, int32_t* n, float* eps, int64_t* bytes)
{
    if (!mesh) return invalid("mesh is NULL");
    if (n) *n = mesh->n;
    if (eps) *eps = mesh->eps;
    if (bytes) *bytes = mesh->bytes;
    return PNDF_OK;
}

pndf_status pndf_mesh_export(const pndf_mesh* mesh, uint8_t* d_deg, float* d_det, void* stream)
{
    if (!mesh) return invalid("mesh is NULL");
    hipStream_t s = (hipStream_t)stream;
    const size_t nc = (size_t)mesh->n * mesh->n;
    hipError_t e = hipSuccess;
    if (d_deg) e = hipMemcpyAsync(d_deg, mesh->deg, nc, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && d_det)
        e = hipMemcpyAsync(d_det, mesh->det, sizeof(float2) * nc, hipMemcpyDeviceToDevice, s);
    return e == hipSuccess ? PNDF_OK : hip_fail(e, "pndf_mesh_export");
}

pndf_status pndf_build_hierarchy(const pndf_mesh* mesh, const pndf_hier_opts* opts, void* stream,
                                 pndf_hier** out)
{
    if (!out) return invalid("out is NULL");
    *out = nullptr;
    if (!mesh) return invalid("mesh is NULL");
    const int cluster = opts ? opts->cluster : 1;
    if (cluster != 0 && cluster != 1) return invalid("cluster must be 0 or 1");
    pndf_status st = check_sticky();
    if (st != PNDF_OK) return st;
    pndf_hier* h = new (std::nothrow) pndf_hier;
    if (!h) return PNDF_ENOMEM;
    pndf_mesh* m = const_cast<pndf_mesh*>(mesh);
    m->refs.fetch_add(1);
    h->mesh = m;
    h->cluster = cluster;
    h->L = m->L;
    int64_t nodes = 0;
    for (int l = 1; l <= m->L; ++l) nodes += (int64_t)(m->n >> l) * (m->n >> l);
    h->nodes = nodes;
    hipError_t e = hipMalloc(&h->bbox, sizeof(float4) * nodes);
    if (e == hipSuccess) e = hipMalloc(&h->bbox_k, sizeof(uint2) * nodes);
    if (e == hipSuccess) e = hipMalloc(&h->quad, sizeof(QuadRec) * (size_t)(m->n >> 1) * (size_t)(m->n >> 1));
    if (cluster) {
        if (e == hipSuccess) e = hipMalloc(&h->bbox_all, sizeof(float4) * nodes);
        if (e == hipSuccess) e = hipMalloc(&h->clu_n, sizeof(float4) * 2 * nodes);
        if (e == hipSuccess) e = hipMalloc(&h->clu_e, sizeof(float) * nodes);
        if (e == hipSuccess) e = hipMalloc(&h->clu_det, sizeof(float2) * nodes);
        if (e == hipSuccess) e = hipMalloc(&h->clu_t, sizeof(float4) * 2 * nodes);
        if (e == hipSuccess) e = hipMalloc(&h->bbox_clu, sizeof(float4) * nodes);
        if (e == hipSuccess) e = hipMalloc(&h->bbox_c, sizeof(uint2) * nodes);
        if (e == hipSuccess) e = hipMalloc(&h->bbox_u, sizeof(uint2) * nodes);
        // whole groups of four (the top level's single node fills one)
        if (e == hipSuccess) e = hipMalloc(&h->grp, sizeof(uint4) * ((nodes + 3) & ~(int64_t)3));
    }
    fill_view(h);
    if (e == hipSuccess) e = build_hierarchy_levels(h, (hipStream_t)stream);
    if (e != hipSuccess) {
        pndf_destroy_hierarchy(h);
        return hip_fail(e, "pndf_build_hierarchy");
    }
    // per node: bbox 16, bbox_k 8; with clusters bbox_all 16, bbox_clu 16, bbox_c 8, bbox_u 8,
    // grp 16, clu_n 32, clu_t 32, clu_e 4, clu_det 8; plus the level-1 leaf records
    h->bytes = (int64_t)nodes * (16 + 8 + (cluster ? 16 + 16 + 8 + 8 + 16 + 32 + 32 + 4 + 8 : 0)) +
               (int64_t)sizeof(QuadRec) * (m->n >> 1) * (m->n >> 1);
    *out = h;
    return PNDF_OK;
}

void pndf_destroy_hierarchy(pndf_hier* h)
{
    if (!h) return;
    (void)hipFree(h->bbox);
    (void)hipFree(h->quad);
    (void)hipFree(h->bbox_all);
    (void)hipFree(h->clu_n);
    (void)hipFree(h->clu_e);
    (void)hipFree(h->clu_det);
    (void)hipFree(h->clu_t);
    (void)hipFree(h->bbox_clu);
    (void)hipFree(h->bbox_c);
    (void)hipFree(h->bbox_u);
    (void)hipFree(h->grp);
    (void)hipFree(h->bbox_k);
    mesh_release(h->mesh);
    delete h;
}

pndf_status pndf_hier_info(const pndf_hier* h, int32_t* levels, int32_t* cluster, int64_t* bytes)
{
    if (!h) return invalid("hierarchy is NULL");
    if (levels) *levels = h->L;
    if (cluster) *cluster = h->cluster;
    if (bytes) *bytes = h->bytes;
    return PNDF_OK;
}

pndf_status pndf_hier_export_level(const pndf_hier* h, int32_t level, float* d_bbox,
                                   float* d_bbox_all, float* d_bbox_clu, float* d_clu_n, float* d_clu_e,
                                   float* d_clu_det, void* stream)
{
    if (!h) return invalid("hierarchy is NULL");
    if (level < 1 || level > h->L) return invalid("level out of range");
    if (!h->cluster && (d_bbox_all || d_bbox_clu || d_clu_n || d_clu_e || d_clu_det))
        return invalid("hierarchy has no clusters");
    hipStream_t s = (hipStream_t)stream;
    const int64_t off = level_offset(h->dev.logn, level);
    const size_t m = (size_t)(h->mesh->n >> level) * (h->mesh->n >> level);
    hipError_t e = hipSuccess;
    const int side = h->mesh->n >> level;
    (void)m;
    auto cp = [&](void* dst, const void* src, int words) {
        if (dst && e == hipSuccess) e = export_rowmajor(src, dst, side, words, s);
    };
    cp(d_bbox, h->bbox + off, 4);
    if (h->cluster) {
        cp(d_bbox_all, h->bbox_all + off, 4);
        cp(d_bbox_clu, h->bbox_clu + off, 4);
        cp(d_clu_n, h->clu_n + 2 * off, 8);
        cp(d_clu_e, h->clu_e + off, 1);
        cp(d_clu_det, h->clu_det + off, 2);
    }
    return e == hipSuccess ? PNDF_OK : hip_fail(e, "pndf_hier_export_level");
}

static pndf_status eval_common(const pndf_hier* h, const pndf_query* d_q, int64_t nq,
                               const pndf_eval_opts* opts, float* d_out, pndf_eval_opts* o)
{
    if (!h) return invalid("hierarchy is NULL");
    if (nq < 0) return invalid("nq < 0");
    if (nq > 0 && (!d_q || !d_out)) return invalid("query or output pointer is NULL");
    if (nq > (int64_t)UINT32_MAX) return invalid("nq above 2^32 - 1 (the spatial order holds 32-bit indices)");
    pndf_status st = resolve_opts(h, opts, o);
    if (st != PNDF_OK) return st;
    return check_sticky();
}

pndf_status pndf_sample_batch(const pndf_hier* h, const pndf_query* d_q, int64_t nq, const double* d_xi,
                              int32_t attempts, const pndf_eval_opts* opts, float* d_m, uint64_t* d_tri,
                              double* d_u, void* stream)
{
    if (!h) return invalid("hierarchy is NULL");
    if (nq < 0) return invalid("nq < 0");
    if (nq > (int64_t)UINT32_MAX) return invalid("nq above 2^32 - 1");
    if (attempts < 1 || attempts > 64) return invalid("attempts must be in [1, 64]");
    if (nq > 0 && (!d_q || !d_xi || !d_m)) return invalid("query, uniform or output pointer is NULL");
    // (the kernel reads the uniforms as pairs of doubles and writes m, u as pairs)
    if (((uintptr_t)d_xi & 15u) || ((uintptr_t)d_m & 7u) || ((uintptr_t)d_u & 15u) || ((uintptr_t)d_tri & 7u) ||
        ((uintptr_t)d_q & 3u))
        return invalid("misaligned pointer (uniforms and u: 16 B, m and tri: 8 B, queries: 4 B)");
    pndf_eval_opts o{PNDF_KERNEL_GAUSSIAN, 0.f, 3.f, PNDF_ALGO_AUTO, 0};
    if (opts) {
        o = *opts;
        o.algo = PNDF_ALGO_AUTO;  // ignored
    }
    if (o.flags != 0) return invalid("sampling takes no flags");
    pndf_eval_opts r;
    pndf_status st = resolve_opts(h, &o, &r);
    if (st != PNDF_OK) return st;
    st = check_sticky();
    if (st != PNDF_OK) return st;
    SampleArgs a{d_q, d_xi, nq, 0, nq, attempts, r.tau, r.sigma_to_r, r.kernel, reinterpret_cast<float2*>(d_m),
                 d_tri, reinterpret_cast<double2*>(d_u)};
    const hipError_t e = launch_sample(h->dev, a, (hipStream_t)stream);
    return e == hipSuccess ? PNDF_OK : hip_fail(e, "pndf_sample_batch");
}

pndf_status pndf_projected_area(const pndf_hier* h, const pndf_query* d_q, int64_t nq, const pndf_eval_opts* opts,
                                float* d_P, float* d_lambda, void* stream)
{
    if (!h) return invalid("hierarchy is NULL");
    if (nq < 0) return invalid("nq < 0");
    if (nq > (int64_t)UINT32_MAX) return invalid("nq above 2^32 - 1");
    if (nq > 0 && (!d_q || !d_P)) return invalid("query or output pointer is NULL");
    pndf_eval_opts o{PNDF_KERNEL_GAUSSIAN, 0.f, 3.f, PNDF_ALGO_AUTO, 0};
    if (opts) {
        o = *opts;
        o.algo = PNDF_ALGO_AUTO;  // ignored
    }
    if (o.flags != 0) return invalid("the projected area takes no flags");
    if (o.tau != 0.f) return invalid("the projected area is brute force: tau must be 0");
    pndf_eval_opts r;
    pndf_status st = resolve_opts(h, &o, &r);
    if (st != PNDF_OK) return st;
    st = check_sticky();
    if (st != PNDF_OK) return st;
    ProjArgs a{d_q, nq, r.sigma_to_r, r.kernel, d_P, d_lambda, nullptr};
    const hipError_t e = launch_projected_area(h->dev, a, (hipStream_t)stream);
    return e == hipSuccess ? PNDF_OK : hip_fail(e, "pndf_projected_area");
}

pndf_status pndf_eval_batch(const pndf_hier* h, const pndf_query* d_q, int64_t nq,
                            const pndf_eval_opts* opts, float* d_out, void* stream)
{
    pndf_eval_opts o;
    pndf_status st = eval_common(h, d_q, nq, opts, d_out, &o);
    if (st != PNDF_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    uint32_t* order = nullptr;
    hipError_t e = hipSuccess;
    if (nq >= kOrderMin && o.algo != PNDF_ALGO_BRUTE && !(o.flags & PNDF_EVAL_INPUT_ORDER))
        e = make_order(h->dev, d_q, nq, &order, s);
    EvalArgs a{d_q, order, nq, 0, 0, d_out, nullptr, nullptr, nullptr, nullptr, o.tau, o.sigma_to_r, o.kernel};
    if (e == hipSuccess) e = launch_eval(h->dev, a, o.algo, s);
    free_order(order, s);
    return e == hipSuccess ? PNDF_OK : hip_fail(e, "pndf_eval_batch");
}

pndf_status pndf_eval_batch_noalloc(const pndf_hier* h, const pndf_query* d_q, int64_t nq,
                                    const pndf_eval_opts* opts, float* d_out, void* stream)
{
    pndf_eval_opts o;
    pndf_status st = eval_common(h, d_q, nq, opts, d_out, &o);
    if (st != PNDF_OK) return st;
    if (nq > kStaticOrderQueries) return invalid("nq above 2^22, the no-allocation workspace's limit");
    hipStream_t s = (hipStream_t)stream;
    uint32_t* order = nullptr;
    hipError_t e = hipSuccess;
    if (nq >= kOrderMin && o.algo != PNDF_ALGO_BRUTE && !(o.flags & PNDF_EVAL_INPUT_ORDER))
        e = make_order_static(h->dev, d_q, nq, &order, s);
    EvalArgs a{d_q, order, nq, 0, 0, d_out, nullptr, nullptr, nullptr, nullptr, o.tau, o.sigma_to_r, o.kernel};
    if (e == hipSuccess) e = launch_eval(h->dev, a, o.algo, s);
    return e == hipSuccess ? PNDF_OK : hip_fail(e, "pndf_eval_batch_noalloc");
}

pndf_status pndf_eval_counts(const pndf_hier* h, const pndf_query* d_q, int64_t nq,
                             const pndf_eval_opts* opts, float* d_out, uint32_t* d_counts,
                             void* stream)
{
    pndf_eval_opts o;
    pndf_status st = eval_common(h, d_q, nq, opts, d_out, &o);
    if (st != PNDF_OK) return st;
    if (nq > 0 && !d_counts) return invalid("counts pointer is NULL");
    EvalArgs a{d_q, nullptr, nq, 0, 0, d_out, d_counts, nullptr, nullptr, nullptr, o.tau, o.sigma_to_r, o.kernel};
    hipError_t e = launch_eval(h->dev, a, o.algo, (hipStream_t)stream);
    return e == hipSuccess ? PNDF_OK : hip_fail(e, "pndf_eval_counts");
}

pndf_status pndf_eval_hits(const pndf_hier* h, const pndf_query* d_q, int64_t nq,
                           const pndf_eval_opts* opts, float* d_out, uint64_t* d_offsets,
                           uint64_t* d_ids, float* d_terms, uint64_t capacity,
                           uint64_t* required, void* stream)
{
    pndf_eval_opts o;
    pndf_status st = eval_common(h, d_q, nq, opts, d_out, &o);
    if (st != PNDF_OK) return st;
    if (!required) return invalid("required is NULL");
    if (nq > 0 && !d_offsets) return invalid("offsets pointer is NULL");
    if (capacity > 0 && (!d_ids || !d_terms)) return invalid("id or term pointer is NULL");
    *required = 0;
    hipStream_t s = (hipStream_t)stream;
    if (nq == 0) return PNDF_OK;
    uint32_t* d_counts = nullptr;
    hipError_t e = hipMalloc(&d_counts, sizeof(uint32_t) * 4 * (size_t)nq);
    if (e != hipSuccess) return hip_fail(e, "pndf_eval_hits");
    EvalArgs a{d_q, nullptr, nq, 0, 0, d_out, d_counts, nullptr, nullptr, nullptr, o.tau, o.sigma_to_r, o.kernel};
    e = launch_eval(h->dev, a, o.algo, s);
    std::vector<uint32_t> counts((size_t)nq * 4);
    if (e == hipSuccess)
        e = hipMemcpyAsync(counts.data(), d_counts, sizeof(uint32_t) * 4 * nq, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    std::vector<uint64_t> offs((size_t)nq + 1, 0);
    for (int64_t k = 0; k < nq; ++k) offs[k + 1] = offs[k] + counts[4 * k + 3];
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_offsets, offs.data(), sizeof(uint64_t) * (nq + 1), hipMemcpyHostToDevice, s);
    *required = offs[nq];
    if (e == hipSuccess && offs[nq] <= capacity && offs[nq] > 0) {
        EvalArgs b{d_q, nullptr, nq, 0, 0, d_out, nullptr, d_offsets, d_ids, d_terms, o.tau, o.sigma_to_r, o.kernel};
        e = launch_eval(h->dev, b, o.algo, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(d_counts);
    if (e != hipSuccess) return hip_fail(e, "pndf_eval_hits");
    if (offs[nq] > capacity) {
        set_error("hit buffer too small");
        return PNDF_EOVERFLOW;
    }
    return PNDF_OK;
}

}  // extern "C"
