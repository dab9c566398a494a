// Host side of the persistent work-stealing evaluation: plans (workspace and
// instantiated launch graph) and the autotuner that picks their shape.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "pndf_internal.h"

struct pndf_plan {
    const pndf_hier* h = nullptr;
    pndf_tuning tuning{};
    pndf_eval_opts opts{};
    pndf::PersistPlan P;
};

namespace pndf {

static pndf_status plan_invalid(const char* msg)
{
    set_error(msg);
    return PNDF_EINVAL;
}

static int compute_units()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        return 256;
    return cus;
}

// Ticks of the device's constant-rate clock in `seconds` (100 MHz if unknown).
static long long wall_ticks(double seconds)
{
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
        khz = 100000;
    return (long long)(seconds * 1e3 * (double)khz);
}

static void plan_free(pndf_plan* p)
{
    if (!p) return;
    PersistPlan& P = p->P;
    if (P.exec) (void)hipGraphExecDestroy(P.exec);
    if (P.graph) (void)hipGraphDestroy(P.graph);
    (void)hipFree(P.ctl);
    (void)hipFree(P.acc);
    (void)hipFree(P.fexp);
    (void)hipFree(P.tasks);
    (void)hipFree(P.flags);
    (void)hipFree(P.order);
    delete p;
}

}  // namespace pndf

using namespace pndf;

extern "C" {

pndf_status pndf_default_tuning(const pndf_hier* h, pndf_tuning* out)
{
    if (!h || !out) return plan_invalid("NULL argument");
    // as many worker blocks as fit on a compute unit (reduced to the resident count
    // when the plan is made), nodes three levels below the root donatable: the best
    // measured setting on the scratched and power-law maps
    out->blocks_per_cu = 8;
    out->split_level = std::max(1, h->L - 3);
    out->queue_factor = 16;
    out->use_graph = 1;
    return PNDF_OK;
}

pndf_status pndf_plan_create(const pndf_hier* h, int64_t max_nq, const pndf_eval_opts* opts,
                             const pndf_tuning* tuning, void* stream, pndf_plan** out)
{
    if (!out) return plan_invalid("out is NULL");
    *out = nullptr;
    if (!h) return plan_invalid("hierarchy is NULL");
    if (max_nq < 1 || max_nq >= ((int64_t)1 << 32)) return plan_invalid("max_nq must be in [1, 2^32)");
    pndf_eval_opts o{PNDF_KERNEL_GAUSSIAN, 0.f, 3.f, PNDF_ALGO_PERSISTENT, 0};
    if (opts) o = *opts;
    if (o.kernel != PNDF_KERNEL_GAUSSIAN && o.kernel != PNDF_KERNEL_DISK && o.kernel != PNDF_KERNEL_BOX)
        return plan_invalid("unknown footprint kernel");
    if (!(std::isfinite(o.tau) && o.tau >= 0.f)) return plan_invalid("tau must be finite and >= 0");
    if (!(std::isfinite(o.sigma_to_r) && o.sigma_to_r > 0.f)) return plan_invalid("sigma_to_r must be > 0");
    if (o.flags & ~PNDF_EVAL_INPUT_ORDER) return plan_invalid("unknown flags");
    if (o.tau > 0.f && !h->cluster) return plan_invalid("tau > 0 needs a hierarchy built with clusters");
    pndf_tuning t;
    pndf_default_tuning(h, &t);
    if (tuning) t = *tuning;
    if (t.blocks_per_cu < 1 || t.blocks_per_cu > 64) return plan_invalid("blocks_per_cu out of range");
    if (t.split_level < 1 || t.split_level > h->L) return plan_invalid("split_level out of range");
    if (t.queue_factor < 1 || t.queue_factor > 1024) return plan_invalid("queue_factor out of range");
    if (t.use_graph != 0 && t.use_graph != 1) return plan_invalid("use_graph must be 0 or 1");
    pndf_plan* p = new (std::nothrow) pndf_plan;
    if (!p) return PNDF_ENOMEM;
    p->h = h;
    p->tuning = t;
    p->opts = o;
    PersistPlan& P = p->P;
    P.max_nq = max_nq;
    P.capacity = (unsigned long long)max_nq * (unsigned long long)t.queue_factor;
    P.split_level = t.split_level;
    // no single piece of undonatable work takes this long; a worker that waits
    // longer reports an error instead of hanging
    P.wait_ticks = wall_ticks(30.0);
    P.tau = o.tau;
    P.s2r = o.sigma_to_r;
    P.kernel = o.kernel;
    // blocks beyond what one compute unit holds at once would only start when
    // resident workers exit, i.e. at the end of the run: use the resident count
    const int resident = persist_resident_blocks(h->dev, P);
    if (resident > 0 && t.blocks_per_cu > resident) p->tuning.blocks_per_cu = resident;
    P.blocks = compute_units() * p->tuning.blocks_per_cu;
    hipError_t e = hipMalloc(&P.ctl, sizeof(QueueCtl));
    if (e == hipSuccess) e = hipMalloc(&P.acc, sizeof(Fix192) * (size_t)max_nq);
    if (e == hipSuccess) e = hipMalloc(&P.fexp, sizeof(int) * (size_t)max_nq);
    if (e == hipSuccess) e = hipMalloc(&P.tasks, sizeof(unsigned long long) * P.capacity);
    if (e == hipSuccess) e = hipMalloc(&P.flags, sizeof(unsigned) * P.capacity);
    if (e == hipSuccess && !(o.flags & PNDF_EVAL_INPUT_ORDER)) {
        // workers take the queries in spatial (Morton bucket) order
        order_shape(h->dev.logn, &P.order_nb, &P.order_bshift);
        e = hipMalloc(&P.order, sizeof(uint32_t) * (2 * (size_t)max_nq + (size_t)P.order_nb));
    }
    // flags start at 0; the first run publishes with epoch 1
    if (e == hipSuccess) e = hipMemsetAsync(P.flags, 0, sizeof(unsigned) * P.capacity, (hipStream_t)stream);
    if (e == hipSuccess) e = hipMemsetAsync(P.ctl, 0, sizeof(QueueCtl), (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e == hipSuccess && t.use_graph) e = persist_graph_build(h->dev, P);
    if (e != hipSuccess) {
        plan_free(p);
        return hip_fail(e, "pndf_plan_create");
    }
    if (!t.use_graph) persist_prepare(h->dev, P);
    *out = p;
    return PNDF_OK;
}

pndf_status pndf_plan_eval(pndf_plan* plan, const pndf_query* d_q, int64_t nq, float* d_out,
                           void* stream)
{
    if (!plan) return plan_invalid("plan is NULL");
    if (nq < 0 || nq > plan->P.max_nq) return plan_invalid("nq out of range for this plan");
    if (nq == 0) return PNDF_OK;
    if (!d_q || !d_out) return plan_invalid("query or output pointer is NULL");
    hipError_t e = hipPeekAtLastError();
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return hip_fail(e, "earlier device error");
    }
    e = persist_run(plan->P, d_q, nq, d_out, plan->tuning.use_graph != 0, (hipStream_t)stream);
    return e == hipSuccess ? PNDF_OK : hip_fail(e, "pndf_plan_eval");
}

pndf_status pndf_plan_get_tuning(const pndf_plan* plan, pndf_tuning* out)
{
    if (!plan || !out) return plan_invalid("NULL argument");
    *out = plan->tuning;
    return PNDF_OK;
}

pndf_status pndf_plan_get_stats(pndf_plan* plan, pndf_plan_stats* out, void* stream)
{
    if (!plan || !out) return plan_invalid("NULL argument");
    QueueCtl c;
    hipError_t e = hipMemcpyAsync(&c, plan->P.ctl, sizeof(c), hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "pndf_plan_get_stats");
    out->spawned = c.spawned;
    out->refused = c.refused;
    out->idle_spins = c.spins;
    out->error = c.error;
    return PNDF_OK;
}

void pndf_plan_destroy(pndf_plan* plan) { plan_free(plan); }

pndf_status pndf_autotune(const pndf_hier* h, const pndf_query* d_q, int64_t nq,
                          const pndf_eval_opts* opts, pndf_tuning* best, double* best_ms,
                          void* stream)
{
    if (!h || !best) return plan_invalid("NULL argument");
    if (nq < 1 || !d_q) return plan_invalid("autotuning needs a non-empty query sample");
    hipStream_t s = (hipStream_t)stream;
    float* d_out = nullptr;
    hipError_t e = hipMalloc(&d_out, sizeof(float) * (size_t)nq);
    if (e != hipSuccess) return hip_fail(e, "pndf_autotune");
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    double best_t = 1e300;
    pndf_tuning bt;
    pndf_default_tuning(h, &bt);
    pndf_status st = PNDF_OK;
    const int lo = std::min(2, h->L), hi = std::min(8, h->L);
    static const int kBpc[] = {1, 2, 4, 6, 8};
    int tried_bpc = 0;  // largest effective blocks per compute unit timed so far
    for (int bpc : kBpc) {
        if (st != PNDF_OK) break;
        for (int sl = lo; sl <= hi && st == PNDF_OK; ++sl) {
            pndf_tuning t{bpc, sl, 16, 1};
            pndf_plan* p = nullptr;
            st = pndf_plan_create(h, nq, opts, &t, stream, &p);
            if (st != PNDF_OK) break;
            // a count beyond what is resident runs as the resident count: timed already
            t = p->tuning;
            if (sl == lo && t.blocks_per_cu <= tried_bpc) {
                pndf_plan_destroy(p);
                break;
            }
            tried_bpc = std::max(tried_bpc, t.blocks_per_cu);
            st = pndf_plan_eval(p, d_q, nq, d_out, stream);  // warm-up
            float ms_best = 1e30f;
            for (int r = 0; r < 2 && st == PNDF_OK; ++r) {
                (void)hipEventRecord(e0, s);
                st = pndf_plan_eval(p, d_q, nq, d_out, stream);
                (void)hipEventRecord(e1, s);
                if (hipEventSynchronize(e1) != hipSuccess) st = PNDF_EDEVICE;
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                ms_best = std::min(ms_best, ms);
            }
            pndf_plan_stats ps{};
            if (st == PNDF_OK) st = pndf_plan_get_stats(p, &ps, stream);
            pndf_plan_destroy(p);
            if (st == PNDF_OK && ps.error) {
                set_error("persistent workers reported an error during autotuning");
                st = PNDF_EDEVICE;
            }
            if (st == PNDF_OK && ms_best < best_t) {
                best_t = ms_best;
                bt = t;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(d_out);
    if (st != PNDF_OK) return st;
    *best = bt;
    if (best_ms) *best_ms = best_t;
    return PNDF_OK;
}

}  // extern "C"
