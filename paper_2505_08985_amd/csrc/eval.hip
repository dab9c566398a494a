// P-NDF evaluation kernels (Eq. ndf_eval).
//
// A wavefront owns a query (or a subtree of one) at a time; its 64 lanes
// cooperate on the candidates:
//   - brute force: lanes stride over the included cells;
//   - hierarchical: a breadth-limited, depth-first quad-tree descent.  Each level
//     has a list in LDS; the wave pops up to 64 nodes of the lowest non-empty level
//     (one per lane), tests the min-max box (and the cluster cut), and pushes the
//     surviving children with a ballot prefix.  Level-1 nodes push their four
//     cells into a leaf queue that is drained 64 cells at a time, so the
//     triangle tests always run with full waves.
//   - persistent: a fixed grid of workers takes queries from a global counter;
//     when a query's descent reaches the split level it donates those subtrees
//     to a global task queue that idle workers steal from.
// Triangle tests run in float32; a float32 hit is confirmed and its barycentrics
// recomputed in FP64 from the float32 vertices, so the recovered uv and the term
// are accurate even for sliver triangles.  Jacobians come from the mesh build
// (FP64, clamped), never from the hot loop.  Terms are summed exactly (128-bit
// fixed point at a per-query binary point), so D does not depend on the order in
// which hits are found: all algorithms, batch compositions and work splits give
// the same bits.
#include <algorithm>

#include "pndf_internal.h"

namespace pndf {

namespace {

enum { kModeValue = 0, kModeCount = 1, kModeRecord = 2 };

struct Acc {
    Fix128 d{0, 0};
    uint32_t nodes = 0, cells = 0, clusters = 0, hits = 0;
};

struct Rec {  // hit-record cursor (record mode)
    uint64_t* ids;
    float* terms;
    uint64_t pos, end;
};

// FP64 confirmation of a float32 hit, barycentrics and term; < 0 if rejected.
__device__ __forceinline__ float confirm_and_term(const QuerySetup& q, const double v[6], int I,
                                                  int J, int lev, int half, float det_used,
                                                  int logn)
{
    double l1, l2;
    if (!tri_bary_f64(v, (double)q.hx, (double)q.hy, &l1, &l2)) return -1.f;
    return hit_term(q, I, J, lev, half, l1, l2, det_used, logn);
}

// Test the two triangles of texel cell (i, j).  Writes up to two (id, term) pairs.
__device__ __forceinline__ int test_cell(const HierDev& H, const QuerySetup& q, int i, int j,
                                         uint64_t ids[2], float terms[2])
{
    const int w = H.n + 1;
    const float2* p = H.nrm + (int64_t)j * w + i;
    const float2 n0 = p[0], n1 = p[1], n2 = p[w], n3 = p[w + 1];
    const uint8_t dg = H.deg[(int64_t)j * H.n + i];
    bool hl, hu;
    float vl[6], vu[6];
    if (dg == 0) {
        // shared offsets and edge functions of the two triangles (they share n1-n2)
        const float q0x = n0.x - q.hx, q0y = n0.y - q.hy, q1x = n1.x - q.hx, q1y = n1.y - q.hy;
        const float q2x = n2.x - q.hx, q2y = n2.y - q.hy, q3x = n3.x - q.hx, q3y = n3.y - q.hy;
        const float c12 = cross2(q1x, q1y, q2x, q2y);
        const float c20 = cross2(q2x, q2y, q0x, q0y);
        const float c01 = cross2(q0x, q0y, q1x, q1y);
        const float c13 = cross2(q1x, q1y, q3x, q3y);
        const float c32 = cross2(q3x, q3y, q2x, q2y);
        hl = (c12 >= 0.f && c20 >= 0.f && c01 >= 0.f) || (c12 <= 0.f && c20 <= 0.f && c01 <= 0.f);
        hu = (c12 <= 0.f && c13 >= 0.f && c32 >= 0.f) || (c12 >= 0.f && c13 <= 0.f && c32 <= 0.f);
        if (!(hl || hu)) return 0;
        vl[0] = n0.x; vl[1] = n0.y; vl[2] = n1.x; vl[3] = n1.y; vl[4] = n2.x; vl[5] = n2.y;
        vu[0] = n3.x; vu[1] = n3.y; vu[2] = n2.x; vu[3] = n2.y; vu[4] = n1.x; vu[5] = n1.y;
    } else {
        const float cx = 0.5f * (n1.x + n2.x), cy = 0.5f * (n1.y + n2.y);
        if (dg & 1) eqtri_f32(cx, cy, H.rho, vl);
        else { vl[0] = n0.x; vl[1] = n0.y; vl[2] = n1.x; vl[3] = n1.y; vl[4] = n2.x; vl[5] = n2.y; }
        if (dg & 2) eqtri_f32(cx, cy, H.rho, vu);
        else { vu[0] = n3.x; vu[1] = n3.y; vu[2] = n2.x; vu[3] = n2.y; vu[4] = n1.x; vu[5] = n1.y; }
        hl = tri_hit_f32(vl, q.hx, q.hy);
        hu = tri_hit_f32(vu, q.hx, q.hy);
        if (!(hl || hu)) return 0;
    }
    int nh = 0;
    const float2 dd = H.det[(int64_t)j * H.n + i];
    for (int half = 0; half < 2; ++half) {
        if (!(half ? hu : hl)) continue;
        double v[6];
        if (dg & (1 << half)) {
            eqtri_f64(0.5 * ((double)n1.x + (double)n2.x), 0.5 * ((double)n1.y + (double)n2.y),
                      (double)H.rho, v);
        } else {
            const float* f = half ? vu : vl;
            for (int k = 0; k < 6; ++k) v[k] = (double)f[k];
        }
        const float t = confirm_and_term(q, v, i, j, 0, half, half ? dd.y : dd.x, H.logn);
        if (t >= 0.f) {
            ids[nh] = tri_id(0, i, j, half);
            terms[nh] = t;
            ++nh;
        }
    }
    return nh;
}

// Test the two cluster triangles of node (lev, I, J) with packed index idx.
__device__ __forceinline__ int test_cluster(const HierDev& H, const QuerySetup& q, int lev, int I,
                                            int J, int64_t idx, uint64_t ids[2], float terms[2])
{
    const float4 a = H.clu_n[2 * idx], b = H.clu_n[2 * idx + 1];
    const uint8_t dg = H.clu_deg[idx];
    const float2 dd = H.clu_det[idx];
    const float rho = H.rho * (float)(1 << lev);
    const float cx = 0.5f * (a.z + b.x), cy = 0.5f * (a.w + b.y);
    float vl[6], vu[6];
    if (dg & 1) eqtri_f32(cx, cy, rho, vl);
    else { vl[0] = a.x; vl[1] = a.y; vl[2] = a.z; vl[3] = a.w; vl[4] = b.x; vl[5] = b.y; }
    if (dg & 2) eqtri_f32(cx, cy, rho, vu);
    else { vu[0] = b.z; vu[1] = b.w; vu[2] = b.x; vu[3] = b.y; vu[4] = a.z; vu[5] = a.w; }
    int nh = 0;
    for (int half = 0; half < 2; ++half) {
        const float* f = half ? vu : vl;
        if (!tri_hit_f32(f, q.hx, q.hy)) continue;
        double v[6];
        if (dg & (1 << half))
            eqtri_f64(0.5 * ((double)a.z + (double)b.x), 0.5 * ((double)a.w + (double)b.y),
                      (double)rho, v);
        else
            for (int k = 0; k < 6; ++k) v[k] = (double)f[k];
        const float t = confirm_and_term(q, v, I, J, lev, half, half ? dd.y : dd.x, H.logn);
        if (t >= 0.f) {
            ids[nh] = tri_id(lev, I, J, half);
            terms[nh] = t;
            ++nh;
        }
    }
    return nh;
}

// Accumulate this lane's hits; in record mode write them in deterministic order,
// never leaving the query's own CSR slot [pos, end).
template <int MODE>
__device__ __forceinline__ void take_hits(const QuerySetup& q, int nh, const uint64_t ids[2],
                                          const float terms[2], Acc& acc, Rec& rec)
{
    for (int k = 0; k < nh; ++k) fix_add_term(acc.d, terms[k], q.fexp);
    acc.hits += nh;
    if (MODE == kModeRecord) {
        int total;
        const int pos = wave_prefix_small(nh, &total);
        for (int k = 0; k < nh; ++k) {
            const uint64_t at = rec.pos + pos + k;
            if (at < rec.end) {
                rec.ids[at] = ids[k];
                rec.terms[at] = terms[k];
            }
        }
        rec.pos += total;
    }
}

// Reserve `count` task slots; returns the first slot or ~0ull if the queue is full.
__device__ __forceinline__ unsigned long long queue_reserve(const TaskQueue& Q, unsigned count)
{
    unsigned long long old = __hip_atomic_load(&Q.ctl->tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while (true) {
        if (old + count > Q.capacity) return ~0ull;
        if (__hip_atomic_compare_exchange_strong(&Q.ctl->tail, &old, old + count, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return old;
    }
}

// The shared descent.  Roots: every lane with root_ok holds a root item of level
// root_level (level 0: texel cells).  With SPAWN, a node of level split_level that
// passes its tests is donated to the task queue instead of being descended (when
// the queue has room; otherwise it is descended here).
template <int MODE, bool CUT, bool SPAWN>
__device__ void descend(const HierDev& H, const QuerySetup& q, uint32_t* lists, uint32_t* cellq,
                        int root_level, bool root_ok, uint32_t root_item, int split_level,
                        unsigned long long qidx, const TaskQueue& Q, Acc& acc, Rec& rec)
{
    const int lane = threadIdx.x & 63;
    const int logn = H.logn;
    const float4* __restrict__ boxes = CUT ? H.bbox_all : H.bbox;
    uint32_t nonempty = 0;   // bit l: list of level l non-empty (wave-uniform)
    int cntv = 0;            // lane l holds the size of list l
    int ncell = 0;
    {
        const bool ok = root_ok;
        const uint64_t bal = __ballot(ok);
        const int pos = __popcll(bal & ((1ull << lane) - 1ull));
        const int tot = __popcll(bal);
        if (root_level == 0) {
            if (ok) cellq[pos] = root_item;
            ncell = tot;
        } else {
            if (ok) lists[(root_level - 1) * kListCap + pos] = root_item;
            if (lane == root_level) cntv = tot;
            if (tot) nonempty |= 1u << root_level;
        }
        wave_sync();
    }
    while (true) {
        if (ncell >= 64 || (nonempty == 0 && ncell > 0)) {
            const int k = min(ncell, 64), base = ncell - k;
            int nh = 0;
            uint64_t ids[2];
            float terms[2];
            if (lane < k) {
                const uint32_t c = cellq[base + lane];
                nh = test_cell(H, q, (int)(c & 0xffffu), (int)(c >> 16), ids, terms);
                acc.cells += 1;
            }
            ncell = base;
            take_hits<MODE>(q, nh, ids, terms, acc, rec);
            wave_sync();
            continue;
        }
        if (nonempty == 0) break;
        const int l = __builtin_ctz(nonempty);
        const int cnt = __builtin_amdgcn_readlane(cntv, l);
        const int k = min(cnt, 64), base = cnt - k;
        if (lane == l) cntv = base;
        if (base == 0) nonempty &= ~(1u << l);
        uint32_t ch[4];
        int nch = 0;
        int nh = 0;
        bool give = false;
        uint32_t item = 0;
        uint64_t ids[2];
        float terms[2];
        if (lane < k) {
            item = lists[(l - 1) * kListCap + base + lane];
            const int I = (int)(item & 0xffffu), J = (int)(item >> 16);
            const int64_t idx = H.off[l] + (int64_t)J * (H.n >> l) + I;
            const float4 bb = boxes[idx];
            acc.nodes += 1;
            if (q.hx >= bb.x && q.hy >= bb.y && q.hx <= bb.z && q.hy <= bb.w) {
                if (CUT && l <= q.l0 && H.clu_e[idx] <= q.t) {
                    nh = test_cluster(H, q, l, I, J, idx, ids, terms);
                    acc.clusters += 1;
                } else if (SPAWN && l == split_level) {
                    give = true;
                } else {
                    const int side = 1 << (l - 1);
                    const bool x0 = axis_overlap(2 * I * side, side, q.cxlo, q.cxhi, logn);
                    const bool x1 = axis_overlap((2 * I + 1) * side, side, q.cxlo, q.cxhi, logn);
                    const bool y0 = axis_overlap(2 * J * side, side, q.cylo, q.cyhi, logn);
                    const bool y1 = axis_overlap((2 * J + 1) * side, side, q.cylo, q.cyhi, logn);
                    const uint32_t ci = 2u * I, cj = 2u * J;
                    if (x0 && y0) ch[nch++] = ci | (cj << 16);
                    if (x1 && y0) ch[nch++] = (ci + 1) | (cj << 16);
                    if (x0 && y1) ch[nch++] = ci | ((cj + 1) << 16);
                    if (x1 && y1) ch[nch++] = (ci + 1) | ((cj + 1) << 16);
                }
            }
        }
        if (CUT) take_hits<MODE>(q, nh, ids, terms, acc, rec);
        if (SPAWN) {
            const uint64_t gb = __ballot(give);
            if (gb) {
                const unsigned total = (unsigned)__popcll(gb);
                unsigned long long slot = 0;
                if (lane == 0) {
                    // count the tasks before they become visible, then reserve
                    __hip_atomic_fetch_add(&Q.ctl->outstanding, (unsigned long long)total,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    slot = queue_reserve(Q, total);
                    if (slot == ~0ull) {
                        __hip_atomic_fetch_add(&Q.ctl->outstanding, (unsigned long long)(-(long long)total),
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        atomicAdd(&Q.ctl->refused, (unsigned long long)total);
                    } else {
                        atomicAdd(&Q.ctl->spawned, (unsigned long long)total);
                    }
                }
                slot = __shfl(slot, 0, 64);
                if (slot != ~0ull) {
                    if (give) {
                        const unsigned long long at = slot + __popcll(gb & ((1ull << lane) - 1ull));
                        Q.tasks[at] = (qidx << 32) | ((unsigned long long)l << 26) |
                                      ((unsigned long long)(item >> 16) << 13) | (item & 0xffffu);
                        __threadfence();
                        __hip_atomic_store(&Q.flags[at], Q.ctl->epoch, __ATOMIC_RELEASE,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    }
                } else if (give) {
                    // queue full: descend this subtree here
                    const int I = (int)(item & 0xffffu), J = (int)(item >> 16);
                    const int side = 1 << (l - 1);
                    const bool x0 = axis_overlap(2 * I * side, side, q.cxlo, q.cxhi, logn);
                    const bool x1 = axis_overlap((2 * I + 1) * side, side, q.cxlo, q.cxhi, logn);
                    const bool y0 = axis_overlap(2 * J * side, side, q.cylo, q.cyhi, logn);
                    const bool y1 = axis_overlap((2 * J + 1) * side, side, q.cylo, q.cyhi, logn);
                    const uint32_t ci = 2u * I, cj = 2u * J;
                    if (x0 && y0) ch[nch++] = ci | (cj << 16);
                    if (x1 && y0) ch[nch++] = (ci + 1) | (cj << 16);
                    if (x0 && y1) ch[nch++] = ci | ((cj + 1) << 16);
                    if (x1 && y1) ch[nch++] = (ci + 1) | ((cj + 1) << 16);
                }
            }
        }
        int total;
        const int pos = wave_prefix_small(nch, &total);
        if (l == 1) {
            for (int c = 0; c < nch; ++c) cellq[ncell + pos + c] = ch[c];
            ncell += total;
        } else {
            uint32_t* dst = lists + (l - 2) * kListCap;
            for (int c = 0; c < nch; ++c) dst[pos + c] = ch[c];
            if (lane == l - 1) cntv = total;
            if (total) nonempty |= 1u << (l - 1);
        }
        wave_sync();
    }
}

// Root items of a query: the entry-level nodes overlapping the box (<= 4 per
// axis), one per lane of lanes 0..15 where *ok is set.
__device__ __forceinline__ uint32_t root_item(const HierDev& H, const QuerySetup& q, bool* ok)
{
    const int lane = threadIdx.x & 63;
    const int l0 = q.l0, M = H.n >> l0, mm = M - 1;
    const int kx0 = q.cxlo >> l0, ky0 = q.cylo >> l0;
    const int nkx = min((q.cxhi >> l0) - kx0 + 1, M), nky = min((q.cyhi >> l0) - ky0 + 1, M);
    const int ra = lane & 3, rb = lane >> 2;
    *ok = lane < 16 && ra < nkx && rb < nky;
    return (uint32_t)((kx0 + ra) & mm) | ((uint32_t)((ky0 + rb) & mm) << 16);
}

template <int MODE>
__device__ __forceinline__ void finish(const EvalArgs& a, int64_t qi, const QuerySetup& q,
                                       const Acc& acc)
{
    const Fix128 d = wave_sum_fix(acc.d);
    if (MODE == kModeCount) {
        const uint32_t nodes = wave_sum_u32(acc.nodes), cells = wave_sum_u32(acc.cells);
        const uint32_t clus = wave_sum_u32(acc.clusters), hits = wave_sum_u32(acc.hits);
        if (lane_id() == 0) {
            uint32_t* c = a.counts + 4 * qi;
            c[0] = nodes; c[1] = cells; c[2] = clus; c[3] = hits;
        }
    }
    if (lane_id() == 0) a.out[qi] = fix_to_float(d, q.fexp);
}

template <int MODE>
__device__ __forceinline__ void invalid(const EvalArgs& a, int64_t qi)
{
    if (lane_id() == 0) {
        a.out[qi] = __int_as_float(0x7fc00000);
        if (MODE == kModeCount) {
            uint32_t* c = a.counts + 4 * qi;
            c[0] = c[1] = c[2] = c[3] = 0;
        }
    }
}

// ------------------------------------------------------------ brute force
template <int MODE>
__global__ __launch_bounds__(256) void k_eval_brute(HierDev H, EvalArgs a)
{
    const int64_t qi = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (qi >= a.nq) return;
    const int lane = threadIdx.x & 63;
    const QuerySetup q = setup_query(a.q[qi], a.s2r, 0.f, H.L, H.eps);
    if (!q.valid) { invalid<MODE>(a, qi); return; }
    const int n = H.n, msk = n - 1;
    const int spanx = q.cxhi - q.cxlo + 1, spany = q.cyhi - q.cylo + 1;
    const int nx = spanx >= n ? n : spanx, ny = spany >= n ? n : spany;
    const int total = nx * ny;  // <= 8192^2
    Acc acc;
    Rec rec{a.ids, a.terms, MODE == kModeRecord ? a.offsets[qi] : 0,
            MODE == kModeRecord ? a.offsets[qi + 1] : 0};
    for (int base = 0; base < total; base += 64) {
        const int idx = base + lane;
        int nh = 0;
        uint64_t ids[2];
        float terms[2];
        if (idx < total) {
            const int ca = idx % nx, cb = idx / nx;
            const int i = spanx >= n ? ca : ((q.cxlo + ca) & msk);
            const int j = spany >= n ? cb : ((q.cylo + cb) & msk);
            nh = test_cell(H, q, i, j, ids, terms);
            acc.cells += 1;
        }
        take_hits<MODE>(q, nh, ids, terms, acc, rec);
    }
    finish<MODE>(a, qi, q, acc);
}

// ------------------------------------------------------------ hierarchical

// LDS per wave: L lists of kListCap node entries (levels 1..L) + the leaf queue.
template <int MODE, bool CUT>
__global__ __launch_bounds__(256) void k_eval_plain(HierDev H, EvalArgs a)
{
    extern __shared__ uint32_t lds[];
    const int wave = threadIdx.x >> 6;
    const int64_t qi = (int64_t)blockIdx.x * 4 + wave;
    if (qi >= a.nq) return;
    uint32_t* lists = lds + (size_t)wave * wave_lds_words(H.L);
    uint32_t* cellq = lists + H.L * kListCap;
    const QuerySetup q = setup_query(a.q[qi], a.s2r, CUT ? a.tau : 0.f, H.L, H.eps);
    if (!q.valid) { invalid<MODE>(a, qi); return; }
    Acc acc;
    Rec rec{a.ids, a.terms, MODE == kModeRecord ? a.offsets[qi] : 0,
            MODE == kModeRecord ? a.offsets[qi + 1] : 0};
    bool ok;
    const uint32_t item = root_item(H, q, &ok);
    TaskQueue none{};
    descend<MODE, CUT, false>(H, q, lists, cellq, q.l0, ok, item, 0, 0, none, acc, rec);
    finish<MODE>(a, qi, q, acc);
}

// ------------------------------------------------------------ persistent
__device__ __forceinline__ void acc_atomic_add(Fix128* dst, const Fix128& v)
{
    if (v.lo == 0 && v.hi == 0) return;
    const unsigned long long old = atomicAdd((unsigned long long*)&dst->lo, (unsigned long long)v.lo);
    const unsigned long long carry = (old + v.lo < old) ? 1ull : 0ull;
    atomicAdd((unsigned long long*)&dst->hi, (unsigned long long)(v.hi + carry));
}

__global__ void k_persist_reset(QueueCtl* ctl, Fix128* acc, int* fexp, const pndf_query* q,
                                long long nq, float* out, unsigned epoch)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    for (long long i = t; i < nq; i += (long long)gridDim.x * blockDim.x) {
        acc[i].lo = 0;
        acc[i].hi = 0;
        fexp[i] = 0;
    }
    if (t == 0) {
        ctl->qhead = 0;
        ctl->head = 0;
        ctl->tail = 0;
        ctl->outstanding = 0;
        ctl->spawned = ctl->refused = ctl->spins = 0;
        ctl->epoch = epoch;
        ctl->error = 0;
        ctl->q = q;
        ctl->out = out;
        ctl->nq = nq;
    }
}

template <bool CUT>
__global__ __launch_bounds__(256) void k_persist(HierDev H, PersistArgs pa)
{
    extern __shared__ uint32_t lds[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint32_t* lists = lds + (size_t)wave * wave_lds_words(H.L);
    uint32_t* cellq = lists + H.L * kListCap;
    QueueCtl* ctl = pa.Q.ctl;
    const long long nq = ctl->nq;
    const pndf_query* qs = ctl->q;
    const unsigned epoch = ctl->epoch;
    Rec rec{nullptr, nullptr, 0, 0};
    const unsigned long long kSpinLimit = 1ull << 24;  // consecutive idle polls before giving up
    unsigned long long idle = 0, spins = 0;
    while (true) {
        // 1) stolen work first: a published task below `tail`
        long long task_slot = -1;
        long long query = -1;
        if (lane == 0) {
            unsigned long long h = __hip_atomic_load(&ctl->head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            while (true) {
                const unsigned long long t = __hip_atomic_load(&ctl->tail, __ATOMIC_RELAXED,
                                                               __HIP_MEMORY_SCOPE_AGENT);
                if (h >= t) break;
                if (__hip_atomic_compare_exchange_strong(&ctl->head, &h, h + 1, __ATOMIC_RELAXED,
                                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    task_slot = (long long)h;
                    break;
                }
            }
            // 2) a new query, counted as outstanding before it is taken
            if (task_slot < 0 && (long long)__hip_atomic_load(&ctl->qhead, __ATOMIC_RELAXED,
                                                              __HIP_MEMORY_SCOPE_AGENT) < nq) {
                __hip_atomic_fetch_add(&ctl->outstanding, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const unsigned long long qn = __hip_atomic_fetch_add(&ctl->qhead, 1ull, __ATOMIC_RELAXED,
                                                                     __HIP_MEMORY_SCOPE_AGENT);
                if ((long long)qn < nq) {
                    query = (long long)qn;
                } else {
                    __hip_atomic_fetch_add(&ctl->outstanding, (unsigned long long)-1ll, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
        task_slot = __shfl(task_slot, 0, 64);
        query = __shfl(query, 0, 64);
        if (task_slot < 0 && query < 0) {
            // nothing available now: finished once every query is taken and nothing
            // is outstanding, otherwise wait for donated tasks
            int done = 0;
            if (lane == 0) {
                const unsigned long long qh = __hip_atomic_load(&ctl->qhead, __ATOMIC_SEQ_CST,
                                                                __HIP_MEMORY_SCOPE_AGENT);
                const unsigned long long os = __hip_atomic_load(&ctl->outstanding, __ATOMIC_SEQ_CST,
                                                                __HIP_MEMORY_SCOPE_AGENT);
                done = ((long long)qh >= nq && os == 0) ? 1 : 0;
                ++spins;
                if (!done && ++idle > kSpinLimit) {
                    atomicOr(&ctl->error, 1u);
                    done = 1;
                }
            }
            done = __shfl(done, 0, 64);
            if (done) break;
            __builtin_amdgcn_s_sleep(8);
            continue;
        }
        idle = 0;
        Acc acc;
        if (task_slot >= 0) {
            // wait for the donor to publish the slot; never use an unpublished or
            // malformed task word
            unsigned long long word = 0;
            int ok = 0;
            if (lane == 0) {
                unsigned long long w = 0;
                ok = 1;
                while (__hip_atomic_load(&pa.Q.flags[task_slot], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) !=
                       epoch) {
                    if (++w > kSpinLimit) {
                        atomicOr(&ctl->error, 2u);
                        ok = 0;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                if (ok) {
                    word = pa.Q.tasks[task_slot];
                    const long long wq = (long long)(word >> 32);
                    const int wl = (int)((word >> 26) & 0x3fu);
                    const int wi = (int)(word & 0x1fffu), wj = (int)((word >> 13) & 0x1fffu);
                    if (wq >= nq || wl < 1 || wl > H.L || wi >= (H.n >> wl) || wj >= (H.n >> wl)) {
                        atomicOr(&ctl->error, 4u);
                        ok = 0;
                    }
                }
            }
            ok = __shfl(ok, 0, 64);
            word = __shfl(word, 0, 64);
            if (ok) {
                const long long qi = (long long)(word >> 32);
                const int lev = (int)((word >> 26) & 0x3fu);
                const uint32_t item = (uint32_t)(word & 0x1fffu) | ((uint32_t)((word >> 13) & 0x1fffu) << 16);
                const QuerySetup q = setup_query(qs[qi], pa.s2r, CUT ? pa.tau : 0.f, H.L, H.eps);
                descend<kModeValue, CUT, false>(H, q, lists, cellq, lev, lane == 0, item, 0, 0, pa.Q, acc,
                                                rec);
                const Fix128 d = wave_sum_fix(acc.d);
                if (lane == 0) acc_atomic_add(&pa.acc[qi], d);
            }
            if (lane == 0) {
                __threadfence();
                __hip_atomic_fetch_add(&ctl->outstanding, (unsigned long long)-1ll, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            }
        } else {
            const QuerySetup q = setup_query(qs[query], pa.s2r, CUT ? pa.tau : 0.f, H.L, H.eps);
            if (q.valid) {
                bool ok;
                const uint32_t item = root_item(H, q, &ok);
                if (q.l0 > pa.split_level)
                    descend<kModeValue, CUT, true>(H, q, lists, cellq, q.l0, ok, item, pa.split_level,
                                                   (unsigned long long)query, pa.Q, acc, rec);
                else
                    descend<kModeValue, CUT, false>(H, q, lists, cellq, q.l0, ok, item, 0, 0, pa.Q, acc,
                                                    rec);
            }
            const Fix128 d = wave_sum_fix(acc.d);
            if (lane == 0) {
                pa.fexp[query] = q.valid ? q.fexp : 0x7fffffff;
                acc_atomic_add(&pa.acc[query], d);
                __threadfence();
                __hip_atomic_fetch_add(&ctl->outstanding, (unsigned long long)-1ll, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
    if (lane == 0 && spins) atomicAdd(&ctl->spins, spins);
}

__global__ void k_persist_finalize(const QueueCtl* ctl, const Fix128* acc, const int* fexp)
{
    const long long nq = ctl->nq;
    float* out = ctl->out;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nq;
         i += (long long)gridDim.x * blockDim.x) {
        const int e = fexp[i];
        out[i] = e == 0x7fffffff ? __int_as_float(0x7fc00000) : fix_to_float(acc[i], e);
    }
}

template <int MODE>
hipError_t launch_mode(const HierDev& H, const EvalArgs& a, int algo, hipStream_t s)
{
    const unsigned blocks = (unsigned)((a.nq + 3) / 4);
    if (algo == PNDF_ALGO_BRUTE) {
        hipLaunchKernelGGL(k_eval_brute<MODE>, dim3(blocks), dim3(256), 0, s, H, a);
    } else {
        const size_t lds = sizeof(uint32_t) * 4 * wave_lds_words(H.L);
        if (a.tau > 0.f)
            hipLaunchKernelGGL((k_eval_plain<MODE, true>), dim3(blocks), dim3(256), lds, s, H, a);
        else
            hipLaunchKernelGGL((k_eval_plain<MODE, false>), dim3(blocks), dim3(256), lds, s, H, a);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_eval(const HierDev& H, const EvalArgs& a, int algo, hipStream_t s)
{
    if (a.nq <= 0) return hipSuccess;
    if (a.offsets) return launch_mode<kModeRecord>(H, a, algo, s);
    if (a.counts) return launch_mode<kModeCount>(H, a, algo, s);
    return launch_mode<kModeValue>(H, a, algo, s);
}

// ---------------------------------------------------------------- persistent
// The launch sequence reset -> workers -> finalize, as a HIP graph.  Only the
// reset node's arguments (queries, count, output, epoch) change between runs; the
// workers and the finalizer read them from the control block.
static void reset_params(PersistPlan& P, const pndf_query* q, long long nq, float* out)
{
    P.rq = q;
    P.rnq = nq;
    P.rout = out;
    P.rargs[0] = &P.ctl;
    P.rargs[1] = &P.acc;
    P.rargs[2] = &P.fexp;
    P.rargs[3] = &P.rq;
    P.rargs[4] = &P.rnq;
    P.rargs[5] = &P.rout;
    P.rargs[6] = &P.epoch;
    P.reset.func = (void*)k_persist_reset;
    P.reset.gridDim = dim3((unsigned)std::min<long long>(1024, (P.max_nq + 255) / 256 + 1));
    P.reset.blockDim = dim3(256);
    P.reset.sharedMemBytes = 0;
    P.reset.kernelParams = P.rargs;
    P.reset.extra = nullptr;
}

hipError_t persist_graph_build(const HierDev& H, PersistPlan& P)
{
    P.H = H;
    P.pa.Q.ctl = P.ctl;
    P.pa.Q.tasks = P.tasks;
    P.pa.Q.flags = P.flags;
    P.pa.Q.capacity = P.capacity;
    P.pa.acc = P.acc;
    P.pa.fexp = P.fexp;
    P.pa.tau = P.tau;
    P.pa.s2r = P.s2r;
    P.pa.split_level = P.split_level;
    reset_params(P, nullptr, 0, nullptr);
    P.wargs[0] = &P.H;
    P.wargs[1] = &P.pa;
    hipKernelNodeParams work{};
    work.func = P.tau > 0.f ? (void*)k_persist<true> : (void*)k_persist<false>;
    work.gridDim = dim3((unsigned)P.blocks);
    work.blockDim = dim3(256);
    work.sharedMemBytes = (unsigned)(sizeof(uint32_t) * 4 * wave_lds_words(H.L));
    work.kernelParams = P.wargs;
    work.extra = nullptr;
    P.fargs[0] = &P.ctl;
    P.fargs[1] = &P.acc;
    P.fargs[2] = &P.fexp;
    hipKernelNodeParams fin{};
    fin.func = (void*)k_persist_finalize;
    fin.gridDim = dim3((unsigned)std::min<long long>(1024, (P.max_nq + 255) / 256 + 1));
    fin.blockDim = dim3(256);
    fin.sharedMemBytes = 0;
    fin.kernelParams = P.fargs;
    fin.extra = nullptr;
    hipError_t e = hipGraphCreate(&P.graph, 0);
    hipGraphNode_t nw, nf;
    if (e == hipSuccess) e = hipGraphAddKernelNode(&P.reset_node, P.graph, nullptr, 0, &P.reset);
    if (e == hipSuccess) e = hipGraphAddKernelNode(&nw, P.graph, &P.reset_node, 1, &work);
    if (e == hipSuccess) e = hipGraphAddKernelNode(&nf, P.graph, &nw, 1, &fin);
    if (e == hipSuccess) e = hipGraphInstantiate(&P.exec, P.graph, nullptr, nullptr, 0);
    return e;
}

hipError_t persist_run(PersistPlan& P, const pndf_query* q, long long nq, float* out, bool use_graph,
                       hipStream_t s)
{
    ++P.epoch;
    reset_params(P, q, nq, out);
    if (use_graph) {
        hipError_t e = hipGraphExecKernelNodeSetParams(P.exec, P.reset_node, &P.reset);
        if (e == hipSuccess) e = hipGraphLaunch(P.exec, s);
        return e;
    }
    hipLaunchKernelGGL(k_persist_reset, P.reset.gridDim, P.reset.blockDim, 0, s, P.ctl, P.acc, P.fexp,
                       q, nq, out, P.epoch);
    const size_t lds = sizeof(uint32_t) * 4 * wave_lds_words(P.H.L);
    if (P.tau > 0.f)
        hipLaunchKernelGGL(k_persist<true>, dim3((unsigned)P.blocks), dim3(256), lds, s, P.H, P.pa);
    else
        hipLaunchKernelGGL(k_persist<false>, dim3((unsigned)P.blocks), dim3(256), lds, s, P.H, P.pa);
    hipLaunchKernelGGL(k_persist_finalize, P.reset.gridDim, dim3(256), 0, s, P.ctl, P.acc, P.fexp);
    return hipGetLastError();
}

}  // namespace pndf
