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
// (FP64, clamped), never from the hot loop.  Terms are summed exactly (192-bit
// fixed point at a per-query binary point), so D does not depend on the order in
// which hits are found: all algorithms, batch compositions and work splits give
// the same bits.
#include <algorithm>

#include "pndf_internal.h"

namespace pndf {

namespace {

enum { kModeValue = 0, kModeCount = 1, kModeRecord = 2 };

struct Acc {
    Fix192 d{0, 0, 0};
    uint32_t nodes = 0, cells = 0, clusters = 0, hits = 0;
};

struct Rec {  // hit-record cursor (record mode)
    uint64_t* ids;
    float* terms;
    uint64_t pos, end;
};

// FP64 confirmation of a float32 hit, barycentrics and term; < 0 if rejected.
__device__ __forceinline__ double confirm_and_term(const QuerySetup& q, const double v[6], int I,
                                                   int J, int lev, int half, float det_used,
                                                   int logn)
{
    double l1, l2;
    if (!tri_bary_f64(v, (double)q.hx, (double)q.hy, &l1, &l2)) return -1.0;
    return hit_term(q, I, J, lev, half, l1, l2, det_used, logn);
}

// Per-lane hit sink: value/count modes add the term to the exact accumulator at
// once; record mode also buffers (id, term) until the wave writes its records in
// lane order.
template <int MODE>
struct HitSink {
    static constexpr int kMax = MODE == kModeRecord ? 8 : 1;
    uint64_t ids[kMax];
    float terms[kMax];
    int n = 0;
    __device__ __forceinline__ void put(const QuerySetup& q, Acc& acc, uint64_t id, double t)
    {
        fix_add_term(acc.d, t, q.fexp);
        acc.hits += 1;
        if (MODE == kModeRecord && n < kMax) {
            ids[n] = id;
            terms[n] = (float)t;
        }
        ++n;
    }
};

// Exclusive prefix over the wave of a per-lane count in [0, 15], and the total.
__device__ __forceinline__ int wave_prefix16(int c, int* total)
{
    const uint64_t b0 = __ballot(c & 1), b1 = __ballot(c & 2), b2 = __ballot(c & 4), b3 = __ballot(c & 8);
    const uint64_t lt = (1ull << lane_id()) - 1ull;
    *total = __popcll(b0) + 2 * __popcll(b1) + 4 * __popcll(b2) + 8 * __popcll(b3);
    return __popcll(b0 & lt) + 2 * __popcll(b1 & lt) + 4 * __popcll(b2 & lt) + 8 * __popcll(b3 & lt);
}

// Write the wave's buffered records in lane order, never leaving the query's own
// CSR slot [pos, end).  Every lane must call it.
template <int MODE>
__device__ __forceinline__ void flush_records(HitSink<MODE>& hs, Rec& rec)
{
    if (MODE == kModeRecord) {
        int total;
        const int pos = wave_prefix16(hs.n, &total);
        for (int k = 0; k < hs.n && k < HitSink<MODE>::kMax; ++k) {
            const uint64_t at = rec.pos + pos + k;
            if (at < rec.end) {
                rec.ids[at] = hs.ids[k];
                rec.terms[at] = hs.terms[k];
            }
        }
        rec.pos += total;
    }
    hs.n = 0;
}

// The two triangles of one cell from its four corner normals and clamp bits.
template <int MODE>
__device__ __forceinline__ void cell_triangles(const HierDev& H, const QuerySetup& q, int i, int j,
                                               float2 n0, float2 n1, float2 n2, float2 n3, uint8_t dg,
                                               Acc& acc, HitSink<MODE>& hs)
{
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
        if (!(hl || hu)) return;
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
        if (!(hl || hu)) return;
    }
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
        const double t = confirm_and_term(q, v, i, j, 0, half, half ? dd.y : dd.x, H.logn);
        if (t >= 0.0) hs.put(q, acc, tri_id(0, i, j, half), t);
    }
}

// A texel cell tested from the padded normal plane (brute force, tiny footprints).
template <int MODE>
__device__ __forceinline__ void plane_cell(const HierDev& H, const QuerySetup& q, int i, int j, Acc& acc,
                                           HitSink<MODE>& hs)
{
    const int w = H.n + 1;
    const float2* p = H.nrm + (int64_t)j * w + i;
    cell_triangles<MODE>(H, q, i, j, p[0], p[1], p[w], p[w + 1], H.deg[(int64_t)j * H.n + i], acc, hs);
    acc.cells += 1;
}

// The 2 x 2 cells of level-1 node (I, J) (leaf record m), those overlapping the box.
template <int MODE>
__device__ __forceinline__ void leaf_quad(const HierDev& H, const QuerySetup& q, int I, int J, uint32_t m,
                                          Acc& acc, HitSink<MODE>& hs)
{
    const float4* r = reinterpret_cast<const float4*>(H.quad + m);
    const float4 a = r[0], b = r[1], c = r[2], d = r[3], e = r[4];
    const float2 t[9] = {make_float2(a.x, a.y), make_float2(a.z, a.w), make_float2(b.x, b.y),
                         make_float2(b.z, b.w), make_float2(c.x, c.y), make_float2(c.z, c.w),
                         make_float2(d.x, d.y), make_float2(d.z, d.w), make_float2(e.x, e.y)};
    const uint32_t dg4 = __float_as_uint(e.z);
    const int logn = H.logn;
    const bool x0 = axis_overlap(2 * I, 1, q.cxlo, q.cxhi, logn);
    const bool x1 = axis_overlap(2 * I + 1, 1, q.cxlo, q.cxhi, logn);
    const bool y0 = axis_overlap(2 * J, 1, q.cylo, q.cyhi, logn);
    const bool y1 = axis_overlap(2 * J + 1, 1, q.cylo, q.cyhi, logn);
#pragma unroll
    for (int c4 = 0; c4 < 4; ++c4) {
        const int di = c4 & 1, dj = c4 >> 1;
        if (!((di ? x1 : x0) && (dj ? y1 : y0))) continue;
        acc.cells += 1;
        cell_triangles<MODE>(H, q, 2 * I + di, 2 * J + dj, t[3 * dj + di], t[3 * dj + di + 1],
                             t[3 * dj + di + 3], t[3 * dj + di + 4], (uint8_t)(dg4 >> (8 * c4)), acc, hs);
    }
}

// The two cluster triangles of node (lev, I, J) with packed index idx.
template <int MODE>
__device__ __forceinline__ void cluster_pair(const HierDev& H, const QuerySetup& q, int lev, int I, int J,
                                             int64_t idx, Acc& acc, HitSink<MODE>& hs)
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
    acc.clusters += 1;
    for (int half = 0; half < 2; ++half) {
        const float* f = half ? vu : vl;
        if (!tri_hit_f32(f, q.hx, q.hy)) continue;
        double v[6];
        if (dg & (1 << half))
            eqtri_f64(0.5 * ((double)a.z + (double)b.x), 0.5 * ((double)a.w + (double)b.y), (double)rho, v);
        else
            for (int k = 0; k < 6; ++k) v[k] = (double)f[k];
        const double t = confirm_and_term(q, v, I, J, lev, half, half ? dd.y : dd.x, H.logn);
        if (t >= 0.0) hs.put(q, acc, tri_id(lev, I, J, half), t);
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

__device__ __forceinline__ bool in_box(const QuerySetup& q, const float4& bb)
{
    return q.hx >= bb.x && q.hy >= bb.y && q.hx <= bb.z && q.hy <= bb.w;
}

// The shared descent.  List items are nodes (Morton codes) whose box contains h
// and whose region meets the support box.  A lane takes one item: a node under the
// cut answers with its cluster triangles; a level-1 node tests its 2 x 2 cells from
// its leaf record; any other node loads its (up to) four overlapping children's
// boxes together and pushes those that contain h.  Roots: every lane with root_ok
// holds a root of level root_level (level 0: texel cell packed i | j << 16; else a
// Morton code), box-tested here unless roots_tested.  With SPAWN, a node of level
// split_level is donated to the task queue instead of expanded (when the queue has
// room; otherwise it is expanded here).
template <int MODE, bool CUT, bool SPAWN>
__device__ void descend(const HierDev& H, const QuerySetup& q, uint32_t* lists, int root_level,
                        bool root_ok, uint32_t root_item, bool roots_tested, int split_level,
                        unsigned long long qidx, const TaskQueue& Q, Acc& acc, Rec& rec)
{
    static_assert(!SPAWN || MODE == kModeValue, "donation is only used by value-mode workers");
    const int lane = threadIdx.x & 63;
    const int logn = H.logn;
    const float4* __restrict__ boxes = CUT ? H.bbox_all : H.bbox;
    HitSink<MODE> hs;
    if (root_level == 0) {
        if (root_ok) plane_cell<MODE>(H, q, (int)(root_item & 0xffffu), (int)(root_item >> 16), acc, hs);
        flush_records<MODE>(hs, rec);
        return;
    }
    uint32_t nonempty = 0;   // bit l: list of level l non-empty (wave-uniform)
    int cntv = 0;            // lane l holds the size of list l
    {
        bool ok = root_ok;
        if (ok && !roots_tested) {
            acc.nodes += 1;
            ok = in_box(q, boxes[H.off[root_level] + root_item]);
        }
        const uint64_t bal = __ballot(ok);
        const int pos = __popcll(bal & ((1ull << lane) - 1ull));
        const int tot = __popcll(bal);
        if (ok) lists[(root_level - 1) * kListCap + pos] = root_item;
        if (lane == root_level) cntv = tot;
        if (tot) nonempty |= 1u << root_level;
        wave_sync();
    }
    while (nonempty) {
        const int l = __builtin_ctz(nonempty);
        const int cnt = __builtin_amdgcn_readlane(cntv, l);
        const int k = min(cnt, 64), base = cnt - k;
        if (lane == l) cntv = base;
        if (base == 0) nonempty &= ~(1u << l);
        uint32_t ch[4];
        int nch = 0;
        bool give = false;
        uint32_t m = 0;
        if (lane < k) {
            m = lists[(l - 1) * kListCap + base + lane];
            const int I = (int)morton_compact(m), J = (int)morton_compact(m >> 1);
            const int64_t idx = H.off[l] + m;
            if (CUT && l <= q.l0 && H.clu_e[idx] <= q.t) {
                cluster_pair<MODE>(H, q, l, I, J, idx, acc, hs);
            } else if (SPAWN && l == split_level) {
                give = true;
            } else if (l == 1) {
                leaf_quad<MODE>(H, q, I, J, m, acc, hs);
            } else {
                const int side = 1 << (l - 1);
                const bool x0 = axis_overlap(2 * I * side, side, q.cxlo, q.cxhi, logn);
                const bool x1 = axis_overlap((2 * I + 1) * side, side, q.cxlo, q.cxhi, logn);
                const bool y0 = axis_overlap(2 * J * side, side, q.cylo, q.cyhi, logn);
                const bool y1 = axis_overlap((2 * J + 1) * side, side, q.cylo, q.cyhi, logn);
                const float4* cb = boxes + H.off[l - 1] + 4 * (int64_t)m;
                float4 b0 = make_float4(1.f, 1.f, -1.f, -1.f), b1 = b0, b2 = b0, b3 = b0;
                if (x0 && y0) b0 = cb[0];
                if (x1 && y0) b1 = cb[1];
                if (x0 && y1) b2 = cb[2];
                if (x1 && y1) b3 = cb[3];
                acc.nodes += (uint32_t)((x0 && y0) + (x1 && y0) + (x0 && y1) + (x1 && y1));
                if (in_box(q, b0)) ch[nch++] = 4 * m;
                if (in_box(q, b1)) ch[nch++] = 4 * m + 1;
                if (in_box(q, b2)) ch[nch++] = 4 * m + 2;
                if (in_box(q, b3)) ch[nch++] = 4 * m + 3;
            }
        }
        if (SPAWN) {
            const uint64_t gb = __ballot(give);
            if (gb) {
                const unsigned total = (unsigned)__popcll(gb);
                unsigned long long slot = 0;
                if (lane == 0) {
                    // count the tasks before they become visible, then reserve
                    __hip_atomic_fetch_add(&Q.ctl->outstanding, (unsigned long long)total, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
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
                        Q.tasks[at] = (qidx << 32) | ((unsigned long long)l << 26) | (unsigned long long)m;
                        __threadfence();
                        __hip_atomic_store(&Q.flags[at], Q.ctl->epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                    }
                } else if (give) {
                    // queue full: handle this node here like any other list item
                    const int I = (int)morton_compact(m), J = (int)morton_compact(m >> 1);
                    if (l == 1) {
                        leaf_quad<MODE>(H, q, I, J, m, acc, hs);
                    } else {
                        const int side = 1 << (l - 1);
                        const bool x0 = axis_overlap(2 * I * side, side, q.cxlo, q.cxhi, logn);
                        const bool x1 = axis_overlap((2 * I + 1) * side, side, q.cxlo, q.cxhi, logn);
                        const bool y0 = axis_overlap(2 * J * side, side, q.cylo, q.cyhi, logn);
                        const bool y1 = axis_overlap((2 * J + 1) * side, side, q.cylo, q.cyhi, logn);
                        const float4* cb = boxes + H.off[l - 1] + 4 * (int64_t)m;
                        acc.nodes += (uint32_t)((x0 && y0) + (x1 && y0) + (x0 && y1) + (x1 && y1));
                        if (x0 && y0 && in_box(q, cb[0])) ch[nch++] = 4 * m;
                        if (x1 && y0 && in_box(q, cb[1])) ch[nch++] = 4 * m + 1;
                        if (x0 && y1 && in_box(q, cb[2])) ch[nch++] = 4 * m + 2;
                        if (x1 && y1 && in_box(q, cb[3])) ch[nch++] = 4 * m + 3;
                    }
                }
            }
        }
        flush_records<MODE>(hs, rec);
        if (l >= 2) {
            int total;
            const int pos = wave_prefix_small(nch, &total);
            uint32_t* dst = lists + (l - 2) * kListCap;
            for (int c = 0; c < nch; ++c) dst[pos + c] = ch[c];
            if (lane == l - 1) cntv = total;
            if (total) nonempty |= 1u << (l - 1);
        }
        wave_sync();
    }
}

// Root items of a query: the entry-level nodes overlapping the box (<= 4 per
// axis), one per lane of lanes 0..15 where *ok is set; Morton codes (level >= 1)
// or packed texel cells (entry level 0).
__device__ __forceinline__ uint32_t root_item(const HierDev& H, const QuerySetup& q, bool* ok)
{
    const int lane = threadIdx.x & 63;
    const int l0 = q.l0, M = H.n >> l0, mm = M - 1;
    const int kx0 = q.cxlo >> l0, ky0 = q.cylo >> l0;
    const int nkx = min((q.cxhi >> l0) - kx0 + 1, M), nky = min((q.cyhi >> l0) - ky0 + 1, M);
    const int ra = lane & 3, rb = lane >> 2;
    *ok = lane < 16 && ra < nkx && rb < nky;
    const uint32_t I = (uint32_t)((kx0 + ra) & mm), J = (uint32_t)((ky0 + rb) & mm);
    return l0 == 0 ? (I | (J << 16)) : morton(I, J);
}

template <int MODE>
__device__ __forceinline__ void finish(const EvalArgs& a, int64_t qi, const QuerySetup& q,
                                       const Acc& acc)
{
    const Fix192 d = wave_sum_fix(acc.d);
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
    const int64_t local = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (local >= a.slots) return;
    const int64_t qi = a.slot0 + local;
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
    HitSink<MODE> hs;
    for (int base = 0; base < total; base += 64) {
        const int idx = base + lane;
        if (idx < total) {
            const int ca = idx % nx, cb = idx / nx;
            const int i = spanx >= n ? ca : ((q.cxlo + ca) & msk);
            const int j = spany >= n ? cb : ((q.cylo + cb) & msk);
            plane_cell<MODE>(H, q, i, j, acc, hs);
        }
        flush_records<MODE>(hs, rec);
    }
    finish<MODE>(a, qi, q, acc);
}

// ------------------------------------------------------------ hierarchical

// One wavefront per workgroup (a long query holds only its own LDS).  LDS: L lists
// of kListCap node entries (levels 1..L) + the leaf queue.
template <int MODE, bool CUT>
__global__ __launch_bounds__(64) void k_eval_plain(HierDev H, EvalArgs a)
{
    extern __shared__ uint32_t lds[];
    const int64_t local = xcd_contiguous(blockIdx.x, gridDim.x);
    if (local >= a.slots) return;
    const int64_t slot = a.slot0 + local;
    const int64_t qi = a.order ? (int64_t)a.order[slot] : slot;
    uint32_t* lists = lds;
    const QuerySetup q = setup_query(a.q[qi], a.s2r, CUT ? a.tau : 0.f, H.L, H.eps);
    if (!q.valid) { invalid<MODE>(a, qi); return; }
    Acc acc;
    Rec rec{a.ids, a.terms, MODE == kModeRecord ? a.offsets[qi] : 0,
            MODE == kModeRecord ? a.offsets[qi + 1] : 0};
    bool ok;
    const uint32_t item = root_item(H, q, &ok);
    TaskQueue none{};
    descend<MODE, CUT, false>(H, q, lists, q.l0, ok, item, false, 0, 0, none, acc, rec);
    finish<MODE>(a, qi, q, acc);
}

// ------------------------------------------------------------ persistent
// Exact atomic accumulation of a 192-bit value: each word is added atomically and
// every carry out of a word is added to the next one, so once all atomics have
// completed the sum is exact whatever their interleaving.
__device__ __forceinline__ void acc_atomic_add(Fix192* dst, const Fix192& v)
{
    unsigned long long* w = (unsigned long long*)dst;
    unsigned long long c1 = 0, c2 = 0;
    if (v.w0) {
        const unsigned long long old = atomicAdd(&w[0], (unsigned long long)v.w0);
        c1 = (old + v.w0 < old) ? 1ull : 0ull;
    }
    if (v.w1) {
        const unsigned long long old = atomicAdd(&w[1], (unsigned long long)v.w1);
        c2 += (old + v.w1 < old) ? 1ull : 0ull;
    }
    if (c1) {
        const unsigned long long old = atomicAdd(&w[1], 1ull);
        c2 += (old + 1ull < old) ? 1ull : 0ull;
    }
    if (v.w2 + c2) atomicAdd(&w[2], (unsigned long long)(v.w2 + c2));
}

__global__ void k_persist_reset(QueueCtl* ctl, Fix192* acc, int* fexp, const pndf_query* q,
                                long long nq, float* out, unsigned epoch)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    for (long long i = t; i < nq; i += (long long)gridDim.x * blockDim.x) {
        acc[i].w0 = 0;
        acc[i].w1 = 0;
        acc[i].w2 = 0;
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
                    const uint64_t wm = word & 0x3ffffffu;
                    if (wq >= nq || wl < 1 || wl > H.L ||
                        wm >= (uint64_t)(H.n >> wl) * (uint64_t)(H.n >> wl)) {
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
                const uint32_t item = (uint32_t)(word & 0x3ffffffu);
                const QuerySetup q = setup_query(qs[qi], pa.s2r, CUT ? pa.tau : 0.f, H.L, H.eps);
                descend<kModeValue, CUT, false>(H, q, lists, lev, lane == 0, item, true, 0, 0, pa.Q, acc, rec);
                const Fix192 d = wave_sum_fix(acc.d);
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
                    descend<kModeValue, CUT, true>(H, q, lists, q.l0, ok, item, false, pa.split_level,
                                                   (unsigned long long)query, pa.Q, acc, rec);
                else
                    descend<kModeValue, CUT, false>(H, q, lists, q.l0, ok, item, false, 0, 0, pa.Q, acc, rec);
            }
            const Fix192 d = wave_sum_fix(acc.d);
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

__global__ void k_persist_finalize(const QueueCtl* ctl, const Fix192* acc, const int* fexp)
{
    const long long nq = ctl->nq;
    float* out = ctl->out;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nq;
         i += (long long)gridDim.x * blockDim.x) {
        const int e = fexp[i];
        out[i] = e == 0x7fffffff ? __int_as_float(0x7fc00000) : fix_to_float(acc[i], e);
    }
}

// Launches cover at most kChunk queries (grid dimensions stay far below 2^32 work-items).
constexpr int64_t kChunk = (int64_t)1 << 24;

template <int MODE>
hipError_t launch_mode(const HierDev& H, const EvalArgs& a0, int algo, hipStream_t s)
{
    for (int64_t off = 0; off < a0.nq; off += kChunk) {
        EvalArgs a = a0;
        a.slot0 = off;
        a.slots = std::min<int64_t>(kChunk, a0.nq - off);
        if (algo == PNDF_ALGO_BRUTE) {
            const unsigned blocks = (unsigned)((a.slots + 3) / 4);
            hipLaunchKernelGGL(k_eval_brute<MODE>, dim3(blocks), dim3(256), 0, s, H, a);
        } else {
            const unsigned blocks = (unsigned)a.slots;
            const size_t lds = sizeof(uint32_t) * wave_lds_words(H.L);
            if (a.tau > 0.f)
                hipLaunchKernelGGL((k_eval_plain<MODE, true>), dim3(blocks), dim3(64), lds, s, H, a);
            else
                hipLaunchKernelGGL((k_eval_plain<MODE, false>), dim3(blocks), dim3(64), lds, s, H, a);
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ------------------------------------------------------------ query order
constexpr int kOrderBits = 6;  // 64 x 64 buckets

__global__ void k_order_zero(uint32_t* hist, int nb)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += gridDim.x * blockDim.x) hist[i] = 0;
}

__global__ void k_order_hist(const pndf_query* __restrict__ q, int64_t nq, int n, int bshift,
                             uint32_t* __restrict__ key, uint32_t* __restrict__ hist)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nq;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float x = q[i].x, y = q[i].y;
        uint32_t k = 0;
        if (fabsf(x) <= 16777216.0f && fabsf(y) <= 16777216.0f) {  // false for NaN
            const uint32_t cx = (uint32_t)((int)floorf(x) & (n - 1)) >> bshift;
            const uint32_t cy = (uint32_t)((int)floorf(y) & (n - 1)) >> bshift;
            k = morton(cx, cy);
        }
        key[i] = k;
        atomicAdd(&hist[k], 1u);
    }
}

// exclusive scan of nb <= 4096 counters by one workgroup of 1024 threads
__global__ __launch_bounds__(1024) void k_order_scan(uint32_t* hist, int nb)
{
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x, per = (nb + 1023) / 1024;
    uint32_t sum = 0;
    for (int k = 0; k < per; ++k) {
        const int i = t * per + k;
        if (i < nb) sum += hist[i];
    }
    part[t] = sum;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const uint32_t v = t >= o ? part[t - o] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = part[t] - sum;
    for (int k = 0; k < per; ++k) {
        const int i = t * per + k;
        if (i < nb) {
            const uint32_t c = hist[i];
            hist[i] = run;
            run += c;
        }
    }
}

__global__ void k_order_scatter(const uint32_t* __restrict__ key, int64_t nq, uint32_t* __restrict__ cursor,
                                uint32_t* __restrict__ order)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nq;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t pos = atomicAdd(&cursor[key[i]], 1u);
        order[pos] = (uint32_t)i;
    }
}

}  // namespace

hipError_t make_order(const HierDev& H, const pndf_query* q, int64_t nq, uint32_t** order, hipStream_t s)
{
    *order = nullptr;
    const int bits = H.logn < kOrderBits ? H.logn : kOrderBits;
    const int nb = 1 << (2 * bits);
    const int bshift = H.logn - bits;
    uint32_t* buf = nullptr;  // order[nq] | key[nq] | hist[nb]
    hipError_t e = hipMallocAsync((void**)&buf, sizeof(uint32_t) * (2 * (size_t)nq + nb), s);
    if (e != hipSuccess) return e;
    uint32_t* key = buf + nq;
    uint32_t* hist = key + nq;
    const unsigned g = (unsigned)std::min<int64_t>(2048, (nq + 255) / 256);
    hipLaunchKernelGGL(k_order_zero, dim3(16), dim3(256), 0, s, hist, nb);
    hipLaunchKernelGGL(k_order_hist, dim3(g), dim3(256), 0, s, q, nq, H.n, bshift, key, hist);
    hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(1024), 0, s, hist, nb);
    hipLaunchKernelGGL(k_order_scatter, dim3(g), dim3(256), 0, s, key, nq, hist, buf);
    e = hipGetLastError();
    if (e != hipSuccess) {
        (void)hipFreeAsync(buf, s);
        return e;
    }
    *order = buf;
    return hipSuccess;
}

void free_order(uint32_t* order, hipStream_t s)
{
    if (order) (void)hipFreeAsync(order, s);
}

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
