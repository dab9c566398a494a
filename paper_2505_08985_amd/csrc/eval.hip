// P-NDF evaluation kernels (Eq. ndf_eval).
//
// One wavefront owns one query at a time, so the order of every floating-point
// operation of a query depends on that query alone (results are bitwise the same
// in any batch).  Lanes cooperate on the query's candidates:
//   - brute force: lanes stride over the included cells;
//   - hierarchical: a breadth-limited, depth-first quad-tree descent.  Each level
//     has a list in LDS; the wave pops up to 64 nodes of the lowest non-empty level
//     (one per lane), tests the min-max box (and the cluster cut), and pushes the
//     surviving children with a ballot prefix.  Level-1 nodes push their four
//     cells into a leaf queue that is drained 64 cells at a time, so the
//     triangle tests always run with full waves.
// Triangle tests run in float32; a float32 hit is confirmed and its barycentrics
// recomputed in FP64 from the float32 vertices, so the recovered uv and the term
// are accurate even for sliver triangles.  Jacobians come from the mesh build
// (FP64, clamped), never from the hot loop.
#include "pndf_internal.h"

namespace pndf {

namespace {

enum { kModeValue = 0, kModeCount = 1, kModeRecord = 2 };

struct Acc {
    double d = 0.0;
    uint32_t nodes = 0, cells = 0, clusters = 0, hits = 0;
};

// Record one candidate hit (float32 test already passed): FP64 confirmation,
// barycentrics and term.  Returns the term, or a negative value if rejected.
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

// Accumulate this lane's hits; in record mode write them in deterministic order.
// Records never leave the query's own CSR slot [offsets[q], offsets[q + 1]).
template <int MODE>
__device__ __forceinline__ void take_hits(int nh, const uint64_t ids[2], const float terms[2],
                                          Acc& acc, uint64_t* rec_ids, float* rec_terms,
                                          uint64_t& rec_pos, uint64_t rec_end)
{
    for (int k = 0; k < nh; ++k) acc.d += (double)terms[k];
    acc.hits += nh;
    if (MODE == kModeRecord) {
        int total;
        const int pos = wave_prefix_small(nh, &total);
        for (int k = 0; k < nh; ++k) {
            const uint64_t at = rec_pos + pos + k;
            if (at < rec_end) {
                rec_ids[at] = ids[k];
                rec_terms[at] = terms[k];
            }
        }
        rec_pos += total;
    }
}

template <int MODE>
__device__ __forceinline__ void finish(const EvalArgs& a, int64_t qi, const Acc& acc)
{
    const double d = wave_sum_f64(acc.d);
    if (MODE == kModeCount) {
        const uint32_t nodes = wave_sum_u32(acc.nodes), cells = wave_sum_u32(acc.cells);
        const uint32_t clus = wave_sum_u32(acc.clusters), hits = wave_sum_u32(acc.hits);
        if (lane_id() == 0) {
            uint32_t* c = a.counts + 4 * qi;
            c[0] = nodes; c[1] = cells; c[2] = clus; c[3] = hits;
        }
    }
    if (lane_id() == 0) a.out[qi] = (float)d;
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
    const QuerySetup q = setup_query(a.q[qi], a.s2r, 0.f, H.L);
    if (!q.valid) { invalid<MODE>(a, qi); return; }
    const int n = H.n, msk = n - 1;
    const int spanx = q.cxhi - q.cxlo + 1, spany = q.cyhi - q.cylo + 1;
    const int nx = spanx >= n ? n : spanx, ny = spany >= n ? n : spany;
    const int total = nx * ny;  // <= 8192^2
    Acc acc;
    uint64_t rec_pos = MODE == kModeRecord ? a.offsets[qi] : 0;
    const uint64_t rec_end = MODE == kModeRecord ? a.offsets[qi + 1] : 0;
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
        take_hits<MODE>(nh, ids, terms, acc, a.ids, a.terms, rec_pos, rec_end);
    }
    finish<MODE>(a, qi, acc);
}

// ------------------------------------------------------------ hierarchical
// LDS per wave: L lists of kListCap node entries (levels 1..L) + the leaf queue.
template <int MODE, bool CUT>
__global__ __launch_bounds__(256) void k_eval_plain(HierDev H, EvalArgs a)
{
    extern __shared__ uint32_t lds[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t qi = (int64_t)blockIdx.x * 4 + wave;
    if (qi >= a.nq) return;
    uint32_t* lists = lds + (size_t)wave * (H.L * kListCap + kCellCap);
    uint32_t* cellq = lists + H.L * kListCap;
    const QuerySetup q = setup_query(a.q[qi], a.s2r, CUT ? a.tau : 0.f, H.L);
    if (!q.valid) { invalid<MODE>(a, qi); return; }
    const int logn = H.logn;
    const float4* __restrict__ boxes = CUT ? H.bbox_all : H.bbox;
    Acc acc;
    uint64_t rec_pos = MODE == kModeRecord ? a.offsets[qi] : 0;
    const uint64_t rec_end = MODE == kModeRecord ? a.offsets[qi + 1] : 0;

    // roots: the entry-level nodes overlapping the box (at most 4 per axis)
    uint32_t nonempty = 0;   // bit l: list of level l non-empty (wave-uniform)
    int cntv = 0;            // lane l holds the size of list l
    int ncell = 0;
    {
        const int l0 = q.l0, M = H.n >> l0, mm = M - 1;
        const int kx0 = q.cxlo >> l0, ky0 = q.cylo >> l0;
        const int nkx = min((q.cxhi >> l0) - kx0 + 1, M), nky = min((q.cyhi >> l0) - ky0 + 1, M);
        const int ra = lane & 3, rb = lane >> 2;
        const bool ok = lane < 16 && ra < nkx && rb < nky;
        const uint32_t item = (uint32_t)((kx0 + ra) & mm) | ((uint32_t)((ky0 + rb) & mm) << 16);
        const uint64_t bal = __ballot(ok);
        const int pos = __popcll(bal & ((1ull << lane) - 1ull));
        const int tot = __popcll(bal);
        if (l0 == 0) {
            if (ok) cellq[pos] = item;
            ncell = tot;
        } else {
            if (ok) lists[(l0 - 1) * kListCap + pos] = item;
            if (lane == l0) cntv = tot;
            if (tot) nonempty |= 1u << l0;
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
            take_hits<MODE>(nh, ids, terms, acc, a.ids, a.terms, rec_pos, rec_end);
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
        uint64_t ids[2];
        float terms[2];
        if (lane < k) {
            const uint32_t item = lists[(l - 1) * kListCap + base + lane];
            const int I = (int)(item & 0xffffu), J = (int)(item >> 16);
            const int64_t idx = H.off[l] + (int64_t)J * (H.n >> l) + I;
            const float4 bb = boxes[idx];
            acc.nodes += 1;
            if (q.hx >= bb.x && q.hy >= bb.y && q.hx <= bb.z && q.hy <= bb.w) {
                if (CUT && l <= q.l0 && H.clu_e[idx] <= q.t) {
                    nh = test_cluster(H, q, l, I, J, idx, ids, terms);
                    acc.clusters += 1;
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
        if (CUT) take_hits<MODE>(nh, ids, terms, acc, a.ids, a.terms, rec_pos, rec_end);
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
    finish<MODE>(a, qi, acc);
}

template <int MODE>
hipError_t launch_mode(const HierDev& H, const EvalArgs& a, int algo, hipStream_t s)
{
    const unsigned blocks = (unsigned)((a.nq + 3) / 4);
    if (algo == PNDF_ALGO_BRUTE) {
        hipLaunchKernelGGL(k_eval_brute<MODE>, dim3(blocks), dim3(256), 0, s, H, a);
    } else {
        const size_t lds = sizeof(uint32_t) * 4 * ((size_t)H.L * kListCap + kCellCap);
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

}  // namespace pndf
