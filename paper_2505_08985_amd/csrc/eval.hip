// P-NDF evaluation kernels (Eq. ndf_eval).
//
// A wavefront owns a query (or a subtree of one) at a time; its 64 lanes
// cooperate on the candidates:
//   - brute force: lanes stride over the included cells;
//   - hierarchical: a breadth-limited, depth-first quad-tree descent.  Each level
//     has a list in LDS; the wave pops up to 64 nodes of the lowest non-empty level
//     (one per lane), tests the min-max box (and the cluster cut), and pushes the
//     surviving children with a ballot prefix.  A level-1 node tests the triangles
//     of its 2 x 2 cells from its leaf record.
//   - persistent: a fixed grid of workers takes chunks of queries (each XCD from
//     its own share of the spatial order); once the queries run out, idle workers
//     ask the busy ones for part of their pending subtrees through a global task
//     queue.
// Triangle tests run in float32 and only queue the hits; a queued hit is confirmed
// and its barycentrics recomputed in FP64 from the float32 vertices 64 at a time
// (one per lane), so the recovered uv and the term are accurate even for sliver
// triangles while the traversal itself stays small.  Jacobians come from the mesh build
// (FP64, clamped), never from the hot loop.  Terms are summed exactly (192-bit
// fixed point at a per-query binary point), so D does not depend on the order in
// which hits are found: all algorithms, batch compositions and work splits give
// the same bits.
#include <algorithm>
#include <mutex>

#include "pndf_internal.h"

namespace pndf {

namespace {

enum { kModeValue = 0, kModeCount = 1, kModeRecord = 2 };

struct Acc {
    Fix192 d{0, 0, 0};
    uint32_t nodes = 0, cells = 0, clusters = 0, hits = 0;
    bool donated = false;  // part of the work was handed to other waves (wave-uniform)
};

struct Rec {  // hit-record cursor (record mode)
    uint64_t* ids;
    float* terms;
    uint64_t pos, end;
};

// FP64 confirmation of a float32 hit, barycentrics and term; < 0 if rejected.  The
// offsets v - h of float32 values are exact in FP64 and the cyclic edge functions
// e_k (as in the float32 test) give the barycentrics l_k = e_k / S, S = e0 + e1 + e2
// (twice the signed area, never 0: clamped triangles are replaced).  One division,
// R = 1 / (S det), serves both quotients: 1 / S = det R and 1 / det = S R.
template <int KER>
__device__ __forceinline__ double confirm_and_term(const QuerySetup& q, const double v[6], int I,
                                                   int J, int lev, int half, float det_used,
                                                   int logn)
{
    const double hx = (double)q.hx, hy = (double)q.hy;
    const double ax = v[0] - hx, ay = v[1] - hy, bx = v[2] - hx, by = v[3] - hy;
    const double cx = v[4] - hx, cy = v[5] - hy;
    const double e0 = bx * cy - by * cx, e1 = cx * ay - cy * ax, e2 = ax * by - ay * bx;
    if (!((e0 >= 0.0 && e1 >= 0.0 && e2 >= 0.0) || (e0 <= 0.0 && e1 <= 0.0 && e2 <= 0.0))) return -1.0;
    const double S = e0 + e1 + e2, dj = (double)det_used;
    const double R = 1.0 / (S * dj);
    const double rs = dj * R;
    return hit_weight<KER>(q, I, J, lev, half, e1 * rs, e2 * rs, logn) * (S * R);
}

// Per-lane hit sink of one hit-processing round: value/count modes add the term to
// the exact accumulator at once; record mode also keeps (id, term) until the wave
// writes its records in lane order.
template <int MODE>
struct HitSink {
    uint64_t id = 0;
    float term = 0.f;
    int n = 0;
    __device__ __forceinline__ void put(const QuerySetup& q, Acc& acc, uint64_t tid, double t)
    {
        fix_add_term(acc.d, t, q.fexp);
        acc.hits += 1;
        if (MODE == kModeRecord) {
            id = tid;
            term = (float)t;
        }
        n = 1;
    }
};

// Write the wave's records in lane order, never leaving the query's own CSR slot
// [pos, end).  Every lane must call it.
template <int MODE>
__device__ __forceinline__ void flush_records(HitSink<MODE>& hs, Rec& rec)
{
    if (MODE == kModeRecord) {
        const uint64_t b = __ballot(hs.n);
        const uint64_t at = rec.pos + __popcll(b & ((1ull << lane_id()) - 1ull));
        if (hs.n && at < rec.end) {
            rec.ids[at] = hs.id;
            rec.terms[at] = hs.term;
        }
        rec.pos += __popcll(b);
    }
    hs.n = 0;
}

// Exclusive prefix over the wave of a per-lane count in [0, 15], and the total.
__device__ __forceinline__ int wave_prefix16(int c, int* total)
{
    const uint64_t b0 = __ballot(c & 1), b1 = __ballot(c & 2), b2 = __ballot(c & 4), b3 = __ballot(c & 8);
    const uint64_t lt = (1ull << lane_id()) - 1ull;
    *total = __popcll(b0) + 2 * __popcll(b1) + 4 * __popcll(b2) + 8 * __popcll(b3);
    return __popcll(b0 & lt) + 2 * __popcll(b1 & lt) + 4 * __popcll(b2 & lt) + 8 * __popcll(b3 & lt);
}

// ---- float32 triangle tests.  They only decide which triangles are hit; every hit
// becomes a 32-bit entry of the wave's hit queue, and the FP64 confirmation,
// barycentrics and term run later with one hit per lane (hit_entry), so the
// traversal keeps few registers and the FP64 work runs with full waves.
//   leaf cell    (0 << 30) | m << 3 | c4 << 1 | half   cell c4 = 2 dj + di of level-1 record m
//   plane cell   (1 << 30) | j << 14 | i << 1 | half   texel cell (i, j), i, j < 8192
//   cluster      (2 << 30) | lev << 25 | m << 1 | half   node m (Morton) of level lev >= 1
// A lane's hits are a bit mask over the low bits of its entry code.
constexpr uint32_t kHitPlane = 1u << 30, kHitCluster = 2u << 30;

// Traversal list items are Morton codes (at most 24 bits); the top bit marks a node
// whose region lies wholly inside the query's box, so that its descendants skip the
// spatial tests.  (With the cluster cut, a node's residual is compared with the
// query's threshold when its parent expands -- the four children's residuals are
// read with their boxes -- and a node under the cut goes to the cluster queue
// instead of a list.  Bit 30 then marks a node whose four children are all under
// the cut: the largest of their residuals, read with the node's own, is within the
// threshold, so its expansion reads only the children's boxes.)
constexpr uint32_t kInside = 1u << 31;
constexpr uint32_t kAllCut = 1u << 30;
constexpr uint32_t kCodeMask = (1u << 30) - 1u;

// Inclusive same-sign test of a triangle's three edge values: h inside or on it.
__device__ __forceinline__ uint32_t same_sign3(float a, float b, float c)
{
    return (uint32_t)(fminf(fminf(a, b), c) >= 0.f) | (uint32_t)(fmaxf(fmaxf(a, b), c) <= 0.f);
}

// A clamped half is replaced by its equilateral triangle (Eq. debias), the same for
// both halves of a cell (centred on the shared diagonal's midpoint): set the bits
// of the clamped halves (dg) of a cell's 2-bit mask from that triangle's test.
__device__ __forceinline__ uint32_t patch_clamped(const QuerySetup& q, float rho, float2 n1, float2 n2,
                                                  uint32_t dg, uint32_t m2)
{
    float v[6];
    eqtri_f32(0.5f * (n1.x + n2.x), 0.5f * (n1.y + n2.y), rho, v);
    const uint32_t e = (uint32_t)tri_hit_f32(v, q.hx, q.hy);
    if (dg & 1u) m2 = (m2 & ~1u) | e;
    if (dg & 2u) m2 = (m2 & ~2u) | (e << 1);
    return m2;
}

// The two triangles of a cell from its four corner normals and clamp bits: bit 0
// lower (n0, n1, n2), bit 1 upper (n3, n2, n1).  Every edge value is computed in
// one canonical direction (bottom and top edges left to right, left and right
// edges upwards, the diagonal from n1 to n2) and only its sign is flipped where a
// triangle runs along it the other way, so a cell tested alone and the same cell
// tested within its 2 x 2 block (which shares edges between cells) decide alike.
__device__ __forceinline__ uint32_t cell_mask(const QuerySetup& q, float rho, float2 n0, float2 n1, float2 n2,
                                              float2 n3, uint32_t dg)
{
    const float q0x = n0.x - q.hx, q0y = n0.y - q.hy, q1x = n1.x - q.hx, q1y = n1.y - q.hy;
    const float q2x = n2.x - q.hx, q2y = n2.y - q.hy, q3x = n3.x - q.hx, q3y = n3.y - q.hy;
    const float h01 = cross2(q0x, q0y, q1x, q1y), h23 = cross2(q2x, q2y, q3x, q3y);
    const float v02 = cross2(q0x, q0y, q2x, q2y), v13 = cross2(q1x, q1y, q3x, q3y);
    const float d12 = cross2(q1x, q1y, q2x, q2y);
    // lower: (d12, -v02, h01); upper: (-d12, v13, -h23), negated as a whole
    uint32_t m = same_sign3(d12, -v02, h01) | (same_sign3(d12, -v13, h23) << 1);
    if (dg & 3u) m = patch_clamped(q, rho, n1, n2, dg, m);
    return m;
}

// A texel cell tested from the padded normal plane (brute force, tiny footprints).
__device__ __forceinline__ uint32_t plane_cell_mask(const HierDev& H, const QuerySetup& q, int i, int j,
                                                    Acc& acc)
{
    const int w = H.n + 1;
    const float2* p = H.nrm + (int64_t)j * w + i;
    acc.cells += 1;
    return cell_mask(q, H.rho, p[0], p[1], p[w], p[w + 1], H.deg[(int64_t)j * H.n + i]);
}

// Along one axis, the level-c node columns (side 2^c; M = N >> c of them on the
// torus) that meet the unrolled cell range [clo, chi] form one cyclic run of n
// columns starting at a, and those with an image wholly inside the range a run of
// ni starting at ai (n or ni = M: every column).  Column X belongs to a run iff
// ((X - a) mod M) < n.  The runs depend only on the query and the level
// (wave-uniform), so each node's spatial tests are a subtraction, a mask and a
// compare per axis and child.
struct AxisRuns {
    int a, n, ai, ni;
};

__device__ __forceinline__ AxisRuns axis_runs(int clo, int chi, int c, int M)
{
    AxisRuns r;
    r.a = clo >> c;
    r.n = min((chi >> c) - r.a + 1, M);
    r.ai = -((-clo) >> c);
    r.ni = max(0, min(((chi + 1) >> c) - r.ai, M));
    return r;
}

// Bits 0 / 1: the columns 2X and 2X + 1 of the level below X (mask mk = M - 1
// there) in the run (a, n).
__device__ __forceinline__ uint32_t pair_in_run(int X, int a, int n, int mk)
{
    const int d = 2 * X - a;
    return (uint32_t)((d & mk) < n) | ((uint32_t)(((d + 1) & mk) < n) << 1);
}

// Bits c = 2 dj + di of the 2 x 2 block from its column bits x and row bits y.
__device__ __forceinline__ uint32_t quad_bits(uint32_t x, uint32_t y)
{
    return (x & (y & 1u ? 3u : 0u)) | ((x & (y & 2u ? 3u : 0u)) << 2);
}

// The 2 x 2 cells of level-1 node m (its leaf record), those overlapping the box
// (all four when the node lies inside it): bit 2 c4 + half for cell c4 = 2 dj + di.
// The block's nine corners give 16 distinct edges (6 horizontal, 6 vertical and 4
// diagonals), each computed once in its canonical direction as in cell_mask, so
// the bits equal cell_mask's for each cell.  rx, ry: the level-0 runs.
__device__ __forceinline__ uint32_t leaf_quad_mask(const HierDev& H, const QuerySetup& q, uint32_t m, bool inside,
                                                   const AxisRuns& rx, const AxisRuns& ry, Acc& acc)
{
    const float4* r = reinterpret_cast<const float4*>(H.quad + m);
    const float4 a = r[0], b = r[1], c = r[2], d = r[3], e = r[4];
    const float tx[9] = {a.x, a.z, b.x, b.z, c.x, c.z, d.x, d.z, e.x};
    const float ty[9] = {a.y, a.w, b.y, b.w, c.y, c.w, d.y, d.w, e.y};
    const uint32_t dg4 = __float_as_uint(e.z);
    uint32_t ov = 0xfu;
    if (!inside) {
        const int mk = H.n - 1;
        ov = quad_bits(pair_in_run((int)morton_compact(m), rx.a, rx.n, mk),
                       pair_in_run((int)morton_compact(m >> 1), ry.a, ry.n, mk));
    }
    acc.cells += (uint32_t)__popc(ov);
    // row by row (rows of corners 0-2 bottom to top), so that only two rows of
    // offsets and their edges are live at a time
    uint32_t mask = 0;
    float bx[3], by[3], bh[2];  // the lower row's offsets and its horizontal edges
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        bx[c] = tx[c] - q.hx;
        by[c] = ty[c] - q.hy;
    }
    bh[0] = cross2(bx[0], by[0], bx[1], by[1]);
    bh[1] = cross2(bx[1], by[1], bx[2], by[2]);
#pragma unroll
    for (int dj = 0; dj < 2; ++dj) {
        float ux[3], uy[3], uh[2], vt[3];  // the upper row, its horizontal edges, the vertical edges
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            ux[c] = tx[3 * dj + 3 + c] - q.hx;
            uy[c] = ty[3 * dj + 3 + c] - q.hy;
            vt[c] = cross2(bx[c], by[c], ux[c], uy[c]);
        }
        uh[0] = cross2(ux[0], uy[0], ux[1], uy[1]);
        uh[1] = cross2(ux[1], uy[1], ux[2], uy[2]);
#pragma unroll
        for (int di = 0; di < 2; ++di) {
            const float d12 = cross2(bx[di + 1], by[di + 1], ux[di], uy[di]);
            mask |= (same_sign3(d12, -vt[di], bh[di]) | (same_sign3(d12, -vt[di + 1], uh[di]) << 1))
                    << (2 * (2 * dj + di));
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            bx[c] = ux[c];
            by[c] = uy[c];
        }
        bh[0] = uh[0];
        bh[1] = uh[1];
    }
    if (dg4 & 0x03030303u) {
        // rare: a clamped triangle (its cell's replacement) is tested on its own; the
        // corners are read again (cached) rather than kept live through the tests
        const QuadRec* rec = H.quad + m;
        for (int c4 = 0; c4 < 4; ++c4) {
            const uint32_t dg = (dg4 >> (8 * c4)) & 3u;
            if (dg) {
                const int k = 3 * (c4 >> 1) + (c4 & 1);
                const uint32_t m2 = patch_clamped(q, H.rho, rec->t[k + 1], rec->t[k + 3], dg, (mask >> (2 * c4)) & 3u);
                mask = (mask & ~(3u << (2 * c4))) | (m2 << (2 * c4));
            }
        }
    }
    const uint32_t ov2 = (ov & 1u) * 3u | ((ov >> 1) & 1u) * 12u | ((ov >> 2) & 1u) * 48u | ((ov >> 3) & 1u) * 192u;
    return mask & ov2;
}

// The two cluster triangles of node idx (level lev): bit half.
__device__ __forceinline__ uint32_t cluster_mask(const HierDev& H, const QuerySetup& q, int lev, int64_t idx,
                                                 Acc& acc)
{
    const float4 a = H.clu_t[2 * idx], b = H.clu_t[2 * idx + 1];
    const uint32_t dg = clamp_bits(a, b);
    const float rho = H.rho * (float)(1 << lev);
    const float cx = 0.5f * (a.z + b.x), cy = 0.5f * (a.w + b.y);
    float vl[6], vu[6];
    if (dg & 1) eqtri_f32(cx, cy, rho, vl);
    else { vl[0] = a.x; vl[1] = a.y; vl[2] = a.z; vl[3] = a.w; vl[4] = b.x; vl[5] = b.y; }
    if (dg & 2) eqtri_f32(cx, cy, rho, vu);
    else { vu[0] = b.z; vu[1] = b.w; vu[2] = b.x; vu[3] = b.y; vu[4] = a.z; vu[5] = a.w; }
    acc.clusters += 1;
    return (uint32_t)tri_hit_f32(vl, q.hx, q.hy) | ((uint32_t)tri_hit_f32(vu, q.hx, q.hy) << 1);
}

// ---- FP64 stage: one queued hit.
template <int MODE, int KER>
__device__ __forceinline__ void hit_entry(const HierDev& H, const QuerySetup& q, uint32_t e, Acc& acc,
                                          HitSink<MODE>& hs)
{
    const int half = (int)(e & 1u);
    const uint32_t kind = e >> 30;
    double v[6];
    float det_used;
    int I, J, lev;
    if (kind == (kHitCluster >> 30)) {
        lev = (int)((e >> 25) & 0xfu);
        const uint32_t m = (e >> 1) & 0xffffffu;
        const int64_t idx = level_offset(H.logn, lev) + m;
        I = (int)morton_compact(m);
        J = (int)morton_compact(m >> 1);
        const float4 a = H.clu_t[2 * idx], b = H.clu_t[2 * idx + 1];
        const float2 dd = H.clu_det[idx];
        det_used = half ? dd.y : dd.x;
        if (clamp_bits(a, b) & (1u << half)) {
            eqtri_f64(0.5 * ((double)a.z + (double)b.x), 0.5 * ((double)a.w + (double)b.y),
                      (double)(H.rho * (float)(1 << lev)), v);
        } else if (half == 0) {
            v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = b.x; v[5] = b.y;
        } else {
            v[0] = b.z; v[1] = b.w; v[2] = b.x; v[3] = b.y; v[4] = a.z; v[5] = a.w;
        }
    } else {
        float2 n0, n1, n2, n3;
        uint32_t dg;
        lev = 0;
        if (kind == 0) {
            const uint32_t m = (e >> 3) & 0xffffffu;
            const int c4 = (int)((e >> 1) & 3u), di = c4 & 1, dj = c4 >> 1;
            const QuadRec* r = H.quad + m;
            const int k = 3 * dj + di;
            n0 = r->t[k]; n1 = r->t[k + 1]; n2 = r->t[k + 3]; n3 = r->t[k + 4];
            dg = r->deg[c4];
            I = 2 * (int)morton_compact(m) + di;
            J = 2 * (int)morton_compact(m >> 1) + dj;
        } else {
            I = (int)((e >> 1) & 0x1fffu);
            J = (int)((e >> 14) & 0x1fffu);
            const int w = H.n + 1;
            const float2* p = H.nrm + (int64_t)J * w + I;
            n0 = p[0]; n1 = p[1]; n2 = p[w]; n3 = p[w + 1];
            dg = H.deg[(int64_t)J * H.n + I];
        }
        const float2 dd = H.det[(int64_t)J * H.n + I];
        det_used = half ? dd.y : dd.x;
        if (dg & (1u << half)) {
            eqtri_f64(0.5 * ((double)n1.x + (double)n2.x), 0.5 * ((double)n1.y + (double)n2.y), (double)H.rho, v);
        } else if (half == 0) {
            v[0] = n0.x; v[1] = n0.y; v[2] = n1.x; v[3] = n1.y; v[4] = n2.x; v[5] = n2.y;
        } else {
            v[0] = n3.x; v[1] = n3.y; v[2] = n2.x; v[3] = n2.y; v[4] = n1.x; v[5] = n1.y;
        }
    }
    const double t = confirm_and_term<KER>(q, v, I, J, lev, half, det_used, H.logn);
    if (t >= 0.0) hs.put(q, acc, tri_id(lev, I, J, half), t);
}

// The wave's hit queue: hq (kHitCap entries in LDS), hn entries (wave-uniform).
// Each lane's float32 hits wait in a bit mask (entry ebase | bit) until they are
// queued; the traversal loops run a round of the FP64 stage (hit_round, one call
// site per kernel so it is inlined once) whenever 64 hits are queued and at the end.
template <int MODE, int KER>
__device__ __forceinline__ void hit_round(const HierDev& H, const QuerySetup& q, const uint32_t* src, int cnt,
                                          Acc& acc, Rec& rec)
{
    HitSink<MODE> hs;
    if (lane_id() < cnt) hit_entry<MODE, KER>(H, q, src[lane_id()], acc, hs);
    flush_records<MODE>(hs, rec);
    wave_sync();
}

// Move the lanes' pending hits into the queue (as many as fit, in lane order).
__device__ __forceinline__ void queue_hits(uint32_t* hq, int& hn, uint32_t& pend, uint32_t ebase)
{
    if (__ballot(pend != 0u) == 0ull) return;
    int total;
    const int pos = wave_prefix16(__popc(pend), &total);
    if (total == 0) return;
    int at = hn + pos;
    while (pend && at < kHitCap) {
        hq[at++] = ebase | (uint32_t)(__ffs(pend) - 1);
        pend &= pend - 1u;
    }
    hn = min(hn + total, kHitCap);
    wave_sync();
}

// Is the query normal inside a box stored as order keys (half_key) of its corners,
// (min x | min y << 16, max x | max y << 16)?  The query's key is that of h rounded
// to the nearest half: rounding is monotone, so a box that contains h contains it.
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ bool key_in_box(uint32_t hk, uint32_t lo, uint32_t hi)
{
    const u16x2 h = __builtin_bit_cast(u16x2, hk);
    const u16x2 a = __builtin_elementwise_max(h, __builtin_bit_cast(u16x2, lo));
    const u16x2 c = __builtin_elementwise_min(h, __builtin_bit_cast(u16x2, hi));
    return (__builtin_bit_cast(uint32_t, a) == hk) & (__builtin_bit_cast(uint32_t, c) == hk);
}

// Nodes under the cut from this level up are tested against the box of their own
// cluster triangles before their cluster test.  Below it that box is about as wide
// as the subtree's (about 60 % of level-1 cluster nodes whose subtree box holds h
// also hold it in their own box, under 25 % from level 3) and the extra 32 B read
// does not pay: from level 1 the scratched 4096^2 map took 7 % longer than from 2.
constexpr int kOwnBoxLevel = 2;

// Cluster queue entry: level (4 bits) << 24 | Morton code of the node (< 2^24).
constexpr int kCluShift = 24;

// A wavefront's node lists in LDS (see list_words): 32-bit items for the levels below
// S, 16-bit items (code in bits 0..13, the flags kAllCut and kInside in bits 14, 15)
// from S up (only with the cut).  The level is wave-uniform wherever a list is read
// or written.
template <bool CUT>
struct NodeLists {
    uint32_t* w;
    uint16_t* h;
    int S;
    __device__ NodeLists(uint32_t* lds, int L)
        : w(lds), h(reinterpret_cast<uint16_t*>(lds + (size_t)(short_list_level(L, CUT) - 1) * kListCap)),
          S(short_list_level(L, CUT))
    {
    }
    __device__ __forceinline__ uint32_t get(int lev, int i) const
    {
        if (!CUT || lev < S) return w[(lev - 1) * kListCap + i];
        const uint32_t v = h[(lev - S) * kListCap + i];
        return (v & 0x3fffu) | ((v & 0xc000u) << 16);
    }
    __device__ __forceinline__ void put(int lev, int i, uint32_t item) const
    {
        if (!CUT || lev < S)
            w[(lev - 1) * kListCap + i] = item;
        else
            h[(lev - S) * kListCap + i] = (uint16_t)((item & 0x3fffu) | ((item >> 16) & 0xc000u));
    }
};

// The shared descent.  List items are nodes (Morton codes) whose box contains h,
// whose region meets the support box and which are not under the cluster cut.  A
// lane takes one item: a level-1 node tests its 2 x 2 cells from its leaf record;
// any other node loads its (up to) four overlapping children's boxes together and
// keeps those that contain h: children under the cut go to the wave's cluster
// queue if the box of their own two cluster triangles contains h, the others to
// the list of the level below.  The cluster queue is taken 64
// nodes at a time, one per lane, each testing its node's two cluster triangles, so
// the cluster tests and the descent never share a step (a step runs every branch
// any lane takes).  Roots: every lane with root_ok holds a root of level
// root_level (level 0: texel cell packed i | j << 16; else a Morton code),
// box-tested here unless roots_tested.  With SPAWN (persistent workers), while
// some worker of the plan is idle the wave gives away part of its pending work
// before each step: half of the items of its highest non-empty list (the largest
// subtrees it holds), if that level is at least split_level, become tasks of the
// global queue.  A full queue simply leaves them here.
template <int MODE, bool CUT, bool SPAWN, int KER>
__device__ void descend(const HierDev& H, const QuerySetup& q, uint32_t* lists, int root_level,
                        bool root_ok, uint32_t root_item, bool roots_tested, int split_level,
                        unsigned long long qidx, const TaskQueue& Q, Acc& acc, Rec& rec)
{
    static_assert(!SPAWN || MODE == kModeValue, "donation is only used by value-mode workers");
    const int lane = threadIdx.x & 63;
    const NodeLists<CUT> nl(lists, H.L);
    uint32_t* hq = lists + list_words(H.L, CUT);  // hit queue
    uint32_t* cq = hq + kHitCap;            // cluster queue (CUT)
    int hn = 0;                             // queued hits (wave-uniform)
    int cn = 0;                             // queued cluster nodes (wave-uniform)
    uint32_t pend = 0, ebase = 0;           // this lane's float32 hits not yet queued
    uint32_t nonempty = 0;   // bit l: list of level l non-empty (wave-uniform)
    int cntv = 0;            // lane l holds the size of list l
    const AxisRuns rx0 = axis_runs(q.cxlo, q.cxhi, 0, H.n), ry0 = axis_runs(q.cylo, q.cyhi, 0, H.n);
    if (root_level == 0) {
        const int i = (int)(root_item & 0xffffu), j = (int)(root_item >> 16);
        if (root_ok) {
            pend = plane_cell_mask(H, q, i, j, acc);
            ebase = kHitPlane | ((uint32_t)j << 14) | ((uint32_t)i << 1);
        }
    } else {
        bool ok = root_ok;
        const uint32_t m = root_item & kCodeMask;
        const int64_t idx = level_offset(H.logn, root_level) + m;
        if (ok && !roots_tested) {
            // the node's box as order keys: of the map triangles, or under the cut of the
            // map and cluster triangles (from its group record)
            acc.nodes += 1;
            const uint2 b = CUT ? reinterpret_cast<const uint2*>(H.grp + (idx & ~(int64_t)3))[idx & 3] : H.bbox_k[idx];
            ok = key_in_box(q.hkey, b.x, b.y);
        }
        bool cut = false;
        // (e^l from the node's group record, the one the root's key test reads; taking it
        // there rather than from the per-node e^l array keeps one array pointer out of the
        // kernel, whose scalar registers are at their limit)
        if (CUT && ok &&
            __uint_as_float(reinterpret_cast<const uint32_t*>(H.grp)[4 * (idx & ~(int64_t)3) + 8 + (idx & 3)]) <= q.t) {
            cut = true;
            if (root_level >= kOwnBoxLevel) {
                // under the cut only the node's own two cluster triangles are tested:
                // their box (inside the subtree's) decides
                const uint2 c = H.bbox_c[idx];
                ok = cut = key_in_box(q.hkey, c.x, c.y);
            }
        }
        const uint64_t bl = __ballot(ok && !cut);
        if (ok && !cut) {
            uint32_t item = root_item;
            if (CUT && root_level >= 2 &&
                __uint_as_float(reinterpret_cast<const uint32_t*>(H.grp)[4 * (idx & ~(int64_t)3) + 12 + (idx & 3)]) <= q.t)
                item |= kAllCut;
            nl.put(root_level, __popcll(bl & ((1ull << lane) - 1ull)), item);
        }
        if (CUT) {
            const uint64_t bc = __ballot(cut);
            if (cut) cq[__popcll(bc & ((1ull << lane) - 1ull))] = ((uint32_t)root_level << kCluShift) | m;
            cn = __popcll(bc);
        }
        const int tot = __popcll(bl);
        if (lane == root_level) cntv = tot;
        if (tot) nonempty |= 1u << root_level;
        wave_sync();
    }
    // SPAWN: the starving flag, loaded at the start of a step (its latency hides behind
    // the step's own loads) and acted on before the next one
    unsigned hungry = 0;
    while (true) {
        queue_hits(hq, hn, pend, ebase);
        if (hn >= 64 || (hn > 0 && !nonempty && cn == 0)) {
            // (lanes still holding hits imply a full queue, so they get here too)
            const int c = min(hn, 64);
            hn -= c;
            hit_round<MODE, KER>(H, q, hq + hn, c, acc, rec);
            continue;
        }
        if (CUT && (cn >= 64 || (cn > 0 && !nonempty))) {
            // a round of cluster nodes, one per lane (every lane's hits are queued)
            const int c = min(cn, 64);
            cn -= c;
            if (lane < c) {
                const uint32_t e = cq[cn + lane];
                const int lev = (int)(e >> kCluShift);
                const uint32_t m = e & ((1u << kCluShift) - 1u);
                pend = cluster_mask(H, q, lev, level_offset(H.logn, lev) + m, acc);
                ebase = kHitCluster | ((uint32_t)lev << 25) | (m << 1);
            }
            wave_sync();
            continue;
        }
        if (!nonempty) break;
        if (SPAWN && hungry) {
            // some workers wait for tasks: give away up to half of the highest list,
            // at most one node per waiting worker
            const int lh = 31 - __builtin_clz(nonempty);
            if (lh >= split_level) {
                const int ch = __builtin_amdgcn_readlane(cntv, lh);
                // keep at least one item: a lone top item is given only when lower lists hold work
                int d = min(ch >= 2 ? ch / 2 : ((nonempty & ~(1u << lh)) ? 1 : 0), 64);
                unsigned long long slot = 0;
                if (lane == 0 && d > 0) {
                    const long long waiting = (long long)__hip_atomic_load(&Q.ctl->head, __ATOMIC_RELAXED,
                                                                           __HIP_MEMORY_SCOPE_AGENT) -
                                              (long long)__hip_atomic_load(&Q.ctl->tail, __ATOMIC_RELAXED,
                                                                           __HIP_MEMORY_SCOPE_AGENT);
                    d = (int)min((long long)d, max(0ll, waiting));
                    if (d > 0) {
                        slot = __hip_atomic_fetch_add(&Q.ctl->tail, (unsigned long long)d, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
                        // slots past the capacity are not used: those nodes stay here
                        const long long room = (long long)Q.capacity - (long long)slot;
                        const int dd = (int)max(0ll, min((long long)d, room));
                        if (dd < d) atomicAdd(&Q.ctl->refused, (unsigned long long)(d - dd));
                        d = dd;
                        if (d > 0) {
                            // counted before they become visible
                            __hip_atomic_fetch_add(&Q.ctl->outstanding, (unsigned long long)d, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
                            atomicAdd(&Q.ctl->spawned, (unsigned long long)d);
                        }
                    }
                    if (d == 0)
                        __hip_atomic_store(&Q.ctl->starving[blockIdx.x & (kStarveCopies - 1)].v, 0u,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                d = __builtin_amdgcn_readfirstlane(d);
                slot = uniform_u64(slot);
                if (d > 0) {
                    if (lane < d) {
                        const uint32_t mm = nl.get(lh, ch - 1 - lane) & kCodeMask;  // the top d items
                        Q.tasks[slot + lane] = (qidx << 32) | ((unsigned long long)lh << 26) | (unsigned long long)mm;
                        // the release store orders the task word before its flag
                        __hip_atomic_store(&Q.flags[slot + lane], Q.ctl->epoch, __ATOMIC_RELEASE,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    }
                    if (lane == lh) cntv = ch - d;
                    if (ch == d) nonempty &= ~(1u << lh);
                    acc.donated = true;
                    wave_sync();
                    if (!nonempty) continue;  // (cannot happen: one item is always kept)
                }
            }
        }
        int l = __builtin_ctz(nonempty);
        int cnt = __builtin_amdgcn_readlane(cntv, l);
        if (cnt < 32) {
            // the lowest list would fill less than half a wave: expand the next higher
            // level first, so the lower levels run with fuller waves (what does not fit
            // is re-queued).  Measured on powerlaw2048: thresholds 8 to 32 all take
            // 3 % less time than deferring every list shorter than a full wave.
            const uint32_t higher = nonempty & ~((2u << l) - 1u);
            if (higher) {
                l = __builtin_ctz(higher);
                cnt = __builtin_amdgcn_readlane(cntv, l);
            }
        }
        const int k = min(cnt, 64), base = cnt - k;
        unsigned hv = 0;
        if (SPAWN && lane == 0 && 31 - __builtin_clz(nonempty) >= split_level)
            hv = __hip_atomic_load(&Q.ctl->starving[blockIdx.x & (kStarveCopies - 1)].v, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        if (lane == l) cntv = base;
        if (base == 0) nonempty &= ~(1u << l);
        uint32_t chm = 0;     // children whose boxes contain h (bit c: child 4m + c)
        uint32_t cin = 0;     // children wholly inside the box (bit c)
        uint32_t m4 = 0;      // 4m: the first child's code
        uint32_t tested = 0;  // child boxes read by this lane
        uint32_t cut4 = 0;    // children under the cut (bit c)
        uint32_t all4 = 0;    // children whose own children are all under the cut (bit c)
        uint32_t entry = 0;   // the lane's list item (Morton code | kInside)
        if (lane < k) {
            entry = nl.get(l, base + lane);
            const uint32_t m = entry & kCodeMask;
            const bool inside = (entry & kInside) != 0u;
            if (l == 1) {
                pend = leaf_quad_mask(H, q, m, inside, rx0, ry0, acc);
                ebase = m << 3;
            } else {
                // the four child boxes are one Morton segment (32 B of keys): loaded
                // whole, children outside the support masked afterwards.  With the cut,
                // the group record (64 B: their keys, residuals and their children's
                // largest residuals), or for a node whose children are all under the
                // cut only the boxes they are tested against.
                const int64_t c0 = level_offset(H.logn, l - 1) + 4 * (int64_t)m;
                // every load is issued before any is used (one memory round trip per
                // expansion): the boxes, then with the cut the residual words
                const bool allc = CUT && (entry & kAllCut) != 0u;
                const uint4* kp = !CUT ? reinterpret_cast<const uint4*>(H.bbox_k + c0)
                                  : (allc && l - 1 >= kOwnBoxLevel) ? reinterpret_cast<const uint4*>(H.bbox_c + c0)
                                                                    : H.grp + c0;
                const uint4 b01 = kp[0], b23 = kp[1];
                uint4 u01 = make_uint4(0u, 0xffffffffu, 0u, 0xffffffffu), u23 = u01;
                if (CUT) {
                    uint4 w2 = make_uint4(0u, 0u, 0u, 0u), w3 = w2;
                    if (!allc) {
                        w2 = H.grp[c0 + 2];
                        w3 = H.grp[c0 + 3];
                        if (l - 1 >= 3) {
                            // the children's union boxes, for those whose own children
                            // all turn out to be under the cut
                            const uint4* up = reinterpret_cast<const uint4*>(H.bbox_u + c0);
                            u01 = up[0];
                            u23 = up[1];
                        }
                    }
                    const float4 ce = __builtin_bit_cast(float4, w2), cm = __builtin_bit_cast(float4, w3);
                    cut4 = allc ? 0xfu
                                : (uint32_t)(ce.x <= q.t) | ((uint32_t)(ce.y <= q.t) << 1) |
                                      ((uint32_t)(ce.z <= q.t) << 2) | ((uint32_t)(ce.w <= q.t) << 3);
                    all4 = allc ? 0u
                                : (uint32_t)(cm.x <= q.t) | ((uint32_t)(cm.y <= q.t) << 1) |
                                      ((uint32_t)(cm.z <= q.t) << 2) | ((uint32_t)(cm.w <= q.t) << 3);
                }
                uint32_t ov = 0xfu;  // children meeting the support box
                cin = 0xfu;
                if (!inside) {
                    const int I = (int)morton_compact(m), J = (int)morton_compact(m >> 1);
                    const int mk = (H.n >> (l - 1)) - 1;
                    const AxisRuns rx = axis_runs(q.cxlo, q.cxhi, l - 1, mk + 1);
                    const AxisRuns ry = axis_runs(q.cylo, q.cyhi, l - 1, mk + 1);
                    ov = quad_bits(pair_in_run(I, rx.a, rx.n, mk), pair_in_run(J, ry.a, ry.n, mk));
                    cin = quad_bits(pair_in_run(I, rx.ai, rx.ni, mk), pair_in_run(J, ry.ai, ry.ni, mk));
                }
                tested = (uint32_t)__popc(ov);
                chm = ((uint32_t)key_in_box(q.hkey, b01.x, b01.y) | ((uint32_t)key_in_box(q.hkey, b01.z, b01.w) << 1) |
                       ((uint32_t)key_in_box(q.hkey, b23.x, b23.y) << 2) |
                       ((uint32_t)key_in_box(q.hkey, b23.z, b23.w) << 3)) & ov;
                if (CUT && all4) {
                    // a child whose children are all under the cut, none of whose
                    // children's own boxes holds h, would only test clusters that
                    // cannot hit: it is not pushed
                    const uint32_t uin = (uint32_t)key_in_box(q.hkey, u01.x, u01.y) |
                                         ((uint32_t)key_in_box(q.hkey, u01.z, u01.w) << 1) |
                                         ((uint32_t)key_in_box(q.hkey, u23.x, u23.y) << 2) |
                                         ((uint32_t)key_in_box(q.hkey, u23.z, u23.w) << 3);
                    // (from level 3, where the union keys are read: a second box test each)
                    const uint32_t utested = l - 1 >= 3 ? all4 & ~cut4 & chm : 0u;
                    tested += (uint32_t)__popc(utested);
                    chm &= ~(utested & ~uin);
                }
                if (CUT && !(entry & kAllCut) && l - 1 >= kOwnBoxLevel && (chm & cut4)) {
                    // children under the cut: the box of their own cluster triangles
                    // (inside the subtree's box) decides instead, another 32 B segment
                    const uint4* cc = reinterpret_cast<const uint4*>(H.bbox_c + c0);
                    const uint4 c01 = cc[0], c23 = cc[1];
                    const uint32_t own = (uint32_t)key_in_box(q.hkey, c01.x, c01.y) |
                                         ((uint32_t)key_in_box(q.hkey, c01.z, c01.w) << 1) |
                                         ((uint32_t)key_in_box(q.hkey, c23.x, c23.y) << 2) |
                                         ((uint32_t)key_in_box(q.hkey, c23.z, c23.w) << 3);
                    chm &= ~cut4 | own;
                }
                m4 = 4 * m;
            }
        }
        if (l >= 2) {
            // Children under the cut go to the cluster queue (which holds fewer than 64
            // entries here, so up to 64 x 4 more fit), the others are appended to the
            // level below (which holds fewer than 64 items: it is empty or the short
            // lowest list).  A parent whose list children would run past the list's end
            // goes back to its own list whole and is expanded again later.  Child
            // positions grow with the lane, so the parents that fit are a prefix and the
            // first one with children always fits.
            const uint32_t chl = CUT ? chm & ~cut4 : chm, chc = CUT ? chm & cut4 : 0u;
            int total;
            const int nch = __popc(chl);
            const int pos = wave_prefix_small(nch, &total);
            const int below = __builtin_amdgcn_readlane(cntv, l - 1);
            const bool back = nch > 0 && below + pos + nch > kListCap;
            const uint64_t bb = __ballot(back);
            if (!back) {
                // child c goes to below + pos + (number of list children before it)
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    if (chl & (1u << c))
                        nl.put(l - 1, below + pos + __popc(chl & ((1u << c) - 1u)),
                               (m4 + c) | ((cin >> c) & 1u ? kInside : 0u) | ((all4 >> c) & 1u ? kAllCut : 0u));
                acc.nodes += tested;
            }
            if (CUT) {
                const uint32_t mine = back ? 0u : chc;
                int ctot;
                const int cpos = cn + wave_prefix_small(__popc(mine), &ctot);
                const uint32_t lev = (uint32_t)(l - 1) << kCluShift;
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    if (mine & (1u << c)) cq[cpos + __popc(mine & ((1u << c) - 1u))] = lev | (m4 + c);
                cn += ctot;
            }
            const int pushed = bb ? __builtin_amdgcn_readlane(pos, __builtin_ctzll(bb)) : total;
            if (lane == l - 1) cntv = below + pushed;
            if (pushed) nonempty |= 1u << (l - 1);
            if (bb) {
                const int nb = __popcll(bb);
                if (back) nl.put(l, base + __popcll(bb & ((1ull << lane) - 1ull)), entry);
                if (lane == l) cntv = base + nb;
                nonempty |= 1u << l;
            }
        }
        if (SPAWN) hungry = (unsigned)__builtin_amdgcn_readfirstlane((int)hv);
        wave_sync();
    }
}

// Root items of a query: the level-lr nodes overlapping the box, one per lane of an
// 8 x 8 lane grid where *ok is set; Morton codes (level >= 1) or packed texel cells
// (level 0).  At the entry level l0 (node side >= r) at most 3 nodes per axis overlap
// the box, at l0 - 1 at most 5.
__device__ __forceinline__ uint32_t root_item(const HierDev& H, const QuerySetup& q, int lr, bool* ok)
{
    const int lane = threadIdx.x & 63;
    const int M = H.n >> lr, mm = M - 1;
    const int kx0 = q.cxlo >> lr, ky0 = q.cylo >> lr;
    const int nkx = min((q.cxhi >> lr) - kx0 + 1, M), nky = min((q.cyhi >> lr) - ky0 + 1, M);
    const int ra = lane & 7, rb = lane >> 3;
    *ok = ra < nkx && rb < nky;
    const uint32_t I = (uint32_t)((kx0 + ra) & mm), J = (uint32_t)((ky0 + rb) & mm);
    if (lr == 0) return I | (J << 16);
    const int side = 1 << lr;
    const bool inside = axis_inside((int)I * side, side, q.cxlo, q.cxhi, H.logn) &&
                        axis_inside((int)J * side, side, q.cylo, q.cyhi, H.logn);
    return morton(I, J) | (inside ? kInside : 0u);
}

// The level a query's descent starts at.  Without the cut it starts below the entry
// level: the entry level's few large boxes seldom prune, and testing their children
// (at most 5 x 5), or their grandchildren when those fit the 8 x 8 lane grid, as
// roots skips steps that would run with at most 9 or 25 of 64 lanes.  (With the cut
// the entry-level nodes' own residuals decide first, so it starts there.)
template <bool CUT>
__device__ __forceinline__ int descent_start(const HierDev& H, const QuerySetup& q)
{
    if (CUT || q.l0 == 0) return q.l0;
    int lr = q.l0 - 1;
    if (lr >= 1) {
        const int l2 = lr - 1, M2 = H.n >> l2;
        if (min((q.cxhi >> l2) - (q.cxlo >> l2) + 1, M2) <= 8 && min((q.cyhi >> l2) - (q.cylo >> l2) + 1, M2) <= 8)
            lr = l2;
    }
    return lr;
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
template <int MODE, int KER>
__global__ __launch_bounds__(256) void k_eval_brute(HierDev H, EvalArgs a)
{
    const int64_t local = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (local >= a.slots) return;
    const int64_t qi = a.slot0 + local;
    const int lane = threadIdx.x & 63;
    const QuerySetup q = uniform_query(setup_query(a.q[qi], a.s2r, 0.f, H.L, H.eps, a.kernel));
    if (!q.valid) { invalid<MODE>(a, qi); return; }
    const int n = H.n, msk = n - 1;
    const int spanx = q.cxhi - q.cxlo + 1, spany = q.cyhi - q.cylo + 1;
    const int nx = spanx >= n ? n : spanx, ny = spany >= n ? n : spany;
    const int total = nx * ny;  // <= 8192^2
    Acc acc;
    Rec rec{a.ids, a.terms, MODE == kModeRecord ? a.offsets[qi] : 0,
            MODE == kModeRecord ? a.offsets[qi + 1] : 0};
    __shared__ uint32_t hq_all[4 * kHitCap];
    uint32_t* hq = hq_all + (threadIdx.x >> 6) * kHitCap;
    int hn = 0;
    uint32_t pend = 0, ebase = 0;
    int base = 0;
    while (true) {
        queue_hits(hq, hn, pend, ebase);
        if (hn >= 64 || (hn > 0 && base >= total)) {
            const int c = min(hn, 64);
            hn -= c;
            hit_round<MODE, KER>(H, q, hq + hn, c, acc, rec);
            continue;
        }
        if (base >= total) break;
        const int idx = base + lane;
        if (idx < total) {
            const int ca = idx % nx, cb = idx / nx;
            const int i = spanx >= n ? ca : ((q.cxlo + ca) & msk);
            const int j = spany >= n ? cb : ((q.cylo + cb) & msk);
            pend = plane_cell_mask(H, q, i, j, acc);
            ebase = kHitPlane | ((uint32_t)j << 14) | ((uint32_t)i << 1);
        }
        base += 64;
    }
    finish<MODE>(a, qi, q, acc);
}

// ------------------------------------------------------------ hierarchical

// One wavefront per workgroup (a long query holds only its own LDS).  LDS: the node
// lists of levels 1..L (NodeLists), the hit queue and, with the cut, the cluster queue.
template <int MODE, bool CUT, int KER>
__global__ __launch_bounds__(64) void k_eval_plain(HierDev H, EvalArgs a)
{
    extern __shared__ uint32_t lds[];
    const int64_t local = xcd_contiguous(blockIdx.x, gridDim.x);
    if (local >= a.slots) return;
    const int64_t slot = a.slot0 + local;
    const int64_t qi = a.order ? (int64_t)a.order[slot] : slot;
    uint32_t* lists = lds;
    const QuerySetup q = uniform_query(setup_query(a.q[qi], a.s2r, CUT ? a.tau : 0.f, H.L, H.eps, a.kernel));
    if (!q.valid) { invalid<MODE>(a, qi); return; }
    Acc acc;
    Rec rec{a.ids, a.terms, MODE == kModeRecord ? a.offsets[qi] : 0,
            MODE == kModeRecord ? a.offsets[qi + 1] : 0};
    const int lr = descent_start<CUT>(H, q);
    bool ok;
    const uint32_t item = root_item(H, q, lr, &ok);
    TaskQueue none{};
    descend<MODE, CUT, false, KER>(H, q, lists, lr, ok, item, false, 0, 0, none, acc, rec);
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
                                long long nq, float* out, unsigned epoch, uint32_t* hist, int nb)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    for (long long i = t; i < nq; i += (long long)gridDim.x * blockDim.x) {
        acc[i].w0 = 0;
        acc[i].w1 = 0;
        acc[i].w2 = 0;
        fexp[i] = 0;
    }
    if (hist)
        for (long long i = t; i < nb; i += (long long)gridDim.x * blockDim.x) hist[i] = 0;
    if (t == 0) {
        for (int x = 0; x < kXcds; ++x) ctl->qhead[x].v = 0;
        ctl->head = 0;
        ctl->tail = 0;
        ctl->outstanding = 0;
        for (int c = 0; c < kStarveCopies; ++c) ctl->starving[c].v = ctl->done[c].v = 0;
        ctl->spawned = ctl->refused = ctl->spins = 0;
        ctl->epoch = epoch;
        ctl->error = 0;
        ctl->q = q;
        ctl->out = out;
        ctl->nq = nq;
    }
}

// Queries taken by one worker per claim: an eighth of the share's remaining queries
// per worker of the XCD, at most kMaxChunk, down to single queries for the share's
// last part (so that no wave ends up holding several large footprints at the end).
// Every claim is an atomic on the share's counter, which all the XCD's workers
// hit: at one claim per few cheap queries its line serialised them (powerlaw2048
// took 18.2 ms with at most 4 queries per claim, 13.6 ms with up to 32; claims
// sized by the time of the previous chunk, or without reading the counter first,
// were slower on the scratched map's heavy tail).
constexpr int kMaxChunk = 32;
constexpr int kChunkDiv = 8;

__device__ __forceinline__ unsigned long long ld_relaxed(const unsigned long long* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void add_relaxed(unsigned long long* p, long long v)
{
    __hip_atomic_fetch_add(p, (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool all_taken(QueueCtl* ctl, long long nq)
{
    for (int x = 0; x < kXcds; ++x)
        if ((long long)ld_relaxed(&ctl->qhead[x].v) < nq * (x + 1) / kXcds - nq * x / kXcds) return false;
    return true;
}

// A unit of work is over: a worker's whole query phase (counted when the worker
// starts, ended when it finds no query left), or a donated task (counted by its
// donor before it is published).  The decrement that leaves nothing outstanding
// after every query was taken ends the run: it raises the done flags the waiting
// workers poll.  (A worker that starts late counts itself before looking for
// queries and finds none, so the count cannot leave zero while work remains.)
__device__ __forceinline__ void unit_done(QueueCtl* ctl, long long nq)
{
    const unsigned long long old = __hip_atomic_fetch_add(&ctl->outstanding, (unsigned long long)-1ll,
                                                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old == 1 && all_taken(ctl, nq))
        for (int c = 0; c < kStarveCopies; ++c)
            __hip_atomic_store(&ctl->done[c].v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Worker waves of a persistent run.  A wave takes chunks of consecutive queries of
// the processing order, from its XCD's eighth of the order first (shrinking towards
// single queries as a share runs out, so the last ones spread over all workers).
// Once no query is left it takes a ticket of the task queue and waits for that
// slot's task (a subtree some busy wave gave away), polling only that slot's flag
// with a short exponential back-off and, now and then, whether the run is over
// (every query taken and nothing outstanding).
// (5 waves per SIMD fit without spilling vector registers)
template <bool CUT, int KER>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_persist(HierDev H, PersistArgs pa)
{
    extern __shared__ uint32_t lds[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint32_t* lists = lds + (size_t)wave * wave_lds_words(H.L, CUT);
    QueueCtl* ctl = pa.Q.ctl;
    const long long nq = ctl->nq;
    const pndf_query* qs = ctl->q;
    const unsigned epoch = ctl->epoch;
    // worker waves per XCD (block b runs on XCD b mod 8)
    const long long xworkers = max(1ll, (long long)gridDim.x * (blockDim.x >> 6) / kXcds);
    const int home = blockIdx.x & (kXcds - 1);
    Rec rec{nullptr, nullptr, 0, 0};
    // a wave that has waited pa.wait_ticks of the constant-rate clock without any
    // work arriving gives up and flags the run (a broken count would otherwise hang)
    long long idle_since = -1;
    int backoff = 1;
    unsigned long long spins = 0;
    long long qb = 0, qe = 0;  // the wave's current chunk of query slots
    long long ticket = -1;     // the wave's place in the task queue while it waits for a task
    int polls = 0;
    bool querying = true;      // in the query phase (counted as one outstanding unit)
    if (lane == 0) add_relaxed(&ctl->outstanding, 1);
    while (true) {
        long long task_slot = -1;
        if (qb >= qe) {
            long long nb = -1, ne = -1;
            if (lane == 0) {
                if (ticket < 0) {
                    // a chunk of queries: from this XCD's share of the processing order
                    // first (neighbouring queries, so the XCD's L2 holds their nodes), then
                    // from the other shares (one atomic per chunk, on the share's own line)
                    for (int k = 0; querying && nb < 0 && k < kXcds; ++k) {
                        const int x = (home + k) & (kXcds - 1);
                        const long long lo = nq * x / kXcds, len = nq * (x + 1) / kXcds - lo;
                        const long long qh = (long long)ld_relaxed(&ctl->qhead[x].v);
                        if (qh >= len) continue;
                        const long long c =
                            max(1ll, min((long long)kMaxChunk, (len - qh) / (kChunkDiv * xworkers)));
                        const long long qn = (long long)__hip_atomic_fetch_add(
                            &ctl->qhead[x].v, (unsigned long long)c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if (qn < len) {
                            nb = lo + qn;
                            ne = lo + min(qn + c, len);
                        }
                    }
                    if (nb < 0 && querying) {
                        // every query is taken: the query phase is over
                        querying = false;
                        unit_done(ctl, nq);
                    }
                    if (nb < 0) {
                        // no query left: take a ticket (the next task slot in order) and tell
                        // the busy waves that workers are waiting
                        ticket = (long long)__hip_atomic_fetch_add(&ctl->head, 1ull, __ATOMIC_RELAXED,
                                                                   __HIP_MEMORY_SCOPE_AGENT);
                        polls = 0;
                        for (int c = 0; c < kStarveCopies; ++c)
                            __hip_atomic_store(&ctl->starving[c].v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
                // a relaxed poll (an acquire load would invalidate this CU's L1 under the
                // busy waves at every poll); the acquire fence only once the task is there
                if (nb < 0 && ticket >= 0 && ticket < (long long)pa.Q.capacity &&
                    __hip_atomic_load(&pa.Q.flags[ticket], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == epoch) {
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    task_slot = ticket;
                    ticket = -1;
                }
            }
            task_slot = (long long)uniform_u64((unsigned long long)task_slot);
            nb = (long long)uniform_u64((unsigned long long)nb);
            ne = (long long)uniform_u64((unsigned long long)ne);
            ticket = (long long)uniform_u64((unsigned long long)ticket);
            if (task_slot < 0 && nb < 0) {
                // waiting for the ticket's task (a slot past the capacity never gets one);
                // the run is over once every query is taken and nothing is outstanding
                int done = 0;
                if (lane == 0) {
                    ++spins;
                    done = __hip_atomic_load(&ctl->done[home].v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
                    if (!done && (++polls & 63) == 0) {
                        // now and then the full condition too, and a reminder to the busy waves
                        done = (all_taken(ctl, nq) && ld_relaxed(&ctl->outstanding) == 0) ? 1 : 0;
                        if (!done)
                            for (int c = 0; c < kStarveCopies; ++c)
                                __hip_atomic_store(&ctl->starving[c].v, 1u, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
                    }
                    const long long now = wall_clock64();
                    if (idle_since < 0) idle_since = now;
                    if (!done && now - idle_since > pa.wait_ticks) {
                        atomicOr(&ctl->error, 1u);
                        done = 1;
                    }
                }
                done = __builtin_amdgcn_readfirstlane(done);
                if (done) break;
                for (int k = 0; k < backoff; ++k) __builtin_amdgcn_s_sleep(16);
                backoff = min(backoff * 2, 8);
                continue;
            }
            idle_since = -1;
            backoff = 1;
            if (nb >= 0) {
                qb = nb;
                qe = ne;
            }
        }
        // one work item: a stolen subtree, or the next query of the chunk
        long long qi;
        int lev;
        uint32_t item;
        bool root_ok, tested;
        if (task_slot >= 0) {
            // the slot is published (its flag carries this run's epoch); never use a
            // malformed task word
            unsigned long long word = 0;
            int ok = 0;
            if (lane == 0) {
                word = pa.Q.tasks[task_slot];
                const long long wq = (long long)(word >> 32);
                const int wl = (int)((word >> 26) & 0x3fu);
                const uint64_t wm = word & 0x3ffffffu;
                ok = 1;
                if (wq >= nq || wl < 1 || wl > H.L || wm >= (uint64_t)(H.n >> wl) * (uint64_t)(H.n >> wl)) {
                    atomicOr(&ctl->error, 4u);
                    ok = 0;
                }
            }
            ok = __builtin_amdgcn_readfirstlane(ok);
            word = uniform_u64(word);
            if (!ok) {
                if (lane == 0) unit_done(ctl, nq);
                continue;
            }
            qi = (long long)(word >> 32);
            lev = (int)((word >> 26) & 0x3fu);
            item = (uint32_t)(word & 0x3ffffffu);
            root_ok = lane == 0;
            tested = true;
        } else {
            qi = pa.order ? (long long)pa.order[qb] : qb;
            qi = (long long)uniform_u64((unsigned long long)qi);
            ++qb;
            lev = -1;  // set below from the query
            item = 0;
            root_ok = false;
            tested = false;
        }
        const QuerySetup q = uniform_query(setup_query(qs[qi], pa.s2r, CUT ? pa.tau : 0.f, H.L, H.eps, pa.kernel));
        Acc acc;
        if (lev < 0) {
            lev = descent_start<CUT>(H, q);
            item = root_item(H, q, lev, &root_ok);
        }
        // a query whose levels are all below split_level never donates; a stolen
        // subtree may be split again
        if (q.valid)
            descend<kModeValue, CUT, true, KER>(H, q, lists, lev, root_ok, item, tested, pa.split_level,
                                           (unsigned long long)qi, pa.Q, acc, rec);
        const Fix192 d = wave_sum_fix(acc.d);
        if (lane == 0) {
            if (task_slot >= 0) {
                acc_atomic_add(&pa.acc[qi], d);
            } else {
                pa.fexp[qi] = q.valid ? q.fexp : 0x7fffffff;
                if (acc.donated)
                    acc_atomic_add(&pa.acc[qi], d);  // tasks of this query add theirs too
                else
                    pa.acc[qi] = d;                  // the only contribution
            }
        }
        if (task_slot >= 0) {
            // the task is finished.  No fence: the count only decides when workers stop;
            // the sums are read after the kernel ends.
            if (lane == 0) unit_done(ctl, nq);
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

// Launches cover at most launch_chunk() queries (grid dimensions stay far below
// 2^32 work-items).
template <int MODE, int KER>
hipError_t launch_mode(const HierDev& H, const EvalArgs& a0, int algo, hipStream_t s)
{
    const int64_t chunk = launch_chunk();
    for (int64_t off = 0; off < a0.nq; off += chunk) {
        EvalArgs a = a0;
        a.slot0 = off;
        a.slots = std::min<int64_t>(chunk, a0.nq - off);
        if (algo == PNDF_ALGO_BRUTE) {
            const unsigned blocks = (unsigned)((a.slots + 3) / 4);
            hipLaunchKernelGGL((k_eval_brute<MODE, KER>), dim3(blocks), dim3(256), 0, s, H, a);
        } else {
            const unsigned blocks = (unsigned)a.slots;
            const size_t lds = sizeof(uint32_t) * wave_lds_words(H.L, a.tau > 0.f);
            if (a.tau > 0.f)
                hipLaunchKernelGGL((k_eval_plain<MODE, true, KER>), dim3(blocks), dim3(64), lds, s, H, a);
            else
                hipLaunchKernelGGL((k_eval_plain<MODE, false, KER>), dim3(blocks), dim3(64), lds, s, H, a);
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int MODE>
hipError_t launch_kernel(const HierDev& H, const EvalArgs& a, int algo, hipStream_t s)
{
    if (a.kernel == PNDF_KERNEL_BOX) return launch_mode<MODE, PNDF_KERNEL_BOX>(H, a, algo, s);
    if (a.kernel == PNDF_KERNEL_DISK) return launch_mode<MODE, PNDF_KERNEL_DISK>(H, a, algo, s);
    return launch_mode<MODE, PNDF_KERNEL_GAUSSIAN>(H, a, algo, s);
}

// ------------------------------------------------------------ query order
constexpr int kOrderBits = 6;  // 64 x 64 buckets

__global__ void k_order_zero(uint32_t* hist, int nb)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += gridDim.x * blockDim.x) hist[i] = 0;
}

// The histogram and the scatter count in LDS first (bins < 4096: at most 64 x 64
// Morton buckets), so the global counters see one atomic per non-empty bin per
// workgroup instead of one per query; a workgroup takes a large strided share of
// the batch (the grid is small, order_blocks).
constexpr int kOrderMaxBins = 4096;

__device__ __forceinline__ void order_hist(const pndf_query* __restrict__ q, int64_t nq, int n, int bshift,
                                           uint32_t* __restrict__ key, uint32_t* __restrict__ hist)
{
    __shared__ uint32_t loc[kOrderMaxBins];
    for (int b = threadIdx.x; b < kOrderMaxBins; b += blockDim.x) loc[b] = 0u;
    __syncthreads();
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
        atomicAdd(&loc[k], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kOrderMaxBins; b += blockDim.x)
        if (loc[b]) atomicAdd(&hist[b], loc[b]);
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

// Each workgroup reserves, per bin, a range of the exact size of its share's count
// (one global atomic per non-empty bin), then places its queries in it.  Within a
// bucket the order is whatever the atomics give: results do not depend on it.
__device__ __forceinline__ void order_scatter(const uint32_t* __restrict__ key, int64_t nq,
                                              uint32_t* __restrict__ cursor, uint32_t* __restrict__ order)
{
    __shared__ uint32_t loc[kOrderMaxBins];
    for (int b = threadIdx.x; b < kOrderMaxBins; b += blockDim.x) loc[b] = 0u;
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = i0; i < nq; i += stride) atomicAdd(&loc[key[i]], 1u);
    __syncthreads();
    for (int b = threadIdx.x; b < kOrderMaxBins; b += blockDim.x)
        if (loc[b]) loc[b] = atomicAdd(&cursor[b], loc[b]);
    __syncthreads();
    for (int64_t i = i0; i < nq; i += stride) order[atomicAdd(&loc[key[i]], 1u)] = (uint32_t)i;
}

__global__ void k_order_hist(const pndf_query* __restrict__ q, int64_t nq, int n, int bshift,
                             uint32_t* __restrict__ key, uint32_t* __restrict__ hist)
{
    order_hist(q, nq, n, bshift, key, hist);
}

__global__ void k_order_scatter(const uint32_t* __restrict__ key, int64_t nq, uint32_t* __restrict__ cursor,
                                uint32_t* __restrict__ order)
{
    order_scatter(key, nq, cursor, order);
}

// The same two passes for a persistent plan, reading the batch from its control
// block (so the launch graph needs no per-run arguments for them).
__global__ void k_porder_hist(const QueueCtl* ctl, int n, int bshift, uint32_t* __restrict__ key,
                              uint32_t* __restrict__ hist)
{
    order_hist(ctl->q, ctl->nq, n, bshift, key, hist);
}

__global__ void k_porder_scatter(const QueueCtl* ctl, const uint32_t* __restrict__ key,
                                 uint32_t* __restrict__ cursor, uint32_t* __restrict__ order)
{
    order_scatter(key, ctl->nq, cursor, order);
}

}  // namespace

void order_shape(int logn, int* nb, int* bshift)
{
    const int bits = logn < kOrderBits ? logn : kOrderBits;
    *nb = 1 << (2 * bits);
    *bshift = logn - bits;
}

// Workgroups (of 256) of the histogram and scatter passes: about 16k queries each,
// at most 256 (one per compute unit), so the LDS counts absorb most atomics.
static unsigned order_blocks(int64_t nq)
{
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(256, (nq + 16383) / 16384));
}

// The four passes of the spatial order into buf = order[nq] | key[nq] | hist[nb]
// (the histogram is cleared by a kernel, never a memset node).
static hipError_t order_passes(const HierDev& H, const pndf_query* q, int64_t nq, uint32_t* buf, hipStream_t s)
{
    int nb, bshift;
    order_shape(H.logn, &nb, &bshift);
    uint32_t* key = buf + nq;
    uint32_t* hist = key + nq;
    const unsigned g = order_blocks(nq);
    hipLaunchKernelGGL(k_order_zero, dim3(16), dim3(256), 0, s, hist, nb);
    hipLaunchKernelGGL(k_order_hist, dim3(g), dim3(256), 0, s, q, nq, H.n, bshift, key, hist);
    hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(1024), 0, s, hist, nb);
    hipLaunchKernelGGL(k_order_scatter, dim3(g), dim3(256), 0, s, key, nq, hist, buf);
    return hipGetLastError();
}

hipError_t make_order(const HierDev& H, const pndf_query* q, int64_t nq, uint32_t** order, hipStream_t s)
{
    *order = nullptr;
    int nb, bshift;
    order_shape(H.logn, &nb, &bshift);
    uint32_t* buf = nullptr;  // order[nq] | key[nq] | hist[nb]
    hipError_t e = hipMallocAsync((void**)&buf, sizeof(uint32_t) * (2 * (size_t)nq + nb), s);
    if (e != hipSuccess) return e;
    e = order_passes(H, q, nq, buf, s);
    if (e != hipSuccess) {
        (void)hipFreeAsync(buf, s);
        return e;
    }
    *order = buf;
    return hipSuccess;
}

// Workspace of the spatial order for callers that cannot allocate: one array per
// GPU, held until the process ends, for batches of up to kStaticOrderQueries
// queries (order, keys and the largest histogram: 32 MiB + 16 KiB).  Its device
// address is looked up once per device; host code uses that address, never the
// array's name.  Every call on a GPU shares it, so calls that overlap on one GPU
// race.
static __device__ __align__(256) uint32_t scratch[2 * kStaticOrderQueries + 4096];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t make_order_static(const HierDev& H, const pndf_query* q, int64_t nq, uint32_t** order, hipStream_t s)
{
    *order = nullptr;
    if (nq > kStaticOrderQueries) return hipErrorInvalidValue;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    uint32_t* buf = nullptr;
    {
        std::lock_guard<std::mutex> g(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            void* p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return e;
            g_scratch_ptr[dev] = static_cast<uint32_t*>(p);
        }
        buf = g_scratch_ptr[dev];
    }
    int nb, bshift;
    order_shape(H.logn, &nb, &bshift);
    if (nb > 4096) return hipErrorInvalidValue;
    e = order_passes(H, q, nq, buf, s);
    if (e == hipSuccess) *order = buf;
    return e;
}

void free_order(uint32_t* order, hipStream_t s)
{
    if (order) (void)hipFreeAsync(order, s);
}

hipError_t launch_eval(const HierDev& H, const EvalArgs& a, int algo, hipStream_t s)
{
    if (a.nq <= 0) return hipSuccess;
    if (a.offsets) return launch_kernel<kModeRecord>(H, a, algo, s);
    if (a.counts) return launch_kernel<kModeCount>(H, a, algo, s);
    return launch_kernel<kModeValue>(H, a, algo, s);
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
    P.rargs[7] = &P.ohist;
    P.rargs[8] = &P.order_nb;
    P.reset.func = (void*)k_persist_reset;
    P.reset.gridDim = dim3((unsigned)std::min<long long>(1024, (P.max_nq + 255) / 256 + 1));
    P.reset.blockDim = dim3(256);
    P.reset.sharedMemBytes = 0;
    P.reset.kernelParams = P.rargs;
    P.reset.extra = nullptr;
}

// The worker kernel for a plan's cut setting and footprint kernel.
static void* persist_func(const PersistPlan& P)
{
    const bool cut = P.tau > 0.f;
    if (P.kernel == PNDF_KERNEL_BOX) return cut ? (void*)k_persist<true, PNDF_KERNEL_BOX> : (void*)k_persist<false, PNDF_KERNEL_BOX>;
    if (P.kernel == PNDF_KERNEL_DISK)
        return cut ? (void*)k_persist<true, PNDF_KERNEL_DISK> : (void*)k_persist<false, PNDF_KERNEL_DISK>;
    return cut ? (void*)k_persist<true, PNDF_KERNEL_GAUSSIAN> : (void*)k_persist<false, PNDF_KERNEL_GAUSSIAN>;
}

// Worker blocks of the plan's kernel that fit on one compute unit at once
// (registers and LDS), 0 if the runtime cannot tell.
int persist_resident_blocks(const HierDev& H, const PersistPlan& P)
{
    int nb = 0;
    const size_t lds = sizeof(uint32_t) * 4 * wave_lds_words(H.L, P.tau > 0.f);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, persist_func(P), 256, lds) != hipSuccess) return 0;
    return nb;
}



// Kernel-node parameters of the three order passes (spatial order of the batch).
static void order_params(PersistPlan& P, hipKernelNodeParams* hist, hipKernelNodeParams* scan,
                         hipKernelNodeParams* scat)
{
    P.hargs[0] = &P.ctl;
    P.hargs[1] = &P.on;
    P.hargs[2] = &P.order_bshift;
    P.hargs[3] = &P.okey;
    P.hargs[4] = &P.ohist;
    P.sargs[0] = &P.ohist;
    P.sargs[1] = &P.order_nb;
    P.cargs[0] = &P.ctl;
    P.cargs[1] = &P.okey;
    P.cargs[2] = &P.ohist;
    P.cargs[3] = &P.order;
    *hist = hipKernelNodeParams{};
    hist->func = (void*)k_porder_hist;
    hist->gridDim = dim3(order_blocks(P.max_nq));
    hist->blockDim = dim3(256);
    hist->kernelParams = P.hargs;
    *scan = hipKernelNodeParams{};
    scan->func = (void*)k_order_scan;
    scan->gridDim = dim3(1);
    scan->blockDim = dim3(1024);
    scan->kernelParams = P.sargs;
    *scat = hipKernelNodeParams{};
    scat->func = (void*)k_porder_scatter;
    scat->gridDim = dim3(order_blocks(P.max_nq));
    scat->blockDim = dim3(256);
    scat->kernelParams = P.cargs;
}

void persist_prepare(const HierDev& H, PersistPlan& P)
{
    P.H = H;
    P.pa.Q.ctl = P.ctl;
    P.pa.Q.tasks = P.tasks;
    P.pa.Q.flags = P.flags;
    P.pa.Q.capacity = P.capacity;
    P.pa.order = P.order;
    P.pa.acc = P.acc;
    P.pa.fexp = P.fexp;
    P.pa.tau = P.tau;
    P.pa.s2r = P.s2r;
    P.pa.kernel = P.kernel;
    P.pa.split_level = P.split_level;
    P.pa.wait_ticks = P.wait_ticks;
    P.okey = P.ohist = nullptr;
    if (P.order) {
        P.okey = P.order + P.max_nq;
        P.ohist = P.okey + P.max_nq;
    }
    P.on = H.n;
}

hipError_t persist_graph_build(const HierDev& H, PersistPlan& P)
{
    persist_prepare(H, P);
    hipKernelNodeParams ohist{}, oscan{}, oscat{};
    if (P.order) order_params(P, &ohist, &oscan, &oscat);
    reset_params(P, nullptr, 0, nullptr);
    P.wargs[0] = &P.H;
    P.wargs[1] = &P.pa;
    hipKernelNodeParams work{};
    work.func = persist_func(P);
    work.gridDim = dim3((unsigned)P.blocks);
    work.blockDim = dim3(256);
    work.sharedMemBytes = (unsigned)(sizeof(uint32_t) * 4 * wave_lds_words(H.L, P.tau > 0.f));
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
    hipGraphNode_t nw = nullptr, nf = nullptr, nh = nullptr, ns = nullptr, nc = nullptr;
    if (e == hipSuccess) e = hipGraphAddKernelNode(&P.reset_node, P.graph, nullptr, 0, &P.reset);
    hipGraphNode_t before_work = P.reset_node;
    if (P.order) {
        if (e == hipSuccess) e = hipGraphAddKernelNode(&nh, P.graph, &P.reset_node, 1, &ohist);
        if (e == hipSuccess) e = hipGraphAddKernelNode(&ns, P.graph, &nh, 1, &oscan);
        if (e == hipSuccess) e = hipGraphAddKernelNode(&nc, P.graph, &ns, 1, &oscat);
        before_work = nc;
    }
    if (e == hipSuccess) e = hipGraphAddKernelNode(&nw, P.graph, &before_work, 1, &work);
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
                       q, nq, out, P.epoch, P.ohist, P.order_nb);
    if (P.order) {
        hipLaunchKernelGGL(k_porder_hist, dim3(order_blocks(P.max_nq)), dim3(256), 0, s, P.ctl, P.on,
                           P.order_bshift, P.okey, P.ohist);
        hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(1024), 0, s, P.ohist, P.order_nb);
        hipLaunchKernelGGL(k_porder_scatter, dim3(order_blocks(P.max_nq)), dim3(256), 0, s, P.ctl, P.okey,
                           P.ohist, P.order);
    }
    const size_t lds = sizeof(uint32_t) * 4 * wave_lds_words(P.H.L, P.tau > 0.f);
    void* args[] = {&P.H, &P.pa};
    const hipError_t e = hipLaunchKernel(persist_func(P), dim3((unsigned)P.blocks), dim3(256), args, lds, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_persist_finalize, P.reset.gridDim, dim3(256), 0, s, P.ctl, P.acc, P.fexp);
    return hipGetLastError();
}

}  // namespace pndf
