// Internal definitions of the gfx950 P-NDF library: handle layouts, the device
// view passed to kernels, and the device helpers shared by the evaluation
// kernels (query setup, periodic-image arithmetic, triangle tests, hit terms).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <atomic>
#include <cstdint>
#include <string>

#include "../../include/pndf.h"

namespace pndf {

constexpr int kMaxLevels = 13;   // N <= 8192
constexpr int kWave = 64;
#ifndef PNDF_LIST_CAP
#define PNDF_LIST_CAP 128
#endif
// Per-level traversal list entries.  A wave expands up to 64 parents at a time;
// parents whose children do not fit wait in their own list.  The roots of a query
// fill up to an 8 x 8 lane grid (64 entries of one list), and children are appended
// to a list that is empty or holds fewer than 32 entries (the short lowest list,
// expanded after the level above it), so with at least 64 entries the first
// parent's four children always fit and the descent progresses.  (Fewer entries
// would mean more waves per CU, but roots would overflow.)
constexpr int kListCap = PNDF_LIST_CAP;
static_assert(kListCap >= 64, "a list holds up to 64 roots; a short list (< 32) plus four children must fit");

// Kernel launches cover at most this many queries (one workgroup or one wavefront
// each), so grids stay far below 2^32 work-items.  PNDF_LAUNCH_CHUNK in the
// environment lowers it (any positive value; used by the tests to force several
// launches per call, which must give the same bits).
constexpr int64_t kLaunchChunk = (int64_t)1 << 24;
int64_t launch_chunk();

// Hit queue of a wavefront: float32 hits wait here for the FP64 stage, which takes
// them 64 at a time (fewer than 64 wait between steps; one step adds at most 64 x 8).
constexpr int kHitCap = 128;

// Cluster queue of a wavefront (with the cluster cut): nodes under the cut wait here
// to be tested 64 at a time; it holds fewer than 64 before a descent step, which adds
// at most 64 x 4.
constexpr int kCluCap = 64 + 4 * 64;

// With the cluster cut, list items of the levels from short_list_level(L, true) up
// take 16 bits: a level-l Morton code is below 4^(L - l), so from l = L - 7 it fits
// 14 bits beside the two flag bits.  Fewer LDS bytes per wavefront let more
// wavefronts reside, which pays where LDS limits them (the cut kernel: powerlaw8192
// 1169 -> 1015 ms); without the cut the kernel is not LDS-limited and the extra
// registers of the 16-bit path cost a wavefront per SIMD, so all its lists stay
// 32-bit (short level L + 1).
__host__ __device__ inline int short_list_level(int L, bool cut)
{
    return !cut ? L + 1 : (L - 7 > 1 ? L - 7 : 1);
}

// 32-bit LDS words of a wavefront's node lists: 32-bit lists of levels 1..S-1, then
// 16-bit lists of levels S..L.
__host__ __device__ inline size_t list_words(int L, bool cut)
{
    const int S = short_list_level(L, cut);
    return (size_t)(S - 1) * kListCap + (size_t)(L - S + 1) * (kListCap / 2);
}
static_assert(kListCap % 2 == 0, "16-bit lists fill whole words");

// 32-bit LDS words per wavefront of the descent: the node lists of levels 1..L, the
// hit queue, and with the cut the cluster queue.
__host__ __device__ inline size_t wave_lds_words(int L, bool cut)
{
    return list_words(L, cut) + kHitCap + (cut ? kCluCap : 0);
}

// Level-1 leaf record: the 3 x 3 texel normals of a 2 x 2 cell block (row-major,
// texel (2I + x, 2J + y) at t[3 y + x], periodic) and the clamp bits of its four
// cells (cell (di, dj) at deg[2 dj + di]), 80 bytes = five 16-byte loads.
struct QuadRec {
    float2 t[9];
    uint8_t deg[4];
    uint32_t pad;
};
static_assert(sizeof(QuadRec) == 80, "QuadRec is five 16-byte words");

// Device-side view of a mesh + hierarchy, passed to kernels by value.  Every
// per-node array is stored per level in Morton (Z) order: node (I, J) of level l at
// level_offset(logn, l) + morton(I, J), so the four children of node m are 4m .. 4m + 3.
struct HierDev {
    const float2* nrm;      // (n+1) x (n+1) padded texel normals (last row/column wrap)
    const uint8_t* deg;     // n x n clamp bits (bit0 lower, bit1 upper)
    const float2* det;      // n x n Jacobians used by the evaluation (lower, upper)
    const float4* bbox;     // all levels packed: min x, min y, max x, max y (map triangles)
    const float4* bbox_all; // same, extended by cluster triangles (nullptr without clusters)
    const uint2* bbox_k;    // bbox as order keys of halves rounded outward (min down, max up): see half_key
    const uint2* bbox_c;    // the node's own two cluster triangles' box, the same way
    const uint2* bbox_u;    // from level 3: the union of its four children's own boxes (bbox_c), the same way
    // (clusters) one 64 B record per group of four sibling nodes 4k..4k+3, in 16 B
    // words: their bbox_all as keys like bbox_k (two nodes per word), their e^l, and
    // per node the largest e^l of its four children (+inf at level 1): what the cut
    // traversal reads when it expands their parent
    const uint4* grp;
    // the cluster test record, 2 float4 per node: (N0.x, N0.y, N1.x, N1.y), (N2.x,
    // N2.y, N3.x, N3.y), except that a clamped triangle's free vertex (N0 of the
    // lower, N3 of the upper: its replacement is built from the shared edge N1 N2
    // alone) holds NaN, so the record carries the clamp bits (clamp_bits)
    const float4* clu_t;
    const float* clu_e;     // e^l per node
    const float2* clu_det;  // cluster triangle Jacobians (lower, upper), eps when clamped
    const QuadRec* quad;    // level-1 leaf records (Morton order)
    int n, L, logn;
    float eps;
    float rho;              // circumradius of the clamp replacement triangle (area eps / 2)
};

// Clamp bits of a cluster test record (a, b) = clu_t[2 idx], clu_t[2 idx + 1]: bit 0
// the lower triangle (N0 stored as NaN), bit 1 the upper (N3 stored as NaN).  (The
// build keeps IEEE semantics, so x != x is the NaN test.)
__device__ __forceinline__ uint32_t clamp_bits(float4 a, float4 b)
{
    return (a.x != a.x ? 1u : 0u) | (b.z != b.z ? 2u : 0u);
}

// Order key of a half-precision value (IEEE binary16 bits): unsigned keys compare
// like the values (negative values mirrored below 0x8000, zero signs aside), so a
// box test is two packed 16-bit integer min / max operations.  Box keys are
// normalised so that the two zeros never exclude: a minimum of +0 is stored as -0
// (key 0x7fff) and a maximum of -0 as +0 (key 0x8000).
__host__ __device__ __forceinline__ uint32_t half_key(uint32_t bits)
{
    return (bits & 0x8000u) ? (~bits & 0xffffu) : (bits | 0x8000u);
}

// First node of level l (1 <= l <= logn + 1) in the packed per-level arrays: the
// levels below hold sum_{k=1}^{l-1} (n / 2^k)^2 = (n^2 - (n / 2^(l-1))^2) / 3 nodes.
__host__ __device__ __forceinline__ int64_t level_offset(int logn, int l)
{
    // 32-bit arithmetic suffices (n <= 8192: 4^13 = 2^26 nodes at most)
    return (int64_t)(((1u << (2 * logn)) - (1u << (2 * (logn - l + 1)))) / 3u);
}

// ---- exact accumulation: unsigned 192-bit fixed point w0 + 2^64 w1 + 2^128 w2, in
// units of 2^fexp.  Adding the float32 terms of a query in any order gives the same
// integer, so every evaluation algorithm (brute force, descent, split across waves)
// returns the same D.
struct Fix192 {
    uint64_t w0, w1, w2;
};

// Global task queue of the persistent traversal, a ticket queue: a worker with no
// query left takes a ticket (fetch-add on `head`) and waits for that slot only; a
// busy wave that sees workers waiting (head > tail) reserves slots with a fetch-add
// on `tail`, writes the tasks and publishes each by storing the launch's epoch into
// its flag.  No CAS retry loop, so thousands of waiting workers do not serialise on
// one word.  `outstanding` counts query chunks and tasks taken or published but not
// finished; a worker exits once every query is taken and nothing is outstanding.
// Every word of the control block that many waves touch sits on its own 128-byte
// line, so the pollers of one do not queue behind the users of another.
constexpr int kStarveCopies = 8;  // replicas of the starving flag (by block index)
constexpr int kXcds = 8;          // workgroups are dispatched to the 8 XCDs round-robin
struct QueueCtl {
    struct alignas(128) Head {
        unsigned long long v;
    } qhead[kXcds];                               // next query slot of each XCD's share of the order
    alignas(128) unsigned long long head;         // tickets handed out (task slots waited for)
    alignas(128) unsigned long long tail;         // task slots reserved by donors
    alignas(128) unsigned long long outstanding;  // query chunks and tasks taken or published, not finished
    struct alignas(128) Flag {
        unsigned int v;
    } starving[kStarveCopies];                    // set by idle workers, cleared by a donation
    Flag done[kStarveCopies];                     // set once every query is taken and nothing is outstanding
    alignas(128) unsigned long long spawned, refused, spins;  // statistics
    unsigned int epoch, error;      // error bit0: idle wait gave up, bit1: slot wait gave up, bit2: bad task
    const pndf_query* q;
    float* out;
    long long nq;
};

struct TaskQueue {
    QueueCtl* ctl;
    unsigned long long* tasks;  // (query << 32) | (level << 26) | Morton code of the node
    unsigned int* flags;        // epoch of the launch that published the slot
    unsigned long long capacity;
};

struct PersistArgs {
    TaskQueue Q;
    const uint32_t* order;  // processing order of the queries (nullptr: input order)
    Fix192* acc;     // per-query exact sums
    int* fexp;       // per-query binary point (written by the query's root task)
    float tau, s2r;
    int kernel;           // PNDF_KERNEL_*
    int split_level;      // smallest level whose nodes may be donated (>= 1)
    long long wait_ticks; // give-up bound of a worker's waits, in wall_clock64 ticks
};

// Device resources and the instantiated launch graph of a persistent plan.
struct PersistPlan {
    QueueCtl* ctl = nullptr;
    Fix192* acc = nullptr;
    int* fexp = nullptr;
    unsigned long long* tasks = nullptr;
    unsigned int* flags = nullptr;
    unsigned long long capacity = 0;
    uint32_t* order = nullptr;  // order[max_nq] | key[max_nq] | hist[order_nb] (nullptr: input order)
    int order_nb = 0, order_bshift = 0;
    long long max_nq = 0;
    int blocks = 0, split_level = 1;
    long long wait_ticks = 0;
    float tau = 0.f, s2r = 3.f;
    int kernel = 0;
    unsigned epoch = 0;
    HierDev H{};
    PersistArgs pa{};
    // graph and the argument storage its kernel nodes point to
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t reset_node = nullptr;
    hipKernelNodeParams reset{};
    const pndf_query* rq = nullptr;
    long long rnq = 0;
    float* rout = nullptr;
    uint32_t* okey = nullptr;   // views into `order`
    uint32_t* ohist = nullptr;
    int on = 0;
    void* rargs[9];
    void* wargs[2];
    void* fargs[3];
    void* hargs[5];  // order passes: histogram, scan, scatter
    void* sargs[2];
    void* cargs[4];
};

// Fill the device arguments of a plan whose buffers are allocated.
void persist_prepare(const HierDev& H, PersistPlan& P);
// Worker blocks of the plan's kernel (cut setting and footprint kernel) resident per
// compute unit at once; 0 if unknown.
int persist_resident_blocks(const HierDev& H, const PersistPlan& P);
// persist_prepare, then build and instantiate the launch graph.
hipError_t persist_graph_build(const HierDev& H, PersistPlan& P);
hipError_t persist_run(PersistPlan& P, const pndf_query* q, long long nq, float* out, bool use_graph,
                       hipStream_t s);

}  // namespace pndf

struct pndf_mesh {
    std::atomic<int> refs{1};
    int device = 0;
    int n = 0, L = 0;
    float eps = 0.f;
    float2* nrm = nullptr;
    uint8_t* deg = nullptr;
    float2* det = nullptr;
    int64_t bytes = 0;
};

struct pndf_hier {
    pndf_mesh* mesh = nullptr;
    int cluster = 0;
    int L = 0;
    int64_t nodes = 0;
    float4* bbox = nullptr;
    float4* bbox_all = nullptr;
    uint2* bbox_k = nullptr;
    float4* bbox_clu = nullptr;   // box of the node's own cluster triangles (float32)
    uint2* bbox_c = nullptr;
    uint2* bbox_u = nullptr;
    uint4* grp = nullptr;
    float4* clu_n = nullptr;      // the fitted normals as float32 (exported; the kernels read clu_t)
    float4* clu_t = nullptr;
    float* clu_e = nullptr;
    float2* clu_det = nullptr;
    pndf::QuadRec* quad = nullptr;
    int64_t bytes = 0;
    pndf::HierDev dev;
};

namespace pndf {

// ---------------------------------------------------------------- host side
void set_error(const std::string& msg);
pndf_status hip_fail(hipError_t e, const char* what);

// launchers implemented in the .hip files
hipError_t launch_build_mesh(const float* in, int n, float eps, float2* nrm, uint8_t* deg,
                             float2* det, unsigned* d_flag, hipStream_t s);
hipError_t build_hierarchy_levels(pndf_hier* h, hipStream_t s);
// Row-major copy of a Morton-ordered per-node array of `words` 32-bit words per node.
hipError_t export_rowmajor(const void* src, void* dst, int m, int words, hipStream_t s);

struct EvalArgs {
    const pndf_query* q;
    const uint32_t* order;     // optional processing order (query index per slot)
    int64_t nq;
    int64_t slot0, slots;      // the launch covers processing slots [slot0, slot0 + slots)
    float* out;
    uint32_t* counts;          // nullptr unless counting
    const uint64_t* offsets;   // hit-record pass only
    uint64_t* ids;
    float* terms;
    float tau;
    float s2r;
    int kernel;                // PNDF_KERNEL_*
};
hipError_t launch_eval(const HierDev& H, const EvalArgs& a, int algo, hipStream_t s);

// One sample of the P-NDF per query (sample.hip).
struct SampleArgs {
    const pndf_query* q;
    const double* xi;          // attempts x nq pairs of uniforms, attempt-major
    int64_t nq;
    int64_t first, end;        // the launch covers queries [first, end)
    int attempts;
    float tau;
    float s2r;
    int kernel;                // PNDF_KERNEL_*
    float2* m;                 // sampled normal per query
    uint64_t* tri;             // optional: triangle id
    double2* u;                // optional: unrolled texture coordinates
};
hipError_t launch_sample(const HierDev& H, const SampleArgs& a, hipStream_t s);

// Projected area P(w) per query (projarea.hip).
struct ProjArgs {
    const pndf_query* q;       // x, y, sx, sy, and w_x, w_y in place of the query normal
    int64_t nq;
    float s2r;
    int kernel;                // PNDF_KERNEL_*
    float* P;
    float* lambda;             // optional: P / w_z - 1
    const uint32_t* order;     // processing order within the launch (heaviest first), or nullptr
};
hipError_t launch_projected_area(const HierDev& H, const ProjArgs& a, hipStream_t s);

// Spatial processing order of a batch: queries bucketed by the Morton code of their
// centre cell (64 x 64 buckets over the torus), stream-ordered workspace.
hipError_t make_order(const HierDev& H, const pndf_query* q, int64_t nq, uint32_t** order, hipStream_t s);
// The same in the library's static per-GPU workspace (no allocation), for batches of
// at most kStaticOrderQueries queries; the order must not be freed.
constexpr int64_t kStaticOrderQueries = (int64_t)1 << 22;
hipError_t make_order_static(const HierDev& H, const pndf_query* q, int64_t nq, uint32_t** order, hipStream_t s);
// Bucket count and coordinate shift of the spatial order for a map of side 2^logn.
void order_shape(int logn, int* nb, int* bshift);
void free_order(uint32_t* order, hipStream_t s);

// ---------------------------------------------------------------- device side
#if defined(__HIPCC__)

__device__ __forceinline__ float cross2(float ax, float ay, float bx, float by)
{
    return fmaf(ax, by, -(ay * bx));
}

__device__ __forceinline__ int floor_div_pow2(int a, int logn) { return a >> logn; }
__device__ __forceinline__ int ceil_div_pow2(int a, int logn) { return -((-a) >> logn); }

// Per-query constants, identical for every lane of the wave that owns the query.
struct QuerySetup {
    int kernel;                  // PNDF_KERNEL_*
    float rx, ry;                // support half-widths (disk / box radii)
    float x, y, hx, hy;
    int cxlo, cxhi, cylo, cyhi;  // included unrolled cell range per axis
    int l0;                      // entry level
    float t;                     // cut threshold fl(fl(rx ry) tau)
    uint32_t hkey;               // order keys (half_key) of h rounded to halves: x | y << 16
    double kx, ky;               // Gaussian: log2(e) / (2 sigma^2)
    double norm;                 // the kernel's peak: 1 / (2 pi sx sy), 1 / (pi rx ry) or 1 / (4 rx ry)
    int fexp;                    // binary point of the exact accumulator (units of 2^fexp)
    bool valid;
};

// Support box, entry level and kernel constants of one query (see pndf.h).
__device__ inline QuerySetup setup_query(const pndf_query& qr, float s2r, float tau, int L,
                                         float eps, int kernel)
{
    QuerySetup q;
    q.kernel = kernel;
    q.x = qr.x; q.y = qr.y; q.hx = qr.hx; q.hy = qr.hy;
    const float lim = 16777216.0f;
    bool ok = isfinite(qr.x) && isfinite(qr.y) && isfinite(qr.sx) && isfinite(qr.sy) &&
              isfinite(qr.hx) && isfinite(qr.hy) && qr.sx > 0.f && qr.sy > 0.f;
    float rx = __fmul_rn(s2r, qr.sx), ry = __fmul_rn(s2r, qr.sy);
    ok = ok && fabsf(qr.x) <= lim && fabsf(qr.y) <= lim && rx <= lim && ry <= lim;
    q.valid = ok;
    q.rx = rx;
    q.ry = ry;
    q.hkey = half_key(__half_as_ushort(__float2half_rn(qr.hx))) |
             (half_key(__half_as_ushort(__float2half_rn(qr.hy))) << 16);
    if (!ok) {
        q.cxlo = q.cylo = 0; q.cxhi = q.cyhi = -1; q.l0 = 0; q.t = -1.f;
        q.kx = q.ky = q.norm = 0.0;
        q.fexp = 0;
        return q;
    }
    float lox = __fsub_rn(qr.x, rx), hix = __fadd_rn(qr.x, rx);
    float loy = __fsub_rn(qr.y, ry), hiy = __fadd_rn(qr.y, ry);
    q.cxlo = (int)ceilf(lox) - 1; q.cxhi = (int)floorf(hix);
    q.cylo = (int)ceilf(loy) - 1; q.cyhi = (int)floorf(hiy);
    float rmax = fmaxf(rx, ry);
    int l0 = 0;
    while (l0 < L && (float)(1 << l0) < rmax) l0++;
    q.l0 = l0;
    q.t = tau > 0.f ? __fmul_rn(__fmul_rn(rx, ry), tau) : -1.f;
    const double log2e = 1.4426950408889634074;
    q.kx = log2e / (2.0 * (double)qr.sx * (double)qr.sx);
    q.ky = log2e / (2.0 * (double)qr.sy * (double)qr.sy);
    const double pi = 3.14159265358979323846;
    const double norm = kernel == PNDF_KERNEL_BOX    ? 1.0 / (4.0 * (double)rx * (double)ry)
                        : kernel == PNDF_KERNEL_DISK ? 1.0 / (pi * (double)rx * (double)ry)
                                                     : 1.0 / (2.0 * pi * (double)qr.sx * (double)qr.sy);
    q.norm = norm;
    // Every term is at most norm / eps per included cell image and triangle (node
    // images of a cluster reach at most one cell beyond the box per side), so
    // D < bound = 2 (nx + 2) (ny + 2) norm / eps.  The exact accumulator counts in
    // units of 2^fexp with bound < 2^(fexp + 190): 192 bits hold any D, and every
    // float32 term down to bound 2^-190 is represented exactly.
    const double bound = 2.0 * ((double)(q.cxhi - q.cxlo) + 3.0) * ((double)(q.cyhi - q.cylo) + 3.0) *
                         norm / (double)eps;
    int e2;
    frexp(bound, &e2);
    q.fexp = e2 + 1 - 190;
    return q;
}

// The setup of a query owned by a whole wave is the same in every lane: keep it in
// scalar registers (frees vector registers for the traversal).
__device__ __forceinline__ float uniform_f32(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double uniform_f64(double v)
{
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ unsigned long long uniform_u64(unsigned long long v)
{
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ QuerySetup uniform_query(const QuerySetup& q)
{
    QuerySetup u;
    u.kernel = __builtin_amdgcn_readfirstlane(q.kernel);
    u.rx = uniform_f32(q.rx); u.ry = uniform_f32(q.ry);
    u.x = uniform_f32(q.x); u.y = uniform_f32(q.y); u.hx = uniform_f32(q.hx); u.hy = uniform_f32(q.hy);
    u.cxlo = __builtin_amdgcn_readfirstlane(q.cxlo); u.cxhi = __builtin_amdgcn_readfirstlane(q.cxhi);
    u.cylo = __builtin_amdgcn_readfirstlane(q.cylo); u.cyhi = __builtin_amdgcn_readfirstlane(q.cyhi);
    u.l0 = __builtin_amdgcn_readfirstlane(q.l0);
    u.t = uniform_f32(q.t);
    u.hkey = (uint32_t)__builtin_amdgcn_readfirstlane((int)q.hkey);
    u.kx = uniform_f64(q.kx); u.ky = uniform_f64(q.ky); u.norm = uniform_f64(q.norm);
    u.fexp = __builtin_amdgcn_readfirstlane(q.fexp);
    u.valid = __builtin_amdgcn_readfirstlane((int)q.valid) != 0;
    return u;
}

// Bits [64 w, 64 w + 64) of m 2^sh for s = sh - 64 w (m < 2^53): m << s for
// 0 <= s < 64, m >> -s for -64 < s < 0, else 0 (the hardware takes shift counts
// mod 64, hence the selects).
__device__ __forceinline__ uint64_t fix_word(uint64_t m, int s)
{
    const uint64_t up = m << (s & 63), dn = m >> ((-s) & 63);
    return s >= 0 ? (s < 64 ? up : 0ull) : (s > -64 ? dn : 0ull);
}

// FP64 term t >= 0 added exactly down to 2^fexp: t = m 2^(ex - 1075) = (m 2^sh) 2^fexp,
// sh <= 136 since t < 2^(fexp + 189).  Branch-free: the lanes of a wave hold terms of
// different magnitudes, and a branch per word range would run every range.
__device__ __forceinline__ void fix_add_term(Fix192& a, double t, int fexp)
{
    const uint64_t b = (uint64_t)__double_as_longlong(t);
    int ex = (int)((b >> 52) & 0x7ffu);
    uint64_t m = b & 0xfffffffffffffull;
    if (ex) m |= 0x10000000000000ull; else ex = 1;
    const int sh = ex - 1075 - fexp;
    const uint64_t v0 = fix_word(m, sh), v1 = fix_word(m, sh - 64), v2 = fix_word(m, sh - 128);
    const uint64_t r0 = a.w0 + v0;
    const uint64_t c0 = r0 < v0 ? 1u : 0u;
    const uint64_t t1 = a.w1 + v1;
    const uint64_t c1 = t1 < v1 ? 1u : 0u;
    const uint64_t r1 = t1 + c0;
    const uint64_t c1b = r1 < c0 ? 1u : 0u;
    a.w0 = r0;
    a.w1 = r1;
    a.w2 += v2 + c1 + c1b;
}

__device__ __forceinline__ void fix_add(Fix192& a, const Fix192& b)
{
    const uint64_t r0 = a.w0 + b.w0;
    const uint64_t c0 = r0 < b.w0 ? 1u : 0u;
    const uint64_t t1 = a.w1 + b.w1;
    const uint64_t c1 = t1 < b.w1 ? 1u : 0u;
    const uint64_t r1 = t1 + c0;
    const uint64_t c1b = r1 < c0 ? 1u : 0u;
    a.w0 = r0;
    a.w1 = r1;
    a.w2 += b.w2 + c1 + c1b;
}

__device__ __forceinline__ float fix_to_float(const Fix192& a, int fexp)
{
    const double d = ((double)a.w2 * 18446744073709551616.0 + (double)a.w1) * 18446744073709551616.0 +
                     (double)a.w0;
    return (float)ldexp(d, fexp);
}

// Does a node of side `side` starting at torus cell `start` have a periodic image
// [start + pN, start + side - 1 + pN] wholly inside the unrolled cell range
// [clo, chi]?  Yes iff the first image starting at or after clo ends by chi.
__device__ __forceinline__ bool axis_inside(int start, int side, int clo, int chi, int logn)
{
    return start + (ceil_div_pow2(clo - start, logn) << logn) + side - 1 <= chi;
}

// Sum over the included periodic images of one axis of exp(-d^2 / (2 sigma^2)),
// d = start + p N + uoff - x; node of side `side` (1 for a texel cell).  The
// exponent a = d^2 log2(e) / (2 sigma^2) is split into floor(a) (an exact power of
// two, ldexp) and a fraction (float32 exp2), so nothing underflows before the
// FP64 product.
__device__ __forceinline__ double exp2_neg_split(double a)
{
    const double ai = floor(a);
    return ldexp((double)exp2f(-(float)(a - ai)), -(int)fmin(ai, 2000.0));
}

__device__ inline double gauss_axis(float x, double k, int start, int side, double uoff, int clo,
                                    int chi, int logn)
{
    int p0 = ceil_div_pow2(clo - start - side + 1, logn);
    int p1 = floor_div_pow2(chi - start, logn);
    double g = 0.0;
    double base = (double)start + uoff - (double)x;
    for (int p = p0; p <= p1; ++p) {
        const double d = base + (double)p * (double)(1 << logn);
        g += exp2_neg_split(d * d * k);
    }
    return g;
}

// Both axes of the Gaussian footprint.  When each axis has a single included image
// (every footprint narrower than the map, away from none of its wraps) the product
// of the two factors is one exponential of the summed exponents.
__device__ inline double gauss_2d(const QuerySetup& q, int sx, int sy, int side, double ux, double uy, int logn)
{
    const int px = ceil_div_pow2(q.cxlo - sx - side + 1, logn), py = ceil_div_pow2(q.cylo - sy - side + 1, logn);
    if (px == floor_div_pow2(q.cxhi - sx, logn) && py == floor_div_pow2(q.cyhi - sy, logn)) {
        const double period = (double)(1 << logn);
        const double dx = (double)sx + ux - (double)q.x + (double)px * period;
        const double dy = (double)sy + uy - (double)q.y + (double)py * period;
        return exp2_neg_split(dx * dx * q.kx + dy * dy * q.ky);
    }
    return gauss_axis(q.x, q.kx, sx, side, ux, q.cxlo, q.cxhi, logn) *
           gauss_axis(q.y, q.ky, sy, side, uy, q.cylo, q.cyhi, logn);
}

// Replacement-triangle vertices (circumradius rho around c, at 90/210/330 degrees).
__device__ __forceinline__ void eqtri_f32(float cx, float cy, float rho, float v[6])
{
    const float c30 = 0.86602540378443864676f;
    v[0] = cx;                     v[1] = cy + rho;
    v[2] = cx - rho * c30;         v[3] = cy - 0.5f * rho;
    v[4] = cx + rho * c30;         v[5] = cy - 0.5f * rho;
}

__device__ __forceinline__ void eqtri_f64(double cx, double cy, double rho, double v[6])
{
    const double c30 = 0.86602540378443864676;
    v[0] = cx;                     v[1] = cy + rho;
    v[2] = cx - rho * c30;         v[3] = cy - 0.5 * rho;
    v[4] = cx + rho * c30;         v[5] = cy - 0.5 * rho;
}

// Inclusive point-in-triangle test in float32 with the cyclic edge functions of the
// vertex offsets q_k = v_k - h: lambda_0 ~ q_b x q_c, lambda_1 ~ q_c x q_a,
// lambda_2 ~ q_a x q_b (all of one sign inside, whatever the orientation).
__device__ __forceinline__ bool tri_hit_f32(const float v[6], float hx, float hy)
{
    float ax = v[0] - hx, ay = v[1] - hy, bx = v[2] - hx, by = v[3] - hy;
    float cx = v[4] - hx, cy = v[5] - hy;
    float e0 = cross2(bx, by, cx, cy), e1 = cross2(cx, cy, ax, ay), e2 = cross2(ax, ay, bx, by);
    return (e0 >= 0.f && e1 >= 0.f && e2 >= 0.f) || (e0 <= 0.f && e1 <= 0.f && e2 <= 0.f);
}

// Contribution of a hit: the triangle's uv vertices are (a, b, c) =
// lower: (U0, U0 + s e_x, U0 + s e_y), upper: (U3, U3 - s e_x, U3 - s e_y) of the node
// (I, J) of side s = 2^lev (lev = 0: texel cell), so u* = corner +- s (l1, l2).
// Box footprint along one axis: the number of included periodic images of the
// point start + uoff within r of x.
__device__ inline double box_axis(float x, float r, int start, int side, double uoff, int clo, int chi, int logn)
{
    const int p0 = ceil_div_pow2(clo - start - side + 1, logn);
    const int p1 = floor_div_pow2(chi - start, logn);
    const double base = (double)start + uoff - (double)x;
    double c = 0.0;
    for (int p = p0; p <= p1; ++p) c += fabs(base + (double)p * (double)(1 << logn)) <= (double)r ? 1.0 : 0.0;
    return c;
}

// Disk footprint: the number of included periodic images of the point inside the
// ellipse of half-axes (rx, ry) around x.
__device__ inline double disk_images(const QuerySetup& q, int sx0, int sy0, int side, double ux, double uy, int logn)
{
    const int p0 = ceil_div_pow2(q.cxlo - sx0 - side + 1, logn), p1 = floor_div_pow2(q.cxhi - sx0, logn);
    const int r0 = ceil_div_pow2(q.cylo - sy0 - side + 1, logn), r1 = floor_div_pow2(q.cyhi - sy0, logn);
    const double bx = (double)sx0 + ux - (double)q.x, by = (double)sy0 + uy - (double)q.y;
    const double period = (double)(1 << logn);
    double c = 0.0;
    for (int p = p0; p <= p1; ++p) {
        const double dx = (bx + (double)p * period) / (double)q.rx;
        for (int r = r0; r <= r1; ++r) {
            const double dy = (by + (double)r * period) / (double)q.ry;
            c += dx * dx + dy * dy <= 1.0 ? 1.0 : 0.0;
        }
    }
    return c;
}

// (the footprint kernel KER is a template parameter: each kernel's evaluation code
// is compiled separately, so the Gaussian path carries none of the others' registers)
// The footprint weight of a hit, norm k(u*), without the division by the Jacobian.
template <int KER>
__device__ inline double hit_weight(const QuerySetup& q, int I, int J, int lev, int half, double l1,
                                    double l2, int logn)
{
    const int s = 1 << lev;
    double ux = half ? (double)s * (1.0 - l1) : (double)s * l1;
    double uy = half ? (double)s * (1.0 - l2) : (double)s * l2;
    double w;
    if constexpr (KER == PNDF_KERNEL_BOX) {
        w = box_axis(q.x, q.rx, I * s, s, ux, q.cxlo, q.cxhi, logn) *
            box_axis(q.y, q.ry, J * s, s, uy, q.cylo, q.cyhi, logn);
    } else if constexpr (KER == PNDF_KERNEL_DISK) {
        w = disk_images(q, I * s, J * s, s, ux, uy, logn);
    } else {
        w = gauss_2d(q, I * s, J * s, s, ux, uy, logn);
    }
    return q.norm * w;
}

template <int KER>
__device__ inline double hit_term(const QuerySetup& q, int I, int J, int lev, int half, double l1,
                                  double l2, float det_used, int logn)
{
    return hit_weight<KER>(q, I, J, lev, half, l1, l2, logn) / (double)det_used;
}

__device__ __forceinline__ uint64_t tri_id(int lev, int I, int J, int half)
{
    return ((uint64_t)lev << 58) | ((uint64_t)J << 29) | ((uint64_t)I << 1) | (uint64_t)half;
}

__host__ __device__ __forceinline__ uint32_t morton_spread(uint32_t v)
{
    v &= 0xffffu;
    v = (v | (v << 8)) & 0x00ff00ffu;
    v = (v | (v << 4)) & 0x0f0f0f0fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

__host__ __device__ __forceinline__ uint32_t morton_compact(uint32_t v)
{
    v &= 0x55555555u;
    v = (v | (v >> 1)) & 0x33333333u;
    v = (v | (v >> 2)) & 0x0f0f0f0fu;
    v = (v | (v >> 4)) & 0x00ff00ffu;
    v = (v | (v >> 8)) & 0x0000ffffu;
    return v;
}

__host__ __device__ __forceinline__ uint32_t morton(uint32_t i, uint32_t j)
{
    return morton_spread(i) | (morton_spread(j) << 1);
}

// Block index -> logical index so that each XCD (workgroups are dispatched to the
// kXcd dies round-robin) walks a contiguous range of the processing order.
constexpr int kXcd = 8;
__device__ __forceinline__ int64_t xcd_contiguous(int64_t b, int64_t nblocks)
{
    const int64_t x = b % kXcd, k = b / kXcd;
    const int64_t per = (nblocks + kXcd - 1) / kXcd, r = nblocks % kXcd;
    if (r == 0) return x * per + k;
    return (x < r ? x * per : r * per + (x - r) * (per - 1)) + k;
}

// Wave-level helpers (wave64).
__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0)); }

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Exclusive prefix over the wave of a per-lane count in [0, 7], and the total.
__device__ __forceinline__ int wave_prefix_small(int c, int* total)
{
    uint64_t b0 = __ballot(c & 1), b1 = __ballot(c & 2), b2 = __ballot(c & 4);
    uint64_t lt = (1ull << lane_id()) - 1ull;
    *total = __popcll(b0) + 2 * __popcll(b1) + 4 * __popcll(b2);
    return __popcll(b0 & lt) + 2 * __popcll(b1 & lt) + 4 * __popcll(b2 & lt);
}

__device__ __forceinline__ double wave_sum_f64(double v)
{
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Row shift of a 64-bit value by DPP (control 0x110 + n: row_shr n; lanes shifted in
// from outside the 16-lane row read 0).
template <int CTRL>
__device__ __forceinline__ uint64_t dpp_row_shr(uint64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, 0xf, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), CTRL, 0xf, 0xf, false);
    return ((uint64_t)hi << 32) | lo;
}

template <int CTRL>
__device__ __forceinline__ void fix_add_row_shr(Fix192& v)
{
    Fix192 w;
    w.w0 = dpp_row_shr<CTRL>(v.w0);
    w.w1 = dpp_row_shr<CTRL>(v.w1);
    w.w2 = dpp_row_shr<CTRL>(v.w2);
    fix_add(v, w);
}

__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int lane)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

// Exact sum over the wave (every lane must be active): within each row of 16 lanes
// by DPP row shifts 1, 2, 4, 8 (lane 15 of the row then holds the row's sum), then
// the four row sums read from lanes 15, 31, 47 and 63.
__device__ __forceinline__ Fix192 wave_sum_fix(Fix192 v)
{
    fix_add_row_shr<0x111>(v);
    fix_add_row_shr<0x112>(v);
    fix_add_row_shr<0x114>(v);
    fix_add_row_shr<0x118>(v);
    Fix192 s;
    s.w0 = readlane_u64(v.w0, 15);
    s.w1 = readlane_u64(v.w1, 15);
    s.w2 = readlane_u64(v.w2, 15);
#pragma unroll
    for (int r = 1; r < 4; ++r) {
        Fix192 t;
        t.w0 = readlane_u64(v.w0, 16 * r + 15);
        t.w1 = readlane_u64(v.w1, 16 * r + 15);
        t.w2 = readlane_u64(v.w2, 16 * r + 15);
        fix_add(s, t);
    }
    return s;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v)
{
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

#endif  // __HIPCC__

}  // namespace pndf
