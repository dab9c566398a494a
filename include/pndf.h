/*
 * pndf.h - C ABI of the MI355X (gfx950) library for batched evaluation of the
 * manifold-based patch normal distribution function (P-NDF) of
 * "Position-Normal Manifold for Efficient Glint Rendering on High-Resolution
 * Normal Maps" (arXiv 2505.08985).
 *
 * The problem, in the paper's notation (section "Preliminaries", Eq. gndf):
 *   D(m, x) = integral of k_r(u - x) delta(n(u) - m) du
 *           = sum over preimages u_i of m of k_r(u_i - x) / |det J(u_i)|,
 * where n(u) is the normal map made continuous by two triangles per texel cell
 * (Eq. interpolation), det J is twice the normal-space triangle area
 * (Eq. jacobian), and the sum is found by point-in-normal-triangle tests with
 * barycentric recovery of u (Eq. ndf_eval), accelerated by a min-max hierarchy and
 * a least-squares cluster hierarchy (section "Acceleration by mesh clustering").
 *
 * Conventions used by every entry point
 *   - Texture coordinates are unnormalised texel units; texel (i, j) sits at (i, j)
 *     (Table notation).  The map is periodic (a torus): cell (N-1, j) connects to
 *     texel column 0, and footprints wider than the map sum every periodic image.
 *   - Normals and query normals are the xy components of unit vectors on the
 *     projected hemisphere (section "Preliminaries").
 *   - The footprint kernel is by default the normalised axis-aligned Gaussian of
 *     standard deviations (sx, sy); its support half-width is r = sigma_to_r * sigma
 *     (3 by default: the "(6 sigma)^2 footprint" of the ablation section), truncated
 *     at texel-cell granularity: every triangle of every periodic cell image whose
 *     closed unit square meets [x - r, x + r] (r, x - r, x + r rounded to float32)
 *     contributes, with the untruncated Gaussian.  Disk and box kernels (see
 *     PNDF_KERNEL_*) use the same cells and weigh each hit point by the kernel.
 *   - Triangles with Jacobian below eps (evaluated in FP64 from the float32 normals,
 *     strict <) are replaced by an equilateral triangle of area eps/2 centred at the
 *     cell-centre normal n(floor(u) + 1/2) = (n1 + n2)/2 (section "Preventing
 *     Jacobian singularity", Eq. debias); its vertices sit at 90, 210, 330 degrees,
 *     assigned to the triangle's (a, b, c).
 *   - Device pointers are HIP device (HBM) addresses; `stream` is a hipStream_t
 *     (NULL = the default stream).  Every call returns a pndf_status and never
 *     aborts; pndf_last_error() gives a thread-local message for the last failure.
 */
#ifndef PNDF_H
#define PNDF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pndf_mesh pndf_mesh; /* opaque, immutable after build */
typedef struct pndf_hier pndf_hier; /* opaque, immutable after build; holds a reference to its mesh */

typedef enum pndf_status {
    PNDF_OK = 0,
    PNDF_EINVAL = 1,      /* invalid argument (null pointer, bad size, out-of-range option or map value) */
    PNDF_ENOMEM = 2,      /* device or host allocation failed */
    PNDF_EDEVICE = 3,     /* a HIP runtime call failed (including an earlier asynchronous fault) */
    PNDF_EOVERFLOW = 4,   /* a caller-provided buffer is too small; the required size is reported */
    PNDF_EUNSUPPORTED = 5,/* valid request that this library does not implement (e.g. N > 8192) */
    PNDF_EAGAIN = 6       /* serving: admission refused for now (memory or slots); retry later */
} pndf_status;

/* One query: footprint centre (x, y) in texel units, Gaussian standard deviations
 * (sx, sy) in texels, query normal (hx, hy) on the projected hemisphere.  24 bytes,
 * arrays of queries are tightly packed.  A query with a non-finite field, sx <= 0,
 * sy <= 0, |x| or |y| above 2^24, or r above 2^24 evaluates to NaN (not a batch
 * error).  A query normal outside every normal triangle evaluates to 0. */
typedef struct pndf_query {
    float x, y, sx, sy, hx, hy;
} pndf_query;

/* Footprint kernels (Table notation: k_r of size 2 r_x x 2 r_y, zero beyond r).
 * r = sigma_to_r * sigma per axis (float32 product) for every kernel.
 *   GAUSSIAN  the normalised Gaussian of standard deviations (sx, sy), evaluated
 *             untruncated at every contributing hit (cells meeting the support box);
 *   DISK      1 / (pi r_x r_y) inside the ellipse of half-axes r around x, 0 outside;
 *   BOX       1 / (4 r_x r_y) where |u - x| <= r per axis, 0 outside.
 * DISK and BOX are truncated at the hit point (u* outside the support weighs 0; the
 * triangle still counts as hit).  The ablation section ("Different footprint
 * kernel") matches a Gaussian's (6 sigma)^2 footprint with a disk / box of
 * (3 sigma)^2, i.e. sigma_to_r = 1.5 for the disk / box against 3 for the Gaussian. */
enum { PNDF_KERNEL_GAUSSIAN = 0, PNDF_KERNEL_DISK = 1, PNDF_KERNEL_BOX = 2 };

/* Evaluation algorithm.  All give the same result (the set of triangles is fixed
 * by the definition, not by the algorithm); they differ in speed. */
enum {
    PNDF_ALGO_AUTO = 0,       /* plain hierarchical traversal */
    PNDF_ALGO_BRUTE = 1,      /* every triangle of every included cell, no hierarchy (tau must be 0) */
    PNDF_ALGO_PLAIN = 2,      /* one wavefront per query, min-max (+ cluster cut) traversal */
    PNDF_ALGO_PERSISTENT = 3  /* persistent work-stealing traversal: needs a plan (pndf_plan_create) */
};

typedef struct pndf_eval_opts {
    int32_t kernel;     /* PNDF_KERNEL_GAUSSIAN, _DISK or _BOX (anything else -> PNDF_EINVAL) */
    float tau;          /* cluster cut threshold: a node of level l >= 1 at or below the entry level is
                         * used as two cluster triangles when e^l <= fl(fl(r_x r_y) tau); 0 = exact */
    float sigma_to_r;   /* support half-width r = sigma_to_r * sigma; the paper's Gaussian uses 3 */
    int32_t algo;       /* PNDF_ALGO_* */
    int32_t flags;      /* PNDF_EVAL_INPUT_ORDER or 0 */
} pndf_eval_opts;

/* Batches of 4096 or more queries are processed in a spatial order (Morton buckets
 * of the footprint centres) for cache locality; results do not depend on the order.
 * This flag keeps the caller's order instead. */
enum { PNDF_EVAL_INPUT_ORDER = 1 };

typedef struct pndf_hier_opts {
    int32_t cluster;    /* 1: fit the cluster hierarchy (needed for tau > 0); 0: min-max only */
} pndf_hier_opts;

/*
 * Build the triangle mesh of a normal map (Fig. normal_map, Eq. interpolation,
 * Eq. jacobian, section "Preventing Jacobian singularity").
 *   normals  device pointer, N*N*2 float32, row-major (x, y) pairs, index (j*N + i)*2 with
 *            i along u; every |n| must be < 1 and finite (else PNDF_EINVAL)
 *   n        map side N: a power of two, 2 <= N <= 8192 (N > 8192: PNDF_EUNSUPPORTED)
 *   eps      Jacobian clamp threshold (the paper uses 1e-6); must be > 0 and finite
 *   out      receives the mesh handle (library-owned HBM: the padded normal planes, per-cell
 *            clamp bits and FP64-derived Jacobians)
 * The input is copied: the caller may free it once this call returns.  The call
 * synchronises `stream` (it validates the map on the device and reads the result).
 */
pndf_status pndf_build_mesh(const float* normals, int32_t n, float eps, void* stream,
                            pndf_mesh** out);

/*
 * Build the acceleration hierarchies of a mesh (section "Acceleration by mesh
 * clustering"; supplement "Derivations of Cluster Normal Optimization"):
 *   - the min-max hierarchy: for every 2^l x 2^l node (l = 1..log2 N) the normal-space
 *     bounding box of every triangle beneath it (clamped triangles by their replacement);
 *   - with opts->cluster: four cluster normals per node minimising the inverse-Jacobian
 *     weighted squared distance between the cluster's two-triangle interpolant and the
 *     map (Eq. normal_optimization), the minimised objective e^l (in texel-area units),
 *     the cluster triangles' Jacobians (2 area / 4^l, clamped at eps like the map's), and
 *     a second bounding-box hierarchy that also covers the cluster triangles.
 * opts may be NULL (cluster = 1).  The mesh must outlive nothing: the hierarchy keeps
 * a reference, so the caller may destroy the mesh handle at any time.  Synchronises
 * `stream`.
 */
pndf_status pndf_build_hierarchy(const pndf_mesh* mesh, const pndf_hier_opts* opts, void* stream,
                                 pndf_hier** out);

/*
 * Evaluate D(m, x) (Eq. ndf_eval) for nq queries.
 *   d_q    device pointer to nq pndf_query records (caller-owned)
 *   nq     number of queries, >= 0 (0 is a no-op)
 *   opts   may be NULL (Gaussian, tau = 0, sigma_to_r = 3, auto algorithm)
 *   d_out  device pointer to nq float32 results (caller-owned)
 * Asynchronous and stream-ordered; the caller keeps d_q and d_out alive until the
 * stream's work completes.  Deterministic: each query's result depends only on that
 * query and the hierarchy, bit for bit, whatever else is in the batch.  tau > 0
 * needs a hierarchy built with clusters (else PNDF_EINVAL).
 */
pndf_status pndf_eval_batch(const pndf_hier* h, const pndf_query* d_q, int64_t nq,
                            const pndf_eval_opts* opts, float* d_out, void* stream);

/*
 * pndf_eval_batch for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * results, bit for bit, with the spatial-order workspace taken from a static
 * array of the library (one per GPU, 32 MiB + 16 KiB, held until the process
 * ends) instead of a stream-ordered allocation.  nq is limited to 2^22 (larger:
 * PNDF_EINVAL, nothing launched); no hipMalloc, hipFree or allocating library call
 * is made (the array's device address is looked up once per device, on the first
 * call there).  Every call on a GPU shares that GPU's array: calls that overlap
 * on one GPU (different streams or threads, not ordered by the caller) race and
 * give wrong results; order them on one stream.  Arguments, ownership and errors
 * as for pndf_eval_batch.
 */
pndf_status pndf_eval_batch_noalloc(const pndf_hier* h, const pndf_query* d_q, int64_t nq,
                                    const pndf_eval_opts* opts, float* d_out, void* stream);

/*
 * As pndf_eval_batch, plus per-query work counters (debug/roofline accounting):
 *   d_counts  device pointer to nq * 4 uint32: nodes tested, leaf cells tested,
 *             cluster nodes used, hit triangles (for the brute-force algorithm the
 *             node count is 0).
 * The values of d_out are identical to pndf_eval_batch's.
 */
pndf_status pndf_eval_counts(const pndf_hier* h, const pndf_query* d_q, int64_t nq,
                             const pndf_eval_opts* opts, float* d_out, uint32_t* d_counts,
                             void* stream);

/*
 * As pndf_eval_batch, plus the list of hit triangles of every query, for parity
 * checks: CSR offsets d_offsets[nq + 1] (uint64, d_offsets[0] = 0), triangle ids
 * d_ids[] and per-hit terms d_terms[] (float32: kernel weight summed over included
 * periodic images, divided by the clamped Jacobian).  A triangle id packs
 * (level << 58) | (J << 29) | (I << 1) | half: level 0 is a texel cell (I, J) and
 * half 0 its lower triangle (u0, u1, u2), 1 its upper (u3, u2, u1); level >= 1 is a
 * cluster node (I, J) of that level and its lower/upper cluster triangle.
 * capacity is the length of d_ids and d_terms.  If the total number of hits exceeds
 * it, returns PNDF_EOVERFLOW with *required set (d_out and d_offsets are still
 * written).  Synchronises `stream` (two passes: count, then fill).
 */
pndf_status pndf_eval_hits(const pndf_hier* h, const pndf_query* d_q, int64_t nq,
                           const pndf_eval_opts* opts, float* d_out, uint64_t* d_offsets,
                           uint64_t* d_ids, float* d_terms, uint64_t capacity,
                           uint64_t* required, void* stream);

/*
 * Sampling of the P-NDF (section "Sampling and evaluation", Eq. debias; with
 * tau > 0 the cluster field of the cut, section "Acceleration by mesh
 * clustering"), consistent with pndf_eval_batch: for query k (x, y, sx, sy used,
 * hx, hy ignored) it draws u from the footprint kernel over the support the
 * evaluation integrates and returns the normal m of the triangle (or, with the
 * cut, the cluster triangle) containing u, warped onto the replacement
 * triangle when that triangle is clamped.  The density of m is D(m) over D's
 * total mass, for each kernel and tau.
 *
 *  d_xi       device, 16-byte aligned, attempts x nq pairs of uniforms in [0, 1), attempt-major:
 *             pair t of query k at d_xi[2 (t nq + k)], d_xi[2 (t nq + k) + 1].
 *             The caller draws them (any generator).  The Gaussian footprint is
 *             drawn by inverse CDF per axis; with tau > 0 a draw whose cut unit
 *             lies outside the included cells is rejected and the next pair is
 *             used (a first draw is rejected with probability of order 1e-2);
 *             disk and box draws (uniform on the ellipse / rectangle) and tau = 0
 *             use the first pair only.
 *  attempts   >= 1 pairs per query.
 *  opts       kernel, tau, sigma_to_r as for pndf_eval_batch (algo ignored,
 *             flags must be 0); tau > 0 needs clusters.
 *  d_m        device, 8-byte aligned, nq float2: the sampled normal; NaN when the query is
 *             invalid (as for the evaluation), a used pair lies outside [0, 1),
 *             or every attempt was rejected.
 *  d_tri      device, nq triangle ids (same encoding as pndf_eval_hits), ~0 when
 *             m is NaN; may be NULL.
 *  d_u        device, 16-byte aligned, nq double2: the drawn texture coordinates (unrolled, not
 *             wrapped onto the torus; the last draw when all were rejected); may
 *             be NULL.
 * Asynchronous on `stream`; deterministic.
 */
pndf_status pndf_sample_batch(const pndf_hier* h, const pndf_query* d_q, int64_t nq, const double* d_xi,
                              int32_t attempts, const pndf_eval_opts* opts, float* d_m, uint64_t* d_tri,
                              double* d_u, void* stream);

/*
 * Projected area of the P-NDF for shadow-masking (section "Shadow-masking",
 * Eq. lambda, Eq. area-integral, Eq. line-integral):
 *   P(w) = integral of D(m, x) max(m~ . w, 0) over the solid angle of the unit
 *          normal m~ = (m, sqrt(1 - |m|^2)),
 * with the footprint kernel taken constant over each triangle (its value at the
 * triangle's uv centroid, summed over the included periodic images; exact for a
 * box whose support contains the triangles).  Computed by brute force over every
 * triangle of every included cell, each by rotation to w_y = 0, clipping to the
 * visible region and closed-form boundary integrals (Stokes).  Then
 *   Lambda(w) = P(w) / w_z - 1,
 *   G(w_i, w_o, m) = H(m~ . w_i) H(m~ . w_o) / ((1 + Lambda(w_i)) (1 + Lambda(w_o))),
 *   aggregated diffuse BRDF f_d = P(w_i) / (pi w_iz).
 *
 *  d_q       device, nq queries: x, y, sx, sy as for pndf_eval_batch; the last two
 *            floats (hx, hy) carry w_x, w_y of the unit direction w, whose w_z is
 *            sqrt(1 - w_x^2 - w_y^2) (the upper hemisphere).
 *  opts      kernel and sigma_to_r; tau must be 0; algo ignored; flags must be 0.
 *  d_P       device, nq floats: P(w); NaN for an invalid query (as for the
 *            evaluation) or w_x^2 + w_y^2 > 1.
 *  d_lambda  device, nq floats: Lambda(w) (+inf at w_z = 0); may be NULL.
 * Queries run heaviest first (by their number of included cells), which changes
 * no result; the order's workspace (8 bytes per query) is allocated and freed
 * stream-ordered.  Asynchronous on `stream`; deterministic.
 */
pndf_status pndf_projected_area(const pndf_hier* h, const pndf_query* d_q, int64_t nq, const pndf_eval_opts* opts,
                                float* d_P, float* d_lambda, void* stream);

/* Release handles (no work may be in flight on them).  NULL is ignored. */
void pndf_destroy_mesh(pndf_mesh* mesh);
void pndf_destroy_hierarchy(pndf_hier* h);

const char* pndf_status_string(pndf_status s);
const char* pndf_last_error(void);

/* ---- persistent work-stealing evaluation ----------------------------------
 *
 * A plan owns the workspace of the persistent traversal for batches of up to
 * max_nq queries: a fixed grid of workers (compute units x blocks_per_cu blocks of
 * four wavefronts) takes queries, in the same spatial order as pndf_eval_batch
 * (unless PNDF_EVAL_INPUT_ORDER), from a global counter.  Once no query is left to
 * take, idle workers wait in a global ticket queue and raise a flag; a busy wave
 * that sees it hands out up to half of the nodes of its highest pending level (if
 * that level is at least split_level), at most one per waiting worker, as tasks of
 * that queue; stolen subtrees are split again
 * the same way, so one huge footprint ends up spread over the whole GPU.  Each
 * query's terms are summed exactly (192-bit fixed point), so the result is
 * bit-identical to pndf_eval_batch whatever the split, the schedule or the batch
 * composition.  The launch sequence (reset, spatial order, workers, finalize) is
 * instantiated once as a HIP graph and replayed per batch.
 */
typedef struct pndf_plan pndf_plan;

typedef struct pndf_tuning {
    int32_t blocks_per_cu; /* worker blocks per compute unit (>= 1; more than fit on a compute
                            * unit at once, given the kernel's registers and LDS, run as that many) */
    int32_t split_level;   /* smallest level whose nodes may be donated, 1..log2 N */
    int32_t queue_factor;  /* task-queue slots per query of max_nq (>= 1); a donation that does not
                            * fit stays with its wave, so capacity only affects balance */
    int32_t use_graph;     /* 1: replay the instantiated graph; 0: three plain launches */
} pndf_tuning;

typedef struct pndf_plan_stats {
    uint64_t spawned;      /* subtrees donated to the queue in the last run */
    uint64_t refused;      /* nodes offered while the queue was full (kept by their wave) */
    uint64_t idle_spins;   /* worker polls that found no work (load-balance diagnostic) */
    uint32_t error;        /* nonzero: a worker gave up after 30 s without work arriving (bit0) or
                            * without a reserved task being published (bit1), or read a malformed
                            * task (bit2); the results of that run are invalid */
} pndf_plan_stats;

/* Default tuning for a hierarchy (used when pndf_plan_create gets tuning == NULL):
 * as many blocks per compute unit as are resident, split level log2 N - 3. */
pndf_status pndf_default_tuning(const pndf_hier* h, pndf_tuning* out);

/*
 * Create a plan for batches of at most max_nq (>= 1) queries with the given options
 * (opts->algo is ignored) and tuning (NULL: pndf_default_tuning).  The hierarchy must
 * outlive the plan.  Allocates device memory; synchronises `stream`.
 */
pndf_status pndf_plan_create(const pndf_hier* h, int64_t max_nq, const pndf_eval_opts* opts,
                             const pndf_tuning* tuning, void* stream, pndf_plan** out);

/*
 * Evaluate nq (0 <= nq <= max_nq) queries with the plan: same contract as
 * pndf_eval_batch (asynchronous, stream-ordered, deterministic).  Runs of one plan
 * must not overlap: order them on one stream (the plan's workspace is reused).
 */
pndf_status pndf_plan_eval(pndf_plan* plan, const pndf_query* d_q, int64_t nq, float* d_out,
                           void* stream);

/* The tuning the plan runs with (blocks_per_cu after the resident limit). */
pndf_status pndf_plan_get_tuning(const pndf_plan* plan, pndf_tuning* out);

/* Statistics of the plan's last run (synchronises `stream`). */
pndf_status pndf_plan_get_stats(pndf_plan* plan, pndf_plan_stats* out, void* stream);

void pndf_plan_destroy(pndf_plan* plan);

/*
 * Autotuner: time the persistent traversal on the given queries (a representative
 * sample of the workload) for every candidate tuning (blocks per compute unit in
 * {1, 2, 4, 6, 8} up to the resident limit, split level 2..8 within the map's levels,
 * graph replay; best of two timed runs after a warm-up) and return the fastest in
 * *best, with its time per batch in *best_ms (may be NULL).  The sample should load
 * the GPU like the batches the plan will run: on a much smaller batch the slowest
 * queries dominate and favour fewer workers.  Synchronises `stream`.
 */
pndf_status pndf_autotune(const pndf_hier* h, const pndf_query* d_q, int64_t nq,
                          const pndf_eval_opts* opts, pndf_tuning* best, double* best_ms,
                          void* stream);

/* ---- serving: continuous batching over resident maps ----------------------
 *
 * A server keeps one or more hierarchies resident and evaluates requests (for
 * example one render tile: a block of queries against one map) as they arrive.
 * A request is admitted when its pinned staging fits the memory budget and the
 * pending queue has room; otherwise pndf_server_submit returns PNDF_EAGAIN.  A
 * scheduler thread packs waiting requests of the same map into batches of up to
 * max_batch_queries: each waiting request gives a piece of at most chunk_queries
 * queries, and a request with queries left goes to the back of the queue, so
 * requests share the device piece by piece and a small request does not wait for
 * the whole of a large one.  Each batch runs on one of `slots` streams (a plain
 * per-batch launch, or the slot's persistent plan), so batches formed while others
 * execute overlap on the device (continuous batching).  Results are bit-identical
 * to pndf_eval_batch for the same queries, whatever batch or piece a query lands
 * in.  Latency is measured from submission (or the trace's arrival time) to the
 * moment all of a request's results are in host memory.
 */
typedef struct pndf_server pndf_server;

typedef struct pndf_server_opts {
    int32_t slots;              /* concurrent batches in flight (streams), 1..16 */
    int64_t max_batch_queries;  /* queries per batch (and the largest request), >= 1 */
    int64_t memory_budget;      /* bytes of pinned staging for admitted requests (28 B per query, plus
                                 * 256 B per request), >= one batch */
    int32_t max_pending;        /* admitted requests not yet finished, >= 1 */
    float tau;                  /* cluster cut threshold for every request (0 = exact) */
    float sigma_to_r;           /* support half-width in standard deviations (3) */
    pndf_tuning tuning;         /* persistent-plan tuning (blocks_per_cu = 0: default) */
    int32_t algo;               /* evaluation of a batch: PNDF_ALGO_PLAIN (or AUTO): one
                                 * pndf_eval_batch on the slot's stream; PNDF_ALGO_PERSISTENT:
                                 * the slot's persistent plan for the batch's map */
    int32_t kernel;             /* footprint kernel of every request (pndf_kernel) */
    int64_t chunk_queries;      /* largest piece of one request in one batch (0: whole requests) */
} pndf_server_opts;

typedef struct pndf_server_stats {
    uint64_t completed, refused;       /* requests finished / refused by admission */
    uint64_t queries, batches;         /* queries evaluated, batches launched */
    double p50_ms, p99_ms, max_ms;     /* request latency percentiles (completed requests) */
    double mean_batch_requests;        /* average requests per batch */
    double busy_s;                     /* wall time from first admission to last completion */
} pndf_server_stats;

/* Create a server over nmaps resident hierarchies (which must outlive it). */
pndf_status pndf_server_create(const pndf_hier* const* maps, int32_t nmaps, const pndf_server_opts* opts,
                               pndf_server** out);

/*
 * Submit a request: nq queries (host memory, copied at submission) against map
 * `map`; results are written to h_out (host memory, nq floats, caller-owned, valid
 * until the request completes).  *ticket identifies it.  PNDF_EAGAIN: not admitted
 * (memory budget or pending limit), nothing was queued.
 */
pndf_status pndf_server_submit(pndf_server* srv, int32_t map, const pndf_query* h_q, int64_t nq,
                               float* h_out, uint64_t* ticket);

/* Wait for a request (timeout_s < 0: forever).  *latency_ms (may be NULL) receives
 * its latency.  PNDF_EAGAIN on timeout. */
pndf_status pndf_server_wait(pndf_server* srv, uint64_t ticket, double timeout_s, double* latency_ms);

/* Wait until every admitted request has completed. */
pndf_status pndf_server_drain(pndf_server* srv);

pndf_status pndf_server_get_stats(pndf_server* srv, pndf_server_stats* out);

/* Clear the statistics (not the resident maps or plans). */
pndf_status pndf_server_reset_stats(pndf_server* srv);

/*
 * Replay an arrival trace: request k (map map_ids[k], nq[k] queries at h_q[k],
 * results to h_out[k]) is submitted arrival_s[k] seconds after the call starts,
 * retrying while it is refused; returns after every submitted request has
 * completed.  latency_ms[k] (may be NULL) receives each latency.  The whole trace
 * is validated first (arrival times finite, >= 0 and non-decreasing; map ids in
 * range; 1 <= nq[k] <= max_batch_queries; non-NULL buffers): PNDF_EINVAL and
 * nothing submitted.  If a submission fails later (a device error), the requests
 * already submitted are still waited for before the call returns that status, so
 * no result is written into h_out after the call.
 */
pndf_status pndf_server_replay(pndf_server* srv, int64_t nreq, const int32_t* map_ids,
                               const double* arrival_s, const pndf_query* const* h_q,
                               const int64_t* nq, float* const* h_out, double* latency_ms);

void pndf_server_destroy(pndf_server* srv);

/* ---- introspection, for parity checks of the build steps ----------------- */

/* Map side, clamp threshold and device bytes held by the mesh. */
pndf_status pndf_mesh_info(const pndf_mesh* mesh, int32_t* n, float* eps, int64_t* bytes);

/* Copy the mesh's per-cell clamp bits (N*N uint8: bit0 lower, bit1 upper clamped)
 * and Jacobians used by the evaluation (N*N*2 float32, lower then upper; eps for
 * clamped triangles) into caller device buffers.  Either pointer may be NULL. */
pndf_status pndf_mesh_export(const pndf_mesh* mesh, uint8_t* d_deg, float* d_det, void* stream);

/* Levels (log2 N), whether clusters were fitted, and device bytes of a hierarchy. */
pndf_status pndf_hier_info(const pndf_hier* h, int32_t* levels, int32_t* cluster, int64_t* bytes);

/* Copy level `level` (1..log2 N) of the hierarchy, (N >> level)^2 nodes in row-major
 * node order (J * (N >> level) + I), into caller device buffers (any may be NULL):
 *   d_bbox      4 float32 per node: min x, min y, max x, max y over the map's triangles
 *   d_bbox_all  the same box extended by every cluster triangle at or below the node
 *   d_bbox_clu  4 float32 per node: the box of the node's own two cluster triangles
 *               (what the cut traversal tests a node under the cut against)
 *   d_clu_n     8 float32 per node: cluster normals N0..N3 (corners (0,0),(1,0),(0,1),(1,1))
 *   d_clu_e     1 float32 per node: e^l
 *   d_clu_det   2 float32 per node: Jacobians of the lower/upper cluster triangle
 *               (eps when clamped)
 * The cluster arrays need a hierarchy built with clusters (else PNDF_EINVAL). */
pndf_status pndf_hier_export_level(const pndf_hier* h, int32_t level, float* d_bbox,
                                   float* d_bbox_all, float* d_bbox_clu, float* d_clu_n, float* d_clu_e,
                                   float* d_clu_det, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PNDF_H */
