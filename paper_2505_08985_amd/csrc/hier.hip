// Hierarchy build: min-max boxes and least-squares cluster normals per quad-tree
// node (section "Acceleration by mesh clustering"; supplement "Derivations of
// Cluster Normal Optimization").
//
// The cluster objective of a node (Eq. normal_optimization) is a quadratic form in
// its four corner normals N0..N3: E(N) = C + tr(N^T B) + tr(N^T A N) / 2 with
//   A = 2 int w lambda lambda^T,  B = -2 int w lambda n^T,  C = int w |n|^2,
// lambda the cluster triangles' barycentric basis and w = 1 / max(Jacobian, eps)
// of each fine triangle.  Both cluster halves (lower: corners 0, 1, 2; upper:
// corners 3, 2, 1) carry these integrals over their own area in their own
// barycentric basis mu: a 3 x 3 Gram matrix G = 2 int w mu mu^T, H = -2 int w mu n^T
// and C.  A child half-triangle lies wholly inside one half of its parent, and the
// parent's barycentrics restricted to it are the child's barycentrics times the
// matrix Lam[i][k] = mu^parent_i(child vertex k), whose entries are 0, 1/2 or 1.  So
//   G_parent += Lam G_child Lam^T,  H_parent += Lam H_child,  C_parent += C_child
// are exact products (powers of two) summed, and every entry of G is a sum of
// non-negative terms: the recurrence is as accurate as integrating each node
// directly, in O(N^2) total work.  Level 0 is the fine triangle itself (area 1/2,
// linear normal field): G = w (1 + delta_ij) / 12, H_i = -(w / 12) (n_i + sum n_k),
// C = (w / 24) (sum |n_k|^2 + |sum n_k|^2).
//
// N* = -A^-1 B by Cholesky.  The residual e^l = E(N*) is then integrated directly
// over the node's fine triangles (the residual is linear on each:
// int w |r|^2 = (w / 24) (sum |r_k|^2 + |sum r_k|^2) from its vertex values), a sum
// of non-negative terms, instead of the difference C + tr(N*^T B) / 2 of large
// numbers.
#include "pndf_internal.h"

namespace pndf {

namespace {

// Statistics of one cluster half: G (00, 01, 02, 11, 12, 22), H (3 x 2, row-major), C.
constexpr int kStat = 13;
constexpr int kG = 0, kH = 6, kC = 12;

__device__ __forceinline__ double jac64(float2 a, float2 b, float2 c)
{
    double p = __dmul_rn((double)c.x - (double)a.x, (double)b.y - (double)a.y);
    double q = __dmul_rn((double)c.y - (double)a.y, (double)b.x - (double)a.x);
    return fabs(__dsub_rn(p, q));
}

__device__ __forceinline__ double fine_weight(double det, double eps) { return 1.0 / (det < eps ? eps : det); }

// Statistics of a fine triangle with vertex normals (a, b, c) and weight w, in its
// own barycentric basis.
__device__ __forceinline__ void fine_stats(double w, float2 a, float2 b, float2 c, double* S)
{
    const double d = w / 6.0, f = w / 12.0;
    S[kG + 0] = d; S[kG + 1] = f; S[kG + 2] = f;
    S[kG + 3] = d; S[kG + 4] = f; S[kG + 5] = d;
    const double ax = a.x, ay = a.y, bx = b.x, by = b.y, cx = c.x, cy = c.y;
    const double sx = ax + bx + cx, sy = ay + by + cy;
    S[kH + 0] = -f * (ax + sx); S[kH + 1] = -f * (ay + sy);
    S[kH + 2] = -f * (bx + sx); S[kH + 3] = -f * (by + sy);
    S[kH + 4] = -f * (cx + sx); S[kH + 5] = -f * (cy + sy);
    const double q = ax * ax + ay * ay + bx * bx + by * by + cx * cx + cy * cy + sx * sx + sy * sy;
    S[kC] = (w / 24.0) * q;
}

// Barycentric basis of a parent half at parent-normalised (U, V): lower half over
// corners (0, 1, 2) = (1 - U - V, U, V); upper half over corners (3, 2, 1) =
// (U + V - 1, 1 - U, 1 - V).
__device__ __forceinline__ void half_basis(int hp, double U, double V, double mu[3])
{
    if (hp == 0) { mu[0] = 1.0 - U - V; mu[1] = U; mu[2] = V; }
    else { mu[0] = U + V - 1.0; mu[1] = 1.0 - U; mu[2] = 1.0 - V; }
}

// Add the statistics S of half hc of child (di, dj) (side 1/2 of the parent) to
// half hp of the parent.  Child lower vertices (in parent-normalised coordinates):
// (di, dj)/2, (di + 1, dj)/2, (di, dj + 1)/2; upper: (di + 1, dj + 1)/2,
// (di, dj + 1)/2, (di + 1, dj)/2.  Called with literal arguments, so Lam folds
// into constants.
__device__ __forceinline__ void add_child(int di, int dj, int hc, int hp, const double* S, double* P)
{
    const double x0 = 0.5 * di, x1 = 0.5 * (di + 1), y0 = 0.5 * dj, y1 = 0.5 * (dj + 1);
    const double vu[3] = {hc ? x1 : x0, hc ? x0 : x1, hc ? x1 : x0};
    const double vv[3] = {hc ? y1 : y0, hc ? y1 : y0, hc ? y0 : y1};
    double Lm[3][3];  // Lm[i][k] = mu^parent_i(child vertex k)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double mu[3];
        half_basis(hp, vu[k], vv[k], mu);
#pragma unroll
        for (int i = 0; i < 3; ++i) Lm[i][k] = mu[i];
    }
    const double G[3][3] = {{S[kG + 0], S[kG + 1], S[kG + 2]},
                            {S[kG + 1], S[kG + 3], S[kG + 4]},
                            {S[kG + 2], S[kG + 4], S[kG + 5]}};
    double T[3][3];  // Lm G
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int m = 0; m < 3; ++m) T[i][m] = Lm[i][0] * G[0][m] + Lm[i][1] * G[1][m] + Lm[i][2] * G[2][m];
    const int gi[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j)
            P[kG + gi[i][j]] += T[i][0] * Lm[j][0] + T[i][1] * Lm[j][1] + T[i][2] * Lm[j][2];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int c = 0; c < 2; ++c)
            P[kH + 2 * i + c] += Lm[i][0] * S[kH + c] + Lm[i][1] * S[kH + 2 + c] + Lm[i][2] * S[kH + 4 + c];
    P[kC] += S[kC];
}

// Add the eight child halves of a node to its two halves: the lower-left child
// (c4 = 0) lies in the lower half, the upper-right one (c4 = 3) in the upper half,
// and the off-diagonal children split along the parent's diagonal (their lower
// halves below it).  C(c4, h) gives half h of child c4 = di + 2 dj.
template <typename ChildFn>
__device__ __forceinline__ void gather_children(ChildFn C, double* lo, double* up)
{
#pragma unroll
    for (int c4 = 0; c4 < 4; ++c4)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int hp = c4 == 0 ? 0 : (c4 == 3 ? 1 : h);
            add_child(c4 & 1, c4 >> 1, h, hp, C(c4, h), hp ? up : lo);
        }
}

// N* = -A^-1 B for the node's 4 x 4 A and 4 x 2 B assembled from its halves (lower
// over corners 0, 1, 2, upper over corners 3, 2, 1), by Cholesky (A is positive
// definite: every fine triangle has a positive weight).
__device__ void solve_cluster(const double* lo, const double* up, double N[4][2])
{
    double A[4][4] = {{0}}, B[4][2] = {{0}};
    const int vi[2][3] = {{0, 1, 2}, {3, 2, 1}};
    const int gi[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
    const double* hs[2] = {lo, up};
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
#pragma unroll
            for (int j = 0; j < 3; ++j) A[vi[h][i]][vi[h][j]] += hs[h][kG + gi[i][j]];
            B[vi[h][i]][0] += hs[h][kH + 2 * i];
            B[vi[h][i]][1] += hs[h][kH + 2 * i + 1];
        }
    double Lm[4][4] = {{0}};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        double d = A[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) d -= Lm[j][k] * Lm[j][k];
        d = sqrt(fmax(d, 1e-300));
        Lm[j][j] = d;
#pragma unroll
        for (int i = j + 1; i < 4; ++i) {
            double v = A[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) v -= Lm[i][k] * Lm[j][k];
            Lm[i][j] = v / d;
        }
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        double y[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            double v = -B[i][c];
#pragma unroll
            for (int k = 0; k < i; ++k) v -= Lm[i][k] * y[k];
            y[i] = v / Lm[i][i];
        }
#pragma unroll
        for (int i = 3; i >= 0; --i) {
            double v = y[i];
#pragma unroll
            for (int k = i + 1; k < 4; ++k) v -= Lm[k][i] * N[k][c];
            N[i][c] = v / Lm[i][i];
        }
    }
}

__device__ __forceinline__ void box_add(float4& b, float x, float y)
{
    b.x = fminf(b.x, x); b.y = fminf(b.y, y); b.z = fmaxf(b.z, x); b.w = fmaxf(b.w, y);
}

__device__ __forceinline__ void box_union(float4& b, const float4& o)
{
    b.x = fminf(b.x, o.x); b.y = fminf(b.y, o.y); b.z = fmaxf(b.z, o.z); b.w = fmaxf(b.w, o.w);
}

// Box of a replacement triangle centred at (cx, cy) with circumradius rho, with a
// margin that covers both the float32 and the FP64 vertex evaluations.
__device__ __forceinline__ void box_add_eqtri(float4& b, float cx, float cy, float rho)
{
    const float r = rho * (1.0f + 1e-6f) + 1e-6f;
    box_add(b, cx - r, cy - r);
    box_add(b, cx + r, cy + r);
}

__device__ __forceinline__ float4 empty_box()
{
    return make_float4(INFINITY, INFINITY, -INFINITY, -INFINITY);
}

struct LevelOut {
    float4* bbox;
    float4* bbox_all;
    float4* bbox_clu;
    float4* clu_n;
    float4* clu_t;
    float* clu_e;
    float2* clu_det;
};

// Store the fitted normals of node idx (level side s): float32 normals, the cluster
// triangles' Jacobians and clamp decisions (FP64 from the stored float32 normals, as
// the evaluation uses them) with the test record that carries them, the FP64 normals
// for the residual pass; returns the box of the cluster triangles.
__device__ float4 store_cluster(const HierDev& H, const LevelOut& o, int64_t idx, int s, const double N[4][2],
                                double* __restrict__ nfit)
{
    float2 f[4];
    for (int k = 0; k < 4; ++k) f[k] = make_float2((float)N[k][0], (float)N[k][1]);
    o.clu_n[2 * idx] = make_float4(f[0].x, f[0].y, f[1].x, f[1].y);
    o.clu_n[2 * idx + 1] = make_float4(f[2].x, f[2].y, f[3].x, f[3].y);
    double* nf = nfit + 8 * idx;
    for (int k = 0; k < 4; ++k) { nf[2 * k] = N[k][0]; nf[2 * k + 1] = N[k][1]; }
    const double s2 = (double)s * (double)s;
    const double dl = jac64(f[0], f[1], f[2]) / s2;
    const double du = jac64(f[3], f[2], f[1]) / s2;
    const double eps = (double)H.eps;
    const bool cl = dl < eps, cu = du < eps;
    o.clu_det[idx] = make_float2(cl ? H.eps : (float)dl, cu ? H.eps : (float)du);
    const float qnan = __int_as_float(0x7fc00000);
    o.clu_t[2 * idx] = make_float4(cl ? qnan : f[0].x, f[0].y, f[1].x, f[1].y);
    o.clu_t[2 * idx + 1] = make_float4(f[2].x, f[2].y, cu ? qnan : f[3].x, f[3].y);
    float4 b = empty_box();
    const float cx = 0.5f * (f[1].x + f[2].x), cy = 0.5f * (f[1].y + f[2].y);
    const float rho = H.rho * (float)s;
    if (cl) box_add_eqtri(b, cx, cy, rho);
    else { box_add(b, f[0].x, f[0].y); box_add(b, f[1].x, f[1].y); box_add(b, f[2].x, f[2].y); }
    if (cu) box_add_eqtri(b, cx, cy, rho);
    else { box_add(b, f[3].x, f[3].y); box_add(b, f[2].x, f[2].y); box_add(b, f[1].x, f[1].y); }
    return b;
}

// Level 1: every node takes its 2 x 2 cells (8 fine triangles), writes its leaf
// record, box and half statistics, and solves its fit.  Thread index = Morton code.
__global__ void k_level1(HierDev H, LevelOut o, QuadRec* __restrict__ quad, double* __restrict__ stat,
                         double* __restrict__ nfit, int cluster)
{
    const int m = H.n >> 1;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)m * m) return;
    const int I = (int)morton_compact((uint32_t)t), J = (int)morton_compact((uint32_t)t >> 1);
    const int w = H.n + 1;
    float2 tx[9];
    {
        QuadRec r;
        for (int y = 0; y < 3; ++y)
            for (int x = 0; x < 3; ++x) tx[3 * y + x] = r.t[3 * y + x] = H.nrm[(int64_t)(2 * J + y) * w + 2 * I + x];
        for (int dj = 0; dj < 2; ++dj)
            for (int di = 0; di < 2; ++di) r.deg[2 * dj + di] = H.deg[(int64_t)(2 * J + dj) * H.n + 2 * I + di];
        r.pad = 0;
        quad[t] = r;
    }
    float4 box = empty_box();
    for (int dj = 0; dj < 2; ++dj)
        for (int di = 0; di < 2; ++di) {
            const int k = 3 * dj + di;
            const float2 n0 = tx[k], n1 = tx[k + 1], n2 = tx[k + 3], n3 = tx[k + 4];
            const uint8_t dg = H.deg[(int64_t)(2 * J + dj) * H.n + 2 * I + di];
            const float cx = 0.5f * (n1.x + n2.x), cy = 0.5f * (n1.y + n2.y);
            if (dg & 1) box_add_eqtri(box, cx, cy, H.rho);
            else { box_add(box, n0.x, n0.y); box_add(box, n1.x, n1.y); box_add(box, n2.x, n2.y); }
            if (dg & 2) box_add_eqtri(box, cx, cy, H.rho);
            else { box_add(box, n3.x, n3.y); box_add(box, n2.x, n2.y); box_add(box, n1.x, n1.y); }
        }
    o.bbox[t] = box;
    if (!cluster) return;
    const double eps = (double)H.eps;
    // the 8 fine triangles (cell c4 = di + 2 dj: lower (n0, n1, n2), upper (n3, n2, n1))
    // gathered into the node's halves
    double lo[kStat] = {0}, up[kStat] = {0};
#pragma unroll
    for (int c4 = 0; c4 < 4; ++c4) {
        const int k = 3 * (c4 >> 1) + (c4 & 1);
        const float2 n0 = tx[k], n1 = tx[k + 1], n2 = tx[k + 3], n3 = tx[k + 4];
        double F[kStat];
        fine_stats(fine_weight(jac64(n0, n1, n2), eps), n0, n1, n2, F);
        add_child(c4 & 1, c4 >> 1, 0, c4 == 3 ? 1 : 0, F, c4 == 3 ? up : lo);
        fine_stats(fine_weight(jac64(n3, n2, n1), eps), n3, n2, n1, F);
        add_child(c4 & 1, c4 >> 1, 1, c4 == 0 ? 0 : 1, F, c4 == 0 ? lo : up);
    }
    double* M = stat + t * (2 * kStat);
    for (int k = 0; k < kStat; ++k) { M[k] = lo[k]; M[kStat + k] = up[k]; }
    double N[4][2];
    solve_cluster(lo, up, N);
    float4 cb = store_cluster(H, o, t, 2, N, nfit);
    o.bbox_clu[t] = cb;
    box_union(cb, box);
    o.bbox_all[t] = cb;
}

// Level l >= 2 from level l-1: boxes are unions of the children, half statistics
// gathered from the children's.  Thread index = Morton code; the children of node
// t are 4t + (di + 2 dj).
__global__ void k_level_up(HierDev H, int level, LevelOut o, const float4* __restrict__ cbox,
                           const float4* __restrict__ cbox_all, const double* __restrict__ cstat,
                           double* __restrict__ stat, double* __restrict__ nfit, int cluster)
{
    const int m = H.n >> level;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)m * m) return;
    const int64_t c00 = 4 * t;
    float4 box = cbox[c00];
    box_union(box, cbox[c00 + 1]);
    box_union(box, cbox[c00 + 2]);
    box_union(box, cbox[c00 + 3]);
    o.bbox[t] = box;
    if (!cluster) return;
    double lo[kStat] = {0}, up[kStat] = {0};
    gather_children([&](int c4, int h) { return cstat + (c00 + c4) * (2 * kStat) + h * kStat; }, lo, up);
    double* M = stat + t * (2 * kStat);
    for (int k = 0; k < kStat; ++k) { M[k] = lo[k]; M[kStat + k] = up[k]; }
    double N[4][2];
    solve_cluster(lo, up, N);
    float4 cb = store_cluster(H, o, t, 1 << level, N, nfit);
    o.bbox_clu[t] = cb;
    box_union(cb, cbox_all[c00]);
    box_union(cb, cbox_all[c00 + 1]);
    box_union(cb, cbox_all[c00 + 2]);
    box_union(cb, cbox_all[c00 + 3]);
    o.bbox_all[t] = cb;
}

// The cluster interpolant of a node at node-normalised (U, V): lower triangle
// N0 (1 - U - V) + N1 U + N2 V, upper N3 (U + V - 1) + N2 (1 - U) + N1 (1 - V)
// (continuous across the diagonal).
__device__ __forceinline__ double2 cluster_field(const double* N, double U, double V)
{
    if (U + V <= 1.0) {
        const double a = 1.0 - U - V;
        return make_double2(N[0] * a + N[2] * U + N[4] * V, N[1] * a + N[3] * U + N[5] * V);
    }
    const double a = U + V - 1.0, b = 1.0 - U, c = 1.0 - V;
    return make_double2(N[6] * a + N[4] * b + N[2] * c, N[7] * a + N[5] * b + N[3] * c);
}

constexpr int kResidBlock = 256;  // leaf records per block of the residual pass (a level-5 node)

// Residual of level `level`: thread t (a level-1 record, Morton order) integrates the
// residual of its 8 fine triangles against the FP64 fit of its level-`level`
// ancestor t >> 2 (level - 1).  The 4^(level - 1) records of a node are consecutive:
// up to a whole block they are summed by a fixed LDS tree and stored as e^l; above,
// each block leaves a partial sum for k_resid_sum.  Deterministic.
__global__ __launch_bounds__(kResidBlock) void k_resid(HierDev H, int level, const double* __restrict__ nfit,
                                                       float* __restrict__ clu_e, double* __restrict__ part)
{
    __shared__ double red[kResidBlock];
    const int64_t m1 = (int64_t)(H.n >> 1) * (H.n >> 1);
    const int64_t t = (int64_t)blockIdx.x * kResidBlock + threadIdx.x;
    const int sh = 2 * (level - 1);
    double r = 0.0;
    if (t < m1) {
        const int64_t node = t >> sh;
        const double* N = nfit + 8 * node;
        const int side = 1 << level;
        const double inv = 1.0 / side;
        const int li = (2 * (int)morton_compact((uint32_t)t)) & (side - 1);
        const int lj = (2 * (int)morton_compact((uint32_t)t >> 1)) & (side - 1);
        const float4* rec = reinterpret_cast<const float4*>(H.quad + t);
        const float4 a = rec[0], b = rec[1], c = rec[2], d = rec[3], e = rec[4];
        const float2 tx[9] = {make_float2(a.x, a.y), make_float2(a.z, a.w), make_float2(b.x, b.y),
                              make_float2(b.z, b.w), make_float2(c.x, c.y), make_float2(c.z, c.w),
                              make_float2(d.x, d.y), make_float2(d.z, d.w), make_float2(e.x, e.y)};
        double rx[9], ry[9];
#pragma unroll
        for (int y = 0; y < 3; ++y)
#pragma unroll
            for (int x = 0; x < 3; ++x) {
                const double2 f = cluster_field(N, (li + x) * inv, (lj + y) * inv);
                rx[3 * y + x] = (double)tx[3 * y + x].x - f.x;
                ry[3 * y + x] = (double)tx[3 * y + x].y - f.y;
            }
        const double eps = (double)H.eps;
#pragma unroll
        for (int c4 = 0; c4 < 4; ++c4) {
            const int k = 3 * (c4 >> 1) + (c4 & 1);
            const int tri[2][3] = {{k, k + 1, k + 3}, {k + 4, k + 3, k + 1}};
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int p = tri[h][0], q = tri[h][1], s = tri[h][2];
                const double wgt = fine_weight(jac64(tx[p], tx[q], tx[s]), eps);
                const double sx = rx[p] + rx[q] + rx[s], sy = ry[p] + ry[q] + ry[s];
                const double qq = rx[p] * rx[p] + ry[p] * ry[p] + rx[q] * rx[q] + ry[q] * ry[q] + rx[s] * rx[s] +
                                  ry[s] * ry[s] + sx * sx + sy * sy;
                r += (wgt / 24.0) * qq;
            }
        }
    }
    if (sh == 0) {
        if (t < m1) clu_e[t] = (float)r;
        return;
    }
    red[threadIdx.x] = r;
    const int group = sh >= 8 ? kResidBlock : 1 << sh;
    for (int st = 1; st < group; st <<= 1) {
        __syncthreads();
        if ((threadIdx.x & (2 * st - 1)) == 0) red[threadIdx.x] += red[threadIdx.x + st];
    }
    if (group < kResidBlock || sh == 8) {
        if ((threadIdx.x & (group - 1)) == 0 && t < m1) clu_e[t >> sh] = (float)red[threadIdx.x];
    } else if (threadIdx.x == 0) {
        part[blockIdx.x] = red[0];
    }
}

// e^l of nodes larger than a block of the residual pass: the sum of the node's
// `per` consecutive block partials, in order.
__global__ void k_resid_sum(const double* __restrict__ part, int64_t nodes, int64_t per, float* __restrict__ clu_e)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nodes) return;
    double s = 0.0;
    for (int64_t i = 0; i < per; ++i) s += part[k * per + i];
    clu_e[k] = (float)s;
}

__global__ void k_export_rowmajor(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst, int m,
                                  int words)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)m * m) return;
    const uint32_t I = (uint32_t)(k % m), J = (uint32_t)(k / m);
    const uint32_t* a = src + (int64_t)morton(I, J) * words;
    uint32_t* b = dst + k * words;
    for (int w = 0; w < words; ++w) b[w] = a[w];
}

}  // namespace

hipError_t export_rowmajor(const void* src, void* dst, int m, int words, hipStream_t s)
{
    const int64_t cnt = (int64_t)m * m;
    hipLaunchKernelGGL(k_export_rowmajor, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s,
                       (const uint32_t*)src, (uint32_t*)dst, m, words);
    return hipGetLastError();
}

// The traversal's boxes in half precision, minima rounded down and maxima up, as
// order keys (half_key): a rounded box contains the exact one, so it prunes a little
// less but never wrongly; four child boxes take 32 B instead of 64 and each test is
// two packed 16-bit integer operations (the float32 boxes stay for the exports).
__device__ __forceinline__ uint2 box_keys(float4 b)
{
    uint32_t x0 = __half_as_ushort(__float2half_rd(b.x)), y0 = __half_as_ushort(__float2half_rd(b.y));
    uint32_t x1 = __half_as_ushort(__float2half_ru(b.z)), y1 = __half_as_ushort(__float2half_ru(b.w));
    // the zeros: a minimum of +0 becomes -0, a maximum of -0 becomes +0
    if (x0 == 0u) x0 = 0x8000u;
    if (y0 == 0u) y0 = 0x8000u;
    if (x1 == 0x8000u) x1 = 0u;
    if (y1 == 0x8000u) y1 = 0u;
    return make_uint2(half_key(x0) | (half_key(y0) << 16), half_key(x1) | (half_key(y1) << 16));
}

__global__ void k_key_boxes(const float4* __restrict__ src, uint2* __restrict__ dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    dst[i] = box_keys(src[i]);
}

// Keys of a box that contains every normal (minimum key 0, maximum key 0xffff).
__global__ void k_fill_keys_all(uint2* __restrict__ dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    dst[i] = make_uint2(0u, 0xffffffffu);
}

// Union keys (HierDev::bbox_u) of one level l >= 3: the box of the node's four
// children's own cluster triangles.  A node whose children are all under the cut
// is skipped when this box misses h: none of their cluster tests could hit.
__global__ void k_union_keys(HierDev H, int level, const float4* __restrict__ bbox_clu, uint2* __restrict__ dst)
{
    const int64_t m = (int64_t)(H.n >> level) * (H.n >> level);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    const float4* c = bbox_clu + level_offset(H.logn, level - 1) + 4 * t;
    float4 u = c[0];
    box_union(u, c[1]);
    box_union(u, c[2]);
    box_union(u, c[3]);
    dst[level_offset(H.logn, level) + t] = box_keys(u);
}

// The cut traversal's sibling-group records (HierDev::grp) of one level: thread t
// writes node t's words (its keys are those of bbox_all, as k_key_boxes forms them).
__global__ void k_group_records(HierDev H, int level, uint32_t* __restrict__ grp)
{
    const int64_t m = (int64_t)(H.n >> level) * (H.n >> level);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    const int64_t idx = level_offset(H.logn, level) + t;
    uint32_t* w = grp + 4 * (idx & ~(int64_t)3);   // 16 words per group
    const int c = (int)(idx & 3);
    const uint2 k = box_keys(H.bbox_all[idx]);
    w[2 * c] = k.x;
    w[2 * c + 1] = k.y;
    w[8 + c] = __float_as_uint(H.clu_e[idx]);
    float emc = INFINITY;
    if (level >= 2) {
        const float* ce = H.clu_e + level_offset(H.logn, level - 1) + 4 * t;
        emc = fmaxf(fmaxf(ce[0], ce[1]), fmaxf(ce[2], ce[3]));
    }
    w[12 + c] = __float_as_uint(emc);
}

hipError_t build_hierarchy_levels(pndf_hier* h, hipStream_t s)
{
    const HierDev& H = h->dev;
    const int n = H.n;
    const int64_t m1 = (int64_t)(n >> 1) * (n >> 1);
    const int64_t rblocks = (m1 + kResidBlock - 1) / kResidBlock;
    // workspace (cluster fits only): half statistics of two consecutive levels, the
    // FP64 normals of the current level, block partials of the residual pass
    double* stat[2] = {nullptr, nullptr};
    double* nfit = nullptr;
    double* part = nullptr;
    hipError_t err = hipSuccess;
    auto release = [&]() {
        (void)hipFree(stat[0]);
        (void)hipFree(stat[1]);
        (void)hipFree(nfit);
        (void)hipFree(part);
    };
    if (h->cluster) {
        const int64_t m2 = n >= 4 ? (int64_t)(n >> 2) * (n >> 2) : 1;
        err = hipMalloc(&stat[0], sizeof(double) * 2 * kStat * m1);
        if (err == hipSuccess) err = hipMalloc(&stat[1], sizeof(double) * 2 * kStat * m2);
        if (err == hipSuccess) err = hipMalloc(&nfit, sizeof(double) * 8 * m1);
        if (err == hipSuccess) err = hipMalloc(&part, sizeof(double) * rblocks);
        if (err != hipSuccess) {
            release();
            return err;
        }
    }
    auto out_for = [&](int level) {
        LevelOut o;
        const int64_t off = level_offset(H.logn, level);
        o.bbox = h->bbox + off;
        o.bbox_all = h->cluster ? h->bbox_all + off : nullptr;
        o.bbox_clu = h->cluster ? h->bbox_clu + off : nullptr;
        o.clu_n = h->cluster ? h->clu_n + 2 * off : nullptr;
        o.clu_e = h->cluster ? h->clu_e + off : nullptr;
        o.clu_t = h->cluster ? h->clu_t + 2 * off : nullptr;
        o.clu_det = h->cluster ? h->clu_det + off : nullptr;
        return o;
    };
    auto residual = [&](int level) {
        // (runs before the next level's fit overwrites nfit: one stream)
        float* e = h->clu_e + level_offset(H.logn, level);
        hipLaunchKernelGGL(k_resid, dim3((unsigned)rblocks), dim3(kResidBlock), 0, s, H, level, nfit, e, part);
        const int sh = 2 * (level - 1);
        if (sh > 8) {
            const int64_t nodes = (int64_t)(n >> level) * (n >> level);
            const int64_t per = ((int64_t)1 << sh) / kResidBlock;
            hipLaunchKernelGGL(k_resid_sum, dim3((unsigned)((nodes + 63) / 64)), dim3(64), 0, s, part, nodes, per, e);
        }
        return hipGetLastError();
    };
    const int bs = 128;
    hipLaunchKernelGGL(k_level1, dim3((unsigned)((m1 + bs - 1) / bs)), dim3(bs), 0, s, H, out_for(1),
                       h->quad, stat[0], nfit, h->cluster);
    err = hipGetLastError();
    if (err == hipSuccess && h->cluster) err = residual(1);
    for (int level = 2; level <= H.L && err == hipSuccess; ++level) {
        const int64_t m = (int64_t)(n >> level) * (n >> level);
        const int64_t coff = level_offset(H.logn, level - 1);
        const double* cs = stat[(level - 2) & 1];
        double* os = stat[(level - 1) & 1];
        hipLaunchKernelGGL(k_level_up, dim3((unsigned)((m + bs - 1) / bs)), dim3(bs), 0, s, H,
                           level, out_for(level), h->bbox + coff,
                           h->cluster ? h->bbox_all + coff : nullptr, cs, os, nfit, h->cluster);
        err = hipGetLastError();
        if (err == hipSuccess && h->cluster) err = residual(level);
    }
    if (err == hipSuccess) {
        const unsigned g = (unsigned)((h->nodes + 255) / 256);
        hipLaunchKernelGGL(k_key_boxes, dim3(g), dim3(256), 0, s, h->bbox, h->bbox_k, h->nodes);
        if (h->cluster) {
            hipLaunchKernelGGL(k_key_boxes, dim3(g), dim3(256), 0, s, h->bbox_clu, h->bbox_c, h->nodes);
            // (levels 1 and 2 keep the all-inclusive box: their children's own boxes are
            // not what those children are tested against)
            hipLaunchKernelGGL(k_fill_keys_all, dim3(g), dim3(256), 0, s, h->bbox_u, h->nodes);
            for (int level = 3; level <= H.L; ++level) {
                const int64_t m = (int64_t)(n >> level) * (n >> level);
                hipLaunchKernelGGL(k_union_keys, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, H, level,
                                   h->bbox_clu, h->bbox_u);
            }
            // (the top level's group holds one node: its other words are never read)
            for (int level = 1; level <= H.L; ++level) {
                const int64_t m = (int64_t)(n >> level) * (n >> level);
                hipLaunchKernelGGL(k_group_records, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, H, level,
                                   reinterpret_cast<uint32_t*>(h->grp));
            }
        }
        err = hipGetLastError();
    }
    if (err == hipSuccess) err = hipStreamSynchronize(s);
    release();
    return err;
}

}  // namespace pndf
