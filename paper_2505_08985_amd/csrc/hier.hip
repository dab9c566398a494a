// Hierarchy build: min-max boxes and least-squares cluster normals per quad-tree
// node (section "Acceleration by mesh clustering"; supplement "Derivations of
// Cluster Normal Optimization").
//
// The cluster objective of a node of side s (Eq. normal_optimization) is a
// quadratic form in its four corner normals.  Its gradient A N + B needs, per
// cluster half (the node's lower and upper triangle), the inverse-Jacobian
// weighted moments of the fine triangles inside that half:
//   int w {1, u, v, u^2, u v, v^2},  int w n {1, u, v},  int w |n|^2.
// These are additive and shift exactly under translation, and the four children
// of a node fall into its halves by a fixed rule (lower-left child and the lower
// halves of the off-diagonal children go to the lower half), so every level is
// assembled from the level below in O(N^2) total work instead of re-integrating
// every fine triangle per level.  Level 1 is integrated directly from its eight
// fine triangles with the three-edge-midpoint rule (exact for quadratics).
#include "pndf_internal.h"

namespace pndf {

namespace {

constexpr int kMom = 13;  // 1, u, v, uu, uv, vv, nx, ny, nxu, nyu, nxv, nyv, |n|^2

__device__ __forceinline__ double jac64(float2 a, float2 b, float2 c)
{
    double p = __dmul_rn((double)c.x - (double)a.x, (double)b.y - (double)a.y);
    double q = __dmul_rn((double)c.y - (double)a.y, (double)b.x - (double)a.x);
    return fabs(__dsub_rn(p, q));
}

// moments of one fine triangle with uv vertices (node-local texel units) and
// normals, weight w, added into M
__device__ void tri_moments(double w, const double u[3], const double v[3], const float2 nn[3],
                            double* M)
{
    const double f = w / 6.0;  // area 1/2, three points
    for (int k = 0; k < 3; ++k) {
        const int k2 = k == 2 ? 0 : k + 1;
        const double mu = 0.5 * (u[k] + u[k2]), mv = 0.5 * (v[k] + v[k2]);
        const double nx = 0.5 * ((double)nn[k].x + (double)nn[k2].x);
        const double ny = 0.5 * ((double)nn[k].y + (double)nn[k2].y);
        M[0] += f;
        M[1] += f * mu;
        M[2] += f * mv;
        M[3] += f * mu * mu;
        M[4] += f * mu * mv;
        M[5] += f * mv * mv;
        M[6] += f * nx;
        M[7] += f * ny;
        M[8] += f * nx * mu;
        M[9] += f * ny * mu;
        M[10] += f * nx * mv;
        M[11] += f * ny * mv;
        M[12] += f * (nx * nx + ny * ny);
    }
}

// add moments S shifted by (ox, oy) into D
__device__ void shift_add(const double* S, double ox, double oy, double* D)
{
    D[0] += S[0];
    D[1] += S[1] + ox * S[0];
    D[2] += S[2] + oy * S[0];
    D[3] += S[3] + 2.0 * ox * S[1] + ox * ox * S[0];
    D[4] += S[4] + ox * S[2] + oy * S[1] + ox * oy * S[0];
    D[5] += S[5] + 2.0 * oy * S[2] + oy * oy * S[0];
    D[6] += S[6];
    D[7] += S[7];
    D[8] += S[8] + ox * S[6];
    D[9] += S[9] + ox * S[7];
    D[10] += S[10] + oy * S[6];
    D[11] += S[11] + oy * S[7];
    D[12] += S[12];
}

// Solve the cluster fit of a node of side s from its half moments.
// Basis: lower lambda = (1-U-V, U, V, 0), upper lambda = (0, 1-V, 1-U, U+V-1),
// U = u / s, V = v / s.  A = 2 int w lam lam^T, B = -2 int w lam n^T, C = int w |n|^2;
// N = -A^-1 B by Cholesky; e = C + tr(B^T N) / 2 (objective at the minimum).
__device__ void solve_cluster(const double* lo, const double* up, int s, double N[4][2],
                              double* e_out)
{
    double A[4][4] = {{0}}, B[4][2] = {{0}};
    const double is = 1.0 / s, is2 = is * is;
    {
        const double M1 = lo[0], MU = lo[1] * is, MV = lo[2] * is;
        const double MUU = lo[3] * is2, MUV = lo[4] * is2, MVV = lo[5] * is2;
        A[0][0] += 2.0 * (M1 - 2.0 * MU - 2.0 * MV + MUU + 2.0 * MUV + MVV);
        A[0][1] += 2.0 * (MU - MUU - MUV);
        A[0][2] += 2.0 * (MV - MUV - MVV);
        A[1][1] += 2.0 * MUU;
        A[1][2] += 2.0 * MUV;
        A[2][2] += 2.0 * MVV;
        for (int c = 0; c < 2; ++c) {
            const double Nn = lo[6 + c], NU = lo[8 + c] * is, NV = lo[10 + c] * is;
            B[0][c] += -2.0 * (Nn - NU - NV);
            B[1][c] += -2.0 * NU;
            B[2][c] += -2.0 * NV;
        }
    }
    {
        const double M1 = up[0], MU = up[1] * is, MV = up[2] * is;
        const double MUU = up[3] * is2, MUV = up[4] * is2, MVV = up[5] * is2;
        A[1][1] += 2.0 * (M1 - 2.0 * MV + MVV);
        A[1][2] += 2.0 * (M1 - MU - MV + MUV);
        A[1][3] += 2.0 * (MU + 2.0 * MV - M1 - MUV - MVV);
        A[2][2] += 2.0 * (M1 - 2.0 * MU + MUU);
        A[2][3] += 2.0 * (2.0 * MU + MV - M1 - MUU - MUV);
        A[3][3] += 2.0 * (MUU + 2.0 * MUV + MVV - 2.0 * MU - 2.0 * MV + M1);
        for (int c = 0; c < 2; ++c) {
            const double Nn = up[6 + c], NU = up[8 + c] * is, NV = up[10 + c] * is;
            B[1][c] += -2.0 * (Nn - NV);
            B[2][c] += -2.0 * (Nn - NU);
            B[3][c] += -2.0 * (NU + NV - Nn);
        }
    }
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < r; ++c) A[r][c] = A[c][r];
    // Cholesky A = L L^T
    double Lm[4][4] = {{0}};
    for (int j = 0; j < 4; ++j) {
        double d = A[j][j];
        for (int k = 0; k < j; ++k) d -= Lm[j][k] * Lm[j][k];
        d = sqrt(fmax(d, 1e-300));
        Lm[j][j] = d;
        for (int i = j + 1; i < 4; ++i) {
            double v = A[i][j];
            for (int k = 0; k < j; ++k) v -= Lm[i][k] * Lm[j][k];
            Lm[i][j] = v / d;
        }
    }
    for (int c = 0; c < 2; ++c) {
        double y[4];
        for (int i = 0; i < 4; ++i) {
            double v = -B[i][c];
            for (int k = 0; k < i; ++k) v -= Lm[i][k] * y[k];
            y[i] = v / Lm[i][i];
        }
        for (int i = 3; i >= 0; --i) {
            double v = y[i];
            for (int k = i + 1; k < 4; ++k) v -= Lm[k][i] * N[k][c];
            N[i][c] = v / Lm[i][i];
        }
    }
    double e = lo[12] + up[12];
    for (int a = 0; a < 4; ++a) e += 0.5 * (B[a][0] * N[a][0] + B[a][1] * N[a][1]);
    *e_out = e > 0.0 ? e : 0.0;
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

// Store the fitted cluster of node idx (level side s) and return its box.
__device__ float4 store_cluster(const HierDev& H, int64_t idx, int s, const double N[4][2], double e,
                                float4* clu_n, float* clu_e, float2* clu_det, uint8_t* clu_deg)
{
    float2 f[4];
    for (int k = 0; k < 4; ++k) f[k] = make_float2((float)N[k][0], (float)N[k][1]);
    clu_n[2 * idx] = make_float4(f[0].x, f[0].y, f[1].x, f[1].y);
    clu_n[2 * idx + 1] = make_float4(f[2].x, f[2].y, f[3].x, f[3].y);
    clu_e[idx] = (float)e;
    const double s2 = (double)s * (double)s;
    const double dl = jac64(f[0], f[1], f[2]) / s2;
    const double du = jac64(f[3], f[2], f[1]) / s2;
    const double eps = (double)H.eps;
    const bool cl = dl < eps, cu = du < eps;
    clu_det[idx] = make_float2(cl ? H.eps : (float)dl, cu ? H.eps : (float)du);
    clu_deg[idx] = (uint8_t)((cl ? 1 : 0) | (cu ? 2 : 0));
    float4 b = empty_box();
    const float cx = 0.5f * (f[1].x + f[2].x), cy = 0.5f * (f[1].y + f[2].y);
    const float rho = H.rho * (float)s;
    if (cl) box_add_eqtri(b, cx, cy, rho);
    else { box_add(b, f[0].x, f[0].y); box_add(b, f[1].x, f[1].y); box_add(b, f[2].x, f[2].y); }
    if (cu) box_add_eqtri(b, cx, cy, rho);
    else { box_add(b, f[3].x, f[3].y); box_add(b, f[2].x, f[2].y); box_add(b, f[1].x, f[1].y); }
    return b;
}

struct LevelOut {
    float4* bbox;
    float4* bbox_all;
    float4* clu_n;
    float* clu_e;
    float2* clu_det;
    uint8_t* clu_deg;
};

// Level 1: every node integrates its 2 x 2 cells (8 fine triangles) directly and
// writes its leaf record.  Thread index = Morton code of the node.
__global__ void k_level1(HierDev H, LevelOut o, QuadRec* __restrict__ quad, double* __restrict__ mom,
                         int cluster)
{
    const int m = H.n >> 1;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)m * m) return;
    const int I = (int)morton_compact((uint32_t)t), J = (int)morton_compact((uint32_t)t >> 1);
    const int w = H.n + 1;
    {
        QuadRec r;
        for (int y = 0; y < 3; ++y)
            for (int x = 0; x < 3; ++x) r.t[3 * y + x] = H.nrm[(int64_t)(2 * J + y) * w + 2 * I + x];
        for (int dj = 0; dj < 2; ++dj)
            for (int di = 0; di < 2; ++di) r.deg[2 * dj + di] = H.deg[(int64_t)(2 * J + dj) * H.n + 2 * I + di];
        r.pad = 0;
        quad[t] = r;
    }
    double lo[kMom] = {0}, up[kMom] = {0};
    float4 box = empty_box();
    for (int dj = 0; dj < 2; ++dj)
        for (int di = 0; di < 2; ++di) {
            const int i = 2 * I + di, j = 2 * J + dj;
            const float2* p = H.nrm + (int64_t)j * w + i;
            const float2 n0 = p[0], n1 = p[1], n2 = p[w], n3 = p[w + 1];
            const uint8_t dg = H.deg[(int64_t)j * H.n + i];
            const float cx = 0.5f * (n1.x + n2.x), cy = 0.5f * (n1.y + n2.y);
            if (dg & 1) box_add_eqtri(box, cx, cy, H.rho);
            else { box_add(box, n0.x, n0.y); box_add(box, n1.x, n1.y); box_add(box, n2.x, n2.y); }
            if (dg & 2) box_add_eqtri(box, cx, cy, H.rho);
            else { box_add(box, n3.x, n3.y); box_add(box, n2.x, n2.y); box_add(box, n1.x, n1.y); }
            if (!cluster) continue;
            const double e = (double)H.eps;
            {   // lower (u0, u1, u2)
                const float2 nn[3] = {n0, n1, n2};
                const double u[3] = {(double)di, di + 1.0, (double)di};
                const double v[3] = {(double)dj, (double)dj, dj + 1.0};
                const double d = jac64(n0, n1, n2);
                tri_moments(1.0 / (d < e ? e : d), u, v, nn, (di + dj <= 1) ? lo : up);
            }
            {   // upper (u3, u2, u1)
                const float2 nn[3] = {n3, n2, n1};
                const double u[3] = {di + 1.0, (double)di, di + 1.0};
                const double v[3] = {dj + 1.0, dj + 1.0, (double)dj};
                const double d = jac64(n3, n2, n1);
                tri_moments(1.0 / (d < e ? e : d), u, v, nn, (di + dj <= 0) ? lo : up);
            }
        }
    o.bbox[t] = box;
    if (!cluster) return;
    double* M = mom + t * (2 * kMom);
    for (int k = 0; k < kMom; ++k) { M[k] = lo[k]; M[kMom + k] = up[k]; }
    double N[4][2], e;
    solve_cluster(lo, up, 2, N, &e);
    float4 cb = store_cluster(H, t, 2, N, e, o.clu_n, o.clu_e, o.clu_det, o.clu_deg);
    box_union(cb, box);
    o.bbox_all[t] = cb;
}

// Level l >= 2 from level l-1: boxes are unions of the children; moments are
// shifted into the parent frame and split over its halves.  Thread index = Morton
// code; the children of node t are 4t + (di + 2 dj).
__global__ void k_level_up(HierDev H, int level, LevelOut o, const float4* __restrict__ cbox,
                           const float4* __restrict__ cbox_all, const double* __restrict__ cmom,
                           double* __restrict__ mom, int cluster)
{
    const int m = H.n >> level;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)m * m) return;
    const int64_t c00 = 4 * t, c10 = c00 + 1, c01 = c00 + 2, c11 = c00 + 3;
    float4 box = cbox[c00];
    box_union(box, cbox[c10]);
    box_union(box, cbox[c01]);
    box_union(box, cbox[c11]);
    o.bbox[t] = box;
    if (!cluster) return;
    const double h = (double)(1 << (level - 1));
    double lo[kMom] = {0}, up[kMom] = {0};
    const double* M00 = cmom + c00 * (2 * kMom);
    const double* M10 = cmom + c10 * (2 * kMom);
    const double* M01 = cmom + c01 * (2 * kMom);
    const double* M11 = cmom + c11 * (2 * kMom);
    shift_add(M00, 0.0, 0.0, lo);
    shift_add(M00 + kMom, 0.0, 0.0, lo);
    shift_add(M10, h, 0.0, lo);
    shift_add(M01, 0.0, h, lo);
    shift_add(M11, h, h, up);
    shift_add(M11 + kMom, h, h, up);
    shift_add(M10 + kMom, h, 0.0, up);
    shift_add(M01 + kMom, 0.0, h, up);
    double* M = mom + t * (2 * kMom);
    for (int k = 0; k < kMom; ++k) { M[k] = lo[k]; M[kMom + k] = up[k]; }
    double N[4][2], e;
    solve_cluster(lo, up, 1 << level, N, &e);
    float4 cb = store_cluster(H, t, 1 << level, N, e, o.clu_n, o.clu_e, o.clu_det, o.clu_deg);
    box_union(cb, cbox_all[c00]);
    box_union(cb, cbox_all[c10]);
    box_union(cb, cbox_all[c01]);
    box_union(cb, cbox_all[c11]);
    o.bbox_all[t] = cb;
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

// The cut traversal's boxes in half precision, minima rounded down and maxima up: a
// rounded box contains the exact one, so it prunes a little less but never wrongly,
// and a parent's four child boxes take 32 B instead of 64 (the traversal under the
// cut is bound by memory traffic; the float32 boxes stay for the exports).
__global__ void k_half_boxes(const float4* __restrict__ src, uint2* __restrict__ dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float4 b = src[i];
    const uint32_t x0 = __half_as_ushort(__float2half_rd(b.x)), y0 = __half_as_ushort(__float2half_rd(b.y));
    const uint32_t x1 = __half_as_ushort(__float2half_ru(b.z)), y1 = __half_as_ushort(__float2half_ru(b.w));
    dst[i] = make_uint2(x0 | (y0 << 16), x1 | (y1 << 16));
}

hipError_t build_hierarchy_levels(pndf_hier* h, hipStream_t s)
{
    const HierDev& H = h->dev;
    const int n = H.n;
    const int64_t m1 = (int64_t)(n >> 1) * (n >> 1);
    double* mom[2] = {nullptr, nullptr};
    hipError_t err = hipSuccess;
    if (h->cluster) {
        const int64_t m2 = n >= 4 ? (int64_t)(n >> 2) * (n >> 2) : 1;
        err = hipMalloc(&mom[0], sizeof(double) * 2 * kMom * m1);
        if (err == hipSuccess) err = hipMalloc(&mom[1], sizeof(double) * 2 * kMom * m2);
        if (err != hipSuccess) {
            (void)hipFree(mom[0]);
            return err;
        }
    }
    auto out_for = [&](int level) {
        LevelOut o;
        const int64_t off = level_offset(H.logn, level);
        o.bbox = h->bbox + off;
        o.bbox_all = h->cluster ? h->bbox_all + off : nullptr;
        o.clu_n = h->cluster ? h->clu_n + 2 * off : nullptr;
        o.clu_e = h->cluster ? h->clu_e + off : nullptr;
        o.clu_det = h->cluster ? h->clu_det + off : nullptr;
        o.clu_deg = h->cluster ? h->clu_deg + off : nullptr;
        return o;
    };
    const int bs = 128;
    hipLaunchKernelGGL(k_level1, dim3((unsigned)((m1 + bs - 1) / bs)), dim3(bs), 0, s, H, out_for(1),
                       h->quad, mom[0], h->cluster);
    err = hipGetLastError();
    for (int level = 2; level <= H.L && err == hipSuccess; ++level) {
        const int64_t m = (int64_t)(n >> level) * (n >> level);
        const int64_t coff = level_offset(H.logn, level - 1);
        const double* cm = mom[(level - 2) & 1];
        double* om = mom[(level - 1) & 1];
        hipLaunchKernelGGL(k_level_up, dim3((unsigned)((m + bs - 1) / bs)), dim3(bs), 0, s, H,
                           level, out_for(level), h->bbox + coff,
                           h->cluster ? h->bbox_all + coff : nullptr, cm, om, h->cluster);
        err = hipGetLastError();
    }
    if (err == hipSuccess && h->cluster) {
        hipLaunchKernelGGL(k_half_boxes, dim3((unsigned)((h->nodes + 255) / 256)), dim3(256), 0, s, h->bbox_all,
                           h->bbox_h, h->nodes);
        err = hipGetLastError();
    }
    if (err == hipSuccess) err = hipStreamSynchronize(s);
    (void)hipFree(mom[0]);
    (void)hipFree(mom[1]);
    return err;
}

}  // namespace pndf
