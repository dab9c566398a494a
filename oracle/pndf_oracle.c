/*
 * FP64 CPU oracle for the manifold-based P-NDF (arXiv 2505.08985).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the GPU
 * library is checked against.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the library never does, and the two
 * share no code, headers, tables or constants.
 *
 * Everything here is double precision, evaluated from the float32 inputs
 * (converted exactly).  The few quantities that the method's definition fixes in
 * the query's own float32 precision (support half-width, support box, cut
 * threshold) are computed in float, as the definition below states.
 *
 * Definitions followed (section / equation names of the paper):
 *   - mesh: two triangles per texel cell, Eq. (interpolation) and Fig. normal_map;
 *     lower triangle (u0,u1,u2) with normals (n0,n1,n2), upper triangle
 *     (u3,u2,u1) with normals (n3,n2,n1); the map is periodic (a torus).
 *   - Jacobian: twice the normal-space triangle area, Eq. (jacobian).
 *   - clamp: triangles with Jacobian below eps are replaced by an equilateral
 *     triangle of area eps/2 centred at n(floor(u)+1/2), section "Preventing
 *     Jacobian singularity" and Eq. (debias).
 *   - evaluation: D(m,x) = sum over triangles in the footprint of
 *     k(a l0 + b l1 + c l2 - x) 1[m in n(tri)] / (2 |n(tri)|), Eq. (ndf_eval),
 *     with barycentrics as signed-area ratios (Table notation, "bary").
 *   - footprint kernel: normalised Gaussian of standard deviation sigma with
 *     support half-width r = 3 sigma (Results: "(6 sigma)^2 footprint"), truncated
 *     at texel-cell granularity: every triangle of every periodic cell image whose
 *     closed unit square meets [x-r, x+r] is included.
 *   - cluster hierarchy: four vertex normals per 2^l x 2^l node minimising the
 *     inverse-Jacobian-weighted L2 distance, Eq. (normal_optimization) and its
 *     supplement derivation; e^l is the minimised objective value.
 *   - cut: starting at the entry level ceil(log2 max(r)) (supplement, "Entry
 *     level"), descend until a node satisfies e^l <= r_x r_y tau (section
 *     "Acceleration by mesh clustering").
 *   - projected area (shadow-masking): Eq. lambda with the kernel constant over
 *     each triangle, the rotation to w_y = 0, clipping to the visible region, and
 *     the boundary integrals of Eq. area-integral / Eq. line-integral (section
 *     "Shadow-masking" and its supplement).
 *   - sampling: u from the footprint kernel over the support the evaluation
 *     integrates, m the normal of the triangle (or, with the cut, the cluster
 *     triangle) containing u, warped onto the replacement triangle when clamped
 *     (section "Sampling and evaluation", Eq. debias, and the remark on sampling
 *     n^l in "Acceleration by mesh clustering").
 *
 * Status of the pins: every function here is pinned by the CPU tests (flat map,
 * tilted triangle pair, linear field, mass invariant, Monte Carlo normal
 * histogram, the supplement's printed coefficient matrices, transpose
 * invariance; for sampling: scipy's normal quantile, the interpolated field,
 * uniformity of disk and box draws, the linear field through clusters, the
 * support kept by rejection, and histograms of samples against D; for the
 * projected area: the hemisphere's clipped-cosine closed form, the triangle
 * area at normal incidence, quadrature of the area integral, the footprint mass
 * at normal incidence, rotation invariance, Monte Carlo and the flat map) except the orientation of the equilateral replacement triangle,
 * which the paper leaves free ("any other shape"): parity unpinned, fixed by
 * convention (vertices at 90, 210, 330 degrees in (a, b, c) order).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_PI 3.14159265358979323846

/* ---------------------------------------------------------------- helpers -- */

static int ilog2_exact(int n)
{
    int l = 0;
    while ((1 << l) < n) l++;
    return ((1 << l) == n) ? l : -1;
}

static long floor_div(long a, long b) /* b > 0 */
{
    long q = a / b;
    if ((a % b != 0) && (a < 0)) q -= 1;
    return q;
}

static long ceil_div(long a, long b) /* b > 0 */
{
    return -floor_div(-a, b);
}

static long wrap(long a, long n) { long r = a % n; return r < 0 ? r + n : r; }

/* normal of texel (i, j), periodic */
static void texel(const float* nrm, int n, long i, long j, double out[2])
{
    long ii = wrap(i, n), jj = wrap(j, n);
    out[0] = (double)nrm[2 * (jj * n + ii) + 0];
    out[1] = (double)nrm[2 * (jj * n + ii) + 1];
}

/* |(c - a) x (b - a)|, the Jacobian of Eq. (jacobian).  Products are rounded
 * before the difference (no fused multiply-add) so the clamp decision is a
 * fixed function of the float inputs. */
static double jac(const double a[2], const double b[2], const double c[2])
{
    double p = (c[0] - a[0]) * (b[1] - a[1]);
    double q = (c[1] - a[1]) * (b[0] - a[0]);
    return fabs(p - q);
}

/* vertices of the equilateral replacement triangle: circumradius rho around
 * centre, vertices at 90, 210, 330 degrees assigned to (a, b, c) */
static void eqtri(const double centre[2], double rho, double v[3][2])
{
    static const double ang[3] = {90.0, 210.0, 330.0};
    for (int k = 0; k < 3; k++) {
        double t = ang[k] * OR_PI / 180.0;
        v[k][0] = centre[0] + rho * cos(t);
        v[k][1] = centre[1] + rho * sin(t);
    }
}

/* circumradius of an equilateral triangle of the given area */
static double eq_rho(double area) { return sqrt(4.0 * area / (3.0 * sqrt(3.0))); }

/* signed double area of (p, q, r) */
static double sarea2(const double p[2], const double q[2], const double r[2])
{
    return (q[0] - p[0]) * (r[1] - p[1]) - (q[1] - p[1]) * (r[0] - p[0]);
}

static double seg_dist(const double h[2], const double a[2], const double b[2])
{
    double ex = b[0] - a[0], ey = b[1] - a[1];
    double px = h[0] - a[0], py = h[1] - a[1];
    double ee = ex * ex + ey * ey;
    double t = ee > 0 ? (px * ex + py * ey) / ee : 0.0;
    if (t < 0) t = 0;
    if (t > 1) t = 1;
    double dx = px - t * ex, dy = py - t * ey;
    return sqrt(dx * dx + dy * dy);
}

/* ------------------------------------------------------------------ mesh -- */

/* Per cell (i, j): Jacobians of the lower and upper triangle and the clamp bits.
 * det[2*(j*n+i)+0] lower, +1 upper; deg bit0 = lower clamped, bit1 = upper. */
int or_mesh(int n, const float* nrm, float eps, double* det, uint8_t* deg)
{
    if (ilog2_exact(n) < 0 || n < 2) return 1;
    const double e = (double)eps;
    for (long j = 0; j < n; j++)
        for (long i = 0; i < n; i++) {
            double n0[2], n1[2], n2[2], n3[2];
            texel(nrm, n, i, j, n0);
            texel(nrm, n, i + 1, j, n1);
            texel(nrm, n, i, j + 1, n2);
            texel(nrm, n, i + 1, j + 1, n3);
            double dl = jac(n0, n1, n2);
            double du = jac(n3, n2, n1);
            det[2 * (j * n + i) + 0] = dl;
            det[2 * (j * n + i) + 1] = du;
            deg[j * n + i] = (uint8_t)((dl < e ? 1 : 0) | (du < e ? 2 : 0));
        }
    return 0;
}

/* --------------------------------------------------------------- cluster -- */

/* cluster barycentric basis lambda^l at node-local normalised coords (U, V) for
 * the cluster half `chalf` (0 lower: U+V<=1, 1 upper) */
static void clu_basis(double U, double V, int chalf, double lam[4])
{
    if (chalf == 0) {
        lam[0] = 1.0 - U - V; lam[1] = U; lam[2] = V; lam[3] = 0.0;
    } else {
        lam[0] = 0.0; lam[1] = 1.0 - V; lam[2] = 1.0 - U; lam[3] = U + V - 1.0;
    }
}

/* fine triangle `half` of local cell (li, lj) inside a node of side s: its uv
 * vertices (node-local), its normals, and which cluster half it lies in */
static int fine_tri(int s, int li, int lj, int half, const double nv[4][2],
                    double uv[3][2], double nn[3][2])
{
    if (half == 0) {
        uv[0][0] = li;     uv[0][1] = lj;
        uv[1][0] = li + 1; uv[1][1] = lj;
        uv[2][0] = li;     uv[2][1] = lj + 1;
        memcpy(nn[0], nv[0], sizeof nn[0]);
        memcpy(nn[1], nv[1], sizeof nn[1]);
        memcpy(nn[2], nv[2], sizeof nn[2]);
        return (li + lj <= s - 1) ? 0 : 1;
    }
    uv[0][0] = li + 1; uv[0][1] = lj + 1;
    uv[1][0] = li;     uv[1][1] = lj + 1;
    uv[2][0] = li + 1; uv[2][1] = lj;
    memcpy(nn[0], nv[3], sizeof nn[0]);
    memcpy(nn[1], nv[2], sizeof nn[1]);
    memcpy(nn[2], nv[1], sizeof nn[2]);
    return (li + lj <= s - 2) ? 0 : 1;
}

/* Contribution of one fine triangle to the gradient terms of the cluster
 * objective: A += w 2 int(lam lam^T), B += -w 2 int(lam n^T), C += w int(|n|^2),
 * by the three-edge-midpoint rule (exact for quadratics on a triangle; area 1/2).
 * With w = 1 these are the supplement's A_ij, B_ij matrices. */
static void fine_contrib(int s, const double uv[3][2], const double nn[3][2], int chalf,
                         double w, double A[4][4], double B[4][2], double* C)
{
    for (int k = 0; k < 3; k++) {
        int k2 = (k + 1) % 3;
        double mu = 0.5 * (uv[k][0] + uv[k2][0]) / s;
        double mv = 0.5 * (uv[k][1] + uv[k2][1]) / s;
        double mn[2] = {0.5 * (nn[k][0] + nn[k2][0]), 0.5 * (nn[k][1] + nn[k2][1])};
        double lam[4];
        clu_basis(mu, mv, chalf, lam);
        /* quadrature weight area/3 = 1/6; A and B carry the factor 2 */
        for (int a = 0; a < 4; a++) {
            for (int b = 0; b < 4; b++) A[a][b] += w * (2.0 / 6.0) * lam[a] * lam[b];
            B[a][0] += -w * (2.0 / 6.0) * lam[a] * mn[0];
            B[a][1] += -w * (2.0 / 6.0) * lam[a] * mn[1];
        }
        *C += w * (1.0 / 6.0) * (mn[0] * mn[0] + mn[1] * mn[1]);
    }
}

/* Exposed for the pin against the supplement's printed matrices: the fine cell
 * (i, j) of a node of side a, triangle `half` (0 = (i,j),(i+1,j),(i,j+1)),
 * corner normals nv = n0..n3 (x,y pairs), weight 1.  Returns the cluster half. */
int or_fine_contrib(int a, int i, int j, int half, const double* nv8,
                    double* A16, double* B8, double* C1)
{
    double nv[4][2], uv[3][2], nn[3][2], A[4][4] = {{0}}, B[4][2] = {{0}}, C = 0;
    for (int k = 0; k < 4; k++) { nv[k][0] = nv8[2 * k]; nv[k][1] = nv8[2 * k + 1]; }
    int ch = fine_tri(a, i, j, half, nv, uv, nn);
    fine_contrib(a, uv, nn, ch, 1.0, A, B, &C);
    memcpy(A16, A, sizeof A);
    memcpy(B8, B, sizeof B);
    *C1 = C;
    return ch;
}

/* plain Gaussian elimination with partial pivoting, A x = rhs (4 x 2) */
static int solve4(double A[4][4], double R[4][2], double X[4][2])
{
    double M[4][6];
    for (int r = 0; r < 4; r++) {
        for (int c = 0; c < 4; c++) M[r][c] = A[r][c];
        M[r][4] = R[r][0];
        M[r][5] = R[r][1];
    }
    for (int c = 0; c < 4; c++) {
        int p = c;
        for (int r = c + 1; r < 4; r++)
            if (fabs(M[r][c]) > fabs(M[p][c])) p = r;
        if (M[p][c] == 0.0) return 1;
        if (p != c)
            for (int k = 0; k < 6; k++) { double t = M[c][k]; M[c][k] = M[p][k]; M[p][k] = t; }
        for (int r = c + 1; r < 4; r++) {
            double f = M[r][c] / M[c][c];
            for (int k = c; k < 6; k++) M[r][k] -= f * M[c][k];
        }
    }
    for (int r = 3; r >= 0; r--)
        for (int q = 0; q < 2; q++) {
            double v = M[r][4 + q];
            for (int k = r + 1; k < 4; k++) v -= M[r][k] * X[k][q];
            X[r][q] = v / M[r][r];
        }
    return 0;
}

/* Cluster fit of node (level, I, J): argmin of Eq. (normal_optimization) with
 * weight 1 / max(Jacobian, eps), solved from A N = -B; e = objective at the
 * optimum, integrated again over every fine triangle.  nstar: N0..N3 (x, y). */
static int cluster_node(int n, const float* nrm, double eps, int level, long I, long J,
                        double nstar[8], double* e_out)
{
    const int s = 1 << level;
    double A[4][4] = {{0}}, B[4][2] = {{0}}, C = 0.0;
    for (int lj = 0; lj < s; lj++)
        for (int li = 0; li < s; li++) {
            double nv[4][2];
            long gi = I * s + li, gj = J * s + lj;
            texel(nrm, n, gi, gj, nv[0]);
            texel(nrm, n, gi + 1, gj, nv[1]);
            texel(nrm, n, gi, gj + 1, nv[2]);
            texel(nrm, n, gi + 1, gj + 1, nv[3]);
            for (int half = 0; half < 2; half++) {
                double uv[3][2], nn[3][2];
                int ch = fine_tri(s, li, lj, half, nv, uv, nn);
                double d = jac(nn[0], nn[1], nn[2]);
                double w = 1.0 / (d < eps ? eps : d);
                fine_contrib(s, uv, nn, ch, w, A, B, &C);
            }
        }
    double R[4][2], X[4][2];
    for (int a = 0; a < 4; a++) { R[a][0] = -B[a][0]; R[a][1] = -B[a][1]; }
    if (solve4(A, R, X)) return 1;
    double E = 0.0;
    for (int lj = 0; lj < s; lj++)
        for (int li = 0; li < s; li++) {
            double nv[4][2];
            long gi = I * s + li, gj = J * s + lj;
            texel(nrm, n, gi, gj, nv[0]);
            texel(nrm, n, gi + 1, gj, nv[1]);
            texel(nrm, n, gi, gj + 1, nv[2]);
            texel(nrm, n, gi + 1, gj + 1, nv[3]);
            for (int half = 0; half < 2; half++) {
                double uv[3][2], nn[3][2];
                int ch = fine_tri(s, li, lj, half, nv, uv, nn);
                double d = jac(nn[0], nn[1], nn[2]);
                double w = 1.0 / (d < eps ? eps : d);
                for (int k = 0; k < 3; k++) {
                    int k2 = (k + 1) % 3;
                    double mu = 0.5 * (uv[k][0] + uv[k2][0]) / s;
                    double mv = 0.5 * (uv[k][1] + uv[k2][1]) / s;
                    double lam[4];
                    clu_basis(mu, mv, ch, lam);
                    double fx = -0.5 * (nn[k][0] + nn[k2][0]);
                    double fy = -0.5 * (nn[k][1] + nn[k2][1]);
                    for (int a = 0; a < 4; a++) { fx += lam[a] * X[a][0]; fy += lam[a] * X[a][1]; }
                    E += w * (1.0 / 6.0) * (fx * fx + fy * fy);
                }
            }
        }
    for (int a = 0; a < 4; a++) { nstar[2 * a] = X[a][0]; nstar[2 * a + 1] = X[a][1]; }
    *e_out = E;
    return 0;
}

/* Cluster fits for `count` nodes of one level (node id = J * (n >> level) + I).
 * Parallel over nodes. */
int or_cluster_nodes(int n, const float* nrm, float eps, int level, const int64_t* ids,
                     int64_t count, double* nstar, double* e)
{
    int L = ilog2_exact(n);
    if (L < 1 || level < 1 || level > L) return 1;
    const long m = n >> level;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(| : bad)
    for (int64_t k = 0; k < count; k++) {
        long id = (long)ids[k];
        if (id < 0 || id >= m * m) { bad |= 1; continue; }
        bad |= cluster_node(n, nrm, (double)eps, level, id % m, id / m, nstar + 8 * k, e + k);
    }
    return bad;
}

/* -------------------------------------------------------------- evaluate -- */

typedef struct {
    int n, L;
    const float* nrm;
    double eps;
    const double* clu_n; /* all levels 1..L packed, 8 FP64 values per node (the oracle's own fit) */
    const double* clu_e; /* all levels 1..L packed, 1 FP64 value per node */
    double emax[32];     /* largest e^l of each level */
} map_t;

static long level_offset(int n, int level) /* first node of `level` in packed arrays */
{
    long off = 0;
    for (int l = 1; l < level; l++) off += (long)(n >> l) * (n >> l);
    return off;
}

typedef struct {
    double x, y, sx, sy, h[2];
    double rx, ry; /* support half-widths r = fl32(sigma_to_r * sigma) */
    long cxlo, cxhi, cylo, cyhi;
    int l0;
    float t; /* cut threshold (float, as fixed by the definition) */
    int use_cut;
    int kernel; /* 0 Gaussian, 1 disk, 2 box */
    double band;
} query_t;

/* relative band around the edge of the disk / box support within which the
 * inclusion of a hit point can flip under rounding (flags bit 1) */
#define OR_KERNEL_BAND 1e-9

/* Agreement of two independent FP64 fits of the cluster objective (the same
 * definition summed in different orders), used to flag the decisions that their
 * float32-rounded values could take differently (flags bit 0): e^l to 1e-10
 * relative plus 1e-20 of the level's largest e^l (for fits that are exact up to
 * rounding), the normals to 1e-10 absolute.  Measured agreement is ~1e-13 and
 * ~1e-12; the GPU tests check these bounds node by node. */
#define OR_FIT_E_REL 1e-10
#define OR_FIT_E_ABS 1e-20
#define OR_FIT_N_ABS 1e-10

typedef struct {
    double D;
    long nhit, namb;
    int flags; /* bit0: a cut decision that matters sits within rounding of the threshold;
                * bit1: a hit point sits within rounding of the disk / box support edge;
                * bit2: a cluster clamp decision that matters sits within rounding */
    /* optional record buffers (NULL = count only) */
    uint64_t* hid; double* hterm;
    uint64_t* aid; double* aterm; uint8_t* ahit;
} acc_t;

#define OR_ID(l, I, J, half) \
    (((uint64_t)(l) << 58) | ((uint64_t)(J) << 29) | ((uint64_t)(I) << 1) | (uint64_t)(half))

/* Could two fits within the agreement bound take the cut decision fl32(e) <= t
 * differently?  fl32(x) <= t exactly when x lies at or below the midpoint between
 * t and the next float32 (up to the tie), so only when e is that close to it. */
static int cut_may_flip(const map_t* m, int level, double e, float t)
{
    const double mid = 0.5 * ((double)t + (double)nextafterf(t, INFINITY));
    const double w = OR_FIT_E_REL * fabs(e) + OR_FIT_E_ABS * m->emax[level];
    return fabs(e - mid) <= w;
}

/* largest e^l of every level (for the absolute part of the agreement bound) */
static void level_emax(map_t* m)
{
    for (int l = 0; l < 32; l++) m->emax[l] = 0.0;
    if (!m->clu_e) return;
    for (int l = 1; l <= m->L; l++) {
        const long off = level_offset(m->n, l), cnt = (long)(m->n >> l) * (m->n >> l);
        double mx = 0.0;
        for (long k = 0; k < cnt; k++) mx = fmax(mx, m->clu_e[off + k]);
        m->emax[l] = mx;
    }
}

/* images p along one axis for a node of side s starting at torus cell `start`:
 * the node's closed square [start + pN, start + s + pN] meets the box iff one of
 * its unit cells lies in the included cell range [clo, chi] */
static void image_range(long start, long s, long clo, long chi, long n, long* p0, long* p1)
{
    *p0 = ceil_div(clo - start - s + 1, n);
    *p1 = floor_div(chi - start, n);
}

static double gauss_sum(double ucoord, long start, long s, long clo, long chi, long n,
                        double x, double sig)
{
    long p0, p1;
    image_range(start, s, clo, chi, n, &p0, &p1);
    double g = 0.0;
    for (long p = p0; p <= p1; p++) {
        double d = ucoord + (double)p * (double)n - x;
        g += exp(-d * d / (2.0 * sig * sig));
    }
    return g;
}

/* Box footprint (Table notation: k_r of size 2r_x x 2r_y, zero beyond r), one axis:
 * the number of included periodic images of the point u within distance r of x */
static double box_count(double ucoord, long start, long s, long clo, long chi, long n, double x, double r,
                        int* amb)
{
    long p0, p1;
    image_range(start, s, clo, chi, n, &p0, &p1);
    double c = 0.0;
    for (long p = p0; p <= p1; p++) {
        double d = fabs(ucoord + (double)p * (double)n - x);
        if (fabs(d - r) <= OR_KERNEL_BAND * r) *amb = 1;
        if (d <= r) c += 1.0;
    }
    return c;
}

/* Disk footprint (an ellipse of half-axes r_x, r_y): the number of included
 * periodic images (p, q) of u inside it */
static double disk_count(double ux, double uy, long I, long J, long s, const query_t* q, long n, int* amb)
{
    long p0, p1, q0, q1;
    image_range(I * s, s, q->cxlo, q->cxhi, n, &p0, &p1);
    image_range(J * s, s, q->cylo, q->cyhi, n, &q0, &q1);
    double c = 0.0;
    for (long p = p0; p <= p1; p++) {
        double dx = (ux + (double)p * (double)n - q->x) / q->rx;
        for (long r = q0; r <= q1; r++) {
            double dy = (uy + (double)r * (double)n - q->y) / q->ry;
            double e = dx * dx + dy * dy;
            if (fabs(e - 1.0) <= OR_KERNEL_BAND) *amb = 1;
            if (e <= 1.0) c += 1.0;
        }
    }
    return c;
}

/* Test one triangle with normal-space vertices nv (a, b, c) and uv vertices
 * (a, b, c); Jacobian det_used; node (level, I, J) of side s for the images. */
static void test_tri(const map_t* m, const query_t* q, acc_t* acc, uint64_t id,
                     const double nv[3][2], const double uv[3][2], double det_used,
                     long I, long J, long s)
{
    double S = sarea2(nv[0], nv[1], nv[2]);
    double l0 = sarea2(q->h, nv[1], nv[2]) / S;
    double l1 = sarea2(nv[0], q->h, nv[2]) / S;
    double l2 = sarea2(nv[0], nv[1], q->h) / S;
    int hit = (l0 >= 0 && l0 <= 1 && l1 >= 0 && l1 <= 1 && l2 >= 0 && l2 <= 1);
    int amb = 0;
    double dmin = seg_dist(q->h, nv[0], nv[1]);
    double d1 = seg_dist(q->h, nv[1], nv[2]);
    double d2 = seg_dist(q->h, nv[2], nv[0]);
    if (d1 < dmin) dmin = d1;
    if (d2 < dmin) dmin = d2;
    amb = dmin < q->band;
    if (!hit && !amb) return;
    double ux = uv[0][0] * l0 + uv[1][0] * l1 + uv[2][0] * l2;
    double uy = uv[0][1] * l0 + uv[1][1] * l1 + uv[2][1] * l2;
    double w; /* footprint kernel k_r(u* - x) summed over the included periodic images */
    if (q->kernel == 0) {
        double gx = gauss_sum(ux, I * s, s, q->cxlo, q->cxhi, m->n, q->x, q->sx);
        double gy = gauss_sum(uy, J * s, s, q->cylo, q->cyhi, m->n, q->y, q->sy);
        w = gx * gy / (2.0 * OR_PI * q->sx * q->sy);
    } else {
        int kamb = 0;
        if (q->kernel == 2) {
            double cx = box_count(ux, I * s, s, q->cxlo, q->cxhi, m->n, q->x, q->rx, &kamb);
            double cy = box_count(uy, J * s, s, q->cylo, q->cyhi, m->n, q->y, q->ry, &kamb);
            w = cx * cy / (4.0 * q->rx * q->ry);
        } else {
            w = disk_count(ux, uy, I, J, s, q, m->n, &kamb) / (OR_PI * q->rx * q->ry);
        }
        if (kamb && hit) acc->flags |= 2;
    }
    double term = w / det_used;
    if (hit) {
        if (acc->hid) { acc->hid[acc->nhit] = id; acc->hterm[acc->nhit] = term; }
        acc->nhit++;
        acc->D += term;
    }
    if (amb) {
        if (acc->aid) {
            acc->aid[acc->namb] = id; acc->aterm[acc->namb] = term;
            acc->ahit[acc->namb] = (uint8_t)hit;
        }
        acc->namb++;
    }
}

/* the two triangles of torus cell (i, j), clamp applied */
static void test_cell(const map_t* m, const query_t* q, acc_t* acc, long i, long j)
{
    double nv4[4][2];
    texel(m->nrm, m->n, i, j, nv4[0]);
    texel(m->nrm, m->n, i + 1, j, nv4[1]);
    texel(m->nrm, m->n, i, j + 1, nv4[2]);
    texel(m->nrm, m->n, i + 1, j + 1, nv4[3]);
    double centre[2] = {0.5 * (nv4[1][0] + nv4[2][0]), 0.5 * (nv4[1][1] + nv4[2][1])};
    for (int half = 0; half < 2; half++) {
        double nv[3][2], uv[3][2];
        if (half == 0) {
            memcpy(nv[0], nv4[0], sizeof nv[0]); memcpy(nv[1], nv4[1], sizeof nv[0]);
            memcpy(nv[2], nv4[2], sizeof nv[0]);
            uv[0][0] = i; uv[0][1] = j; uv[1][0] = i + 1; uv[1][1] = j; uv[2][0] = i; uv[2][1] = j + 1;
        } else {
            memcpy(nv[0], nv4[3], sizeof nv[0]); memcpy(nv[1], nv4[2], sizeof nv[0]);
            memcpy(nv[2], nv4[1], sizeof nv[0]);
            uv[0][0] = i + 1; uv[0][1] = j + 1; uv[1][0] = i; uv[1][1] = j + 1; uv[2][0] = i + 1; uv[2][1] = j;
        }
        double d = jac(nv[0], nv[1], nv[2]);
        double du = d;
        if (d < m->eps) {
            eqtri(centre, eq_rho(0.5 * m->eps), nv);
            du = m->eps;
        }
        test_tri(m, q, acc, OR_ID(0, i, j, half), nv, uv, du, i, j, 1);
    }
}

/* Could another fit, whose normals round to float32 values within
 * [fl32(x - 1e-10), fl32(x + 1e-10)] of this fit's FP64 normals x, take the clamp
 * decision Jacobian < lim of the cluster triangle with FP64 vertices v (a, b, c)
 * differently?  The Jacobian |(c - a) x (b - a)| over those intervals, by interval
 * arithmetic (with a relative slack for its own FP64 rounding), must contain lim. */
static void ivl_mul(double a0, double a1, double b0, double b1, double* lo, double* hi)
{
    double p[4] = {a0 * b0, a0 * b1, a1 * b0, a1 * b1};
    *lo = *hi = p[0];
    for (int k = 1; k < 4; k++) {
        if (p[k] < *lo) *lo = p[k];
        if (p[k] > *hi) *hi = p[k];
    }
}

static int clamp_may_flip(const double v[3][2], double lim)
{
    double lo[3][2], hi[3][2];
    for (int k = 0; k < 3; k++)
        for (int c = 0; c < 2; c++) {
            lo[k][c] = (double)(float)(v[k][c] - OR_FIT_N_ABS);
            hi[k][c] = (double)(float)(v[k][c] + OR_FIT_N_ABS);
        }
    double pl, ph, ql, qh;
    ivl_mul(lo[2][0] - hi[0][0], hi[2][0] - lo[0][0], lo[1][1] - hi[0][1], hi[1][1] - lo[0][1], &pl, &ph);
    ivl_mul(lo[2][1] - hi[0][1], hi[2][1] - lo[0][1], lo[1][0] - hi[0][0], hi[1][0] - lo[0][0], &ql, &qh);
    const double dl = pl - qh, dh = ph - ql;
    double al, ah;
    if (dl >= 0.0) { al = dl; ah = dh; }
    else if (dh <= 0.0) { al = -dh; ah = -dl; }
    else { al = 0.0; ah = fmax(-dl, dh); }
    const double slack = 1e-14 * (fmax(fabs(pl), fabs(ph)) + fmax(fabs(ql), fabs(qh)));
    return al - slack <= lim && lim <= ah + slack;
}

/* the two cluster triangles of node (level, I, J): corners at spacing s, normals
 * from the cluster fit; Jacobian with respect to u is 2 area_n / s^2, clamped at
 * eps with an equilateral triangle of area eps s^2 / 2 */
static void test_cluster(const map_t* m, const query_t* q, acc_t* acc, int level, long I, long J)
{
    const long s = 1L << level;
    const long mm = m->n >> level;
    const double* cn = m->clu_n + 8 * (level_offset(m->n, level) + J * mm + I);
    double N[4][2], N64[4][2];
    for (int k = 0; k < 4; k++)
        for (int c = 0; c < 2; c++) {
            N64[k][c] = cn[2 * k + c];
            N[k][c] = (double)(float)cn[2 * k + c];
        }
    double centre[2] = {0.5 * (N[1][0] + N[2][0]), 0.5 * (N[1][1] + N[2][1])};
    const double s2 = (double)s * (double)s;
    for (int half = 0; half < 2; half++) {
        double nv[3][2], uv[3][2], eq[3][2], v64[3][2];
        double X0 = (double)(I * s), Y0 = (double)(J * s), X1 = X0 + s, Y1 = Y0 + s;
        const int vi[2][3] = {{0, 1, 2}, {3, 2, 1}};
        for (int k = 0; k < 3; k++) {
            memcpy(nv[k], N[vi[half][k]], sizeof nv[k]);
            memcpy(v64[k], N64[vi[half][k]], sizeof v64[k]);
        }
        if (half == 0) {
            uv[0][0] = X0; uv[0][1] = Y0; uv[1][0] = X1; uv[1][1] = Y0; uv[2][0] = X0; uv[2][1] = Y1;
        } else {
            uv[0][0] = X1; uv[0][1] = Y1; uv[1][0] = X0; uv[1][1] = Y1; uv[2][0] = X1; uv[2][1] = Y0;
        }
        double jn = jac(nv[0], nv[1], nv[2]);
        double du = jn / s2;
        eqtri(centre, eq_rho(0.5 * m->eps * s2), eq);
        if (clamp_may_flip(v64, m->eps * s2)) {
            /* the clamp decision could differ: it matters if either version of the
             * triangle holds a hit or an edge-ambiguous query normal */
            acc_t a, b;
            memset(&a, 0, sizeof a);
            memset(&b, 0, sizeof b);
            test_tri(m, q, &a, OR_ID(level, I, J, half), nv, uv, du, I, J, s);
            test_tri(m, q, &b, OR_ID(level, I, J, half), eq, uv, m->eps, I, J, s);
            if (a.nhit || a.namb || b.nhit || b.namb) acc->flags |= 4;
        }
        if (du < m->eps)
            test_tri(m, q, acc, OR_ID(level, I, J, half), eq, uv, m->eps, I, J, s);
        else
            test_tri(m, q, acc, OR_ID(level, I, J, half), nv, uv, du, I, J, s);
    }
}

/* does node (level, I, J) overlap the box in some periodic image (per axis) */
static int node_in(const query_t* q, int n, int level, long I, long J)
{
    long s = 1L << level, p0, p1;
    image_range(I * s, s, q->cxlo, q->cxhi, n, &p0, &p1);
    if (p0 > p1) return 0;
    image_range(J * s, s, q->cylo, q->cyhi, n, &p0, &p1);
    return p0 <= p1;
}

/* top-down cut: from a node at or below the entry level, stop at the first node
 * with e^l <= t (levels >= 1), else descend; cells represent themselves */
static void descend(const map_t* m, const query_t* q, acc_t* acc, int level, long I, long J)
{
    if (!node_in(q, m->n, level, I, J)) return;
    if (level == 0) { test_cell(m, q, acc, I, J); return; }
    long mm = m->n >> level;
    const double e64 = m->clu_e[level_offset(m->n, level) + J * mm + I];
    const float e = (float)e64;
    if (cut_may_flip(m, level, e64, q->t)) {
        /* the decision sits within rounding of the threshold; it can change the
         * result only if one of its two outcomes (this node's cluster triangles,
         * or the cut beneath it) holds a hit or an edge-ambiguous triangle */
        acc_t a, b;
        memset(&a, 0, sizeof a);
        memset(&b, 0, sizeof b);
        test_cluster(m, q, &a, level, I, J);
        for (int dj = 0; dj < 2; dj++)
            for (int di = 0; di < 2; di++) descend(m, q, &b, level - 1, 2 * I + di, 2 * J + dj);
        if (a.nhit || a.namb || b.nhit || b.namb) acc->flags |= 1;
        acc->flags |= b.flags;
    }
    if (e <= q->t) { test_cluster(m, q, acc, level, I, J); return; }
    for (int dj = 0; dj < 2; dj++)
        for (int di = 0; di < 2; di++) descend(m, q, acc, level - 1, 2 * I + di, 2 * J + dj);
}

static int setup_query(const map_t* m, const float* qr, float tau, float s2r, double band, int kernel,
                       query_t* q)
{
    float x = qr[0], y = qr[1], sx = qr[2], sy = qr[3], hx = qr[4], hy = qr[5];
    const float lim = 16777216.0f; /* 2^24 */
    if (!(isfinite(x) && isfinite(y) && isfinite(sx) && isfinite(sy) && isfinite(hx) &&
          isfinite(hy)))
        return 1;
    if (!(sx > 0.0f && sy > 0.0f)) return 1;
    float rx = s2r * sx, ry = s2r * sy; /* float products */
    if (!(fabsf(x) <= lim && fabsf(y) <= lim && rx <= lim && ry <= lim)) return 1;
    float lox = x - rx, hix = x + rx, loy = y - ry, hiy = y + ry;
    q->x = x; q->y = y; q->sx = sx; q->sy = sy; q->h[0] = hx; q->h[1] = hy;
    q->rx = rx; q->ry = ry;
    q->kernel = kernel;
    q->cxlo = (long)ceilf(lox) - 1; q->cxhi = (long)floorf(hix);
    q->cylo = (long)ceilf(loy) - 1; q->cyhi = (long)floorf(hiy);
    float rmax = rx > ry ? rx : ry;
    int l0 = 0;
    while (l0 < m->L && (float)(1L << l0) < rmax) l0++;
    q->l0 = l0;
    float rr = rx * ry;
    q->t = rr * tau;
    q->use_cut = tau > 0.0f;
    q->band = band;
    return 0;
}

/* included torus indices along one axis: all of them when the cell range is at
 * least one period long, else the range itself (each unrolled cell is then a
 * distinct torus cell) */
static long axis_cells(long clo, long chi, long n, long* idx)
{
    long cnt = 0;
    if (chi - clo + 1 >= n) {
        for (long i = 0; i < n; i++) idx[cnt++] = i;
    } else {
        for (long c = clo; c <= chi; c++) idx[cnt++] = wrap(c, n);
    }
    return cnt;
}

static void eval_one(const map_t* m, const query_t* q, acc_t* acc)
{
    const long n = m->n;
    long* xi = (long*)malloc(sizeof(long) * (size_t)n);
    long* yj = (long*)malloc(sizeof(long) * (size_t)n);
    long nx = axis_cells(q->cxlo, q->cxhi, n, xi);
    long ny = axis_cells(q->cylo, q->cyhi, n, yj);
    if (!q->use_cut) {
        /* brute force over every included periodic cell (Eq. ndf_eval) */
        for (long b = 0; b < ny; b++)
            for (long a = 0; a < nx; a++) test_cell(m, q, acc, xi[a], yj[b]);
    } else {
        /* roots: every node of the entry level that overlaps the box */
        const long mm = n >> q->l0;
        uint8_t* rx = (uint8_t*)calloc((size_t)mm, 1);
        uint8_t* ry = (uint8_t*)calloc((size_t)mm, 1);
        for (long a = 0; a < nx; a++) rx[xi[a] >> q->l0] = 1;
        for (long b = 0; b < ny; b++) ry[yj[b] >> q->l0] = 1;
        for (long J = 0; J < mm; J++)
            for (long I = 0; I < mm; I++)
                if (rx[I] && ry[J]) descend(m, q, acc, q->l0, I, J);
        free(rx);
        free(ry);
    }
    free(xi);
    free(yj);
}

/*
 * Evaluate nq queries (6 floats each: x, y, sx, sy, hx, hy).
 *  D[k]      the P-NDF value (NaN for an invalid query: non-finite input, sigma <= 0,
 *            |x|, |y| or r above 2^24)
 *  nhit[k]   number of hit triangles, namb[k] number of triangles within `band` of h
 *  flags[k]  bit0 = a cut decision that another FP64 fit (within the agreement
 *            bound above) could take differently after float32 rounding, with a hit or
 *            an edge-ambiguous triangle in one of its two outcomes;
 *            bit2 = likewise a cluster triangle's clamp decision, with either version
 *            hit or edge-ambiguous;
 *            bit1 = (disk / box) a hit point lies within 1e-9 relative of the support edge
 * kernel: 0 Gaussian (sigma the standard deviation, support r = s2r sigma), 1 disk
 * (the ellipse of half-axes r), 2 box (|u - x| <= r per axis); disk and box are
 * normalised over their support and truncated at the hit point (Table notation:
 * k_r is zero beyond r), the cells included are those meeting the support box.
 * If hoff/aoff (prefix offsets from a previous counting call) are given, the
 * records are written: hit ids + terms, ambiguous ids + terms + hit flags.
 * tau > 0 requires clu_n / clu_e: the FP64 cluster fit, all levels packed (the
 * evaluation uses their float32 roundings, as stored by a hierarchy).
 */
int or_eval_k(int n, const float* nrm, float eps, const double* clu_n, const double* clu_e,
              const float* queries, int64_t nq, float tau, float s2r, double band, int kernel,
              double* D, int64_t* nhit, int64_t* namb, int32_t* flags,
              const int64_t* hoff, uint64_t* hid, double* hterm,
              const int64_t* aoff, uint64_t* aid, double* aterm, uint8_t* ahit)
{
    if (kernel < 0 || kernel > 2) return 3;
    map_t m;
    m.n = n;
    m.L = ilog2_exact(n);
    if (m.L < 1) return 1;
    m.nrm = nrm;
    m.eps = (double)eps;
    m.clu_n = clu_n;
    m.clu_e = clu_e;
    level_emax(&m);
    if (tau > 0.0f && (!clu_n || !clu_e)) return 2;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < nq; k++) {
        query_t q;
        acc_t acc;
        memset(&acc, 0, sizeof acc);
        if (setup_query(&m, queries + 6 * k, tau, s2r, band, kernel, &q)) {
            D[k] = NAN;
            if (nhit) nhit[k] = 0;
            if (namb) namb[k] = 0;
            if (flags) flags[k] = 0;
            continue;
        }
        if (hoff && hid) { acc.hid = hid + hoff[k]; acc.hterm = hterm + hoff[k]; }
        if (aoff && aid) { acc.aid = aid + aoff[k]; acc.aterm = aterm + aoff[k]; acc.ahit = ahit + aoff[k]; }
        eval_one(&m, &q, &acc);
        D[k] = acc.D;
        if (nhit) nhit[k] = acc.nhit;
        if (namb) namb[k] = acc.namb;
        if (flags) flags[k] = acc.flags;
    }
    return 0;
}

/* or_eval_k with the Gaussian footprint kernel */
int or_eval(int n, const float* nrm, float eps, const double* clu_n, const double* clu_e,
            const float* queries, int64_t nq, float tau, float s2r, double band,
            double* D, int64_t* nhit, int64_t* namb, int32_t* flags,
            const int64_t* hoff, uint64_t* hid, double* hterm,
            const int64_t* aoff, uint64_t* aid, double* aterm, uint8_t* ahit)
{
    return or_eval_k(n, nrm, eps, clu_n, clu_e, queries, nq, tau, s2r, band, 0, D, nhit, namb, flags, hoff, hid,
                     hterm, aoff, aid, aterm, ahit);
}

/* the normal field n(u) of Eq. (interpolation) at texture coordinates u (periodic),
 * and the clamp-consistent sampling map of Eq. (debias) for clamped triangles:
 * a point of a clamped triangle goes to the same barycentric point of its
 * equilateral replacement.  Used by the Monte Carlo histogram pin. */
int or_sample_normals(int n, const float* nrm, float eps, const double* u, int64_t count,
                      double* mout)
{
    if (ilog2_exact(n) < 0) return 1;
    for (int64_t k = 0; k < count; k++) {
        double fx = floor(u[2 * k]), fy = floor(u[2 * k + 1]);
        double a = u[2 * k] - fx, b = u[2 * k + 1] - fy;
        long i = (long)fx, j = (long)fy;
        double nv4[4][2];
        texel(nrm, n, i, j, nv4[0]);
        texel(nrm, n, i + 1, j, nv4[1]);
        texel(nrm, n, i, j + 1, nv4[2]);
        texel(nrm, n, i + 1, j + 1, nv4[3]);
        double nv[3][2], w[3];
        if (a + b < 1.0) {
            memcpy(nv[0], nv4[0], sizeof nv[0]); memcpy(nv[1], nv4[1], sizeof nv[0]);
            memcpy(nv[2], nv4[2], sizeof nv[0]);
            w[0] = 1.0 - a - b; w[1] = a; w[2] = b;
        } else {
            memcpy(nv[0], nv4[3], sizeof nv[0]); memcpy(nv[1], nv4[2], sizeof nv[0]);
            memcpy(nv[2], nv4[1], sizeof nv[0]);
            w[0] = a + b - 1.0; w[1] = 1.0 - a; w[2] = 1.0 - b;
        }
        if (jac(nv[0], nv[1], nv[2]) < (double)eps) {
            double centre[2] = {0.5 * (nv4[1][0] + nv4[2][0]), 0.5 * (nv4[1][1] + nv4[2][1])};
            eqtri(centre, eq_rho(0.5 * (double)eps), nv);
        }
        mout[2 * k] = w[0] * nv[0][0] + w[1] * nv[1][0] + w[2] * nv[2][0];
        mout[2 * k + 1] = w[0] * nv[0][1] + w[1] * nv[1][1] + w[2] * nv[2][1];
    }
    return 0;
}

/* ------------------------------------------------------------- sampling -- */
/*
 * Sampling of the P-NDF (section "Sampling and evaluation", Eq. debias; with the
 * cut, section "Acceleration by mesh clustering": sampling uses the same normal
 * field n^l as the evaluation).  u is drawn from the footprint kernel over the
 * same support the evaluation integrates, then m is the normal of the triangle
 * containing u: n(u) by barycentric interpolation, or the same barycentric point
 * of the equilateral replacement for a clamped triangle.  The density of m is
 * then D(m) divided by D's total mass.
 *
 * Support (the evaluation's, R2 and R10): at tau = 0, the included cells
 * [cxlo, cxhi + 1] per axis; with the cut, the units of the cut (cells or
 * cluster nodes) whose unrolled image meets the included cells.  The Gaussian is
 * drawn by inverse CDF on a per-axis range S (the included cells at tau = 0; the
 * entry-level nodes over them with the cut) and, with the cut, rejected when its
 * unit does not meet the included cells (the next uniform pair is then used).
 * Disk and box supports lie inside the included cells, so their draws are
 * direct: uniform on the ellipse (radius sqrt(xi0), angle 2 pi xi1) or rectangle.
 */

/* standard normal CDF */
static double std_cdf(double z) { return 0.5 * erfc(-z / sqrt(2.0)); }

/* its inverse, by bisection on the monotone CDF (slow, plain) */
static double std_cdf_inv(double p)
{
    double lo = -40.0, hi = 40.0;
    for (int it = 0; it < 400; it++) {
        double mid = 0.5 * (lo + hi);
        if (hi - lo <= 1e-15 * (fabs(mid) > 1.0 ? fabs(mid) : 1.0)) break;
        if (std_cdf(mid) < p) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* u on [a, b) from the Gaussian N(x, sig^2) truncated to [a, b), by inverse CDF */
static double trunc_gauss(double x, double sig, double a, double b, double xi)
{
    double pa = std_cdf((a - x) / sig), pb = std_cdf((b - x) / sig);
    double u = x + sig * std_cdf_inv(pa + xi * (pb - pa));
    if (u < a) u = a;
    if (u >= b) u = nextafter(b, a);
    return u;
}

/* the unit of the cut that contains u: level (0 = a cell) and its torus node;
 * flag bit0 when another fit could take a decision on the way differently */
static int cut_unit(const map_t* m, const query_t* q, const double u[2], long* I, long* J, int* flag)
{
    if (q->use_cut)
        for (int l = q->l0; l >= 1; l--) {
            long s = 1L << l, mm = m->n >> l;
            long Il = wrap((long)floor(u[0] / (double)s), mm), Jl = wrap((long)floor(u[1] / (double)s), mm);
            const double e64 = m->clu_e[level_offset(m->n, l) + Jl * mm + Il];
            const float e = (float)e64;
            if (cut_may_flip(m, l, e64, q->t)) *flag |= 1;
            if (e <= q->t) { *I = Il; *J = Jl; return l; }
        }
    *I = wrap((long)floor(u[0]), m->n);
    *J = wrap((long)floor(u[1]), m->n);
    return 0;
}

/* does the unrolled image of the level-l unit holding coordinate c meet [clo, chi]
 * (cells) */
static int unit_meets(double c, int l, long clo, long chi)
{
    long s = 1L << l;
    long start = (long)floor(c / (double)s) * s;
    return start <= chi && start + s - 1 >= clo;
}

/* m at u inside unit (level, I, J): the two triangles of the cell (level 0, the
 * map's normals, Eq. interpolation) or of the cluster node (normals N0..N3);
 * clamped triangles are replaced as in the evaluation.  Returns the half; flag
 * bit1 when u lies within `band` (unit-local) of the unit's edges or diagonal. */
static int unit_normal(const map_t* m, int level, long I, long J, const double u[2], double band, double mo[2],
                       int* flag)
{
    const double s = (double)(1L << level);
    double U = (u[0] - floor(u[0] / s) * s) / s, V = (u[1] - floor(u[1] / s) * s) / s;
    double dmin = U;
    if (1.0 - U < dmin) dmin = 1.0 - U;
    if (V < dmin) dmin = V;
    if (1.0 - V < dmin) dmin = 1.0 - V;
    if (fabs(U + V - 1.0) < dmin) dmin = fabs(U + V - 1.0);
    if (dmin < band) *flag |= 2;
    double N[4][2], N64[4][2];
    if (level == 0) {
        texel(m->nrm, m->n, I, J, N[0]);
        texel(m->nrm, m->n, I + 1, J, N[1]);
        texel(m->nrm, m->n, I, J + 1, N[2]);
        texel(m->nrm, m->n, I + 1, J + 1, N[3]);
    } else {
        const double* cn = m->clu_n + 8 * (level_offset(m->n, level) + J * (m->n >> level) + I);
        for (int k = 0; k < 4; k++)
            for (int c = 0; c < 2; c++) {
                N64[k][c] = cn[2 * k + c];
                N[k][c] = (double)(float)cn[2 * k + c];
            }
    }
    int half = U + V < 1.0 ? 0 : 1;
    double nv[3][2], w[3];
    if (half == 0) {
        memcpy(nv[0], N[0], sizeof nv[0]); memcpy(nv[1], N[1], sizeof nv[0]); memcpy(nv[2], N[2], sizeof nv[0]);
        w[0] = 1.0 - U - V; w[1] = U; w[2] = V;
    } else {
        memcpy(nv[0], N[3], sizeof nv[0]); memcpy(nv[1], N[2], sizeof nv[0]); memcpy(nv[2], N[1], sizeof nv[0]);
        w[0] = U + V - 1.0; w[1] = 1.0 - U; w[2] = 1.0 - V;
    }
    /* the clamp of the evaluation (test_cell / test_cluster): Jacobian per unit uv area;
     * a cluster's decision within rounding of eps is flagged as in the evaluation */
    const double jn = jac(nv[0], nv[1], nv[2]);
    if (level > 0) {
        const int vi[2][3] = {{0, 1, 2}, {3, 2, 1}};
        double v64[3][2];
        for (int k = 0; k < 3; k++) memcpy(v64[k], N64[vi[half][k]], sizeof v64[k]);
        if (clamp_may_flip(v64, m->eps * s * s)) *flag |= 1;
    }
    if (jn / (s * s) < m->eps) {
        double centre[2] = {0.5 * (N[1][0] + N[2][0]), 0.5 * (N[1][1] + N[2][1])};
        eqtri(centre, eq_rho(0.5 * m->eps * s * s), nv);
    }
    mo[0] = w[0] * nv[0][0] + w[1] * nv[1][0] + w[2] * nv[2][0];
    mo[1] = w[0] * nv[0][1] + w[1] * nv[1][1] + w[2] * nv[2][1];
    return half;
}

/*
 * Draw nq samples (queries as for or_sample_k's evaluation: x, y, sx, sy used).
 * xi: attempts pairs of uniforms in [0, 1) per query, row-major (nq x 2 attempts).
 * Outputs: u (2 per query, unrolled texture coordinates), m (2 per query), tri
 * (triangle id as in the evaluation's hit lists), flags: bit0 a cut decision on
 * the way, or a cluster clamp decision, that another fit could take differently
 * (as for the evaluation); bit1 u within `band` of a unit edge or
 * diagonal (the triangle may differ under rounding) or of the rejection
 * boundary; bit2 every attempt was rejected (m = NaN).  Invalid queries, or a
 * pair of uniforms outside [0, 1) among those used, give NaN with tri = ~0.
 */
int or_sample_k(int n, const float* nrm, float eps, const double* clu_n, const double* clu_e,
                const float* queries, const double* xi, int64_t nq, int attempts, float tau, float s2r,
                double band, int kernel, double* uout, double* mout, uint64_t* tri, int32_t* flags)
{
    if (kernel < 0 || kernel > 2) return 3;
    if (attempts < 1) return 4;
    map_t m;
    m.n = n;
    m.L = ilog2_exact(n);
    if (m.L < 1) return 1;
    m.nrm = nrm;
    m.eps = (double)eps;
    m.clu_n = clu_n;
    m.clu_e = clu_e;
    level_emax(&m);
    if (tau > 0.0f && (!clu_n || !clu_e)) return 2;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < nq; k++) {
        query_t q;
        int fl = 0;
        double u[2] = {NAN, NAN}, mo[2] = {NAN, NAN};
        uint64_t id = ~(uint64_t)0;
        int bad = setup_query(&m, queries + 6 * k, tau, s2r, 0.0, kernel, &q);
        int done = 0;
        for (int a = 0; !bad && a < attempts && !done; a++) {
            double x0 = xi[(2 * k) * attempts + 2 * a], x1 = xi[(2 * k) * attempts + 2 * a + 1];
            /* a pair that is used must be uniforms in [0, 1) */
            if (!(x0 >= 0.0 && x0 < 1.0 && x1 >= 0.0 && x1 < 1.0)) { bad = 1; break; }
            if (kernel == 1) {
                double rad = sqrt(x0), ang = 2.0 * OR_PI * x1;
                u[0] = q.x + q.rx * rad * cos(ang);
                u[1] = q.y + q.ry * rad * sin(ang);
            } else if (kernel == 2) {
                u[0] = q.x + q.rx * (2.0 * x0 - 1.0);
                u[1] = q.y + q.ry * (2.0 * x1 - 1.0);
            } else {
                /* the per-axis range S: included cells, or the entry-level nodes over them */
                int l = q.use_cut ? q.l0 : 0;
                long sl = 1L << l;
                double ax = (double)(floor_div(q.cxlo, sl) * sl), bx = (double)((floor_div(q.cxhi, sl) + 1) * sl);
                double ay = (double)(floor_div(q.cylo, sl) * sl), by = (double)((floor_div(q.cyhi, sl) + 1) * sl);
                u[0] = trunc_gauss(q.x, q.sx, ax, bx, x0);
                u[1] = trunc_gauss(q.y, q.sy, ay, by, x1);
            }
            long I, J;
            int ufl = 0;
            int lev = cut_unit(&m, &q, u, &I, &J, &ufl);
            /* (flags u near the unit's edges, which also decide the rejection) */
            int half = unit_normal(&m, lev, I, J, u, band, mo, &ufl);
            fl |= ufl;
            if (kernel == 0 && q.use_cut &&
                !(unit_meets(u[0], lev, q.cxlo, q.cxhi) && unit_meets(u[1], lev, q.cylo, q.cyhi)))
                continue; /* rejected: the unit lies outside the support */
            id = OR_ID(lev, I, J, half);
            done = 1;
        }
        if (bad) {
            u[0] = u[1] = NAN;
            mo[0] = mo[1] = NAN;
            id = ~(uint64_t)0;
            fl = 0;
        } else if (!done) {
            fl |= 4;
            mo[0] = mo[1] = NAN;
            id = ~(uint64_t)0;
        }
        uout[2 * k] = u[0];
        uout[2 * k + 1] = u[1];
        mout[2 * k] = mo[0];
        mout[2 * k + 1] = mo[1];
        tri[k] = id;
        flags[k] = fl;
    }
    return 0;
}

/* ------------------------------------------------------- projected area -- */
/*
 * Projected area of the P-NDF (section "Shadow-masking", Eq. lambda):
 *   P(w) = integral of D(m) max(m~ . w, 0) over the solid angle of m~, m~ the unit
 * normal (m_x, m_y, sqrt(1 - |m|^2)) over the projected normal m.  With the
 * footprint kernel taken constant over each triangle (its value at the
 * triangle's uv centroid), Eq. area-integral gives
 *   P(w) = sum over triangles k(tri) / J(tri) * integral over n+(tri) of
 *          (w_x m_x / m~_z + w_z) dm
 * in the frame rotated about z so that w_y = 0 and w_x >= 0; J is the (clamped)
 * Jacobian and n+(tri) the part of the normal triangle where m~ . w >= 0 and
 * |m| <= 1.  That region V is bounded on the right by the unit circle and on the
 * left by the semi-ellipse m_x = -w_z sqrt(1 - m_y^2), and is convex.
 *
 * The integral over n+(tri) is a boundary integral by Stokes' theorem, the curl of
 * (0, w_z m_x - w_x m~_z, 0) being the integrand (supplement, "Correctness of the
 * area-line integral conversion"): the counter-clockwise boundary integral of
 * F dm_y, F = w_z m_x - w_x m~_z, over the clipped edges of the triangle and the
 * pieces of the boundary of V between them.  Closed forms, with
 * S(y) = (asin y + y sqrt(1 - y^2)) / 2 (the integral of sqrt(1 - t^2) from 0):
 *   segment P -> Q: w_z (Q_y - P_y)(Q_x + P_x) / 2 - w_x d_y r^2 [S(p/r)] from
 *     p = d.P to d.Q, d the unit direction, r = sqrt(1 - s^2), s the line's
 *     distance to the origin (on the line, m~_z = sqrt(r^2 - p^2));
 *   unit-circle arc (m~_z = 0, m_x = sqrt(1 - y^2)): w_z [S(y)] between its ends;
 *   ellipse arc (F = -sqrt(1 - y^2) there): -[S(y)] between its ends.
 * (The supplement's printed sign of the segment's arcsine term and its "d_x"
 * disagree with its own derivation; these follow the mathematics.)
 */

static double S_half(double y)
{
    if (y > 1.0) y = 1.0;
    if (y < -1.0) y = -1.0;
    return 0.5 * (asin(y) + y * sqrt(1.0 - y * y));
}

/* in the region V (closed), for the canonical w = (wx, 0, wz) */
static int in_vis(double x, double y, double wz)
{
    if (x * x + y * y > 1.0) return 0;
    if (x >= 0.0) return 1;
    return x * x + wz * wz * y * y <= wz * wz;
}

/* the boundary integral of F dm_y along the segment P -> Q (inside V) */
static double seg_term(const double P[2], const double Q[2], double wx, double wz)
{
    double dx = Q[0] - P[0], dy = Q[1] - P[1];
    double len = sqrt(dx * dx + dy * dy);
    if (len == 0.0) return 0.0;
    double t = 0.5 * wz * dy * (Q[0] + P[0]);
    dx /= len;
    dy /= len;
    double s = dy * P[0] - dx * P[1];
    double r2 = 1.0 - s * s;
    if (r2 <= 0.0) return t; /* tangent to the unit circle: m~_z = 0 on it */
    double r = sqrt(r2);
    double p0 = dx * P[0] + dy * P[1], p1 = dx * Q[0] + dy * Q[1];
    return t - wx * dy * r2 * (S_half(p1 / r) - S_half(p0 / r));
}

/* position of a boundary point of V along its counter-clockwise traversal,
 * starting at (0, -1): the right semicircle (y from -1 to 1) maps to y + 1 in
 * [0, 2], the left semi-ellipse (y from 1 to -1) to 3 - y in [2, 4].  A point is
 * on the semicircle when x >= 0 and it lies on the unit circle (at w_z = 0 the
 * semi-ellipse is the segment x = 0 inside the disk) */
static double vis_pos(double x, double y)
{
    if (y > 1.0) y = 1.0;
    if (y < -1.0) y = -1.0;
    return (x >= 0.0 && x * x + y * y >= 1.0 - 1e-9) ? y + 1.0 : 3.0 - y;
}

/* the boundary integral of F dm_y along the boundary of V counter-clockwise
 * from position a to position b (a <= b < a + 4, positions modulo 4) */
static double arc_term(double a, double b, double wz)
{
    double sum = 0.0;
    while (b - a > 1e-300) {
        double base = floor(a / 2.0) * 2.0; /* start of the current half */
        double end = base + 2.0 < b ? base + 2.0 : b;
        double la = a - base, lb = end - base; /* in [0, 2] */
        if (fmod(base, 4.0) == 0.0) {
            /* right semicircle: y = pos - 1, F = w_z sqrt(1 - y^2) */
            sum += wz * (S_half(lb - 1.0) - S_half(la - 1.0));
        } else {
            /* left semi-ellipse: y = 1 - pos, F = -sqrt(1 - y^2), y decreasing */
            sum += -(S_half(1.0 - lb) - S_half(1.0 - la));
        }
        a = end;
    }
    return sum;
}

/* parameters t in [0, 1] where the segment P + t D meets the unit circle or the
 * full ellipse; the boundary of V is made of parts of these two curves, so its
 * crossings are among them (the others only split the segment further) */
static int vis_crossings(const double P[2], const double D[2], double wz, double t[4])
{
    int n = 0;
    /* unit circle */
    double a = D[0] * D[0] + D[1] * D[1], b = 2.0 * (P[0] * D[0] + P[1] * D[1]), c = P[0] * P[0] + P[1] * P[1] - 1.0;
    for (int pass = 0; pass < 2; pass++) {
        double disc = b * b - 4.0 * a * c;
        if (a > 0.0 && disc >= 0.0) {
            double sq = sqrt(disc);
            double r[2] = {(-b - sq) / (2.0 * a), (-b + sq) / (2.0 * a)};
            for (int k = 0; k < 2; k++)
                if (r[k] >= 0.0 && r[k] <= 1.0) t[n++] = r[k];
        }
        /* then the ellipse x^2 + wz^2 y^2 = wz^2 */
        a = D[0] * D[0] + wz * wz * D[1] * D[1];
        b = 2.0 * (P[0] * D[0] + wz * wz * P[1] * D[1]);
        c = P[0] * P[0] + wz * wz * P[1] * P[1] - wz * wz;
    }
    /* and the line x = 0, which the ellipse becomes as wz -> 0 (where its
     * discriminant is a difference of equal products and can round below 0) */
    if (D[0] != 0.0) {
        double r = -P[0] / D[0];
        if (r >= 0.0 && r <= 1.0) t[n++] = r;
    }
    return n;
}

/* integral of (w_x m_x / m~_z + w_z) over (triangle v) intersected with V, the
 * triangle given in the canonical frame */
static double tri_projected(const double v0[3][2], double wx, double wz)
{
    double v[3][2];
    memcpy(v, v0, sizeof v);
    double area2 = sarea2(v[0], v[1], v[2]);
    if (area2 < 0.0) { /* counter-clockwise */
        double tmp[2];
        memcpy(tmp, v[1], sizeof tmp); memcpy(v[1], v[2], sizeof tmp); memcpy(v[2], tmp, sizeof tmp);
    }
    /* per edge: the part inside V (V convex: one interval) */
    double ent[3][2], ext[3][2];
    int has[3];
    int any = 0;
    for (int e = 0; e < 3; e++) {
        const double* P = v[e];
        const double* Q = v[(e + 1) % 3];
        double D[2] = {Q[0] - P[0], Q[1] - P[1]};
        double ts[9];
        int nt = 0;
        ts[nt++] = 0.0;
        ts[nt++] = 1.0;
        nt += vis_crossings(P, D, wz, ts + nt);
        /* sort */
        for (int i = 1; i < nt; i++)
            for (int j = i; j > 0 && ts[j] < ts[j - 1]; j--) { double x = ts[j]; ts[j] = ts[j - 1]; ts[j - 1] = x; }
        double t0 = 2.0, t1 = -1.0;
        for (int i = 0; i + 1 < nt; i++) {
            double tm = 0.5 * (ts[i] + ts[i + 1]);
            if (ts[i + 1] - ts[i] <= 0.0) continue;
            if (in_vis(P[0] + tm * D[0], P[1] + tm * D[1], wz)) {
                if (ts[i] < t0) t0 = ts[i];
                if (ts[i + 1] > t1) t1 = ts[i + 1];
            }
        }
        has[e] = t1 > t0;
        if (has[e]) {
            /* (the vertices themselves at t = 0 and 1, so that consecutive edges meet
             * exactly at a vertex inside V) */
            if (t0 == 0.0) { ent[e][0] = P[0]; ent[e][1] = P[1]; }
            else { ent[e][0] = P[0] + t0 * D[0]; ent[e][1] = P[1] + t0 * D[1]; }
            if (t1 == 1.0) { ext[e][0] = Q[0]; ext[e][1] = Q[1]; }
            else { ext[e][0] = P[0] + t1 * D[0]; ext[e][1] = P[1] + t1 * D[1]; }
            any = 1;
        }
    }
    if (!any) {
        /* no edge inside V: V lies inside the triangle, or they are disjoint
         * (the origin, a point of V, decides) */
        double o[2] = {0.0, 0.0};
        double a0 = sarea2(o, v[1], v[2]), a1 = sarea2(v[0], o, v[2]), a2 = sarea2(v[0], v[1], o);
        if (a0 >= 0.0 && a1 >= 0.0 && a2 >= 0.0) return arc_term(0.0, 4.0, wz);
        return 0.0;
    }
    double sum = 0.0;
    for (int e = 0; e < 3; e++) {
        if (!has[e]) continue;
        sum += seg_term(ent[e], ext[e], wx, wz);
        /* from this edge's exit along the boundary of V to the next edge's entry,
         * unless the exit is the next edge's start (a vertex inside V) */
        int f = (e + 1) % 3;
        while (!has[f]) f = (f + 1) % 3;
        if (ext[e][0] == ent[f][0] && ext[e][1] == ent[f][1]) continue;
        double a = vis_pos(ext[e][0], ext[e][1]), b = vis_pos(ent[f][0], ent[f][1]);
        if (b < a) b += 4.0;
        sum += arc_term(a, b, wz);
    }
    return sum;
}

/* exposed for the pins: the integral for one triangle (3 x 2 normals) and a
 * direction w (x, y, z), w_z >= 0 */
double or_tri_projected(const double* tri, const double* w)
{
    double len = sqrt(w[0] * w[0] + w[1] * w[1]);
    double c = len > 0.0 ? w[0] / len : 1.0, sn = len > 0.0 ? w[1] / len : 0.0;
    double v[3][2];
    for (int k = 0; k < 3; k++) {
        v[k][0] = c * tri[2 * k] + sn * tri[2 * k + 1];
        v[k][1] = -sn * tri[2 * k] + c * tri[2 * k + 1];
    }
    return tri_projected((const double(*)[2])v, len, w[2]);
}

/* the footprint kernel at uv point (ux, uy) of the cell (i, j) (torus indices),
 * summed over the cell's included periodic images */
static double kernel_at(const map_t* m, const query_t* q, double ux, double uy, long i, long j)
{
    int amb = 0;
    if (q->kernel == 2)
        return box_count(ux, i, 1, q->cxlo, q->cxhi, m->n, q->x, q->rx, &amb) *
               box_count(uy, j, 1, q->cylo, q->cyhi, m->n, q->y, q->ry, &amb) / (4.0 * q->rx * q->ry);
    if (q->kernel == 1) return disk_count(ux, uy, i, j, 1, q, m->n, &amb) / (OR_PI * q->rx * q->ry);
    return gauss_sum(ux, i, 1, q->cxlo, q->cxhi, m->n, q->x, q->sx) *
           gauss_sum(uy, j, 1, q->cylo, q->cyhi, m->n, q->y, q->sy) / (2.0 * OR_PI * q->sx * q->sy);
}

/*
 * Projected area P(w) (see above) for nq queries: x, y, sx, sy as for the
 * evaluation; the last two floats are w_x, w_y of the unit direction w, with
 * w_z = sqrt(1 - w_x^2 - w_y^2) >= 0.  Brute force over every triangle of every
 * included cell (the paper's own implementation is brute force too).  P[k] is NaN
 * for an invalid query or |(w_x, w_y)| > 1.
 */
int or_projected_area(int n, const float* nrm, float eps, const float* queries, int64_t nq, float s2r,
                      int kernel, double* Pout)
{
    if (kernel < 0 || kernel > 2) return 3;
    map_t m;
    m.n = n;
    m.L = ilog2_exact(n);
    if (m.L < 1) return 1;
    m.nrm = nrm;
    m.eps = (double)eps;
    m.clu_n = NULL;
    m.clu_e = NULL;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < nq; k++) {
        query_t q;
        const float* qr = queries + 6 * k;
        double wx = qr[4], wy = qr[5];
        double wl2 = wx * wx + wy * wy;
        if (setup_query(&m, qr, 0.0f, s2r, 0.0, kernel, &q) || !(wl2 <= 1.0)) {
            Pout[k] = NAN;
            continue;
        }
        double wz = sqrt(1.0 - wl2), wl = sqrt(wl2);
        /* rotation about z taking w to (wl, 0, wz) */
        double c = wl > 0.0 ? wx / wl : 1.0, sn = wl > 0.0 ? wy / wl : 0.0;
        long* xi = (long*)malloc(sizeof(long) * (size_t)n);
        long* yj = (long*)malloc(sizeof(long) * (size_t)n);
        long nx = axis_cells(q.cxlo, q.cxhi, n, xi);
        long ny = axis_cells(q.cylo, q.cyhi, n, yj);
        double P = 0.0;
        for (long b = 0; b < ny; b++)
            for (long a = 0; a < nx; a++) {
                long i = xi[a], j = yj[b];
                double nv4[4][2];
                texel(m.nrm, n, i, j, nv4[0]);
                texel(m.nrm, n, i + 1, j, nv4[1]);
                texel(m.nrm, n, i, j + 1, nv4[2]);
                texel(m.nrm, n, i + 1, j + 1, nv4[3]);
                double centre[2] = {0.5 * (nv4[1][0] + nv4[2][0]), 0.5 * (nv4[1][1] + nv4[2][1])};
                for (int half = 0; half < 2; half++) {
                    double nv[3][2];
                    if (half == 0) {
                        memcpy(nv[0], nv4[0], sizeof nv[0]); memcpy(nv[1], nv4[1], sizeof nv[0]);
                        memcpy(nv[2], nv4[2], sizeof nv[0]);
                    } else {
                        memcpy(nv[0], nv4[3], sizeof nv[0]); memcpy(nv[1], nv4[2], sizeof nv[0]);
                        memcpy(nv[2], nv4[1], sizeof nv[0]);
                    }
                    double J = jac(nv[0], nv[1], nv[2]);
                    if (J < m.eps) {
                        eqtri(centre, eq_rho(0.5 * m.eps), nv);
                        J = m.eps;
                    }
                    /* the kernel, constant over the triangle: its value at the uv centroid */
                    double third = half == 0 ? 1.0 / 3.0 : 2.0 / 3.0;
                    double kv = kernel_at(&m, &q, (double)i + third, (double)j + third, i, j);
                    if (kv == 0.0) continue;
                    double rv[3][2];
                    for (int v = 0; v < 3; v++) {
                        rv[v][0] = c * nv[v][0] + sn * nv[v][1];
                        rv[v][1] = -sn * nv[v][0] + c * nv[v][1];
                    }
                    P += kv / J * tri_projected((const double(*)[2])rv, wl, wz);
                }
            }
        free(xi);
        free(yj);
        Pout[k] = P;
    }
    return 0;
}

/* number of OpenMP threads the evaluation uses (for reporting CPU baselines) */
#ifdef _OPENMP
#include <omp.h>
#endif
int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* threads of the oracle's parallel loops from now on (n >= 1) */
void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
