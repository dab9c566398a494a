// Projected area of the P-NDF on gfx950 (section "Shadow-masking", Eq. lambda,
// Eq. area-integral, Eq. line-integral and the supplement's derivations).
//
//   P(w) = integral of D(m) max(m~ . w, 0) over the solid angle of m~,
//
// with the footprint kernel constant over each triangle (its value at the uv
// centroid).  Per triangle, after rotating about z so that w = (w_l, 0, w_z),
// w_l >= 0, the contribution is k / J times the integral of (w_l m_x / m~_z + w_z)
// over the part of the normal triangle inside the visible region V = {|m| <= 1,
// m~ . w >= 0}: the unit disk cut on the left by the semi-ellipse
// m_x = -w_z sqrt(1 - m_y^2).  V is convex.  By Stokes' theorem the area integral
// is the counter-clockwise boundary integral of F dm_y, F = w_z m_x - w_l m~_z,
// over the triangle's edges clipped to V and the pieces of V's boundary between
// them, all in closed form with A(y) = (asin y + y sqrt(1 - y^2)) / 2:
//   segment P -> Q:  w_z (Q_y - P_y)(P_x + Q_x) / 2 - w_l d_y rho^2 [A(p / rho)],
//                    d the unit direction, p the abscissa along d, rho^2 = 1 - s^2
//                    with s the line's distance to the origin;
//   circle piece:    w_z [A(y)] (m~_z = 0, m_x = sqrt(1 - y^2), y increasing);
//   ellipse piece:   -[A(y)] (F = -sqrt(1 - y^2) there, y decreasing).
// A triangle with its three vertices in V lies in V (convexity): three segments.
//
// Brute force like the paper's implementation: one wavefront per query, lanes over
// the included cells (two triangles each), FP64 throughout; the lanes' partial
// sums are reduced in the wave.  V lies right of the line m_x = -w_z (the
// ellipse's leftmost point), so a triangle left of it adds nothing; a triangle
// with its three vertices in V takes three segment terms at once (a cell whose two
// triangles both lie in V five: the shared diagonal once); only the others need
// clipping, and they wait in a per-wave LDS queue until 64 of them fill a round with
// one per lane (a lane's clipping would otherwise stall its wave).
#include <algorithm>

#include "pndf_internal.h"

namespace pndf {
namespace {

__device__ __forceinline__ double arc_prim(double y)
{
    y = fmin(1.0, fmax(-1.0, y));
    return 0.5 * (asin(y) + y * sqrt(fmax(0.0, 1.0 - y * y)));
}

__device__ __forceinline__ bool visible(double x, double y, double wz)
{
    return x * x + y * y <= 1.0 && (x >= 0.0 || x * x + wz * wz * y * y <= wz * wz);
}

// 1 / sqrt(x), x > 0, in FP64: the hardware estimate refined by two Newton steps
// y <- y (3/2 - x y^2 / 2) (each step squares the relative error), so the segment
// terms need no FP64 square root or division (unit direction, 1/rho, sqrt(1 - y^2)).
__device__ __forceinline__ double rsqrt_f64(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = y * fma(-h * y, y, 1.5);
    y = y * fma(-h * y, y, 1.5);
    return y;
}

// sqrt(z) for 0 <= z <= 1 as z / sqrt(z) (exactly 0 at 0)
__device__ __forceinline__ double sqrt_unit(double z)
{
    return z > 0.0 ? z * rsqrt_f64(z) : 0.0;
}

// A(b) - A(a) with one arcsine: asin b - asin a = asin(b sqrt(1 - a^2) - a sqrt(1 - b^2))
// while the difference of the angles is within [-pi/2, pi/2], i.e. while
// sqrt(1 - a^2) sqrt(1 - b^2) + a b >= 0; else two
__device__ __forceinline__ double arc_prim_diff(double a, double b)
{
    a = fmin(1.0, fmax(-1.0, a));
    b = fmin(1.0, fmax(-1.0, b));
    const double ca = sqrt_unit(1.0 - a * a), cb = sqrt_unit(1.0 - b * b);
    const double d = ca * cb + a * b >= 0.0 ? asin(fmin(1.0, fmax(-1.0, b * ca - a * cb))) : asin(b) - asin(a);
    return 0.5 * (d + b * cb - a * ca);
}

// F dm_y along the segment P -> Q
__device__ inline double segment_int(double px, double py, double qx, double qy, double wl, double wz)
{
    double dx = qx - px, dy = qy - py;
    const double l2 = dx * dx + dy * dy;
    if (l2 == 0.0) return 0.0;
    const double lin = 0.5 * wz * dy * (px + qx);
    const double il = rsqrt_f64(l2);
    dx *= il;
    dy *= il;
    const double s = dy * px - dx * py;
    const double rho2 = 1.0 - s * s;
    if (rho2 <= 0.0) return lin;
    const double ir = rsqrt_f64(rho2);
    return lin - wl * dy * rho2 * arc_prim_diff((dx * px + dy * py) * ir, (dx * qx + dy * qy) * ir);
}

// place of a point of V's boundary on its counter-clockwise loop from (0, -1):
// right semicircle -> [0, 2], left semi-ellipse -> [2, 4].  On the semicircle
// means x >= 0 and on the unit circle (at w_z = 0 the semi-ellipse degenerates to
// the segment x = 0 inside the disk).
__device__ __forceinline__ double loop_pos(double x, double y)
{
    y = fmin(1.0, fmax(-1.0, y));
    return (x >= 0.0 && x * x + y * y >= 1.0 - 1e-9) ? 1.0 + y : 3.0 - y;
}

// F dm_y along V's boundary from loop place a to b (a <= b < a + 4)
__device__ inline double boundary_int(double a, double b, double wz)
{
    double sum = 0.0;
    for (int guard = 0; guard < 5 && a < b; ++guard) {
        const double half = floor(a * 0.5);
        const double stop = fmin(b, 2.0 * half + 2.0);
        const double ya = a - 2.0 * half, yb = stop - 2.0 * half;  // in [0, 2]
        if (((int)half & 1) == 0)
            sum += wz * (arc_prim(yb - 1.0) - arc_prim(ya - 1.0));   // circle, y = place - 1
        else
            sum += arc_prim(1.0 - ya) - arc_prim(1.0 - yb);         // ellipse, y = 1 - place
        a = stop;
    }
    return sum;
}

__device__ __forceinline__ void cswap(double& a, double& b)
{
    const double lo = fmin(a, b), hi = fmax(a, b);
    a = lo;
    b = hi;
}

// parameter interval [t0, t1] of the segment P + t D (t in [0, 1]) inside V;
// false if empty.  The candidates: the ends, every meeting with the unit circle or
// the whole ellipse x^2 + wz^2 y^2 = wz^2 (V's boundary crossings are among them,
// the others only split the segment), and the line x = 0, the ellipse's limit as
// wz -> 0 (its discriminant is then a difference of equal products and may round
// below 0).  Unused slots repeat t = 1.  Sorted by a fixed network (registers
// only); V convex: the visible pieces between consecutive candidates form one
// interval.
__device__ inline bool clip_edge(double px, double py, double dx, double dy, double wz, double* t0, double* t1)
{
    double ts[7] = {0.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0};
#pragma unroll
    for (int curve = 0; curve < 2; ++curve) {
        const double ey = curve == 0 ? 1.0 : wz * wz, rhs = curve == 0 ? 1.0 : wz * wz;
        const double qa = dx * dx + ey * dy * dy;
        const double qb = 2.0 * (px * dx + ey * py * dy);
        const double qc = px * px + ey * py * py - rhs;
        const double disc = qb * qb - 4.0 * qa * qc;
        if (qa > 0.0 && disc >= 0.0) {
            const double sq = sqrt(disc);
            const double ra = (-qb - sq) / (2.0 * qa), rb = (-qb + sq) / (2.0 * qa);
            ts[2 + 2 * curve] = (ra > 0.0 && ra < 1.0) ? ra : 1.0;
            ts[3 + 2 * curve] = (rb > 0.0 && rb < 1.0) ? rb : 1.0;
        }
    }
    if (dx != 0.0) {
        const double t = -px / dx;
        ts[6] = (t > 0.0 && t < 1.0) ? t : 1.0;
    }
    // sorting network for 7 values
    cswap(ts[0], ts[6]); cswap(ts[2], ts[3]); cswap(ts[4], ts[5]);
    cswap(ts[0], ts[2]); cswap(ts[1], ts[4]); cswap(ts[3], ts[6]);
    cswap(ts[0], ts[1]); cswap(ts[2], ts[5]); cswap(ts[3], ts[4]);
    cswap(ts[1], ts[2]); cswap(ts[4], ts[6]);
    cswap(ts[2], ts[3]); cswap(ts[4], ts[5]);
    cswap(ts[1], ts[2]); cswap(ts[3], ts[4]); cswap(ts[5], ts[6]);
    double lo = 2.0, hi = -1.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        if (!(ts[i + 1] > ts[i])) continue;
        const double tm = 0.5 * (ts[i] + ts[i + 1]);
        if (visible(px + tm * dx, py + tm * dy, wz)) {
            lo = fmin(lo, ts[i]);
            hi = fmax(hi, ts[i + 1]);
        }
    }
    *t0 = lo;
    *t1 = hi;
    return hi > lo;
}

// counter-clockwise vertex order
__device__ __forceinline__ void orient_ccw(double v[6])
{
    const double a2 = (v[2] - v[0]) * (v[5] - v[1]) - (v[3] - v[1]) * (v[4] - v[0]);
    if (a2 < 0.0) {
        double t = v[2]; v[2] = v[4]; v[4] = t;
        t = v[3]; v[3] = v[5]; v[5] = t;
    }
}

// integral of (w_l m_x / m~_z + w_z) over (triangle v, canonical frame,
// counter-clockwise) within V, by clipping
__device__ inline double triangle_int_clipped(const double v[6], double wl, double wz)
{
    double ex[3], ey[3], xx[3], xy[3];  // entry and exit point of each edge
    bool in[3];
    bool any = false;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const int f = (e + 1) % 3;
        const double px = v[2 * e], py = v[2 * e + 1], qx = v[2 * f], qy = v[2 * f + 1];
        double t0, t1;
        in[e] = clip_edge(px, py, qx - px, qy - py, wz, &t0, &t1);
        if (in[e]) {
            ex[e] = t0 == 0.0 ? px : px + t0 * (qx - px);
            ey[e] = t0 == 0.0 ? py : py + t0 * (qy - py);
            xx[e] = t1 == 1.0 ? qx : px + t1 * (qx - px);
            xy[e] = t1 == 1.0 ? qy : py + t1 * (qy - py);
            any = true;
        }
    }
    if (!any) {
        // V inside the triangle (it holds the origin, a point of V) or disjoint
        const bool o0 = v[2] * v[5] - v[3] * v[4] >= 0.0;               // (0, v1, v2)
        const bool o1 = v[4] * v[1] - v[5] * v[0] >= 0.0;               // (0, v2, v0)
        const bool o2 = v[0] * v[3] - v[1] * v[2] >= 0.0;               // (0, v0, v1)
        return (o0 && o1 && o2) ? boundary_int(0.0, 4.0, wz) : 0.0;
    }
    double sum = 0.0;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        if (!in[e]) continue;
        sum += segment_int(ex[e], ey[e], xx[e], xy[e], wl, wz);
        int f = (e + 1) % 3;
        if (!in[f]) f = (f + 1) % 3;
        if (!in[f]) f = e;
        if (xx[e] == ex[f] && xy[e] == ey[f]) continue;  // meets the next edge at a vertex
        const double a = loop_pos(xx[e], xy[e]);
        double b = loop_pos(ex[f], ey[f]);
        if (b < a) b += 4.0;
        sum += boundary_int(a, b, wz);
    }
    return sum;
}

// A triangle of cell (i, j) and its weight k / J: normals in the canonical frame.
__device__ __forceinline__ void cell_triangle(const HierDev& H, int i, int j, int half, double c, double sn,
                                              double r[6])
{
    const int wdt = H.n + 1;
    const float2* p = H.nrm + (int64_t)j * wdt + i;
    const float2 n1 = p[1], n2 = p[wdt];
    const float2 nc = half ? p[wdt + 1] : p[0];
    double v[6];
    if ((H.deg[(int64_t)j * H.n + i] >> half) & 1u) {
        eqtri_f64(0.5 * ((double)n1.x + (double)n2.x), 0.5 * ((double)n1.y + (double)n2.y), (double)H.rho, v);
    } else if (half == 0) {
        v[0] = nc.x; v[1] = nc.y; v[2] = n1.x; v[3] = n1.y; v[4] = n2.x; v[5] = n2.y;
    } else {
        v[0] = nc.x; v[1] = nc.y; v[2] = n2.x; v[3] = n2.y; v[4] = n1.x; v[5] = n1.y;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        r[2 * k] = c * v[2 * k] + sn * v[2 * k + 1];
        r[2 * k + 1] = -sn * v[2 * k] + c * v[2 * k + 1];
    }
    orient_ccw(r);
}

constexpr int kClipCap = 256;  // queued triangles per wave (a step adds at most 128)

template <int KER>
// One wavefront per workgroup: queries differ in cost by up to 64x (the support
// grows with sigma^2), and a workgroup of four held its slot until its slowest query
// ended (7.4 resident waves per CU of the 16 the registers allow; one per workgroup:
// -18 %).
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_projected_area(HierDev H, ProjArgs a)
{
    __shared__ uint32_t clip_cell[kClipCap];
    __shared__ double clip_w[kClipCap];
    if ((int64_t)blockIdx.x >= a.nq) return;
    const int64_t qi = a.order ? (int64_t)a.order[blockIdx.x] : (int64_t)blockIdx.x;
    const int lane = threadIdx.x & 63;
    const pndf_query qr = a.q[qi];
    const QuerySetup q = uniform_query(setup_query(qr, a.s2r, 0.f, H.L, H.eps, KER));
    const double wx = qr.hx, wy = qr.hy;
    const double wl2 = wx * wx + wy * wy;
    if (!q.valid || !(wl2 <= 1.0)) {
        if (lane == 0) {
            a.P[qi] = __int_as_float(0x7fc00000);
            if (a.lambda) a.lambda[qi] = __int_as_float(0x7fc00000);
        }
        return;
    }
    const double wz = sqrt(1.0 - wl2), wl = sqrt(wl2);
    const double c = wl > 0.0 ? wx / wl : 1.0, sn = wl > 0.0 ? wy / wl : 0.0;
    const int n = H.n, msk = n - 1;
    const int spanx = q.cxhi - q.cxlo + 1, spany = q.cyhi - q.cylo + 1;
    const int nx = spanx >= n ? n : spanx, ny = spany >= n ? n : spany;
    const int total = nx * ny;
    double acc = 0.0;
    int qn = 0;  // queued triangles (wave-uniform)
    for (int base = 0; base < total || qn > 0; base += 64) {
        uint32_t clip = 0;          // bit h: this lane's triangle h needs clipping
        double kw[2] = {0.0, 0.0};
        uint32_t cell = 0;
        const int idx = base + lane;
        if (idx < total) {
            const int ca = idx % nx, cb = idx / nx;
            const int i = spanx >= n ? ca : ((q.cxlo + ca) & msk);
            const int j = spany >= n ? cb : ((q.cylo + cb) & msk);
            cell = (uint32_t)i | ((uint32_t)j << 13);
            const float2 dd = H.det[(int64_t)j * n + i];
            // kernel at the uv centroid over the included images, divided by J
            double kh[2];
            kh[0] = hit_term<KER>(q, i, j, 0, 0, 1.0 / 3.0, 1.0 / 3.0, dd.x, H.logn);
            kh[1] = hit_term<KER>(q, i, j, 0, 1, 1.0 / 3.0, 1.0 / 3.0, dd.y, H.logn);
            if ((H.deg[(int64_t)j * n + i] & 3u) == 0u) {
                // both halves regular: lower (n0, n1, n2) and upper (n3, n2, n1) share the
                // diagonal n1 -> n2, which the upper runs backwards.  The corners are rotated
                // once; a triangle's CCW boundary integral is its orientation sign times
                // the integral in vertex order, so with both triangles inside V the
                // diagonal's term is computed once with weight s_l k_l - s_u k_u.
                const int wdt = n + 1;
                const float2* p = H.nrm + (int64_t)j * wdt + i;
                const float2 nn[4] = {p[0], p[1], p[wdt], p[wdt + 1]};
                double x[4], y[4];
                bool vis[4], left[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    x[k] = c * (double)nn[k].x + sn * (double)nn[k].y;
                    y[k] = -sn * (double)nn[k].x + c * (double)nn[k].y;
                    vis[k] = visible(x[k], y[k], wz);
                    left[k] = x[k] < -wz;
                }
                const double sl = (x[1] - x[0]) * (y[2] - y[0]) - (y[1] - y[0]) * (x[2] - x[0]) < 0.0 ? -1.0 : 1.0;
                const double su = (x[2] - x[3]) * (y[1] - y[3]) - (y[2] - y[3]) * (x[1] - x[3]) < 0.0 ? -1.0 : 1.0;
                const bool lo_live = kh[0] != 0.0 && !(left[0] && left[1] && left[2]);
                const bool up_live = kh[1] != 0.0 && !(left[3] && left[2] && left[1]);
                const bool lo_full = lo_live && vis[0] && vis[1] && vis[2];
                const bool up_full = up_live && vis[3] && vis[2] && vis[1];
                double wd = 0.0;
                if (lo_full) {
                    acc += kh[0] * sl * (segment_int(x[0], y[0], x[1], y[1], wl, wz) +
                                         segment_int(x[2], y[2], x[0], y[0], wl, wz));
                    wd += kh[0] * sl;
                }
                if (up_full) {
                    acc += kh[1] * su * (segment_int(x[3], y[3], x[2], y[2], wl, wz) +
                                         segment_int(x[1], y[1], x[3], y[3], wl, wz));
                    wd -= kh[1] * su;
                }
                if (wd != 0.0) acc += wd * segment_int(x[1], y[1], x[2], y[2], wl, wz);
                if (lo_live && !lo_full) {
                    clip |= 1u;
                    kw[0] = kh[0];
                }
                if (up_live && !up_full) {
                    clip |= 2u;
                    kw[1] = kh[1];
                }
            } else {
                // a clamped half (its replacement triangle): each triangle on its own
#pragma unroll
                for (int half = 0; half < 2; ++half) {
                    const double kj = kh[half];
                    if (kj == 0.0) continue;
                    double r[6];
                    cell_triangle(H, i, j, half, c, sn, r);
                    if (r[0] < -wz && r[2] < -wz && r[4] < -wz) continue;  // left of V
                    if (visible(r[0], r[1], wz) && visible(r[2], r[3], wz) && visible(r[4], r[5], wz)) {
                        acc += kj * (segment_int(r[0], r[1], r[2], r[3], wl, wz) +
                                     segment_int(r[2], r[3], r[4], r[5], wl, wz) +
                                     segment_int(r[4], r[5], r[0], r[1], wl, wz));
                    } else {
                        clip |= 1u << half;
                        kw[half] = kj;
                    }
                }
            }
        }
        // queue the triangles that need clipping (lane order)
        int tot;
        const int pos = wave_prefix_small(__popc(clip), &tot);
        int at = qn + pos;
#pragma unroll
        for (int half = 0; half < 2; ++half)
            if (clip & (1u << half)) {
                clip_cell[at] = cell | ((uint32_t)half << 26);
                clip_w[at] = kw[half];
                ++at;
            }
        qn += tot;
        wave_sync();
        // full rounds, and at the end whatever is left
        while (qn >= 64 || (qn > 0 && base + 64 >= total)) {
            const int cnt = min(qn, 64);
            qn -= cnt;
            if (lane < cnt) {
                const uint32_t e = clip_cell[qn + lane];
                double r[6];
                cell_triangle(H, (int)(e & 0x1fffu), (int)((e >> 13) & 0x1fffu), (int)(e >> 26), c, sn, r);
                acc += clip_w[qn + lane] * triangle_int_clipped(r, wl, wz);
            }
            wave_sync();
        }
    }
    const double P = wave_sum_f64(acc);
    if (lane == 0) {
        a.P[qi] = (float)P;
        if (a.lambda) a.lambda[qi] = (float)(P / wz - 1.0);
    }
}

// ---- heaviest-first order.  A query's cost grows with its number of included
// cells; the launch takes queries in decreasing cost class, so the longest ones
// start first and the batch does not end on a few long queries with the GPU
// otherwise idle.  Counting sort on 64 classes of log2 of the cell count (half
// octaves: up to 2^32 cells), in LDS per workgroup like the evaluation's spatial
// order.
constexpr int kCostBins = 64;

__device__ __forceinline__ uint32_t cost_class(const pndf_query& qr, float s2r, int n, int kernel, float eps, int L)
{
    const QuerySetup q = setup_query(qr, s2r, 0.f, L, eps, kernel);
    if (!q.valid) return 0u;
    const double cx = fmin((double)(q.cxhi - q.cxlo + 1), (double)n), cy = fmin((double)(q.cyhi - q.cylo + 1), (double)n);
    const int c = (int)floor(2.0 * log2(cx * cy));
    return (uint32_t)min(max(c, 0), kCostBins - 1);
}

__global__ void k_cost_hist(const pndf_query* __restrict__ q, int64_t nq, float s2r, int kernel, HierDev H,
                            uint32_t* __restrict__ key, uint32_t* __restrict__ hist)
{
    __shared__ uint32_t loc[kCostBins];
    if (threadIdx.x < kCostBins) loc[threadIdx.x] = 0u;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nq; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t k = (kCostBins - 1) - cost_class(q[i], s2r, H.n, kernel, H.eps, H.L);  // heaviest first
        key[i] = k;
        atomicAdd(&loc[k], 1u);
    }
    __syncthreads();
    if (threadIdx.x < kCostBins && loc[threadIdx.x]) atomicAdd(&hist[threadIdx.x], loc[threadIdx.x]);
}

// exclusive scan of the 64 counters, one wavefront
__global__ void k_cost_scan(uint32_t* hist)
{
    const int t = threadIdx.x;
    uint32_t v = hist[t], run = v;
    for (int o = 1; o < kCostBins; o <<= 1) {
        const uint32_t u = __shfl_up(run, o);
        if (t >= o) run += u;
    }
    hist[t] = run - v;
}

__global__ void k_cost_scatter(const uint32_t* __restrict__ key, int64_t nq, uint32_t* __restrict__ cursor,
                               uint32_t* __restrict__ order)
{
    __shared__ uint32_t loc[kCostBins];
    if (threadIdx.x < kCostBins) loc[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = i0; i < nq; i += stride) atomicAdd(&loc[key[i]], 1u);
    __syncthreads();
    if (threadIdx.x < kCostBins && loc[threadIdx.x]) loc[threadIdx.x] = atomicAdd(&cursor[threadIdx.x], loc[threadIdx.x]);
    __syncthreads();
    for (int64_t i = i0; i < nq; i += stride) order[atomicAdd(&loc[key[i]], 1u)] = (uint32_t)i;
}

__global__ void k_cost_zero(uint32_t* hist)
{
    if (threadIdx.x < kCostBins) hist[threadIdx.x] = 0u;
}

}  // namespace

hipError_t launch_projected_area(const HierDev& H, const ProjArgs& a, hipStream_t s)
{
    // one wavefront-sized workgroup per query, in launches of at most launch_chunk()
    // workgroups (2^24 x 64 = 2^30 work-items), each in heaviest-first order
    // (workspace: order, keys and counters of one launch, stream-ordered)
    const int64_t chunk = launch_chunk();
    const int64_t most = std::min(chunk, a.nq);
    uint32_t* buf = nullptr;
    if (most > 0) {
        const hipError_t e = hipMallocAsync((void**)&buf, sizeof(uint32_t) * (2 * (size_t)most + kCostBins), s);
        if (e != hipSuccess) return e;
    }
    for (int64_t off = 0; off < a.nq; off += chunk) {
        ProjArgs c = a;
        c.q = a.q + off;
        c.P = a.P + off;
        if (a.lambda) c.lambda = a.lambda + off;
        c.nq = std::min(chunk, a.nq - off);
        uint32_t* key = buf + most;
        uint32_t* hist = key + most;
        const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(256, (c.nq + 4095) / 4096));
        hipLaunchKernelGGL(k_cost_zero, dim3(1), dim3(64), 0, s, hist);
        hipLaunchKernelGGL(k_cost_hist, dim3(g), dim3(256), 0, s, c.q, c.nq, c.s2r, c.kernel, H, key, hist);
        hipLaunchKernelGGL(k_cost_scan, dim3(1), dim3(kCostBins), 0, s, hist);
        hipLaunchKernelGGL(k_cost_scatter, dim3(g), dim3(256), 0, s, key, c.nq, hist, buf);
        c.order = buf;
        const dim3 grid((unsigned)c.nq), block(64);
        if (a.kernel == PNDF_KERNEL_DISK)
            hipLaunchKernelGGL(k_projected_area<PNDF_KERNEL_DISK>, grid, block, 0, s, H, c);
        else if (a.kernel == PNDF_KERNEL_BOX)
            hipLaunchKernelGGL(k_projected_area<PNDF_KERNEL_BOX>, grid, block, 0, s, H, c);
        else
            hipLaunchKernelGGL(k_projected_area<PNDF_KERNEL_GAUSSIAN>, grid, block, 0, s, H, c);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            (void)hipFreeAsync(buf, s);
            return e;
        }
    }
    return buf ? hipFreeAsync(buf, s) : hipSuccess;
}

}  // namespace pndf
