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
// sums are reduced in the wave.
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

// F dm_y along the segment P -> Q
__device__ inline double segment_int(double px, double py, double qx, double qy, double wl, double wz)
{
    double dx = qx - px, dy = qy - py;
    const double len = sqrt(dx * dx + dy * dy);
    if (len == 0.0) return 0.0;
    const double lin = 0.5 * wz * dy * (px + qx);
    dx /= len;
    dy /= len;
    const double s = dy * px - dx * py;
    const double rho2 = 1.0 - s * s;
    if (rho2 <= 0.0) return lin;
    const double rho = sqrt(rho2);
    return lin - wl * dy * rho2 * (arc_prim((dx * qx + dy * qy) / rho) - arc_prim((dx * px + dy * py) / rho));
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

// parameter interval [t0, t1] of the segment P + t D (t in [0, 1]) inside V;
// false if empty
__device__ inline bool clip_edge(double px, double py, double dx, double dy, double wz, double* t0, double* t1)
{
    double ts[7];
    int nt = 0;
    ts[nt++] = 0.0;
    ts[nt++] = 1.0;
    // every meeting with the unit circle or the whole ellipse x^2 + wz^2 y^2 = wz^2:
    // V's boundary crossings are among them, the others only split the segment
#pragma unroll
    for (int curve = 0; curve < 2; ++curve) {
        const double ey = curve == 0 ? 1.0 : wz * wz, rhs = curve == 0 ? 1.0 : wz * wz;
        const double qa = dx * dx + ey * dy * dy;
        const double qb = 2.0 * (px * dx + ey * py * dy);
        const double qc = px * px + ey * py * py - rhs;
        const double disc = qb * qb - 4.0 * qa * qc;
        if (qa > 0.0 && disc >= 0.0) {
            const double sq = sqrt(disc);
#pragma unroll
            for (int sgn = -1; sgn <= 1; sgn += 2) {
                const double t = (-qb + sgn * sq) / (2.0 * qa);
                if (t > 0.0 && t < 1.0) ts[nt++] = t;
            }
        }
    }
    // the line x = 0, the ellipse's limit as wz -> 0 (its discriminant is then a
    // difference of equal products and may round below 0)
    if (dx != 0.0) {
        const double t = -px / dx;
        if (t > 0.0 && t < 1.0) ts[nt++] = t;
    }
    // sort (at most 7 values)
    for (int i = 1; i < nt; ++i)
        for (int j = i; j > 0 && ts[j] < ts[j - 1]; --j) {
            const double tmp = ts[j];
            ts[j] = ts[j - 1];
            ts[j - 1] = tmp;
        }
    double lo = 2.0, hi = -1.0;
    for (int i = 0; i + 1 < nt; ++i) {
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

// integral of (w_l m_x / m~_z + w_z) over (triangle v, canonical frame) within V
__device__ inline double triangle_int(double v[6], double wl, double wz)
{
    // counter-clockwise
    const double a2 = (v[2] - v[0]) * (v[5] - v[1]) - (v[3] - v[1]) * (v[4] - v[0]);
    if (a2 < 0.0) {
        double t = v[2]; v[2] = v[4]; v[4] = t;
        t = v[3]; v[3] = v[5]; v[5] = t;
    }
    if (visible(v[0], v[1], wz) && visible(v[2], v[3], wz) && visible(v[4], v[5], wz))
        return segment_int(v[0], v[1], v[2], v[3], wl, wz) + segment_int(v[2], v[3], v[4], v[5], wl, wz) +
               segment_int(v[4], v[5], v[0], v[1], wl, wz);
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

__device__ __forceinline__ double wave_sum_f64(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int KER>
__global__ __launch_bounds__(256) void k_projected_area(HierDev H, ProjArgs a)
{
    const int64_t qi = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (qi >= a.nq) return;
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
    for (int idx = lane; idx < total; idx += 64) {
        const int ca = idx % nx, cb = idx / nx;
        const int i = spanx >= n ? ca : ((q.cxlo + ca) & msk);
        const int j = spany >= n ? cb : ((q.cylo + cb) & msk);
        const int wdt = n + 1;
        const float2* p = H.nrm + (int64_t)j * wdt + i;
        const float2 n0 = p[0], n1 = p[1], n2 = p[wdt], n3 = p[wdt + 1];
        const uint8_t dg = H.deg[(int64_t)j * n + i];
        const float2 dd = H.det[(int64_t)j * n + i];
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const double J = (double)(half ? dd.y : dd.x);
            // kernel at the uv centroid over the included images, divided by J
            const double kj = hit_term<KER>(q, i, j, 0, half, 1.0 / 3.0, 1.0 / 3.0, (float)J, H.logn);
            if (kj == 0.0) continue;
            double v[6];
            if ((dg >> half) & 1u) {
                eqtri_f64(0.5 * ((double)n1.x + (double)n2.x), 0.5 * ((double)n1.y + (double)n2.y),
                          (double)H.rho, v);
            } else if (half == 0) {
                v[0] = n0.x; v[1] = n0.y; v[2] = n1.x; v[3] = n1.y; v[4] = n2.x; v[5] = n2.y;
            } else {
                v[0] = n3.x; v[1] = n3.y; v[2] = n2.x; v[3] = n2.y; v[4] = n1.x; v[5] = n1.y;
            }
            double r[6];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                r[2 * k] = c * v[2 * k] + sn * v[2 * k + 1];
                r[2 * k + 1] = -sn * v[2 * k] + c * v[2 * k + 1];
            }
            acc += kj * triangle_int(r, wl, wz);
        }
    }
    const double P = wave_sum_f64(acc);
    if (lane == 0) {
        a.P[qi] = (float)P;
        if (a.lambda) a.lambda[qi] = (float)(P / wz - 1.0);
    }
}

}  // namespace

hipError_t launch_projected_area(const HierDev& H, const ProjArgs& a, hipStream_t s)
{
    if (a.nq == 0) return hipSuccess;
    const dim3 grid((unsigned)((a.nq + 3) / 4)), block(256);
    if (a.kernel == PNDF_KERNEL_DISK)
        hipLaunchKernelGGL(k_projected_area<PNDF_KERNEL_DISK>, grid, block, 0, s, H, a);
    else if (a.kernel == PNDF_KERNEL_BOX)
        hipLaunchKernelGGL(k_projected_area<PNDF_KERNEL_BOX>, grid, block, 0, s, H, a);
    else
        hipLaunchKernelGGL(k_projected_area<PNDF_KERNEL_GAUSSIAN>, grid, block, 0, s, H, a);
    return hipGetLastError();
}

}  // namespace pndf
