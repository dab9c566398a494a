// Sampling of the manifold P-NDF on gfx950: one thread per sample.
//
// A sample draws u from the footprint kernel over the support that the evaluation
// integrates and returns the normal m of the triangle containing u (section
// "Sampling and evaluation"): n(u) interpolated from the texel normals, the same
// barycentric point of the equilateral replacement for a clamped triangle
// (Eq. debias), and with the cut the cluster field n^l of the unit the evaluation
// uses at u (section "Acceleration by mesh clustering").  The density of m is then
// D(m) divided by D's total mass, for every footprint kernel and cut threshold.
//
// Support.  Without the cut, the included cells [cxlo, cxhi + 1] per axis; with
// it, the units of the cut (cells or cluster nodes) whose unrolled image meets the
// included cells.  The Gaussian is drawn per axis by inverse CDF on a range S
// (the included cells, or with the cut the entry-level nodes over them) and with
// the cut rejected when its unit misses the included cells; the caller supplies
// `attempts` uniform pairs per sample for that.  Disk and box supports lie inside
// the included cells and are drawn directly from the first pair.
//
// Work per sample: the query (24 B), one uniform pair (16 B), the cut levels'
// residuals (4 B each, from the entry level down to the cut), the unit's four corner
// normals and clamp bits (for a texel cell from its leaf record), and the outputs.
// Nothing is shared between samples: the kernel is a gather-bound stream.
#include <algorithm>

#include "pndf_internal.h"

namespace pndf {
namespace {

// u on [a, b) from N(x, sig^2) truncated to [a, b), by inverse CDF
__device__ inline double trunc_gauss(double x, double sig, double a, double b, double xi)
{
    const double pa = normcdf((a - x) / sig), pb = normcdf((b - x) / sig);
    double u = x + sig * normcdfinv(pa + xi * (pb - pa));
    if (u < a) u = a;
    if (u >= b) u = nextafter(b, a);
    return u;
}

// unit-local coordinates of u in a unit of side s = 2^l, and its torus node
__device__ __forceinline__ void unit_coords(double u, int l, int mask, int* node, double* frac)
{
    const double s = (double)(1 << l);
    const double f = floor(u / s);
    *node = (int)((long long)f & (long long)mask);
    *frac = (u - f * s) / s;
}

// does the unrolled image of the level-l unit holding u meet the cells [clo, chi]
__device__ __forceinline__ bool unit_meets(double u, int l, int clo, int chi)
{
    const long long s = 1ll << l;
    const long long start = (long long)floor(u / (double)s) * s;
    return start <= (long long)chi && start + s - 1 >= (long long)clo;
}

template <int KER, bool CUT>
__global__ __launch_bounds__(256) void k_sample(HierDev H, SampleArgs a)
{
    const int64_t k = a.first + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.end) return;
    const QuerySetup q = setup_query(a.q[k], a.s2r, CUT ? a.tau : 0.f, H.L, H.eps, KER);
    bool ok = q.valid;
    const double2* xi = reinterpret_cast<const double2*>(a.xi);
    double2 u = make_double2(__longlong_as_double(0x7ff8000000000000ll), __longlong_as_double(0x7ff8000000000000ll));
    float2 mo = make_float2(__int_as_float(0x7fc00000), __int_as_float(0x7fc00000));
    uint64_t id = ~0ull;
    // attempts that may be needed: only the Gaussian with the cut rejects
    const int tries = (KER == PNDF_KERNEL_GAUSSIAN && CUT) ? a.attempts : 1;
    for (int t = 0; ok && t < tries; ++t) {
        const double2 x = xi[(int64_t)t * a.nq + k];
        if (!(x.x >= 0.0 && x.x < 1.0 && x.y >= 0.0 && x.y < 1.0)) {
            ok = false;
            break;
        }
        if constexpr (KER == PNDF_KERNEL_DISK) {
            double sn, cs;
            sincospi(2.0 * x.y, &sn, &cs);
            const double rad = sqrt(x.x);
            u.x = (double)q.x + (double)q.rx * rad * cs;
            u.y = (double)q.y + (double)q.ry * rad * sn;
        } else if constexpr (KER == PNDF_KERNEL_BOX) {
            u.x = (double)q.x + (double)q.rx * (2.0 * x.x - 1.0);
            u.y = (double)q.y + (double)q.ry * (2.0 * x.y - 1.0);
        } else {
            const int l = CUT ? q.l0 : 0;
            const double ax = (double)(floor_div_pow2(q.cxlo, l) << l);
            const double bx = (double)((floor_div_pow2(q.cxhi, l) + 1) << l);
            const double ay = (double)(floor_div_pow2(q.cylo, l) << l);
            const double by = (double)((floor_div_pow2(q.cyhi, l) + 1) << l);
            u.x = trunc_gauss((double)q.x, (double)a.q[k].sx, ax, bx, x.x);
            u.y = trunc_gauss((double)q.y, (double)a.q[k].sy, ay, by, x.y);
        }
        // the unit of the cut that holds u: the first level from the entry level down
        // whose residual is within the threshold, else the cell
        int lev = 0;
        if constexpr (CUT) {
            // (a short dependent chain per thread; the many threads in flight hide it)
            for (int l = q.l0; l >= 1; --l) {
                int I, J;
                double fx, fy;
                const int mask = (H.n >> l) - 1;
                unit_coords(u.x, l, mask, &I, &fx);
                unit_coords(u.y, l, mask, &J, &fy);
                if (H.clu_e[level_offset(H.logn, l) + morton((uint32_t)I, (uint32_t)J)] <= q.t) {
                    lev = l;
                    break;
                }
            }
            if (KER == PNDF_KERNEL_GAUSSIAN &&
                !(unit_meets(u.x, lev, q.cxlo, q.cxhi) && unit_meets(u.y, lev, q.cylo, q.cyhi)))
                continue;  // rejected: the unit lies outside the support
        }
        int I, J;
        double U, V;
        unit_coords(u.x, lev, (H.n >> lev) - 1, &I, &U);
        unit_coords(u.y, lev, (H.n >> lev) - 1, &J, &V);
        const int half = U + V < 1.0 ? 0 : 1;
        double w0, w1, w2;
        if (half == 0) {
            w0 = 1.0 - U - V; w1 = U; w2 = V;
        } else {
            w0 = U + V - 1.0; w1 = 1.0 - U; w2 = 1.0 - V;
        }
        float2 n0, n1, n2, n3;
        bool clamped;
        if (lev == 0) {
            // from the cell's 2 x 2 leaf record (its 3 x 3 corners and clamp bytes in
            // 80 B), not from two rows of the normal plane and the clamp array: one
            // scattered record instead of three scattered lines per sample
            const QuadRec* r = H.quad + morton((uint32_t)I >> 1, (uint32_t)J >> 1);
            const int di = I & 1, dj = J & 1, k = 3 * dj + di;
            n0 = r->t[k]; n1 = r->t[k + 1]; n2 = r->t[k + 3]; n3 = r->t[k + 4];
            clamped = (r->deg[2 * dj + di] >> half) & 1u;
        } else {
            const int64_t ix = level_offset(H.logn, lev) + morton((uint32_t)I, (uint32_t)J);
            const float4 ca = H.clu_t[2 * ix], cb = H.clu_t[2 * ix + 1];
            n0 = make_float2(ca.x, ca.y); n1 = make_float2(ca.z, ca.w);
            n2 = make_float2(cb.x, cb.y); n3 = make_float2(cb.z, cb.w);
            clamped = (clamp_bits(ca, cb) >> half) & 1u;
        }
        double v[6];
        if (clamped) {
            eqtri_f64(0.5 * ((double)n1.x + (double)n2.x), 0.5 * ((double)n1.y + (double)n2.y),
                      (double)(H.rho * (float)(1 << lev)), v);
        } else if (half == 0) {
            v[0] = n0.x; v[1] = n0.y; v[2] = n1.x; v[3] = n1.y; v[4] = n2.x; v[5] = n2.y;
        } else {
            v[0] = n3.x; v[1] = n3.y; v[2] = n2.x; v[3] = n2.y; v[4] = n1.x; v[5] = n1.y;
        }
        mo.x = (float)(w0 * v[0] + w1 * v[2] + w2 * v[4]);
        mo.y = (float)(w0 * v[1] + w1 * v[3] + w2 * v[5]);
        id = tri_id(lev, I, J, half);
        break;
    }
    if (!ok) u = make_double2(__longlong_as_double(0x7ff8000000000000ll), __longlong_as_double(0x7ff8000000000000ll));
    a.m[k] = mo;
    if (a.tri) a.tri[k] = id;
    if (a.u) a.u[k] = u;
}

// One thread per sample, in launches of at most launch_chunk() samples (the
// uniforms keep their stride nq: attempt t of sample k at t nq + k).
template <int KER>
void launch_kernel(const HierDev& H, const SampleArgs& a0, hipStream_t s)
{
    const int64_t chunk = launch_chunk();
    for (int64_t off = 0; off < a0.nq; off += chunk) {
        SampleArgs a = a0;
        a.first = off;
        a.end = std::min(a0.nq, off + chunk);
        const dim3 grid((unsigned)((a.end - a.first + 255) / 256)), block(256);
        if (a.tau > 0.f)
            hipLaunchKernelGGL((k_sample<KER, true>), grid, block, 0, s, H, a);
        else
            hipLaunchKernelGGL((k_sample<KER, false>), grid, block, 0, s, H, a);
        if (hipPeekAtLastError() != hipSuccess) return;
    }
}

}  // namespace

hipError_t launch_sample(const HierDev& H, const SampleArgs& a, hipStream_t s)
{
    if (a.nq == 0) return hipSuccess;
    if (a.kernel == PNDF_KERNEL_DISK)
        launch_kernel<PNDF_KERNEL_DISK>(H, a, s);
    else if (a.kernel == PNDF_KERNEL_BOX)
        launch_kernel<PNDF_KERNEL_BOX>(H, a, s);
    else
        launch_kernel<PNDF_KERNEL_GAUSSIAN>(H, a, s);
    return hipGetLastError();
}

}  // namespace pndf
