// Mesh build: padded texel-normal plane, per-cell clamp bits and Jacobians.
//
// Each texel cell (i, j) carries two triangles (Fig. normal_map, Eq. interpolation):
// lower (u0, u1, u2) with normals (n0, n1, n2) and upper (u3, u2, u1) with
// normals (n3, n2, n1).  Their Jacobian is twice the normal-space area
// (Eq. jacobian), evaluated here once in FP64 from the float32 normals; triangles
// below eps are clamped (section "Preventing Jacobian singularity").
#include "pndf_internal.h"

namespace pndf {

// |(c - a) x (b - a)| in FP64 with each product rounded before the difference, so
// the clamp decision is a fixed function of the float inputs.
__device__ __forceinline__ double jac64(float2 a, float2 b, float2 c)
{
    double p = __dmul_rn((double)c.x - (double)a.x, (double)b.y - (double)a.y);
    double q = __dmul_rn((double)c.y - (double)a.y, (double)b.x - (double)a.x);
    return fabs(__dsub_rn(p, q));
}

__global__ void k_build_mesh(const float* __restrict__ in, int n, float eps,
                             float2* __restrict__ nrm, uint8_t* __restrict__ deg,
                             float2* __restrict__ det, unsigned* __restrict__ flag)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= n) return;
    const int m = n - 1;  // n is a power of two
    auto tex = [&](int ii, int jj) {
        const int k = 2 * ((jj & m) * n + (ii & m));
        return make_float2(in[k], in[k + 1]);
    };
    const float2 n0 = tex(i, j), n1 = tex(i + 1, j), n2 = tex(i, j + 1), n3 = tex(i + 1, j + 1);
    const double r2 = (double)n0.x * (double)n0.x + (double)n0.y * (double)n0.y;
    if (!(isfinite(n0.x) && isfinite(n0.y)) || !(r2 < 1.0)) atomicOr(flag, 1u);
    const double dl = jac64(n0, n1, n2);
    const double du = jac64(n3, n2, n1);
    const double e = (double)eps;
    const bool cl = dl < e, cu = du < e;
    deg[j * n + i] = (uint8_t)((cl ? 1 : 0) | (cu ? 2 : 0));
    det[j * n + i] = make_float2(cl ? eps : (float)dl, cu ? eps : (float)du);
    const int w = n + 1;
    nrm[j * w + i] = n0;
    if (i == 0) nrm[j * w + n] = n0;
    if (j == 0) nrm[n * w + i] = n0;
    if (i == 0 && j == 0) nrm[n * w + n] = n0;
}

hipError_t launch_build_mesh(const float* in, int n, float eps, float2* nrm, uint8_t* deg,
                             float2* det, unsigned* d_flag, hipStream_t s)
{
    const int bx = n < 256 ? n : 256;
    dim3 grid((n + bx - 1) / bx, n);
    hipLaunchKernelGGL(k_build_mesh, grid, dim3(bx), 0, s, in, n, eps, nrm, deg, det, d_flag);
    return hipGetLastError();
}

}  // namespace pndf
