// amrmg_transform.hip -- the domain transform of Sec. 4.1 (arXiv:1812.03689)
// between particle space S_p and computation space S_c = [-l0,l0] x [-l1,l1]
// x [-l2,l2]: the scale s = max over the particles of
// Gamma(x, l) = max_d |x_d - c_d| / l_d (c: the reference particle), the map
// x* = (x - c) / s, and the rescaling on the grid after the solve in S_c:
// phi = phi* / s and E = E* / s^2 (Eqs. potential_transform,
// efield_transform, three dimensions).
//
// Memory-bound elementwise passes: the scale reads the positions once
// (24 B per particle in FP64), the map reads and writes them (48 B), the
// rescale reads and writes each field value (16 B).  Grid-stride loops with
// a grid capped at a few workgroups per CU; the scale reduces in registers,
// then across the wavefront, then one atomic per workgroup.
#include <hip/hip_runtime.h>

#include <cmath>

#include "amrmg_kernels.hpp"

namespace amrmg {

namespace {

constexpr int TB = 256;

unsigned grid_for(int64_t n)
{
    int64_t g = (n + TB - 1) / TB;
    return (unsigned)(g < 2048 ? (g < 1 ? 1 : g) : 2048);
}

template <typename P>
__global__ __launch_bounds__(TB) void k_domain_scale(const P *__restrict__ x, const P *__restrict__ y,
                                                     const P *__restrict__ z, int64_t n, double3 c, double3 l,
                                                     unsigned long long *out)
{
    double g = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB) {
        double gx = fabs((double)x[i] - c.x) / l.x;
        double gy = fabs((double)y[i] - c.y) / l.y;
        double gz = fabs((double)z[i] - c.z) / l.z;
        // a NaN coordinate becomes +inf so that the caller sees a non-finite scale
        gx = gx == gx ? gx : INFINITY;
        gy = gy == gy ? gy : INFINITY;
        gz = gz == gz ? gz : INFINITY;
        g = fmax(g, fmax(gx, fmax(gy, gz)));
    }
    for (int o = 32; o > 0; o >>= 1) g = fmax(g, __shfl_xor(g, o));
    __shared__ double part[TB / 64];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = g;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < TB / 64; ++w) g = fmax(g, part[w]);
        // non-negative doubles order like their bit patterns
        atomicMax(out, (unsigned long long)__double_as_longlong(g));
    }
}

template <typename P>
__global__ __launch_bounds__(TB) void k_to_computation(const P *x, const P *y, const P *z, int64_t n, double3 c,
                                                       double s, P *xs, P *ys, P *zs)
{
    for (int64_t i = blockIdx.x * (int64_t)TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB) {
        const double a = ((double)x[i] - c.x) / s;
        const double b = ((double)y[i] - c.y) / s;
        const double d = ((double)z[i] - c.z) / s;
        xs[i] = (P)a;
        ys[i] = (P)b;
        zs[i] = (P)d;
    }
}

__global__ __launch_bounds__(TB) void k_divide(double *v, int64_t n, double div)
{
    for (int64_t i = blockIdx.x * (int64_t)TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB) v[i] = v[i] / div;
}

}  // namespace

void launch_domain_scale(hipStream_t st, int pos_f32, int64_t n, const void *x, const void *y, const void *z,
                         const double *c, const double *l, unsigned long long *out)
{
    if (n <= 0) return;
    const double3 cc = make_double3(c[0], c[1], c[2]), ll = make_double3(l[0], l[1], l[2]);
    if (pos_f32)
        hipLaunchKernelGGL(k_domain_scale<float>, dim3(grid_for(n)), dim3(TB), 0, st, (const float *)x,
                           (const float *)y, (const float *)z, n, cc, ll, out);
    else
        hipLaunchKernelGGL(k_domain_scale<double>, dim3(grid_for(n)), dim3(TB), 0, st, (const double *)x,
                           (const double *)y, (const double *)z, n, cc, ll, out);
}

void launch_to_computation(hipStream_t st, int pos_f32, int64_t n, const void *x, const void *y, const void *z,
                           const double *c, double s, void *xs, void *ys, void *zs)
{
    if (n <= 0) return;
    const double3 cc = make_double3(c[0], c[1], c[2]);
    if (pos_f32)
        hipLaunchKernelGGL(k_to_computation<float>, dim3(grid_for(n)), dim3(TB), 0, st, (const float *)x,
                           (const float *)y, (const float *)z, n, cc, s, (float *)xs, (float *)ys, (float *)zs);
    else
        hipLaunchKernelGGL(k_to_computation<double>, dim3(grid_for(n)), dim3(TB), 0, st, (const double *)x,
                           (const double *)y, (const double *)z, n, cc, s, (double *)xs, (double *)ys,
                           (double *)zs);
}

void launch_divide(hipStream_t st, double *v, int64_t n, double div)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_divide, dim3(grid_for(n)), dim3(TB), 0, st, v, n, div);
}

}  // namespace amrmg
