// amrmg_sort.hip -- spatial visiting order of the particles for the deposit:
// a Morton (Z-order) key of each particle's cell at a fine resolution, sorted
// with the rocPRIM radix sort (through hipCUB).  In Z-order every cell of
// every coarser level is a contiguous key range, so after the sort the
// particles that a workgroup deposits or gathers fall into a few cells and
// the deposit of a workgroup stays inside a small LDS tile on every level.
#include <hip/hip_runtime.h>

#include <hipcub/hipcub.hpp>

#include "amrmg_kernels.hpp"

namespace amrmg {

__device__ __forceinline__ uint64_t spread3(uint32_t v)
{
    uint64_t x = v & 0x1fffff;  // 21 bits
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

template <class P, class K>
__global__ void __launch_bounds__(256) k_morton_keys(int64_t n, const P *x, const P *y, const P *z, double lo0,
                                                     double lo1, double lo2, double hi0, double hi1, double hi2,
                                                     int3 nf, K *keys, uint32_t *vals)
{
    int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    double X[3] = {(double)x[p], (double)y[p], (double)z[p]};
    double lo[3] = {lo0, lo1, lo2}, hi[3] = {hi0, hi1, hi2};
    int nn[3] = {nf.x, nf.y, nf.z};
    uint64_t key = 0;
    bool inside = true;
    for (int d = 0; d < 3; ++d) {
        if (!(X[d] >= lo[d] && X[d] < hi[d])) inside = false;
        double s = (X[d] - lo[d]) / (hi[d] - lo[d]) * nn[d];
        int c = (int)floor(s);
        c = c < 0 ? 0 : (c >= nn[d] ? nn[d] - 1 : c);
        key |= spread3((uint32_t)c) << d;
    }
    keys[p] = inside ? (K)key : ~(K)0;  // particles outside the domain go last
    vals[p] = (uint32_t)p;
}

// Keys are 32-bit when the Morton code of the grid fits (up to 1024 cells per
// axis), 64-bit beyond.
size_t sort_temp_bytes(int64_t n)
{
    size_t b32 = 0, b64 = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, b32, (const uint32_t *)nullptr, (uint32_t *)nullptr,
                                             (const uint32_t *)nullptr, (uint32_t *)nullptr, (int)n, 0, 32);
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, b64, (const uint64_t *)nullptr, (uint64_t *)nullptr,
                                             (const uint32_t *)nullptr, (uint32_t *)nullptr, (int)n, 0, 63);
    return b32 > b64 ? b32 : b64;
}

template <class K>
static hipError_t order_with(hipStream_t st, int pos_f32, int64_t n, const void *x, const void *y, const void *z,
                             const double *lo, const double *hi, int3 nn, int end_bit, K *keys, uint32_t *vals,
                             void *temp, size_t temp_bytes)
{
    unsigned g = (unsigned)((n + 255) / 256);
    if (pos_f32)
        hipLaunchKernelGGL((k_morton_keys<float, K>), dim3(g), dim3(256), 0, st, n, (const float *)x,
                           (const float *)y, (const float *)z, lo[0], lo[1], lo[2], hi[0], hi[1], hi[2], nn, keys,
                           vals);
    else
        hipLaunchKernelGGL((k_morton_keys<double, K>), dim3(g), dim3(256), 0, st, n, (const double *)x,
                           (const double *)y, (const double *)z, lo[0], lo[1], lo[2], hi[0], hi[1], hi[2], nn, keys,
                           vals);
    size_t tb = temp_bytes;
    return hipcub::DeviceRadixSort::SortPairs(temp, tb, keys, keys + n, vals, vals + n, (int)n, 0, end_bit, st);
}

hipError_t particle_order(hipStream_t st, int pos_f32, int64_t n, const void *x, const void *y, const void *z,
                          const double *lo, const double *hi, const int *nf, uint64_t *keys, uint32_t *vals,
                          void *temp, size_t temp_bytes, uint32_t **perm_out)
{
    *perm_out = nullptr;
    if (n <= 0) return hipSuccess;
    int3 nn = make_int3(nf[0], nf[1], nf[2]);
    int bits = 0;
    int m = nf[0] > nf[1] ? nf[0] : nf[1];
    m = m > nf[2] ? m : nf[2];
    while ((1 << bits) < m) ++bits;
    hipError_t e;
    if (3 * bits <= 32)
        e = order_with<uint32_t>(st, pos_f32, n, x, y, z, lo, hi, nn, 3 * bits, (uint32_t *)keys, vals, temp,
                                 temp_bytes);
    else
        e = order_with<uint64_t>(st, pos_f32, n, x, y, z, lo, hi, nn, 3 * bits < 63 ? 3 * bits : 63, keys, vals,
                                 temp, temp_bytes);
    if (e != hipSuccess) return e;
    *perm_out = vals + n;
    return hipGetLastError();
}

template <class P>
__global__ void __launch_bounds__(256) k_permute(int64_t n, const uint32_t *perm, const P *x, const P *y, const P *z,
                                                 const double *q, P *xs, P *ys, P *zs, double *qs)
{
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    int64_t p = perm[i];
    xs[i] = x[p];
    ys[i] = y[p];
    zs[i] = z[p];
    qs[i] = q[p];
}

void launch_permute(hipStream_t st, int pos_f32, int64_t n, const uint32_t *perm, const void *x, const void *y,
                    const void *z, const double *q, void *xs, void *ys, void *zs, double *qs)
{
    if (n <= 0) return;
    unsigned g = (unsigned)((n + 255) / 256);
    if (pos_f32)
        hipLaunchKernelGGL((k_permute<float>), dim3(g), dim3(256), 0, st, n, perm, (const float *)x,
                           (const float *)y, (const float *)z, q, (float *)xs, (float *)ys, (float *)zs, qs);
    else
        hipLaunchKernelGGL((k_permute<double>), dim3(g), dim3(256), 0, st, n, perm, (const double *)x,
                           (const double *)y, (const double *)z, q, (double *)xs, (double *)ys, (double *)zs, qs);
}

}  // namespace amrmg
