// amrmg_sort.hip -- spatial visiting order of the particles for the deposit,
// the gather and the tagging passes: a counting sort of the particles into
// buckets, the cells of a grid of at most 128 cells per axis (the level-0
// cells, merged 2^3 at a time while an axis has more), numbered in Morton
// (Z) order.  In Z-order the buckets of any aligned block are contiguous, so
// consecutive particles fall into a few neighbouring buckets and the
// deposit of a workgroup stays inside a small LDS tile on every level; the
// order inside a bucket does not matter (it is the order in which the
// particles claimed their slots).  Passes: count with slot claims, the
// counts in bucket order, exclusive scan (amrmg_scan.hip), scatter of the
// order (which also leaves its inverse), ordered copy.
#include <hip/hip_runtime.h>

#include "amrmg_kernels.hpp"

namespace amrmg {

__device__ __forceinline__ uint32_t spread3_10(uint32_t v)
{
    uint32_t x = v & 0x3ff;  // 10 bits
    x = (x | (x << 16)) & 0x030000ffu;
    x = (x | (x << 8)) & 0x0300f00fu;
    x = (x | (x << 4)) & 0x030c30c3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

struct BucketGrid {
    double lo[3], scale[3];  // cell = floor((x - lo) * scale) on the level-0 grid
    int n[3];                // level-0 cells per axis
    int shift;               // bucket = cell >> shift
    uint32_t nbkt;           // Morton space of the buckets; bucket nbkt holds the particles outside
    int sbits;               // counters of 2^sbits consecutive buckets lie on different cache lines
};

// Counter of bucket k: consecutive buckets are spread over distant counters
// (a transpose of nbkt / 2^sbits rows of 2^sbits), so that the slot claims
// of a dense region, many buckets with consecutive Morton codes, do not
// queue on a few cache lines.  A bijection on [0, nbkt); nbkt maps to itself.
__host__ __device__ __forceinline__ uint32_t counter_of(const BucketGrid &G, uint32_t k)
{
    if (k >= G.nbkt) return k;
    const uint32_t S = 1u << G.sbits;
    return (k & (S - 1)) * (G.nbkt >> G.sbits) + (k >> G.sbits);
}

template <class P>
__global__ void __launch_bounds__(256) k_bucket_count(int64_t n, const P *x, const P *y, const P *z, BucketGrid G,
                                                      uint32_t *count, uint32_t *key, uint32_t *slot)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    const double X[3] = {(double)x[p], (double)y[p], (double)z[p]};
    uint32_t k = 0;
    bool inside = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double s = (X[d] - G.lo[d]) * G.scale[d];
        if (!(s >= 0.0 && s < (double)G.n[d])) inside = false;
        int c = (int)floor(s);
        c = c < 0 ? 0 : (c >= G.n[d] ? G.n[d] - 1 : c);
        k |= spread3_10((uint32_t)(c >> G.shift)) << d;
    }
    if (!inside) k = G.nbkt;
    key[p] = k;
    slot[p] = atomicAdd(&count[counter_of(G, k)], 1u);
}

// the counts in bucket order, for the scan
__global__ void __launch_bounds__(256) k_bucket_gather(BucketGrid G, const uint32_t *count, uint32_t *ordered)
{
    const uint32_t k = blockIdx.x * 256 + threadIdx.x;
    if (k <= G.nbkt) ordered[k] = count[counter_of(G, k)];
}

// perm[dst] = p at dst = start of p's bucket + p's slot; the slot is then
// replaced by dst, so that slot holds the inverse order (a coalesced write)
__global__ void __launch_bounds__(256) k_bucket_scatter(int64_t n, const uint32_t *key, uint32_t *slot,
                                                        const uint32_t *start, uint32_t *perm)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    const uint32_t dst = start[key[p]] + slot[p];
    perm[dst] = (uint32_t)p;
    slot[p] = dst;
}

// the particles in visiting order (random reads, coalesced writes: faster
// than scattering them with perm)
template <class P>
__global__ void __launch_bounds__(256) k_copy_ordered(int64_t n, const uint32_t *perm, const P *x, const P *y,
                                                      const P *z, const double *q, P *xs, P *ys, P *zs, double *qs)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const uint32_t p = perm[i];
    xs[i] = x[p];
    ys[i] = y[p];
    zs[i] = z[p];
    qs[i] = q[p];
}

static BucketGrid bucket_grid(const double *lo, const double *hi, const int *n0)
{
    BucketGrid G{};
    int m = 1;
    for (int d = 0; d < 3; ++d) {
        G.lo[d] = lo[d];
        G.scale[d] = (double)n0[d] / (hi[d] - lo[d]);
        G.n[d] = n0[d];
        m = n0[d] > m ? n0[d] : m;
    }
    int bits = 0;
    while ((1 << bits) < m) ++bits;
    G.shift = bits > 7 ? bits - 7 : 0;
    bits -= G.shift;
    G.nbkt = 1u << (3 * bits);
    G.sbits = 3 * bits < 10 ? 3 * bits : 10;
    return G;
}

size_t order_count_entries(const double *lo, const double *hi, const int *n0)
{
    return (size_t)bucket_grid(lo, hi, n0).nbkt + 1;
}

int order_bucket_shift(const double *lo, const double *hi, const int *n0) { return bucket_grid(lo, hi, n0).shift; }

size_t order_temp_bytes(size_t entries) { return scan_temp_bytes<uint32_t>((int64_t)entries); }

hipError_t particle_order(hipStream_t st, int pos_f32, int64_t n, const void *x, const void *y, const void *z,
                          const double *q, const double *lo, const double *hi, const int *n0, uint32_t *key,
                          uint32_t *slot, uint32_t *count, uint32_t *start, uint32_t *perm, void *temp,
                          size_t temp_bytes, void *xs, void *ys, void *zs, double *qs)
{
    if (n <= 0) return hipSuccess;
    const BucketGrid G = bucket_grid(lo, hi, n0);
    const int entries = (int)G.nbkt + 1;
    hipError_t e = hipMemsetAsync(count, 0, sizeof(uint32_t) * entries, st);
    if (e != hipSuccess) return e;
    const unsigned g = (unsigned)((n + 255) / 256);
    if (pos_f32)
        hipLaunchKernelGGL((k_bucket_count<float>), dim3(g), dim3(256), 0, st, n, (const float *)x, (const float *)y,
                           (const float *)z, G, count, key, slot);
    else
        hipLaunchKernelGGL((k_bucket_count<double>), dim3(g), dim3(256), 0, st, n, (const double *)x,
                           (const double *)y, (const double *)z, G, count, key, slot);
    uint32_t *ordered = count + entries;
    hipLaunchKernelGGL(k_bucket_gather, dim3((entries + 255) / 256), dim3(256), 0, st, G, count, ordered);
    e = exclusive_scan<uint32_t>(st, ordered, start, entries, temp, temp_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bucket_scatter, dim3(g), dim3(256), 0, st, n, key, slot, start, perm);
    if (xs) launch_copy_ordered(st, pos_f32, n, perm, x, y, z, q, xs, ys, zs, qs);
    return hipGetLastError();
}

void launch_copy_ordered(hipStream_t st, int pos_f32, int64_t n, const uint32_t *perm, const void *x, const void *y,
                         const void *z, const double *q, void *xs, void *ys, void *zs, double *qs)
{
    if (n <= 0) return;
    const unsigned g = (unsigned)((n + 255) / 256);
    if (pos_f32)
        hipLaunchKernelGGL((k_copy_ordered<float>), dim3(g), dim3(256), 0, st, n, perm, (const float *)x,
                           (const float *)y, (const float *)z, q, (float *)xs, (float *)ys, (float *)zs, qs);
    else
        hipLaunchKernelGGL((k_copy_ordered<double>), dim3(g), dim3(256), 0, st, n, perm, (const double *)x,
                           (const double *)y, (const double *)z, q, (double *)xs, (double *)ys, (double *)zs, qs);
}

}  // namespace amrmg
