// amrmg_scan.hip -- exclusive prefix sums of unsigned integers on the device,
// used by the particle visiting order (the radix sort's tile offsets) and the
// brick-table build (face and update-list offsets).  Up to 16384 values, one
// workgroup in one launch; beyond, two launches:
//   1. every workgroup sums its tile of SCAN_TILE consecutive values;
//   2. every workgroup adds the sums of all tiles before its own (read by the
//      whole workgroup and reduced in LDS) to the exclusive scan of its tile.
// The result is exact (integer arithmetic) and does not depend on the launch
// shape.
#include <hip/hip_runtime.h>

#include "amrmg_kernels.hpp"

namespace amrmg {

constexpr int SCAN_NT = 256, SCAN_PER = 8, SCAN_TILE = SCAN_NT * SCAN_PER;

// inclusive sum over the workgroup of one value per thread; returns the
// thread's inclusive prefix and writes the workgroup total to *total
template <class V>
__device__ V block_inclusive_scan(V v, V *lds, V *total)
{
    const int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int off = 1; off < SCAN_NT; off <<= 1) {
        const V add = t >= off ? lds[t - off] : (V)0;
        __syncthreads();
        lds[t] += add;
        __syncthreads();
    }
    const V r = lds[t];
    if (total) *total = lds[SCAN_NT - 1];
    __syncthreads();
    return r;
}

template <class V>
__global__ void __launch_bounds__(SCAN_NT) k_scan_tiles(const V *in, int64_t n, V *tile_sum)
{
    __shared__ V lds[SCAN_NT];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_PER;
    V s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_PER; ++i)
        if (base + i < n) s += in[base + i];
    V total;
    (void)block_inclusive_scan(s, lds, &total);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

template <class V>
__global__ void __launch_bounds__(SCAN_NT) k_scan_apply(const V *in, int64_t n, const V *tile_sum, V *out)
{
    __shared__ V lds[SCAN_NT];
    // the sums of the tiles before this one
    V before = 0;
    for (int t = threadIdx.x; t < (int)blockIdx.x; t += SCAN_NT) before += tile_sum[t];
    V prefix;
    (void)block_inclusive_scan(before, lds, &prefix);
    // the tile: each thread scans its SCAN_PER values, the threads' totals are
    // scanned across the workgroup
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_PER;
    V v[SCAN_PER], s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_PER; ++i) {
        v[i] = base + i < n ? in[base + i] : (V)0;
        s += v[i];
    }
    const V incl = block_inclusive_scan(s, lds, (V *)nullptr);
    V run = prefix + incl - s;
#pragma unroll
    for (int i = 0; i < SCAN_PER; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
}

// Up to SCAN_ONE values: one workgroup of 1024 threads, each scanning 16
// consecutive values, the threads' totals scanned across the workgroup (one
// launch instead of two: short scans are launch-bound).
constexpr int SCAN_ONE_NT = 1024, SCAN_ONE_PER = 16, SCAN_ONE = SCAN_ONE_NT * SCAN_ONE_PER;

template <class V>
__global__ void __launch_bounds__(SCAN_ONE_NT) k_scan_one(const V *in, int64_t n, V *out)
{
    __shared__ V lds[SCAN_ONE_NT];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)t * SCAN_ONE_PER;
    V v[SCAN_ONE_PER], s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ONE_PER; ++i) {
        v[i] = base + i < n ? in[base + i] : (V)0;
        s += v[i];
    }
    lds[t] = s;
    __syncthreads();
    for (int off = 1; off < SCAN_ONE_NT; off <<= 1) {
        const V add = t >= off ? lds[t - off] : (V)0;
        __syncthreads();
        lds[t] += add;
        __syncthreads();
    }
    V run = lds[t] - s;
#pragma unroll
    for (int i = 0; i < SCAN_ONE_PER; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
}

template <class V>
size_t scan_temp_bytes(int64_t n)
{
    return sizeof(V) * (size_t)((n + SCAN_TILE - 1) / SCAN_TILE + 1);
}

template <class V>
hipError_t exclusive_scan(hipStream_t st, const V *in, V *out, int64_t n, void *temp, size_t temp_bytes)
{
    if (n <= 0) return hipSuccess;
    if (n <= SCAN_ONE) {
        hipLaunchKernelGGL((k_scan_one<V>), dim3(1), dim3(SCAN_ONE_NT), 0, st, in, n, out);
        return hipGetLastError();
    }
    if (!temp || temp_bytes < scan_temp_bytes<V>(n)) return hipErrorInvalidValue;
    const int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (tiles > INT32_MAX) return hipErrorInvalidValue;
    V *sums = (V *)temp;
    hipLaunchKernelGGL((k_scan_tiles<V>), dim3((unsigned)tiles), dim3(SCAN_NT), 0, st, in, n, sums);
    hipLaunchKernelGGL((k_scan_apply<V>), dim3((unsigned)tiles), dim3(SCAN_NT), 0, st, in, n, sums, out);
    return hipGetLastError();
}

template size_t scan_temp_bytes<uint32_t>(int64_t);
template size_t scan_temp_bytes<uint64_t>(int64_t);
template hipError_t exclusive_scan<uint32_t>(hipStream_t, const uint32_t *, uint32_t *, int64_t, void *, size_t);
template hipError_t exclusive_scan<uint64_t>(hipStream_t, const uint64_t *, uint64_t *, int64_t, void *, size_t);

}  // namespace amrmg
