// amrmg_sort.hip -- spatial visiting order of the particles for the deposit,
// the gather and the tagging passes: a stable least-significant-digit radix
// sort of the particles by the Morton (Z-order) code of their cell on a sort
// grid (sort_grid: the level-0 grid refined towards about four particles per
// cell, at most to the finest level, merged 2^3 at a time while an axis has
// more than 1024 cells, so at most 30 key bits), 6 to 10 bits per pass.  In Z-order the cells
// of any aligned block are contiguous, so consecutive particles lie in a few
// neighbouring cells and the deposit of a workgroup stays inside a small LDS
// tile on every level.  Stable: particles of one cell keep their order, so
// the visiting order is a function of the positions alone.
//
// Per pass: a histogram of the pass's digit per tile of consecutive keys
// (in LDS), an exclusive scan of the histograms in
// (digit, tile) order (amrmg_scan.hip), which gives every tile its output
// start per digit, and the scatter: each tile walks its keys in order, 256 at
// a time, ranks them among the keys of the same digit with wavefront ballots
// (one per digit bit) into LDS in digit order, then writes each digit's run
// of keys to consecutive places from its start.  The first
// histogram comes with the keys; the last pass writes the order and its
// inverse instead of keys.
#include <hip/hip_runtime.h>

#include "amrmg_kernels.hpp"

namespace amrmg {

// a tile is RADIX_NT * IT keys: IT = 16 for large sorts, 4 below 4M keys,
// where 16 would leave fewer tiles than the chip has compute units and each
// tile's rounds (separated by barriers) would set the pace alone
constexpr int RADIX_NT = 256, ITEMS_LARGE = 16, ITEMS_SMALL = 4;
constexpr int RADIX_WAVES = RADIX_NT / 64;
constexpr int SORT_AXIS_BITS = 10, DIGIT_MIN = 6, DIGIT_MAX = 10;

__device__ __forceinline__ uint32_t spread3_10(uint32_t v)
{
    uint32_t x = v & 0x3ff;  // 10 bits
    x = (x | (x << 16)) & 0x030000ffu;
    x = (x | (x << 8)) & 0x0300f00fu;
    x = (x | (x << 4)) & 0x030c30c3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

struct SortGrid {
    double lo[3], scale[3];  // cell = floor((x - lo) * scale) on the sort grid, clamped
    int n[3];                // sort-grid cells per axis
    int shift;               // sort cell = cell >> shift
    int bits;                // key bits (three per axis bit)
};

// The sort grid: the level-0 grid refined until its cells hold about four
// particles on average (about n / 4 cells), but not beyond the finest
// level, and then merged 2^3 at a time while an axis has more than 1024
// cells.  Finer orders keep a deposit workgroup's particles in fewer cells,
// but on the coarse levels those then collide in the LDS tile, and every
// three key bits more can cost a sort pass.
static SortGrid sort_grid(const double *lo, const double *hi, const int *n0, int levels, int64_t n)
{
    SortGrid G{};
    int m0 = 1;
    for (int d = 0; d < 3; ++d) m0 = n0[d] > m0 ? n0[d] : m0;
    int r = 0;
    while (r < levels && (double)m0 * (double)(1 << r) * (double)m0 * (double)(1 << r) * (double)m0 * (double)(1 << r) <
                             (double)n / 4.0)
        ++r;
    int m = 1;
    for (int d = 0; d < 3; ++d) {
        G.lo[d] = lo[d];
        G.n[d] = n0[d] << r;
        G.scale[d] = (double)G.n[d] / (hi[d] - lo[d]);
        m = G.n[d] > m ? G.n[d] : m;
    }
    int b = 0;
    while ((1 << b) < m) ++b;
    G.shift = b > SORT_AXIS_BITS ? b - SORT_AXIS_BITS : 0;
    G.bits = 3 * (b - G.shift);
    return G;
}

static int radix_items(int64_t n) { return n < ((int64_t)4 << 20) ? ITEMS_SMALL : ITEMS_LARGE; }
static int radix_tiles(int64_t n)
{
    const int64_t tile = (int64_t)RADIX_NT * radix_items(n);
    return (int)((n + tile - 1) / tile);
}
// passes of at most DIGIT_MAX bits, the digit as wide as the passes need
static int radix_passes(const SortGrid &G) { return G.bits <= DIGIT_MAX ? 1 : (G.bits + DIGIT_MAX - 1) / DIGIT_MAX; }
static int radix_digit(const SortGrid &G)
{
    const int p = radix_passes(G), d = (G.bits + p - 1) / p;
    return d < DIGIT_MIN ? DIGIT_MIN : d;
}
static size_t sort_align(size_t x) { return (x + 255) & ~(size_t)255; }

// keys of the particles (a particle outside the domain takes the nearest
// cell: the deposit skips it wherever it is visited) and the histogram of
// their lowest digit per tile, hist[digit * tiles + tile]
template <class P, int DB, int IT>
__global__ void __launch_bounds__(RADIX_NT) k_sort_keys(int64_t n, const P *x, const P *y, const P *z, SortGrid G,
                                                        int tiles, uint32_t *key, uint32_t *hist)
{
    constexpr int BINS = 1 << DB;
    __shared__ uint32_t h[BINS];
    for (int b = threadIdx.x; b < BINS; b += RADIX_NT) h[b] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * (RADIX_NT * IT);
    for (int r = 0; r < IT; ++r) {
        const int64_t p = base + r * RADIX_NT + threadIdx.x;
        if (p >= n) break;
        const double X[3] = {(double)x[p], (double)y[p], (double)z[p]};
        uint32_t k = 0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            // clamped in floating point first (fmax takes 0 for a NaN)
            const double s = fmin(fmax((X[d] - G.lo[d]) * G.scale[d], 0.0), (double)(G.n[d] - 1));
            k |= spread3_10((uint32_t)s >> G.shift) << d;
        }
        key[p] = k;
        atomicAdd(&h[k & (BINS - 1)], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < BINS; b += RADIX_NT) hist[(size_t)b * tiles + blockIdx.x] = h[b];
}

template <int DB, int IT>
__global__ void __launch_bounds__(RADIX_NT) k_radix_hist(int64_t n, const uint32_t *key, int shift, int tiles,
                                                         uint32_t *hist)
{
    constexpr int BINS = 1 << DB;
    __shared__ uint32_t h[BINS];
    for (int b = threadIdx.x; b < BINS; b += RADIX_NT) h[b] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * (RADIX_NT * IT);
    for (int r = 0; r < IT; ++r) {
        const int64_t i = base + r * RADIX_NT + threadIdx.x;
        if (i >= n) break;
        atomicAdd(&h[(key[i] >> shift) & (BINS - 1)], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < BINS; b += RADIX_NT) hist[(size_t)b * tiles + blockIdx.x] = h[b];
}

// One pass's scatter with digits of DB bits.  hist[digit * tiles + tile]: the
// tile's count of each digit; offs: the exclusive scan of hist, where the
// tile's keys of that digit start in the output.  The tile's keys are first
// ranked into LDS in digit order (stably: 256 at a time, ranked within each
// wavefront by ballots on the digit bits, then across the wavefronts), so
// that the keys of one digit leave in one run of consecutive addresses.
// vin == nullptr: the values are the indices (first pass).  kout == nullptr:
// no keys written (last pass); iperm: also the inverse order, iperm[value] =
// position (last pass).
template <int DB, int IT>
__global__ void __launch_bounds__(RADIX_NT) k_radix_scatter(int64_t n, const uint32_t *kin, const uint32_t *vin,
                                                            int shift, int tiles, const uint32_t *hist,
                                                            const uint32_t *offs, uint32_t *kout, uint32_t *vout,
                                                            uint32_t *iperm)
{
    constexpr int BINS = 1 << DB, BPT = BINS > RADIX_NT ? BINS / RADIX_NT : 1;  // bins per thread
    constexpr int TILE = RADIX_NT * IT;
    __shared__ uint32_t kbuf[TILE], vbuf[TILE];
    __shared__ uint32_t wcnt[RADIX_WAVES][BINS];  // this round's count per wavefront and digit
    __shared__ uint32_t run[BINS];                // next place in the tile per digit
    __shared__ uint32_t lstart[BINS];             // where the digit's keys start in the tile
    __shared__ uint32_t part[RADIX_NT];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    for (int b = t; b < BINS; b += RADIX_NT)
        for (int w = 0; w < RADIX_WAVES; ++w) wcnt[w][b] = 0;
    // exclusive scan of the tile's histogram over the digits: each thread
    // sums BPT consecutive digits, then a scan of the 256 sums
    uint32_t c[BPT], own = 0;
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
        const int b = t * BPT + j;
        c[j] = b < BINS ? hist[(size_t)b * tiles + blockIdx.x] : 0u;
        own += c[j];
    }
    part[t] = own;
    __syncthreads();
    for (int off = 1; off < RADIX_NT; off <<= 1) {
        const uint32_t add = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += add;
        __syncthreads();
    }
    uint32_t acc = part[t] - own;
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
        const int b = t * BPT + j;
        if (b < BINS) {
            lstart[b] = acc;
            run[b] = acc;
        }
        acc += c[j];
    }
    __syncthreads();
    const uint64_t below = (1ull << lane) - 1;
    const int64_t base = (int64_t)blockIdx.x * TILE;
    // the tile's keys and values, all loaded before the first round (a
    // load per round would wait a memory latency behind each round's barriers)
    uint32_t kr[IT], vr[IT];
#pragma unroll
    for (int r = 0; r < IT; ++r) {
        const int64_t i = base + r * RADIX_NT + t;
        kr[r] = i < n ? kin[i] : 0u;
        vr[r] = i < n ? (vin ? vin[i] : (uint32_t)i) : 0u;
    }
#pragma unroll
    for (int r = 0; r < IT; ++r) {
        const int64_t i = base + r * RADIX_NT + t;
        const bool valid = i < n;
        const uint32_t k = kr[r], v = vr[r];
        const uint32_t d = (k >> shift) & (BINS - 1);
        // the valid lanes of the wavefront with this lane's digit
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < DB; ++b) {
            const uint64_t bal = __ballot((d >> b) & 1u);
            m &= ((d >> b) & 1u) ? bal : ~bal;
        }
        const uint32_t rank = (uint32_t)__popcll(m & below);
        if (valid && rank == 0) wcnt[wave][d] = (uint32_t)__popcll(m);
        __syncthreads();
        if (valid) {
            uint32_t pos = run[d] + rank;
            for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
            kbuf[pos] = k;
            vbuf[pos] = v;
        }
        __syncthreads();
        for (int b = t; b < BINS; b += RADIX_NT) {
            uint32_t add = 0;
#pragma unroll
            for (int w = 0; w < RADIX_WAVES; ++w) {
                add += wcnt[w][b];
                wcnt[w][b] = 0;
            }
            run[b] += add;
        }
        __syncthreads();
    }
    // the tile in digit order to the output: a digit's keys go to
    // consecutive places from its start
    const int cnt_tile = (int)(n - base < TILE ? n - base : TILE);
    for (int j = t; j < cnt_tile; j += RADIX_NT) {
        const uint32_t k = kbuf[j], v = vbuf[j];
        const uint32_t d = (k >> shift) & (BINS - 1);
        const uint32_t pos = offs[(size_t)d * tiles + blockIdx.x] + (uint32_t)j - lstart[d];
        if (kout) kout[pos] = k;
        vout[pos] = v;
        if (iperm) iperm[v] = pos;
    }
}

// the particles in visiting order (random reads, coalesced writes: faster
// than scattering them with the order)
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

int order_cell_shift(const double *lo, const double *hi, const int *n0, int levels, int64_t n)
{
    const SortGrid G = sort_grid(lo, hi, n0, levels, n);
    int r = 0;
    while ((n0[0] << r) < G.n[0]) ++r;
    return G.shift - r;
}

// scratch layout: keys A, keys B, values A, values B [n each], histograms
// and offsets [2^DIGIT_MAX * tiles each], the scan's temporary
struct SortScratch {
    uint32_t *ka, *kb, *va, *vb, *hist, *offs;
    void *temp;
    size_t temp_bytes, total;
};

static SortScratch sort_scratch(int64_t n, void *base)
{
    SortScratch S{};
    const size_t entries = ((size_t)1 << DIGIT_MAX) * (size_t)radix_tiles(n);
    const size_t nb = sort_align(sizeof(uint32_t) * (size_t)n), hb = sort_align(sizeof(uint32_t) * entries);
    char *p = (char *)base;
    size_t o = 0;
    auto at = [&](size_t bytes) -> char * {
        const size_t q = o;
        o += bytes;
        return p ? p + q : nullptr;
    };
    S.ka = (uint32_t *)at(nb);
    S.kb = (uint32_t *)at(nb);
    S.va = (uint32_t *)at(nb);
    S.vb = (uint32_t *)at(nb);
    S.hist = (uint32_t *)at(hb);
    S.offs = (uint32_t *)at(hb);
    S.temp_bytes = sort_align(scan_temp_bytes<uint32_t>((int64_t)entries));
    S.temp = at(S.temp_bytes);
    S.total = o;
    return S;
}

size_t order_scratch_bytes(int64_t n) { return n > 0 ? sort_scratch(n, nullptr).total : 0; }

template <int DB, int IT>
static hipError_t sort_passes(hipStream_t st, int pos_f32, int64_t n, const void *x, const void *y, const void *z,
                              const SortGrid &G, const SortScratch &S, uint32_t *perm, uint32_t *iperm)
{
    const int tiles = radix_tiles(n), passes = radix_passes(G);
    if (pos_f32)
        hipLaunchKernelGGL((k_sort_keys<float, DB, IT>), dim3(tiles), dim3(RADIX_NT), 0, st, n, (const float *)x,
                           (const float *)y, (const float *)z, G, tiles, S.ka, S.hist);
    else
        hipLaunchKernelGGL((k_sort_keys<double, DB, IT>), dim3(tiles), dim3(RADIX_NT), 0, st, n, (const double *)x,
                           (const double *)y, (const double *)z, G, tiles, S.ka, S.hist);
    const uint32_t *kin = S.ka, *vin = nullptr;
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = DB * pass;
        const bool last = pass == passes - 1;
        if (pass > 0)
            hipLaunchKernelGGL((k_radix_hist<DB, IT>), dim3(tiles), dim3(RADIX_NT), 0, st, n, kin, shift, tiles, S.hist);
        hipError_t e = exclusive_scan<uint32_t>(st, S.hist, S.offs, ((int64_t)1 << DB) * tiles, S.temp, S.temp_bytes);
        if (e != hipSuccess) return e;
        uint32_t *kout = last ? nullptr : (kin == S.ka ? S.kb : S.ka);
        uint32_t *vout = last ? perm : (vin == S.va ? S.vb : S.va);
        hipLaunchKernelGGL((k_radix_scatter<DB, IT>), dim3(tiles), dim3(RADIX_NT), 0, st, n, kin, vin, shift, tiles,
                           S.hist, S.offs, kout, vout, last ? iperm : nullptr);
        kin = kout;
        vin = vout;
    }
    return hipGetLastError();
}

hipError_t particle_order(hipStream_t st, int pos_f32, int64_t n, const void *x, const void *y, const void *z,
                          const double *lo, const double *hi, const int *n0, int levels, void *scratch,
                          size_t scratch_bytes, uint32_t *perm, uint32_t *iperm)
{
    if (n <= 0) return hipSuccess;
    if (n > (int64_t)0x7fffffff || !scratch || scratch_bytes < order_scratch_bytes(n)) return hipErrorInvalidValue;
    const SortGrid G = sort_grid(lo, hi, n0, levels, n);
    const SortScratch S = sort_scratch(n, scratch);
    const bool large = radix_items(n) == ITEMS_LARGE;
    switch (radix_digit(G)) {
    case 6: return large ? sort_passes<6, ITEMS_LARGE>(st, pos_f32, n, x, y, z, G, S, perm, iperm)
                         : sort_passes<6, ITEMS_SMALL>(st, pos_f32, n, x, y, z, G, S, perm, iperm);
    case 7: return large ? sort_passes<7, ITEMS_LARGE>(st, pos_f32, n, x, y, z, G, S, perm, iperm)
                         : sort_passes<7, ITEMS_SMALL>(st, pos_f32, n, x, y, z, G, S, perm, iperm);
    case 8: return large ? sort_passes<8, ITEMS_LARGE>(st, pos_f32, n, x, y, z, G, S, perm, iperm)
                         : sort_passes<8, ITEMS_SMALL>(st, pos_f32, n, x, y, z, G, S, perm, iperm);
    case 9: return large ? sort_passes<9, ITEMS_LARGE>(st, pos_f32, n, x, y, z, G, S, perm, iperm)
                         : sort_passes<9, ITEMS_SMALL>(st, pos_f32, n, x, y, z, G, S, perm, iperm);
    default: return large ? sort_passes<10, ITEMS_LARGE>(st, pos_f32, n, x, y, z, G, S, perm, iperm)
                          : sort_passes<10, ITEMS_SMALL>(st, pos_f32, n, x, y, z, G, S, perm, iperm);
    }
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
