// amrmg_kernels.hip -- HIP kernels for gfx950 of the composite AMR multigrid
// path (arXiv:1812.03689): CIC deposit and gather, charge tagging, the FP64
// composite residual with flux matching (Alg. 1; Eqs. lap_flux_differencing,
// coarse_fluxes, flux_differencing), coarse-fine ghost interpolation (Eq.
// 2d_lagrange, Tab. bit_pattern), smoothers, restriction, prolongation and
// coarse-fine residual update of the V-cycle (Alg. 3), the CG bottom solve,
// average down and E = -grad phi (Alg. 2).
//
// Every stencil kernel works on 8^3 bricks (one workgroup per brick, or four
// bricks per workgroup where a thread owns a coarse cell).  The brick a
// workgroup takes is remapped so that each of the chip's eight XCDs (which
// receive workgroups round robin) walks a contiguous run of bricks and keeps
// neighbouring halos in its own L2.  Arithmetic is FP64; the cycle arrays are
// stored in T (float in mixed precision, double otherwise).
#include <hip/hip_ext.h>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <hip/hip_runtime.h>

#include "amrmg_internal.hpp"
#include "amrmg_kernels.hpp"

namespace amrmg {

// step-1 weights of the coarse-fine ghost, already multiplied by the step-2
// weight 8/15 of the coarse node: [pattern 0..13][quadrant 0..3][node 0..8]
__constant__ double c_cfw[14 * 4 * 9];

// optional kernel-execution timestamps for the next launch (profiling)
static thread_local hipEvent_t g_ev_start = nullptr, g_ev_stop = nullptr;

void set_launch_timing(hipEvent_t start, hipEvent_t stop)
{
    g_ev_start = start;
    g_ev_stop = stop;
}

bool launch_timing_pending() { return g_ev_start != nullptr; }

#define AMRMG_LAUNCH(kernel, grid, block, shmem, stream, ...)                                              \
    do {                                                                                                   \
        if (g_ev_start) {                                                                                  \
            hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, g_ev_start, g_ev_stop, 0, __VA_ARGS__); \
            g_ev_start = g_ev_stop = nullptr;                                                              \
        } else {                                                                                           \
            hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);                           \
        }                                                                                                  \
    } while (0)

hipError_t upload_cf_weights(const double *w)
{
    return hipMemcpyToSymbol(HIP_SYMBOL(c_cfw), w, sizeof(double) * 14 * 4 * 9, 0, hipMemcpyHostToDevice);
}

// workgroup i -> logical index, so that XCD (i mod 8) gets one contiguous run
__device__ __forceinline__ int xcd_remap(int i, int n)
{
    int x = i & 7, q = n >> 3, r = n & 7;
    return x * q + (x < r ? x : r) + (i >> 3);
}

// brick of workgroup i in a range or in an explicit list
__device__ __forceinline__ int pick_brick(int b0, int nb, const int32_t *list, int i)
{
    int k = xcd_remap(i, nb);
    return list ? list[k] : b0 + k;
}

__device__ __forceinline__ int oct_of(int x, int y, int z) { return (x >> 2) | ((y >> 2) << 1) | ((z >> 2) << 2); }

__device__ __forceinline__ void transverse(int d, int &du, int &dv)
{
    du = (d == 0) ? 1 : 0;
    dv = (d == 2) ? 1 : 2;
}

// ---------------------------------------------------------------------------
// accessors: value of local cell l of brick b
// ---------------------------------------------------------------------------
template <class T>
struct BrickAcc {
    const T *u;
    __device__ double operator()(int b, const int *l) const
    {
        return (double)u[(size_t)b * BRICK_CELLS + l[0] + 8 * l[1] + 64 * l[2]];
    }
};

struct OffsetAcc {  // contiguous double slab starting at brick b0
    const double *u;
    int b0;
    __device__ double operator()(int b, const int *l) const
    {
        return u[(size_t)(b - b0) * BRICK_CELLS + l[0] + 8 * l[1] + 64 * l[2]];
    }
};

struct ZeroAcc {
    __device__ double operator()(int, const int *) const { return 0.0; }
};

// The neighbour value that cell l of brick b sees across face (d, s), written
// as a * u_c + bv:
//   same level (in this brick or the face neighbour brick): a = 0, bv = u_nb
//   physical boundary: Dirichlet ghost 2 g - u_c, a = -1, bv = 2 g (g = 0 when
//     !inhom); Robin ghost (central difference of d phi/dn + phi/d = 0),
//     a = (2 d - h)/(2 d + h), bv = 0 (the level's abnd)
//   coarse-fine face, fine side: ghost = cpart + 2/3 u_c - 1/5 u_in, with
//     cpart the coarse part precomputed per ghost (zero when cp == nullptr):
//     a = 2/3, bv = cpart - u_in / 5.
template <class U>
__device__ __forceinline__ void face_nb(const DevMeta &M, int b, const int *lc, int d, int s, const U &u,
                                        const double *cp_d, const float *cp_f, bool inhom, double &a, double &bv)
{
    int l[3] = {lc[0], lc[1], lc[2]};
    int n = l[d] + s;
    if (n >= 0 && n < BRICK) {
        l[d] = n;
        a = 0.0;
        bv = u(b, l);
        return;
    }
    int f = M.nbr[b * 6 + 2 * d + (s > 0)];
    if (f >= 0) {
        l[d] = (s > 0) ? 0 : BRICK - 1;
        a = 0.0;
        bv = u(f, l);
        return;
    }
    int g = -1 - f;
    int du, dv;
    transverse(d, du, dv);
    int t = l[du] + 8 * l[dv];
    if (g < M.nbc) {
        a = M.lc[M.org[b].w].abnd[d];
        bv = inhom ? 2.0 * M.gbc[(size_t)g * 64 + t] : 0.0;
        return;
    }
    size_t cf = (size_t)(g - M.nbc);
    l[d] -= s;  // the fine cell further inside
    double cpv = cp_d ? cp_d[cf * 64 + t] : (cp_f ? (double)cp_f[cf * 64 + t] : 0.0);
    a = 2.0 / 3.0;
    bv = cpv - 0.2 * u(b, l);
}

template <class T>
struct CpPtr;
template <>
struct CpPtr<double> {
    static __device__ const double *d(const double *p) { return p; }
    static __device__ const float *f(const double *) { return nullptr; }
};
template <>
struct CpPtr<float> {
    static __device__ const double *d(const float *) { return nullptr; }
    static __device__ const float *f(const float *p) { return p; }
};

// sum (op 0) or max (op 1) over a workgroup of up to 1024 threads
__device__ double block_reduce(double v, int op)
{
    __shared__ double sh[16];
    for (int o = 32; o > 0; o >>= 1) {
        double w = __shfl_xor(v, o, 64);
        v = op ? fmax(v, w) : v + w;
    }
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = sh[0];
    const int nw = blockDim.x >> 6;
    for (int i = 1; i < nw; ++i) r = op ? fmax(r, sh[i]) : r + sh[i];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------
// LDS tile of one brick: the 8^3 cells plus one halo layer on the six faces
// (edges and corners are never read by the 7-point stencil).  A halo cell
// across a same-level face holds the neighbour's value; across a boundary or
// coarse-fine face it holds bv of the ghost a*u_c + bv, and alpha[face] holds
// a, stored as a - 2 on a boundary face so that its sign tells the kinds
// apart (coarse-fine 2/3 > 0, same level 0, boundary a - 2 < -1 since
// |a| < 1 or a = -1; tile_ab and ghost_shift take the 2 back).  All loads of
// a tile are independent and issued before one barrier.
// ---------------------------------------------------------------------------
constexpr int TE = 10;
__device__ __forceinline__ int tix(int x, int y, int z) { return (x + 1) + TE * ((y + 1) + TE * (z + 1)); }

template <class T>
struct SrcB {  // brick-layout array
    const T *u;
    __device__ double operator()(int b, int c) const { return (double)u[(size_t)b * BRICK_CELLS + c]; }
};
struct SrcZ {
    __device__ double operator()(int, int) const { return 0.0; }
};
// coarse parts of coarse-fine ghosts, by face id and face-local cell
struct CpNone {
    __device__ double operator()(size_t, int) const { return 0.0; }
};
template <class T>
struct CpArr {
    const T *cp;
    __device__ double operator()(size_t cf, int fl) const { return cp ? (double)cp[cf * 64 + fl] : 0.0; }
};
// computed on the spot from the coarse level's cycle array (step 1 of the
// two-step interpolation times 8/15), optionally stored for later sweeps
template <class T>
struct CpInline {
    const DevMeta *M;
    const T *ec;
    T *store;
    __device__ double operator()(size_t cf, int fl) const
    {
        int iu = fl & 7, iv = fl >> 3;
        int m = (iu >> 1) + 4 * (iv >> 1), q = (iu & 1) + 2 * (iv & 1);
        size_t e = cf * 16 + m;
        int pat = M->cf_pat[e];
        const double *W = c_cfw + (pat * 4 + q) * 9;
        double v = 0.0;
        for (int w = 0; w < 9; ++w) v += W[w] * (double)ec[M->cf_idx[e * 9 + w]];
        if (store) store[cf * 64 + fl] = (T)v;
        return v;
    }
};

// NT = threads of the workgroup.  Every load of the tile is issued before the
// first LDS store, so a thread waits for memory once.
template <class S, bool ZERO = false, class CP = CpNone, int NT = 256, class V = double>
__device__ void stage_tile(const DevMeta &M, int b, const S &src, const CP &cp, bool inhom, V *tile, V *alpha)
{
    constexpr int NI = BRICK_CELLS / NT, NH = (384 + NT - 1) / NT;
    double vi[NI], vh[NH], ah[NH];
#pragma unroll
    for (int j = 0; j < NI; ++j) vi[j] = ZERO ? 0.0 : src(b, (int)threadIdx.x + NT * j);
#pragma unroll
    for (int j = 0; j < NH; ++j) {
        const int t = threadIdx.x + NT * j;
        vh[j] = 0.0;
        ah[j] = 0.0;
        if (t >= 384) continue;
        const int f = t >> 6, d = f >> 1;
        const bool plus = f & 1;
        const int fl = t & 63;
        const int nb = M.nbr[b * 6 + f];
        if (nb >= 0) {
            if (!ZERO) {
                int du, dv;
                transverse(d, du, dv);
                int m[3];
                m[du] = fl & 7;
                m[dv] = fl >> 3;
                m[d] = plus ? 0 : 7;
                vh[j] = src(nb, m[0] + 8 * m[1] + 64 * m[2]);
            }
        } else {
            const int g = -1 - nb;
            if (g < M.nbc) {
                ah[j] = M.lc[M.org[b].w].abnd[d] - 2.0;
                vh[j] = inhom ? 2.0 * M.gbc[(size_t)g * 64 + fl] : 0.0;
            } else {
                ah[j] = 2.0 / 3.0;
                vh[j] = cp((size_t)(g - M.nbc), fl);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < NI; ++j) {
        const int c = threadIdx.x + NT * j;
        tile[tix(c & 7, (c >> 3) & 7, c >> 6)] = (V)vi[j];
    }
#pragma unroll
    for (int j = 0; j < NH; ++j) {
        const int t = threadIdx.x + NT * j;
        if (t >= 384) continue;
        const int f = t >> 6, d = f >> 1;
        int du, dv;
        transverse(d, du, dv);
        int l[3];
        l[du] = t & 7;
        l[dv] = (t >> 3) & 7;
        l[d] = (f & 1) ? 8 : -1;
        tile[tix(l[0], l[1], l[2])] = (V)vh[j];
        if ((t & 63) == 0) alpha[f] = (V)ah[j];
    }
    __syncthreads();
}

// Ghost form a * u_c + bv of the neighbour of tile cell (x,y,z) across
// (d, s).  A coarse-fine halo slot holds the coarse part; the -u_in/5 term
// uses the current value of the cell further inside.
template <class V>
__device__ __forceinline__ void tile_ab(const V *tile, const V *alpha, int x, int y, int z, int d, int s, V &a, V &bv)
{
    int l[3] = {x, y, z};
    l[d] += s;
    bv = tile[tix(l[0], l[1], l[2])];
    a = (V)0;
    if (l[d] < 0 || l[d] > 7) {
        a = alpha[2 * d + (s > 0)];
        if (a > (V)0) {
            int in[3] = {x, y, z};
            in[d] -= s;
            bv -= (V)0.2 * tile[tix(in[0], in[1], in[2])];
        } else if (a < (V)0) {
            a += (V)2;  // boundary
        }
    }
}

// ---------------------------------------------------------------------------
// FP64 composite residual (Alg. 1) on a range of bricks of the AMR levels
// ---------------------------------------------------------------------------

// Fine part of the flux through a coarse-fine face, per coarse cell of the
// face: over the four fine cells next to the face, sum (u_f/3 + u_in/5 -
// cpart) with u_in the fine cell further inside and cpart the coarse part of
// the fine cell's ghost; the coarse operator gets -1/(2 h_d^2) times it (the
// flux through the coarse face is the mean of the four fine fluxes).  The
// fine side computes these sums (it holds the fine values) into
// ffs[(F * 6 + face) * 16 + m], F the fine brick, face its face towards the
// coarse cell, m = mu + 4 mv the coarse cell's position on that face; the
// coarse side reads them through the children of its brick and of its face
// neighbours, staged in LDS.

// kids[8 f + o]: child o of face neighbour f of brick b, kids[48 + o]: child
// o of b (-1 where none).  Threads 0..55 load; a barrier must follow.
__device__ __forceinline__ void stage_kids(const DevMeta &M, int b, int *kids)
{
    const int t = threadIdx.x;
    if (t < 48) {
        const int nb = M.nbr[b * 6 + (t >> 3)];
        kids[t] = nb >= 0 ? M.child[nb * 8 + (t & 7)] : -1;
    } else if (t < 56) {
        kids[t] = M.child[b * 8 + (t - 48)];
    }
}

// the fine sum of the face (d, s) of a coarse cell whose neighbour nl (local
// cell of the brick inside, or of face neighbour f) is covered
__device__ __forceinline__ double ffs_at(const double *ffs, const int *kids, bool inside, int f, const int *nl, int d,
                                         int s)
{
    const int o = oct_of(nl[0], nl[1], nl[2]);
    const int F = kids[inside ? 48 + o : 8 * f + o];
    int du, dv;
    transverse(d, du, dv);
    const int m = (nl[du] & 3) + 4 * (nl[dv] & 3);
    return ffs[((size_t)F * 6 + 2 * d + (s < 0)) * 16 + m];
}

// the sum of coarse cell m of face dir of fine brick F from fine values u
// (brick layout) and the coarse parts c[q] of its four fine ghosts (q = the
// fine cell's offsets along the two face axes, first axis fastest)
template <class U>
__device__ __forceinline__ double face_sum(const U &u, int F, int dir, int m, const double *c)
{
    const int d = dir >> 1;
    const bool plus = dir & 1;
    int du, dv;
    transverse(d, du, dv);
    int l[3], li[3];
    l[d] = plus ? 7 : 0;
    li[d] = plus ? 6 : 1;
    double sum = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        l[du] = li[du] = 2 * (m & 3) + (q & 1);
        l[dv] = li[dv] = 2 * (m >> 2) + (q >> 1);
        sum += (1.0 / 3.0) * u(F, l[0] + 8 * l[1] + 64 * l[2]) + 0.2 * u(F, li[0] + 8 * li[1] + 64 * li[2]) - c[q];
    }
    return sum;
}

// The row layout of the sweep and the outer residual: one wavefront per
// brick.  Lane (y, z) = (lane & 7, lane >> 3) owns the brick's x-row (y, z):
// its 8 cells, their right-hand sides and, for x = 0 and x = 7, the x halo
// slots stay in registers, so x-neighbours need no LDS.  The rows of the
// brick and the y and z halo rows sit in LDS, row (y', z') for y', z' in
// -1..8 at rows[((y' + 1) + 10 (z' + 1)) * 9]: rows are 9 words apart, so the
// 64 lanes reading the same x of their neighbouring rows fall in different
// banks.  Row r of the brick starts at cell 8 r of its slab, so the global
// row loads and stores are whole coalesced vectors.  A workgroup holds BPW
// bricks (one per wavefront).
constexpr int RW = 10, RS = 9;
__device__ __forceinline__ int rrow(int y, int z) { return ((y + 1) + RW * (z + 1)) * RS; }

template <class T>
struct Row8;
template <>
struct Row8<float> {
    static __device__ __forceinline__ void load(const float *p, float (&v)[8])
    {
        const float4 a = *(const float4 *)p, b = *(const float4 *)(p + 4);
        v[0] = a.x, v[1] = a.y, v[2] = a.z, v[3] = a.w, v[4] = b.x, v[5] = b.y, v[6] = b.z, v[7] = b.w;
    }
    static __device__ __forceinline__ void store(float *p, const float (&v)[8])
    {
        *(float4 *)p = make_float4(v[0], v[1], v[2], v[3]);
        *(float4 *)(p + 4) = make_float4(v[4], v[5], v[6], v[7]);
    }
};
template <>
struct Row8<double> {
    static __device__ __forceinline__ void load(const double *p, double (&v)[8])
    {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const double2 a = *(const double2 *)(p + 2 * i);
            v[2 * i] = a.x, v[2 * i + 1] = a.y;
        }
    }
    static __device__ __forceinline__ void store(double *p, const double (&v)[8])
    {
#pragma unroll
        for (int i = 0; i < 4; ++i) *(double2 *)(p + 2 * i) = make_double2(v[2 * i], v[2 * i + 1]);
    }
};

// Composite residual r = rho/eps0 - A_comp phi on uncovered cells (zero on
// covered ones) of a range or list of AMR bricks, from FP64 phi and rho in
// brick layout, written as T in brick layout (r_out) and/or FP64 in the
// caller's layout (r_user), with one partial norm per wavefront (part[2 b],
// part[2 b + 1]).  A face towards a covered cell takes the mean of the four
// fine fluxes through it (flux matching), from the fine sums ffs of phi.  Bricks with no covered cell and no
// covered face neighbour (every brick of the finest level) take the plain
// 7-point stencil on the tile, corrected on brick faces whose halo is a
// boundary or coarse-fine ghost.  Two wavefronts per brick, one barrier.
constexpr int RT = 128;

// a u_c + bv - bv_halo for a ghost a u_c + bv whose halo slot holds bv_halo
// (bv = bv_halo - u_in / 5 on a coarse-fine face), from the stored alpha
// (a, or a - 2 on a boundary face)
__device__ __forceinline__ double ghost_shift(double a, double uc, double uin)
{
    return a > 0.0 ? a * uc - 0.2 * uin : (a < 0.0 ? (a + 2.0) * uc : 0.0);
}

// One wavefront per brick, lane (y, z) holding the x-row (y, z) of phi and
// rho in registers and the rows of phi with the y and z halo rows in LDS, as
// the sweep kernel does (rrow); the face kinds and the covered-octant masks
// of the brick and of its face neighbours come through scalar loads.  Each lane writes its row of r and one partial norm per brick
// (part[2 b]; part[2 b + 1] = 0).
template <class T, bool ZERO, int BPW>
__global__ void __launch_bounds__(64 * BPW) k_outer_residual(DevMeta M, int b0, int nb, const double *phib,
                                                             const double *rhob, double inv_eps0,
                                                             const double *cp_phi, T *r_out, double *part, int norm_p,
                                                             const int32_t *list, double *const *r_user,
                                                             const double *ffs)
{
    __shared__ double rows_all[BPW][RW * RW * RS];
    __shared__ int kids_all[BPW][56];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int k0 = xcd_remap(blockIdx.x, (nb + BPW - 1) / BPW) * BPW + w;
    const bool active = k0 < nb;
    const int kk = active ? k0 : nb - 1;
    const int b = __builtin_amdgcn_readfirstlane(list ? list[kk] : b0 + kk);
    double *rows = rows_all[w];
    int *kids = kids_all[w];
    const int y = lane & 7, z = lane >> 3;
    const int lev = M.org[b].w;
    const LevelConst L = M.lc[lev];
    const uint32_t cm = M.cmask[b];
    int nbf[6], kind[6];
    uint32_t ncm[6];
    bool any_cov = cm != 0;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        nbf[f] = M.nbr[b * 6 + f];
        kind[f] = nbf[f] >= 0 ? 0 : ((-1 - nbf[f]) < M.nbc ? 1 : 2);
        ncm[f] = kind[f] == 0 ? (uint32_t)M.cmask[nbf[f]] : 0u;
        any_cov = any_cov || ncm[f] != 0;
    }
    const size_t rb = (size_t)b * BRICK_CELLS + 8 * lane;
    // every cell covered (wavefront-uniform): r = 0, nothing to load; the
    // wavefront still takes part in the workgroup's barrier
    const bool all_cov = cm == 0xffu;
    // the children of the brick and of its face neighbours, for the fine
    // sums of covered faces: kids[8 f + o] of face neighbour f, kids[48 + o]
    // of the brick (-1 where none); read after the barrier below
    if (!ZERO && any_cov && !all_cov && lane < 56) {
        const int nbl = lane < 48 ? M.nbr[b * 6 + (lane >> 3)] : b;
        kids[lane] = nbl >= 0 ? M.child[nbl * 8 + (lane & 7)] : -1;
    }
    double rv[8], u[8], hs[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < 8; ++i) rv[i] = u[i] = 0.0;
    if (!all_cov) {
        Row8<double>::load(rhob + rb, rv);
        if (!ZERO) Row8<double>::load(phib + rb, u);
    }
    // halo slots: the neighbour's phi, 2 g on the boundary (the Dirichlet
    // data enter here), or the coarse part of the coarse-fine ghost
#pragma unroll
    for (int f = 0; f < 6 && !all_cov; ++f) {
        const int d = f >> 1, md = (f & 1) ? 0 : 7;
        const int uu = lane & 7, vv = lane >> 3;
        if (kind[f] == 0) {
            const int c = d == 0 ? md + 8 * uu + 64 * vv : (d == 1 ? uu + 8 * md + 64 * vv : uu + 8 * vv + 64 * md);
            hs[f] = ZERO ? 0.0 : phib[(size_t)nbf[f] * BRICK_CELLS + c];
        } else if (kind[f] == 1) {
            hs[f] = 2.0 * M.gbc[(size_t)(-1 - nbf[f]) * 64 + lane];
        } else {
            hs[f] = (ZERO || !cp_phi) ? 0.0 : cp_phi[(size_t)(-1 - nbf[f] - M.nbc) * 64 + lane];
        }
    }
    const int rym = rrow(y - 1, z), ryp = rrow(y + 1, z), rzm = rrow(y, z - 1), rzp = rrow(y, z + 1), rme = rrow(y, z);
#pragma unroll
    for (int i = 0; i < 8; ++i) rows[rme + i] = u[i];
    rows[rrow(-1, lane >> 3) + (lane & 7)] = hs[2];
    rows[rrow(8, lane >> 3) + (lane & 7)] = hs[3];
    rows[rrow(lane >> 3, -1) + (lane & 7)] = hs[4];
    rows[rrow(lane >> 3, 8) + (lane & 7)] = hs[5];
    // ghost coefficients and the per-row weights (as in the sweep)
    double ag[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) ag[f] = kind[f] == 1 ? L.abnd[f >> 1] : (kind[f] == 2 ? 2.0 / 3.0 : 0.0);
    const double ih2x = L.ih2[0], ih2y = L.ih2[1], ih2z = L.ih2[2];
    const double aym = y == 0 ? ag[2] : 0.0, ayp = y == 7 ? ag[3] : 0.0;
    const double azm = z == 0 ? ag[4] : 0.0, azp = z == 7 ? ag[5] : 0.0;
    const double wyp = (y == 0 && kind[2] == 2) ? 0.8 : 1.0, wym = (y == 7 && kind[3] == 2) ? 0.8 : 1.0;
    const double wzp = (z == 0 && kind[4] == 2) ? 0.8 : 1.0, wzm = (z == 7 && kind[5] == 2) ? 0.8 : 1.0;
    const double wxp0 = kind[0] == 2 ? 0.8 : 1.0, wxm7 = kind[1] == 2 ? 0.8 : 1.0;
    const double den = ih2y * (2.0 - aym - ayp) + ih2z * (2.0 - azm - azp) + 2.0 * ih2x;
    __syncthreads();
    double r[8], acc = 0.0;
#pragma unroll
    for (int x = 0; x < 8; ++x) {
        r[x] = 0.0;
        if (all_cov) continue;
        const double uc = u[x];
        const double xm = x == 0 ? hs[0] : u[x - 1], xp = x == 7 ? hs[1] : u[x + 1];
        const double wxm = x == 7 ? wxm7 : 1.0, wxp = x == 0 ? wxp0 : 1.0;
        const double dc = den - (x == 0 ? ih2x * ag[0] : 0.0) - (x == 7 ? ih2x * ag[1] : 0.0);
        const double ym = rows[rym + x], yp = rows[ryp + x], zm = rows[rzm + x], zp = rows[rzp + x];
        double Au = dc * uc - (ih2x * (wxm * xm + wxp * xp) + ih2y * (wym * ym + wyp * yp) +
                               ih2z * (wzm * zm + wzp * zp));
        const int oc = (x >> 2) | ((y >> 2) << 1) | ((z >> 2) << 2);
        const bool mine_cov = (cm >> oc) & 1;
        if (any_cov && !mine_cov) {
            // a face towards a covered cell of this level: the flux through
            // it is the mean of the four fine fluxes (the fine sums), in
            // place of the same-level term ih2 (u_c - u_nb)
#pragma unroll
            for (int f = 0; f < 6; ++f) {
                const int d = f >> 1, sg = (f & 1) ? 1 : -1;
                const int qx = x + (d == 0 ? sg : 0), qy = y + (d == 1 ? sg : 0), qz = z + (d == 2 ? sg : 0);
                const bool inside = ((qx | qy | qz) & ~7) == 0;
                if (!inside && kind[f] != 0) continue;
                const int lx = qx & 7, ly = qy & 7, lz = qz & 7;
                const int qo = (lx >> 2) | ((ly >> 2) << 1) | ((lz >> 2) << 2);
                if (!(((inside ? cm : ncm[f]) >> qo) & 1)) continue;
                const double unb = d == 0 ? (f & 1 ? xp : xm) : (d == 1 ? (f & 1 ? yp : ym) : (f & 1 ? zp : zm));
                const double ih2 = d == 0 ? ih2x : (d == 1 ? ih2y : ih2z);
                Au -= ih2 * (uc - unb);
                if (!ZERO) {
                    // the child covering that cell: of this brick, or of the face neighbour
                    const int F = kids[inside ? 48 + qo : 8 * f + qo];
                    const int m = d == 0 ? (ly & 3) + 4 * (lz & 3) : (d == 1 ? (lx & 3) + 4 * (lz & 3)
                                                                                 : (lx & 3) + 4 * (ly & 3));
                    Au += -0.5 * ih2 * ffs[((size_t)F * 6 + 2 * d + (sg < 0)) * 16 + m];
                }
            }
        }
        r[x] = mine_cov ? 0.0 : rv[x] * inv_eps0 - Au;
        const double av = fabs(r[x]);
        acc = norm_p == 2 ? acc + av * av : norm_p == 1 ? acc + av : fmax(acc, av);
    }
    if (active) {
        if (r_out) {
            T rt[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) rt[i] = (T)r[i];
            Row8<T>::store(r_out + rb, rt);
        }
        if (r_user) {
            const int2 us = M.ustr[b];
            double *ru = r_user[lev] + M.ubase[b] + (int64_t)us.x * y + (int64_t)us.y * z;
#pragma unroll
            for (int i = 0; i < 8; ++i) ru[i] = r[i];
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double v = __shfl_xor(acc, o, 64);
        acc = norm_p == 0 ? fmax(acc, v) : acc + v;
    }
    if (active && lane == 0) {
        part[2 * (size_t)b] = acc;
        part[2 * (size_t)b + 1] = 0.0;
    }
}

// Copies between the caller's box-list layout and brick layout on a range or
// list of AMR bricks: to_brick: a -> ab and (when set) b -> bb; else ab -> a.
__global__ void __launch_bounds__(256) k_user_brick(DevMeta M, int b0, int nb, const int32_t *list, int to_brick,
                                                    double *const *a, double *ab, double *const *bu, double *bb)
{
    const int b = pick_brick(b0, nb, list, blockIdx.x);
    const int w = M.org[b].w;
    const int64_t ub = M.ubase[b];
    const int2 us = M.ustr[b];
    for (int c = threadIdx.x; c < BRICK_CELLS; c += 256) {
        int64_t ui = ub + (c & 7) + (int64_t)us.x * ((c >> 3) & 7) + (int64_t)us.y * (c >> 6);
        size_t bi = (size_t)b * BRICK_CELLS + c;
        if (to_brick) {
            ab[bi] = a[w][ui];
            if (bb) bb[bi] = bu[w][ui];
        } else {
            a[w][ui] = ab[bi];
        }
    }
}

// Norm of each listed brick range (one AMR level of one problem) from the
// partials (two per brick), in a fixed order, by one workgroup.  The ranges
// go in chunks of NORM_CHUNK: every wavefront sums its share of each range
// of the chunk, then one thread per range adds the 16 wavefront sums (one
// barrier per chunk, not two per range).  With hout set, the norms are also
// written to host-visible memory followed by a sequence number (the device
// counter plus one, read at the start so that its latency overlaps the
// sums), so that the host can poll for them without synchronising the
// stream.  The host copy goes to hout + alt when the counter is odd: two
// publications in a row land in different slots, so the host can still read
// one while the next is being written.
constexpr int NORM_CHUNK = 64;
__global__ void __launch_bounds__(1024) k_level_norms(const int2 *ranges, int n, const double *part, double *out,
                                                      int norm_p, double *hout, int alt, unsigned *hseq,
                                                      unsigned *counter)
{
    __shared__ double sh[16][NORM_CHUNK];
    __shared__ unsigned sseq;
    const bool mx = norm_p == 0;
    const int wave = threadIdx.x >> 6;
    unsigned seq = 0;
    if (hout && threadIdx.x == 0) {
        seq = *counter;
        sseq = seq;
    }
    for (int l0 = 0; l0 < n; l0 += NORM_CHUNK) {
        const int nl = n - l0 < NORM_CHUNK ? n - l0 : NORM_CHUNK;
        for (int j = 0; j < nl; ++j) {
            // the range's partials as pairs (two per brick, 16-byte aligned):
            // pair q of the range to thread q mod 1024, eight pairs in flight
            const int2 rg = ranges[l0 + j];
            const double2 *pp = (const double2 *)part + rg.x;
            const int np = rg.y;
            double a[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) a[u] = 0.0;
            int q = (int)threadIdx.x;
            for (; q + 7 * 1024 < np; q += 8 * 1024) {
                double2 v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = pp[q + u * 1024];
#pragma unroll
                for (int u = 0; u < 8; ++u) a[u] = mx ? fmax(a[u], fmax(v[u].x, v[u].y)) : a[u] + (v[u].x + v[u].y);
            }
            {  // the last fewer than eight pairs of this thread, also in flight together (partials are >= 0)
                double2 v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = q + u * 1024 < np ? pp[q + u * 1024] : make_double2(0.0, 0.0);
#pragma unroll
                for (int u = 0; u < 8; ++u) a[u] = mx ? fmax(a[u], fmax(v[u].x, v[u].y)) : a[u] + (v[u].x + v[u].y);
            }
            double acc = mx ? fmax(fmax(fmax(a[0], a[1]), fmax(a[2], a[3])), fmax(fmax(a[4], a[5]), fmax(a[6], a[7])))
                            : ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
            for (int o = 32; o > 0; o >>= 1) {
                double w = __shfl_xor(acc, o, 64);
                acc = mx ? fmax(acc, w) : acc + w;
            }
            if ((threadIdx.x & 63) == 0) sh[wave][j] = acc;
        }
        __syncthreads();
        if ((int)threadIdx.x < nl) {
            const int j = threadIdx.x;
            double r = sh[0][j];
            for (int i = 1; i < 16; ++i) r = mx ? fmax(r, sh[i][j]) : r + sh[i][j];
            r = norm_p == 2 ? sqrt(r) : r;
            out[l0 + j] = r;
            if (hout) {
                hout[(sseq & 1u) * alt + l0 + j] = r;
                __threadfence_system();
            }
        }
        __syncthreads();
    }
    if (hout && threadIdx.x == 0) {
        __threadfence_system();
        *counter = seq + 1;
        *(volatile unsigned *)hseq = seq + 1;
    }
}

// ---------------------------------------------------------------------------
// coarse parts of the coarse-fine ghosts (step 1 of Eq. 2d_lagrange, times
// the step-2 weight 8/15)
// ---------------------------------------------------------------------------
template <class T>
struct SrcBrick {
    const T *u;
    __device__ double operator()(int32_t g) const { return (double)u[g]; }
};

template <class T, class S>
__global__ void __launch_bounds__(256) k_cpart(DevMeta M, int cf0, int ncf, S src, T *cp, const T *fine,
                                               double *ffs)
{
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= ncf * 16) return;
    int cf = cf0 + (i >> 4), m = i & 15;
    size_t e = (size_t)cf * 16 + m;
    const int ow = ffs ? M.gf_owner[M.nbc + cf] : 0;
    int pat = M.cf_pat[e];
    double v[9];
    for (int w = 0; w < 9; ++w) v[w] = src(M.cf_idx[e * 9 + w]);
    int mu = m & 3, mv = m >> 2;
    double c[4];
    for (int q = 0; q < 4; ++q) {
        const double *W = c_cfw + (pat * 4 + q) * 9;
        double s = 0.0;
        for (int w = 0; w < 9; ++w) s += W[w] * v[w];
        int t = (2 * mu + (q & 1)) + 8 * (2 * mv + (q >> 1));
        cp[(size_t)cf * 64 + t] = (T)s;
        c[q] = (double)(T)s;
    }
    // with ffs: the fine sum of this coarse cell from the fine values and these coarse parts
    if (ffs) ffs[((size_t)(ow >> 3) * 6 + (ow & 7)) * 16 + m] = face_sum(SrcB<T>{fine}, ow >> 3, ow & 7, m, c);
}

// fine sums (zero coarse parts) of the coarse-fine faces [cf0, cf0 + ncf) from e
template <class T>
__global__ void __launch_bounds__(256) k_face_sums(DevMeta M, int cf0, int ncf, const T *e, double *ffs)
{
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= ncf * 16) return;
    const int ow = M.gf_owner[M.nbc + cf0 + (i >> 4)], m = i & 15;
    const double c[4] = {0.0, 0.0, 0.0, 0.0};
    ffs[((size_t)(ow >> 3) * 6 + (ow & 7)) * 16 + m] = face_sum(SrcB<T>{e}, ow >> 3, ow & 7, m, c);
}

// ---------------------------------------------------------------------------
// V-cycle kernels on the correction equation (Alg. 3)
// ---------------------------------------------------------------------------

// Gauss-Seidel red-black, one colour: cells with (i+j+k) mod 2 == colour in
// level indices.  Each of the 256 threads owns one cell of that colour.
// init: e is undefined and taken as zero; the other colour is written 0.
template <class T>
__global__ void __launch_bounds__(256) k_gsrb(DevMeta M, int b0, int nb, T *e, const T *r, const T *cp,
                                              int colour, int init)
{
    __shared__ double tile[TE * TE * TE];
    __shared__ double alpha[6];
    int b = b0 + xcd_remap(blockIdx.x, nb);
    int lev = M.org[b].w;
    LevelConst L = M.lc[lev];
    int t = threadIdx.x;
    int z = t >> 5, y = (t >> 2) & 7, xx = (t & 3) << 1;
    int x = xx + (((y + z) & 1) ^ colour);  // brick origins are even
    size_t li = (size_t)b * BRICK_CELLS + x + 8 * y + 64 * z;
    double rv = (double)r[li];
    if (init)
        stage_tile<SrcZ, true>(M, b, SrcZ{}, CpNone{}, false, tile, alpha);
    else
        stage_tile<SrcB<T>, false, CpArr<T>>(M, b, SrcB<T>{e}, CpArr<T>{cp}, false, tile, alpha);
    double num = rv, den = 0.0;
    for (int d = 0; d < 3; ++d)
        for (int s = -1; s <= 1; s += 2) {
            double a, bv;
            tile_ab(tile, alpha, x, y, z, d, s, a, bv);
            num += L.ih2[d] * bv;
            den += L.ih2[d] * (1.0 - a);
        }
    e[li] = (T)(num / den);
    if (init) e[li ^ 1] = (T)0;
}

// damped Jacobi sweep: eout = ein + omega (D^-1 (r - (A - D) ein) - ein)
template <class T>
__global__ void __launch_bounds__(256) k_jacobi(DevMeta M, int b0, int nb, const T *ein, T *eout, const T *r,
                                                const T *cp, double omega, int init)
{
    __shared__ double tile[TE * TE * TE];
    __shared__ double alpha[6];
    int b = b0 + xcd_remap(blockIdx.x, nb);
    int lev = M.org[b].w;
    LevelConst L = M.lc[lev];
    double rv[2];
    for (int k = 0; k < 2; ++k) rv[k] = (double)r[(size_t)b * BRICK_CELLS + threadIdx.x + 256 * k];
    if (init)
        stage_tile<SrcZ, true>(M, b, SrcZ{}, CpNone{}, false, tile, alpha);
    else
        stage_tile<SrcB<T>, false, CpArr<T>>(M, b, SrcB<T>{ein}, CpArr<T>{cp}, false, tile, alpha);
    for (int k = 0; k < 2; ++k) {
        int c = threadIdx.x + 256 * k;
        int x = c & 7, y = (c >> 3) & 7, z = c >> 6;
        double num = rv[k], den = 0.0;
        for (int d = 0; d < 3; ++d)
            for (int s = -1; s <= 1; s += 2) {
                double a, bv;
                tile_ab(tile, alpha, x, y, z, d, s, a, bv);
                num += L.ih2[d] * bv;
                den += L.ih2[d] * (1.0 - a);
            }
        double uc = tile[tix(x, y, z)];
        eout[(size_t)b * BRICK_CELLS + c] = (T)(uc + omega * (num / den - uc));
    }
}

// cycle array plus the injected parent value (prolongation I e^{l-1})
template <class T>
struct SrcProl {
    const T *u;
    const int32_t *par;
    __device__ double operator()(int b, int c) const
    {
        int p = par[b];
        int pb = p >> 3, oc = p & 7;
        int x = c & 7, y = (c >> 3) & 7, z = c >> 6;
        int pc = ((oc & 1) * 4 + (x >> 1)) + 8 * (((oc >> 1) & 1) * 4 + (y >> 1)) + 64 * ((oc >> 2) * 4 + (z >> 1));
        return (double)u[(size_t)b * BRICK_CELLS + c] + (double)u[(size_t)pb * BRICK_CELLS + pc];
    }
};

// Brick-hybrid Gauss-Seidel sweep: red then black over the cells of one
// brick in LDS, with the halo taken from the previous sweep (Gauss-Seidel
// inside a brick, Jacobi between bricks, as a parallel Gauss-Seidel works
// inside and between subdomains).  Reads ein, writes eout.
// MODE bits: 1 input is zero; 2 input plus the parent correction (fused
// prolongation); 4 coarse parts of the coarse-fine ghosts computed from the
// coarse level's values in ein and stored into cp (else read from cp);
// 8 phi += result on AMR bricks (fused phi update; phi in brick layout);
// 16 the fine sums of the result on the brick's coarse-fine faces into ffs.
enum { HG_ZERO = 1, HG_PROL = 2, HG_CPIN = 4, HG_PHI = 8, HG_FFS = 16 };

// face_sum of a brick held in the row layout with zero coarse parts: over the
// four fine cells of coarse cell m of face f, u_f/3 + u_in/5 (u_in the cell
// further inside along the face normal)
template <class T>
__device__ __forceinline__ double row_face_sum(const T *rows, int f, int m)
{
    const int d = f >> 1, at = (f & 1) ? 7 : 0, in = (f & 1) ? 6 : 1;
    double sum = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int u = 2 * (m & 3) + (q & 1), v = 2 * (m >> 2) + (q >> 1);
        // (x, y, z) of the face cell and of the cell inside, for the normal d
        // with u, v along the two other axes in x < y < z order
        const int x0 = d == 0 ? at : u, y0 = d == 1 ? at : (d == 0 ? u : v), z0 = d == 2 ? at : v;
        const int x1 = d == 0 ? in : u, y1 = d == 1 ? in : (d == 0 ? u : v), z1 = d == 2 ? in : v;
        sum += (1.0 / 3.0) * (double)rows[rrow(y0, z0) + x0] + 0.2 * (double)rows[rrow(y1, z1) + x1];
    }
    return sum;
}

// parent cell of local cell (x, y, z) of a brick whose parent entry is p
// (parent brick << 3 | octant), as a cell index of the parent's slab
__device__ __forceinline__ size_t parent_cell(int p, int x, int y, int z)
{
    const int oc = p & 7;
    return (size_t)(p >> 3) * BRICK_CELLS + ((oc & 1) * 4 + (x >> 1)) + 8 * (((oc >> 1) & 1) * 4 + (y >> 1)) +
           64 * ((oc >> 2) * 4 + (z >> 1));
}

// Lane-wise choice of a (lane's bit of m clear) or b (set), m a wavefront
// mask from a ballot, as v_cndmask in asm: a choice between two elements of
// a register array written as C++ is rewritten by the compiler into one
// access at a computed index, which moves the array into private memory.
__device__ __forceinline__ float lane_pick(uint64_t m, float a, float b)
{
    float r;
    asm("v_cndmask_b32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(m));
    return r;
}
__device__ __forceinline__ double lane_pick(uint64_t m, double a, double b)
{
    const uint64_t ia = (uint64_t)__double_as_longlong(a), ib = (uint64_t)__double_as_longlong(b);
    uint32_t lo, hi;
    asm("v_cndmask_b32 %0, %1, %2, %3" : "=v"(lo) : "v"((uint32_t)ia), "v"((uint32_t)ib), "s"(m));
    asm("v_cndmask_b32 %0, %1, %2, %3" : "=v"(hi) : "v"((uint32_t)(ia >> 32)), "v"((uint32_t)(ib >> 32)), "s"(m));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

template <class T, int MODE, int BPW>
__global__ void __launch_bounds__(64 * BPW) k_hgs(DevMeta M, int b0, int nb, const T *ein, T *eout, const T *r,
                                                  T *cp, double *phib, double *ffs)
{
    __shared__ T rows_all[BPW][RW * RW * RS];
    // the wavefront's brick, wavefront-uniform (so its table entries come
    // through scalar loads and the face kinds branch on the scalar unit)
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int k0 = xcd_remap(blockIdx.x, (nb + BPW - 1) / BPW) * BPW + w;
    const bool active = k0 < nb;  // the last workgroup may hold fewer bricks
    const int b = __builtin_amdgcn_readfirstlane(b0 + (active ? k0 : nb - 1));
    T *rows = rows_all[w];
    const int y = lane & 7, z = lane >> 3;
    // face kinds: 0 a brick of the level, 1 the physical boundary (ghost
    // abnd u_c), 2 coarse-fine (ghost 2/3 u_c + cp - u_in/5)
    int nbf[6], kind[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        nbf[f] = M.nbr[b * 6 + f];
        kind[f] = nbf[f] >= 0 ? 0 : ((-1 - nbf[f]) < M.nbc ? 1 : 2);
    }
    // the value of cell c of brick bb as this sweep starts from it (input,
    // plus the injected parent correction with the fused prolongation)
    auto src = [&](int bb, int c) -> T {
        if (MODE & HG_ZERO) return (T)0;
        double v = (double)ein[(size_t)bb * BRICK_CELLS + c];
        if (MODE & HG_PROL) v += (double)ein[parent_cell(M.par[bb], c & 7, (c >> 3) & 7, c >> 6)];
        return (T)v;
    };
    // halo slot of face f at face-local cell fl (first transverse axis
    // fastest): the neighbour's value, 0 on the boundary (homogeneous cycle),
    // or the coarse part of the coarse-fine ghost
    auto slot = [&](int f, int fl) -> T {
        const int d = f >> 1, md = (f & 1) ? 0 : 7;
        if (kind[f] == 0) {
            const int u = fl & 7, v = fl >> 3;
            const int c = d == 0 ? md + 8 * u + 64 * v : (d == 1 ? u + 8 * md + 64 * v : u + 8 * v + 64 * md);
            return src(nbf[f], c);
        }
        if (kind[f] == 1 || (MODE & HG_ZERO)) return (T)0;
        const size_t cf = (size_t)(-1 - nbf[f] - M.nbc);
        if (MODE & HG_CPIN) return (T)CpInline<T>{&M, ein, active ? cp : nullptr}(cf, fl);
        return cp ? cp[cf * 64 + fl] : (T)0;
    };
    // every load first: right-hand sides, input, halo slots
    const size_t rb = (size_t)b * BRICK_CELLS + 8 * lane;
    T rr[8], er[8], hs[6];
    Row8<T>::load(r + rb, rr);
    if (MODE & HG_ZERO) {
#pragma unroll
        for (int i = 0; i < 8; ++i) er[i] = (T)0;
    } else {
        Row8<T>::load(ein + rb, er);
    }
    if (MODE & HG_PROL) {
        const size_t pc = parent_cell(M.par[b], 0, y, z);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const T pv = ein[pc + k];
            er[2 * k] = (T)((double)er[2 * k] + (double)pv);
            er[2 * k + 1] = (T)((double)er[2 * k + 1] + (double)pv);
        }
    }
    // x-neighbours held by the previous or the next wavefront of the
    // workgroup (bricks are numbered x-fastest within a box): their starting
    // values are the rows those wavefronts put in LDS, read from there below
    // instead of from memory
    const bool lx_m = BPW > 1 && w > 0 && kind[0] == 0 && nbf[0] == b - 1;
    const bool lx_p = BPW > 1 && w + 1 < BPW && k0 + 1 < nb && kind[1] == 0 && nbf[1] == b + 1;
#pragma unroll
    for (int f = 0; f < 6; ++f) hs[f] = (f == 0 && lx_m) || (f == 1 && lx_p) ? (T)0 : slot(f, lane);
    const LevelConst L = M.lc[M.org[b].w];
    const T ih2x = (T)L.ih2[0], ih2y = (T)L.ih2[1], ih2z = (T)L.ih2[2];
    const int rym = rrow(y - 1, z), ryp = rrow(y + 1, z), rzm = rrow(y, z - 1), rzp = rrow(y, z + 1), rme = rrow(y, z);
#pragma unroll
    for (int i = 0; i < 8; ++i) rows[rme + i] = er[i];
    // y halo rows: face-local cell (x, z); z halo rows: (x, y)
    rows[rrow(-1, lane >> 3) + (lane & 7)] = hs[2];
    rows[rrow(8, lane >> 3) + (lane & 7)] = hs[3];
    rows[rrow(lane >> 3, -1) + (lane & 7)] = hs[4];
    rows[rrow(lane >> 3, 8) + (lane & 7)] = hs[5];
    T hxm = hs[0], hxp = hs[1];
    // ghost coefficients a of the faces, and per row the weights that fold a
    // coarse-fine ghost's -u_in/5 into the neighbour inside
    const T cf5 = (T)0.2;
    T ag[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) ag[f] = kind[f] == 1 ? (T)L.abnd[f >> 1] : (kind[f] == 2 ? (T)(2.0 / 3.0) : (T)0);
    const T aym = y == 0 ? ag[2] : (T)0, ayp = y == 7 ? ag[3] : (T)0;
    const T azm = z == 0 ? ag[4] : (T)0, azp = z == 7 ? ag[5] : (T)0;
    const T wyp = (y == 0 && kind[2] == 2) ? (T)1 - cf5 : (T)1, wym = (y == 7 && kind[3] == 2) ? (T)1 - cf5 : (T)1;
    const T wzp = (z == 0 && kind[4] == 2) ? (T)1 - cf5 : (T)1, wzm = (z == 7 && kind[5] == 2) ? (T)1 - cf5 : (T)1;
    const T wxp0 = kind[0] == 2 ? (T)1 - cf5 : (T)1, wxm7 = kind[1] == 2 ? (T)1 - cf5 : (T)1;
    const T den = ih2y * ((T)2 - aym - ayp) + ih2z * ((T)2 - azm - azp) + (T)2 * ih2x;
    const T inv_mid = (T)1 / den, inv_x0 = (T)1 / (den - ih2x * ag[0]), inv_x7 = (T)1 / (den - ih2x * ag[1]);
    __syncthreads();
    if (BPW > 1) {
        // the neighbours' rows are read before any wavefront starts updating its own
        if (lx_m) hxm = rows_all[w - 1][rme + 7];
        if (lx_p) hxp = rows_all[w + 1][rme];
        __syncthreads();
    }
    // red (colour 0) then black: cell x of row (y, z) has colour (x + y + z)
    // & 1, so in each pair of cells (2k, 2k + 1) of the row exactly one
    // takes part in a pass, the one at x = 2k + p with p = (y + z + pass) &
    // 1.  Its operands are chosen from the row's registers by selects
    // between fixed elements (a lane-dependent register index would be
    // turned into an indexed access to private memory); its LDS neighbours
    // are read at the lane's own offset.
    const int q = (y + z) & 1;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const bool p = ((q + c) & 1) != 0;
        const uint64_t pm = __builtin_amdgcn_ballot_w64(p);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int x = 2 * k + (p ? 1 : 0);
            const T xm = lane_pick(pm, k == 0 ? hxm : er[2 * k - 1], er[2 * k]);
            const T xp = lane_pick(pm, er[2 * k + 1], k == 3 ? hxp : er[2 * k + 2]);
            const T rx = lane_pick(pm, rr[2 * k], rr[2 * k + 1]);
            const T wxm = k == 3 ? lane_pick(pm, (T)1, wxm7) : (T)1;
            const T wxp = k == 0 ? lane_pick(pm, wxp0, (T)1) : (T)1;
            const T inv = k == 0 ? lane_pick(pm, inv_x0, inv_mid) : (k == 3 ? lane_pick(pm, inv_mid, inv_x7) : inv_mid);
            const T num = rx + ih2x * (wxm * xm + wxp * xp) +
                          ih2y * (wym * rows[rym + x] + wyp * rows[ryp + x]) +
                          ih2z * (wzm * rows[rzm + x] + wzp * rows[rzp + x]);
            const T nv = num * inv;
            er[2 * k] = p ? er[2 * k] : nv;
            er[2 * k + 1] = p ? nv : er[2 * k + 1];
            rows[rme + x] = nv;
        }
        __syncthreads();
    }
    if (!active) return;
    Row8<T>::store(eout + rb, er);
    if ((MODE & HG_PHI) && L.amr >= 0) {
        double ph[8];
        Row8<double>::load(phib + rb, ph);
#pragma unroll
        for (int i = 0; i < 8; ++i) ph[i] += (double)er[i];
        Row8<double>::store(phib + rb, ph);
    }
    // fine sums of the new e on the brick's coarse-fine faces (the coarse
    // correction, and so the ghosts' coarse parts, are zero at the
    // restriction that reads them)
    if (MODE & HG_FFS) {
        for (int t = lane; t < 96; t += 64) {
            const int f = t >> 4;
            if (kind[f] == 2) ffs[((size_t)b * 6 + f) * 16 + (t & 15)] = row_face_sum(rows, f, t & 15);
        }
    }
}

// residual of the homogeneous problem at one cell: r - A e (zero coarse data)
template <class T>
__device__ __forceinline__ double cell_residual(const DevMeta &M, const LevelConst &L, int b, const int *lc,
                                                const T *e, const T *r)
{
    size_t li = (size_t)b * BRICK_CELLS + lc[0] + 8 * lc[1] + 64 * lc[2];
    double uc = (double)e[li], Au = 0.0;
    for (int d = 0; d < 3; ++d)
        for (int s = -1; s <= 1; s += 2) {
            double a, bv;
            face_nb(M, b, lc, d, s, BrickAcc<T>{e}, nullptr, nullptr, false, a, bv);
            Au += L.ih2[d] * ((1.0 - a) * uc - bv);
        }
    return (double)r[li] - Au;
}

// r^{l-1} on covered cells = mean over the 8 children of (r^l - A_nf e^l)
// (Alg. 3, restriction onto the covered domain; e^{l-1} = 0 at that point,
// so the coarse parts of the coarse-fine ghosts are zero).  One wavefront
// per fine brick in the row layout: lane (y, z) computes the residual of its
// row, adds x pairs, then the y and z pairs of the lanes 1 and 8 apart; the
// lanes with even y and z write four coarse cells of their parent's row.
template <class T>
__device__ __forceinline__ void restrict_brick(const DevMeta &M, int b, bool active, const T *e, T *r, T *rows)
{
    const int lane = threadIdx.x & 63, y = lane & 7, z = lane >> 3;
    const LevelConst L = M.lc[M.org[b].w];
    int nbf[6], kind[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        nbf[f] = M.nbr[b * 6 + f];
        kind[f] = nbf[f] >= 0 ? 0 : ((-1 - nbf[f]) < M.nbc ? 1 : 2);
    }
    const size_t rb = (size_t)b * BRICK_CELLS + 8 * lane;
    T rr[8], u[8], hs[6];
    Row8<T>::load(r + rb, rr);
    Row8<T>::load(e + rb, u);
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        const int d = f >> 1, md = (f & 1) ? 0 : 7, uu = lane & 7, vv = lane >> 3;
        const int c = d == 0 ? md + 8 * uu + 64 * vv : (d == 1 ? uu + 8 * md + 64 * vv : uu + 8 * vv + 64 * md);
        hs[f] = kind[f] == 0 ? e[(size_t)nbf[f] * BRICK_CELLS + c] : (T)0;
    }
    const int rym = rrow(y - 1, z), ryp = rrow(y + 1, z), rzm = rrow(y, z - 1), rzp = rrow(y, z + 1), rme = rrow(y, z);
#pragma unroll
    for (int i = 0; i < 8; ++i) rows[rme + i] = u[i];
    rows[rrow(-1, lane >> 3) + (lane & 7)] = hs[2];
    rows[rrow(8, lane >> 3) + (lane & 7)] = hs[3];
    rows[rrow(lane >> 3, -1) + (lane & 7)] = hs[4];
    rows[rrow(lane >> 3, 8) + (lane & 7)] = hs[5];
    T ag[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) ag[f] = kind[f] == 1 ? (T)L.abnd[f >> 1] : (kind[f] == 2 ? (T)(2.0 / 3.0) : (T)0);
    const T ih2x = (T)L.ih2[0], ih2y = (T)L.ih2[1], ih2z = (T)L.ih2[2], cf5 = (T)0.2;
    const T aym = y == 0 ? ag[2] : (T)0, ayp = y == 7 ? ag[3] : (T)0;
    const T azm = z == 0 ? ag[4] : (T)0, azp = z == 7 ? ag[5] : (T)0;
    const T wyp = (y == 0 && kind[2] == 2) ? (T)1 - cf5 : (T)1, wym = (y == 7 && kind[3] == 2) ? (T)1 - cf5 : (T)1;
    const T wzp = (z == 0 && kind[4] == 2) ? (T)1 - cf5 : (T)1, wzm = (z == 7 && kind[5] == 2) ? (T)1 - cf5 : (T)1;
    const T wxp0 = kind[0] == 2 ? (T)1 - cf5 : (T)1, wxm7 = kind[1] == 2 ? (T)1 - cf5 : (T)1;
    const T den = ih2y * ((T)2 - aym - ayp) + ih2z * ((T)2 - azm - azp) + (T)2 * ih2x;
    __syncthreads();
    T s4[4];
#pragma unroll
    for (int cx = 0; cx < 4; ++cx) {
        T pair = (T)0;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int x = 2 * cx + q;
            const T xm = x == 0 ? hs[0] : u[x - 1], xp = x == 7 ? hs[1] : u[x + 1];
            const T wxm = x == 7 ? wxm7 : (T)1, wxp = x == 0 ? wxp0 : (T)1;
            const T dc = den - (x == 0 ? ih2x * ag[0] : (T)0) - (x == 7 ? ih2x * ag[1] : (T)0);
            const T Au = dc * u[x] - (ih2x * (wxm * xm + wxp * xp) + ih2y * (wym * rows[rym + x] + wyp * rows[ryp + x]) +
                                      ih2z * (wzm * rows[rzm + x] + wzp * rows[rzp + x]));
            pair += rr[x] - Au;
        }
        pair += __shfl_xor(pair, 1, 64);
        pair += __shfl_xor(pair, 8, 64);
        s4[cx] = (T)0.125 * pair;
    }
    if (active && !(y & 1) && !(z & 1)) {
        const int p = M.par[b], oc = p & 7;
        const int Y = ((oc >> 1) & 1) * 4 + (y >> 1), Z = (oc >> 2) * 4 + (z >> 1);
        T *dst = r + (size_t)(p >> 3) * BRICK_CELLS + (oc & 1) * 4 + 8 * Y + 64 * Z;
#pragma unroll
        for (int cx = 0; cx < 4; ++cx) dst[cx] = s4[cx];
    }
}

// Uncovered coarse cells next to covered ones: r -= B_fine e^l, i.e. add
// 1/(2 h_d^2) * sum over the 4 fine faces of (e_f/3 + e_in/5) per coarse-fine
// face (the coarse correction is still zero), from the fine sums ffs of e.
// FP64 arithmetic.
template <class T>
__device__ __forceinline__ void reflux_brick(const DevMeta &M, int b, const double *ffs, T *r, int *kids,
                                             uint8_t *ncm)
{
    const LevelConst L = M.lc[M.org[b].w];
    const uint8_t cm = M.cmask[b];
    if (threadIdx.x < 6) {
        int f = M.nbr[b * 6 + threadIdx.x];
        ncm[threadIdx.x] = f >= 0 ? M.cmask[f] : 0;
    }
    stage_kids(M, b, kids);
    __syncthreads();
    for (int c = threadIdx.x; c < BRICK_CELLS; c += blockDim.x) {
        const int x = c & 7, y = (c >> 3) & 7, z = c >> 6;
        if ((cm >> oct_of(x, y, z)) & 1) continue;
        double add = 0.0;
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            const int d = f >> 1, s = (f & 1) ? 1 : -1;
            int qx = x + (d == 0 ? s : 0), qy = y + (d == 1 ? s : 0), qz = z + (d == 2 ? s : 0);
            bool inside = ((qx | qy | qz) & ~7) == 0;
            bool cov = ((inside ? cm : ncm[f]) >> oct_of(qx & 7, qy & 7, qz & 7)) & 1;
            if (cov) {
                const int nl[3] = {qx & 7, qy & 7, qz & 7};
                add += 0.5 * L.ih2[d] * ffs_at(ffs, kids, inside, f, nl, d, s);
            }
        }
        if (add != 0.0) {
            size_t li = (size_t)b * BRICK_CELLS + c;
            r[li] = (T)((double)r[li] + add);
        }
    }
}

// One launch per level step: the restriction of the nb fine bricks from b0
// into their parents (covered coarse cells), then the coarse-fine update of
// the nrf listed coarse bricks (uncovered cells) -- disjoint cells, so the
// two kinds of workgroups run together.
// Workgroups of 128 threads: the first (nb + 1) / 2 restrict two fine bricks
// each (one per wavefront), the others update one listed coarse brick each.
template <class T>
__global__ void __launch_bounds__(128) k_restrict(DevMeta M, int b0, int nb, const int32_t *rlist, int nrf,
                                                  const T *e, T *r, const double *ffs)
{
    __shared__ T rows[2][RW * RW * RS];
    __shared__ int kids[56];
    __shared__ uint8_t ncm[6];
    const int nwr = (nb + 1) / 2;
    if ((int)blockIdx.x < nwr) {
        const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        const int k = xcd_remap(blockIdx.x, nwr) * 2 + w;
        restrict_brick<T>(M, __builtin_amdgcn_readfirstlane(b0 + (k < nb ? k : nb - 1)), k < nb, e, r, rows[w]);
    } else {
        reflux_brick<T>(M, rlist[xcd_remap(blockIdx.x - nwr, nrf)], ffs, r, kids, ncm);
    }
}

// e^l += I e^{l-1}: piecewise-constant injection of the parent value
template <class T>
__global__ void __launch_bounds__(256) k_prolong(DevMeta M, int b0, int nb, T *e)
{
    int b = b0 + xcd_remap(blockIdx.x, nb);
    int par = M.par[b];
    int pb = par >> 3, oc = par & 7;
    int ox = (oc & 1) * 4, oy = ((oc >> 1) & 1) * 4, oz = (oc >> 2) * 4;
    for (int c = threadIdx.x; c < BRICK_CELLS; c += 256) {
        int x = c & 7, y = (c >> 3) & 7, z = c >> 6;
        size_t li = (size_t)b * BRICK_CELLS + c;
        size_t pi = (size_t)pb * BRICK_CELLS + (ox + (x >> 1)) + 8 * (oy + (y >> 1)) + 64 * (oz + (z >> 1));
        e[li] = (T)((double)e[li] + (double)e[pi]);
    }
}

// phi += e on AMR bricks (FP64 accumulation of the correction; brick layout)
template <class T>
__global__ void __launch_bounds__(256) k_phi_update(DevMeta M, int b0, int nb, double *phib, const T *e,
                                                    const int32_t *list)
{
    int b = pick_brick(b0, nb, list, blockIdx.x);
    for (int c = threadIdx.x; c < BRICK_CELLS; c += 256) {
        size_t i = (size_t)b * BRICK_CELLS + c;
        phib[i] += (double)e[i];
    }
}

// phi^{l} <- U phi^l + R phi^{l+1} for the covered cells under a range of
// fine bricks (Alg. 2, average down; brick layout)
__global__ void __launch_bounds__(256) k_avgdown(DevMeta M, int b0, int nb, double *phib)
{
    int nwg = (nb + 3) >> 2;
    int w = xcd_remap(blockIdx.x, nwg);
    int k = w * 4 + (threadIdx.x >> 6);
    if (k >= nb) return;
    int b = b0 + k;
    int t = threadIdx.x & 63;
    int cx = t & 3, cy = (t >> 2) & 3, cz = t >> 4;
    const double *u = phib + (size_t)b * BRICK_CELLS;
    double s = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) s += u[(2 * cx + dx) + 8 * (2 * cy + dy) + 64 * (2 * cz + dz)];
    int par = M.par[b];
    int pb = par >> 3, oc = par & 7;
    int X = (oc & 1) * 4 + cx, Y = ((oc >> 1) & 1) * 4 + cy, Z = (oc >> 2) * 4 + cz;
    phib[(size_t)pb * BRICK_CELLS + X + 8 * Y + 64 * Z] = 0.125 * s;
}

// E_d = -(u_+ - u_-) / (2 h_d) on every cell of a range of AMR bricks (phi in
// brick layout, E in the caller's layout)
__global__ void __launch_bounds__(256) k_efield(DevMeta M, int b0, int nb, const double *phib, const double *cp_phi,
                                                double *const *E, const int32_t *list)
{
    __shared__ double tile[TE * TE * TE];
    __shared__ double alpha[6];
    int b = pick_brick(b0, nb, list, blockIdx.x);
    int lev = M.org[b].w;
    LevelConst L = M.lc[lev];
    stage_tile<SrcB<double>, false, CpArr<double>>(M, b, SrcB<double>{phib}, CpArr<double>{cp_phi}, true, tile,
                                                   alpha);
    int64_t ub = M.ubase[b];
    int2 us = M.ustr[b];
    for (int c = threadIdx.x; c < BRICK_CELLS; c += 256) {
        int x = c & 7, y = (c >> 3) & 7, z = c >> 6;
        int64_t ui = ub + x + (int64_t)us.x * y + (int64_t)us.y * z;
        double uc = tile[tix(x, y, z)];
        for (int d = 0; d < 3; ++d) {
            double a, bv;
            tile_ab(tile, alpha, x, y, z, d, +1, a, bv);
            double up = a * uc + bv;
            tile_ab(tile, alpha, x, y, z, d, -1, a, bv);
            double um = a * uc + bv;
            E[3 * lev + d][ui] = -(up - um) / (2.0 * L.h[d]);
        }
    }
}

// ---------------------------------------------------------------------------
// CG on the coarsest grid, one workgroup of 1024 threads (FP64 vectors and
// dot products).  Homogeneous boundary data, no coarse-fine faces.
// ---------------------------------------------------------------------------
__device__ double block_reduce_1024(double v)
{
    __shared__ double sh[16];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    const int nw = blockDim.x >> 6;
    for (int i = 0; i < nw; ++i) r += sh[i];
    __syncthreads();
    return r;
}

// CG on bricks [b0, b0+nb) of one level with four FP64 work vectors; called
// by a whole workgroup of 1024 threads.  Returns the iteration count.
template <class T>
__device__ int cg_solve(const DevMeta &M, int b0, int nb, const T *rhs, T *e, double *work, double rtol, int maxit)
{
    const int n = nb * BRICK_CELLS;
    double *x = work, *r = x + n, *p = x + 2 * (size_t)n, *q = x + 3 * (size_t)n;
    double rho = 0.0;
    for (int i = threadIdx.x; i < n; i += (int)blockDim.x) {
        double v = (double)rhs[(size_t)b0 * BRICK_CELLS + i];
        x[i] = 0.0;
        r[i] = v;
        p[i] = v;
        rho += v * v;
    }
    rho = block_reduce_1024(rho);
    double stop = rtol * rtol * rho;
    int it = 0;
    OffsetAcc pacc{p, b0};
    const LevelConst L = M.lc[M.org[b0].w];
    while (it < maxit && rho > stop && rho > 0.0) {
        double pq = 0.0;
        for (int i = threadIdx.x; i < n; i += (int)blockDim.x) {
            int b = b0 + (i >> 9), c = i & 511;
            int lc[3] = {c & 7, (c >> 3) & 7, c >> 6};
            double pc = p[i], Ap = 0.0;
            for (int d = 0; d < 3; ++d)
                for (int s = -1; s <= 1; s += 2) {
                    double a, bv;
                    face_nb(M, b, lc, d, s, pacc, nullptr, nullptr, false, a, bv);
                    Ap += L.ih2[d] * ((1.0 - a) * pc - bv);
                }
            q[i] = Ap;
            pq += pc * Ap;
        }
        pq = block_reduce_1024(pq);
        double alpha = rho / pq;
        double rho1 = 0.0;
        for (int i = threadIdx.x; i < n; i += (int)blockDim.x) {
            x[i] += alpha * p[i];
            double rv = r[i] - alpha * q[i];
            r[i] = rv;
            rho1 += rv * rv;
        }
        rho1 = block_reduce_1024(rho1);
        double beta = rho1 / rho;
        for (int i = threadIdx.x; i < n; i += (int)blockDim.x) p[i] = r[i] + beta * p[i];
        rho = rho1;
        ++it;
        __syncthreads();
    }
    for (int i = threadIdx.x; i < n; i += (int)blockDim.x) e[(size_t)b0 * BRICK_CELLS + i] = (T)x[i];
    __syncthreads();
    return it;
}

// CG as above for grids of at most 4096 cells: the search direction lives in
// LDS, each thread keeps its (at most four) cells of x, r and q in registers,
// and a reduction costs one barrier.
constexpr int CG_LDS_MAX = 4096;
constexpr int CG_PER = 8;  // cells per thread: CG_LDS_MAX / CG_PER threads at least

__device__ __forceinline__ double wg_sum_1024(double v, double *red, int slot)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) red[slot * 16 + (threadIdx.x >> 6)] = v;
    __syncthreads();
    double s = 0.0;
    const int nw = blockDim.x >> 6;
    for (int i = 0; i < nw; ++i) s += red[slot * 16 + i];
    return s;
}

template <class T>
__device__ int cg_solve_lds(const DevMeta &M, int b0, int nb, const T *rhs, T *e, double rtol, int maxit, double *p)
{
    __shared__ double red[3 * 16];
    const int n = nb * BRICK_CELLS;
    const LevelConst L = M.lc[M.org[b0].w];
    // neighbours of each owned cell (at most CG_PER per thread), resolved once: LDS index, or -1 for a
    // homogeneous boundary ghost (abnd p_c, in the diagonal); the coarsest
    // grid has no coarse-fine faces
    int nbi[CG_PER][6];
    double diag[CG_PER];
    for (int k = 0; k < CG_PER; ++k) {
        int i = threadIdx.x + (int)blockDim.x * k;
        diag[k] = 0.0;
        for (int f = 0; f < 6; ++f) nbi[k][f] = -1;
        if (i >= n) continue;
        int b = b0 + (i >> 9), c = i & 511;
        int l[3] = {c & 7, (c >> 3) & 7, c >> 6};
        for (int f = 0; f < 6; ++f) {
            int d = f >> 1, s = (f & 1) ? 1 : -1;
            int m[3] = {l[0], l[1], l[2]};
            m[d] += s;
            int bb = b;
            if (m[d] < 0 || m[d] > 7) {
                bb = M.nbr[b * 6 + f];
                m[d] = s > 0 ? 0 : 7;
            }
            if (bb >= 0) {
                nbi[k][f] = (bb - b0) * BRICK_CELLS + m[0] + 8 * m[1] + 64 * m[2];
                diag[k] += L.ih2[d];
            } else {
                diag[k] += (1.0 - L.abnd[d]) * L.ih2[d];
            }
        }
    }
    double x[CG_PER], r[CG_PER];
    double rho = 0.0;
    for (int k = 0; k < CG_PER; ++k) {
        int i = threadIdx.x + (int)blockDim.x * k;
        double v = i < n ? (double)rhs[(size_t)b0 * BRICK_CELLS + i] : 0.0;
        x[k] = 0.0;
        r[k] = v;
        if (i < n) p[i] = v;
        rho += v * v;
    }
    int slot = 0;
    rho = wg_sum_1024(rho, red, slot);
    slot = (slot + 1) % 3;
    double stop = rtol * rtol * rho;
    int it = 0;
    while (it < maxit && rho > stop && rho > 0.0) {
        double q[CG_PER], pk[CG_PER], pq = 0.0;
        for (int k = 0; k < CG_PER; ++k) {
            int i = threadIdx.x + (int)blockDim.x * k;
            q[k] = 0.0;
            pk[k] = 0.0;
            if (i >= n) continue;
            double pc = p[i], off = 0.0;
            for (int f = 0; f < 6; ++f)
                if (nbi[k][f] >= 0) off += L.ih2[f >> 1] * p[nbi[k][f]];
            pk[k] = pc;
            q[k] = diag[k] * pc - off;
            pq += pc * q[k];
        }
        pq = wg_sum_1024(pq, red, slot);
        slot = (slot + 1) % 3;
        double alpha = rho / pq;
        double rho1 = 0.0;
        for (int k = 0; k < CG_PER; ++k) {
            x[k] += alpha * pk[k];
            r[k] -= alpha * q[k];
            rho1 += r[k] * r[k];
        }
        rho1 = wg_sum_1024(rho1, red, slot);
        slot = (slot + 1) % 3;
        double beta = rho1 / rho;
        for (int k = 0; k < CG_PER; ++k) {
            int i = threadIdx.x + (int)blockDim.x * k;
            if (i < n) p[i] = r[k] + beta * pk[k];
        }
        __syncthreads();
        rho = rho1;
        ++it;
    }
    for (int k = 0; k < CG_PER; ++k) {
        int i = threadIdx.x + (int)blockDim.x * k;
        if (i < n) e[(size_t)b0 * BRICK_CELLS + i] = (T)x[k];
    }
    __syncthreads();
    return it;
}

// ---------------------------------------------------------------------------
// Exact solve of the coarsest grid (one box, homogeneous boundary ghosts) by
// its separable eigendecomposition: e = Q diag(1/lambda) Q^T r with Q the
// tensor product of the per-axis orthonormal eigenvector matrices.  Three
// launches over all jobs: forward transforms along x and y per (z plane, block
// of 16 x frequencies); along z per group of 16 columns (forward, division by
// the eigenvalue sum, inverse); inverse along x and y per (plane, block).  The
// work is dense FP64 products, bound by the matrix-core rate, so it is cut
// into 16-wide blocks to occupy every CU (a 64^3 grid gives 256 workgroups per
// launch).  FP64 scratch in natural order (x fastest).
// ---------------------------------------------------------------------------
__device__ __forceinline__ size_t direct_cell(const DirectJob &J, int x, int y, int z)
{
    const int nbx = J.dn[0] >> 3, nby = J.dn[1] >> 3;
    int b = J.b0 + (x >> 3) + nbx * ((y >> 3) + nby * (z >> 3));
    return (size_t)b * BRICK_CELLS + (x & 7) + 8 * (y & 7) + 64 * (z & 7);
}

__device__ __forceinline__ int pad16(int n) { return (n + 15) & ~15; }

typedef double dbl4 __attribute__((ext_vector_type(4)));

// Products on the FP64 matrix cores, one 16 x 16 output tile per wavefront:
// C[r][k] = sum_i Tb[r][i] D[k][i] with the table Tb (K x K, zero-padded, in
// global memory in operand order) and the data D (rows of K values in LDS,
// row stride ld).  v_mfma_f64 16x16x4 takes Tb[r0 + l%16][i0 + l/16] and
// D[k0 + l%16][i0 + l/16] from lane l and returns C[r0 + l/16 + 4j][k0 + l%16]
// in element j, so consecutive lanes hold consecutive k.
// The wavefronts of a workgroup take the (R/16) x (N/16) output tiles in
// turn; the K columns go in chunks of 64 (16 matrix-core steps, two
// accumulation chains).  A wavefront can take its first tile's first chunk
// of table rows early (dst_pre), so that those loads overlap the data loads.
struct DPre {
    double tb[16];
};
// this lane's operands of table rows r0.. for columns kc..kc+63:
// tb[s] = Tb[r0 + l%16][kc + 4s + l/16], from the table stored in that order
// (64 consecutive values per row block and step)
__device__ __forceinline__ void dst_rows(const double *Tb, int K, int r0, int kc, double (&tb)[16])
{
    const double *p = Tb + ((size_t)(r0 >> 4) * (K >> 2) + (kc >> 2)) * 64 + (threadIdx.x & 63);
#pragma unroll
    for (int s = 0; s < 16; ++s) tb[s] = kc + 4 * s < K ? p[64 * s] : 0.0;
}
__device__ __forceinline__ void dst_pre(const double *Tb, int R, int N, int K, DPre &pre)
{
    const int u = threadIdx.x >> 6, tr = R >> 4;
    if (u < tr * (N >> 4)) dst_rows(Tb, K, (u % tr) << 4, 0, pre.tb);
}
template <class F>
__device__ __forceinline__ void dst_product(const DPre &pre, const double *Tb, int R, int N, int K, const double *D,
                                            int ld, F out)
{
    const int lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
    const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6, tr = R >> 4, tiles = tr * (N >> 4);
    for (int u = wave; u < tiles; u += nw) {
        const int r0 = (u % tr) << 4, k0 = (u / tr) << 4;
        dbl4 a0 = {0.0, 0.0, 0.0, 0.0}, a1 = {0.0, 0.0, 0.0, 0.0};  // two chains (even and odd steps)
        for (int kc = 0; kc < K; kc += 64) {
            double tb[16];
            if (u == wave && kc == 0) {
#pragma unroll
                for (int q = 0; q < 16; ++q) tb[q] = pre.tb[q];
            } else {
                dst_rows(Tb, K, r0, kc, tb);
            }
            const double *d = D + (k0 + lr) * ld + lk + kc;
#pragma unroll
            for (int q = 0; q < 16; q += 2) {
                if (kc + 4 * q < K) a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(tb[q], d[4 * q], a0, 0, 0, 0);
                if (kc + 4 * q + 4 < K) a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(tb[q + 1], d[4 * q + 4], a1, 0, 0, 0);
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) out(r0 + lk + 4 * j, k0 + lr, j, a0[j] + a1[j]);
    }
}

// table pool layout per job: forward and inverse matrices of x, y, z, each
// P_d x P_d with P_d = pad16(n_d), zero-padded, in matrix-core operand order
// (dst_rows); then the eigenvalues of x, y, z (n_d each)
__device__ __forceinline__ const double *dst_table(const DirectJob &J, const double *tab, int d, bool inv)
{
    const int px = pad16(J.dn[0]), py = pad16(J.dn[1]), pz = pad16(J.dn[2]);
    int off = J.tab;
    if (d >= 1) off += 2 * px * px;
    if (d >= 2) off += 2 * py * py;
    const int p = d == 0 ? px : (d == 1 ? py : pz);
    return tab + off + (inv ? p * p : 0);
}

// transforms along x and y of one z plane for one block of 16 x-frequencies
// kx (x positions on the inverse), forward (r -> W) or inverse (W -> e,
// phi += e): the x transform of the whole plane restricted to the block,
// then the y transform of the block.  planes[i] = (job, z | block << 8), or
// with jobs == nullptr the one job J1 and workgroup z * blocks + block.
// Dynamic LDS: rows + 16 rows of ld doubles, rows = pad16(largest edge).
template <class T, bool INV>
__global__ void __launch_bounds__(256) k_dst_plane(const DirectJob *jobs, const int2 *planes, DirectJob J1,
                                                  const double *tab, double *W, const T *r, T *e, double *phib,
                                                  int phi_update, int ld, int rows)
{
    extern __shared__ double sm[];
    // one job (jobs == nullptr): J1, workgroup = z * blocks + block; else from the lists
    int z, kb;
    DirectJob J;
    if (!jobs) {
        J = J1;
        const int nkb = pad16(J.dn[0]) >> 4;
        z = blockIdx.x / nkb;
        kb = blockIdx.x - z * nkb;
    } else {
        const int2 pl = planes[blockIdx.x];
        J = jobs[pl.x];
        z = pl.y & 255;
        kb = pl.y >> 8;
    }
    const int nx = J.dn[0], ny = J.dn[1], kx0 = kb << 4, np = nx * ny;
    const int px = pad16(nx), py = pad16(ny);
    double *A = sm, *Bt = sm + rows * ld;  // plane [y][x]; x-transformed block [kx - kx0][y]
    double *w = W + J.w + (size_t)np * z;
    // the x table's first rows first, then the plane: those loads in flight together
    const double *Mx = dst_table(J, tab, 0, INV) + (size_t)(kx0 >> 4) * (px >> 2) * 64, *My = dst_table(J, tab, 1, INV);
    DPre p1;
    dst_pre(Mx, 16, py, px, p1);
    // the plane in rows of 64: x = xb + thread % 64, y = yb + thread / 64 + 4 q
    for (int xb = 0; xb < px; xb += 64)
        for (int yb = 0; yb < py; yb += 64) {
            const int x = xb + (threadIdx.x & 63), y0 = yb + (threadIdx.x >> 6);
            double v[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int y = y0 + 4 * q;
                v[q] = 0.0;
                if (y < ny && x < nx) v[q] = INV ? w[y * nx + x] : (double)r[direct_cell(J, x, y, z)];
            }
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int y = y0 + 4 * q;
                if (y < py && x < px) A[y * ld + x] = v[q];
            }
        }
    DPre p2;
    dst_pre(My, py, 16, py, p2);
    __syncthreads();
    // along x: Bt[kx - kx0][y] = sum_x Mx[kx][x] A[y][x]
    dst_product(p1, Mx, 16, py, px, A, ld, [&](int kx, int y, int, double s) { Bt[kx * ld + y] = s; });
    __syncthreads();
    // along y: out[ky][kx] = sum_y My[ky][y] Bt[kx - kx0][y]
    dst_product(p2, My, py, 16, py, Bt, ld, [&](int y, int xl, int, double s) {
        const int x = kx0 + xl;
        if (x >= nx || y >= ny) return;
        if (!INV) {
            w[y * nx + x] = s;
        } else {
            const size_t bi = direct_cell(J, x, y, z);
            e[bi] = (T)s;
            if (phi_update && J.amr) phib[bi] += s;
        }
    });
}

// transform along z of a group of DIRECT_COLS columns: forward, division by
// the eigenvalue sum, inverse.  groups[i] = (job, first column), or with
// jobs == nullptr the one job J1 and columns from DIRECT_COLS * workgroup.  Dynamic
// LDS: two arrays of DIRECT_COLS rows of ld doubles.
__global__ void __launch_bounds__(256) k_dst_column(const DirectJob *jobs, const int2 *groups, DirectJob J1,
                                                   const double *tab, double *W, int ld)
{
    extern __shared__ double sm[];
    double *A = sm, *C = sm + DIRECT_COLS * ld;  // [col][z], [col][kz]
    DirectJob J;
    int c0;  // np is a multiple of DIRECT_COLS
    if (!jobs) {  // one job: J1, workgroup = column group
        J = J1;
        c0 = blockIdx.x * DIRECT_COLS;
    } else {
        const int2 gr = groups[blockIdx.x];
        J = jobs[gr.x];
        c0 = gr.y;
    }
    const int nx = J.dn[0], ny = J.dn[1], nz = J.dn[2], np = nx * ny, pz = pad16(nz);
    const double *mux = dst_table(J, tab, 2, false) + 2 * pz * pz, *muy = mux + nx, *muz = muy + ny;
    const double *Fz = dst_table(J, tab, 2, false), *Bz = dst_table(J, tab, 2, true);
    double *w = W + J.w;
    DPre pf;
    dst_pre(Fz, pz, DIRECT_COLS, pz, pf);
    constexpr int NV = DIRECT_DIM * DIRECT_COLS / 256;
    double v[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const int i = threadIdx.x + 256 * q, zz = i / DIRECT_COLS, c = i % DIRECT_COLS;
        v[q] = zz < nz ? w[(size_t)np * zz + c0 + c] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const int i = threadIdx.x + 256 * q, zz = i / DIRECT_COLS, c = i % DIRECT_COLS;
        if (zz < pz) A[c * ld + zz] = v[q];
    }
    DPre pb;
    dst_pre(Bz, pz, DIRECT_COLS, pz, pb);
    __syncthreads();
    // forward, then the division by the eigenvalue sum of (column, kz)
    dst_product(pf, Fz, pz, DIRECT_COLS, pz, A, ld, [&](int kz, int c, int, double s) {
        const int col = c0 + c;
        C[c * ld + kz] = kz < nz ? s / (mux[col % nx] + muy[col / nx] + muz[kz]) : 0.0;
    });
    __syncthreads();
    dst_product(pb, Bz, pz, DIRECT_COLS, pz, C, ld, [&](int zz, int c, int, double s) {
        if (zz < nz) w[(size_t)np * zz + c0 + c] = s;
    });
}

// one workgroup per job: jobs[i] = (first brick, bricks, offset of its four
// work vectors in doubles)
template <class T>
__global__ void __launch_bounds__(1024) k_bottom_cg(DevMeta M, const int4 *jobs, const T *rhs, T *e, double *work,
                                                    double rtol, int maxit, int *iters)
{
    int4 jb = jobs[blockIdx.x];
    int it = cg_solve<T>(M, jb.x, jb.y, rhs, e, work + jb.z, rtol, maxit);
    if (threadIdx.x == 0 && iters) atomicMax(iters, it);
}

// exact red-black Gauss-Seidel pass over a whole level by one workgroup
template <class T>
__device__ void wg_gs_pass(const DevMeta &M, int b0, int nb, T *e, const T *r, int colour)
{
    const LevelConst L = M.lc[M.org[b0].w];
    for (int i = threadIdx.x; i < nb * 256; i += (int)blockDim.x) {
        int b = b0 + (i >> 8), t = i & 255;
        int z = t >> 5, y = (t >> 2) & 7, xx = (t & 3) << 1;
        int lc[3] = {xx + (((y + z) & 1) ^ colour), y, z};
        size_t li = (size_t)b * BRICK_CELLS + lc[0] + 8 * y + 64 * z;
        double num = (double)r[li], den = 0.0;
        for (int d = 0; d < 3; ++d)
            for (int s = -1; s <= 1; s += 2) {
                double a, bv;
                face_nb(M, b, lc, d, s, BrickAcc<T>{e}, nullptr, nullptr, false, a, bv);
                num += L.ih2[d] * bv;
                den += L.ih2[d] * (1.0 - a);
            }
        e[li] = (T)(num / den);
    }
    __syncthreads();
}

// The part of the V-cycle on the small levels 0..nlev-1 of one problem (no
// coarse-fine faces there) in one workgroup: pre-smoothing and restriction
// down, CG on level 0, prolongation and post-smoothing up, and phi += e on
// AMR levels when phi_update is set.
template <class T>
__global__ void __launch_bounds__(1024) k_coarse_cycle(DevMeta M, const CoarseJob *jobs, T *e, T *r, double *work,
                                                       int nu1, int nu2, double rtol, int maxit, int *iters,
                                                       double *phib, int phi_update)
{
    __shared__ double lds[CG_LDS_MAX];
    const CoarseJob J = jobs[blockIdx.x];
    if (J.direct) return;  // solved by the transform kernels
    for (int k = J.nlev - 1; k >= 1; --k) {
        const int b0 = J.b0[k], nb = J.nb[k];
        for (int i = threadIdx.x; i < nb * BRICK_CELLS; i += (int)blockDim.x) e[(size_t)b0 * BRICK_CELLS + i] = (T)0;
        __syncthreads();
        for (int it = 0; it < nu1; ++it) {
            wg_gs_pass<T>(M, b0, nb, e, r, 0);
            wg_gs_pass<T>(M, b0, nb, e, r, 1);
        }
        const LevelConst L = M.lc[M.org[b0].w];
        for (int i = threadIdx.x; i < nb * 64; i += (int)blockDim.x) {
            int b = b0 + (i >> 6), t = i & 63;
            int cx = t & 3, cy = (t >> 2) & 3, cz = t >> 4;
            double sum = 0.0;
            for (int dz = 0; dz < 2; ++dz)
                for (int dy = 0; dy < 2; ++dy)
                    for (int dx = 0; dx < 2; ++dx) {
                        int lc[3] = {2 * cx + dx, 2 * cy + dy, 2 * cz + dz};
                        sum += cell_residual(M, L, b, lc, e, r);
                    }
            int par = M.par[b];
            int pb = par >> 3, oc = par & 7;
            int X = (oc & 1) * 4 + cx, Y = ((oc >> 1) & 1) * 4 + cy, Z = (oc >> 2) * 4 + cz;
            r[(size_t)pb * BRICK_CELLS + X + 8 * Y + 64 * Z] = (T)(0.125 * sum);
        }
        __syncthreads();
    }
    int it;
    if (J.nb[0] * BRICK_CELLS <= CG_PER * (int)blockDim.x && J.nb[0] * BRICK_CELLS <= CG_LDS_MAX)
        it = cg_solve_lds<T>(M, J.b0[0], J.nb[0], r, e, rtol, maxit, lds);
    else
        it = cg_solve<T>(M, J.b0[0], J.nb[0], r, e, work + J.cg_off, rtol, maxit);
    if (threadIdx.x == 0 && iters) atomicMax(iters, it);
    for (int k = 0; k < J.nlev; ++k) {
        const int b0 = J.b0[k], nb = J.nb[k];
        if (k > 0) {
            for (int i = threadIdx.x; i < nb * BRICK_CELLS; i += (int)blockDim.x) {
                int b = b0 + (i >> 9), c = i & 511;
                int par = M.par[b];
                int pb = par >> 3, oc = par & 7;
                int x = c & 7, y = (c >> 3) & 7, z = c >> 6;
                size_t pi = (size_t)pb * BRICK_CELLS + ((oc & 1) * 4 + (x >> 1)) +
                            8 * (((oc >> 1) & 1) * 4 + (y >> 1)) + 64 * ((oc >> 2) * 4 + (z >> 1));
                size_t li = (size_t)b * BRICK_CELLS + c;
                e[li] = (T)((double)e[li] + (double)e[pi]);
            }
            __syncthreads();
            for (int it2 = 0; it2 < nu2; ++it2) {
                wg_gs_pass<T>(M, b0, nb, e, r, 0);
                wg_gs_pass<T>(M, b0, nb, e, r, 1);
            }
        }
        if (phi_update && M.lc[M.org[b0].w].amr >= 0)
            for (int i = threadIdx.x; i < nb * BRICK_CELLS; i += (int)blockDim.x)
                phib[(size_t)b0 * BRICK_CELLS + i] += (double)e[(size_t)b0 * BRICK_CELLS + i];
    }
}

// ---------------------------------------------------------------------------
// particles
// ---------------------------------------------------------------------------
template <class P>
__device__ __forceinline__ bool cic_stencil(const DepLevel &D, double X, double Y, double Z, int *i0, int *i1,
                                            double *f)
{
    double xs[3] = {X, Y, Z};
    for (int d = 0; d < 3; ++d) {
        if (!(xs[d] >= D.lo[d] && xs[d] < D.hi[d])) return false;
        double s = (xs[d] - D.lo[d]) / D.h[d] - 0.5;
        double fl = floor(s);
        int a = (int)fl;
        f[d] = s - fl;
        int b = a + 1;
        a = a < 0 ? 0 : (a > D.n[d] - 1 ? D.n[d] - 1 : a);
        b = b < 0 ? 0 : (b > D.n[d] - 1 ? D.n[d] - 1 : b);
        i0[d] = a;
        i1[d] = b;
    }
    return true;
}

__device__ __forceinline__ int64_t user_index(const DepLevel &D, const int64_t *ubase, const int2 *ustr, int i,
                                              int j, int k)
{
    int g = D.bmap[(i >> 3) + D.nbk[0] * ((j >> 3) + D.nbk[1] * (k >> 3))];
    if (g < 0) return -1;
    int2 s = ustr[g];
    return ubase[g] + (i & 7) + (int64_t)s.x * (j & 7) + (int64_t)s.y * (k & 7);
}

// Corners of a CIC stencil: bit d of c selects the upper cell along axis d;
// st[d]: the stencil crosses a brick face along d.  A corner is "fresh"
// when every upper axis of it crosses, so that its brick differs from the
// bricks of the corners below it; spread_corners copies the value of each
// fresh corner to the corners in the same brick (the bits of axes without a
// crossing cleared), with fixed indices only.
__device__ __forceinline__ bool corner_fresh(int c, const bool *st)
{
    return (!(c & 1) || st[0]) && (!(c & 2) || st[1]) && (!(c & 4) || st[2]);
}

template <class V>
__device__ __forceinline__ void spread_corners(const bool *st, V *v)
{
    v[1] = st[0] ? v[1] : v[0];
    v[2] = st[1] ? v[2] : v[0];
    v[3] = st[1] ? (st[0] ? v[3] : v[2]) : v[1];
    v[4] = st[2] ? v[4] : v[0];
    v[5] = st[2] ? (st[0] ? v[5] : v[4]) : v[1];
    v[6] = st[2] ? (st[1] ? v[6] : v[4]) : v[2];
    v[7] = st[2] ? (st[1] ? (st[0] ? v[7] : v[6]) : v[5]) : v[3];
}

// Caller's-layout index of each corner of the CIC stencil (i0, i1) on level
// D, -1 outside the level's boxes or for every corner when !ok.  Each
// distinct brick of the stencil is looked up once (at most two per axis),
// every lookup issued before any is used.
__device__ __forceinline__ void corner_addresses(const DepLevel &D, const int64_t *ubase, const int2 *ustr, bool ok,
                                                 const int *i0, const int *i1, int64_t (&u)[8])
{
    const bool st[3] = {(i0[0] >> 3) != (i1[0] >> 3), (i0[1] >> 3) != (i1[1] >> 3), (i0[2] >> 3) != (i1[2] >> 3)};
    int g[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        g[c] = -1;
        if (ok && corner_fresh(c, st)) {
            const int bx = ((c & 1) ? i1[0] : i0[0]) >> 3, by = ((c & 2) ? i1[1] : i0[1]) >> 3,
                      bz = ((c & 4) ? i1[2] : i0[2]) >> 3;
            g[c] = D.bmap[bx + D.nbk[0] * (by + D.nbk[1] * bz)];
        }
    }
    spread_corners(st, g);
    int64_t ub[8];
    int usx[8], usy[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        ub[c] = 0;
        usx[c] = usy[c] = 0;
        if (corner_fresh(c, st) && g[c] >= 0) {
            ub[c] = ubase[g[c]];
            const int2 s2 = ustr[g[c]];
            usx[c] = s2.x;
            usy[c] = s2.y;
        }
    }
    spread_corners(st, ub);
    spread_corners(st, usx);
    spread_corners(st, usy);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int ii = (c & 1) ? i1[0] : i0[0], jj = (c & 2) ? i1[1] : i0[1], kk = (c & 4) ? i1[2] : i0[2];
        u[c] = g[c] < 0 ? -1 : ub[c] + (ii & 7) + (int64_t)usx[c] * (jj & 7) + (int64_t)usy[c] * (kk & 7);
    }
}

// Add v to rho[addr] for every active lane (addr >= 0), combining lanes of
// the wavefront that share an address: up to 8 distinct addresses are summed
// across the wavefront and issued as one atomic each by their first lane; the
// remaining lanes issue their own atomics.
__device__ __forceinline__ void wave_atomic_add(double *rho, int64_t addr, double v)
{
    const int lane = threadIdx.x & 63;
    uint64_t active = __ballot(addr >= 0);
    for (int round = 0; round < 8 && active; ++round) {
        int leader = __builtin_ctzll(active);
        int64_t A = __shfl(addr, leader, 64);
        uint64_t match = __ballot(addr == A) & active;
        double s = ((match >> lane) & 1) ? v : 0.0;
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if (lane == leader) atomicAdd(rho + A, s);
        active &= ~match;
    }
    if ((active >> lane) & 1) atomicAdd(rho + addr, v);
}

// Deposit every particle on every listed level.  A workgroup takes 256 PPT
// consecutive particles of the visiting order (spatially sorted, so they are
// close together) and, per level, accumulates their CIC weights in an LDS
// tile over the bounding box of their stencils, then adds the tile's nonzero
// cells to rho with one FP64 atomic each.  When the box exceeds the tile the
// workgroup adds its weights with wavefront-combined global atomics instead.
// Two tile sizes: 4096 cells (32 KB), and 8192 cells (64 KB, fewer
// workgroups per CU) for levels on which a visiting-order bucket spans 8 or
// more cells per axis, so that the boxes of those levels still fit (576^3
// benchmark: deposit 8.7 -> 5.3 ms; on the levels with small buckets the
// larger tile only costs occupancy).
constexpr int DEP_TILE = 4096, DEP_TILE_BIG = 8192;
// bricks whose layout a tile flush stages in LDS (a tile of 4096 cells spans
// at most 4 x 4 x 4 bricks unless it is elongated; longer ones look up each cell)
constexpr int DEP_BRICKS = 64;
// particles from which a deposit launch takes the per-wavefront tile passes
constexpr int64_t DEP_WAVES_MIN = (int64_t)4 << 20;

// v[0..2] minima, v[3..5] maxima over the wavefront
__device__ __forceinline__ void wave_minmax6(int *v)
{
    for (int o = 32; o > 0; o >>= 1)
        for (int a = 0; a < 6; ++a) {
            int w = __shfl_xor(v[a], o, 64);
            v[a] = a < 3 ? min(v[a], w) : max(v[a], w);
        }
}

__device__ __forceinline__ void wg_minmax6(int *v, int *red)
{
    // v[0..2] minima, v[3..5] maxima over the workgroup of 256 threads
    for (int o = 32; o > 0; o >>= 1)
        for (int a = 0; a < 6; ++a) {
            int w = __shfl_xor(v[a], o, 64);
            v[a] = a < 3 ? min(v[a], w) : max(v[a], w);
        }
    const int wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int a = 0; a < 6; ++a) red[a * 4 + wid] = v[a];
    __syncthreads();
    for (int a = 0; a < 6; ++a) {
        int r = red[a * 4];
        for (int k = 1; k < 4; ++k) r = a < 3 ? min(r, red[a * 4 + k]) : max(r, red[a * 4 + k]);
        v[a] = r;
    }
    __syncthreads();
}

template <class P, int PPT, int TILE, bool WAVES>
__global__ void __launch_bounds__(256) k_deposit(int64_t n, const P *x, const P *y, const P *z, const double *q,
                                                 const uint32_t *perm, DepArgs A, const int64_t *ubase,
                                                 const int2 *ustr, unsigned long long *nout, P *xs, P *ys, P *zs,
                                                 double *qs)
{
    __shared__ double acc[TILE];
    __shared__ int red[24];
    // the caller's-layout base and strides of the bricks the tile spans
    // (when they are at most DEP_BRICKS), looked up once per tile
    __shared__ int64_t tub[DEP_BRICKS];
    __shared__ int2 tus[DEP_BRICKS];
    __shared__ int wbox[4][6];  // the wavefronts' boxes when the workgroup's exceeds the tile
    const int64_t first = (int64_t)blockIdx.x * 256 * PPT;
    double X[PPT], Y[PPT], Z[PPT], Q[PPT];
    bool valid[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        int64_t i = first + (int64_t)threadIdx.x * PPT + k;  // consecutive particles per thread
        valid[k] = i < n;
        int64_t p = valid[k] ? (perm ? (int64_t)perm[i] : i) : 0;
        X[k] = valid[k] ? (double)x[p] : 0.0;
        Y[k] = valid[k] ? (double)y[p] : 0.0;
        Z[k] = valid[k] ? (double)z[p] : 0.0;
        Q[k] = valid[k] ? q[p] : 0.0;
        if (xs && valid[k]) {  // the visiting-order copy (exact: P -> double -> P)
            xs[i] = (P)X[k];
            ys[i] = (P)Y[k];
            zs[i] = (P)Z[k];
            qs[i] = Q[k];
        }
    }
    for (int l = 0; l < A.nlev; ++l) {
        const DepLevel &D = A.lev[l];
        int i0[PPT][3], i1[PPT][3];
        double f[PPT][3];
        bool ok[PPT];
        int bb[6] = {INT_MAX, INT_MAX, INT_MAX, INT_MIN, INT_MIN, INT_MIN};
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            ok[k] = valid[k] && cic_stencil<P>(D, X[k], Y[k], Z[k], i0[k], i1[k], f[k]);
            if (valid[k] && !ok[k] && l == 0 && nout) atomicAdd(nout, 1ull);
            if (ok[k])
                for (int d = 0; d < 3; ++d) {
                    bb[d] = min(bb[d], i0[k][d]);
                    bb[3 + d] = max(bb[3 + d], i1[k][d]);
                }
        }
        // this lane's own bounds, kept for the wavefront boxes below
        int lb[6];
#pragma unroll
        for (int a = 0; a < 6; ++a) lb[a] = bb[a];
        wg_minmax6(bb, red);
        if (bb[0] > bb[3]) continue;  // no particle of the workgroup inside the domain
        // One pass through the LDS tile over the box tb of cells: clear, add
        // the stencils of the taking part lanes' particles (mine), add the
        // tile's nonzero cells to rho.  Every thread of the workgroup runs it.
        auto tile_pass = [&](const int *tb, bool mine) {
            const int ex = tb[3] - tb[0] + 1, ey = tb[4] - tb[1] + 1, ez = tb[5] - tb[2] + 1;
            const int vol = ex * ey * ez;
            for (int t = threadIdx.x; t < vol; t += 256) acc[t] = 0.0;
            __syncthreads();
            // the 8 corners of each stencil, in an order rotated by the
            // lane: the particles of a wavefront often share a stencil (the
            // visiting order keeps them together), and the same corner of
            // one cell from every lane at once would serialise the LDS
            // atomics on one address
            const int rot = threadIdx.x & 7;
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                if (!mine || !ok[k]) continue;
                const double qv = Q[k] * D.ivol;
                const int b = (i0[k][0] - tb[0]) + ex * ((i0[k][1] - tb[1]) + ey * (i0[k][2] - tb[2]));
                const int ox = i1[k][0] - i0[k][0], oy = i1[k][1] - i0[k][1], oz = i1[k][2] - i0[k][2];
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const int ce = (c + rot) & 7;
                    const bool ux = ce & 1, uy = ce & 2, uz = ce & 4;
                    const double w = (ux ? f[k][0] : 1.0 - f[k][0]) * (uy ? f[k][1] : 1.0 - f[k][1]) *
                                     (uz ? f[k][2] : 1.0 - f[k][2]);
                    atomicAdd(&acc[b + (ux ? ox : 0) + ex * ((uy ? oy : 0) + ey * (uz ? oz : 0))], qv * w);
                }
            }
            // the tile's bricks: (bx0, by0, bz0) + (0..nbx-1, 0..nby-1, 0..nbz-1)
            const int bx0 = tb[0] >> 3, by0 = tb[1] >> 3, bz0 = tb[2] >> 3;
            const int nbx = (tb[3] >> 3) - bx0 + 1, nby = (tb[4] >> 3) - by0 + 1, nbz = (tb[5] >> 3) - bz0 + 1;
            const int nbt = nbx * nby * nbz;
            if (nbt <= DEP_BRICKS && (int)threadIdx.x < nbt) {
                const int t = threadIdx.x, ix = t % nbx, iy = (t / nbx) % nby, iz = t / (nbx * nby);
                const int g = D.bmap[(bx0 + ix) + D.nbk[0] * ((by0 + iy) + D.nbk[1] * (bz0 + iz))];
                tub[t] = g >= 0 ? ubase[g] : -1;
                tus[t] = g >= 0 ? ustr[g] : make_int2(0, 0);
            }
            __syncthreads();
            for (int t = threadIdx.x; t < vol; t += 256) {
                double v = acc[t];
                if (v == 0.0) continue;
                const int ii = tb[0] + t % ex, r = t / ex, jj = tb[1] + r % ey, kk = tb[2] + r / ey;
                int64_t u;
                if (nbt <= DEP_BRICKS) {
                    const int k = ((ii >> 3) - bx0) + nbx * (((jj >> 3) - by0) + nby * ((kk >> 3) - bz0));
                    const int64_t b = tub[k];
                    const int2 us = tus[k];
                    u = b < 0 ? -1 : b + (ii & 7) + (int64_t)us.x * (jj & 7) + (int64_t)us.y * (kk & 7);
                } else {
                    u = user_index(D, ubase, ustr, ii, jj, kk);
                }
                if (u >= 0) atomicAdd(A.rho[l] + u, v);
            }
            __syncthreads();
        };
        const int64_t vol = (int64_t)(bb[3] - bb[0] + 1) * (bb[4] - bb[1] + 1) * (bb[5] - bb[2] + 1);
        if (vol <= TILE) {
            tile_pass(bb, true);
            continue;
        }
        // The stencils span more than the tile (sparse particles).  With
        // WAVES the wavefronts take the tile in turn, each over the box of its
        // own particles.  A wavefront whose box still exceeds the tile (every
        // wavefront without WAVES) adds each corner with a global atomic, the
        // addresses found first with every table load in flight together.
        bool sparse = true;
        if (WAVES) {
            wave_minmax6(lb);
            const int wave = threadIdx.x >> 6;
            if ((threadIdx.x & 63) == 0)
#pragma unroll
                for (int a = 0; a < 6; ++a) wbox[wave][a] = lb[a];
            __syncthreads();
            sparse = false;  // this wavefront's box exceeds the tile too
#pragma unroll 1
            for (int wv = 0; wv < 4; ++wv) {
                int tb[6];
#pragma unroll
                for (int a = 0; a < 6; ++a) tb[a] = wbox[wv][a];
                if (tb[0] > tb[3]) continue;  // no particle of that wavefront inside the domain
                const int64_t wvol = (int64_t)(tb[3] - tb[0] + 1) * (tb[4] - tb[1] + 1) * (tb[5] - tb[2] + 1);
                if (wvol <= TILE) tile_pass(tb, wave == wv);
                else if (wave == wv) sparse = true;
            }
        }
        if (!sparse) continue;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const double qv = ok[k] ? Q[k] * D.ivol : 0.0;
            int64_t u[8];
            corner_addresses(D, ubase, ustr, ok[k], i0[k], i1[k], u);
            // all lanes stay in the loop: the combination uses wavefront shuffles
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                double w = ((c & 1) ? f[k][0] : 1.0 - f[k][0]) * ((c & 2) ? f[k][1] : 1.0 - f[k][1]) *
                           ((c & 4) ? f[k][2] : 1.0 - f[k][2]);
                wave_atomic_add(A.rho[l], u[c], qv * w);
            }
        }
    }
}

// Two cells adjacent along x in one row of a box: one 16-byte load (8-byte
// alignment is enough for a global load on CDNA).
typedef double dpair __attribute__((ext_vector_type(2)));
typedef dpair dpair_a8 __attribute__((aligned(8)));

// E at every particle from the finest level whose boxes hold all 8 cells of
// its CIC stencil; particles are visited in the given (spatially sorted)
// order so that neighbouring threads read neighbouring field cells.  ORD:
// the positions are already in that order (x[i] is particle perm[i]), so
// only the writes go through perm, or, with rec, E goes to rec[i] in the
// visiting order for k_unpermute.  Boxes are unions of whole bricks, so the
// stencil's 8 cells lie in at most two bricks per axis: each distinct brick
// is looked up once (mostly one brick in all), and when the two x cells of
// the stencil share a brick row they are read together.  Same sums in the
// same order as cell by cell.
template <class P, bool ORD>
__global__ void __launch_bounds__(256) k_gather(int64_t n, const P *x, const P *y, const P *z, const uint32_t *perm,
                                                GatherArgs G, const int64_t *ubase, const int2 *ustr, double *Ex,
                                                double *Ey, double *Ez, double4 *rec)
{
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    int64_t p = perm ? (int64_t)perm[i] : i;
    int64_t s = ORD ? i : p;
    double X = (double)x[s], Y = (double)y[s], Z = (double)z[s];
    double e[3] = {0.0, 0.0, 0.0};
    for (int l = G.nlev - 1; l >= 0; --l) {
        const DepLevel &D = G.lev[l];
        int i0[3], i1[3];
        double f[3];
        if (!cic_stencil<P>(D, X, Y, Z, i0, i1, f)) break;
        // st[d]: the stencil crosses a brick face along d
        const int bstride[3] = {1, D.nbk[0], D.nbk[0] * D.nbk[1]};
        bool st[3];
        int base = 0, off[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            base += (i0[d] >> 3) * bstride[d];
            st[d] = (i1[d] >> 3) != (i0[d] >> 3);
            off[d] = st[d] ? bstride[d] : 0;
        }
        // brick of corner c (bit d of c: the upper cell along d), looked up
        // for the corners whose upper axes all cross a brick face; every
        // other corner shares the brick of one of those
        int g[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            g[c] = -1;
            if (corner_fresh(c, st))
                g[c] = D.bmap[base + ((c & 1) ? off[0] : 0) + ((c & 2) ? off[1] : 0) + ((c & 4) ? off[2] : 0)];
        }
        spread_corners(st, g);
        bool ok = true;
#pragma unroll
        for (int c = 0; c < 8; ++c) ok = ok && g[c] >= 0;
        if (!ok) continue;
        int64_t u[8];
        {
            int64_t ub[8];
            int usx[8], usy[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                ub[c] = 0;
                usx[c] = usy[c] = 0;
                if (corner_fresh(c, st)) {
                    ub[c] = ubase[g[c]];
                    const int2 t = ustr[g[c]];
                    usx[c] = t.x;
                    usy[c] = t.y;
                }
            }
            spread_corners(st, ub);
            spread_corners(st, usx);
            spread_corners(st, usy);
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const int ci = (c & 1) ? i1[0] : i0[0], cj = (c & 2) ? i1[1] : i0[1], ck = (c & 4) ? i1[2] : i0[2];
                u[c] = ub[c] + (ci & 7) + (int64_t)usx[c] * (cj & 7) + (int64_t)usy[c] * (ck & 7);
            }
        }
        // the field values of the 8 cells, x pairs with one load each when
        // the upper x cell follows the lower one in the same brick row
        double v[3][8];
        if (!st[0] && i1[0] == i0[0] + 1) {
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int c = 0; c < 8; c += 2) {
                    const dpair t = *(const dpair_a8 *)(G.E[3 * l + d] + u[c]);
                    v[d][c] = t.x;
                    v[d][c + 1] = t.y;
                }
        } else {
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int c = 0; c < 8; ++c) v[d][c] = G.E[3 * l + d][u[c]];
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            double w = ((c & 1) ? f[0] : 1.0 - f[0]) * ((c & 2) ? f[1] : 1.0 - f[1]) *
                       ((c & 4) ? f[2] : 1.0 - f[2]);
#pragma unroll
            for (int d = 0; d < 3; ++d) e[d] += w * v[d][c];
        }
        break;
    }
    if (rec) {
        rec[i] = make_double4(e[0], e[1], e[2], 0.0);
        return;
    }
    Ex[p] = e[0];
    Ey[p] = e[1];
    Ez[p] = e[2];
}

// E of particle p from its record in the visiting order (iperm[p] = its
// place there): one 32-byte read at a scattered place, three coalesced writes
__global__ void __launch_bounds__(256) k_unpermute(int64_t n, const uint32_t *iperm, const double4 *rec, double *Ex,
                                                   double *Ey, double *Ez)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    const double4 r = rec[iperm[p]];
    Ex[p] = r.x;
    Ey[p] = r.y;
    Ez[p] = r.z;
}

// max |rho| over a level (per-workgroup partials, then one workgroup)
__global__ void __launch_bounds__(256) k_absmax_part(const double *v, int64_t n, double *part)
{
    double m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        m = fmax(m, fabs(v[i]));
    m = block_reduce(m, 1);
    if (threadIdx.x == 0) part[blockIdx.x] = m;
}

__global__ void __launch_bounds__(256) k_absmax_final(const double *part, int n, double *out)
{
    double m = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) m = fmax(m, part[i]);
    m = block_reduce(m, 1);
    if (threadIdx.x == 0) *out = m;
}

// tag |rho| > lambda * max |rho| (the max read from device memory)
__global__ void __launch_bounds__(256) k_tag(const double *v, int64_t n, const double *vmax, double lambda,
                                             uint8_t *tags)
{
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    tags[i] = fabs(v[i]) > lambda * (*vmax) ? 1 : 0;
}

template <class T>
__global__ void __launch_bounds__(256) k_copy(const T *a, T *b, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) b[i] = a[i];
}

// Tag cells of one level (|rho| > lambda * max|rho|) and mark the blocks of
// the finer level (bf fine cells = half coarse cells per edge) that a tag
// dilated by nbuf cells reaches.  Same value written by every marker.
__global__ void __launch_bounds__(256) k_mark_blocks(const double *rho, const int4 *borg, const int64_t *ubase,
                                                     const int2 *ustr, int nb, const double *vmax, double lambda,
                                                     int nbuf, int half, int3 n, int3 g, uint8_t *marks)
{
    int b = xcd_remap(blockIdx.x, nb);
    int4 o = borg[b];
    int64_t ub = ubase[b];
    int2 us = ustr[b];
    double thr = lambda * (*vmax);
    for (int c = threadIdx.x; c < BRICK_CELLS; c += 256) {
        int x = c & 7, y = (c >> 3) & 7, z = c >> 6;
        double v = rho[ub + x + (int64_t)us.x * y + (int64_t)us.y * z];
        if (!(fabs(v) > thr)) continue;
        int gi = o.x + x, gj = o.y + y, gk = o.z + z;
        int x0 = max(0, gi - nbuf) / half, x1 = min(n.x - 1, gi + nbuf) / half;
        int y0 = max(0, gj - nbuf) / half, y1 = min(n.y - 1, gj + nbuf) / half;
        int z0 = max(0, gk - nbuf) / half, z1 = min(n.z - 1, gk + nbuf) / half;
        for (int bz = z0; bz <= z1; ++bz)
            for (int by = y0; by <= y1; ++by)
                for (int bx = x0; bx <= x1; ++bx) marks[(size_t)bx + (size_t)g.x * ((size_t)by + (size_t)g.y * bz)] = 1;
    }
}

__global__ void __launch_bounds__(256) k_fill_multi(DepArgs A, int64_t total, const int64_t *dummy)
{
    (void)dummy;
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    for (int l = 0; l < A.nlev; ++l) {
        if (i < A.ncell[l]) {
            A.rho[l][i] = 0.0;
            return;
        }
        i -= A.ncell[l];
    }
    (void)total;
}

// Proper nesting of the marked blocks of the finer level: a block stays
// marked when its footprint on the coarse level (half coarse cells per block
// edge), grown by np cells and clipped to the level's index space cn, lies
// in bricks of the coarse level (cbmap over its brick grid cnbk).  The marks
// are packed into bits in linear block order, word t / 64 holding block t at
// bit t % 64, for the greedy merge on the host.
__global__ void __launch_bounds__(256) k_nest_pack(const uint8_t *marks, int64_t total, int3 g, const int32_t *cbmap,
                                                   int3 cn, int3 cnbk, int half, int np, uint64_t *bits)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    bool keep = false;
    if (t < total && marks[t]) {
        const int blk[3] = {(int)(t % g.x), (int)((t / g.x) % g.y), (int)(t / ((int64_t)g.x * g.y))};
        const int nn[3] = {cn.x, cn.y, cn.z};
        int b0[3], b1[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int lo = max(0, blk[d] * half - np), hi = min(nn[d], (blk[d] + 1) * half + np);
            b0[d] = lo >> 3;
            b1[d] = (hi - 1) >> 3;
        }
        keep = true;
        for (int bz = b0[2]; bz <= b1[2] && keep; ++bz)
            for (int by = b0[1]; by <= b1[1] && keep; ++by)
                for (int bx = b0[0]; bx <= b1[0] && keep; ++bx)
                    keep = cbmap[bx + (int64_t)cnbk.x * (by + (int64_t)cnbk.y * bz)] >= 0;
    }
    const uint64_t m = __ballot(keep);
    if ((threadIdx.x & 63) == 0 && t < total) bits[t >> 6] = m;
}

__global__ void __launch_bounds__(256) k_fill(double *v, int64_t n, double val)
{
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) v[i] = val;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

template <class T>
void launch_outer_residual(hipStream_t st, const DevMeta &M, int b0, int nb, const int32_t *list, const double *phib,
                           const double *rhob, double inv_eps0, const double *cp_phi, T *r_out, double *part,
                           int norm_p, bool zero_phi, double *const *r_user, const double *ffs)
{
    if (nb <= 0) return;
    // four bricks per workgroup on levels far larger than the chip (the
    // sweep's tuning finds the same), one otherwise
    if (nb > 16384) {
        const dim3 g((nb + 3) / 4), blk(256);
        if (zero_phi)
            AMRMG_LAUNCH((k_outer_residual<T, true, 4>), g, blk, 0, st, M, b0, nb, phib, rhob, inv_eps0, cp_phi,
                         r_out, part, norm_p, list, r_user, ffs);
        else
            AMRMG_LAUNCH((k_outer_residual<T, false, 4>), g, blk, 0, st, M, b0, nb, phib, rhob, inv_eps0, cp_phi,
                         r_out, part, norm_p, list, r_user, ffs);
    } else {
        if (zero_phi)
            AMRMG_LAUNCH((k_outer_residual<T, true, 1>), dim3(nb), dim3(64), 0, st, M, b0, nb, phib, rhob, inv_eps0,
                         cp_phi, r_out, part, norm_p, list, r_user, ffs);
        else
            AMRMG_LAUNCH((k_outer_residual<T, false, 1>), dim3(nb), dim3(64), 0, st, M, b0, nb, phib, rhob,
                         inv_eps0, cp_phi, r_out, part, norm_p, list, r_user, ffs);
    }
}

void launch_user_brick(hipStream_t st, const DevMeta &M, int b0, int nb, const int32_t *list, bool to_brick,
                       double *const *a, double *ab, double *const *bu, double *bb)
{
    if (nb <= 0) return;
    AMRMG_LAUNCH(k_user_brick, dim3(nb), dim3(256), 0, st, M, b0, nb, list, (int)to_brick, a, ab, bu, bb);
}

void launch_level_norms(hipStream_t st, const int2 *ranges, int n, const double *part, double *out, int norm_p,
                        double *hout, int alt, unsigned *hseq, unsigned *counter)
{
    if (n <= 0) return;
    AMRMG_LAUNCH(k_level_norms, dim3(1), dim3(1024), 0, st, ranges, n, part, out, norm_p, hout, alt, hseq,
                 counter);
}

template <class T>
void launch_cpart_brick(hipStream_t st, const DevMeta &M, int cf0, int ncf, const T *src, T *cp, const T *fine,
                        double *ffs)
{
    if (ncf <= 0) return;
    SrcBrick<T> s{src};
    AMRMG_LAUNCH((k_cpart<T, SrcBrick<T>>), dim3(blocks_for((int64_t)ncf * 16, 256)), dim3(256), 0, st, M,
                       cf0, ncf, s, cp, fine, ffs);
}

template <class T>
void launch_face_sums(hipStream_t st, const DevMeta &M, int cf0, int ncf, const T *e, double *ffs)
{
    if (ncf <= 0) return;
    AMRMG_LAUNCH((k_face_sums<T>), dim3(blocks_for((int64_t)ncf * 16, 256)), dim3(256), 0, st, M, cf0, ncf, e,
                 ffs);
}

template <class T>
void launch_gsrb(hipStream_t st, const DevMeta &M, int b0, int nb, T *e, const T *r, const T *cp, int colour,
                 bool init)
{
    if (nb <= 0) return;
    AMRMG_LAUNCH((k_gsrb<T>), dim3(nb), dim3(256), 0, st, M, b0, nb, e, r, cp, colour, (int)init);
}

template <class T>
void launch_jacobi(hipStream_t st, const DevMeta &M, int b0, int nb, const T *ein, T *eout, const T *r, const T *cp,
                   double omega, bool init)
{
    if (nb <= 0) return;
    AMRMG_LAUNCH((k_jacobi<T>), dim3(nb), dim3(256), 0, st, M, b0, nb, ein, eout, r, cp, omega, (int)init);
}

template <class T>
void launch_restrict(hipStream_t st, const DevMeta &M, int b0, int nb, const int32_t *rlist, int nrf, const T *e,
                     T *r, const double *ffs)
{
    if (nb + nrf <= 0) return;
    AMRMG_LAUNCH((k_restrict<T>), dim3((nb + 1) / 2 + nrf), dim3(128), 0, st, M, b0, nb, rlist, nrf, e, r, ffs);
}

template <class T>
void launch_prolong(hipStream_t st, const DevMeta &M, int b0, int nb, T *e)
{
    if (nb <= 0) return;
    AMRMG_LAUNCH((k_prolong<T>), dim3(nb), dim3(256), 0, st, M, b0, nb, e);
}

template <class T>
void launch_phi_update(hipStream_t st, const DevMeta &M, int b0, int nb, const int32_t *list, double *phib,
                       const T *e)
{
    if (nb <= 0) return;
    AMRMG_LAUNCH((k_phi_update<T>), dim3(nb), dim3(256), 0, st, M, b0, nb, phib, e, list);
}

void launch_avgdown(hipStream_t st, const DevMeta &M, int b0, int nb, double *phib)
{
    if (nb <= 0) return;
    AMRMG_LAUNCH(k_avgdown, dim3((nb + 3) / 4), dim3(256), 0, st, M, b0, nb, phib);
}

void launch_efield(hipStream_t st, const DevMeta &M, int b0, int nb, const int32_t *list, const double *phib,
                   const double *cp_phi, double *const *E)
{
    if (nb <= 0) return;
    AMRMG_LAUNCH(k_efield, dim3(nb), dim3(256), 0, st, M, b0, nb, phib, cp_phi, E, list);
}

template <class T>
void launch_bottom_cg(hipStream_t st, const DevMeta &M, const int4 *jobs, int njobs, const T *rhs, T *e,
                      double *work, double rtol, int maxit, int *iters)
{
    if (njobs <= 0) return;
    AMRMG_LAUNCH((k_bottom_cg<T>), dim3(njobs), dim3(1024), 0, st, M, jobs, rhs, e, work, rtol, maxit, iters);
}

template <class P, int PPT>
static void launch_deposit_tile(hipStream_t st, unsigned g, bool big, int64_t n, const void *x, const void *y,
                                const void *z, const double *q, const uint32_t *perm, const DepArgs &A,
                                const int64_t *ubase, const int2 *ustr, unsigned long long *nout, void *xs, void *ys,
                                void *zs, double *qs)
{
    // the per-wavefront tile passes for sparse workgroups: measured faster
    // with 9e6 and 1e7 particles (128^3 + 2 and + 3 levels: deposit -10 %
    // and -5 %), slower with 1e6 (64^3 + 2: +3 %, and +15 us in the build),
    // where a launch is a few rounds of workgroups and the serial passes of
    // the sparse ones lengthen it
    const bool waves = n >= DEP_WAVES_MIN;
#define AMRMG_DEPOSIT(TL, WV)                                                                                     \
    AMRMG_LAUNCH((k_deposit<P, PPT, TL, WV>), dim3(g), dim3(256), 0, st, n, (const P *)x, (const P *)y,            \
                 (const P *)z, q, perm, A, ubase, ustr, nout, (P *)xs, (P *)ys, (P *)zs, qs)
    if (big) {
        if (waves) AMRMG_DEPOSIT(DEP_TILE_BIG, true);
        else AMRMG_DEPOSIT(DEP_TILE_BIG, false);
    } else {
        if (waves) AMRMG_DEPOSIT(DEP_TILE, true);
        else AMRMG_DEPOSIT(DEP_TILE, false);
    }
#undef AMRMG_DEPOSIT
}

void launch_deposit(hipStream_t st, int pos_f32, int64_t n, const void *x, const void *y, const void *z,
                    const double *q, const uint32_t *perm, const DepArgs &A, const int64_t *ubase, const int2 *ustr,
                    unsigned long long *nout, void *xs, void *ys, void *zs, double *qs, bool big_tile)
{
    if (n <= 0 || A.nlev <= 0) return;
    // one particle per thread: the most workgroups in flight measured fastest
    // at 1e6 to 1e7 particles (ahead of two and four per thread, whose fewer
    // tile flushes per particle do not make up for the lost parallelism)
    const unsigned g = blocks_for(n, 256);
    if (pos_f32)
        launch_deposit_tile<float, 1>(st, g, big_tile, n, x, y, z, q, perm, A, ubase, ustr, nout, xs, ys, zs, qs);
    else
        launch_deposit_tile<double, 1>(st, g, big_tile, n, x, y, z, q, perm, A, ubase, ustr, nout, xs, ys, zs, qs);
}

template <class P, bool ORD>
static void launch_gather_t(hipStream_t st, unsigned g, int64_t n, const void *x, const void *y, const void *z,
                            const uint32_t *perm, const GatherArgs &G, const int64_t *ubase, const int2 *ustr,
                            double *Ex, double *Ey, double *Ez, double4 *rec)
{
    AMRMG_LAUNCH((k_gather<P, ORD>), dim3(g), dim3(256), 0, st, n, (const P *)x, (const P *)y, (const P *)z, perm, G,
                 ubase, ustr, Ex, Ey, Ez, rec);
}

void launch_gather(hipStream_t st, int pos_f32, int64_t n, const void *x, const void *y, const void *z,
                   const uint32_t *perm, const uint32_t *iperm, const GatherArgs &G, const int64_t *ubase,
                   const int2 *ustr, double *Ex, double *Ey, double *Ez, double4 *rec, bool ordered)
{
    if (n <= 0) return;
    unsigned g = blocks_for(n, 256);
    if (!perm || !iperm) rec = nullptr;
    if (ordered && perm) {
        if (pos_f32)
            launch_gather_t<float, true>(st, g, n, x, y, z, perm, G, ubase, ustr, Ex, Ey, Ez, rec);
        else
            launch_gather_t<double, true>(st, g, n, x, y, z, perm, G, ubase, ustr, Ex, Ey, Ez, rec);
    } else if (pos_f32) {
        launch_gather_t<float, false>(st, g, n, x, y, z, perm, G, ubase, ustr, Ex, Ey, Ez, rec);
    } else {
        launch_gather_t<double, false>(st, g, n, x, y, z, perm, G, ubase, ustr, Ex, Ey, Ez, rec);
    }
    if (rec) AMRMG_LAUNCH(k_unpermute, dim3(g), dim3(256), 0, st, n, iperm, rec, Ex, Ey, Ez);
}

void launch_tag(hipStream_t st, const double *v, int64_t n, double lambda, double *scratch, uint8_t *tags)
{
    if (n <= 0) return;
    int parts = (int)blocks_for(n, 256);
    if (parts > 1024) parts = 1024;
    AMRMG_LAUNCH(k_absmax_part, dim3(parts), dim3(256), 0, st, v, n, scratch + 1);
    AMRMG_LAUNCH(k_absmax_final, dim3(1), dim3(256), 0, st, scratch + 1, parts, scratch);
    AMRMG_LAUNCH(k_tag, dim3(blocks_for(n, 256)), dim3(256), 0, st, v, n, scratch, lambda, tags);
}

// the size rule: one wavefront (brick) per workgroup
int hgs_rule_threads(int) { return 64; }

template <class T>
void launch_hgs(hipStream_t st, const DevMeta &M, int b0, int nb, const T *ein, T *eout, const T *r, T *cp,
                double *phib, double *ffs, int mode, int nt)
{
    if (nb <= 0) return;
    const int bpw = (nt ? nt : hgs_rule_threads(nb)) / 64;
    const dim3 blk(64 * bpw), grid((nb + bpw - 1) / bpw);
#define AMRMG_HGS_BPW(MD, B)                                                                                     \
    if (bpw == B) {                                                                                              \
        AMRMG_LAUNCH((k_hgs<T, MD, B>), grid, blk, 0, st, M, b0, nb, ein, eout, r, cp, phib, ffs);               \
        return;                                                                                                  \
    }
#define AMRMG_HGS(MD)        \
    case MD:                 \
        AMRMG_HGS_BPW(MD, 1) \
        AMRMG_HGS_BPW(MD, 2) \
        AMRMG_HGS_BPW(MD, 4) \
        break;
    switch (mode) {
        AMRMG_HGS(0)
        AMRMG_HGS(HG_ZERO)
        AMRMG_HGS(HG_FFS)
        AMRMG_HGS(HG_ZERO | HG_FFS)
        AMRMG_HGS(HG_PHI)
        AMRMG_HGS(HG_PROL | HG_CPIN)
        AMRMG_HGS(HG_PROL | HG_CPIN | HG_PHI)
    default: break;
    }
#undef AMRMG_HGS
#undef AMRMG_HGS_BPW
    fprintf(stderr, "libamrmg: no sweep kernel for mode %d and %d threads per workgroup\n", mode, 64 * bpw);
    abort();
}

template <class T>
void launch_coarse_cycle(hipStream_t st, const DevMeta &M, const CoarseJob *jobs, int njobs, T *e, T *r,
                         double *work, int nu1, int nu2, double rtol, int maxit, int *iters, double *phib,
                         bool phi_update, int threads_hint)
{
    if (njobs <= 0) return;
    int threads = threads_hint > 0 ? threads_hint : 1024;
    AMRMG_LAUNCH((k_coarse_cycle<T>), dim3(njobs), dim3(threads), 0, st, M, jobs, e, r, work, nu1, nu2, rtol, maxit,
                 iters, phib, (int)phi_update);
}

template <class T>
void launch_direct(hipStream_t st, const DirectJob *jobs, const int2 *planes, int nplanes, const int2 *groups,
                   int ngroups, const double *tab, double *W, const T *r, T *e, double *phib, bool phi_update,
                   int maxdim, const DirectJob *one)
{
    if (nplanes <= 0) return;
    const int rows = (maxdim + 15) & ~15, ld = rows + 1;
    const size_t sp = sizeof(double) * (rows + 16) * ld, sc = sizeof(double) * 2 * DIRECT_COLS * ld;
    static bool attr = false;  // allow more than 64 KiB of dynamic LDS
    if (!attr) {
        const int lim = (int)(sizeof(double) * (DIRECT_DIM + 16) * (DIRECT_DIM + 1));
        (void)hipFuncSetAttribute((const void *)k_dst_plane<T, false>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
        (void)hipFuncSetAttribute((const void *)k_dst_plane<T, true>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
        attr = true;
    }
    // one job: its record goes by value and the workgroups' lists are not read
    const DirectJob J1 = one ? *one : DirectJob{};
    const DirectJob *jl = one ? nullptr : jobs;
    AMRMG_LAUNCH((k_dst_plane<T, false>), dim3(nplanes), dim3(256), sp, st, jl, planes, J1, tab, W, r, e, phib,
                 (int)phi_update, ld, rows);
    AMRMG_LAUNCH(k_dst_column, dim3(ngroups), dim3(256), sc, st, jl, groups, J1, tab, W, ld);
    AMRMG_LAUNCH((k_dst_plane<T, true>), dim3(nplanes), dim3(256), sp, st, jl, planes, J1, tab, W, r, e, phib,
                 (int)phi_update, ld, rows);
}

template <class T>
void launch_copy(hipStream_t st, const T *a, T *b, int64_t n)
{
    if (n <= 0) return;
    AMRMG_LAUNCH((k_copy<T>), dim3(blocks_for(n, 256)), dim3(256), 0, st, a, b, n);
}

void launch_nest_pack(hipStream_t st, const uint8_t *marks, int64_t total, int3 g, const int32_t *cbmap, int3 cn,
                      int3 cnbk, int half, int np, uint64_t *bits)
{
    if (total <= 0) return;
    AMRMG_LAUNCH(k_nest_pack, dim3(blocks_for(total, 256)), dim3(256), 0, st, marks, total, g, cbmap, cn, cnbk, half, np,
                 bits);
}

void launch_mark_blocks(hipStream_t st, const double *rho, int64_t ncell, const int4 *borg, const int64_t *ubase,
                        const int2 *ustr, int nb, double lambda, int nbuf, int half, int3 n, int3 g, double *scratch,
                        uint8_t *marks)
{
    if (nb <= 0) return;
    int parts = (int)blocks_for(ncell, 256);
    if (parts > 1024) parts = 1024;
    AMRMG_LAUNCH(k_absmax_part, dim3(parts), dim3(256), 0, st, rho, ncell, scratch + 1);
    AMRMG_LAUNCH(k_absmax_final, dim3(1), dim3(256), 0, st, scratch + 1, parts, scratch);
    AMRMG_LAUNCH(k_mark_blocks, dim3(nb), dim3(256), 0, st, rho, borg, ubase, ustr, nb, scratch, lambda, nbuf,
                       half, n, g, marks);
}

void launch_zero_levels(hipStream_t st, const DepArgs &A)
{
    int64_t total = 0;
    for (int l = 0; l < A.nlev; ++l) total += A.ncell[l];
    if (total <= 0) return;
    hipLaunchKernelGGL(k_fill_multi, dim3(blocks_for(total, 256)), dim3(256), 0, st, A, total, nullptr);
}

void launch_fill(hipStream_t st, double *v, int64_t n, double val)
{
    if (n <= 0) return;
    AMRMG_LAUNCH(k_fill, dim3(blocks_for(n, 256)), dim3(256), 0, st, v, n, val);
}

#define AMRMG_INST(T)                                                                                            \
    template void launch_outer_residual<T>(hipStream_t, const DevMeta &, int, int, const int32_t *,               \
                                           const double *, const double *, double, const double *, T *, double *, \
                                           int, bool, double *const *, const double *);                           \
    template void launch_cpart_brick<T>(hipStream_t, const DevMeta &, int, int, const T *, T *, const T *,      \
                                        double *);                                                              \
    template void launch_face_sums<T>(hipStream_t, const DevMeta &, int, int, const T *, double *);             \
    template void launch_gsrb<T>(hipStream_t, const DevMeta &, int, int, T *, const T *, const T *, int, bool);  \
    template void launch_jacobi<T>(hipStream_t, const DevMeta &, int, int, const T *, T *, const T *, const T *, \
                                   double, bool);                                                                \
    template void launch_restrict<T>(hipStream_t, const DevMeta &, int, int, const int32_t *, int, const T *,   \
                                     T *, const double *);                                                      \
    template void launch_prolong<T>(hipStream_t, const DevMeta &, int, int, T *);                                \
    template void launch_phi_update<T>(hipStream_t, const DevMeta &, int, int, const int32_t *, double *,         \
                                       const T *);                                                               \
    template void launch_bottom_cg<T>(hipStream_t, const DevMeta &, const int4 *, int, const T *, T *, double *, \
                                      double, int, int *);                                                      \
    template void launch_copy<T>(hipStream_t, const T *, T *, int64_t);                                         \
    template void launch_hgs<T>(hipStream_t, const DevMeta &, int, int, const T *, T *, const T *, T *,         \
                                double *, double *, int, int);                                                       \
    template void launch_coarse_cycle<T>(hipStream_t, const DevMeta &, const CoarseJob *, int, T *, T *,        \
                                         double *, int, int, double, int, int *, double *, bool, int);          \
    template void launch_direct<T>(hipStream_t, const DirectJob *, const int2 *, int, const int2 *, int,         \
                                   const double *, double *, const T *, T *, double *, bool, int, const DirectJob *);
AMRMG_INST(float)
AMRMG_INST(double)
#undef AMRMG_INST

}  // namespace amrmg
