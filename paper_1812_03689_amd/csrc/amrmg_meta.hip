// amrmg_meta.hip -- brick tables and face data of a new hierarchy, built on
// the device.  Face data: the Dirichlet values at the centres of the physical-boundary faces of the
// AMR levels, and for every coarse-fine face the interpolation pattern and
// window cells of each of its 16 coarse cells (Sec. 5.1 of arXiv:1812.03689,
// Tab. bit_pattern and the bilinear table after it).
//
// Pattern selection: the coarse layer across a fine brick face, 5x5 cells
// around each coarse cell, gives a 25-bit availability mask (bit iu + 5 jv,
// set when the coarse cell exists and is not covered by the fine level).  The
// first of the nine quadratic windows (printed order) whose cells are all
// available wins; then the four bilinear windows; else the centre cell alone
// (pattern 13).  Window masks and origins come from the host tables, so host
// and device select from one definition.
#include <hip/hip_runtime.h>

#include "amrmg_internal.hpp"
#include "amrmg_kernels.hpp"

namespace amrmg {

// [0..12]: 25-bit window masks; origins (u0, v0) and node count per pattern
__constant__ uint32_t c_winmask[13];
__constant__ int c_winorg[14 * 3];

hipError_t upload_pattern_tables(const uint32_t *masks13, const int *org14x3)
{
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_winmask), masks13, sizeof(uint32_t) * 13, 0, hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    return hipMemcpyToSymbol(HIP_SYMBOL(c_winorg), org14x3, sizeof(int) * 14 * 3, 0, hipMemcpyHostToDevice);
}

__device__ __forceinline__ void face_axes(int d, int &du, int &dv)
{
    du = (d == 0) ? 1 : 0;
    dv = (d == 2) ? 1 : 2;
}

// global brick id of cell (i, j, k) of level E, or -1 (also outside the level)
__device__ __forceinline__ int brick_of(const EntryDev &E, const int32_t *pool, int i, int j, int k)
{
    if (i < 0 || j < 0 || k < 0 || i >= E.n[0] || j >= E.n[1] || k >= E.n[2]) return -1;
    return pool[E.bmap_off + (i >> 3) + E.nbk[0] * ((j >> 3) + E.nbk[1] * (k >> 3))];
}

// One thread per (coarse-fine face, coarse cell m of its 4x4 coarse cells).
__global__ void __launch_bounds__(256) k_cf_windows(DevMeta M, const EntryDev *ent, const int32_t *pool,
                                                    uint8_t *cf_pat, int32_t *cf_idx, int *err)
{
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= M.ncf * 16) return;
    int t = i >> 4, m = i & 15;
    int ow = M.gf_owner[M.nbc + t];
    int g = ow >> 3, dir = ow & 7, d = dir >> 1;
    bool plus = dir & 1;
    int du, dv;
    face_axes(d, du, dv);
    int4 o = M.org[g];
    const EntryDev F = ent[o.w];
    const EntryDev C = ent[F.crse];
    int O[3] = {o.x, o.y, o.z};
    int ghost = plus ? O[d] + 8 : O[d] - 1;
    int P[3];
    P[d] = ghost >> 1;
    const int cu = O[du] / 2 + (m & 3), cv = O[dv] / 2 + (m >> 2);  // the coarse cell of this thread
    uint32_t mask = 0;
    for (int jv = 0; jv < 5; ++jv)
        for (int iu = 0; iu < 5; ++iu) {
            P[du] = cu + iu - 2;
            P[dv] = cv + jv - 2;
            if (brick_of(C, pool, P[0], P[1], P[2]) < 0) continue;
            if (brick_of(F, pool, 2 * P[0], 2 * P[1], 2 * P[2]) >= 0) continue;
            mask |= 1u << (iu + 5 * jv);
        }
    int pat = 13;
    for (int p = 0; p < 13; ++p)
        if ((mask & c_winmask[p]) == c_winmask[p]) {
            pat = p;
            break;
        }
    cf_pat[i] = (uint8_t)pat;
    const int u0 = c_winorg[3 * pat], v0 = c_winorg[3 * pat + 1], np = c_winorg[3 * pat + 2];
    for (int b = 0; b < 3; ++b)
        for (int a = 0; a < 3; ++a) {
            int ou = 0, ov = 0;  // unused nodes point at the centre (weight 0)
            if (a < np && b < np) {
                ou = u0 + a;
                ov = v0 + b;
            }
            P[du] = cu + ou;
            P[dv] = cv + ov;
            int q = brick_of(C, pool, P[0], P[1], P[2]);
            int gi = 0;
            if (q < 0)
                *err = 1;  // the window leaves the coarser level: nesting is violated
            else
                gi = q * BRICK_CELLS + (P[0] & 7) + 8 * (P[1] & 7) + 64 * (P[2] & 7);
            cf_idx[(size_t)i * 9 + a + 3 * b] = gi;
        }
}

// One thread per (boundary face, face cell): the Dirichlet value of the sum
// of the problem's monopoles q / (4 pi eps0 |x - x_m|) at the face centre;
// zero below AMR level 0 (the correction equation there is homogeneous).
__global__ void __launch_bounds__(256) k_bc_values(DevMeta M, const EntryDev *ent, const double *mono, double *gbc)
{
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= M.nbc * 64) return;
    int t = i >> 6, f = i & 63;
    int ow = M.gf_owner[t];
    int g = ow >> 3, dir = ow & 7, d = dir >> 1;
    bool plus = dir & 1;
    int du, dv;
    face_axes(d, du, dv);
    int4 o = M.org[g];
    const EntryDev E = ent[o.w];
    double v = 0.0;
    if (E.amr >= 0 && E.mono_n > 0) {
        int l[3];
        l[d] = plus ? 7 : 0;
        l[du] = f & 7;
        l[dv] = f >> 3;
        const int O[3] = {o.x, o.y, o.z};
        double x[3];
        for (int a = 0; a < 3; ++a) x[a] = E.lo[a] + ((double)(O[a] + l[a]) + 0.5) * E.h[a];
        x[d] += (plus ? 0.5 : -0.5) * E.h[d];
        for (int k = 0; k < E.mono_n; ++k) {
            const double *q = mono + 4 * (size_t)(E.mono_off + k);
            double dx = x[0] - q[1], dy = x[1] - q[2], dz = x[2] - q[3];
            v += q[0] / (4.0 * 3.14159265358979323846 * E.eps0 * sqrt(dx * dx + dy * dy + dz * dz));
        }
    }
    gbc[i] = v;
}

// ---------------------------------------------------------------------------
// Brick tables of a new hierarchy, built on the device from the box lists
// (the same tables, bit for bit, as the host reference build_meta):
// 1. per brick: origin, level id, caller's-layout base and strides, brick
//    map entry; children and parent cleared;
// 2. per brick: face neighbours (or boundary / coarse-fine markers, counted),
//    parent and octant, the parent's child slot;
// 3. scan of the (boundary, coarse-fine) face counts in brick order;
// 4. per brick: face ids (boundary faces first, then coarse-fine faces, both
//    in brick and face order) with their owners; covered-octant mask;
// 5. per AMR brick: coarse-fine update flag (an uncovered cell next to a
//    covered one), composite cell count per level, the list of AMR bricks;
// 6. scan of the flags and the update list; per-level summary to the host.
// ---------------------------------------------------------------------------
constexpr int32_t NBR_BND = -1, NBR_CF = -2;  // markers between steps 2 and 4

__device__ __forceinline__ int pool_at(const EntryDev &E, const int32_t *pool, int bx, int by, int bz)
{
    return pool[E.bmap_off + bx + E.nbk[0] * (by + E.nbk[1] * bz)];
}

// the brick maps to -1, the composite cell counts and the error flag to 0
__global__ void __launch_bounds__(256) k_meta_clear(int64_t npool, int32_t *pool, int nent, unsigned long long *dof,
                                                    int *err)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < npool) pool[i] = -1;
    if (i < nent) dof[i] = 0;
    if (i == 0) *err = 0;
}

__global__ void __launch_bounds__(256) k_meta_bricks(int nbrick, int nbox, const BoxDev *boxes, const EntryDev *ent,
                                                     int32_t *pool, int4 *org, int64_t *ubase, int2 *ustr,
                                                     int32_t *child, int32_t *par)
{
    const int g = blockIdx.x * 256 + threadIdx.x;
    if (g >= nbrick) return;
    int lo = 0, hi = nbox - 1;  // the last box starting at or before g
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (boxes[mid].g0 <= g) lo = mid;
        else hi = mid - 1;
    }
    const BoxDev B = boxes[lo];
    const int li = g - B.g0, ix = li % B.ext[0], r = li / B.ext[0], iy = r % B.ext[1], iz = r / B.ext[1];
    const int P[3] = {B.lo[0] + ix, B.lo[1] + iy, B.lo[2] + iz};
    const EntryDev &E = ent[B.ent];
    org[g] = make_int4(8 * P[0], 8 * P[1], 8 * P[2], B.ent);
    pool[E.bmap_off + P[0] + E.nbk[0] * (P[1] + E.nbk[1] * P[2])] = g;
    if (E.amr >= 0) {
        ubase[g] = B.uoff + 8 * ix + (int64_t)B.nx * (8 * iy + (int64_t)B.ny * 8 * iz);
        ustr[g] = make_int2(B.nx, B.nx * B.ny);
    } else {
        ubase[g] = 0;
        ustr[g] = make_int2(0, 0);
    }
    par[g] = -1;
#pragma unroll
    for (int o = 0; o < 8; ++o) child[(size_t)g * 8 + o] = -1;
}

__global__ void __launch_bounds__(256) k_meta_links(int nbrick, const EntryDev *ent, const int32_t *pool,
                                                    const int4 *org, int32_t *nbr, int32_t *child, int32_t *par,
                                                    uint64_t *cnt, int *err)
{
    const int g = blockIdx.x * 256 + threadIdx.x;
    if (g >= nbrick) {
        if (g == nbrick) cnt[g] = 0;
        return;
    }
    const int4 o = org[g];
    const EntryDev &E = ent[o.w];
    const int P[3] = {o.x >> 3, o.y >> 3, o.z >> 3};
    uint32_t nbnd = 0, ncf = 0;
#pragma unroll
    for (int dir = 0; dir < 6; ++dir) {
        const int d = dir >> 1;
        int Q[3] = {P[0], P[1], P[2]};
        Q[d] += (dir & 1) ? 1 : -1;
        int32_t v;
        if (Q[d] < 0 || Q[d] >= E.nbk[d]) {
            v = NBR_BND;
            ++nbnd;
        } else {
            v = pool_at(E, pool, Q[0], Q[1], Q[2]);
            if (v < 0) {
                v = NBR_CF;
                ++ncf;
            }
        }
        nbr[(size_t)g * 6 + dir] = v;
    }
    cnt[g] = (uint64_t)nbnd | ((uint64_t)ncf << 32);
    if (E.crse >= 0) {
        const EntryDev &C = ent[E.crse];
        int q = pool_at(C, pool, P[0] >> 1, P[1] >> 1, P[2] >> 1);
        const int oc = (P[0] & 1) | ((P[1] & 1) << 1) | ((P[2] & 1) << 2);
        if (q < 0) {  // no parent: nesting is violated
            *err = 1;
            q = C.b0;
        }
        par[g] = (q << 3) | oc;
        child[(size_t)q * 8 + oc] = g;
    }
}

__global__ void __launch_bounds__(256) k_meta_faces(int nbrick, const EntryDev *ent, const int4 *org,
                                                    const uint64_t *off, int32_t *nbr, int32_t *gf_owner,
                                                    const int32_t *child, uint8_t *cmask)
{
    const int g = blockIdx.x * 256 + threadIdx.x;
    if (g >= nbrick) return;
    const uint64_t of = off[g], tot = off[nbrick];
    uint32_t jb = (uint32_t)of, jc = (uint32_t)(of >> 32);
    const uint32_t nbc = (uint32_t)tot;
#pragma unroll
    for (int dir = 0; dir < 6; ++dir) {
        const int32_t v = nbr[(size_t)g * 6 + dir];
        if (v >= 0) continue;
        const uint32_t gf = v == NBR_BND ? jb++ : nbc + jc++;
        nbr[(size_t)g * 6 + dir] = -1 - (int32_t)gf;
        gf_owner[gf] = (g << 3) | dir;
    }
    uint32_t cm = 0;
    if (ent[org[g].w].amr >= 0)
#pragma unroll
        for (int o = 0; o < 8; ++o) cm |= (child[(size_t)g * 8 + o] >= 0 ? 1u : 0u) << o;
    cmask[g] = (uint8_t)cm;
}

__global__ void __launch_bounds__(256) k_meta_reflux(int nbrick, const EntryDev *ent, const int4 *org,
                                                     const int32_t *nbr, const uint8_t *cmask, uint32_t *flag,
                                                     unsigned long long *dof, int32_t *amr_list)
{
    const int gi = blockIdx.x * 256 + threadIdx.x;
    if (gi == nbrick) flag[gi] = 0;
    if (nbrick <= 0) return;
    // lanes past the last brick take its level and count nothing
    const bool live = gi < nbrick;
    const int g = live ? gi : nbrick - 1;
    const int w = org[g].w;
    const EntryDev &E = ent[w];
    uint32_t want = 0;
    // composite cells: one atomic per wavefront when its bricks share a level
    // (the usual case; per-brick atomics on a few counters would queue)
    const uint32_t cells = live && E.amr >= 0 ? 64 * (8 - __popc((uint32_t)cmask[g])) : 0;
    const int w0 = __shfl(w, 0, 64);
    if (__all(w == w0)) {
        unsigned long long sum = cells;
        for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
        if ((threadIdx.x & 63) == 0 && sum) atomicAdd(&dof[w0], sum);
    } else if (cells) {
        atomicAdd(&dof[w], (unsigned long long)cells);
    }
    if (!live) return;
    if (E.amr >= 0) {
        const uint32_t cm = cmask[g];
        amr_list[E.amr_pos + (g - E.b0)] = g;
        int32_t nb[6];
        uint32_t ncm[6];
        bool near = cm != 0;
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            nb[f] = nbr[(size_t)g * 6 + f];
            ncm[f] = nb[f] >= 0 ? cmask[nb[f]] : 0;
            near = near || ncm[f] != 0;
        }
        // an uncovered octant with a covered face neighbour (in the brick or across a face)
        for (int o = 0; o < 8 && near && !want && cm != 0xFF; ++o) {
            if ((cm >> o) & 1) continue;
            for (int d = 0; d < 3 && !want; ++d) {
                const int od = (o >> d) & 1, on = o ^ (1 << d);
                // the face neighbour inside the brick, then the one across the brick face
                if ((cm >> on) & 1) want = 1;
                const uint32_t across = ncm[2 * d + (od ? 1 : 0)];
                if ((across >> on) & 1) want = 1;
            }
        }
    }
    flag[g] = want;
}

// The update list (every brick with its flag set, at its scanned place),
// and, by the first workgroup, the summary for the host: per level id (cf0,
// ncf, rf0, nrf) and the composite cell count; then the totals (boundary
// faces, coarse-fine faces, update list length, nesting error) and, last,
// the sequence number seq, all in host-visible memory.  (The list's writes
// need not be seen by the host; later kernels are ordered after this one.)
__global__ void __launch_bounds__(256) k_meta_list_summary(int nbrick, const uint32_t *flag, int32_t *reflux, int nent,
                                                           const EntryDev *ent, const uint64_t *off,
                                                           const uint32_t *roff, const unsigned long long *dof,
                                                           const int *err, int32_t *hout, int64_t *hdof,
                                                           unsigned *hseq, unsigned seq)
{
    const int g = blockIdx.x * 256 + threadIdx.x;
    if (g < nbrick && flag[g]) reflux[roff[g]] = g;
    if (blockIdx.x != 0) return;
    for (int e = threadIdx.x; e < nent; e += blockDim.x) {
        const EntryDev &E = ent[e];
        const uint32_t c0 = (uint32_t)(off[E.b0] >> 32), c1 = (uint32_t)(off[E.b0 + E.nb] >> 32);
        hout[4 * e] = (int32_t)c0;
        hout[4 * e + 1] = (int32_t)(c1 - c0);
        hout[4 * e + 2] = (int32_t)roff[E.b0];
        hout[4 * e + 3] = (int32_t)(roff[E.b0 + E.nb] - roff[E.b0]);
        hdof[e] = (int64_t)dof[e];
    }
    if (threadIdx.x == 0) {
        const uint64_t tot = off[nbrick];
        hout[4 * nent] = (int32_t)(uint32_t)tot;
        hout[4 * nent + 1] = (int32_t)(tot >> 32);
        hout[4 * nent + 2] = (int32_t)roff[nbrick];
        hout[4 * nent + 3] = *err;
    }
    // every writer's host-visible stores complete before the sequence number
    if ((int)threadIdx.x < nent || threadIdx.x == 0) __threadfence_system();
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence_system();
        *(volatile unsigned *)hseq = seq;
    }
}

size_t meta_scan_temp_bytes(int nbrick)
{
    const size_t a = scan_temp_bytes<uint64_t>(nbrick + 1), b = scan_temp_bytes<uint32_t>(nbrick + 1);
    return a > b ? a : b;
}

hipError_t launch_meta_build(hipStream_t st, const MetaBuild &B)
{
    const unsigned g1 = (unsigned)((B.nbrick + 256) / 256);  // one thread more than bricks
    const int64_t nclear = B.npool > B.nent ? B.npool : B.nent;
    hipLaunchKernelGGL(k_meta_clear, dim3((unsigned)((nclear + 256) / 256)), dim3(256), 0, st, B.npool, B.pool,
                       B.nent, B.dof, B.err);
    hipError_t e;
    hipLaunchKernelGGL(k_meta_bricks, dim3(g1), dim3(256), 0, st, B.nbrick, B.nbox, B.boxes, B.ent, B.pool, B.org,
                       B.ubase, B.ustr, B.child, B.par);
    hipLaunchKernelGGL(k_meta_links, dim3(g1), dim3(256), 0, st, B.nbrick, B.ent, B.pool, B.org, B.nbr, B.child,
                       B.par, B.cnt, B.err);
    e = exclusive_scan<uint64_t>(st, B.cnt, B.off, B.nbrick + 1, B.temp, B.temp_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_meta_faces, dim3(g1), dim3(256), 0, st, B.nbrick, B.ent, B.org, B.off, B.nbr, B.gf_owner,
                       B.child, B.cmask);
    hipLaunchKernelGGL(k_meta_reflux, dim3(g1), dim3(256), 0, st, B.nbrick, B.ent, B.org, B.nbr, B.cmask, B.flag,
                       B.dof, B.amr_list);
    e = exclusive_scan<uint32_t>(st, B.flag, B.roff, B.nbrick + 1, B.temp, B.temp_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_meta_list_summary, dim3(g1), dim3(256), 0, st, B.nbrick, B.flag, B.reflux, B.nent, B.ent,
                       B.off, B.roff, B.dof, B.err, B.hout, B.hdof, B.hseq, B.seq);
    return hipGetLastError();
}

void launch_face_data(hipStream_t st, const DevMeta &M, const EntryDev *ent, const int32_t *pool,
                      const double *mono, double *gbc, uint8_t *cf_pat, int32_t *cf_idx, int *err)
{
    if (M.nbc > 0)
        hipLaunchKernelGGL(k_bc_values, dim3((M.nbc * 64 + 255) / 256), dim3(256), 0, st, M, ent, mono, gbc);
    if (M.ncf > 0)
        hipLaunchKernelGGL(k_cf_windows, dim3((M.ncf * 16 + 255) / 256), dim3(256), 0, st, M, ent, pool, cf_pat,
                           cf_idx, err);
}

}  // namespace amrmg
