// amrmg_meta.hip -- face data of a new hierarchy generated on the device:
// the Dirichlet values at the centres of the physical-boundary faces of the
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
