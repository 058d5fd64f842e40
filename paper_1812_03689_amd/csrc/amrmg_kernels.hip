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
#include <hip/hip_runtime.h>

#include "amrmg_internal.hpp"
#include "amrmg_kernels.hpp"

namespace amrmg {

// step-1 weights of the coarse-fine ghost, already multiplied by the step-2
// weight 8/15 of the coarse node: [pattern 0..13][quadrant 0..3][node 0..8]
__constant__ double c_cfw[14 * 4 * 9];

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

struct UserAcc {  // caller's box-list layout of one level
    const double *base;
    const int64_t *ubase;
    const int2 *ustr;
    __device__ double operator()(int b, const int *l) const
    {
        int2 s = ustr[b];
        return base[ubase[b] + l[0] + (int64_t)s.x * l[1] + (int64_t)s.y * l[2]];
    }
};

struct UserAccL {  // caller's layout, level looked up from the brick
    double *const *p;
    const int4 *org;
    const int64_t *ubase;
    const int2 *ustr;
    __device__ double operator()(int b, const int *l) const
    {
        int2 s = ustr[b];
        return p[org[b].w][ubase[b] + l[0] + (int64_t)s.x * l[1] + (int64_t)s.y * l[2]];
    }
};

// The neighbour value that cell l of brick b sees across face (d, s), written
// as a * u_c + bv:
//   same level (in this brick or the face neighbour brick): a = 0, bv = u_nb
//   physical boundary, Dirichlet ghost 2 g - u_c: a = -1, bv = 2 g (g = 0 when
//     !inhom)
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
        a = -1.0;
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

// sum over a workgroup of 256 threads (op 0: sum, 1: max)
__device__ double block_reduce_256(double v, int op)
{
    __shared__ double sh[4];
    for (int o = 32; o > 0; o >>= 1) {
        double w = __shfl_xor(v, o, 64);
        v = op ? fmax(v, w) : v + w;
    }
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = sh[0];
    for (int i = 1; i < 4; ++i) r = op ? fmax(r, sh[i]) : r + sh[i];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------
// FP64 composite residual (Alg. 1) on a range of bricks of the AMR levels
// ---------------------------------------------------------------------------

// Fine part of the flux through the coarse face (d, s) of a coarse cell whose
// neighbour nl (local cell of coarse brick nb) is covered: the four fine cells
// next to the face and their inner neighbours, and the coarse parts of their
// ghosts.  Returns sum over the 4 fine faces of (u_f/3 + u_in/5 - cpart);
// the coarse operator gets -1/(2 h_d^2) times it.
template <class UF>
__device__ double fine_face_sum(const DevMeta &M, int nb, const int *nl, int d, int s, const UF &uf,
                                const double *cp)
{
    int F = M.child[nb * 8 + oct_of(nl[0], nl[1], nl[2])];
    int4 co = M.org[nb], fo = M.org[F];
    int gn[3] = {co.x + nl[0], co.y + nl[1], co.z + nl[2]};
    int fob[3] = {fo.x, fo.y, fo.z};
    int du, dv;
    transverse(d, du, dv);
    int gfc = -1 - M.nbr[F * 6 + 2 * d + (s < 0)];  // F's face towards the coarse cell
    size_t cf = (size_t)(gfc - M.nbc);
    double sum = 0.0;
    for (int bb = 0; bb < 2; ++bb)
        for (int aa = 0; aa < 2; ++aa) {
            int fl[3];
            fl[d] = 2 * gn[d] + (s > 0 ? 0 : 1) - fob[d];
            fl[du] = 2 * gn[du] + aa - fob[du];
            fl[dv] = 2 * gn[dv] + bb - fob[dv];
            int f2[3] = {fl[0], fl[1], fl[2]};
            f2[d] += s;
            int t = fl[du] + 8 * fl[dv];
            double c = cp ? cp[cf * 64 + t] : 0.0;
            sum += (1.0 / 3.0) * uf(F, fl) + 0.2 * uf(F, f2) - c;
        }
    return sum;
}

template <class T, bool ZERO>
__global__ void __launch_bounds__(256) k_outer_residual(DevMeta M, int b0, int nb, double *const *phi, double *const *rho,
                                                        double inv_eps0, const double *cp_phi, T *r_out,
                                                        double *part, int norm_p, const int32_t *list,
                                                        double *const *r_user)
{
    int b = pick_brick(b0, nb, list, blockIdx.x);
    int4 o = M.org[b];
    int lev = o.w;
    LevelConst L = M.lc[lev];
    uint8_t cm = M.cmask[b];
    UserAcc uacc{phi[lev], M.ubase, M.ustr};
    UserAccL facc{phi, M.org, M.ubase, M.ustr};
    const double *rh = rho[lev];
    int64_t ub = M.ubase[b];
    int2 us = M.ustr[b];
    double acc = 0.0;
    for (int c = threadIdx.x; c < BRICK_CELLS; c += 256) {
        int lc[3] = {c & 7, (c >> 3) & 7, c >> 6};
        int64_t ui = ub + lc[0] + (int64_t)us.x * lc[1] + (int64_t)us.y * lc[2];
        double rv = 0.0;
        if (!((cm >> oct_of(lc[0], lc[1], lc[2])) & 1)) {
            double uc = 0.0;
            if (!ZERO) uc = uacc(b, lc);
            double Au = 0.0;
            for (int d = 0; d < 3; ++d)
                for (int s = -1; s <= 1; s += 2) {
                    int nl[3] = {lc[0], lc[1], lc[2]};
                    int n = nl[d] + s, nbk = b;
                    bool cov = false;
                    if (n >= 0 && n < BRICK) {
                        nl[d] = n;
                        cov = (cm >> oct_of(nl[0], nl[1], nl[2])) & 1;
                    } else {
                        int f = M.nbr[b * 6 + 2 * d + (s > 0)];
                        if (f >= 0) {
                            nl[d] = (s > 0) ? 0 : BRICK - 1;
                            nbk = f;
                            cov = (M.cmask[f] >> oct_of(nl[0], nl[1], nl[2])) & 1;
                        }
                    }
                    if (cov) {
                        if (!ZERO) Au += -0.5 * L.ih2[d] * fine_face_sum(M, nbk, nl, d, s, facc, cp_phi);
                    } else {
                        double a, bv;
                        if (ZERO)
                            face_nb(M, b, lc, d, s, ZeroAcc{}, nullptr, nullptr, true, a, bv);
                        else
                            face_nb(M, b, lc, d, s, uacc, cp_phi, nullptr, true, a, bv);
                        Au += L.ih2[d] * ((1.0 - a) * uc - bv);
                    }
                }
            rv = rh[ui] * inv_eps0 - Au;
        }
        if (r_out) r_out[(size_t)b * BRICK_CELLS + c] = (T)rv;
        if (r_user) r_user[lev][ui] = rv;
        double av = fabs(rv);
        acc = norm_p == 2 ? acc + av * av : norm_p == 1 ? acc + av : fmax(acc, av);
    }
    acc = block_reduce_256(acc, norm_p == 0);
    if (threadIdx.x == 0) part[b] = acc;
}

// norm of each listed brick range (one AMR level of one problem) from the
// per-brick partials, in a fixed order
__global__ void k_level_norms(const int2 *ranges, int n, const double *part, double *out, int norm_p)
{
    int l = blockIdx.x;
    if (l >= n) return;
    int b0 = ranges[l].x, b1 = ranges[l].x + ranges[l].y;
    double acc = 0.0;
    for (int b = b0 + (int)threadIdx.x; b < b1; b += 256) acc = norm_p == 0 ? fmax(acc, part[b]) : acc + part[b];
    acc = block_reduce_256(acc, norm_p == 0);
    if (threadIdx.x == 0) out[l] = norm_p == 2 ? sqrt(acc) : acc;
}

// ---------------------------------------------------------------------------
// coarse parts of the coarse-fine ghosts (step 1 of Eq. 2d_lagrange, times
// the step-2 weight 8/15)
// ---------------------------------------------------------------------------
struct SrcUser {
    double *const *p;
    const int4 *org;
    const int64_t *ubase;
    const int2 *ustr;
    __device__ double operator()(int32_t g) const
    {
        int b = g >> 9, c = g & 511;
        int2 s = ustr[b];
        return p[org[b].w][ubase[b] + (c & 7) + (int64_t)s.x * ((c >> 3) & 7) + (int64_t)s.y * (c >> 6)];
    }
};
template <class T>
struct SrcBrick {
    const T *u;
    __device__ double operator()(int32_t g) const { return (double)u[g]; }
};

template <class T, class S>
__global__ void __launch_bounds__(256) k_cpart(DevMeta M, int cf0, int ncf, S src, T *cp)
{
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= ncf * 16) return;
    int cf = cf0 + (i >> 4), m = i & 15;
    size_t e = (size_t)cf * 16 + m;
    int pat = M.cf_pat[e];
    double v[9];
    for (int w = 0; w < 9; ++w) v[w] = src(M.cf_idx[e * 9 + w]);
    int mu = m & 3, mv = m >> 2;
    for (int q = 0; q < 4; ++q) {
        const double *W = c_cfw + (pat * 4 + q) * 9;
        double s = 0.0;
        for (int w = 0; w < 9; ++w) s += W[w] * v[w];
        int t = (2 * mu + (q & 1)) + 8 * (2 * mv + (q >> 1));
        cp[(size_t)cf * 64 + t] = (T)s;
    }
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
    int b = b0 + xcd_remap(blockIdx.x, nb);
    int lev = M.org[b].w;
    LevelConst L = M.lc[lev];
    int t = threadIdx.x;
    int z = t >> 5, y = (t >> 2) & 7, xx = (t & 3) << 1;
    int x = xx + (((y + z) & 1) ^ colour);  // brick origins are even
    int lc[3] = {x, y, z};
    size_t li = (size_t)b * BRICK_CELLS + x + 8 * y + 64 * z;
    double num = (double)r[li], den = 0.0;
    const double *cpd = CpPtr<T>::d(cp);
    const float *cpf = CpPtr<T>::f(cp);
    for (int d = 0; d < 3; ++d)
        for (int s = -1; s <= 1; s += 2) {
            double a, bv;
            if (init)
                face_nb(M, b, lc, d, s, ZeroAcc{}, nullptr, nullptr, false, a, bv);
            else
                face_nb(M, b, lc, d, s, BrickAcc<T>{e}, cpd, cpf, false, a, bv);
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
    int b = b0 + xcd_remap(blockIdx.x, nb);
    int lev = M.org[b].w;
    LevelConst L = M.lc[lev];
    const double *cpd = CpPtr<T>::d(cp);
    const float *cpf = CpPtr<T>::f(cp);
    for (int c = threadIdx.x; c < BRICK_CELLS; c += 256) {
        int lc[3] = {c & 7, (c >> 3) & 7, c >> 6};
        size_t li = (size_t)b * BRICK_CELLS + c;
        double num = (double)r[li], den = 0.0;
        for (int d = 0; d < 3; ++d)
            for (int s = -1; s <= 1; s += 2) {
                double a, bv;
                if (init)
                    face_nb(M, b, lc, d, s, ZeroAcc{}, nullptr, nullptr, false, a, bv);
                else
                    face_nb(M, b, lc, d, s, BrickAcc<T>{ein}, cpd, cpf, false, a, bv);
                num += L.ih2[d] * bv;
                den += L.ih2[d] * (1.0 - a);
            }
        double uc = init ? 0.0 : (double)ein[li];
        eout[li] = (T)(uc + omega * (num / den - uc));
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
// (Alg. 3, restriction onto the covered domain; e^{l-1} = 0 at that point).
// Four fine bricks per workgroup, one coarse cell per thread.
template <class T>
__global__ void __launch_bounds__(256) k_restrict(DevMeta M, int b0, int nb, const T *e, const T *r, T *rc)
{
    int nwg = (nb + 3) >> 2;
    int w = xcd_remap(blockIdx.x, nwg);
    int k = w * 4 + (threadIdx.x >> 6);
    if (k >= nb) return;
    int b = b0 + k;
    int lev = M.org[b].w;
    LevelConst L = M.lc[lev];
    int t = threadIdx.x & 63;
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
    rc[(size_t)pb * BRICK_CELLS + X + 8 * Y + 64 * Z] = (T)(0.125 * sum);
}

// Uncovered coarse cells next to covered ones: r -= B_fine e^l, i.e. add
// 1/(2 h_d^2) * sum over the 4 fine faces of (e_f/3 + e_in/5) per coarse-fine
// face (the coarse correction is still zero).  FP64 arithmetic.
template <class T>
__global__ void __launch_bounds__(256) k_reflux(DevMeta M, const int32_t *list, int n, const T *e, T *r)
{
    int b = list[xcd_remap(blockIdx.x, n)];
    int lev = M.org[b].w;
    LevelConst L = M.lc[lev];
    uint8_t cm = M.cmask[b];
    for (int c = threadIdx.x; c < BRICK_CELLS; c += 256) {
        int lc[3] = {c & 7, (c >> 3) & 7, c >> 6};
        if ((cm >> oct_of(lc[0], lc[1], lc[2])) & 1) continue;
        double add = 0.0;
        for (int d = 0; d < 3; ++d)
            for (int s = -1; s <= 1; s += 2) {
                int nl[3] = {lc[0], lc[1], lc[2]};
                int nn = nl[d] + s, nbk = b;
                bool cov = false;
                if (nn >= 0 && nn < BRICK) {
                    nl[d] = nn;
                    cov = (cm >> oct_of(nl[0], nl[1], nl[2])) & 1;
                } else {
                    int f = M.nbr[b * 6 + 2 * d + (s > 0)];
                    if (f >= 0) {
                        nl[d] = (s > 0) ? 0 : BRICK - 1;
                        nbk = f;
                        cov = (M.cmask[f] >> oct_of(nl[0], nl[1], nl[2])) & 1;
                    }
                }
                if (cov) add += 0.5 * L.ih2[d] * fine_face_sum(M, nbk, nl, d, s, BrickAcc<T>{e}, nullptr);
            }
        if (add != 0.0) {
            size_t li = (size_t)b * BRICK_CELLS + c;
            r[li] = (T)((double)r[li] + add);
        }
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

// phi += e on AMR bricks (FP64 accumulation of the correction)
template <class T>
__global__ void __launch_bounds__(256) k_phi_update(DevMeta M, int b0, int nb, double *const *phi, const T *e,
                                                    const int32_t *list)
{
    int b = pick_brick(b0, nb, list, blockIdx.x);
    double *ph = phi[M.org[b].w];
    int64_t ub = M.ubase[b];
    int2 us = M.ustr[b];
    for (int c = threadIdx.x; c < BRICK_CELLS; c += 256) {
        int64_t ui = ub + (c & 7) + (int64_t)us.x * ((c >> 3) & 7) + (int64_t)us.y * (c >> 6);
        ph[ui] += (double)e[(size_t)b * BRICK_CELLS + c];
    }
}

// phi^{l} <- U phi^l + R phi^{l+1} for the covered cells under a range of
// fine bricks (Alg. 2, average down)
__global__ void __launch_bounds__(256) k_avgdown(DevMeta M, int b0, int nb, double *const *phi)
{
    int nwg = (nb + 3) >> 2;
    int w = xcd_remap(blockIdx.x, nwg);
    int k = w * 4 + (threadIdx.x >> 6);
    if (k >= nb) return;
    int b = b0 + k;
    int lev = M.org[b].w;
    int t = threadIdx.x & 63;
    int cx = t & 3, cy = (t >> 2) & 3, cz = t >> 4;
    UserAcc uf{phi[lev], M.ubase, M.ustr};
    double s = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                int l[3] = {2 * cx + dx, 2 * cy + dy, 2 * cz + dz};
                s += uf(b, l);
            }
    int par = M.par[b];
    int pb = par >> 3, oc = par & 7;
    int X = (oc & 1) * 4 + cx, Y = ((oc >> 1) & 1) * 4 + cy, Z = (oc >> 2) * 4 + cz;
    int2 us = M.ustr[pb];
    phi[M.org[pb].w][M.ubase[pb] + X + (int64_t)us.x * Y + (int64_t)us.y * Z] = 0.125 * s;
}

// E_d = -(u_+ - u_-) / (2 h_d) on every cell of a range of AMR bricks
__global__ void __launch_bounds__(256) k_efield(DevMeta M, int b0, int nb, double *const *phi, const double *cp_phi,
                                                double *const *E, const int32_t *list)
{
    int b = pick_brick(b0, nb, list, blockIdx.x);
    int lev = M.org[b].w;
    LevelConst L = M.lc[lev];
    UserAcc uacc{phi[lev], M.ubase, M.ustr};
    int64_t ub = M.ubase[b];
    int2 us = M.ustr[b];
    for (int c = threadIdx.x; c < BRICK_CELLS; c += 256) {
        int lc[3] = {c & 7, (c >> 3) & 7, c >> 6};
        int64_t ui = ub + lc[0] + (int64_t)us.x * lc[1] + (int64_t)us.y * lc[2];
        double uc = uacc(b, lc);
        for (int d = 0; d < 3; ++d) {
            double a, bv, up, um;
            face_nb(M, b, lc, d, +1, uacc, cp_phi, nullptr, true, a, bv);
            up = a * uc + bv;
            face_nb(M, b, lc, d, -1, uacc, cp_phi, nullptr, true, a, bv);
            um = a * uc + bv;
            E[3 * lev + d][ui] = -(up - um) / (2.0 * L.h[d]);
        }
    }
}

// ---------------------------------------------------------------------------
// CG on the coarsest grid, one workgroup of 1024 threads (FP64 vectors and
// dot products).  Homogeneous Dirichlet data, no coarse-fine faces.
// ---------------------------------------------------------------------------
__device__ double block_reduce_1024(double v)
{
    __shared__ double sh[16];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    for (int i = 0; i < 16; ++i) r += sh[i];
    __syncthreads();
    return r;
}

// one workgroup per job: jobs[i] = (first brick, bricks, offset of its four
// work vectors in doubles)
template <class T>
__global__ void __launch_bounds__(1024) k_bottom_cg(DevMeta M, const int4 *jobs, const T *rhs, T *e, double *work,
                                                    double rtol, int maxit, int *iters)
{
    int4 jb = jobs[blockIdx.x];
    const int b0 = jb.x, nb = jb.y;
    const int n = nb * BRICK_CELLS;
    double *x = work + jb.z, *r = x + n, *p = x + 2 * (size_t)n, *q = x + 3 * (size_t)n;
    double rho = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) {
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
    while (it < maxit && rho > stop && rho > 0.0) {
        double pq = 0.0;
        for (int i = threadIdx.x; i < n; i += 1024) {
            int b = b0 + (i >> 9), c = i & 511;
            int lc[3] = {c & 7, (c >> 3) & 7, c >> 6};
            LevelConst L = M.lc[M.org[b].w];
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
        for (int i = threadIdx.x; i < n; i += 1024) {
            x[i] += alpha * p[i];
            double rv = r[i] - alpha * q[i];
            r[i] = rv;
            rho1 += rv * rv;
        }
        rho1 = block_reduce_1024(rho1);
        double beta = rho1 / rho;
        for (int i = threadIdx.x; i < n; i += 1024) p[i] = r[i] + beta * p[i];
        rho = rho1;
        ++it;
        __syncthreads();
    }
    for (int i = threadIdx.x; i < n; i += 1024) e[(size_t)b0 * BRICK_CELLS + i] = (T)x[i];
    if (threadIdx.x == 0 && iters) atomicMax(iters, it);
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

template <class P>
__global__ void __launch_bounds__(256) k_deposit(int64_t n, const P *x, const P *y, const P *z, const double *q,
                                                 DepLevel D, const int64_t *ubase, const int2 *ustr, double *rho,
                                                 unsigned long long *nout)
{
    int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    int i0[3], i1[3];
    double f[3];
    if (!cic_stencil<P>(D, (double)x[p], (double)y[p], (double)z[p], i0, i1, f)) {
        if (nout) atomicAdd(nout, 1ull);
        return;
    }
    double qv = q[p] * D.ivol;
    for (int c = 0; c < 8; ++c) {
        int ii = (c & 1) ? i1[0] : i0[0];
        int jj = (c & 2) ? i1[1] : i0[1];
        int kk = (c & 4) ? i1[2] : i0[2];
        double w = ((c & 1) ? f[0] : 1.0 - f[0]) * ((c & 2) ? f[1] : 1.0 - f[1]) * ((c & 4) ? f[2] : 1.0 - f[2]);
        int64_t u = user_index(D, ubase, ustr, ii, jj, kk);
        if (u >= 0) atomicAdd(rho + u, qv * w);
    }
}

template <class P>
__global__ void __launch_bounds__(256) k_gather(int64_t n, const P *x, const P *y, const P *z, GatherArgs G,
                                                const int64_t *ubase, const int2 *ustr, double *Ex, double *Ey,
                                                double *Ez)
{
    int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    double X = (double)x[p], Y = (double)y[p], Z = (double)z[p];
    double e[3] = {0.0, 0.0, 0.0};
    for (int l = G.nlev - 1; l >= 0; --l) {
        const DepLevel &D = G.lev[l];
        int i0[3], i1[3];
        double f[3];
        if (!cic_stencil<P>(D, X, Y, Z, i0, i1, f)) break;
        int64_t u[8];
        bool ok = true;
        for (int c = 0; c < 8; ++c) {
            u[c] = user_index(D, ubase, ustr, (c & 1) ? i1[0] : i0[0], (c & 2) ? i1[1] : i0[1],
                              (c & 4) ? i1[2] : i0[2]);
            ok = ok && u[c] >= 0;
        }
        if (!ok) continue;
        for (int c = 0; c < 8; ++c) {
            double w = ((c & 1) ? f[0] : 1.0 - f[0]) * ((c & 2) ? f[1] : 1.0 - f[1]) *
                       ((c & 4) ? f[2] : 1.0 - f[2]);
            for (int d = 0; d < 3; ++d) e[d] += w * G.E[3 * l + d][u[c]];
        }
        break;
    }
    Ex[p] = e[0];
    Ey[p] = e[1];
    Ez[p] = e[2];
}

// max |rho| over a level (per-workgroup partials, then one workgroup)
__global__ void __launch_bounds__(256) k_absmax_part(const double *v, int64_t n, double *part)
{
    double m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        m = fmax(m, fabs(v[i]));
    m = block_reduce_256(m, 1);
    if (threadIdx.x == 0) part[blockIdx.x] = m;
}

__global__ void __launch_bounds__(256) k_absmax_final(const double *part, int n, double *out)
{
    double m = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) m = fmax(m, part[i]);
    m = block_reduce_256(m, 1);
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
void launch_outer_residual(hipStream_t st, const DevMeta &M, int b0, int nb, const int32_t *list,
                           double *const *phi, double *const *rho, double inv_eps0, const double *cp_phi, T *r_out,
                           double *part, int norm_p, bool zero_phi, double *const *r_user)
{
    if (nb <= 0) return;
    if (zero_phi)
        hipLaunchKernelGGL((k_outer_residual<T, true>), dim3(nb), dim3(256), 0, st, M, b0, nb, phi, rho, inv_eps0,
                           cp_phi, r_out, part, norm_p, list, r_user);
    else
        hipLaunchKernelGGL((k_outer_residual<T, false>), dim3(nb), dim3(256), 0, st, M, b0, nb, phi, rho,
                           inv_eps0, cp_phi, r_out, part, norm_p, list, r_user);
}

void launch_level_norms(hipStream_t st, const int2 *ranges, int n, const double *part, double *out, int norm_p)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_level_norms, dim3(n), dim3(256), 0, st, ranges, n, part, out, norm_p);
}

void launch_cpart_user(hipStream_t st, const DevMeta &M, int cf0, int ncf, double *const *phi, double *cp)
{
    if (ncf <= 0) return;
    SrcUser s{phi, M.org, M.ubase, M.ustr};
    hipLaunchKernelGGL((k_cpart<double, SrcUser>), dim3(blocks_for((int64_t)ncf * 16, 256)), dim3(256), 0, st, M,
                       cf0, ncf, s, cp);
}

template <class T>
void launch_cpart_brick(hipStream_t st, const DevMeta &M, int cf0, int ncf, const T *src, T *cp)
{
    if (ncf <= 0) return;
    SrcBrick<T> s{src};
    hipLaunchKernelGGL((k_cpart<T, SrcBrick<T>>), dim3(blocks_for((int64_t)ncf * 16, 256)), dim3(256), 0, st, M,
                       cf0, ncf, s, cp);
}

template <class T>
void launch_gsrb(hipStream_t st, const DevMeta &M, int b0, int nb, T *e, const T *r, const T *cp, int colour,
                 bool init)
{
    if (nb <= 0) return;
    hipLaunchKernelGGL((k_gsrb<T>), dim3(nb), dim3(256), 0, st, M, b0, nb, e, r, cp, colour, (int)init);
}

template <class T>
void launch_jacobi(hipStream_t st, const DevMeta &M, int b0, int nb, const T *ein, T *eout, const T *r, const T *cp,
                   double omega, bool init)
{
    if (nb <= 0) return;
    hipLaunchKernelGGL((k_jacobi<T>), dim3(nb), dim3(256), 0, st, M, b0, nb, ein, eout, r, cp, omega, (int)init);
}

template <class T>
void launch_restrict(hipStream_t st, const DevMeta &M, int b0, int nb, const T *e, const T *r, T *rc)
{
    if (nb <= 0) return;
    hipLaunchKernelGGL((k_restrict<T>), dim3((nb + 3) / 4), dim3(256), 0, st, M, b0, nb, e, r, rc);
}

template <class T>
void launch_reflux(hipStream_t st, const DevMeta &M, const int32_t *list, int n, const T *e, T *r)
{
    if (n <= 0) return;
    hipLaunchKernelGGL((k_reflux<T>), dim3(n), dim3(256), 0, st, M, list, n, e, r);
}

template <class T>
void launch_prolong(hipStream_t st, const DevMeta &M, int b0, int nb, T *e)
{
    if (nb <= 0) return;
    hipLaunchKernelGGL((k_prolong<T>), dim3(nb), dim3(256), 0, st, M, b0, nb, e);
}

template <class T>
void launch_phi_update(hipStream_t st, const DevMeta &M, int b0, int nb, const int32_t *list, double *const *phi,
                       const T *e)
{
    if (nb <= 0) return;
    hipLaunchKernelGGL((k_phi_update<T>), dim3(nb), dim3(256), 0, st, M, b0, nb, phi, e, list);
}

void launch_avgdown(hipStream_t st, const DevMeta &M, int b0, int nb, double *const *phi)
{
    if (nb <= 0) return;
    hipLaunchKernelGGL(k_avgdown, dim3((nb + 3) / 4), dim3(256), 0, st, M, b0, nb, phi);
}

void launch_efield(hipStream_t st, const DevMeta &M, int b0, int nb, const int32_t *list, double *const *phi,
                   const double *cp_phi, double *const *E)
{
    if (nb <= 0) return;
    hipLaunchKernelGGL(k_efield, dim3(nb), dim3(256), 0, st, M, b0, nb, phi, cp_phi, E, list);
}

template <class T>
void launch_bottom_cg(hipStream_t st, const DevMeta &M, const int4 *jobs, int njobs, const T *rhs, T *e,
                      double *work, double rtol, int maxit, int *iters)
{
    if (njobs <= 0) return;
    hipLaunchKernelGGL((k_bottom_cg<T>), dim3(njobs), dim3(1024), 0, st, M, jobs, rhs, e, work, rtol, maxit, iters);
}

void launch_deposit(hipStream_t st, int pos_f32, int64_t n, const void *x, const void *y, const void *z,
                    const double *q, const DepLevel &D, const int64_t *ubase, const int2 *ustr, double *rho,
                    unsigned long long *nout)
{
    if (n <= 0) return;
    unsigned g = blocks_for(n, 256);
    if (pos_f32)
        hipLaunchKernelGGL((k_deposit<float>), dim3(g), dim3(256), 0, st, n, (const float *)x, (const float *)y,
                           (const float *)z, q, D, ubase, ustr, rho, nout);
    else
        hipLaunchKernelGGL((k_deposit<double>), dim3(g), dim3(256), 0, st, n, (const double *)x, (const double *)y,
                           (const double *)z, q, D, ubase, ustr, rho, nout);
}

void launch_gather(hipStream_t st, int pos_f32, int64_t n, const void *x, const void *y, const void *z,
                   const GatherArgs &G, const int64_t *ubase, const int2 *ustr, double *Ex, double *Ey, double *Ez)
{
    if (n <= 0) return;
    unsigned g = blocks_for(n, 256);
    if (pos_f32)
        hipLaunchKernelGGL((k_gather<float>), dim3(g), dim3(256), 0, st, n, (const float *)x, (const float *)y,
                           (const float *)z, G, ubase, ustr, Ex, Ey, Ez);
    else
        hipLaunchKernelGGL((k_gather<double>), dim3(g), dim3(256), 0, st, n, (const double *)x, (const double *)y,
                           (const double *)z, G, ubase, ustr, Ex, Ey, Ez);
}

void launch_tag(hipStream_t st, const double *v, int64_t n, double lambda, double *scratch, uint8_t *tags)
{
    if (n <= 0) return;
    int parts = (int)blocks_for(n, 256);
    if (parts > 1024) parts = 1024;
    hipLaunchKernelGGL(k_absmax_part, dim3(parts), dim3(256), 0, st, v, n, scratch + 1);
    hipLaunchKernelGGL(k_absmax_final, dim3(1), dim3(256), 0, st, scratch + 1, parts, scratch);
    hipLaunchKernelGGL(k_tag, dim3(blocks_for(n, 256)), dim3(256), 0, st, v, n, scratch, lambda, tags);
}

template <class T>
void launch_copy(hipStream_t st, const T *a, T *b, int64_t n)
{
    if (n <= 0) return;
    hipLaunchKernelGGL((k_copy<T>), dim3(blocks_for(n, 256)), dim3(256), 0, st, a, b, n);
}

void launch_fill(hipStream_t st, double *v, int64_t n, double val)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(n, 256)), dim3(256), 0, st, v, n, val);
}

#define AMRMG_INST(T)                                                                                            \
    template void launch_outer_residual<T>(hipStream_t, const DevMeta &, int, int, const int32_t *,               \
                                           double *const *, double *const *, double, const double *, T *,         \
                                           double *, int, bool, double *const *);                                 \
    template void launch_cpart_brick<T>(hipStream_t, const DevMeta &, int, int, const T *, T *);                \
    template void launch_gsrb<T>(hipStream_t, const DevMeta &, int, int, T *, const T *, const T *, int, bool);  \
    template void launch_jacobi<T>(hipStream_t, const DevMeta &, int, int, const T *, T *, const T *, const T *, \
                                   double, bool);                                                                \
    template void launch_restrict<T>(hipStream_t, const DevMeta &, int, int, const T *, const T *, T *);         \
    template void launch_reflux<T>(hipStream_t, const DevMeta &, const int32_t *, int, const T *, T *);          \
    template void launch_prolong<T>(hipStream_t, const DevMeta &, int, int, T *);                                \
    template void launch_phi_update<T>(hipStream_t, const DevMeta &, int, int, const int32_t *, double *const *, \
                                       const T *);                                                               \
    template void launch_bottom_cg<T>(hipStream_t, const DevMeta &, const int4 *, int, const T *, T *, double *, \
                                      double, int, int *);                                                      \
    template void launch_copy<T>(hipStream_t, const T *, T *, int64_t);
AMRMG_INST(float)
AMRMG_INST(double)
#undef AMRMG_INST

}  // namespace amrmg
