// amrmg_particles.cpp -- particle entry points of libamrmg: the visiting
// order, cloud-in-cell deposit and gather (Sec. 1, Fig. 2), and the domain
// transform with the field rescale (Sec. 4.1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "amrmg_state.hpp"


// the deposit's larger LDS tile on levels where a cell of the visiting
// order (that of the last build's particle count) spans 8 or more cells per
// axis
bool big_tile(const amrmg_ctx *ctx, int level)
{
    const int64_t n = ctx->perm_n > 0 ? ctx->perm_n : 1;
    return order_cell_shift(ctx->P.lo, ctx->P.hi, ctx->P.n0, ctx->P.max_level, n) + level >= 3;
}

DepLevel dep_level(const Problem &P, const HostLevel &L, const int32_t *bmap)
{
    DepLevel D{};
    for (int d = 0; d < 3; ++d) {
        D.lo[d] = P.lo[d];
        D.hi[d] = P.hi[d];
        D.h[d] = L.h[d];
        D.n[d] = L.n[d];
        D.nbk[d] = L.nbk[d];
    }
    D.ivol = 1.0 / (L.h[0] * L.h[1] * L.h[2]);
    D.bmap = bmap;
    return D;
}

// Visiting order of the particles (sorted by the Morton code of their cell
// on the finest level's grid) and its inverse; with copy, also room for the
// particles in that order in
// ctx->sorted (charges first, then x, y, z), returned through xs, ys, zs,
// qs: the caller writes the copy (the first tagging deposit does, while it
// reads the particles anyway, or launch_copy_ordered)
amrmg_status compute_order(amrmg_ctx *ctx, int pos_dtype, const void *x, const void *y, const void *z,
                                  const double *q, int64_t n, bool copy, const void **xs, const void **ys,
                                  const void **zs, const double **qs)
{
    ctx->perm = nullptr;
    ctx->iperm = nullptr;
    ctx->perm_n = -1;
    if (n <= 0 || n > (int64_t)0x7fffffff) return AMRMG_OK;
    const amrmg_params &P = ctx->P;
    const size_t sb = order_scratch_bytes(n);
    HIP_TRY(ctx->sort_scratch.ensure(sb));
    HIP_TRY(ctx->sort_vals.ensure(sizeof(uint32_t) * 2 * (size_t)n));
    char *cx = nullptr, *cy = nullptr, *cz = nullptr;
    double *cq = nullptr;
    if (copy) {
        const size_t ps = pos_dtype == AMRMG_POS_F32 ? 4 : 8;
        HIP_TRY(ctx->sorted.ensure((size_t)n * (3 * ps + 8) + 1024));
        char *base = (char *)ctx->sorted.p;
        cq = (double *)base;
        cx = base + align256((size_t)n * 8);
        cy = cx + align256((size_t)n * ps);
        cz = cy + align256((size_t)n * ps);
    }
    uint32_t *perm = (uint32_t *)ctx->sort_vals.p;
    HIP_TRY(particle_order(ctx->st, pos_dtype == AMRMG_POS_F32, n, x, y, z, P.lo, P.hi, P.n0, P.max_level,
                           ctx->sort_scratch.p, ctx->sort_scratch.cap, perm, perm + n));
    ctx->perm = perm;
    ctx->iperm = perm + n;
    ctx->perm_n = n;
    if (copy) {
        *xs = cx;
        *ys = cy;
        *zs = cz;
        *qs = cq;
    }
    return AMRMG_OK;
}

extern "C" amrmg_status amrmg_deposit(amrmg_ctx *ctx, int pos_dtype, const void *x, const void *y, const void *z,
                                      const double *q, int64_t n, double *const *rho, int64_t *n_outside)
{
    if (!ctx) return fail(AMRMG_E_INVALID, "ctx is NULL");
    if (!ctx->built) return fail(AMRMG_E_STATE, "hierarchy not built");
    if (pos_dtype != AMRMG_POS_F64 && pos_dtype != AMRMG_POS_F32) return fail(AMRMG_E_INVALID, "bad pos_dtype");
    if (!rho || n < 0 || (n > 0 && (!x || !y || !z || !q))) return fail(AMRMG_E_INVALID, "bad arguments");
    const Problem &pr = ctx->prob;
    unsigned long long *dout = nullptr;
    if (n_outside) {
        HIP_TRY(ctx->dep_count.ensure(sizeof(unsigned long long)));
        dout = (unsigned long long *)ctx->dep_count.p;
        HIP_TRY(hipMemsetAsync(dout, 0, sizeof(unsigned long long), ctx->st));
    }
    DepArgs A{};
    A.nlev = pr.namr();
    for (int l = 0; l < pr.namr(); ++l) {
        if (!rho[l]) return fail(AMRMG_E_INVALID, "rho[l] is NULL");
        const HostLevel &L = pr.lev[pr.kg + l];
        A.lev[l] = dep_level(pr, L, ctx->ds.d_bmap[l]);
        A.rho[l] = rho[l];
        A.ncell[l] = L.ncells();
    }
    launch_zero_levels(ctx->st, A);
    int64_t cells = 0;
    for (int l = 0; l < A.nlev; ++l) cells += A.ncell[l];
    ctx->prof.begin(AMRMG_K_DEPOSIT);
    launch_deposit(ctx->st, pos_dtype == AMRMG_POS_F32, n, x, y, z, q, ctx->perm_n == n ? ctx->perm : nullptr, A,
                   ctx->ds.M.ubase, ctx->ds.M.ustr, dout, nullptr, nullptr, nullptr, nullptr,
                   big_tile(ctx, pr.namr() - 1));
    ctx->prof.end(AMRMG_K_DEPOSIT, (double)n * (3.0 * (pos_dtype == AMRMG_POS_F32 ? 4 : 8) + 8.0) + 8.0 * (double)cells);
    HIP_TRY(hipGetLastError());
    if (n_outside) {
        unsigned long long h = 0;
        HIP_TRY(hipMemcpyAsync(&h, dout, sizeof(h), hipMemcpyDeviceToHost, ctx->st));
        HIP_TRY(hipStreamSynchronize(ctx->st));
        *n_outside = (int64_t)h;
    }
    return AMRMG_OK;
}

extern "C" amrmg_status amrmg_deposit_built(amrmg_ctx *ctx, double *const *rho, int64_t *n_outside)
{
    if (!ctx) return fail(AMRMG_E_INVALID, "ctx is NULL");
    if (!ctx->built) return fail(AMRMG_E_STATE, "hierarchy not built");
    if (ctx->built_n < 0) return fail(AMRMG_E_STATE, "the last build kept no ordered copy of its particles");
    if (!rho) return fail(AMRMG_E_INVALID, "rho is NULL");
    const Problem &pr = ctx->prob;
    const int64_t n = ctx->built_n;
    const int pos = ctx->built_pos;
    // levels deposited by the build are copied; the others are deposited
    // together from the ordered copy (positions after the charges)
    DepArgs A{};
    int finest = 0;
    for (int l = 0; l < pr.namr(); ++l) {
        if (!rho[l]) return fail(AMRMG_E_INVALID, "rho[l] is NULL");
        const HostLevel &L = pr.lev[pr.kg + l];
        if (l < (int)ctx->lev_rho_ok.size() && ctx->lev_rho_ok[l]) {
            HIP_TRY(hipMemcpyAsync(rho[l], ctx->lev_rho[l].p, sizeof(double) * L.ncells(), hipMemcpyDeviceToDevice,
                                   ctx->st));
            continue;
        }
        finest = l;
        A.lev[A.nlev] = dep_level(pr, L, ctx->ds.d_bmap[l]);
        A.rho[A.nlev] = rho[l];
        A.ncell[A.nlev] = L.ncells();
        ++A.nlev;
    }
    unsigned long long *dout = nullptr;
    const bool level0_kept = !ctx->lev_rho_ok.empty() && ctx->lev_rho_ok[0];
    if (A.nlev > 0) {
        launch_zero_levels(ctx->st, A);
        if (n_outside && !level0_kept) {
            HIP_TRY(ctx->dep_count.ensure(sizeof(unsigned long long)));
            dout = (unsigned long long *)ctx->dep_count.p;
            HIP_TRY(hipMemsetAsync(dout, 0, sizeof(unsigned long long), ctx->st));
        }
        const size_t ps = pos == AMRMG_POS_F32 ? 4 : 8;
        const char *base = (const char *)ctx->sorted.p;
        const double *qs = (const double *)base;
        const char *xs = base + align256((size_t)n * 8), *ys = xs + align256((size_t)n * ps),
                   *zs = ys + align256((size_t)n * ps);
        int64_t cells = 0;
        for (int l = 0; l < A.nlev; ++l) cells += A.ncell[l];
        ctx->prof.begin(AMRMG_K_DEPOSIT);
        launch_deposit(ctx->st, pos == AMRMG_POS_F32, n, xs, ys, zs, qs, nullptr, A, ctx->ds.M.ubase, ctx->ds.M.ustr,
                       dout, nullptr, nullptr, nullptr, nullptr, big_tile(ctx, finest));
        ctx->prof.end(AMRMG_K_DEPOSIT, (double)n * (3.0 * ps + 8.0) + 8.0 * (double)cells);
    }
    HIP_TRY(hipGetLastError());
    if (n_outside) {
        unsigned long long h = 0;
        if (level0_kept) dout = (unsigned long long *)ctx->built_nout.p;
        if (dout) HIP_TRY(hipMemcpyAsync(&h, dout, sizeof(h), hipMemcpyDeviceToHost, ctx->st));
        HIP_TRY(hipStreamSynchronize(ctx->st));
        *n_outside = (int64_t)h;
    }
    return AMRMG_OK;
}

extern "C" amrmg_status amrmg_visiting_order(amrmg_ctx *ctx, uint32_t *perm, int64_t n)
{
    if (!ctx) return fail(AMRMG_E_INVALID, "ctx is NULL");
    if (!ctx->built || ctx->perm_n < 0 || !ctx->perm) return fail(AMRMG_E_STATE, "no visiting order kept");
    if (n != ctx->perm_n) return fail(AMRMG_E_INVALID, "n differs from the build's particle count");
    if (n > 0 && !perm) return fail(AMRMG_E_INVALID, "perm is NULL");
    if (n > 0)
        HIP_TRY(hipMemcpyAsync(perm, ctx->perm, sizeof(uint32_t) * (size_t)n, hipMemcpyDeviceToDevice, ctx->st));
    return AMRMG_OK;
}

// the levels and E pointers a gather reads
static amrmg_status gather_args(const amrmg_ctx *ctx, double *const *E, GatherArgs &G)
{
    const Problem &pr = ctx->prob;
    G = GatherArgs{};
    G.nlev = pr.namr();
    for (int l = 0; l < G.nlev; ++l) {
        G.lev[l] = dep_level(pr, pr.lev[pr.kg + l], ctx->ds.d_bmap[l]);
        for (int d = 0; d < 3; ++d) {
            if (!E[3 * l + d]) return fail(AMRMG_E_INVALID, "E component is NULL");
            G.E[3 * l + d] = E[3 * l + d];
        }
    }
    return AMRMG_OK;
}

// staging records of a gather of n particles in visiting order, or nullptr
// (then the gather writes E at its scattered places directly)
static double4 *gather_records(amrmg_ctx *ctx, int64_t n)
{
    if (n <= 0 || !ctx->iperm) return nullptr;
    if (ctx->gather_rec.ensure(sizeof(double4) * (size_t)n) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return (double4 *)ctx->gather_rec.p;
}

extern "C" amrmg_status amrmg_gather(amrmg_ctx *ctx, int pos_dtype, const void *x, const void *y, const void *z,
                                     int64_t n, double *const *E, double *Ex, double *Ey, double *Ez)
{
    if (!ctx) return fail(AMRMG_E_INVALID, "ctx is NULL");
    if (!ctx->built) return fail(AMRMG_E_STATE, "hierarchy not built");
    if (pos_dtype != AMRMG_POS_F64 && pos_dtype != AMRMG_POS_F32) return fail(AMRMG_E_INVALID, "bad pos_dtype");
    if (!E || n < 0 || (n > 0 && (!x || !y || !z || !Ex || !Ey || !Ez))) return fail(AMRMG_E_INVALID, "bad arguments");
    GatherArgs G;
    ST_TRY(gather_args(ctx, E, G));
    const bool ord = ctx->perm_n == n;
    double4 *rec = ord ? gather_records(ctx, n) : nullptr;
    ctx->prof.begin(AMRMG_K_GATHER);
    launch_gather(ctx->st, pos_dtype == AMRMG_POS_F32, n, x, y, z, ord ? ctx->perm : nullptr,
                  ord ? ctx->iperm : nullptr, G, ctx->ds.M.ubase, ctx->ds.M.ustr, Ex, Ey, Ez, rec);
    ctx->prof.end(AMRMG_K_GATHER, (double)n * (3.0 * (pos_dtype == AMRMG_POS_F32 ? 4 : 8) + 24.0));
    HIP_TRY(hipGetLastError());
    return AMRMG_OK;
}

extern "C" amrmg_status amrmg_gather_built(amrmg_ctx *ctx, double *const *E, double *Ex, double *Ey, double *Ez)
{
    if (!ctx) return fail(AMRMG_E_INVALID, "ctx is NULL");
    if (!ctx->built) return fail(AMRMG_E_STATE, "hierarchy not built");
    if (ctx->built_n < 0) return fail(AMRMG_E_STATE, "the last build kept no ordered copy of its particles");
    const int64_t n = ctx->built_n;
    if (!E || (n > 0 && (!Ex || !Ey || !Ez))) return fail(AMRMG_E_INVALID, "bad arguments");
    if (n > 0 && (ctx->perm_n != n || !ctx->perm)) return fail(AMRMG_E_STATE, "visiting order of the build lost");
    GatherArgs G;
    ST_TRY(gather_args(ctx, E, G));
    const int pos = ctx->built_pos;
    const size_t ps = pos == AMRMG_POS_F32 ? 4 : 8;
    const char *base = (const char *)ctx->sorted.p;
    const char *xs = base + align256((size_t)n * 8), *ys = xs + align256((size_t)n * ps),
               *zs = ys + align256((size_t)n * ps);
    double4 *rec = gather_records(ctx, n);
    ctx->prof.begin(AMRMG_K_GATHER);
    launch_gather(ctx->st, pos == AMRMG_POS_F32, n, xs, ys, zs, ctx->perm, ctx->iperm, G, ctx->ds.M.ubase,
                  ctx->ds.M.ustr, Ex, Ey, Ez, rec, true);
    ctx->prof.end(AMRMG_K_GATHER, (double)n * (3.0 * ps + 4.0 + 24.0));
    HIP_TRY(hipGetLastError());
    return AMRMG_OK;
}

// ---------------------------------------------------------------------------
// domain transform (Sec. 4.1)
// ---------------------------------------------------------------------------
extern "C" amrmg_status amrmg_transform_particles(amrmg_ctx *ctx, int pos_dtype, const void *x, const void *y,
                                                  const void *z, int64_t n, const double *center, const double *l,
                                                  void *xs, void *ys, void *zs, double *s)
{
    if (!ctx) return fail(AMRMG_E_INVALID, "ctx is NULL");
    if (pos_dtype != AMRMG_POS_F64 && pos_dtype != AMRMG_POS_F32) return fail(AMRMG_E_INVALID, "bad pos_dtype");
    if (!center || !l || !s) return fail(AMRMG_E_INVALID, "center, l and s must not be NULL");
    if (n < 0 || (n > 0 && (!x || !y || !z || !xs || !ys || !zs))) return fail(AMRMG_E_INVALID, "bad particle arrays");
    for (int d = 0; d < 3; ++d) {
        if (!(l[d] > 0.0) || !std::isfinite(l[d])) return fail(AMRMG_E_INVALID, "l must be positive and finite");
        if (!std::isfinite(center[d])) return fail(AMRMG_E_INVALID, "center must be finite");
    }
    *s = 0.0;
    if (n == 0) return AMRMG_OK;
    HIP_TRY(ctx->tag_scratch.ensure(sizeof(double) * 1040));
    unsigned long long *d_bits = (unsigned long long *)ctx->tag_scratch.p;
    HIP_TRY(hipMemsetAsync(d_bits, 0, sizeof(unsigned long long), ctx->st));
    launch_domain_scale(ctx->st, pos_dtype == AMRMG_POS_F32, n, x, y, z, center, l, d_bits);
    HIP_TRY(hipGetLastError());
    double v = 0.0;
    HIP_TRY(hipMemcpyAsync(&v, d_bits, sizeof(double), hipMemcpyDeviceToHost, ctx->st));
    HIP_TRY(hipStreamSynchronize(ctx->st));
    if (!std::isfinite(v)) return fail(AMRMG_E_INVALID, "a particle coordinate is not finite");
    if (!(v > 0.0)) return fail(AMRMG_E_INVALID, "every particle sits at the centre: the scale is zero");
    launch_to_computation(ctx->st, pos_dtype == AMRMG_POS_F32, n, x, y, z, center, v, xs, ys, zs);
    HIP_TRY(hipGetLastError());
    *s = v;
    return AMRMG_OK;
}

extern "C" amrmg_status amrmg_rescale_fields(amrmg_ctx *ctx, double s, double *const *phi, double *const *E)
{
    if (!ctx) return fail(AMRMG_E_INVALID, "ctx is NULL");
    if (!ctx->built) return fail(AMRMG_E_STATE, "hierarchy not built");
    if (!(s > 0.0) || !std::isfinite(s)) return fail(AMRMG_E_INVALID, "s must be positive and finite");
    const Problem &pr = ctx->prob;
    const int L = pr.namr();
    for (int l = 0; l < L; ++l) {
        if ((phi && !phi[l]) || (E && (!E[3 * l] || !E[3 * l + 1] || !E[3 * l + 2])))
            return fail(AMRMG_E_INVALID, "a level array is NULL");
    }
    const double s2 = s * s;
    for (int l = 0; l < L; ++l) {
        const int64_t nc = pr.lev[pr.kg + l].ncells();
        if (phi) launch_divide(ctx->st, phi[l], nc, s);
        if (E)
            for (int d = 0; d < 3; ++d) launch_divide(ctx->st, E[3 * l + d], nc, s2);
    }
    HIP_TRY(hipGetLastError());
    return AMRMG_OK;
}
