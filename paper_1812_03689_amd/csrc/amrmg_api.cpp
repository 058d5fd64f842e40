// amrmg_api.cpp -- the C ABI of libamrmg (include/amrmg.h): parameters,
// contexts, the last-error message and per-launch profiling.  The hierarchy
// build is in amrmg_build.cpp, deposit, gather and the domain transform in
// amrmg_particles.cpp, the solve driver in amrmg_solver.cpp.
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

static thread_local std::string g_err;

amrmg_status fail(amrmg_status s, const std::string &m)
{
    g_err = m;
    return s;
}

extern "C" void amrmg_default_params(amrmg_params *p)
{
    std::memset(p, 0, sizeof(*p));
    for (int d = 0; d < 3; ++d) {
        p->lo[d] = 0.0;
        p->hi[d] = 1.0;
        p->n0[d] = 32;
    }
    p->max_level = 2;
    p->ref_ratio = 2;
    p->blocking_factor = 8;
    p->max_grid_size = 32;
    p->n_buffer = 1;
    p->n_proper = 2;
    p->eps0 = 1.0;
    p->n_monopoles = 0;
    p->monopoles = nullptr;
    p->precision = AMRMG_MIXED;
    p->smoother = AMRMG_GSRB;
    p->nu1 = 2;
    p->nu2 = 4;
    p->omega = 6.0 / 7.0;
    p->norm_p = 2;
    p->max_iters = 50;
    p->bottom_rtol = 1e-2;
    p->bottom = AMRMG_BOTTOM_AUTO;
    p->tag_policy = AMRMG_TAG_CHARGE;
    p->robin_d = 0.0;
}

extern "C" const char *amrmg_last_error(void) { return g_err.c_str(); }

static amrmg_status check_params(const amrmg_params *p)
{
    if (!p) return fail(AMRMG_E_INVALID, "params is NULL");
    for (int d = 0; d < 3; ++d) {
        if (p->n0[d] <= 0 || p->n0[d] % 8) return fail(AMRMG_E_INVALID, "n0 must be positive multiples of 8");
        if (!(p->hi[d] > p->lo[d])) return fail(AMRMG_E_INVALID, "domain must have hi > lo");
    }
    if (p->ref_ratio != 2) return fail(AMRMG_E_INVALID, "only refinement ratio 2 is supported");
    if (p->blocking_factor != 8) return fail(AMRMG_E_INVALID, "blocking factor must be 8");
    if (p->max_grid_size < 8 || p->max_grid_size % 8) return fail(AMRMG_E_INVALID, "max_grid_size must be a multiple of 8");
    if (p->max_level < 0 || p->max_level >= AMRMG_MAX_LEVELS) return fail(AMRMG_E_INVALID, "max_level out of range");
    if (p->n_buffer < 0 || p->n_proper < 1) return fail(AMRMG_E_INVALID, "n_buffer >= 0 and n_proper >= 1 required");
    if (!(p->eps0 > 0)) return fail(AMRMG_E_INVALID, "eps0 must be positive");
    if (p->n_monopoles < 0 || (p->n_monopoles > 0 && !p->monopoles)) return fail(AMRMG_E_INVALID, "bad monopoles");
    if (p->precision != AMRMG_FP64 && p->precision != AMRMG_MIXED) return fail(AMRMG_E_INVALID, "bad precision");
    if (p->smoother != AMRMG_GSRB && p->smoother != AMRMG_JACOBI && p->smoother != AMRMG_GSRB_GLOBAL)
        return fail(AMRMG_E_INVALID, "bad smoother");
    if (p->nu1 < 1 || p->nu2 < 1 || p->nu1 > 64 || p->nu2 > 64) return fail(AMRMG_E_INVALID, "nu1, nu2 in [1, 64]");
    if (p->norm_p != 0 && p->norm_p != 1 && p->norm_p != 2) return fail(AMRMG_E_INVALID, "norm_p must be 0, 1 or 2");
    if (p->max_iters < 0) return fail(AMRMG_E_INVALID, "max_iters must be >= 0");
    if (!(p->bottom_rtol > 0 && p->bottom_rtol < 1)) return fail(AMRMG_E_INVALID, "bottom_rtol in (0, 1)");
    if (p->bottom != AMRMG_BOTTOM_AUTO && p->bottom != AMRMG_BOTTOM_CG) return fail(AMRMG_E_INVALID, "bad bottom");
    if (!(p->omega > 0 && p->omega <= 1)) return fail(AMRMG_E_INVALID, "omega in (0, 1]");
    if (p->tag_policy != AMRMG_TAG_CHARGE && p->tag_policy != AMRMG_TAG_POTENTIAL && p->tag_policy != AMRMG_TAG_EFIELD)
        return fail(AMRMG_E_INVALID, "bad tag_policy");
    if (!(p->robin_d >= 0.0) || !std::isfinite(p->robin_d)) return fail(AMRMG_E_INVALID, "robin_d must be >= 0");
    if (p->robin_d > 0.0 && p->n_monopoles > 0)
        return fail(AMRMG_E_INVALID, "Robin boundaries are homogeneous: no Dirichlet monopoles");
    return AMRMG_OK;
}

extern "C" amrmg_status amrmg_create(const amrmg_params *p, void *hip_stream, amrmg_ctx **out)
{
    if (!out) return fail(AMRMG_E_INVALID, "out is NULL");
    *out = nullptr;
    ST_TRY(check_params(p));
    amrmg_ctx *c = new amrmg_ctx();
    c->P = *p;
    if (p->n_monopoles > 0) c->mono.assign(p->monopoles, p->monopoles + 4 * p->n_monopoles);
    c->P.monopoles = nullptr;
    c->st = (hipStream_t)hip_stream;
    // the device of the stream: the no-allocation solve's scratch array is
    // looked up there (once per device, with that device current) and its
    // timing events are made there; a failure only disables that solve
    int dev = -1, cur = -1;
    hipError_t ed = c->st ? hipStreamGetDevice(c->st, &dev) : hipGetDevice(&dev);
    if (ed == hipSuccess && dev >= 0 && hipGetDevice(&cur) == hipSuccess) {
        c->device = dev;
        (void)noalloc_setup(dev);
        if (cur == dev || hipSetDevice(dev) == hipSuccess) {
            for (auto &e : c->ev_solve)
                if (hipEventCreate(&e) != hipSuccess) e = nullptr;
            if (cur != dev) (void)hipSetDevice(cur);
        }
    }
    *out = c;
    return AMRMG_OK;
}

extern "C" void amrmg_destroy(amrmg_ctx *ctx) { delete ctx; }

extern "C" amrmg_status amrmg_profile_enable(amrmg_ctx *ctx, uint32_t mask)
{
    if (!ctx) return fail(AMRMG_E_INVALID, "ctx is NULL");
    HIP_TRY(hipStreamSynchronize(ctx->st));
    ctx->prof.reset(mask);
    return AMRMG_OK;
}

extern "C" amrmg_status amrmg_profile_read(amrmg_ctx *ctx, int32_t kclass, double *ms, int64_t *launches,
                                           double *bytes)
{
    if (!ctx) return fail(AMRMG_E_INVALID, "ctx is NULL");
    if (kclass < 0 || kclass >= AMRMG_K_NCLASS) return fail(AMRMG_E_INVALID, "bad kernel class");
    HIP_TRY(hipStreamSynchronize(ctx->st));
    ctx->prof.flush();
    if (ms) *ms = ctx->prof.tot_ms[kclass];
    if (launches) *launches = ctx->prof.tot_n[kclass];
    if (bytes) *bytes = ctx->prof.tot_bytes[kclass];
    return AMRMG_OK;
}

extern "C" amrmg_status amrmg_profile_launches(amrmg_ctx *ctx, int32_t kclass, double *ms, double *bytes,
                                               int64_t cap, int64_t *count)
{
    if (!ctx || !count) return fail(AMRMG_E_INVALID, "ctx and count must be set");
    if (kclass < 0 || kclass >= AMRMG_K_NCLASS) return fail(AMRMG_E_INVALID, "bad kernel class");
    if (cap < 0 || (cap > 0 && (!ms || !bytes))) return fail(AMRMG_E_INVALID, "cap > 0 needs ms and bytes");
    HIP_TRY(hipStreamSynchronize(ctx->st));
    ctx->prof.flush();
    const auto &k = ctx->prof.kept[kclass];
    *count = (int64_t)k.size();
    for (int64_t i = 0; i < cap && i < (int64_t)k.size(); ++i) {
        ms[i] = k[i].first;
        bytes[i] = k[i].second;
    }
    return AMRMG_OK;
}
