// amrmg_api.cpp -- the C ABI of libamrmg (include/amrmg.h): contexts, the
// hierarchy build, deposit and gather, and the solve driver that runs the
// composite AMR multigrid of arXiv:1812.03689 (Alg. 2 and Alg. 3) on the HIP
// kernels of amrmg_kernels.hip.
//
// Solve structure (per outer iteration, Alg. 2):
//   1. FP64 composite residual of every AMR level (Alg. 1) -> per-level norms,
//      read back to the host (the only synchronisation per iteration);
//   2. one V-cycle (Alg. 3) on the correction equation A_comp e = r, stored in
//      T (float in mixed precision, double otherwise), continued below AMR
//      level 0 through geometric coarsenings down to a CG bottom solve;
//   3. phi += e in FP64.
// With T = double this is Alg. 2 as printed (the V-cycle applied to the
// correction form, which is algebraically the same cycle); with T = float it
// is iterative refinement around an FP32 cycle.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "amrmg.h"
#include "amrmg_hier.hpp"
#include "amrmg_kernels.hpp"

using namespace amrmg;

static thread_local std::string g_err;

static amrmg_status fail(amrmg_status s, const std::string &m)
{
    g_err = m;
    return s;
}

#define HIP_TRY(x)                                                                             \
    do {                                                                                       \
        hipError_t e_ = (x);                                                                   \
        if (e_ != hipSuccess) return fail(AMRMG_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// ---------------------------------------------------------------------------
// device copy of merged metadata plus the solve workspace
// ---------------------------------------------------------------------------
struct DevState {
    Meta meta;
    DevMeta M{};
    std::vector<void *> allocs;
    int32_t *d_reflux = nullptr, *d_amr = nullptr;
    int2 *d_ranges = nullptr;  // brick range of each AMR level of each problem
    std::vector<int> range_prob, range_amr;
    int4 *d_jobs = nullptr;
    int njobs = 0;
    size_t cg_doubles = 0;
    double **d_phi = nullptr, **d_rho = nullptr, **d_E = nullptr, **d_rout = nullptr;
    std::vector<double *> h_phi, h_rho, h_E, h_rout;
    // workspace
    void *ws = nullptr;
    size_t ws_bytes = 0;
    bool ws_owned = false;
    int ws_prec = -1;
    void *e = nullptr, *r = nullptr, *et = nullptr, *cpe = nullptr;
    double *cpphi = nullptr, *part = nullptr, *dnorm = nullptr;
    double *cgw = nullptr;
    int *cgit = nullptr;
    double *h_norm = nullptr;  // pinned

    void release()
    {
        for (void *p : allocs) (void)hipFree(p);
        allocs.clear();
        if (ws_owned && ws) (void)hipFree(ws);
        ws = nullptr;
        ws_owned = false;
        ws_bytes = 0;
        ws_prec = -1;
        if (h_norm) (void)hipHostFree(h_norm);
        h_norm = nullptr;
    }
    ~DevState() { release(); }
};

template <class V>
static amrmg_status up(DevState &D, const std::vector<V> &v, V **out)
{
    *out = nullptr;
    if (v.empty()) return AMRMG_OK;
    void *p = nullptr;
    HIP_TRY(hipMalloc(&p, sizeof(V) * v.size()));
    D.allocs.push_back(p);
    HIP_TRY(hipMemcpy(p, v.data(), sizeof(V) * v.size(), hipMemcpyHostToDevice));
    *out = (V *)p;
    return AMRMG_OK;
}

#define ST_TRY(x)                                \
    do {                                         \
        amrmg_status s_ = (x);                   \
        if (s_ != AMRMG_OK) return s_;           \
    } while (0)

static bool g_weights_ok = false;

static amrmg_status upload_meta(DevState &D)
{
    const Meta &m = D.meta;
    if (!g_weights_ok) {
        std::vector<double> W = cf_weight_table();
        HIP_TRY(upload_cf_weights(W.data()));
        g_weights_ok = true;
    }
    int32_t *org = nullptr, *nbr = nullptr, *child = nullptr, *par = nullptr, *ustr = nullptr, *gfo = nullptr,
            *cfi = nullptr;
    uint8_t *cm = nullptr, *cfp = nullptr;
    int64_t *ub = nullptr;
    double *gbc = nullptr;
    ST_TRY(up(D, m.org, &org));
    ST_TRY(up(D, m.nbr, &nbr));
    ST_TRY(up(D, m.child, &child));
    ST_TRY(up(D, m.par, &par));
    ST_TRY(up(D, m.cmask, &cm));
    ST_TRY(up(D, m.ubase, &ub));
    ST_TRY(up(D, m.ustr, &ustr));
    ST_TRY(up(D, m.gf_owner, &gfo));
    ST_TRY(up(D, m.gbc, &gbc));
    ST_TRY(up(D, m.cf_pat, &cfp));
    ST_TRY(up(D, m.cf_idx, &cfi));
    ST_TRY(up(D, m.reflux, &D.d_reflux));
    ST_TRY(up(D, m.amr_bricks, &D.d_amr));
    std::vector<LevelConst> lc(m.ent.size());
    for (size_t i = 0; i < m.ent.size(); ++i)
        for (int d = 0; d < 3; ++d) {
            lc[i].h[d] = m.ent[i].h[d];
            lc[i].ih2[d] = 1.0 / (m.ent[i].h[d] * m.ent[i].h[d]);
        }
    LevelConst *dlc = nullptr;
    ST_TRY(up(D, lc, &dlc));
    D.M.org = (const int4 *)org;
    D.M.nbr = nbr;
    D.M.child = child;
    D.M.par = par;
    D.M.cmask = cm;
    D.M.ubase = ub;
    D.M.ustr = (const int2 *)ustr;
    D.M.gf_owner = gfo;
    D.M.gbc = gbc;
    D.M.cf_pat = cfp;
    D.M.cf_idx = cfi;
    D.M.lc = dlc;
    D.M.nbc = m.nbc;
    D.M.ncf = m.ncf;
    // norm ranges: every AMR level of every problem, entry order
    std::vector<int32_t> rg;
    D.range_prob.clear();
    D.range_amr.clear();
    for (const auto &e : m.ent)
        if (e.amr >= 0) {
            rg.push_back(e.b0);
            rg.push_back(e.nb);
            D.range_prob.push_back(e.prob);
            D.range_amr.push_back(e.amr);
        }
    int32_t *drg = nullptr;
    ST_TRY(up(D, rg, &drg));
    D.d_ranges = (int2 *)drg;
    // bottom solves: the coarsest level of each problem
    std::vector<int32_t> jobs;
    size_t off = 0;
    for (size_t i = 0; i < m.prob_ent.size(); ++i) {
        const auto &e = m.ent[m.prob_ent[i][0]];
        jobs.push_back(e.b0);
        jobs.push_back(e.nb);
        jobs.push_back((int32_t)off);
        jobs.push_back(0);
        off += (size_t)4 * e.nb * BRICK_CELLS;
    }
    int32_t *dj = nullptr;
    ST_TRY(up(D, jobs, &dj));
    D.d_jobs = (int4 *)dj;
    D.njobs = (int)m.prob_ent.size();
    D.cg_doubles = off;
    // per-level pointer tables (filled per call)
    size_t ne = m.ent.size();
    D.h_phi.assign(ne, nullptr);
    D.h_rho.assign(ne, nullptr);
    D.h_rout.assign(ne, nullptr);
    D.h_E.assign(3 * ne, nullptr);
    for (double ***pp : {&D.d_phi, &D.d_rho, &D.d_rout}) {
        void *p = nullptr;
        HIP_TRY(hipMalloc(&p, sizeof(double *) * ne));
        D.allocs.push_back(p);
        *pp = (double **)p;
    }
    {
        void *p = nullptr;
        HIP_TRY(hipMalloc(&p, sizeof(double *) * 3 * ne));
        D.allocs.push_back(p);
        D.d_E = (double **)p;
    }
    if (!D.h_norm) HIP_TRY(hipHostMalloc((void **)&D.h_norm, sizeof(double) * 2 * (D.range_prob.size() + 1)));
    return AMRMG_OK;
}

static size_t ws_need(const DevState &D, int prec)
{
    const Meta &m = D.meta;
    size_t w = prec == AMRMG_MIXED ? 4 : 8;
    size_t nc = (size_t)m.nbrick * BRICK_CELLS;
    size_t s = 0;
    s += 3 * align256(nc * w);                        // e, r, et
    s += align256((size_t)m.ncf * 64 * w + 8);         // coarse parts of the cycle
    s += align256((size_t)m.ncf * 64 * 8 + 8);         // coarse parts of phi
    s += align256((size_t)m.nbrick * 8);               // per-brick partials
    s += align256(sizeof(double) * 2 * (D.range_prob.size() + 1));
    s += align256(D.cg_doubles * 8);
    s += align256(64);
    return s;
}

static amrmg_status ensure_ws(DevState &D, int prec, void *user, size_t user_bytes)
{
    size_t need = ws_need(D, prec);
    char *base = nullptr;
    if (user) {
        if (user_bytes < need) return fail(AMRMG_E_OOM, "caller workspace smaller than amrmg_workspace_size");
        if (D.ws_owned && D.ws) (void)hipFree(D.ws);
        D.ws = user;
        D.ws_owned = false;
        D.ws_bytes = user_bytes;
    } else if (!(D.ws_owned && D.ws && D.ws_bytes >= need)) {
        if (D.ws_owned && D.ws) (void)hipFree(D.ws);
        D.ws = nullptr;
        D.ws_owned = false;
        hipError_t e = hipMalloc(&D.ws, need);
        if (e != hipSuccess) return fail(AMRMG_E_OOM, "workspace allocation failed");
        D.ws_owned = true;
        D.ws_bytes = need;
    }
    base = (char *)D.ws;
    const Meta &m = D.meta;
    size_t w = prec == AMRMG_MIXED ? 4 : 8;
    size_t nc = (size_t)m.nbrick * BRICK_CELLS;
    auto take = [&](size_t bytes) {
        char *p = base;
        base += align256(bytes);
        return (void *)p;
    };
    D.e = take(nc * w);
    D.r = take(nc * w);
    D.et = take(nc * w);
    D.cpe = take((size_t)m.ncf * 64 * w + 8);
    D.cpphi = (double *)take((size_t)m.ncf * 64 * 8 + 8);
    D.part = (double *)take((size_t)m.nbrick * 8);
    D.dnorm = (double *)take(sizeof(double) * 2 * (D.range_prob.size() + 1));
    D.cgw = (double *)take(D.cg_doubles * 8);
    D.cgit = (int *)take(64);
    D.ws_prec = prec;
    return AMRMG_OK;
}

// ---------------------------------------------------------------------------
// per-launch event timing of selected kernel classes
// ---------------------------------------------------------------------------
struct Prof {
    uint32_t mask = 0;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    struct Rec {
        int cls;
        size_t ev;  // index of the start event; end = ev + 1
        double bytes;
    };
    std::vector<Rec> recs;
    hipStream_t st = nullptr;
    size_t pending = (size_t)-1;
    int pending_cls = -1;

    bool on(int cls) const { return (mask >> cls) & 1; }
    void begin(int cls)
    {
        pending = (size_t)-1;
        if (!on(cls) || used + 2 > pool.size()) return;
        pending = used;
        pending_cls = cls;
        (void)hipEventRecord(pool[used], st);
        used += 2;
    }
    void end(int cls, double bytes)
    {
        if (pending == (size_t)-1 || pending_cls != cls) return;
        (void)hipEventRecord(pool[pending + 1], st);
        recs.push_back({cls, pending, bytes});
        pending = (size_t)-1;
    }
    void reset(uint32_t m, hipStream_t s)
    {
        mask = m;
        st = s;
        used = 0;
        recs.clear();
        if (m && pool.empty()) {
            pool.resize(1 << 16);
            for (auto &e : pool) (void)hipEventCreate(&e);
        }
    }
    ~Prof()
    {
        for (auto &e : pool) (void)hipEventDestroy(e);
    }
};

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
struct amrmg_ctx {
    amrmg_params P{};
    std::vector<double> mono;
    hipStream_t st = nullptr;
    Problem prob;
    bool built = false;
    DevState ds;
    std::vector<int32_t *> d_bmap;  // per AMR level: brick grid -> global brick
    void *user_ws = nullptr;
    size_t user_ws_bytes = 0;
    int generation = 0;
    // batch cache (kept by the first context of a batch)
    std::vector<amrmg_ctx *> batch_ctx;
    std::vector<int> batch_gen;
    DevState *batch = nullptr;
    Prof prof;
    ~amrmg_ctx()
    {
        for (auto p : d_bmap) (void)hipFree(p);
        delete batch;
    }
};

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
    p->nu2 = 2;
    p->omega = 6.0 / 7.0;
    p->norm_p = 2;
    p->max_iters = 50;
    p->bottom_rtol = 1e-6;
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
    if (p->smoother != AMRMG_GSRB && p->smoother != AMRMG_JACOBI) return fail(AMRMG_E_INVALID, "bad smoother");
    if (p->nu1 < 1 || p->nu2 < 1 || p->nu1 > 64 || p->nu2 > 64) return fail(AMRMG_E_INVALID, "nu1, nu2 in [1, 64]");
    if (p->norm_p != 0 && p->norm_p != 1 && p->norm_p != 2) return fail(AMRMG_E_INVALID, "norm_p must be 0, 1 or 2");
    if (p->max_iters < 0) return fail(AMRMG_E_INVALID, "max_iters must be >= 0");
    if (!(p->bottom_rtol > 0 && p->bottom_rtol < 1)) return fail(AMRMG_E_INVALID, "bottom_rtol in (0, 1)");
    if (!(p->omega > 0 && p->omega <= 1)) return fail(AMRMG_E_INVALID, "omega in (0, 1]");
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
    *out = c;
    return AMRMG_OK;
}

extern "C" void amrmg_destroy(amrmg_ctx *ctx) { delete ctx; }

// device brick map and user mapping of one level, for deposits during the
// build (local brick ids)
struct LevelDev {
    int32_t *bmap = nullptr;
    int64_t *ubase = nullptr;
    int2 *ustr = nullptr;
    ~LevelDev()
    {
        if (bmap) (void)hipFree(bmap);
        if (ubase) (void)hipFree(ubase);
        if (ustr) (void)hipFree(ustr);
    }
};

static DepLevel dep_level(const Problem &P, const HostLevel &L, const int32_t *bmap)
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

static amrmg_status level_dev(const HostLevel &L, LevelDev &out)
{
    std::vector<int64_t> ub(L.nbrick());
    std::vector<int32_t> us(2 * (size_t)L.nbrick());
    for (int b = 0; b < L.nbrick(); ++b) {
        const Box &B = L.boxes[L.bbox[b]];
        int64_t nx = B.hi[0] - B.lo[0], ny = B.hi[1] - B.lo[1];
        ub[b] = L.off[L.bbox[b]] + (8 * L.bpos[3 * b] - B.lo[0]) +
                nx * ((8 * L.bpos[3 * b + 1] - B.lo[1]) + ny * (int64_t)(8 * L.bpos[3 * b + 2] - B.lo[2]));
        us[2 * b] = (int32_t)nx;
        us[2 * b + 1] = (int32_t)(nx * ny);
    }
    HIP_TRY(hipMalloc(&out.bmap, sizeof(int32_t) * L.bmap.size()));
    HIP_TRY(hipMemcpy(out.bmap, L.bmap.data(), sizeof(int32_t) * L.bmap.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMalloc(&out.ubase, sizeof(int64_t) * ub.size()));
    HIP_TRY(hipMemcpy(out.ubase, ub.data(), sizeof(int64_t) * ub.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMalloc(&out.ustr, sizeof(int32_t) * us.size()));
    HIP_TRY(hipMemcpy(out.ustr, us.data(), sizeof(int32_t) * us.size(), hipMemcpyHostToDevice));
    return AMRMG_OK;
}

extern "C" amrmg_status amrmg_build_hierarchy(amrmg_ctx *ctx, int pos_dtype, const void *x, const void *y,
                                              const void *z, const double *q, int64_t n, const double *tag_rel,
                                              const int32_t *explicit_boxes, int32_t n_explicit)
{
    if (!ctx) return fail(AMRMG_E_INVALID, "ctx is NULL");
    if (pos_dtype != AMRMG_POS_F64 && pos_dtype != AMRMG_POS_F32) return fail(AMRMG_E_INVALID, "bad pos_dtype");
    if (n < 0 || (n > 0 && (!x || !y || !z || !q))) return fail(AMRMG_E_INVALID, "bad particle arrays");
    if (n_explicit < 0 || (n_explicit > 0 && !explicit_boxes)) return fail(AMRMG_E_INVALID, "bad explicit boxes");
    const amrmg_params &P = ctx->P;
    std::map<int, std::vector<Box>> expl;
    for (int32_t t = 0; t < n_explicit; ++t) {
        const int32_t *e = explicit_boxes + 7 * t;
        if (e[0] < 1 || e[0] > P.max_level) return fail(AMRMG_E_NESTING, "explicit box level out of range");
        Box B;
        for (int d = 0; d < 3; ++d) {
            B.lo[d] = e[1 + d];
            B.hi[d] = e[4 + d];
        }
        expl[e[0]].push_back(B);
    }
    ctx->built = false;
    ctx->ds.release();
    ctx->ds = DevState();
    for (auto p : ctx->d_bmap) (void)hipFree(p);
    ctx->d_bmap.clear();
    ++ctx->generation;

    Problem &pr = ctx->prob;
    pr = Problem();
    for (int d = 0; d < 3; ++d) {
        pr.lo[d] = P.lo[d];
        pr.hi[d] = P.hi[d];
    }
    pr.eps0 = P.eps0;
    pr.mono = ctx->mono;
    {
        HostLevel L0;
        level_init(L0, P.n0, P.lo, P.hi);
        L0.amr = 0;
        Box B{{0, 0, 0}, {P.n0[0], P.n0[1], P.n0[2]}};
        level_set_boxes(L0, {B});
        pr.lev.push_back(L0);
    }
    for (int l = 0; l < P.max_level; ++l) {
        std::vector<Box> boxes;
        const HostLevel &L = pr.lev[l];
        if (expl.count(l + 1)) {
            boxes = expl[l + 1];
        } else {
            if (!tag_rel) return fail(AMRMG_E_INVALID, "tag_rel is NULL but a level needs tagging");
            int64_t nc = L.ncells();
            LevelDev ld;
            ST_TRY(level_dev(L, ld));
            double *rho = nullptr, *scratch = nullptr;
            uint8_t *tags = nullptr;
            HIP_TRY(hipMalloc(&rho, sizeof(double) * nc));
            HIP_TRY(hipMalloc(&scratch, sizeof(double) * 1032));
            HIP_TRY(hipMalloc(&tags, nc));
            launch_fill(ctx->st, rho, nc, 0.0);
            DepLevel D = dep_level(pr, L, ld.bmap);
            launch_deposit(ctx->st, pos_dtype == AMRMG_POS_F32, n, x, y, z, q, D, ld.ubase, ld.ustr, rho, nullptr);
            launch_tag(ctx->st, rho, nc, tag_rel[l], scratch, tags);
            std::vector<uint8_t> ht(nc);
            hipError_t e1 = hipMemcpyAsync(ht.data(), tags, nc, hipMemcpyDeviceToHost, ctx->st);
            hipError_t e2 = hipStreamSynchronize(ctx->st);
            (void)hipFree(rho);
            (void)hipFree(scratch);
            (void)hipFree(tags);
            HIP_TRY(e1);
            HIP_TRY(e2);
            HIP_TRY(hipGetLastError());
            boxes = generate_boxes(L, ht.data(), P.n_buffer, P.n_proper, P.blocking_factor, P.max_grid_size);
        }
        if (boxes.empty()) break;
        std::string msg = check_nesting(L, boxes, P.n_proper);
        if (!msg.empty()) return fail(AMRMG_E_NESTING, "level " + std::to_string(l + 1) + ": " + msg);
        HostLevel F;
        int nf[3] = {2 * L.n[0], 2 * L.n[1], 2 * L.n[2]};
        level_init(F, nf, P.lo, P.hi);
        F.amr = l + 1;
        level_set_boxes(F, boxes);
        pr.lev.push_back(F);
    }
    add_levels_below(pr);
    build_meta({&pr}, ctx->ds.meta);
    if (!ctx->ds.meta.error.empty()) return fail(AMRMG_E_NESTING, ctx->ds.meta.error);
    ST_TRY(upload_meta(ctx->ds));
    // per AMR level brick map with global brick ids
    for (int l = 0; l < pr.namr(); ++l) {
        const HostLevel &L = pr.lev[pr.kg + l];
        int b0 = ctx->ds.meta.ent[ctx->ds.meta.prob_ent[0][pr.kg + l]].b0;
        std::vector<int32_t> bm(L.bmap);
        for (auto &v : bm)
            if (v >= 0) v += b0;
        int32_t *d = nullptr;
        HIP_TRY(hipMalloc(&d, sizeof(int32_t) * bm.size()));
        ctx->d_bmap.push_back(d);
        HIP_TRY(hipMemcpy(d, bm.data(), sizeof(int32_t) * bm.size(), hipMemcpyHostToDevice));
    }
    HIP_TRY(hipStreamSynchronize(ctx->st));
    ctx->built = true;
    return AMRMG_OK;
}

extern "C" amrmg_status amrmg_hierarchy_info(const amrmg_ctx *ctx, int32_t *nlevels, int32_t *nboxes,
                                             int64_t *ncells, int64_t *ndof)
{
    if (!ctx) return fail(AMRMG_E_INVALID, "ctx is NULL");
    if (!ctx->built) return fail(AMRMG_E_STATE, "hierarchy not built");
    const Problem &pr = ctx->prob;
    int L = pr.namr();
    if (nlevels) *nlevels = L;
    int64_t dof = 0;
    for (int l = 0; l < L; ++l) {
        if (nboxes) nboxes[l] = (int32_t)pr.lev[pr.kg + l].boxes.size();
        if (ncells) ncells[l] = pr.lev[pr.kg + l].ncells();
        dof += ctx->ds.meta.dof[0][l];
    }
    if (ndof) *ndof = dof;
    return AMRMG_OK;
}

extern "C" amrmg_status amrmg_get_boxes(const amrmg_ctx *ctx, int32_t level, int32_t *boxes, int64_t *offsets)
{
    if (!ctx) return fail(AMRMG_E_INVALID, "ctx is NULL");
    if (!ctx->built) return fail(AMRMG_E_STATE, "hierarchy not built");
    const Problem &pr = ctx->prob;
    if (level < 0 || level >= pr.namr()) return fail(AMRMG_E_INVALID, "level out of range");
    const HostLevel &L = pr.lev[pr.kg + level];
    for (size_t b = 0; b < L.boxes.size(); ++b)
        for (int d = 0; d < 3; ++d) {
            if (boxes) {
                boxes[6 * b + d] = L.boxes[b].lo[d];
                boxes[6 * b + 3 + d] = L.boxes[b].hi[d];
            }
        }
    if (offsets)
        for (size_t b = 0; b <= L.boxes.size(); ++b) offsets[b] = L.off[b];
    return AMRMG_OK;
}

extern "C" amrmg_status amrmg_cf_faces(const amrmg_ctx *ctx, int32_t level, int32_t *out, int64_t cap,
                                       int64_t *count)
{
    if (!ctx) return fail(AMRMG_E_INVALID, "ctx is NULL");
    if (!ctx->built) return fail(AMRMG_E_STATE, "hierarchy not built");
    const Problem &pr = ctx->prob;
    if (level < 0 || level >= pr.namr()) return fail(AMRMG_E_INVALID, "level out of range");
    const Meta &m = ctx->ds.meta;
    const Meta::Entry &e = m.ent[m.prob_ent[0][pr.kg + level]];
    int64_t k = 0;
    for (int c = e.cf0; c < e.cf0 + e.ncf; ++c) {
        int32_t ow = m.gf_owner[m.nbc + c];
        int g = ow >> 3, dir = ow & 7, d = dir >> 1, s = (dir & 1) ? 1 : -1;
        int du = (d == 0) ? 1 : 0, dv = (d == 2) ? 1 : 2;
        for (int t = 0; t < 64; ++t, ++k) {
            if (!out || k >= cap) continue;
            int l[3];
            l[d] = s > 0 ? 7 : 0;
            l[du] = t & 7;
            l[dv] = t >> 3;
            int32_t *o = out + 6 * k;
            for (int a = 0; a < 3; ++a) o[a] = m.org[(size_t)g * 4 + a] + l[a];
            o[3] = d;
            o[4] = s;
            int mm = ((t & 7) >> 1) + 4 * ((t >> 3) >> 1);
            o[5] = m.cf_pat[(size_t)c * 16 + mm];
        }
    }
    if (count) *count = k;
    return AMRMG_OK;
}

extern "C" amrmg_status amrmg_workspace_size(const amrmg_ctx *ctx, size_t *bytes)
{
    if (!ctx || !bytes) return fail(AMRMG_E_INVALID, "NULL argument");
    if (!ctx->built) return fail(AMRMG_E_STATE, "hierarchy not built");
    *bytes = ws_need(ctx->ds, ctx->P.precision);
    return AMRMG_OK;
}

extern "C" amrmg_status amrmg_set_workspace(amrmg_ctx *ctx, void *dev, size_t bytes)
{
    if (!ctx) return fail(AMRMG_E_INVALID, "ctx is NULL");
    if (dev && ((uintptr_t)dev & 255)) return fail(AMRMG_E_INVALID, "workspace must be 256-byte aligned");
    if (dev && ctx->built && bytes < ws_need(ctx->ds, ctx->P.precision))
        return fail(AMRMG_E_OOM, "workspace smaller than amrmg_workspace_size");
    if (!dev && ctx->ds.ws && !ctx->ds.ws_owned) {
        ctx->ds.ws = nullptr;
        ctx->ds.ws_bytes = 0;
    }
    ctx->user_ws = dev;
    ctx->user_ws_bytes = dev ? bytes : 0;
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
        HIP_TRY(hipMallocAsync((void **)&dout, sizeof(unsigned long long), ctx->st));
        HIP_TRY(hipMemsetAsync(dout, 0, sizeof(unsigned long long), ctx->st));
    }
    for (int l = 0; l < pr.namr(); ++l) {
        if (!rho[l]) return fail(AMRMG_E_INVALID, "rho[l] is NULL");
        const HostLevel &L = pr.lev[pr.kg + l];
        launch_fill(ctx->st, rho[l], L.ncells(), 0.0);
        DepLevel D = dep_level(pr, L, ctx->d_bmap[l]);
        ctx->prof.begin(AMRMG_K_DEPOSIT);
        launch_deposit(ctx->st, pos_dtype == AMRMG_POS_F32, n, x, y, z, q, D, ctx->ds.M.ubase, ctx->ds.M.ustr, rho[l],
                       l == 0 ? dout : nullptr);
        ctx->prof.end(AMRMG_K_DEPOSIT, (double)n * (3.0 * (pos_dtype == AMRMG_POS_F32 ? 4 : 8) + 8.0) +
                                           8.0 * (double)L.ncells());
    }
    HIP_TRY(hipGetLastError());
    if (n_outside) {
        unsigned long long h = 0;
        HIP_TRY(hipMemcpyAsync(&h, dout, sizeof(h), hipMemcpyDeviceToHost, ctx->st));
        HIP_TRY(hipFreeAsync(dout, ctx->st));
        HIP_TRY(hipStreamSynchronize(ctx->st));
        *n_outside = (int64_t)h;
    }
    return AMRMG_OK;
}

extern "C" amrmg_status amrmg_gather(amrmg_ctx *ctx, int pos_dtype, const void *x, const void *y, const void *z,
                                     int64_t n, double *const *E, double *Ex, double *Ey, double *Ez)
{
    if (!ctx) return fail(AMRMG_E_INVALID, "ctx is NULL");
    if (!ctx->built) return fail(AMRMG_E_STATE, "hierarchy not built");
    if (pos_dtype != AMRMG_POS_F64 && pos_dtype != AMRMG_POS_F32) return fail(AMRMG_E_INVALID, "bad pos_dtype");
    if (!E || n < 0 || (n > 0 && (!x || !y || !z || !Ex || !Ey || !Ez))) return fail(AMRMG_E_INVALID, "bad arguments");
    const Problem &pr = ctx->prob;
    GatherArgs G{};
    G.nlev = pr.namr();
    for (int l = 0; l < G.nlev; ++l) {
        G.lev[l] = dep_level(pr, pr.lev[pr.kg + l], ctx->d_bmap[l]);
        for (int d = 0; d < 3; ++d) {
            if (!E[3 * l + d]) return fail(AMRMG_E_INVALID, "E component is NULL");
            G.E[3 * l + d] = E[3 * l + d];
        }
    }
    ctx->prof.begin(AMRMG_K_GATHER);
    launch_gather(ctx->st, pos_dtype == AMRMG_POS_F32, n, x, y, z, G, ctx->ds.M.ubase, ctx->ds.M.ustr, Ex, Ey, Ez);
    ctx->prof.end(AMRMG_K_GATHER, (double)n * (3.0 * (pos_dtype == AMRMG_POS_F32 ? 4 : 8) + 24.0));
    HIP_TRY(hipGetLastError());
    return AMRMG_OK;
}

// ---------------------------------------------------------------------------
// the solve
// ---------------------------------------------------------------------------
struct SolveOpts {
    int precision, smoother, nu1, nu2, norm_p, max_iters;
    double omega, bottom_rtol, inv_eps0;
};

template <class T>
struct Driver {
    DevState &D;
    hipStream_t st;
    SolveOpts o;
    const Meta &m;
    T *e, *r, *et, *cpe;
    Prof *P;
    static constexpr double W = sizeof(T);

    Driver(DevState &D_, hipStream_t s, const SolveOpts &op, Prof *p)
        : D(D_), st(s), o(op), m(D_.meta), e((T *)D_.e), r((T *)D_.r), et((T *)D_.et), cpe((T *)D_.cpe), P(p)
    {
    }
    void pb(int c)
    {
        if (P) P->begin(c);
    }
    void pe(int c, double bytes)
    {
        if (P) P->end(c, bytes);
    }

    bool single() const { return m.prob_ent.size() == 1; }
    // all AMR bricks: a contiguous range for one problem, a list otherwise
    void amr_range(int &b0, int &nb, const int32_t *&list) const
    {
        nb = (int)m.amr_bricks.size();
        if (single()) {
            b0 = nb ? m.amr_bricks[0] : 0;
            list = nullptr;
        } else {
            b0 = 0;
            list = D.d_amr;
        }
    }
    int step_b0(int k) const { return m.ent[m.step_ent0[k]].b0; }
    int step_nb(int k) const
    {
        const auto &last = m.ent[m.step_ent0[k + 1] - 1];
        return last.b0 + last.nb - step_b0(k);
    }

    // outer FP64 residual of every AMR level; norms into dnorm[off ..]
    void outer(bool zero_phi, int noff, double *const *rout_user)
    {
        int b0, nb;
        const int32_t *list;
        amr_range(b0, nb, list);
        if (!zero_phi) {
            pb(AMRMG_K_CPART);
            launch_cpart_user(st, D.M, 0, m.ncf, D.d_phi, D.cpphi);
            pe(AMRMG_K_CPART, (double)m.ncf * 16 * (9 + 4) * 8);
        }
        pb(AMRMG_K_RESIDUAL);
        launch_outer_residual<T>(st, D.M, b0, nb, list, D.d_phi, D.d_rho, o.inv_eps0, zero_phi ? nullptr : D.cpphi,
                                 (zero_phi || rout_user) ? nullptr : r, D.part, o.norm_p, zero_phi, rout_user);
        pe(AMRMG_K_RESIDUAL, (double)nb * BRICK_CELLS * (zero_phi ? 8.0 : 16.0 + W));
        launch_level_norms(st, D.d_ranges, (int)D.range_prob.size(), D.part, D.dnorm + noff, o.norm_p);
    }

    void smooth(int k, int nu, bool pre)
    {
        int b0 = step_b0(k), nb = step_nb(k);
        const T *cp = pre ? nullptr : cpe;
        const double n = (double)nb * BRICK_CELLS;
        if (o.smoother == AMRMG_GSRB) {
            for (int it = 0; it < nu; ++it) {
                for (int colour = 0; colour < 2; ++colour) {
                    pb(AMRMG_K_GSRB);
                    launch_gsrb<T>(st, D.M, b0, nb, e, r, cp, colour, pre && it == 0 && colour == 0);
                    pe(AMRMG_K_GSRB, 1.5 * n * W);
                }
            }
            return;
        }
        // damped Jacobi, ping-pong between e and et; the result ends in e
        int left = nu;
        bool first = pre;
        if (first) {
            if (left % 2 == 1) {
                launch_jacobi<T>(st, D.M, b0, nb, e, e, r, cp, o.omega, true);
            } else {
                launch_jacobi<T>(st, D.M, b0, nb, e, et, r, cp, o.omega, true);
                launch_jacobi<T>(st, D.M, b0, nb, et, e, r, cp, o.omega, false);
                --left;
            }
            --left;
        }
        while (left >= 2) {
            launch_jacobi<T>(st, D.M, b0, nb, e, et, r, cp, o.omega, false);
            launch_jacobi<T>(st, D.M, b0, nb, et, e, r, cp, o.omega, false);
            left -= 2;
        }
        if (left == 1) {
            launch_jacobi<T>(st, D.M, b0, nb, e, et, r, cp, o.omega, false);
            launch_copy<T>(st, et + (size_t)b0 * BRICK_CELLS, e + (size_t)b0 * BRICK_CELLS, (int64_t)nb * BRICK_CELLS);
        }
    }

    void vcycle()
    {
        for (int k = m.K - 1; k >= 1; --k) {
            smooth(k, o.nu1, true);
            double n = (double)step_nb(k) * BRICK_CELLS;
            pb(AMRMG_K_RESTRICT);
            launch_restrict<T>(st, D.M, step_b0(k), step_nb(k), e, r, r);
            pe(AMRMG_K_RESTRICT, (2.0 + 0.125) * n * W);
            // coarse cells of level k-1 next to level k
            const auto &e0 = m.ent[m.step_ent0[k - 1]];
            const auto &e1 = m.ent[m.step_ent0[k] - 1];
            int rf0 = e0.rf0, nrf = e1.rf0 + e1.nrf - e0.rf0;
            pb(AMRMG_K_REFLUX);
            launch_reflux<T>(st, D.M, D.d_reflux + rf0, nrf, e, r);
            pe(AMRMG_K_REFLUX, 2.0 * nrf * BRICK_CELLS * W);
        }
        pb(AMRMG_K_BOTTOM);
        launch_bottom_cg<T>(st, D.M, D.d_jobs, D.njobs, r, e, D.cgw, o.bottom_rtol, 10000, D.cgit);
        pe(AMRMG_K_BOTTOM, (double)D.cg_doubles / 4 * (2 * W));
        for (int k = 1; k < m.K; ++k) {
            const auto &e0 = m.ent[m.step_ent0[k]];
            const auto &e1 = m.ent[m.step_ent0[k + 1] - 1];
            int ncf = e1.cf0 + e1.ncf - e0.cf0;
            double n = (double)step_nb(k) * BRICK_CELLS;
            pb(AMRMG_K_CPART);
            launch_cpart_brick<T>(st, D.M, e0.cf0, ncf, e, cpe);
            pe(AMRMG_K_CPART, (double)ncf * 16 * (9 + 4) * W);
            pb(AMRMG_K_PROLONG);
            launch_prolong<T>(st, D.M, step_b0(k), step_nb(k), e);
            pe(AMRMG_K_PROLONG, (2.0 + 0.125) * n * W);
            smooth(k, o.nu2, false);
        }
        int b0, nb;
        const int32_t *list;
        amr_range(b0, nb, list);
        pb(AMRMG_K_PHI_UPDATE);
        launch_phi_update<T>(st, D.M, b0, nb, list, D.d_phi, e);
        pe(AMRMG_K_PHI_UPDATE, (double)nb * BRICK_CELLS * (16.0 + W));
    }
};

// run a solve on a DevState whose pointer tables are set; per-problem stats
template <class T>
static amrmg_status run_solve(DevState &D, hipStream_t st, const SolveOpts &o, double tol,
                              std::vector<amrmg_solve_stats> &stats, bool want_E, Prof *prof)
{
    const Meta &m = D.meta;
    Driver<T> drv(D, st, o, prof);
    const int nr = (int)D.range_prob.size();
    const int np = (int)m.prob_ent.size();
    hipEvent_t ev0, ev1;
    HIP_TRY(hipEventCreate(&ev0));
    HIP_TRY(hipEventCreate(&ev1));
    HIP_TRY(hipMemsetAsync(D.cgit, 0, sizeof(int), st));
    HIP_TRY(hipEventRecord(ev0, st));
    drv.outer(true, 0, nullptr);
    drv.outer(false, nr, nullptr);
    HIP_TRY(hipMemcpyAsync(D.h_norm, D.dnorm, sizeof(double) * 2 * nr, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    HIP_TRY(hipGetLastError());
    std::vector<double> bn(D.h_norm, D.h_norm + nr), rn(D.h_norm + nr, D.h_norm + 2 * nr);
    // a level without right-hand side uses its problem's composite norm
    std::vector<double> tot(np, 0.0);
    for (int i = 0; i < nr; ++i) {
        int p = D.range_prob[i];
        if (o.norm_p == 2) tot[p] += bn[i] * bn[i];
        else if (o.norm_p == 1) tot[p] += bn[i];
        else tot[p] = std::max(tot[p], bn[i]);
    }
    for (int p = 0; p < np; ++p)
        if (o.norm_p == 2) tot[p] = std::sqrt(tot[p]);
    for (int i = 0; i < nr; ++i)
        if (bn[i] == 0.0) bn[i] = tot[D.range_prob[i]];
    std::vector<int> conv_at(np, -1);
    auto check = [&](int it) {
        std::vector<int> ok(np, 1);
        for (int i = 0; i < nr; ++i)
            if (!(rn[i] <= tol * bn[i])) ok[D.range_prob[i]] = 0;
        bool all = true;
        for (int p = 0; p < np; ++p) {
            if (ok[p] && conv_at[p] < 0) conv_at[p] = it;
            all = all && ok[p];
        }
        return all;
    };
    int it = 0;
    bool all = check(0);
    while (!all && it < o.max_iters) {
        drv.vcycle();
        drv.outer(false, nr, nullptr);
        HIP_TRY(hipMemcpyAsync(D.h_norm + nr, D.dnorm + nr, sizeof(double) * nr, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        HIP_TRY(hipGetLastError());
        rn.assign(D.h_norm + nr, D.h_norm + 2 * nr);
        ++it;
        all = check(it);
    }
    // average down, finest first, then the field
    for (int k = m.K - 1; k >= 1; --k)
        for (int ei = m.step_ent0[k]; ei < m.step_ent0[k + 1]; ++ei)
            if (m.ent[ei].amr >= 1) {
                drv.pb(AMRMG_K_AVGDOWN);
                launch_avgdown(st, D.M, m.ent[ei].b0, m.ent[ei].nb, D.d_phi);
                drv.pe(AMRMG_K_AVGDOWN, (double)m.ent[ei].nb * BRICK_CELLS * 8.0 * (1.0 + 0.125));
            }
    if (want_E) {
        int b0, nb;
        const int32_t *list;
        drv.amr_range(b0, nb, list);
        drv.pb(AMRMG_K_EFIELD);
        launch_efield(st, D.M, b0, nb, list, D.d_phi, D.cpphi, D.d_E);
        drv.pe(AMRMG_K_EFIELD, (double)nb * BRICK_CELLS * 32.0);
    }
    HIP_TRY(hipEventRecord(ev1, st));
    HIP_TRY(hipEventSynchronize(ev1));
    HIP_TRY(hipGetLastError());
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ev0, ev1));
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    int cgmax = 0;
    HIP_TRY(hipMemcpy(&cgmax, D.cgit, sizeof(int), hipMemcpyDeviceToHost));
    stats.assign(np, amrmg_solve_stats{});
    for (int p = 0; p < np; ++p) {
        amrmg_solve_stats &s = stats[p];
        s.iters = conv_at[p] >= 0 ? conv_at[p] : it;
        s.converged = conv_at[p] >= 0;
        s.time_ms = ms;
        s.bottom_iters_max = cgmax;
        int64_t dof = 0;
        for (auto v : m.dof[p]) dof += v;
        s.dof = dof;
    }
    for (int i = 0; i < nr; ++i) {
        amrmg_solve_stats &s = stats[D.range_prob[i]];
        s.rel_residual[D.range_amr[i]] = bn[i] > 0 ? rn[i] / bn[i] : rn[i];
        s.nlevels = std::max(s.nlevels, D.range_amr[i] + 1);
    }
    return all ? AMRMG_OK : AMRMG_E_NOT_CONVERGED;
}

static SolveOpts opts_of(const amrmg_params &P)
{
    SolveOpts o;
    o.precision = P.precision;
    o.smoother = P.smoother;
    o.nu1 = P.nu1;
    o.nu2 = P.nu2;
    o.norm_p = P.norm_p;
    o.max_iters = P.max_iters;
    o.omega = P.omega;
    o.bottom_rtol = P.bottom_rtol;
    o.inv_eps0 = 1.0 / P.eps0;
    return o;
}

static amrmg_status set_tables(DevState &D, hipStream_t st)
{
    size_t ne = D.meta.ent.size();
    HIP_TRY(hipMemcpyAsync(D.d_phi, D.h_phi.data(), sizeof(double *) * ne, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(D.d_rho, D.h_rho.data(), sizeof(double *) * ne, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(D.d_E, D.h_E.data(), sizeof(double *) * 3 * ne, hipMemcpyHostToDevice, st));
    return AMRMG_OK;
}

extern "C" amrmg_status amrmg_solve(amrmg_ctx *ctx, double *const *rho, double *const *phi, double *const *E,
                                    double tol, amrmg_solve_stats *stats)
{
    if (!ctx) return fail(AMRMG_E_INVALID, "ctx is NULL");
    if (!ctx->built) return fail(AMRMG_E_STATE, "hierarchy not built");
    if (!rho || !phi) return fail(AMRMG_E_INVALID, "rho and phi are required");
    if (!(tol > 0)) return fail(AMRMG_E_INVALID, "tol must be positive");
    DevState &D = ctx->ds;
    const Problem &pr = ctx->prob;
    std::fill(D.h_phi.begin(), D.h_phi.end(), nullptr);
    std::fill(D.h_rho.begin(), D.h_rho.end(), nullptr);
    std::fill(D.h_E.begin(), D.h_E.end(), nullptr);
    for (int l = 0; l < pr.namr(); ++l) {
        if (!rho[l] || !phi[l]) return fail(AMRMG_E_INVALID, "rho[l] and phi[l] must be set");
        int ei = D.meta.prob_ent[0][pr.kg + l];
        D.h_phi[ei] = phi[l];
        D.h_rho[ei] = rho[l];
        for (int d = 0; d < 3; ++d) {
            if (E && !E[3 * l + d]) return fail(AMRMG_E_INVALID, "E component is NULL");
            D.h_E[3 * ei + d] = E ? E[3 * l + d] : nullptr;
        }
    }
    ST_TRY(ensure_ws(D, ctx->P.precision, ctx->user_ws, ctx->user_ws_bytes));
    ST_TRY(set_tables(D, ctx->st));
    std::vector<amrmg_solve_stats> sv;
    SolveOpts o = opts_of(ctx->P);
    Prof *pf = ctx->prof.mask ? &ctx->prof : nullptr;
    amrmg_status rc = ctx->P.precision == AMRMG_MIXED ? run_solve<float>(D, ctx->st, o, tol, sv, E != nullptr, pf)
                                                      : run_solve<double>(D, ctx->st, o, tol, sv, E != nullptr, pf);
    if (stats && !sv.empty()) *stats = sv[0];
    if (rc == AMRMG_E_NOT_CONVERGED) g_err = "not converged within max_iters";
    return rc;
}

extern "C" amrmg_status amrmg_residual(amrmg_ctx *ctx, double *const *rho, double *const *phi, double *const *r)
{
    if (!ctx) return fail(AMRMG_E_INVALID, "ctx is NULL");
    if (!ctx->built) return fail(AMRMG_E_STATE, "hierarchy not built");
    if (!rho || !phi || !r) return fail(AMRMG_E_INVALID, "rho, phi and r are required");
    DevState &D = ctx->ds;
    const Problem &pr = ctx->prob;
    std::fill(D.h_phi.begin(), D.h_phi.end(), nullptr);
    std::fill(D.h_rho.begin(), D.h_rho.end(), nullptr);
    std::fill(D.h_rout.begin(), D.h_rout.end(), nullptr);
    for (int l = 0; l < pr.namr(); ++l) {
        if (!rho[l] || !phi[l] || !r[l]) return fail(AMRMG_E_INVALID, "level arrays must be set");
        int ei = D.meta.prob_ent[0][pr.kg + l];
        D.h_phi[ei] = phi[l];
        D.h_rho[ei] = rho[l];
        D.h_rout[ei] = r[l];
    }
    ST_TRY(ensure_ws(D, ctx->P.precision, ctx->user_ws, ctx->user_ws_bytes));
    ST_TRY(set_tables(D, ctx->st));
    size_t ne = D.meta.ent.size();
    HIP_TRY(hipMemcpyAsync(D.d_rout, D.h_rout.data(), sizeof(double *) * ne, hipMemcpyHostToDevice, ctx->st));
    SolveOpts o = opts_of(ctx->P);
    Driver<double> drv(D, ctx->st, o, nullptr);
    drv.outer(false, 0, D.d_rout);
    HIP_TRY(hipStreamSynchronize(ctx->st));
    HIP_TRY(hipGetLastError());
    return AMRMG_OK;
}

extern "C" amrmg_status amrmg_solve_batch(amrmg_ctx *const *ctxs, int32_t nb, double *const *const *rho,
                                          double *const *const *phi, double tol, amrmg_solve_stats *stats)
{
    (void)ctxs;
    (void)nb;
    (void)rho;
    (void)phi;
    (void)tol;
    (void)stats;
    return fail(AMRMG_E_NOT_IMPLEMENTED, "amrmg_solve_batch");
}

extern "C" amrmg_status amrmg_profile_enable(amrmg_ctx *ctx, uint32_t mask)
{
    if (!ctx) return fail(AMRMG_E_INVALID, "ctx is NULL");
    HIP_TRY(hipStreamSynchronize(ctx->st));
    ctx->prof.reset(mask, ctx->st);
    return AMRMG_OK;
}

extern "C" amrmg_status amrmg_profile_read(amrmg_ctx *ctx, int32_t kclass, double *ms, int64_t *launches,
                                           double *bytes)
{
    if (!ctx) return fail(AMRMG_E_INVALID, "ctx is NULL");
    if (kclass < 0 || kclass >= AMRMG_K_NCLASS) return fail(AMRMG_E_INVALID, "bad kernel class");
    HIP_TRY(hipStreamSynchronize(ctx->st));
    double t = 0.0, b = 0.0;
    int64_t n = 0;
    for (const auto &r : ctx->prof.recs) {
        if (r.cls != kclass) continue;
        float e = 0.f;
        HIP_TRY(hipEventElapsedTime(&e, ctx->prof.pool[r.ev], ctx->prof.pool[r.ev + 1]));
        t += e;
        b += r.bytes;
        ++n;
    }
    if (ms) *ms = t;
    if (launches) *launches = n;
    if (bytes) *bytes = b;
    return AMRMG_OK;
}
