// amrmg_solver.cpp -- the solve driver of libamrmg, which runs the composite
// AMR multigrid of arXiv:1812.03689 (Alg. 2 and Alg. 3) on the HIP kernels
// of amrmg_kernels.hip; the workspace, amrmg_solve, amrmg_residual and
// amrmg_solve_batch.
//
// Solve structure (per outer iteration, Alg. 2):
//   1. FP64 composite residual of every AMR level (Alg. 1) -> per-level norms,
//      which the norms kernel writes into host memory with a sequence number
//      that the host polls (no stream synchronisation per iteration);
//   2. one V-cycle (Alg. 3) on the correction equation A_comp e = r, stored in
//      T (float in mixed precision, double otherwise), continued below AMR
//      level 0 through geometric coarsenings down to a grid of at most 64
//      cells per edge, solved exactly (separable transforms) or by CG;
//   3. phi += e in FP64.
// With T = double this is Alg. 2 as printed (the V-cycle applied to the
// correction form, which is algebraically the same cycle); with T = float it
// is iterative refinement around an FP32 cycle.
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

size_t ws_need(const DevState &D, int prec)
{
    const Meta &m = D.meta;
    size_t w = prec == AMRMG_MIXED ? 4 : 8;
    size_t nc = (size_t)m.nbrick * BRICK_CELLS;
    size_t s = 0;
    s += 3 * align256(nc * w);                        // e, r, et
    s += 2 * align256(nc * 8);                        // phi, rho in brick layout
    s += align256((size_t)m.ncf * 64 * w + 8);         // coarse parts of the cycle
    s += align256((size_t)m.ncf * 64 * 8 + 8);         // coarse parts of phi
    s += align256((size_t)m.nbrick * 16);              // per-wavefront partial norms (two per brick)
    s += align256((size_t)m.nbrick * 96 * 8);          // fine sums of the coarse-fine faces
    s += align256(sizeof(double) * 2 * (D.range_prob.size() + 1));
    s += align256(D.cg_doubles * 8);
    s += align256(D.dw_doubles * 8 + 8);             // direct-solve scratch
    s += align256(64);
    return s;
}

amrmg_status ensure_ws(DevState &D, int prec, void *user, size_t user_bytes)
{
    size_t need = ws_need(D, prec);
    char *base = nullptr;
    if (user) {
        if (user_bytes < need) return fail(AMRMG_E_OOM, "caller workspace smaller than amrmg_workspace_size");
        if (D.ws == user && D.ws_prec == prec) return AMRMG_OK;
        D.ws = user;
        D.ws_bytes = user_bytes;
    } else {
        if (D.ws == D.ws_own.p && D.ws && D.ws_bytes >= need && D.ws_prec == prec) return AMRMG_OK;
        if (D.ws_own.ensure(need) != hipSuccess) return fail(AMRMG_E_OOM, "workspace allocation failed");
        D.ws = D.ws_own.p;
        D.ws_bytes = D.ws_own.cap;
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
    D.phib = (double *)take(nc * 8);
    D.rhob = (double *)take(nc * 8);
    D.cpe = take((size_t)m.ncf * 64 * w + 8);
    D.cpphi = (double *)take((size_t)m.ncf * 64 * 8 + 8);
    D.part = (double *)take((size_t)m.nbrick * 16);
    D.ffs = (double *)take((size_t)m.nbrick * 96 * 8);
    D.dnorm = (double *)take(sizeof(double) * 2 * (D.range_prob.size() + 1));
    D.cgw = (double *)take(D.cg_doubles * 8);
    D.dw = (double *)take(D.dw_doubles * 8 + 8);
    D.cgit = (int *)take(64);
    D.d_seqc = (unsigned *)((char *)D.cgit + 32);
    D.ws_prec = prec;
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
    if (!dev && ctx->ds.ws && ctx->ds.ws != ctx->ds.ws_own.p) {
        ctx->ds.ws = nullptr;
        ctx->ds.ws_bytes = 0;
        ctx->ds.ws_prec = -1;
    }
    ctx->user_ws = dev;
    ctx->user_ws_bytes = dev ? bytes : 0;
    return AMRMG_OK;
}

// ---------------------------------------------------------------------------
// the solve
// ---------------------------------------------------------------------------
// replay the outer iteration as a hipGraph (AMRMG_NO_GRAPH=1 disables)
static bool g_use_graphs = getenv("AMRMG_NO_GRAPH") == nullptr;
// an outer iteration is queued one ahead while the residual is this many
// times above its target (a cycle reduces it by far less than this factor)
constexpr double kAhead = 100.0;

// Workgroup shape of the sweep kernel (one wavefront per brick, 1, 2 or 4
// bricks per workgroup), tuned on the device: for each launch size class
// (bricks per launch, rounded up to a power of two) and cycle precision the
// first solve that meets it times a plain sweep with each shape and keeps the
// fastest unless the size rule's is within 3 %; later solves and captured
// graphs read the choice.  Process-wide (one GPU per process);
// AMRMG_NO_TUNE=1 keeps the size rule instead.
static std::mutex g_tune_mu;
static std::map<std::pair<int, int>, int> g_hgs_nt;  // (sizeof(T), log2 bricks) -> threads per workgroup
static const bool g_tune = getenv("AMRMG_NO_TUNE") == nullptr;

static int size_class(int nb)
{
    int c = 0;
    while ((1 << c) < nb) ++c;
    return c;
}

static int tuned_nt(int wbytes, int nb)
{
    if (!g_tune) return 0;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_hgs_nt.find({wbytes, size_class(nb)});
    return it == g_hgs_nt.end() ? 0 : it->second;
}

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
        nb = D.n_amr;
        if (single()) {
            b0 = D.amr_first;
            list = nullptr;
        } else {
            b0 = 0;
            list = D.d_amr;
        }
    }
    int step_b0(int k) const { return m.ent[m.step_ent0[k]].b0; }
    double step_amr_cells(int k) const
    {
        double c = 0.0;
        for (int ei = m.step_ent0[k]; ei < m.step_ent0[k + 1]; ++ei)
            if (m.ent[ei].amr >= 0) c += (double)m.ent[ei].nb * BRICK_CELLS;
        return c;
    }
    int step_nb(int k) const
    {
        const auto &last = m.ent[m.step_ent0[k + 1] - 1];
        return last.b0 + last.nb - step_b0(k);
    }
    int hgs_nt(int k) const { return tuned_nt((int)sizeof(T), step_nb(k)); }

    // time the sweep of every level with each workgroup shape (1, 2 or 4
    // bricks per workgroup, one wavefront each) not yet tuned for its size
    // class (plain sweeps from e into et: both are scratch before the cycle
    // starts)
    amrmg_status tune()
    {
        if (!g_tune) return AMRMG_OK;
        for (int k = D.kc + 1; k < m.K; ++k) {
            const int b0 = step_b0(k), nb = step_nb(k);
            if (nb <= 0 || tuned_nt((int)sizeof(T), nb)) continue;
            hipEvent_t a, z;
            HIP_TRY(hipEventCreate(&a));
            HIP_TRY(hipEventCreate(&z));
            constexpr int REPS = 5, NC = 3;
            const int cand[NC] = {64, 128, 256};
            float each[NC] = {0.f, 0.f, 0.f};
            for (int i = 0; i < NC; ++i) {
                launch_hgs<T>(st, D.M, b0, nb, e, et, r, cpe, D.phib, D.ffs, 0, cand[i]);  // warm
                HIP_TRY(hipEventRecord(a, st));
                for (int rep = 0; rep < REPS; ++rep)
                    launch_hgs<T>(st, D.M, b0, nb, e, et, r, cpe, D.phib, D.ffs, 0, cand[i]);
                HIP_TRY(hipEventRecord(z, st));
                HIP_TRY(hipEventSynchronize(z));
                HIP_TRY(hipEventElapsedTime(&each[i], a, z));
            }
            // the size rule's shape unless another is clearly faster
            int rule = 0;
            for (int i = 0; i < NC; ++i)
                if (cand[i] == hgs_rule_threads(nb)) rule = i;
            int best = rule;
            for (int i = 0; i < NC; ++i)
                if (each[i] < each[best]) best = i;
            const int pick = each[best] < 0.97f * each[rule] ? cand[best] : cand[rule];
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(z);
            HIP_TRY(hipGetLastError());
            if (getenv("AMRMG_TUNE_LOG"))
                fprintf(stderr,
                        "libamrmg: sweep of %d bricks (%d-byte cycle): 1, 2, 4 bricks per workgroup %.4f, %.4f, "
                        "%.4f ms -> %d threads\n",
                        nb, (int)sizeof(T), each[0] / REPS, each[1] / REPS, each[2] / REPS, pick);
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_hgs_nt.emplace(std::make_pair((int)sizeof(T), size_class(nb)), pick);
        }
        return AMRMG_OK;
    }

    // outer FP64 residual of every AMR level; norms into dnorm[off ..] (and
    // published to the host at h_pub[pub_off ..] when publish is set, or
    // pub_alt further on when the publication's sequence number is even)
    void outer(bool zero_phi, int noff, double *const *rout_user, bool publish = false, int pub_off = 0,
               int pub_alt = 0)
    {
        int b0, nb;
        const int32_t *list;
        amr_range(b0, nb, list);
        if (!zero_phi) {
            pb(AMRMG_K_CPART);
            launch_cpart_brick<double>(st, D.M, 0, m.ncf, D.phib, D.cpphi, D.phib, D.ffs);
            pe(AMRMG_K_CPART, (double)m.ncf * 16 * (9 + 4) * 8);
        }
        // (a last-workgroup reduction inside the residual kernel would need a
        // device-scope fence per workgroup, which costs far more than this
        // extra launch on a chip whose XCDs have separate L2 caches)
        pb(AMRMG_K_RESIDUAL);
        launch_outer_residual<T>(st, D.M, b0, nb, list, D.phib, D.rhob, o.inv_eps0, zero_phi ? nullptr : D.cpphi,
                                 (zero_phi || rout_user) ? nullptr : r, D.part, o.norm_p, zero_phi, rout_user, D.ffs);
        pe(AMRMG_K_RESIDUAL, (double)nb * BRICK_CELLS * (zero_phi ? 8.0 : 16.0 + W));
        launch_level_norms(st, D.d_ranges, (int)D.range_prob.size(), D.part, D.dnorm + noff, o.norm_p,
                           publish ? D.h_pub + pub_off : nullptr, pub_alt, D.h_seq, D.d_seqc);
    }

    void smooth(int k, int nu, bool pre)
    {
        int b0 = step_b0(k), nb = step_nb(k);
        const T *cp = pre ? nullptr : cpe;
        const double n = (double)nb * BRICK_CELLS;
        if (o.smoother == AMRMG_GSRB_GLOBAL) {
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

    bool hybrid() const { return o.smoother == AMRMG_GSRB; }

    void pre_hybrid(int k)
    {
        int b0 = step_b0(k), nb = step_nb(k);
        const double n = (double)nb * BRICK_CELLS;
        T *out = (o.nu1 % 2 == 1) ? e : et;
        // the last pre-smoothing sweep also writes the fine sums of e that the
        // restriction's coarse-fine update reads
        pb(AMRMG_K_GSRB);
        launch_hgs<T>(st, D.M, b0, nb, nullptr, out, r, nullptr, D.phib, D.ffs, o.nu1 <= 1 ? 1 | 16 : 1, hgs_nt(k));
        pe(AMRMG_K_GSRB, 2.0 * n * W);
        T *src = out;
        for (int i = 1; i < o.nu1; ++i) {
            T *dst = (src == e) ? et : e;
            pb(AMRMG_K_GSRB);
            launch_hgs<T>(st, D.M, b0, nb, src, dst, r, nullptr, D.phib, D.ffs, i == o.nu1 - 1 ? 16 : 0, hgs_nt(k));
            pe(AMRMG_K_GSRB, 3.0 * n * W);
            src = dst;
        }
    }

    void post_hybrid(int k)
    {
        int b0 = step_b0(k), nb = step_nb(k);
        const double n = (double)nb * BRICK_CELLS;
        T *src = e;
        for (int i = 0; i < o.nu2; ++i) {
            T *dst = (src == e) ? et : e;
            int mode = (i == 0 ? 2 | 4 : 0) | (i == o.nu2 - 1 ? 8 : 0);
            pb(AMRMG_K_GSRB);
            launch_hgs<T>(st, D.M, b0, nb, src, dst, r, cpe, D.phib, D.ffs, mode, hgs_nt(k));
            // e, r in; e out; the parent value with the fused prolongation;
            // phi read and written on AMR bricks with the fused update
            pe(AMRMG_K_GSRB, (3.0 + (i == 0 ? 0.125 : 0.0)) * n * W + ((mode & 8) ? 16.0 * step_amr_cells(k) : 0.0));
            src = dst;
        }
        if (src != e) launch_copy<T>(st, et + (size_t)b0 * BRICK_CELLS, e + (size_t)b0 * BRICK_CELLS, (int64_t)nb * BRICK_CELLS);
    }

    void vcycle()
    {
        const int kc = D.kc;
        for (int k = m.K - 1; k > kc; --k) {
            if (hybrid())
                pre_hybrid(k);
            else
                smooth(k, o.nu1, true);
            double n = (double)step_nb(k) * BRICK_CELLS;
            // restriction into level k-1 together with the coarse-fine
            // update of its cells next to level k
            const auto &e0 = m.ent[m.step_ent0[k - 1]];
            const auto &e1 = m.ent[m.step_ent0[k] - 1];
            int rf0 = e0.rf0, nrf = e1.rf0 + e1.nrf - e0.rf0;
            if (!hybrid()) {  // the hybrid sweep writes the fine sums itself
                const auto &f0 = m.ent[m.step_ent0[k]];
                const auto &f1 = m.ent[m.step_ent0[k + 1] - 1];
                launch_face_sums<T>(st, D.M, f0.cf0, f1.cf0 + f1.ncf - f0.cf0, e, D.ffs);
            }
            pb(AMRMG_K_RESTRICT);
            launch_restrict<T>(st, D.M, step_b0(k), step_nb(k), D.d_reflux + rf0, nrf, e, r, D.ffs);
            pe(AMRMG_K_RESTRICT, (2.0 + 0.125) * n * W + 2.0 * nrf * BRICK_CELLS * W);
        }
        pb(AMRMG_K_BOTTOM);
        launch_direct<T>(st, D.d_djobs, D.d_planes, D.n_planes, D.d_groups, D.n_groups, D.d_dtab, D.dw, r, e, D.phib,
                         hybrid(), D.direct_maxdim, D.n_djobs == 1 ? &D.djob0 : nullptr);
        if (D.n_cg > 0)
            launch_coarse_cycle<T>(st, D.M, D.d_cjobs, D.njobs, e, r, D.cgw, o.nu1, o.nu2, o.bottom_rtol, 10000,
                                   D.cgit, D.phib, hybrid(), D.cg_threads);
        pe(AMRMG_K_BOTTOM, (double)D.cg_doubles / 4 * (2 * W));
        for (int k = kc + 1; k < m.K; ++k) {
            if (hybrid()) {
                post_hybrid(k);
                continue;
            }
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
        if (hybrid()) return;  // phi updated by the last sweep of each level and in the coarse cycle
        int b0, nb;
        const int32_t *list;
        amr_range(b0, nb, list);
        pb(AMRMG_K_PHI_UPDATE);
        launch_phi_update<T>(st, D.M, b0, nb, list, D.phib, e);
        pe(AMRMG_K_PHI_UPDATE, (double)nb * BRICK_CELLS * (16.0 + W));
    }

    // phi (and rho) between the caller's layout and brick layout
    void to_bricks(bool with_rho)
    {
        int b0, nb;
        const int32_t *list;
        amr_range(b0, nb, list);
        launch_user_brick(st, D.M, b0, nb, list, true, D.d_phi, D.phib, with_rho ? D.d_rho : nullptr,
                          with_rho ? D.rhob : nullptr);
    }
    void from_bricks()
    {
        int b0, nb;
        const int32_t *list;
        amr_range(b0, nb, list);
        launch_user_brick(st, D.M, b0, nb, list, false, D.d_phi, D.phib, nullptr, nullptr);
    }

    // one outer iteration: V-cycle, phi += e, FP64 residual and its norms
    // (published to h_pub[2 nr ..] or h_pub[3 nr ..] in turn)
    void iteration(int nr)
    {
        vcycle();
        outer(false, nr, nullptr, true, 2 * nr, nr);
    }
};

// The graph of one outer iteration, captured and instantiated once per
// hierarchy, workspace and option set; iterate launches it (or the kernels
// themselves when graphs are off or launches are being timed).
template <class T>
static amrmg_status ensure_graph(DevState &D, int nr, const SolveOpts &o)
{
    std::vector<int64_t> key = {D.meta_gen, (int64_t)(intptr_t)D.ws, (int64_t)sizeof(T), o.smoother, o.nu1, o.nu2,
                                o.norm_p, (int64_t)(o.omega * 1e12), (int64_t)(o.bottom_rtol * 1e15),
                                (int64_t)(o.inv_eps0 * 1e12)};
    if (D.gexec && D.gkey == key) return AMRMG_OK;
    D.drop_graph();
    if (!D.cap_stream) HIP_TRY(hipStreamCreateWithFlags(&D.cap_stream, hipStreamNonBlocking));
    Driver<T> cap(D, D.cap_stream, o, nullptr);
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(D.cap_stream, hipStreamCaptureModeThreadLocal));
    cap.iteration(nr);
    hipError_t ec = hipStreamEndCapture(D.cap_stream, &g);
    if (ec != hipSuccess) return fail(AMRMG_E_HIP, std::string("graph capture: ") + hipGetErrorString(ec));
    hipError_t ei = hipGraphInstantiate(&D.gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
        D.gexec = nullptr;
        return fail(AMRMG_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(ei));
    }
    D.gkey = key;
    return AMRMG_OK;
}

template <class T>
static amrmg_status iterate(DevState &D, Driver<T> &drv, hipStream_t st, int nr, const SolveOpts &o, bool graphs)
{
    if (!graphs || drv.P) {
        drv.iteration(nr);
        return AMRMG_OK;
    }
    ST_TRY(ensure_graph<T>(D, nr, o));
    HIP_TRY(hipGraphLaunch(D.gexec, st));
    return AMRMG_OK;
}

// run a solve on a DevState whose pointer tables are set; per-problem stats
// Events that time a solve: two made for it (and destroyed with it), or the
// caller's pair when it may make none.
struct SolveTimers {
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool own = false;
    ~SolveTimers()
    {
        if (own)
            for (auto e : ev)
                if (e) (void)hipEventDestroy(e);
    }
};

// ev_fixed: the context's pair of timing events (made with it), or nullptr
// (two are made for this solve).  noalloc: the solve may allocate nothing --
// no sweep tuning (the tuned or the size rule's threads per brick), no graph
// (eager launches), the events of ev_fixed
template <class T>
static amrmg_status run_solve(DevState &D, hipStream_t st, const SolveOpts &o, double tol,
                              std::vector<amrmg_solve_stats> &stats, bool want_E, Prof *prof,
                              const hipEvent_t *ev_fixed, bool noalloc)
{
    const Meta &m = D.meta;
    Driver<T> drv(D, st, o, prof);
    const int nr = (int)D.range_prob.size();
    const int np = (int)m.prob_ent.size();
    if (noalloc && !ev_fixed) return fail(AMRMG_E_HIP, "a solve without allocation needs the context's events");
    SolveTimers evs;
    if (ev_fixed && ev_fixed[0] && ev_fixed[1]) {
        evs.ev[0] = ev_fixed[0];
        evs.ev[1] = ev_fixed[1];
    } else {
        evs.own = true;
        HIP_TRY(hipEventCreate(&evs.ev[0]));
        HIP_TRY(hipEventCreate(&evs.ev[1]));
    }
    hipEvent_t ev0 = evs.ev[0], ev1 = evs.ev[1];
    const bool graphs = g_use_graphs && !noalloc;
    // the iteration's graph is captured and instantiated first, while the
    // stream may still be busy with the caller's earlier work (the deposit)
    if (o.smoother == AMRMG_GSRB && !noalloc) ST_TRY(drv.tune());
    if (graphs && !prof && o.max_iters > 0) ST_TRY(ensure_graph<T>(D, nr, o));
    HIP_TRY(hipMemsetAsync(D.cgit, 0, 64, st));  // CG iteration count and the norm sequence counter
    D.seq = 0;
    *(volatile unsigned *)D.h_seq = 0;
    HIP_TRY(hipEventRecord(ev0, st));
    // norms of b (zero phi) to h_pub[nr ..], of the initial residual to
    // h_pub[0 ..]; each publication bumps the sequence number, and those of
    // the iterations alternate between two slots after these
    drv.to_bricks(true);
    drv.outer(true, 0, nullptr, true, nr);
    drv.outer(false, nr, nullptr, true, 0);
    HIP_TRY(hipGetLastError());
    // the first iteration is queued before the initial norms are read; when
    // the initial guess already meets the tolerance it only refines phi, and
    // the norms reported are those after it
    const bool first_queued = o.max_iters > 0;
    if (first_queued) ST_TRY(iterate<T>(D, drv, st, nr, o, graphs));
    // wait for publication number want in host memory (no stream
    // synchronisation); after a second without it, synchronise and look again
    auto wait_pub = [&](unsigned want) -> amrmg_status {
        auto t0 = std::chrono::steady_clock::now();
        for (unsigned spin = 0; *(volatile unsigned *)D.h_seq < want; ++spin) {
            if ((spin & 1023) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::seconds(1)) {
                HIP_TRY(hipStreamSynchronize(st));
                if (*(volatile unsigned *)D.h_seq < want)
                    return fail(AMRMG_E_HIP, "the iteration's norms did not reach the host");
                break;
            }
        }
        HIP_TRY(hipGetLastError());
        return AMRMG_OK;
    };
    D.seq = 2;
    ST_TRY(wait_pub(D.seq));
    std::vector<double> bn(D.h_pub + nr, D.h_pub + 2 * nr), rn(D.h_pub, D.h_pub + nr);
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
    // the least converged level's residual in units of its target
    auto worst = [&]() {
        double w = 0.0;
        for (int i = 0; i < nr; ++i) {
            const double lim = tol * bn[i];
            w = std::max(w, lim > 0.0 ? rn[i] / lim : (rn[i] > 0.0 ? HUGE_VAL : 0.0));
        }
        return w;
    };
    // the norms of the iteration whose publication was the last awaited
    // (sequence numbers 3, 5, ... in h_pub[2 nr ..], 4, 6, ... in h_pub[3 nr ..])
    auto read_iter = [&]() {
        const double *src = D.h_pub + (2 + (D.seq & 1u ? 0 : 1)) * nr;
        rn.assign(src, src + nr);
    };
    int it = 0, queued = first_queued ? 1 : 0;
    bool all = check(0);
    if (first_queued) {
        ST_TRY(wait_pub(++D.seq));
        read_iter();
        it = 1;
        if (!all) all = check(1);
    }
    while (!all && it < o.max_iters) {
        if (queued == it) {
            ST_TRY(iterate<T>(D, drv, st, nr, o, graphs));
            ++queued;
        }
        // While the last norms lie more than kAhead times above the target,
        // the iteration already queued cannot reach it (a V-cycle reduces
        // the residual about tenfold), so the one after it will run too:
        // queue it now, and the GPU does not wait for the host between them.
        if (queued == it + 1 && queued < o.max_iters && worst() > kAhead) {
            ST_TRY(iterate<T>(D, drv, st, nr, o, graphs));
            ++queued;
        }
        ST_TRY(wait_pub(++D.seq));
        read_iter();
        ++it;
        all = check(it);
    }
    // an iteration queued beyond the last one read runs all the same: its
    // norms are the solve's
    while (it < queued) {
        ST_TRY(wait_pub(++D.seq));
        read_iter();
        ++it;
        all = check(it) || all;
    }
    // average down, finest first, then the field
    for (int k = m.K - 1; k >= 1; --k)
        for (int ei = m.step_ent0[k]; ei < m.step_ent0[k + 1]; ++ei)
            if (m.ent[ei].amr >= 1) {
                drv.pb(AMRMG_K_AVGDOWN);
                launch_avgdown(st, D.M, m.ent[ei].b0, m.ent[ei].nb, D.phib);
                drv.pe(AMRMG_K_AVGDOWN, (double)m.ent[ei].nb * BRICK_CELLS * 8.0 * (1.0 + 0.125));
            }
    if (want_E) {
        int b0, nb;
        const int32_t *list;
        drv.amr_range(b0, nb, list);
        drv.pb(AMRMG_K_EFIELD);
        launch_efield(st, D.M, b0, nb, list, D.phib, D.cpphi, D.d_E);
        drv.pe(AMRMG_K_EFIELD, (double)nb * BRICK_CELLS * 32.0);
    }
    drv.from_bricks();
    HIP_TRY(hipEventRecord(ev1, st));
    HIP_TRY(hipEventSynchronize(ev1));
    HIP_TRY(hipGetLastError());
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ev0, ev1));
    int cgmax = 0;  // only a CG bottom solve counts iterations
    if (D.n_cg > 0) HIP_TRY(hipMemcpy(&cgmax, D.cgit, sizeof(int), hipMemcpyDeviceToHost));
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
    double **h = (double **)D.ptrstage.p;
    std::memcpy(h, D.h_phi.data(), sizeof(double *) * ne);
    std::memcpy(h + ne, D.h_rho.data(), sizeof(double *) * ne);
    std::memcpy(h + 2 * ne, D.h_rout.data(), sizeof(double *) * ne);
    std::memcpy(h + 3 * ne, D.h_E.data(), sizeof(double *) * 3 * ne);
    HIP_TRY(hipMemcpyAsync(D.ptrbuf.p, h, sizeof(double *) * 6 * ne, hipMemcpyHostToDevice, st));
    return AMRMG_OK;
}

// check the arguments of a solve and record the caller's level arrays in the
// pointer tables of the context's DevState
static amrmg_status bind_solve_levels(amrmg_ctx *ctx, double *const *rho, double *const *phi, double *const *E,
                                      double tol)
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
    std::fill(D.h_rout.begin(), D.h_rout.end(), nullptr);
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
    return AMRMG_OK;
}

static amrmg_status solve_bound(amrmg_ctx *ctx, bool want_E, double tol, amrmg_solve_stats *stats, bool noalloc)
{
    DevState &D = ctx->ds;
    ST_TRY(set_tables(D, ctx->st));
    std::vector<amrmg_solve_stats> sv;
    SolveOpts o = opts_of(ctx->P);
    Prof *pf = ctx->prof.mask ? &ctx->prof : nullptr;
    amrmg_status rc = ctx->P.precision == AMRMG_MIXED
                          ? run_solve<float>(D, ctx->st, o, tol, sv, want_E, pf, ctx->ev_solve, noalloc)
                          : run_solve<double>(D, ctx->st, o, tol, sv, want_E, pf, ctx->ev_solve, noalloc);
    if (stats && !sv.empty()) *stats = sv[0];
    if (rc == AMRMG_E_NOT_CONVERGED) (void)fail(rc, "not converged within max_iters");
    return rc;
}

extern "C" amrmg_status amrmg_solve(amrmg_ctx *ctx, double *const *rho, double *const *phi, double *const *E,
                                    double tol, amrmg_solve_stats *stats)
{
    ST_TRY(bind_solve_levels(ctx, rho, phi, E, tol));
    ST_TRY(ensure_ws(ctx->ds, ctx->P.precision, ctx->user_ws, ctx->user_ws_bytes));
    return solve_bound(ctx, E != nullptr, tol, stats, false);
}

static_assert(NOALLOC_SCRATCH_BYTES == AMRMG_NOALLOC_SCRATCH_BYTES, "header and array sizes differ");

extern "C" amrmg_status amrmg_solve_noalloc(amrmg_ctx *ctx, double *const *rho, double *const *phi,
                                            double *const *E, double tol, amrmg_solve_stats *stats)
{
    ST_TRY(bind_solve_levels(ctx, rho, phi, E, tol));
    hipError_t se = hipSuccess;
    void *scr = noalloc_scratch(ctx->device, &se);
    if (!scr)
        return fail(AMRMG_E_HIP, "the no-allocation scratch array has no address on device " +
                                     std::to_string(ctx->device) + ": " + hipGetErrorString(se));
    if (!ctx->ev_solve[0] || !ctx->ev_solve[1])
        return fail(AMRMG_E_HIP, "the context's timing events were not created");
    const size_t need = ws_need(ctx->ds, ctx->P.precision);
    if (need > NOALLOC_SCRATCH_BYTES)
        return fail(AMRMG_E_OOM, "the hierarchy needs " + std::to_string(need) + " bytes of workspace; "
                                 "amrmg_solve_noalloc has " + std::to_string(NOALLOC_SCRATCH_BYTES));
    ST_TRY(ensure_ws(ctx->ds, ctx->P.precision, scr, NOALLOC_SCRATCH_BYTES));
    return solve_bound(ctx, E != nullptr, tol, stats, true);
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
    std::fill(D.h_E.begin(), D.h_E.end(), nullptr);
    for (int l = 0; l < pr.namr(); ++l) {
        if (!rho[l] || !phi[l] || !r[l]) return fail(AMRMG_E_INVALID, "level arrays must be set");
        int ei = D.meta.prob_ent[0][pr.kg + l];
        D.h_phi[ei] = phi[l];
        D.h_rho[ei] = rho[l];
        D.h_rout[ei] = r[l];
    }
    ST_TRY(ensure_ws(D, ctx->P.precision, ctx->user_ws, ctx->user_ws_bytes));
    ST_TRY(set_tables(D, ctx->st));
    SolveOpts o = opts_of(ctx->P);
    Driver<double> drv(D, ctx->st, o, nullptr);
    drv.to_bricks(true);
    drv.outer(false, 0, D.d_rout);
    HIP_TRY(hipStreamSynchronize(ctx->st));
    HIP_TRY(hipGetLastError());
    return AMRMG_OK;
}

extern "C" amrmg_status amrmg_solve_batch(amrmg_ctx *const *ctxs, int32_t nb, double *const *const *rho,
                                          double *const *const *phi, double tol, amrmg_solve_stats *stats)
{
    if (!ctxs || nb <= 0) return fail(AMRMG_E_INVALID, "need at least one context");
    if (!rho || !phi) return fail(AMRMG_E_INVALID, "rho and phi are required");
    if (!(tol > 0)) return fail(AMRMG_E_INVALID, "tol must be positive");
    amrmg_ctx *c0 = ctxs[0];
    for (int i = 0; i < nb; ++i) {
        const amrmg_ctx *c = ctxs[i];
        if (!c) return fail(AMRMG_E_INVALID, "context " + std::to_string(i) + " is NULL");
        if (!c->built) return fail(AMRMG_E_STATE, "context " + std::to_string(i) + ": hierarchy not built");
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == c) return fail(AMRMG_E_INVALID, "a context appears twice in the batch");
        const amrmg_params &a = c0->P, &b = c->P;
        if (c->st != c0->st || a.precision != b.precision || a.smoother != b.smoother || a.nu1 != b.nu1 ||
            a.nu2 != b.nu2 || a.norm_p != b.norm_p || a.omega != b.omega || a.max_iters != b.max_iters ||
            a.bottom != b.bottom || a.bottom_rtol != b.bottom_rtol || a.eps0 != b.eps0)
            return fail(AMRMG_E_INVALID, "context " + std::to_string(i) + ": stream or solver settings differ");
        if (!rho[i] || !phi[i]) return fail(AMRMG_E_INVALID, "rho[i] and phi[i] are required");
    }
    // merged metadata of the batch, kept by the first context until one of
    // the contexts builds a new hierarchy
    std::vector<amrmg_ctx *> key(ctxs, ctxs + nb);
    std::vector<int> gen(nb);
    for (int i = 0; i < nb; ++i) gen[i] = ctxs[i]->generation;
    if (!c0->batch || c0->batch_ctx != key || c0->batch_gen != gen) {
        delete c0->batch;
        c0->batch = new DevState();
        c0->batch_ctx.clear();
        std::vector<const Problem *> probs;
        for (int i = 0; i < nb; ++i) probs.push_back(&ctxs[i]->prob);
        ST_TRY(upload_meta(*c0->batch, c0->st, probs, c0->P.bottom == AMRMG_BOTTOM_AUTO));
        HIP_TRY(hipStreamSynchronize(c0->st));
        if (!c0->batch->meta.error.empty()) return fail(AMRMG_E_NESTING, c0->batch->meta.error);
        if (*(int *)c0->batch->h_face_err.p)
            return fail(AMRMG_E_NESTING, "coarse-fine window leaves the coarser level (nesting violated)");
        c0->batch_ctx = key;
        c0->batch_gen = gen;
    }
    DevState &D = *c0->batch;
    std::fill(D.h_phi.begin(), D.h_phi.end(), nullptr);
    std::fill(D.h_rho.begin(), D.h_rho.end(), nullptr);
    std::fill(D.h_E.begin(), D.h_E.end(), nullptr);
    std::fill(D.h_rout.begin(), D.h_rout.end(), nullptr);
    for (int i = 0; i < nb; ++i) {
        const Problem &pr = ctxs[i]->prob;
        for (int l = 0; l < pr.namr(); ++l) {
            if (!rho[i][l] || !phi[i][l]) return fail(AMRMG_E_INVALID, "rho[i][l] and phi[i][l] must be set");
            int ei = D.meta.prob_ent[i][pr.kg + l];
            D.h_phi[ei] = phi[i][l];
            D.h_rho[ei] = rho[i][l];
        }
    }
    ST_TRY(ensure_ws(D, c0->P.precision, nullptr, 0));
    ST_TRY(set_tables(D, c0->st));
    std::vector<amrmg_solve_stats> sv;
    SolveOpts o = opts_of(c0->P);
    amrmg_status rc = c0->P.precision == AMRMG_MIXED
                          ? run_solve<float>(D, c0->st, o, tol, sv, false, nullptr, c0->ev_solve, false)
                          : run_solve<double>(D, c0->st, o, tol, sv, false, nullptr, c0->ev_solve, false);
    if (stats)
        for (int i = 0; i < nb && i < (int)sv.size(); ++i) stats[i] = sv[i];
    if (rc == AMRMG_E_NOT_CONVERGED) (void)fail(rc, "not every problem converged within max_iters");
    return rc;
}
