// amrmg_api.cpp -- the C ABI of libamrmg (include/amrmg.h): contexts, the
// hierarchy build, deposit and gather, and the solve driver that runs the
// composite AMR multigrid of arXiv:1812.03689 (Alg. 2 and Alg. 3) on the HIP
// kernels of amrmg_kernels.hip.
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
static size_t align8(size_t x) { return (x + 7) & ~(size_t)7; }

// ---------------------------------------------------------------------------
// grow-only device and pinned host buffers (allocation happens only when a
// hierarchy outgrows its predecessor, so regrids do not reallocate)
// ---------------------------------------------------------------------------
struct DBuf {
    void *p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t n)
    {
        if (n <= cap && p) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
        size_t c = n + n / 4 + 4096;
        hipError_t e = hipMalloc(&p, c);
        if (e == hipSuccess) cap = c;
        return e;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
    ~DBuf() { release(); }
};

// host memory the device writes and the host polls (coherent, mapped)
struct CBuf {
    void *p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t n)
    {
        if (n <= cap && p) return hipSuccess;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
        hipError_t e = hipHostMalloc(&p, n, hipHostMallocCoherent | hipHostMallocMapped);
        if (e == hipSuccess) {
            cap = n;
            std::memset(p, 0, n);
        }
        return e;
    }
    ~CBuf()
    {
        if (p) (void)hipHostFree(p);
    }
};

struct PBuf {
    void *p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t n)
    {
        if (n <= cap && p) return hipSuccess;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
        size_t c = n + n / 4 + 4096;
        hipError_t e = hipHostMalloc(&p, c);
        if (e == hipSuccess) cap = c;
        return e;
    }
    ~PBuf()
    {
        if (p) (void)hipHostFree(p);
    }
};

// Packs host arrays into one pinned staging buffer and one device buffer
// with a single host-to-device copy.
struct Packer {
    struct Item {
        const void *src;
        size_t bytes, off;
        void **dst;
    };
    std::vector<Item> items;
    size_t total = 0;
    template <class V>
    void add(const std::vector<V> &v, V **dst)
    {
        add_raw(v.data(), sizeof(V) * v.size(), (void **)dst);
    }
    void add_raw(const void *src, size_t bytes, void **dst)
    {
        items.push_back({src, bytes, total, dst});
        total += align256(bytes ? bytes : 1);
    }
    amrmg_status run(DBuf &dev, PBuf &stage, hipStream_t st)
    {
        HIP_TRY(stage.ensure(total));
        HIP_TRY(dev.ensure(total));
        for (auto &it : items) {
            if (it.bytes) std::memcpy((char *)stage.p + it.off, it.src, it.bytes);
            *it.dst = (char *)dev.p + it.off;
        }
        HIP_TRY(hipMemcpyAsync(dev.p, stage.p, total, hipMemcpyHostToDevice, st));
        return AMRMG_OK;
    }
};

#define ST_TRY(x)                                \
    do {                                         \
        amrmg_status s_ = (x);                   \
        if (s_ != AMRMG_OK) return s_;           \
    } while (0)

// ---------------------------------------------------------------------------
// device copy of merged metadata plus the solve workspace
// ---------------------------------------------------------------------------
struct DevState {
    Meta meta;
    DevMeta M{};
    DBuf metabuf;
    PBuf stage;
    // brick tables built on the device (org, nbr, child, ... and the scan
    // scratch); per-level counts come back through bsum
    DBuf brickbuf;
    CBuf bsum;
    unsigned bseq = 0;
    int n_amr = 0, amr_first = 0, n_reflux = 0;  // AMR bricks (list d_amr), update list length
    int32_t *d_reflux = nullptr, *d_amr = nullptr;
    int2 *d_ranges = nullptr;  // brick range of each AMR level of each problem
    std::vector<int> range_prob, range_amr;
    int4 *d_jobs = nullptr;
    int njobs = 0;
    size_t cg_doubles = 0;
    CoarseJob *d_cjobs = nullptr;
    int n_cg = 0;  // problems whose coarsest grid is solved by CG
    // direct solves of the coarsest grids: tables, jobs, work lists, scratch
    double *d_dtab = nullptr;
    DirectJob *d_djobs = nullptr;
    int2 *d_planes = nullptr, *d_groups = nullptr;
    int n_planes = 0, n_groups = 0, direct_maxdim = 0;
    int n_djobs = 0;
    DirectJob djob0{};  // host copy of the job when there is one
    size_t dw_doubles = 0;
    double *dw = nullptr;
    int kc = 0;  // levels 0..kc of every problem run in the one-workgroup coarse cycle
    // per-level pointer tables: phi[ne], rho[ne], rout[ne], E[3 ne]
    DBuf ptrbuf;
    PBuf ptrstage;
    double **d_phi = nullptr, **d_rho = nullptr, **d_E = nullptr, **d_rout = nullptr;
    std::vector<double *> h_phi, h_rho, h_E, h_rout;
    // workspace
    DBuf ws_own;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    int ws_prec = -1;
    void *e = nullptr, *r = nullptr, *et = nullptr, *cpe = nullptr;
    double *cpphi = nullptr, *part = nullptr, *dnorm = nullptr;
    double *ffs = nullptr;  // fine sums of coarse-fine faces, 96 per brick
    double *phib = nullptr, *rhob = nullptr;  // FP64 phi and rho in brick layout during a solve
    double *cgw = nullptr;
    int *cgit = nullptr;
    int cg_threads = 1024;
    PBuf h_normbuf;
    double *h_norm = nullptr;
    // norms of each outer iteration, published by the norms kernel: values,
    // then a sequence number; the device keeps the count at d_seqc
    CBuf pubbuf;
    double *h_pub = nullptr;
    unsigned *h_seq = nullptr, *d_seqc = nullptr;
    unsigned seq = 0;
    // AMR-level brick maps with global brick ids of the first problem (views
    // into the map pool)
    std::vector<int32_t *> d_bmap;
    // face data generated on the device: gbc, cf_pat, cf_idx, error flag
    DBuf facebuf;
    int *d_face_err = nullptr;
    PBuf h_face_err;
    // captured outer iteration (V-cycle, phi update, FP64 residual, norms)
    hipGraphExec_t gexec = nullptr;
    std::vector<int64_t> gkey;
    int meta_gen = 0;
    hipStream_t cap_stream = nullptr;  // capture needs a stream other than the null stream
    void drop_graph()
    {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        gexec = nullptr;
        gkey.clear();
    }
    ~DevState()
    {
        drop_graph();
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }
};

static bool g_weights_ok = false;

// direct-solve tables by grid shape and spacing (they depend on nothing else;
// a regrid keeps level 0 and so its coarsest grid)
static const std::vector<double> &cached_direct_tables(const int n[3], const double h[3], const double a[3])
{
    struct Key {
        int n[3];
        double h[3], a[3];
        bool operator<(const Key &o) const
        {
            for (int d = 0; d < 3; ++d) {
                if (n[d] != o.n[d]) return n[d] < o.n[d];
                if (h[d] != o.h[d]) return h[d] < o.h[d];
                if (a[d] != o.a[d]) return a[d] < o.a[d];
            }
            return false;
        }
    };
    static thread_local std::map<Key, std::vector<double>> cache;
    Key k{{n[0], n[1], n[2]}, {h[0], h[1], h[2]}, {a[0], a[1], a[2]}};
    auto it = cache.find(k);
    if (it == cache.end()) {
        if (cache.size() > 64) cache.clear();
        it = cache.emplace(k, direct_tables(n, h, a)).first;
    }
    return it->second;
}

// the direct_tables layout with every matrix zero-padded to P x P, P = n
// rounded up to a multiple of 16 (the matrix-core tile), and stored in the
// order the matrix cores take it: for row block rb and step s, 64 values,
// value l = M[16 rb + l % 16][4 s + l / 16]; eigenvalues as they are
static void append_padded_tables(std::vector<double> &out, const int n[3], const std::vector<double> &t)
{
    size_t off = 0;
    for (int d = 0; d < 3; ++d) {
        const int N = n[d], P = (N + 15) & ~15;
        for (int m = 0; m < 2; ++m, off += (size_t)N * N) {
            const size_t base = out.size();
            out.resize(base + (size_t)P * P, 0.0);
            for (int rb = 0; rb < P / 16; ++rb)
                for (int s = 0; s < P / 4; ++s)
                    for (int l = 0; l < 64; ++l) {
                        const int a = 16 * rb + l % 16, b = 4 * s + l / 16;
                        if (a < N && b < N)
                            out[base + ((size_t)rb * (P / 4) + s) * 64 + l] = t[off + (size_t)a * N + b];
                    }
        }
    }
    out.insert(out.end(), t.begin() + off, t.end());
}

// Upload D.meta (built without face data) in one copy, then generate the
// face data (boundary values, coarse-fine windows) on the device.
static amrmg_status upload_meta(DevState &D, hipStream_t st, const std::vector<const Problem *> &probs,
                                bool direct)
{
    Meta &m = D.meta;
    meta_entries(probs, m);
    if (!g_weights_ok) {
        std::vector<double> W = cf_weight_table();
        HIP_TRY(upload_cf_weights(W.data()));
        uint32_t masks[13];
        int org[42];
        pattern_tables(masks, org);
        HIP_TRY(upload_pattern_tables(masks, org));
        g_weights_ok = true;
    }
    // level table, box table, monopoles; the brick maps of every level are
    // built on the device into the map pool
    static thread_local std::vector<EntryDev> ed;
    static thread_local std::vector<BoxDev> bx;
    static thread_local std::vector<double> mono;
    static thread_local std::vector<int> mono_off;
    ed.assign(m.ent.size(), EntryDev{});
    bx.clear();
    mono.clear();
    mono_off.assign(probs.size(), 0);
    for (size_t i = 0; i < probs.size(); ++i) {
        mono_off[i] = (int)(mono.size() / 4);
        mono.insert(mono.end(), probs[i]->mono.begin(), probs[i]->mono.begin() + (probs[i]->mono.size() / 4) * 4);
    }
    std::vector<int64_t> amr_off;  // pool offset of AMR level l of problem 0
    int64_t npool = 0;
    int n_amr = 0;
    for (size_t ei = 0; ei < m.ent.size(); ++ei) {
        const Meta::Entry &e = m.ent[ei];
        const Problem &P = *probs[e.prob];
        const HostLevel &L = P.lev[e.k];
        EntryDev &E = ed[ei];
        for (int d = 0; d < 3; ++d) {
            E.lo[d] = P.lo[d];
            E.h[d] = L.h[d];
            E.n[d] = L.n[d];
            E.nbk[d] = L.nbk[d];
        }
        E.eps0 = P.eps0;
        E.amr = L.amr;
        E.crse = e.k > 0 ? m.prob_ent[e.prob][e.k - 1] : -1;
        E.mono_off = mono_off[e.prob];
        E.mono_n = (int)(P.mono.size() / 4);
        E.b0 = e.b0;
        E.nb = e.nb;
        E.bmap_off = (int)npool;
        if (L.amr >= 0 && e.prob == 0) amr_off.push_back(npool);
        npool += (int64_t)L.nbk[0] * L.nbk[1] * L.nbk[2];
        E.amr_pos = L.amr >= 0 ? n_amr : 0;
        if (L.amr >= 0) n_amr += e.nb;
        int g0 = e.b0;
        for (size_t b = 0; b < L.boxes.size(); ++b) {
            const Box &B = L.boxes[b];
            BoxDev t{};
            for (int d = 0; d < 3; ++d) {
                t.lo[d] = B.lo[d] / 8;
                t.ext[d] = (B.hi[d] - B.lo[d]) / 8;
            }
            t.g0 = g0;
            t.ent = (int)ei;
            t.uoff = L.off.size() > b ? L.off[b] : 0;
            t.nx = B.hi[0] - B.lo[0];
            t.ny = B.hi[1] - B.lo[1];
            g0 += t.ext[0] * t.ext[1] * t.ext[2];
            bx.push_back(t);
        }
    }
    if (npool > (int64_t)INT32_MAX) return fail(AMRMG_E_INVALID, "brick maps exceed 2^31 entries");
    D.n_amr = n_amr;
    D.amr_first = 0;
    for (const auto &e : m.ent)
        if (e.amr >= 0) {
            D.amr_first = e.b0;
            break;
        }
    if (mono.empty()) mono.push_back(0.0);
    static thread_local std::vector<LevelConst> lc;
    lc.assign(m.ent.size(), LevelConst{});
    for (size_t i = 0; i < m.ent.size(); ++i) {
        for (int d = 0; d < 3; ++d) {
            lc[i].h[d] = m.ent[i].h[d];
            lc[i].ih2[d] = 1.0 / (m.ent[i].h[d] * m.ent[i].h[d]);
        }
        boundary_ghost(*probs[m.ent[i].prob], m.ent[i].h, lc[i].abnd);
        lc[i].amr = m.ent[i].amr;
    }
    // norm ranges: every AMR level of every problem, entry order
    static thread_local std::vector<int32_t> rg, jobs;
    rg.clear();
    D.range_prob.clear();
    D.range_amr.clear();
    for (const auto &e : m.ent)
        if (e.amr >= 0) {
            rg.push_back(e.b0);
            rg.push_back(e.nb);
            D.range_prob.push_back(e.prob);
            D.range_amr.push_back(e.amr);
        }
    // bottom solves: the coarsest level of each problem
    jobs.clear();
    size_t off = 0;
    for (size_t i = 0; i < m.prob_ent.size(); ++i) {
        const auto &e = m.ent[m.prob_ent[i][0]];
        jobs.push_back(e.b0);
        jobs.push_back(e.nb);
        jobs.push_back((int32_t)off);
        jobs.push_back(0);
        off += (size_t)4 * e.nb * BRICK_CELLS;
    }
    D.njobs = (int)m.prob_ent.size();
    D.cg_doubles = off;
    // coarse part: levels 0..kc with at most 8 bricks above level 0 and no
    // coarse-fine faces (at most AMR level 0), the same kc for all problems
    const int kMaxCoarseBricks = 0;  // the coarse kernel runs the CG on the coarsest grid only
    int kc = 1 << 20;
    for (size_t i = 0; i < m.prob_ent.size(); ++i) {
        int ki = 0;
        const auto &pe = m.prob_ent[i];
        for (int k = 1; k < (int)pe.size() && k < 8; ++k) {
            const auto &e = m.ent[pe[k]];
            if (e.amr > 0 || e.nb > kMaxCoarseBricks) break;
            ki = k;
        }
        kc = std::min(kc, ki);
    }
    D.kc = kc;
    {
        int maxn = 0;
        for (size_t i = 0; i < m.prob_ent.size(); ++i) maxn = std::max(maxn, m.ent[m.prob_ent[i][0]].nb * BRICK_CELLS);
        D.cg_threads = maxn <= 512 ? 512 : 1024;
    }
    static thread_local std::vector<CoarseJob> cj;
    static thread_local std::vector<double> dtab;
    static thread_local std::vector<DirectJob> djl;
    static thread_local std::vector<int2> planes, groups;
    cj.assign(m.prob_ent.size(), CoarseJob{});
    dtab.clear();
    djl.clear();
    planes.clear();
    groups.clear();
    D.n_cg = 0;
    D.dw_doubles = 0;
    D.direct_maxdim = 0;
    for (size_t i = 0; i < m.prob_ent.size(); ++i) {
        cj[i].nlev = kc + 1;
        for (int k = 0; k <= kc; ++k) {
            cj[i].b0[k] = m.ent[m.prob_ent[i][k]].b0;
            cj[i].nb[k] = m.ent[m.prob_ent[i][k]].nb;
        }
        cj[i].cg_off = jobs[4 * i + 2];
        // direct solve of the coarsest grid when it is one full box of at
        // most DIRECT_DIM cells per axis (the levels below level 0 stop there)
        const auto &e0 = m.ent[m.prob_ent[i][0]];
        const HostLevel &L = probs[e0.prob]->lev[0];
        bool fits = direct && L.boxes.size() == 1;
        for (int d = 0; d < 3 && fits; ++d)
            fits = L.boxes[0].lo[d] == 0 && L.boxes[0].hi[d] == L.n[d] && L.n[d] <= DIRECT_DIM && L.n[d] % 4 == 0;
        cj[i].direct = fits ? 1 : 0;
        if (!fits) {
            ++D.n_cg;
            continue;
        }
        DirectJob J{};
        J.b0 = e0.b0;
        for (int d = 0; d < 3; ++d) {
            J.dn[d] = L.n[d];
            D.direct_maxdim = std::max(D.direct_maxdim, L.n[d]);
        }
        J.tab = (int)dtab.size();
        J.w = (int)D.dw_doubles;
        J.amr = L.amr >= 0 ? 1 : 0;
        double ab[3];
        boundary_ghost(*probs[e0.prob], L.h, ab);
        const std::vector<double> &t = cached_direct_tables(L.n, L.h, ab);
        append_padded_tables(dtab, L.n, t);
        D.dw_doubles += (size_t)L.n[0] * L.n[1] * L.n[2];
        const int jid = (int)djl.size();
        djl.push_back(J);
        // one workgroup per (z plane, block of 16 x frequencies)
        for (int z = 0; z < L.n[2]; ++z)
            for (int kb = 0; kb < (L.n[0] + 15) / 16; ++kb) planes.push_back(make_int2(jid, z | kb << 8));
        for (int c = 0; c < L.n[0] * L.n[1]; c += DIRECT_COLS) groups.push_back(make_int2(jid, c));
    }
    D.n_planes = (int)planes.size();
    D.n_groups = (int)groups.size();
    D.n_djobs = (int)djl.size();
    if (D.n_djobs == 1) D.djob0 = djl[0];
    if (dtab.empty()) dtab.push_back(0.0);
    if (djl.empty()) djl.push_back(DirectJob{});
    if (planes.empty()) planes.push_back(make_int2(0, 0));
    if (groups.empty()) groups.push_back(make_int2(0, 0));

    Packer P;
    int32_t *drg = nullptr, *dj = nullptr, *cfi = nullptr;
    uint8_t *cfp = nullptr;
    double *gbc = nullptr;
    LevelConst *dlc = nullptr;
    P.add(lc, &dlc);
    P.add(rg, &drg);
    P.add(jobs, &dj);
    P.add(cj, &D.d_cjobs);
    EntryDev *dent = nullptr;
    BoxDev *dbox = nullptr;
    double *dmono = nullptr;
    P.add(dtab, &D.d_dtab);
    P.add(djl, &D.d_djobs);
    P.add(planes, &D.d_planes);
    P.add(groups, &D.d_groups);
    P.add(ed, &dent);
    P.add(bx, &dbox);
    P.add(mono, &dmono);
    ST_TRY(P.run(D.metabuf, D.stage, st));

    // brick tables on the device
    const int nbr_ = m.nbrick, nent = (int)m.ent.size();
    const size_t nbp = (size_t)nbr_ + 1;
    MetaBuild B{};
    B.nbrick = nbr_;
    B.nbox = (int)bx.size();
    B.nent = nent;
    B.npool = npool;
    B.boxes = dbox;
    B.ent = dent;
    B.temp_bytes = meta_scan_temp_bytes(nbr_);
    {
        size_t o = 0;
        auto at = [&](size_t bytes) {
            size_t p = o;
            o += align256(bytes + 8);
            return p;
        };
        const size_t o_pool = at(4 * (size_t)npool), o_org = at(16 * nbp), o_ub = at(8 * nbp), o_us = at(8 * nbp),
                     o_ch = at(32 * nbp), o_par = at(4 * nbp), o_nbr = at(24 * nbp), o_gfo = at(24 * nbp),
                     o_rf = at(4 * nbp), o_amr = at(4 * nbp), o_cm = at(nbp), o_cnt = at(8 * nbp),
                     o_off = at(8 * nbp), o_flag = at(4 * nbp), o_roff = at(4 * nbp), o_dof = at(8 * (size_t)nent),
                     o_err = at(4), o_tmp = at(B.temp_bytes);
        HIP_TRY(D.brickbuf.ensure(o));
        char *p = (char *)D.brickbuf.p;
        B.pool = (int32_t *)(p + o_pool);
        B.org = (int4 *)(p + o_org);
        B.ubase = (int64_t *)(p + o_ub);
        B.ustr = (int2 *)(p + o_us);
        B.child = (int32_t *)(p + o_ch);
        B.par = (int32_t *)(p + o_par);
        B.nbr = (int32_t *)(p + o_nbr);
        B.gf_owner = (int32_t *)(p + o_gfo);
        B.reflux = (int32_t *)(p + o_rf);
        B.amr_list = (int32_t *)(p + o_amr);
        B.cmask = (uint8_t *)(p + o_cm);
        B.cnt = (uint64_t *)(p + o_cnt);
        B.off = (uint64_t *)(p + o_off);
        B.flag = (uint32_t *)(p + o_flag);
        B.roff = (uint32_t *)(p + o_roff);
        B.dof = (unsigned long long *)(p + o_dof);
        B.err = (int *)(p + o_err);
        B.temp = p + o_tmp;
    }
    HIP_TRY(D.bsum.ensure(sizeof(int32_t) * (4 * (size_t)nent + 8) + sizeof(int64_t) * ((size_t)nent + 1) + 64));
    unsigned *hseq = (unsigned *)D.bsum.p;
    B.hout = (int32_t *)((char *)D.bsum.p + 64);
    B.hdof = (int64_t *)((char *)D.bsum.p + 64 + align8(sizeof(int32_t) * (4 * (size_t)nent + 8)));
    B.hseq = hseq;
    B.seq = ++D.bseq;
    HIP_TRY(launch_meta_build(st, B));
    // the per-level counts, by polling host memory (no stream synchronisation)
    {
        auto t0 = std::chrono::steady_clock::now();
        for (unsigned spin = 0; *(volatile unsigned *)hseq != B.seq; ++spin) {
            if ((spin & 1023) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::seconds(1)) {
                HIP_TRY(hipStreamSynchronize(st));
                if (*(volatile unsigned *)hseq != B.seq)
                    return fail(AMRMG_E_HIP, "the brick-table build did not report to the host");
                break;
            }
        }
    }
    const int32_t *h = B.hout;
    m.nbc = h[4 * nent];
    m.ncf = h[4 * nent + 1];
    D.n_reflux = h[4 * nent + 2];
    if (h[4 * nent + 3]) m.error = "a brick has no parent on the coarser level (nesting violated)";
    m.dof.assign(probs.size(), std::vector<int64_t>());
    for (int ei = 0; ei < nent; ++ei) {
        Meta::Entry &e = m.ent[ei];
        e.cf0 = h[4 * ei];
        e.ncf = h[4 * ei + 1];
        e.rf0 = h[4 * ei + 2];
        e.nrf = h[4 * ei + 3];
        if (e.amr >= 0) {
            auto &dv = m.dof[e.prob];
            if ((int)dv.size() <= e.amr) dv.resize(e.amr + 1, 0);
            dv[e.amr] = B.hdof[ei];
        }
    }
    D.d_reflux = B.reflux;
    D.d_amr = B.amr_list;
    D.d_bmap.assign(amr_off.size(), nullptr);
    for (size_t l = 0; l < amr_off.size(); ++l) D.d_bmap[l] = B.pool + amr_off[l];
    // face data buffers: gbc [nbc*64], cf_idx [ncf*144], cf_pat [ncf*16], error flag
    size_t o_gbc = 0, o_idx = align256((size_t)m.nbc * 64 * 8 + 8);
    size_t o_pat = o_idx + align256((size_t)m.ncf * 144 * 4 + 4);
    size_t o_err = o_pat + align256((size_t)m.ncf * 16 + 1);
    HIP_TRY(D.facebuf.ensure(o_err + 256));
    HIP_TRY(D.h_face_err.ensure(sizeof(int)));
    char *fb = (char *)D.facebuf.p;
    gbc = (double *)(fb + o_gbc);
    cfi = (int32_t *)(fb + o_idx);
    cfp = (uint8_t *)(fb + o_pat);
    D.d_face_err = (int *)(fb + o_err);
    D.M.org = B.org;
    D.M.nbr = B.nbr;
    D.M.child = B.child;
    D.M.par = B.par;
    D.M.cmask = B.cmask;
    D.M.ubase = B.ubase;
    D.M.ustr = B.ustr;
    D.M.gf_owner = B.gf_owner;
    D.M.gbc = gbc;
    D.M.cf_pat = cfp;
    D.M.cf_idx = cfi;
    D.M.lc = dlc;
    D.M.nbc = m.nbc;
    D.M.ncf = m.ncf;
    D.d_ranges = (int2 *)drg;
    D.d_jobs = (int4 *)dj;
    int32_t *dpool = B.pool;
    HIP_TRY(hipMemsetAsync(D.d_face_err, 0, sizeof(int), st));
    launch_face_data(st, D.M, dent, dpool, dmono, gbc, cfp, cfi, D.d_face_err);
    HIP_TRY(hipGetLastError());
    *(int *)D.h_face_err.p = 0;
    HIP_TRY(hipMemcpyAsync(D.h_face_err.p, D.d_face_err, sizeof(int), hipMemcpyDeviceToHost, st));
    // per-level pointer tables (filled per call)
    size_t ne = m.ent.size();
    D.h_phi.assign(ne, nullptr);
    D.h_rho.assign(ne, nullptr);
    D.h_rout.assign(ne, nullptr);
    D.h_E.assign(3 * ne, nullptr);
    HIP_TRY(D.ptrbuf.ensure(sizeof(double *) * 6 * ne));
    HIP_TRY(D.ptrstage.ensure(sizeof(double *) * 6 * ne));
    D.d_phi = (double **)D.ptrbuf.p;
    D.d_rho = D.d_phi + ne;
    D.d_rout = D.d_rho + ne;
    D.d_E = D.d_rout + ne;
    HIP_TRY(D.h_normbuf.ensure(sizeof(double) * 2 * (D.range_prob.size() + 1)));
    D.h_norm = (double *)D.h_normbuf.p;
    HIP_TRY(D.pubbuf.ensure(sizeof(double) * (2 * D.range_prob.size() + 8)));
    D.h_seq = (unsigned *)D.pubbuf.p;
    D.h_pub = (double *)D.pubbuf.p + 1;
    D.ws_prec = -1;  // carve the workspace again for the new hierarchy
    D.drop_graph();
    ++D.meta_gen;
    return AMRMG_OK;
}

static size_t ws_need(const DevState &D, int prec)
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

static amrmg_status ensure_ws(DevState &D, int prec, void *user, size_t user_bytes)
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
    double tot_ms[AMRMG_K_NCLASS] = {}, tot_bytes[AMRMG_K_NCLASS] = {};
    int64_t tot_n[AMRMG_K_NCLASS] = {};
    // per-launch (ms, bytes) of each class, the first kMaxKept launches
    static constexpr size_t kMaxKept = 65536;
    std::vector<std::pair<double, double>> kept[AMRMG_K_NCLASS];
    size_t pending = (size_t)-1;
    int pending_cls = -1;

    bool on(int cls) const { return (mask >> cls) & 1; }
    void begin(int cls)
    {
        pending = (size_t)-1;
        if (!on(cls)) return;
        if (used + 2 > pool.size()) flush();
        if (used + 2 > pool.size()) return;
        pending = used;
        pending_cls = cls;
        set_launch_timing(pool[used], pool[used + 1]);
        used += 2;
    }
    void end(int cls, double bytes)
    {
        if (pending == (size_t)-1 || pending_cls != cls) return;
        if (launch_timing_pending()) {  // the launcher launched nothing
            set_launch_timing(nullptr, nullptr);
            used -= 2;
        } else {
            recs.push_back({cls, pending, bytes});
        }
        pending = (size_t)-1;
    }
    // fold the recorded launches into the totals (waits for them)
    void flush()
    {
        for (const auto &r : recs) {
            float e = 0.f;
            if (hipEventSynchronize(pool[r.ev + 1]) == hipSuccess &&
                hipEventElapsedTime(&e, pool[r.ev], pool[r.ev + 1]) == hipSuccess) {
                tot_ms[r.cls] += e;
                tot_bytes[r.cls] += r.bytes;
                tot_n[r.cls] += 1;
                if (kept[r.cls].size() < kMaxKept) kept[r.cls].emplace_back((double)e, r.bytes);
            }
        }
        recs.clear();
        used = 0;
    }
    void reset(uint32_t m)
    {
        mask = m;
        used = 0;
        recs.clear();
        for (int c = 0; c < AMRMG_K_NCLASS; ++c) tot_ms[c] = tot_bytes[c] = 0.0, tot_n[c] = 0, kept[c].clear();
        if (m && pool.empty()) {
            pool.resize(1 << 12);
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
    // scratch of the tagging passes of build_hierarchy
    DBuf tag_marks, tag_scratch, tag_geom, tag_fields;
    PBuf tag_stage, tag_host;
    // spatial visiting order of the particles (a performance hint for the
    // deposit; any order gives the same sums up to rounding)
    DBuf sort_keys, sort_vals, sort_cnt, sort_tmp;
    DBuf sorted;  // the particles of the last build in visiting order (charges, x, y, z)
    uint32_t *perm = nullptr;
    int64_t perm_n = -1;
    DBuf dep_count;
    // what the last build keeps for amrmg_deposit_built: the charge of each
    // level it deposited for tagging (caller's layout), the particle count
    // and position type of the ordered copy, and its count of particles
    // outside the domain (device, valid when level 0 was deposited)
    std::vector<DBuf> lev_rho;
    std::vector<char> lev_rho_ok;
    int64_t built_n = -1;
    int built_pos = -1;
    DBuf built_nout;
    void *user_ws = nullptr;
    size_t user_ws_bytes = 0;
    int generation = 0;
    // batch cache (kept by the first context of a batch)
    std::vector<amrmg_ctx *> batch_ctx;
    std::vector<int> batch_gen;
    DevState *batch = nullptr;
    Prof prof;
    ~amrmg_ctx() { delete batch; }
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
    *out = c;
    return AMRMG_OK;
}

extern "C" void amrmg_destroy(amrmg_ctx *ctx) { delete ctx; }

// the deposit's larger LDS tile on levels where a visiting-order bucket spans
// 8 or more cells per axis
static bool big_tile(const amrmg_ctx *ctx, int level)
{
    return order_bucket_shift(ctx->P.lo, ctx->P.hi, ctx->P.n0) + level >= 3;
}

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

// Visiting order of the particles (Morton-ordered buckets of the level-0
// grid); with copy, also room for the particles in that order in
// ctx->sorted (charges first, then x, y, z), returned through xs, ys, zs,
// qs: the caller writes the copy (the first tagging deposit does, while it
// reads the particles anyway, or launch_copy_ordered)
static amrmg_status compute_order(amrmg_ctx *ctx, int pos_dtype, const void *x, const void *y, const void *z,
                                  const double *q, int64_t n, bool copy, const void **xs, const void **ys,
                                  const void **zs, const double **qs)
{
    ctx->perm = nullptr;
    ctx->perm_n = -1;
    if (n <= 0 || n > (int64_t)0x7fffffff) return AMRMG_OK;
    const amrmg_params &P = ctx->P;
    const size_t entries = order_count_entries(P.lo, P.hi, P.n0);
    HIP_TRY(ctx->sort_keys.ensure(sizeof(uint32_t) * 2 * (size_t)n));
    HIP_TRY(ctx->sort_vals.ensure(sizeof(uint32_t) * (size_t)n));
    HIP_TRY(ctx->sort_cnt.ensure(sizeof(uint32_t) * 3 * entries));
    HIP_TRY(ctx->sort_tmp.ensure(order_temp_bytes(entries) + 256));
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
    uint32_t *key = (uint32_t *)ctx->sort_keys.p, *cnt = (uint32_t *)ctx->sort_cnt.p;
    HIP_TRY(particle_order(ctx->st, pos_dtype == AMRMG_POS_F32, n, x, y, z, q, P.lo, P.hi, P.n0, key, key + n, cnt,
                           cnt + 2 * entries, (uint32_t *)ctx->sort_vals.p, ctx->sort_tmp.p, ctx->sort_tmp.cap, nullptr,
                           nullptr, nullptr, nullptr));
    ctx->perm = (uint32_t *)ctx->sort_vals.p;
    ctx->perm_n = n;
    if (copy) {
        *xs = cx;
        *ys = cy;
        *zs = cz;
        *qs = cq;
    }
    return AMRMG_OK;
}

// Geometry of the tagging passes on level L: per brick its origin, its
// caller's-layout base and strides, and the level's brick map, uploaded to
// the device; the block marks of level l+1 cleared.
struct TagGeom {
    int32_t *borg = nullptr, *us = nullptr, *bmap = nullptr;
    int64_t *ub = nullptr;
    int nb = 0;
    int64_t nc = 0;
    int3 nn{}, g{};
    size_t ng = 0;
};

static amrmg_status tag_geometry(amrmg_ctx *ctx, const HostLevel &L, TagGeom &G)
{
    const amrmg_params &P = ctx->P;
    hipStream_t st = ctx->st;
    int nb = L.nbrick();
    static thread_local std::vector<int32_t> borg;
    static thread_local std::vector<int64_t> ub;
    static thread_local std::vector<int32_t> us;
    borg.resize(4 * (size_t)nb);
    ub.resize(nb);
    us.resize(2 * (size_t)nb);
    for (int b = 0; b < nb; ++b) {
        const Box &B = L.boxes[L.bbox[b]];
        int64_t nx = B.hi[0] - B.lo[0], ny = B.hi[1] - B.lo[1];
        for (int d = 0; d < 3; ++d) borg[4 * b + d] = 8 * L.bpos[3 * b + d];
        borg[4 * b + 3] = 0;
        ub[b] = L.off[L.bbox[b]] + (8 * L.bpos[3 * b] - B.lo[0]) +
                nx * ((8 * L.bpos[3 * b + 1] - B.lo[1]) + ny * (int64_t)(8 * L.bpos[3 * b + 2] - B.lo[2]));
        us[2 * b] = (int32_t)nx;
        us[2 * b + 1] = (int32_t)(nx * ny);
    }
    Packer pk;
    pk.add(borg, &G.borg);
    pk.add(ub, &G.ub);
    pk.add(us, &G.us);
    pk.add(L.bmap, &G.bmap);
    ST_TRY(pk.run(ctx->tag_geom, ctx->tag_stage, st));
    G.nb = nb;
    G.nc = L.ncells();
    G.nn = make_int3(L.n[0], L.n[1], L.n[2]);
    G.g = make_int3(2 * L.n[0] / P.blocking_factor, 2 * L.n[1] / P.blocking_factor, 2 * L.n[2] / P.blocking_factor);
    G.ng = (size_t)G.g.x * G.g.y * G.g.z;
    HIP_TRY(ctx->tag_scratch.ensure(sizeof(double) * 1040));
    HIP_TRY(ctx->tag_marks.ensure(G.ng));
    HIP_TRY(ctx->tag_host.ensure(G.ng));
    HIP_TRY(hipMemsetAsync(ctx->tag_marks.p, 0, G.ng, st));
    return AMRMG_OK;
}

// mark the blocks of level l+1 reached by the (dilated) cells of level L
// with |v| > lambda * max |v|; the marks of several arrays accumulate
static void tag_mark(amrmg_ctx *ctx, const TagGeom &G, const double *v, double lambda)
{
    launch_mark_blocks(ctx->st, v, G.nc, (const int4 *)G.borg, G.ub, (const int2 *)G.us, G.nb, lambda, ctx->P.n_buffer,
                       ctx->P.blocking_factor / 2, G.nn, G.g, (double *)ctx->tag_scratch.p,
                       (uint8_t *)ctx->tag_marks.p);
}

// the marks to the host, then proper nesting and the greedy merge
static amrmg_status tag_boxes(amrmg_ctx *ctx, const HostLevel &L, const TagGeom &G, std::vector<Box> &boxes)
{
    const amrmg_params &P = ctx->P;
    HIP_TRY(hipMemcpyAsync(ctx->tag_host.p, ctx->tag_marks.p, G.ng, hipMemcpyDeviceToHost, ctx->st));
    HIP_TRY(hipStreamSynchronize(ctx->st));
    HIP_TRY(hipGetLastError());
    boxes = merge_blocks(L, (uint8_t *)ctx->tag_host.p, P.n_proper, P.blocking_factor, P.max_grid_size);
    return AMRMG_OK;
}

// Charge tagging of level l (Sec. 4.2, Eq. tag_charge in relative form):
// deposit level l alone, tag, dilate and mark the blocks of level l+1 on the
// device; the host then applies nesting and the greedy merge.
static amrmg_status tag_level(amrmg_ctx *ctx, const HostLevel &L, int pos_dtype, const void *x, const void *y,
                              const void *z, const double *q, int64_t n, double lambda, std::vector<Box> &boxes,
                              const uint32_t *perm, unsigned long long *nout, void *cx = nullptr,
                              void *cy = nullptr, void *cz = nullptr, double *cq = nullptr)
{
    hipStream_t st = ctx->st;
    TagGeom G;
    ST_TRY(tag_geometry(ctx, L, G));
    // the level's charge is kept for amrmg_deposit_built
    HIP_TRY(ctx->lev_rho[L.amr].ensure(sizeof(double) * G.nc));
    double *rho = (double *)ctx->lev_rho[L.amr].p;
    launch_fill(st, rho, G.nc, 0.0);
    Problem &pr = ctx->prob;
    DepArgs A{};
    A.nlev = 1;
    A.lev[0] = dep_level(pr, L, G.bmap);
    A.rho[0] = rho;
    A.ncell[0] = G.nc;
    launch_deposit(st, pos_dtype == AMRMG_POS_F32, n, x, y, z, q, perm, A, G.ub, (const int2 *)G.us, nout, cx, cy,
                   cz, cq, big_tile(ctx, L.amr));
    tag_mark(ctx, G, rho, lambda);
    return tag_boxes(ctx, L, G, boxes);
}

// Potential or field tagging of level l (Sec. 4.2, the relative criteria on
// phi and on each component E_w): the hierarchy built so far (levels 0..l)
// is finished, every particle deposited on it and the composite problem
// solved to a relative residual of AMRMG_TAG_SOLVE_TOL; a cell of level l is
// tagged when |phi| > lambda max|phi| over the level, or (field) when
// |E_w| > lambda max|E_w| for some component w.  The levels below level 0
// are removed again afterwards.
static amrmg_status tag_level_field(amrmg_ctx *ctx, int l, int pos_dtype, const void *x, const void *y,
                                    const void *z, const double *q, int64_t n, double lambda,
                                    std::vector<Box> &boxes)
{
    const amrmg_params &P = ctx->P;
    hipStream_t st = ctx->st;
    Problem &pr = ctx->prob;
    add_levels_below(pr);
    auto restore = [&]() {
        pr.lev.erase(pr.lev.begin(), pr.lev.begin() + pr.kg);
        pr.kg = 0;
        pr.lev.reserve(P.max_level + 16);
        ctx->built = false;
    };
    amrmg_status rc = upload_meta(ctx->ds, st, {&pr}, P.bottom == AMRMG_BOTTOM_AUTO);
    if (rc == AMRMG_OK && hipStreamSynchronize(st) != hipSuccess) rc = fail(AMRMG_E_HIP, "hipStreamSynchronize failed");
    if (rc == AMRMG_OK && !ctx->ds.meta.error.empty()) rc = fail(AMRMG_E_NESTING, ctx->ds.meta.error);
    if (rc == AMRMG_OK && *(int *)ctx->ds.h_face_err.p)
        rc = fail(AMRMG_E_NESTING, "coarse-fine window leaves the coarser level (nesting violated)");
    if (rc != AMRMG_OK) {
        restore();
        return rc;
    }
    ctx->built = true;
    const bool field = P.tag_policy == AMRMG_TAG_EFIELD;
    const int nv = field ? 5 : 2;  // rho, phi (, E)
    int64_t total = 0;
    for (int k = 0; k <= l; ++k) total += pr.lev[pr.kg + k].ncells();
    std::vector<double *> rho(l + 1), phi(l + 1), E(3 * (l + 1));
    if (ctx->tag_fields.ensure(sizeof(double) * (size_t)(nv * total + 1)) != hipSuccess) {
        restore();
        return fail(AMRMG_E_OOM, "tagging fields");
    }
    double *cur = (double *)ctx->tag_fields.p;
    for (int k = 0; k <= l; ++k) {
        const int64_t nc = pr.lev[pr.kg + k].ncells();
        rho[k] = cur;
        phi[k] = cur + nc;
        cur += 2 * nc;
        if (field)
            for (int d = 0; d < 3; ++d, cur += nc) E[3 * k + d] = cur;
    }
    launch_fill(st, (double *)ctx->tag_fields.p, nv * total, 0.0);
    rc = amrmg_deposit(ctx, pos_dtype, x, y, z, q, n, rho.data(), nullptr);
    if (rc == AMRMG_OK)
        rc = amrmg_solve(ctx, rho.data(), phi.data(), field ? E.data() : nullptr, AMRMG_TAG_SOLVE_TOL, nullptr);
    if (rc == AMRMG_E_NOT_CONVERGED)
        rc = fail(AMRMG_E_NOT_CONVERGED, "the solve for tagging level " + std::to_string(l) + " did not converge");
    TagGeom G;
    if (rc == AMRMG_OK) rc = tag_geometry(ctx, pr.lev[pr.kg + l], G);
    if (rc == AMRMG_OK) {
        if (field)
            for (int d = 0; d < 3; ++d) tag_mark(ctx, G, E[3 * l + d], lambda);
        else
            tag_mark(ctx, G, phi[l], lambda);
        rc = tag_boxes(ctx, pr.lev[pr.kg + l], G, boxes);
    }
    restore();
    return rc;
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
    ++ctx->generation;
    // the tagging passes (and amrmg_deposit_built) read the particles in
    // visiting order from a copy made with the order
    const void *tx = x, *ty = y, *tz = z;
    const double *tq = q;
    ctx->built_n = -1;
    ctx->lev_rho.resize(P.max_level + 1);
    ctx->lev_rho_ok.assign(P.max_level + 1, 0);
    ST_TRY(compute_order(ctx, pos_dtype, x, y, z, q, n, true, &tx, &ty, &tz, &tq));
    const bool copied = ctx->perm_n == n && n > 0;
    // the ordered copy: written by the first charge-tagging deposit of level
    // 0, else by a copy before the first pass that reads it
    bool copy_done = !copied;
    auto ensure_copy = [&]() {
        if (copy_done) return;
        launch_copy_ordered(ctx->st, pos_dtype == AMRMG_POS_F32, n, ctx->perm, x, y, z, q, (void *)tx, (void *)ty,
                            (void *)tz, (double *)tq);
        copy_done = true;
    };
    HIP_TRY(ctx->built_nout.ensure(sizeof(unsigned long long)));
    HIP_TRY(hipMemsetAsync(ctx->built_nout.p, 0, sizeof(unsigned long long), ctx->st));
    const uint32_t *tperm = nullptr;

    Problem &pr = ctx->prob;
    // the previous build's AMR levels lend their storage to the new ones
    // (same level number), so that a regrid touches no fresh pages
    std::vector<HostLevel> pool(P.max_level + 1);
    for (auto &L : pr.lev)
        if (L.amr >= 0 && L.amr <= P.max_level) pool[L.amr] = std::move(L);
    pr.lev.clear();
    pr.lev.reserve(P.max_level + 16);  // references into it stay valid while levels are added
    pr.kg = 0;
    for (int d = 0; d < 3; ++d) {
        pr.lo[d] = P.lo[d];
        pr.hi[d] = P.hi[d];
    }
    pr.eps0 = P.eps0;
    pr.robin = P.robin_d;
    pr.mono = ctx->mono;
    {
        HostLevel L0 = std::move(pool[0]);
        level_init(L0, P.n0, P.lo, P.hi);
        L0.amr = 0;
        Box B{{0, 0, 0}, {P.n0[0], P.n0[1], P.n0[2]}};
        level_set_boxes(L0, {B});
        pr.lev.push_back(std::move(L0));
    }
    for (int l = 0; l < P.max_level; ++l) {
        std::vector<Box> boxes;
        if (expl.count(l + 1)) {
            boxes = expl[l + 1];
        } else {
            if (!tag_rel) return fail(AMRMG_E_INVALID, "tag_rel is NULL but a level needs tagging");
            if (P.tag_policy == AMRMG_TAG_CHARGE) {
                if (!copy_done && l == 0) {
                    // read through the order, write the ordered copy on the way
                    ST_TRY(tag_level(ctx, pr.lev[l], pos_dtype, x, y, z, q, n, tag_rel[l], boxes, ctx->perm,
                                     (unsigned long long *)ctx->built_nout.p, (void *)tx, (void *)ty, (void *)tz,
                                     (double *)tq));
                    copy_done = true;
                } else {
                    ensure_copy();
                    ST_TRY(tag_level(ctx, pr.lev[l], pos_dtype, tx, ty, tz, tq, n, tag_rel[l], boxes, tperm,
                                     l == 0 ? (unsigned long long *)ctx->built_nout.p : nullptr));
                }
                ctx->lev_rho_ok[l] = 1;
            } else {
                // moves the levels (the reference below is taken afterwards)
                ST_TRY(tag_level_field(ctx, l, pos_dtype, x, y, z, q, n, tag_rel[l], boxes));
            }
        }
        const HostLevel &L = pr.lev[l];
        if (boxes.empty()) break;
        if (expl.count(l + 1)) {  // generated boxes are aligned, disjoint and nested by construction
            std::string msg = check_nesting(L, boxes, P.n_proper);
            if (!msg.empty()) return fail(AMRMG_E_NESTING, "level " + std::to_string(l + 1) + ": " + msg);
        }
        HostLevel F = std::move(pool[l + 1]);
        int nf[3] = {2 * L.n[0], 2 * L.n[1], 2 * L.n[2]};
        level_init(F, nf, P.lo, P.hi);
        F.amr = l + 1;
        level_set_boxes(F, boxes);
        pr.lev.push_back(std::move(F));
    }
    ensure_copy();
    add_levels_below(pr);
    ST_TRY(upload_meta(ctx->ds, ctx->st, {&pr}, P.bottom == AMRMG_BOTTOM_AUTO));
    HIP_TRY(hipStreamSynchronize(ctx->st));
    if (!ctx->ds.meta.error.empty()) return fail(AMRMG_E_NESTING, ctx->ds.meta.error);
    if (*(int *)ctx->ds.h_face_err.p)
        return fail(AMRMG_E_NESTING, "coarse-fine window leaves the coarser level (nesting violated)");
    ctx->built = true;
    if (copied || n == 0) {
        ctx->built_n = n;
        ctx->built_pos = pos_dtype;
    }
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
    // the level's faces (owners, their origins, patterns) from the device tables
    std::vector<uint8_t> pat((size_t)e.ncf * 16);
    std::vector<int32_t> owner(e.ncf);
    std::vector<int4> org((size_t)e.nb);
    HIP_TRY(hipStreamSynchronize(ctx->st));
    if (e.ncf > 0) {
        HIP_TRY(hipMemcpy(pat.data(), ctx->ds.M.cf_pat + (size_t)e.cf0 * 16, pat.size(), hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(owner.data(), ctx->ds.M.gf_owner + m.nbc + e.cf0, sizeof(int32_t) * e.ncf,
                          hipMemcpyDeviceToHost));
    }
    if (e.nb > 0)
        HIP_TRY(hipMemcpy(org.data(), ctx->ds.M.org + e.b0, sizeof(int4) * e.nb, hipMemcpyDeviceToHost));
    int64_t k = 0;
    for (int c = e.cf0; c < e.cf0 + e.ncf; ++c) {
        int32_t ow = owner[c - e.cf0];
        int g = ow >> 3, dir = ow & 7, d = dir >> 1, s = (dir & 1) ? 1 : -1;
        int du = (d == 0) ? 1 : 0, dv = (d == 2) ? 1 : 2;
        for (int t = 0; t < 64; ++t, ++k) {
            if (!out || k >= cap) continue;
            int l[3];
            l[d] = s > 0 ? 7 : 0;
            l[du] = t & 7;
            l[dv] = t >> 3;
            int32_t *o = out + 6 * k;
            const int4 og = org[g - e.b0];
            const int O[3] = {og.x, og.y, og.z};
            for (int a = 0; a < 3; ++a) o[a] = O[a] + l[a];
            o[3] = d;
            o[4] = s;
            int mm = ((t & 7) >> 1) + 4 * ((t >> 3) >> 1);
            o[5] = pat[(size_t)(c - e.cf0) * 16 + mm];
        }
    }
    if (count) *count = k;
    return AMRMG_OK;
}

extern "C" amrmg_status amrmg_brick_tables(const amrmg_ctx *ctx, int64_t *counts, int32_t *org, int32_t *nbr,
                                           int32_t *child, int32_t *parent, uint8_t *cmask, int64_t *ubase,
                                           int32_t *ustr, int32_t *owner, int32_t *update)
{
    if (!ctx || !counts) return fail(AMRMG_E_INVALID, "NULL argument");
    if (!ctx->built) return fail(AMRMG_E_STATE, "hierarchy not built");
    const DevState &D = ctx->ds;
    const Meta &m = D.meta;
    const size_t nb = (size_t)m.nbrick;
    counts[0] = m.nbrick;
    counts[1] = m.nbc;
    counts[2] = m.ncf;
    counts[3] = D.n_reflux;
    HIP_TRY(hipStreamSynchronize(ctx->st));
    auto get = [&](void *dst, const void *src, size_t bytes) -> amrmg_status {
        if (dst && bytes) HIP_TRY(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost));
        return AMRMG_OK;
    };
    ST_TRY(get(org, D.M.org, 16 * nb));
    ST_TRY(get(nbr, D.M.nbr, 24 * nb));
    ST_TRY(get(child, D.M.child, 32 * nb));
    ST_TRY(get(parent, D.M.par, 4 * nb));
    ST_TRY(get(cmask, D.M.cmask, nb));
    ST_TRY(get(ubase, D.M.ubase, 8 * nb));
    ST_TRY(get(ustr, D.M.ustr, 8 * nb));
    ST_TRY(get(owner, D.M.gf_owner, 4 * (size_t)(m.nbc + m.ncf)));
    ST_TRY(get(update, D.d_reflux, 4 * (size_t)D.n_reflux));
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

extern "C" amrmg_status amrmg_gather(amrmg_ctx *ctx, int pos_dtype, const void *x, const void *y, const void *z,
                                     int64_t n, double *const *E, double *Ex, double *Ey, double *Ez)
{
    if (!ctx) return fail(AMRMG_E_INVALID, "ctx is NULL");
    if (!ctx->built) return fail(AMRMG_E_STATE, "hierarchy not built");
    if (pos_dtype != AMRMG_POS_F64 && pos_dtype != AMRMG_POS_F32) return fail(AMRMG_E_INVALID, "bad pos_dtype");
    if (!E || n < 0 || (n > 0 && (!x || !y || !z || !Ex || !Ey || !Ez))) return fail(AMRMG_E_INVALID, "bad arguments");
    GatherArgs G;
    ST_TRY(gather_args(ctx, E, G));
    ctx->prof.begin(AMRMG_K_GATHER);
    launch_gather(ctx->st, pos_dtype == AMRMG_POS_F32, n, x, y, z, ctx->perm_n == n ? ctx->perm : nullptr, G,
                  ctx->ds.M.ubase, ctx->ds.M.ustr, Ex, Ey, Ez);
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
    ctx->prof.begin(AMRMG_K_GATHER);
    launch_gather(ctx->st, pos == AMRMG_POS_F32, n, xs, ys, zs, ctx->perm, G, ctx->ds.M.ubase, ctx->ds.M.ustr, Ex, Ey,
                  Ez, true);
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

// ---------------------------------------------------------------------------
// the solve
// ---------------------------------------------------------------------------
// replay the outer iteration as a hipGraph (AMRMG_NO_GRAPH=1 disables)
static bool g_use_graphs = getenv("AMRMG_NO_GRAPH") == nullptr;

struct SolveOpts {
    int precision, smoother, nu1, nu2, norm_p, max_iters;
    double omega, bottom_rtol, inv_eps0;
};

// Threads per brick of the sweep kernel, tuned on the device: for each
// launch size class (bricks per launch, rounded up to a power of two) and
// cycle precision the first solve that meets it times a plain sweep with
// 128 and with 256 threads per brick and keeps the faster; later solves and
// captured graphs read the choice.  Process-wide (one GPU per process);
// AMRMG_NO_TUNE=1 keeps the size rule instead.
static std::mutex g_tune_mu;
static std::map<std::pair<int, int>, int> g_hgs_nt;  // (sizeof(T), log2 bricks) -> threads
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

    // time the sweep of every level with each block size not yet tuned for
    // its size class (plain sweeps from e into et: both are scratch before
    // the cycle starts)
    amrmg_status tune()
    {
        if (!g_tune) return AMRMG_OK;
        for (int k = D.kc + 1; k < m.K; ++k) {
            const int b0 = step_b0(k), nb = step_nb(k);
            if (nb <= 0 || tuned_nt((int)sizeof(T), nb)) continue;
            hipEvent_t a, z;
            HIP_TRY(hipEventCreate(&a));
            HIP_TRY(hipEventCreate(&z));
            constexpr int REPS = 5;
            float each[2] = {0.f, 0.f};
            const int cand[2] = {128, 256};
            for (int i = 0; i < 2; ++i) {
                launch_hgs<T>(st, D.M, b0, nb, e, et, r, cpe, D.phib, D.ffs, 0, cand[i]);  // warm
                HIP_TRY(hipEventRecord(a, st));
                for (int rep = 0; rep < REPS; ++rep)
                    launch_hgs<T>(st, D.M, b0, nb, e, et, r, cpe, D.phib, D.ffs, 0, cand[i]);
                HIP_TRY(hipEventRecord(z, st));
                HIP_TRY(hipEventSynchronize(z));
                HIP_TRY(hipEventElapsedTime(&each[i], a, z));
            }
            // the size rule's choice unless the other is clearly faster
            const int rule = hgs_rule_threads(nb) == cand[1] ? 1 : 0, other = 1 - rule;
            const int pick = each[other] < 0.97f * each[rule] ? cand[other] : cand[rule];
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(z);
            HIP_TRY(hipGetLastError());
            if (getenv("AMRMG_TUNE_LOG"))
                fprintf(stderr, "libamrmg: sweep of %d bricks (%d-byte cycle): 128 threads %.4f ms, 256 threads %.4f ms -> %d\n",
                        nb, (int)sizeof(T), each[0] / REPS, each[1] / REPS, pick);
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_hgs_nt.emplace(std::make_pair((int)sizeof(T), size_class(nb)), pick);
        }
        return AMRMG_OK;
    }

    // outer FP64 residual of every AMR level; norms into dnorm[off ..] (and
    // published to the host at h_pub[pub_off ..] when publish is set)
    void outer(bool zero_phi, int noff, double *const *rout_user, bool publish = false, int pub_off = 0)
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
                           publish ? D.h_pub + pub_off : nullptr, D.h_seq, D.d_seqc);
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
    void iteration(int nr)
    {
        vcycle();
        outer(false, nr, nullptr, true);
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
    // the iteration's graph is captured and instantiated first, while the
    // stream may still be busy with the caller's earlier work (the deposit)
    if (o.smoother == AMRMG_GSRB) ST_TRY(drv.tune());
    if (g_use_graphs && !prof && o.max_iters > 0) ST_TRY(ensure_graph<T>(D, nr, o));
    HIP_TRY(hipMemsetAsync(D.cgit, 0, 64, st));  // CG iteration count and the norm sequence counter
    D.seq = 0;
    *(volatile unsigned *)D.h_seq = 0;
    HIP_TRY(hipEventRecord(ev0, st));
    // norms of b (zero phi) to h_pub[nr ..], of the initial residual to
    // h_pub[0 ..]; each publication bumps the sequence number
    drv.to_bricks(true);
    drv.outer(true, 0, nullptr, true, nr);
    drv.outer(false, nr, nullptr, true, 0);
    HIP_TRY(hipGetLastError());
    // the first iteration is queued before the initial norms are read; when
    // the initial guess already meets the tolerance it only refines phi, and
    // the norms reported are those after it
    const bool first_queued = o.max_iters > 0;
    if (first_queued) ST_TRY(iterate<T>(D, drv, st, nr, o, g_use_graphs));
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
    int it = 0;
    bool all = check(0);
    if (first_queued) {
        ST_TRY(wait_pub(++D.seq));
        rn.assign(D.h_pub, D.h_pub + nr);
        it = 1;
        if (!all) all = check(1);
    }
    while (!all && it < o.max_iters) {
        ST_TRY(iterate<T>(D, drv, st, nr, o, g_use_graphs));
        ST_TRY(wait_pub(++D.seq));
        rn.assign(D.h_pub, D.h_pub + nr);
        ++it;
        all = check(it);
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
    double **h = (double **)D.ptrstage.p;
    std::memcpy(h, D.h_phi.data(), sizeof(double *) * ne);
    std::memcpy(h + ne, D.h_rho.data(), sizeof(double *) * ne);
    std::memcpy(h + 2 * ne, D.h_rout.data(), sizeof(double *) * ne);
    std::memcpy(h + 3 * ne, D.h_E.data(), sizeof(double *) * 3 * ne);
    HIP_TRY(hipMemcpyAsync(D.ptrbuf.p, h, sizeof(double *) * 6 * ne, hipMemcpyHostToDevice, st));
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
    amrmg_status rc = c0->P.precision == AMRMG_MIXED ? run_solve<float>(D, c0->st, o, tol, sv, false, nullptr)
                                                     : run_solve<double>(D, c0->st, o, tol, sv, false, nullptr);
    if (stats)
        for (int i = 0; i < nb && i < (int)sv.size(); ++i) stats[i] = sv[i];
    if (rc == AMRMG_E_NOT_CONVERGED) g_err = "not every problem converged within max_iters";
    return rc;
}

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
