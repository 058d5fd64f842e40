// amrmg_build.cpp -- the hierarchy build of libamrmg: charge, potential and
// field tagging (Sec. 4.2), box generation, the levels below level 0, the
// upload of the merged metadata and the device build of the brick tables,
// and the read-back entry points (hierarchy info, boxes, coarse-fine faces,
// brick tables).
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
amrmg_status upload_meta(DevState &D, hipStream_t st, const std::vector<const Problem *> &probs,
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
    HIP_TRY(D.pubbuf.ensure(sizeof(double) * (4 * D.range_prob.size() + 8)));
    D.h_seq = (unsigned *)D.pubbuf.p;
    D.h_pub = (double *)D.pubbuf.p + 1;
    D.ws_prec = -1;  // carve the workspace again for the new hierarchy
    D.drop_graph();
    ++D.meta_gen;
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

// proper nesting on the device, the nested marks to the host as bits (one
// per block), then the greedy merge
static amrmg_status tag_boxes(amrmg_ctx *ctx, const HostLevel &L, const TagGeom &G, std::vector<Box> &boxes)
{
    const amrmg_params &P = ctx->P;
    const size_t nw = (G.ng + 63) / 64;
    HIP_TRY(ctx->tag_bits.ensure(8 * nw));
    HIP_TRY(ctx->tag_host.ensure(8 * nw));
    launch_nest_pack(ctx->st, (const uint8_t *)ctx->tag_marks.p, (int64_t)G.ng, G.g, G.bmap,
                     make_int3(L.n[0], L.n[1], L.n[2]), make_int3(L.nbk[0], L.nbk[1], L.nbk[2]),
                     P.blocking_factor / 2, P.n_proper, (uint64_t *)ctx->tag_bits.p);
    HIP_TRY(hipMemcpyAsync(ctx->tag_host.p, ctx->tag_bits.p, 8 * nw, hipMemcpyDeviceToHost, ctx->st));
    HIP_TRY(hipStreamSynchronize(ctx->st));
    HIP_TRY(hipGetLastError());
    const int g[3] = {G.g.x, G.g.y, G.g.z};
    boxes = merge_block_bits(g, (uint64_t *)ctx->tag_host.p, P.blocking_factor, P.max_grid_size);
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
