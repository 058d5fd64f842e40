// Test shim: exposes the product's host hierarchy code (amrmg_hier.cpp) to
// Python on a machine without a GPU.  Links only product code.
#include <cstring>
#include <vector>

#include "amrmg_hier.hpp"

using namespace amrmg;

extern "C" int hs_generate_boxes(const int32_t *n, int nb, const int32_t *boxes, const uint8_t *tags, int nbuf,
                                 int nprop, int bf, int mgs, int32_t *out, int cap)
{
    HostLevel L;
    double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
    int nn[3] = {n[0], n[1], n[2]};
    level_init(L, nn, lo, hi);
    std::vector<Box> bx(nb);
    for (int b = 0; b < nb; ++b)
        for (int d = 0; d < 3; ++d) {
            bx[b].lo[d] = boxes[6 * b + d];
            bx[b].hi[d] = boxes[6 * b + 3 + d];
        }
    level_set_boxes(L, bx);
    std::vector<Box> o = generate_boxes(L, tags, nbuf, nprop, bf, mgs);
    if ((int)o.size() > cap) return -1;
    for (size_t b = 0; b < o.size(); ++b)
        for (int d = 0; d < 3; ++d) {
            out[6 * b + d] = o[b].lo[d];
            out[6 * b + 3 + d] = o[b].hi[d];
        }
    return (int)o.size();
}

// greedy merge of a block mask (bytes, 1 = available, x fastest over g[0] x
// g[1] x g[2] blocks) through the product's bit-array merge; returns the box
// count (boxes in block units: lo, hi) or -1 when out holds too few rows
extern "C" int hs_merge_block_bits(const int32_t *g, const uint8_t *mask, int maxb, int32_t *out, int cap)
{
    const size_t total = (size_t)g[0] * g[1] * g[2];
    std::vector<uint64_t> bits((total + 63) / 64, 0);
    for (size_t t = 0; t < total; ++t)
        if (mask[t]) bits[t >> 6] |= 1ull << (t & 63);
    const int gg[3] = {g[0], g[1], g[2]};
    std::vector<Box> o = merge_block_bits(gg, bits.data(), 1, maxb);
    if ((int)o.size() > cap) return -1;
    for (size_t b = 0; b < o.size(); ++b)
        for (int d = 0; d < 3; ++d) {
            out[6 * b + d] = o[b].lo[d];
            out[6 * b + 3 + d] = o[b].hi[d];
        }
    return (int)o.size();
}

// levels given as box lists; returns rows (i,j,k,d,s,pattern) of the CF ghost
// faces of AMR level `level`
extern "C" long hs_cf_patterns(const int32_t *n0, int nlev, const int32_t *nbox, const int32_t *boxes, int level,
                               int32_t *out, long cap)
{
    Problem P;
    for (int d = 0; d < 3; ++d) {
        P.lo[d] = 0;
        P.hi[d] = 1;
    }
    const int32_t *bp = boxes;
    for (int l = 0; l < nlev; ++l) {
        HostLevel L;
        int n[3] = {n0[0] << l, n0[1] << l, n0[2] << l};
        level_init(L, n, P.lo, P.hi);
        L.amr = l;
        std::vector<Box> bx(nbox[l]);
        for (int b = 0; b < nbox[l]; ++b, bp += 6)
            for (int d = 0; d < 3; ++d) {
                bx[b].lo[d] = bp[d];
                bx[b].hi[d] = bp[3 + d];
            }
        level_set_boxes(L, bx);
        P.lev.push_back(L);
    }
    add_levels_below(P);
    Meta M;
    build_meta({&P}, M);
    const Meta::Entry &e = M.ent[M.prob_ent[0][P.kg + level]];
    long k = 0;
    for (int c = e.cf0; c < e.cf0 + e.ncf; ++c) {
        int ow = M.gf_owner[M.nbc + c];
        int g = ow >> 3, dir = ow & 7, d = dir >> 1, s = (dir & 1) ? 1 : -1;
        int du = (d == 0) ? 1 : 0, dv = (d == 2) ? 1 : 2;
        for (int t = 0; t < 64; ++t, ++k) {
            if (k >= cap) continue;
            int l[3];
            l[d] = s > 0 ? 7 : 0;
            l[du] = t & 7;
            l[dv] = t >> 3;
            for (int a = 0; a < 3; ++a) out[6 * k + a] = M.org[(size_t)g * 4 + a] + l[a];
            out[6 * k + 3] = d;
            out[6 * k + 4] = s;
            out[6 * k + 5] = M.cf_pat[(size_t)c * 16 + ((t & 7) >> 1) + 4 * ((t >> 3) >> 1)];
        }
    }
    return k;
}

// the brick tables of the host reference build_meta for the same box lists
// (counts[4] = bricks, boundary faces, coarse-fine faces, update list length;
// arrays sized as amrmg_brick_tables documents; call with NULL arrays for
// the counts first)
extern "C" void hs_brick_tables(const int32_t *n0, int nlev, const int32_t *nbox, const int32_t *boxes,
                                int64_t *counts, int32_t *org, int32_t *nbr, int32_t *child, int32_t *par,
                                uint8_t *cmask, int64_t *ubase, int32_t *ustr, int32_t *owner, int32_t *update,
                                int32_t *lev_counts)
{
    Problem P;
    for (int d = 0; d < 3; ++d) {
        P.lo[d] = 0;
        P.hi[d] = 1;
    }
    const int32_t *bp = boxes;
    for (int l = 0; l < nlev; ++l) {
        HostLevel L;
        int n[3] = {n0[0] << l, n0[1] << l, n0[2] << l};
        level_init(L, n, P.lo, P.hi);
        L.amr = l;
        std::vector<Box> bx(nbox[l]);
        for (int b = 0; b < nbox[l]; ++b, bp += 6)
            for (int d = 0; d < 3; ++d) {
                bx[b].lo[d] = bp[d];
                bx[b].hi[d] = bp[3 + d];
            }
        level_set_boxes(L, bx);
        P.lev.push_back(L);
    }
    add_levels_below(P);
    Meta M;
    build_meta({&P}, M, false);
    counts[0] = M.nbrick;
    counts[1] = M.nbc;
    counts[2] = M.ncf;
    counts[3] = (int64_t)M.reflux.size();
    if (!org) return;
    std::memcpy(org, M.org.data(), 4 * M.org.size());
    std::memcpy(nbr, M.nbr.data(), 4 * M.nbr.size());
    std::memcpy(child, M.child.data(), 4 * M.child.size());
    std::memcpy(par, M.par.data(), 4 * M.par.size());
    std::memcpy(cmask, M.cmask.data(), M.cmask.size());
    std::memcpy(ubase, M.ubase.data(), 8 * M.ubase.size());
    std::memcpy(ustr, M.ustr.data(), 4 * M.ustr.size());
    std::memcpy(owner, M.gf_owner.data(), 4 * M.gf_owner.size());
    std::memcpy(update, M.reflux.data(), 4 * M.reflux.size());
    // per level (coarsest first): cf0, ncf, rf0, nrf, composite cells (AMR levels, else -1)
    for (size_t e = 0; e < M.ent.size(); ++e) {
        int32_t *o = lev_counts + 5 * e;
        o[0] = M.ent[e].cf0;
        o[1] = M.ent[e].ncf;
        o[2] = M.ent[e].rf0;
        o[3] = M.ent[e].nrf;
        o[4] = M.ent[e].amr >= 0 ? (int32_t)M.dof[0][M.ent[e].amr] : -1;
    }
}

// the weight table and quadratic masks, for checks against the printed table
extern "C" void hs_tables(double *w, uint32_t *qmask)
{
    std::vector<double> W = cf_weight_table();
    std::memcpy(w, W.data(), sizeof(double) * W.size());
    for (int p = 0; p < 9; ++p) qmask[p] = quadratic_mask(p);
}

// the direct-solve tables of an n[0] x n[1] x n[2] grid with spacing h
extern "C" long hs_direct_tables(const int32_t *n, const double *h, const double *abnd, double *out, long cap)
{
    int nn[3] = {n[0], n[1], n[2]};
    const double dir[3] = {-1.0, -1.0, -1.0};
    std::vector<double> t = direct_tables(nn, h, abnd ? abnd : dir);
    if ((long)t.size() > cap) return -1;
    std::memcpy(out, t.data(), sizeof(double) * t.size());
    return (long)t.size();
}
