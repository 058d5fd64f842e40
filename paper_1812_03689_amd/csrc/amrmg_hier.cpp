// amrmg_hier.cpp -- host-side hierarchy construction of libamrmg.
//
// Box generation: the paper leaves box generation to its AMR library (Sec.
// 3, Sec. 4.2).  Here it is a fixed integer procedure on 8-cell blocks of the
// finer level: tag dilation, block marking, proper nesting, greedy merge.
//
// Coarse-fine metadata follows Sec. 5.1 of the paper: for each fine brick face
// on the coarse-fine interface, each of the 16 coarse cells of the coarse
// layer across it gets the 5x5 availability mask of its layer (bit i + 5 j,
// set when the coarse cell exists and is not covered), the first window of
// Tab. bit_pattern that fits (or a bilinear window of the following table, or
// the centre alone), and the coarse cells of that window.
#include "amrmg_hier.hpp"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <iterator>

namespace amrmg {

static const double kPi = 3.14159265358979323846;

int HostLevel::brick_at(int bx, int by, int bz) const
{
    if (bx < 0 || by < 0 || bz < 0 || bx >= nbk[0] || by >= nbk[1] || bz >= nbk[2]) return -1;
    return bmap[(size_t)bx + (size_t)nbk[0] * ((size_t)by + (size_t)nbk[1] * (size_t)bz)];
}

bool HostLevel::has_cell(int i, int j, int k) const
{
    if (i < 0 || j < 0 || k < 0 || i >= n[0] || j >= n[1] || k >= n[2]) return false;
    return brick_at(i >> 3, j >> 3, k >> 3) >= 0;
}

void level_init(HostLevel &L, const int n[3], const double lo[3], const double hi[3])
{
    for (int d = 0; d < 3; ++d) {
        L.n[d] = n[d];
        L.h[d] = (hi[d] - lo[d]) / n[d];
        L.nbk[d] = n[d] / 8;
    }
}

void level_set_boxes(HostLevel &L, const std::vector<Box> &boxes)
{
    L.boxes = boxes;
    L.off.assign(boxes.size() + 1, 0);
    const size_t nmap = (size_t)L.nbk[0] * L.nbk[1] * L.nbk[2];
    if (L.bmap.size() == nmap && L.map_nbk[0] == L.nbk[0] && L.map_nbk[1] == L.nbk[1] && L.map_nbk[2] == L.nbk[2]) {
        // the same brick grid as the previous box list (a regrid): clear only its bricks
        for (size_t k = 0; k + 2 < L.bpos.size(); k += 3)
            L.bmap[(size_t)L.bpos[k] + (size_t)L.nbk[0] * ((size_t)L.bpos[k + 1] + (size_t)L.nbk[1] * L.bpos[k + 2])] = -1;
    } else {
        L.bmap.assign(nmap, -1);
        for (int d = 0; d < 3; ++d) L.map_nbk[d] = L.nbk[d];
    }
    L.bpos.clear();
    L.bbox.clear();
    size_t nbr = 0;
    for (const Box &B : boxes) nbr += (size_t)(B.volume() / 512);
    L.bpos.reserve(3 * nbr);
    L.bbox.reserve(nbr);
    for (size_t b = 0; b < boxes.size(); ++b) {
        const Box &B = boxes[b];
        L.off[b + 1] = L.off[b] + B.volume();
        for (int bz = B.lo[2] / 8; bz < B.hi[2] / 8; ++bz)
            for (int by = B.lo[1] / 8; by < B.hi[1] / 8; ++by)
                for (int bx = B.lo[0] / 8; bx < B.hi[0] / 8; ++bx) {
                    L.bmap[(size_t)bx + (size_t)L.nbk[0] * ((size_t)by + (size_t)L.nbk[1] * bz)] =
                        (int32_t)L.bbox.size();
                    L.bpos.push_back(bx);
                    L.bpos.push_back(by);
                    L.bpos.push_back(bz);
                    L.bbox.push_back((int32_t)b);
                }
    }
}

// every cell of the axis-aligned cell box [lo, hi) belongs to level L
static bool region_inside(const HostLevel &L, const int lo[3], const int hi[3])
{
    for (int bz = lo[2] >> 3; bz <= (hi[2] - 1) >> 3; ++bz)
        for (int by = lo[1] >> 3; by <= (hi[1] - 1) >> 3; ++by)
            for (int bx = lo[0] >> 3; bx <= (hi[0] - 1) >> 3; ++bx)
                if (L.brick_at(bx, by, bz) < 0) return false;
    return true;
}

// coarse footprint of fine block (bx,by,bz), grown by np cells and clipped to
// the coarse index space
static void grown_footprint(const HostLevel &C, const int blk[3], int half, int np, int lo[3], int hi[3])
{
    for (int d = 0; d < 3; ++d) {
        lo[d] = std::max(0, blk[d] * half - np);
        hi[d] = std::min(C.n[d], (blk[d] + 1) * half + np);
    }
}

void mark_blocks(const HostLevel &L, const uint8_t *tags, int n_buffer, int bf, std::vector<uint8_t> &mark)
{
    const int half = bf / 2;  // coarse cells per fine block edge
    int g[3];
    for (int d = 0; d < 3; ++d) g[d] = 2 * L.n[d] / bf;
    auto at = [&](int x, int y, int z) { return (size_t)x + (size_t)g[0] * ((size_t)y + (size_t)g[1] * z); };
    mark.assign((size_t)g[0] * g[1] * g[2], 0);
    for (size_t b = 0; b < L.boxes.size(); ++b) {
        const Box &B = L.boxes[b];
        int64_t t = L.off[b];
        for (int k = B.lo[2]; k < B.hi[2]; ++k)
            for (int j = B.lo[1]; j < B.hi[1]; ++j)
                for (int i = B.lo[0]; i < B.hi[0]; ++i, ++t) {
                    if (!tags[t]) continue;
                    int zlo = std::max(0, k - n_buffer), zhi = std::min(L.n[2] - 1, k + n_buffer);
                    int ylo = std::max(0, j - n_buffer), yhi = std::min(L.n[1] - 1, j + n_buffer);
                    int xlo = std::max(0, i - n_buffer), xhi = std::min(L.n[0] - 1, i + n_buffer);
                    for (int z = zlo / half; z <= zhi / half; ++z)
                        for (int y = ylo / half; y <= yhi / half; ++y)
                            for (int x = xlo / half; x <= xhi / half; ++x) mark[at(x, y, z)] = 1;
                }
    }
}

void nest_blocks(const HostLevel &L, uint8_t *mark, int n_proper, int bf)
{
    const int half = bf / 2;
    int g[3];
    for (int d = 0; d < 3; ++d) g[d] = 2 * L.n[d] / bf;
    const size_t total = (size_t)g[0] * g[1] * g[2];
    // skip eight blocks at a time where a word of marks holds none
    for (size_t t0 = 0; t0 < total; t0 += 8) {
        if (t0 + 8 <= total) {
            uint64_t w;
            std::memcpy(&w, mark + t0, 8);
            if (w == 0) continue;
        }
        for (size_t t = t0; t < std::min(t0 + 8, total); ++t) {
            if (!mark[t]) continue;
            int blk[3] = {(int)(t % g[0]), (int)((t / g[0]) % g[1]), (int)(t / ((size_t)g[0] * g[1]))}, lo[3], hi[3];
            grown_footprint(L, blk, half, n_proper, lo, hi);
            if (!region_inside(L, lo, hi)) mark[t] = 0;
        }
    }
}

// bit t of a block bit array (block t = x + g0 (y + g1 z)): word t / 64, bit t % 64
static bool bits_all_set(const uint64_t *b, size_t t, int e)
{
    while (e > 0) {
        const size_t w = t >> 6;
        const int o = (int)(t & 63), k = std::min(e, 64 - o);
        const uint64_t m = (k == 64 ? ~0ull : ((1ull << k) - 1)) << o;
        if ((b[w] & m) != m) return false;
        t += k;
        e -= k;
    }
    return true;
}

static void bits_clear(uint64_t *b, size_t t, int e)
{
    while (e > 0) {
        const size_t w = t >> 6;
        const int o = (int)(t & 63), k = std::min(e, 64 - o);
        b[w] &= ~((k == 64 ? ~0ull : ((1ull << k) - 1)) << o);
        t += k;
        e -= k;
    }
}

// the number of consecutive set bits from t, at most lim
static int bits_run(const uint64_t *b, size_t t, int lim)
{
    int run = 0;
    while (run < lim) {
        const size_t w = t >> 6;
        const int o = (int)(t & 63), k = std::min(lim - run, 64 - o);
        const uint64_t v = ~(b[w] >> o);  // clear where the bits are set; the o vacated top bits read as clear blocks
        const int ones = std::min(v == 0 ? 64 : __builtin_ctzll(v), k);
        run += ones;
        if (ones < k) break;
        t += k;
    }
    return run;
}

std::vector<Box> merge_block_bits(const int g[3], uint64_t *bits, int bf, int max_grid_size)
{
    const int maxb = max_grid_size / bf;
    const size_t total = (size_t)g[0] * g[1] * g[2], nw = (total + 63) / 64;
    auto at = [&](int x, int y, int z) { return (size_t)x + (size_t)g[0] * ((size_t)y + (size_t)g[1] * z); };
    std::vector<Box> out;
    for (size_t w = 0; w < nw; ++w) {
        // the lowest available block starts a box; a box clears only blocks
        // after it in linear order, so taking the lowest set bit of the word
        // again visits the blocks in the same order as a linear scan
        while (bits[w]) {
            const size_t t = w * 64 + (size_t)__builtin_ctzll(bits[w]);
            const int x = (int)(t % g[0]), y = (int)((t / g[0]) % g[1]), z = (int)(t / ((size_t)g[0] * g[1]));
            const int ex = bits_run(bits, t, std::min(maxb, g[0] - x));
            int ey = 1, ez = 1;
            while (y + ey < g[1] && ey < maxb && bits_all_set(bits, at(x, y + ey, z), ex)) ++ey;
            while (z + ez < g[2] && ez < maxb) {
                bool slab = true;
                for (int c = 0; c < ey && slab; ++c) slab = bits_all_set(bits, at(x, y + c, z + ez), ex);
                if (!slab) break;
                ++ez;
            }
            for (int c3 = 0; c3 < ez; ++c3)
                for (int c2 = 0; c2 < ey; ++c2) bits_clear(bits, at(x, y + c2, z + c3), ex);
            Box B;
            B.lo[0] = x * bf;
            B.lo[1] = y * bf;
            B.lo[2] = z * bf;
            B.hi[0] = (x + ex) * bf;
            B.hi[1] = (y + ey) * bf;
            B.hi[2] = (z + ez) * bf;
            out.push_back(B);
        }
    }
    return out;
}

std::vector<Box> merge_blocks(const HostLevel &L, uint8_t *mark, int n_proper, int bf, int max_grid_size)
{
    nest_blocks(L, mark, n_proper, bf);
    int g[3];
    for (int d = 0; d < 3; ++d) g[d] = 2 * L.n[d] / bf;
    const size_t total = (size_t)g[0] * g[1] * g[2];
    std::vector<uint64_t> bits((total + 63) / 64, 0);
    for (size_t t = 0; t < total; ++t)
        if (mark[t] == 1) bits[t >> 6] |= 1ull << (t & 63);
    return merge_block_bits(g, bits.data(), bf, max_grid_size);
}

std::vector<Box> generate_boxes(const HostLevel &L, const uint8_t *tags, int n_buffer, int n_proper, int bf,
                                int max_grid_size)
{
    std::vector<uint8_t> mark;
    mark_blocks(L, tags, n_buffer, bf, mark);
    return merge_blocks(L, mark.data(), n_proper, bf, max_grid_size);
}

std::string check_nesting(const HostLevel &C, const std::vector<Box> &fine, int n_proper)
{
    char msg[256];
    int nf[3] = {2 * C.n[0], 2 * C.n[1], 2 * C.n[2]};
    int g[3] = {nf[0] / 8, nf[1] / 8, nf[2] / 8};
    std::vector<uint8_t> used((size_t)g[0] * g[1] * g[2], 0);
    for (size_t b = 0; b < fine.size(); ++b) {
        const Box &B = fine[b];
        for (int d = 0; d < 3; ++d) {
            if (B.lo[d] % 8 || B.hi[d] % 8) {
                snprintf(msg, sizeof msg, "box %zu is not aligned to 8 cells", b);
                return msg;
            }
            if (B.lo[d] < 0 || B.hi[d] > nf[d] || B.lo[d] >= B.hi[d]) {
                snprintf(msg, sizeof msg, "box %zu is empty or outside the level", b);
                return msg;
            }
        }
        for (int z = B.lo[2] / 8; z < B.hi[2] / 8; ++z)
            for (int y = B.lo[1] / 8; y < B.hi[1] / 8; ++y)
                for (int x = B.lo[0] / 8; x < B.hi[0] / 8; ++x) {
                    size_t t = (size_t)x + (size_t)g[0] * ((size_t)y + (size_t)g[1] * z);
                    if (used[t]) {
                        snprintf(msg, sizeof msg, "box %zu overlaps an earlier box", b);
                        return msg;
                    }
                    used[t] = 1;
                    int blk[3] = {x, y, z}, lo[3], hi[3];
                    grown_footprint(C, blk, 4, n_proper, lo, hi);
                    if (!region_inside(C, lo, hi)) {
                        snprintf(msg, sizeof msg, "box %zu is not properly nested in the coarser level", b);
                        return msg;
                    }
                }
    }
    return "";
}

// ---------------------------------------------------------------------------
// interpolation patterns
// ---------------------------------------------------------------------------

// window origins (first node offset along u, v from the centre cell) of the
// nine quadratic cases in the order of Tab. bit_pattern: centred, shifted
// towards -v, -u, +v, +u, then the corners (+u,-v), (-u,-v), (-u,+v), (+u,+v)
static const int kQuadWin[9][2] = {{-1, -1}, {-1, -2}, {-2, -1}, {-1, 0}, {0, -1},
                                   {0, -2},  {-2, -2}, {-2, 0},  {0, 0}};
// the four bilinear windows in the printed order: (-u,-v), (-u,+v), (+u,+v), (+u,-v)
static const int kLinWin[4][2] = {{-1, -1}, {-1, 0}, {0, 0}, {0, -1}};

void pattern_window(int pat, int &u0, int &v0, int &np)
{
    if (pat < 9) {
        u0 = kQuadWin[pat][0];
        v0 = kQuadWin[pat][1];
        np = 3;
    } else if (pat < 13) {
        u0 = kLinWin[pat - 9][0];
        v0 = kLinWin[pat - 9][1];
        np = 2;
    } else {
        u0 = 0;
        v0 = 0;
        np = 1;
    }
}

static uint32_t window_mask(int pat)
{
    int u0, v0, np;
    pattern_window(pat, u0, v0, np);
    uint32_t m = 0;
    for (int b = 0; b < np; ++b)
        for (int a = 0; a < np; ++a) m |= 1u << ((u0 + a + 2) + 5 * (v0 + b + 2));
    return m;
}

uint32_t quadratic_mask(int pat) { return window_mask(pat); }

void pattern_tables(uint32_t masks13[13], int org14x3[42])
{
    for (int p = 0; p < 14; ++p) {
        if (p < 13) masks13[p] = window_mask(p);
        pattern_window(p, org14x3[3 * p], org14x3[3 * p + 1], org14x3[3 * p + 2]);
    }
}

int select_pattern(uint32_t mask5)
{
    static const struct Masks {
        uint32_t m[13];
        Masks()
        {
            for (int p = 0; p < 13; ++p) m[p] = window_mask(p);
        }
    } W;
    for (int p = 0; p < 13; ++p)
        if ((mask5 & W.m[p]) == W.m[p]) return p;
    return 13;
}

// Lagrange basis of node a (offset u0 + a) over nodes u0 .. u0+np-1 at t
static double lagrange_basis(int a, int u0, int np, double t)
{
    double v = 1.0;
    for (int m = 0; m < np; ++m)
        if (m != a) v *= (t - (u0 + m)) / (double)(a - m);
    return v;
}

std::vector<double> cf_weight_table()
{
    std::vector<double> W(14 * 4 * 9, 0.0);
    for (int p = 0; p < 14; ++p) {
        int u0, v0, np;
        pattern_window(p, u0, v0, np);
        for (int q = 0; q < 4; ++q) {
            double tu = (q & 1) ? 0.25 : -0.25, tv = (q >> 1) ? 0.25 : -0.25;
            for (int b = 0; b < np; ++b)
                for (int a = 0; a < np; ++a)
                    W[(p * 4 + q) * 9 + a + 3 * b] =
                        (8.0 / 15.0) * lagrange_basis(a, u0, np, tu) * lagrange_basis(b, v0, np, tv);
        }
    }
    return W;
}

// Eigendecomposition of a symmetric matrix (row-major N x N, destroyed) by
// cyclic Jacobi rotations: A = V diag(w) V^T, V column k the k-th
// eigenvector.  Each rotation zeroes A[p][q] with t = tan(angle) the smaller
// root of t^2 + 2 theta t - 1 = 0, theta = (A_qq - A_pp) / (2 A_pq); sweeps
// over all p < q until the off-diagonal part is negligible.
static void jacobi_eigen(std::vector<double> &A, int N, std::vector<double> &V, std::vector<double> &w)
{
    V.assign((size_t)N * N, 0.0);
    for (int i = 0; i < N; ++i) V[(size_t)i * N + i] = 1.0;
    auto at = [&](int i, int j) -> double & { return A[(size_t)i * N + j]; };
    double scale = 0.0;
    for (double v : A) scale += v * v;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < N; ++p)
            for (int q = p + 1; q < N; ++q) off += at(p, q) * at(p, q);
        if (off <= 1e-32 * scale) break;
        for (int p = 0; p < N; ++p)
            for (int q = p + 1; q < N; ++q) {
                const double apq = at(p, q);
                if (apq == 0.0) continue;
                const double theta = (at(q, q) - at(p, p)) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < N; ++k) {  // columns p, q
                    const double akp = at(k, p), akq = at(k, q);
                    at(k, p) = c * akp - s * akq;
                    at(k, q) = s * akp + c * akq;
                }
                for (int k = 0; k < N; ++k) {  // rows p, q
                    const double apk = at(p, k), aqk = at(q, k);
                    at(p, k) = c * apk - s * aqk;
                    at(q, k) = s * apk + c * aqk;
                }
                for (int k = 0; k < N; ++k) {
                    const double vkp = V[(size_t)k * N + p], vkq = V[(size_t)k * N + q];
                    V[(size_t)k * N + p] = c * vkp - s * vkq;
                    V[(size_t)k * N + q] = s * vkp + c * vkq;
                }
            }
    }
    w.resize(N);
    for (int i = 0; i < N; ++i) w[i] = at(i, i);
}

std::vector<double> direct_tables(const int n[3], const double h[3], const double abnd[3])
{
    std::vector<double> t, lam;
    for (int d = 0; d < 3; ++d) {
        const int N = n[d];
        std::vector<double> S((size_t)N * N), w(N);
        if (abnd[d] == -1.0) {
            for (int i = 0; i < N; ++i)
                for (int k = 0; k < N; ++k) {
                    double c = (k == N - 1) ? std::sqrt(1.0 / N) : std::sqrt(2.0 / N);
                    S[(size_t)i * N + k] = c * std::sin(kPi * (k + 1) * (i + 0.5) / N);
                }
            for (int k = 0; k < N; ++k) {
                double s = std::sin(kPi * (k + 1) / (2.0 * N));
                w[k] = 4.0 * s * s;
            }
        } else {
            // 2 on the diagonal, 2 - abnd at both ends, -1 off the diagonal
            std::vector<double> A((size_t)N * N, 0.0);
            for (int i = 0; i < N; ++i) {
                A[(size_t)i * N + i] = 2.0 - ((i == 0) ? abnd[d] : 0.0) - ((i == N - 1) ? abnd[d] : 0.0);
                if (i + 1 < N) A[(size_t)i * N + i + 1] = A[(size_t)(i + 1) * N + i] = -1.0;
            }
            jacobi_eigen(A, N, S, w);
        }
        for (int k = 0; k < N; ++k)
            for (int i = 0; i < N; ++i) t.push_back(S[(size_t)i * N + k]);
        for (int i = 0; i < N; ++i)
            for (int k = 0; k < N; ++k) t.push_back(S[(size_t)i * N + k]);
        for (int k = 0; k < N; ++k) lam.push_back(w[k] / (h[d] * h[d]));
    }
    t.insert(t.end(), lam.begin(), lam.end());
    return t;
}

void boundary_ghost(const Problem &P, const double h[3], double a[3])
{
    for (int d = 0; d < 3; ++d) a[d] = P.robin > 0.0 ? (2.0 * P.robin - h[d]) / (2.0 * P.robin + h[d]) : -1.0;
}

void add_levels_below(Problem &P)
{
    std::vector<HostLevel> below;
    int n[3] = {P.lev[0].n[0], P.lev[0].n[1], P.lev[0].n[2]};
    while (n[0] % 16 == 0 && n[1] % 16 == 0 && n[2] % 16 == 0 && std::max(n[0], std::max(n[1], n[2])) > 64) {
        for (int d = 0; d < 3; ++d) n[d] /= 2;
        HostLevel L;
        level_init(L, n, P.lo, P.hi);
        L.amr = -1;
        Box B{{0, 0, 0}, {n[0], n[1], n[2]}};
        level_set_boxes(L, {B});
        below.insert(below.begin(), L);
    }
    P.kg = (int)below.size();
    below.insert(below.end(), std::make_move_iterator(P.lev.begin()), std::make_move_iterator(P.lev.end()));
    P.lev.swap(below);
}

// ---------------------------------------------------------------------------
// merged metadata
// ---------------------------------------------------------------------------
static double dirichlet_value(const Problem &P, const double x[3])
{
    double g = 0.0;
    for (size_t m = 0; m + 3 < P.mono.size(); m += 4) {
        double dx = x[0] - P.mono[m + 1], dy = x[1] - P.mono[m + 2], dz = x[2] - P.mono[m + 3];
        g += P.mono[m] / (4.0 * kPi * P.eps0 * std::sqrt(dx * dx + dy * dy + dz * dz));
    }
    return g;
}

static inline void tdirs(int d, int &du, int &dv)
{
    du = (d == 0) ? 1 : 0;
    dv = (d == 2) ? 1 : 2;
}

// bricks of a level from its box list alone
static int level_bricks(const HostLevel &L)
{
    int64_t nb = 0;
    for (const Box &B : L.boxes)
        nb += (int64_t)((B.hi[0] - B.lo[0]) / 8) * ((B.hi[1] - B.lo[1]) / 8) * ((B.hi[2] - B.lo[2]) / 8);
    return (int)nb;
}

void meta_entries(const std::vector<const Problem *> &probs, Meta &M)
{
    // start over, keeping the vectors' storage (a regrid reuses it without
    // fresh page faults)
    M.ent.clear();
    M.step_ent0.clear();
    M.K = 0;
    M.nbrick = 0;
    M.nbc = M.ncf = 0;
    M.gf_owner.clear();
    M.gbc.clear();
    M.cf_pat.clear();
    M.cf_idx.clear();
    M.reflux.clear();
    M.amr_bricks.clear();
    M.prob_ent.clear();
    M.dof.clear();
    M.error.clear();
    const int np = (int)probs.size();
    M.K = 0;
    for (auto *p : probs) M.K = std::max(M.K, (int)p->lev.size());
    M.prob_ent.assign(np, std::vector<int>());
    for (int i = 0; i < np; ++i) M.prob_ent[i].assign(probs[i]->lev.size(), -1);
    // entries and brick ranges
    int nb = 0;
    for (int k = 0; k < M.K; ++k) {
        M.step_ent0.push_back((int)M.ent.size());
        for (int i = 0; i < np; ++i) {
            const Problem &P = *probs[i];
            if (k >= (int)P.lev.size()) continue;
            const HostLevel &L = P.lev[k];
            Meta::Entry e{};
            e.prob = i;
            e.k = k;
            e.amr = L.amr;
            e.b0 = nb;
            e.nb = level_bricks(L);
            for (int d = 0; d < 3; ++d) e.h[d] = L.h[d];
            nb += e.nb;
            M.prob_ent[i][k] = (int)M.ent.size();
            M.ent.push_back(e);
        }
    }
    M.step_ent0.push_back((int)M.ent.size());
    M.nbrick = nb;
    M.org.clear();
    M.nbr.clear();
    M.child.clear();
    M.par.clear();
    M.cmask.clear();
    M.ubase.clear();
    M.ustr.clear();
}

void build_meta(const std::vector<const Problem *> &probs, Meta &M, bool face_data)
{
    meta_entries(probs, M);
    const int np = (int)probs.size();
    const int nb = M.nbrick;
    M.org.assign((size_t)nb * 4, 0);
    M.nbr.assign((size_t)nb * 6, 0);
    M.child.assign((size_t)nb * 8, -1);
    M.par.assign(nb, -1);
    M.cmask.assign(nb, 0);
    M.ubase.assign(nb, 0);
    M.ustr.assign((size_t)nb * 2, 0);

    struct Face {
        int brick, dir, ent;
    };
    std::vector<Face> bcf, cff;
    const int CF_TAG = INT_MIN / 2;
    for (size_t ei = 0; ei < M.ent.size(); ++ei) {
        Meta::Entry &e = M.ent[ei];
        const Problem &P = *probs[e.prob];
        const HostLevel &L = P.lev[e.k];
        const HostLevel *Cc = (e.k > 0) ? &P.lev[e.k - 1] : nullptr;
        int ecrse = Cc ? M.prob_ent[e.prob][e.k - 1] : -1;
        e.cf0 = (int)cff.size();
        // bricks are numbered box by box, x fastest inside a box: a face
        // neighbour inside the same box is found without the brick map
        int bcur = -1, bfirst = 0, blo[3] = {0, 0, 0}, bhi[3] = {0, 0, 0};
        for (int lb = 0; lb < L.nbrick(); ++lb) {
            int g = e.b0 + lb;
            int Pb[3] = {L.bpos[3 * lb], L.bpos[3 * lb + 1], L.bpos[3 * lb + 2]};
            if (L.bbox[lb] != bcur) {
                bcur = L.bbox[lb];
                bfirst = lb;
                for (int d = 0; d < 3; ++d) {
                    blo[d] = L.boxes[bcur].lo[d] / 8;
                    bhi[d] = L.boxes[bcur].hi[d] / 8;
                }
            }
            const int ex = bhi[0] - blo[0], ey = bhi[1] - blo[1];
            for (int d = 0; d < 3; ++d) M.org[(size_t)g * 4 + d] = 8 * Pb[d];
            M.org[(size_t)g * 4 + 3] = (int32_t)ei;
            for (int d = 0; d < 3; ++d)
                for (int s = -1; s <= 1; s += 2) {
                    int Q[3] = {Pb[0], Pb[1], Pb[2]};
                    Q[d] += s;
                    int dir = 2 * d + (s > 0);
                    int32_t v;
                    if (Q[d] < 0 || Q[d] >= L.nbk[d]) {
                        v = -1 - (int32_t)bcf.size();
                        bcf.push_back({g, dir, (int)ei});
                    } else {
                        int q;
                        if (Q[d] >= blo[d] && Q[d] < bhi[d])
                            q = bfirst + (Q[0] - blo[0]) + ex * ((Q[1] - blo[1]) + ey * (Q[2] - blo[2]));
                        else
                            q = L.brick_at(Q[0], Q[1], Q[2]);
                        if (q >= 0) {
                            v = e.b0 + q;
                        } else {
                            v = CF_TAG + (int32_t)cff.size();
                            cff.push_back({g, dir, (int)ei});
                        }
                    }
                    M.nbr[(size_t)g * 6 + dir] = v;
                }
            // parent and octant; the parent's child table and covered mask
            // are filled from here (levels are visited coarse to fine)
            if (Cc) {
                int q = Cc->brick_at(Pb[0] >> 1, Pb[1] >> 1, Pb[2] >> 1);
                int oc = (Pb[0] & 1) | ((Pb[1] & 1) << 1) | ((Pb[2] & 1) << 2);
                if (q < 0) {
                    M.error = "a brick has no parent on the coarser level (nesting violated)";
                    q = 0;
                }
                const int pg = M.ent[ecrse].b0 + q;
                M.par[g] = (pg << 3) | oc;
                M.child[(size_t)pg * 8 + oc] = g;
                if (Cc->amr >= 0) M.cmask[pg] |= (uint8_t)(1u << oc);
            }
            if (L.amr >= 0) {
                const Box &B = L.boxes[L.bbox[lb]];
                int64_t nx = B.hi[0] - B.lo[0], ny = B.hi[1] - B.lo[1];
                M.ubase[g] = L.off[L.bbox[lb]] + (8 * Pb[0] - B.lo[0]) +
                             nx * ((8 * Pb[1] - B.lo[1]) + ny * (int64_t)(8 * Pb[2] - B.lo[2]));
                M.ustr[(size_t)g * 2] = (int32_t)nx;
                M.ustr[(size_t)g * 2 + 1] = (int32_t)(nx * ny);
            }
        }
        e.ncf = (int)cff.size() - e.cf0;
    }
    M.nbc = (int)bcf.size();
    M.ncf = (int)cff.size();
    for (auto &v : M.nbr)
        if (v < 0 && v <= CF_TAG + (int32_t)cff.size() && v >= CF_TAG) v = -1 - (M.nbc + (v - CF_TAG));
    M.gf_owner.resize(M.nbc + M.ncf);
    for (int t = 0; t < M.nbc; ++t) M.gf_owner[t] = (bcf[t].brick << 3) | bcf[t].dir;
    for (int t = 0; t < M.ncf; ++t) M.gf_owner[M.nbc + t] = (cff[t].brick << 3) | cff[t].dir;

    // Dirichlet data at the centres of the boundary faces of AMR levels
    M.gbc.assign(face_data ? (size_t)M.nbc * 64 : 0, 0.0);
    for (int t = 0; t < M.nbc && face_data; ++t) {
        const Meta::Entry &e = M.ent[bcf[t].ent];
        const Problem &P = *probs[e.prob];
        if (e.amr < 0 || P.mono.empty()) continue;
        int g = bcf[t].brick, d = bcf[t].dir >> 1, s = (bcf[t].dir & 1) ? 1 : -1;
        int du, dv;
        tdirs(d, du, dv);
        for (int f = 0; f < 64; ++f) {
            int l[3];
            l[d] = s > 0 ? 7 : 0;
            l[du] = f & 7;
            l[dv] = f >> 3;
            double x[3];
            for (int a = 0; a < 3; ++a) x[a] = P.lo[a] + (M.org[(size_t)g * 4 + a] + l[a] + 0.5) * e.h[a];
            x[d] += 0.5 * s * e.h[d];
            M.gbc[(size_t)t * 64 + f] = dirichlet_value(P, x);
        }
    }

    // coarse-fine faces: pattern and window cells per coarse cell
    M.cf_pat.assign(face_data ? (size_t)M.ncf * 16 : 0, 0);
    M.cf_idx.assign(face_data ? (size_t)M.ncf * 16 * 9 : 0, 0);
    for (int t = 0; t < M.ncf && face_data; ++t) {
        const Meta::Entry &e = M.ent[cff[t].ent];
        const Problem &P = *probs[e.prob];
        const HostLevel &Lf = P.lev[e.k];
        const HostLevel &Lc = P.lev[e.k - 1];
        const Meta::Entry &ec = M.ent[M.prob_ent[e.prob][e.k - 1]];
        int g = cff[t].brick, d = cff[t].dir >> 1, s = (cff[t].dir & 1) ? 1 : -1;
        int du, dv;
        tdirs(d, du, dv);
        int O[3] = {M.org[(size_t)g * 4], M.org[(size_t)g * 4 + 1], M.org[(size_t)g * 4 + 2]};
        int ghost_d = s > 0 ? O[d] + 8 : O[d] - 1;
        // the coarse layer cells within 2 of the face's 4x4 coarse cells:
        // their cycle-array index (or -1 when not on the coarser level) and
        // availability (on the coarser level and not covered)
        int32_t gidx[8][8];
        uint8_t av[8][8];
        for (int jv = 0; jv < 8; ++jv)
            for (int iu = 0; iu < 8; ++iu) {
                int Pc[3];
                Pc[d] = ghost_d >> 1;
                Pc[du] = O[du] / 2 - 2 + iu;
                Pc[dv] = O[dv] / 2 - 2 + jv;
                int q = -1;
                if (Pc[0] >= 0 && Pc[1] >= 0 && Pc[2] >= 0 && Pc[0] < Lc.n[0] && Pc[1] < Lc.n[1] && Pc[2] < Lc.n[2])
                    q = Lc.brick_at(Pc[0] >> 3, Pc[1] >> 3, Pc[2] >> 3);
                gidx[jv][iu] = q < 0 ? -1 : (ec.b0 + q) * 512 + (Pc[0] & 7) + 8 * (Pc[1] & 7) + 64 * (Pc[2] & 7);
                av[jv][iu] = q >= 0 && !Lf.has_cell(2 * Pc[0], 2 * Pc[1], 2 * Pc[2]);
            }
        for (int m = 0; m < 16; ++m) {
            int mu = m & 3, mv = m >> 2;
            uint32_t mask = 0;
            for (int jv = 0; jv < 5; ++jv)
                for (int iu = 0; iu < 5; ++iu)
                    if (av[mv + jv][mu + iu]) mask |= 1u << (iu + 5 * jv);
            int pat = select_pattern(mask);
            int u0, v0, npn;
            pattern_window(pat, u0, v0, npn);
            M.cf_pat[(size_t)t * 16 + m] = (uint8_t)pat;
            for (int b = 0; b < 3; ++b)
                for (int a = 0; a < 3; ++a) {
                    int ou = 0, ov = 0;  // unused nodes point at the centre (weight 0)
                    if (a < npn && b < npn) {
                        ou = u0 + a;
                        ov = v0 + b;
                    }
                    int32_t gi = gidx[mv + 2 + ov][mu + 2 + ou];
                    if (gi < 0) {
                        M.error = "coarse-fine window leaves the coarser level (nesting violated)";
                        gi = 0;
                    }
                    M.cf_idx[((size_t)t * 16 + m) * 9 + a + 3 * b] = gi;
                }
        }
    }

    // bricks of AMR levels with uncovered cells next to covered ones; AMR
    // brick list; composite cell counts
    M.dof.assign(np, std::vector<int64_t>());
    for (size_t ei = 0; ei < M.ent.size(); ++ei) {
        Meta::Entry &e = M.ent[ei];
        e.rf0 = (int)M.reflux.size();
        const Problem &P = *probs[e.prob];
        if (e.amr >= 0) {
            int64_t dof = 0;
            for (int g = e.b0; g < e.b0 + e.nb; ++g) {
                M.amr_bricks.push_back(g);
                uint8_t cm = M.cmask[g];
                dof += 64 * (8 - __builtin_popcount(cm));
                // a brick needs the update only next to a covered cell: in
                // itself or in a face neighbour
                bool near = cm != 0;
                for (int f = 0; f < 6 && !near; ++f) {
                    int q = M.nbr[(size_t)g * 6 + f];
                    near = q >= 0 && M.cmask[q] != 0;
                }
                bool want = false;
                for (int o = 0; o < 8 && near && !want && cm != 0xFF; ++o) {
                    if ((cm >> o) & 1) continue;
                    for (int d = 0; d < 3 && !want; ++d)
                        for (int s = -1; s <= 1 && !want; s += 2) {
                            int od = (o >> d) & 1;
                            int on = o ^ (1 << d);
                            bool inside = (s > 0) ? od == 0 : od == 1;
                            if (inside) {
                                want = (cm >> on) & 1;
                            } else {
                                int f = M.nbr[(size_t)g * 6 + 2 * d + (s > 0)];
                                if (f >= 0) want = (M.cmask[f] >> on) & 1;
                            }
                        }
                }
                if (want) M.reflux.push_back(g);
            }
            if ((int)M.dof[e.prob].size() <= e.amr) M.dof[e.prob].resize(e.amr + 1, 0);
            M.dof[e.prob][e.amr] = dof;
        }
        e.nrf = (int)M.reflux.size() - e.rf0;
        (void)P;
    }
}

}  // namespace amrmg
