// Sanitizer driver for the product's host hierarchy code
// (paper_1812_03689_amd/csrc/amrmg_hier.cpp), built with
// -fsanitize=address,undefined by tests/test_sanitizers.py: box generation
// from random tags on boxes of several shapes, nesting checks (valid and
// invalid), pattern tables, direct-solve tables (Dirichlet and Robin), the
// levels below level 0, and the whole host metadata (brick tables, faces,
// coarse-fine windows) of one problem and of a batch of two.  Links only
// product code.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "amrmg_hier.hpp"

using namespace amrmg;

static uint64_t rng = 0x9E3779B97F4A7C15ull;
static double unif()
{
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (double)(rng >> 11) * (1.0 / 9007199254740992.0);
}

// a problem with levels tagged around a centre (tags: cells within r of c)
static Problem make_problem(const int n0[3], int levels, double robin, double c0)
{
    Problem P;
    for (int d = 0; d < 3; ++d) {
        P.lo[d] = 0.0;
        P.hi[d] = 1.0;
    }
    P.robin = robin;
    if (robin == 0.0) P.mono = {1.0, c0, 0.5, 0.5};
    HostLevel L0;
    level_init(L0, n0, P.lo, P.hi);
    L0.amr = 0;
    level_set_boxes(L0, {Box{{0, 0, 0}, {n0[0], n0[1], n0[2]}}});
    P.lev.push_back(L0);
    for (int l = 0; l < levels; ++l) {
        const HostLevel &L = P.lev.back();
        std::vector<uint8_t> tags(L.ncells(), 0);
        int64_t t = 0;
        for (const Box &B : L.boxes)
            for (int k = B.lo[2]; k < B.hi[2]; ++k)
                for (int j = B.lo[1]; j < B.hi[1]; ++j)
                    for (int i = B.lo[0]; i < B.hi[0]; ++i, ++t) {
                        const double x = (i + 0.5) / L.n[0] - c0, y = (j + 0.5) / L.n[1] - 0.5,
                                     z = (k + 0.5) / L.n[2] - 0.5;
                        tags[t] = (x * x + y * y + z * z < 0.03 || unif() < 0.002) ? 1 : 0;
                    }
        std::vector<Box> boxes = generate_boxes(L, tags.data(), 1, 2, 8, 16);
        if (boxes.empty()) break;
        if (!check_nesting(L, boxes, 2).empty()) {
            std::fprintf(stderr, "generated boxes break nesting\n");
            std::exit(3);
        }
        HostLevel F;
        const int nf[3] = {2 * L.n[0], 2 * L.n[1], 2 * L.n[2]};
        level_init(F, nf, P.lo, P.hi);
        F.amr = (int)P.lev.size();
        level_set_boxes(F, boxes);
        P.lev.push_back(F);
    }
    add_levels_below(P);
    return P;
}

int main()
{
    // pattern selection over every 5x5 mask with the centre available
    for (uint32_t m = 0; m < (1u << 25); m += 4099) (void)select_pattern(m | (1u << 12));
    std::vector<double> w = cf_weight_table();
    uint32_t masks[13];
    int org[42];
    pattern_tables(masks, org);
    for (int p = 0; p < 9; ++p) (void)quadratic_mask(p);
    // direct-solve tables
    const int nd[3] = {24, 40, 16};
    const double h[3] = {1.0 / 24, 1.0 / 40, 1.0 / 16}, ad[3] = {-1, -1, -1}, ar[3] = {0.9, 0.95, 0.85};
    std::vector<double> t1 = direct_tables(nd, h, ad), t2 = direct_tables(nd, h, ar);
    // an invalid explicit box list (misaligned, overlapping, outside, not nested)
    {
        HostLevel L;
        const int n[3] = {32, 32, 32};
        const double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
        level_init(L, n, lo, hi);
        level_set_boxes(L, {Box{{8, 8, 8}, {24, 24, 24}}});
        const std::vector<std::vector<Box>> bad = {{Box{{3, 16, 16}, {19, 32, 32}}},
                                                   {Box{{16, 16, 16}, {40, 40, 40}}, Box{{32, 32, 32}, {48, 48, 48}}},
                                                   {Box{{56, 56, 56}, {72, 72, 72}}},
                                                   {Box{{16, 16, 16}, {24, 24, 24}}}};
        for (const auto &B : bad)
            if (check_nesting(L, B, 2).empty()) {
                std::fprintf(stderr, "an invalid box list passed the nesting check\n");
                return 4;
            }
    }
    // one problem (Dirichlet), another (Robin), and the two as a batch
    const int na[3] = {32, 32, 32}, nb[3] = {16, 24, 40};
    Problem A = make_problem(na, 2, 0.0, 0.5), B = make_problem(nb, 2, 0.7, 0.4);
    Meta M1, M2, M3;
    build_meta({&A}, M1, true);
    build_meta({&B}, M2, true);
    build_meta({&A, &B}, M3, true);
    meta_entries({&A, &B}, M3);
    for (const Meta *M : {&M1, &M2, &M3})
        if (!M->error.empty()) {
            std::fprintf(stderr, "metadata error: %s\n", M->error.c_str());
            return 5;
        }
    double ab[3];
    boundary_ghost(B, h, ab);
    std::printf("hier sanitize ok: %d + %d bricks, %zu weights\n", M1.nbrick, M2.nbrick, w.size());
    return 0;
}
