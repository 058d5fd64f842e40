// amrmg_hier.hpp -- host-side hierarchy of libamrmg: box lists, the brick
// decomposition, box generation from tags, and the metadata the kernels read
// (neighbour and parent/child tables, boundary and coarse-fine faces with
// their interpolation patterns).  Plain C++ (no HIP), so that it also builds
// and runs on a machine without a GPU.
#pragma once
#include <array>
#include <cstdint>
#include <string>
#include <vector>

namespace amrmg {

struct Box {
    int lo[3], hi[3];
    int64_t volume() const { return (int64_t)(hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]); }
};

// One level of one problem.  AMR levels carry the caller's box list; the
// multigrid levels below level 0 are a single box of the coarsened domain.
struct HostLevel {
    int n[3] = {0, 0, 0};       // index extent
    double h[3] = {0, 0, 0};
    int amr = -1;               // AMR level number, -1 below level 0
    std::vector<Box> boxes;
    std::vector<int64_t> off;   // user-layout offsets (nb + 1)
    int nbk[3] = {0, 0, 0};     // brick grid extent
    std::vector<int32_t> bmap;  // brick grid -> local brick or -1
    int map_nbk[3] = {0, 0, 0}; // brick grid extent bmap was built for (its entries
                                // other than those of bpos are -1)
    std::vector<int32_t> bpos;  // local brick -> brick grid position (3 each)
    std::vector<int32_t> bbox;  // local brick -> box
    int nbrick() const { return (int)bbox.size(); }
    int64_t ncells() const { return off.empty() ? (int64_t)nbrick() * 512 : off.back(); }
    int brick_at(int bx, int by, int bz) const;  // local brick or -1 (also outside the grid)
    bool has_cell(int i, int j, int k) const;
};

// build offsets and bricks of a level from its boxes (boxes must be 8-aligned)
void level_set_boxes(HostLevel &L, const std::vector<Box> &boxes);
// make level geometry: index extent n, spacing from the domain
void level_init(HostLevel &L, const int n[3], const double lo[3], const double hi[3]);

// Box generation for level l+1 from the tags (user layout) of level L: dilate
// by n_buffer cells, mark 8-fine-cell blocks, drop blocks that break proper
// nesting by n_proper coarse cells, and merge greedily along x, then y, then z
// with edges of at most max_grid_size cells.
std::vector<Box> generate_boxes(const HostLevel &L, const uint8_t *tags, int n_buffer, int n_proper, int bf,
                                int max_grid_size);
// the same procedure split in two: marking the blocks of the finer level
// (size (2 n / bf)^3, 1 = tagged) from cell tags, and nesting + merge of a
// block mask (which it modifies)
void mark_blocks(const HostLevel &L, const uint8_t *tags, int n_buffer, int bf, std::vector<uint8_t> &mark);
std::vector<Box> merge_blocks(const HostLevel &L, uint8_t *mark, int n_proper, int bf, int max_grid_size);
// the two steps of merge_blocks: proper nesting (unmarks blocks whose coarse
// footprint grown by n_proper cells leaves the bricks of L), and the greedy
// merge of a nested mask given as bits in linear block order (bit t % 64 of
// word t / 64 for block t = x + g0 (y + g1 z), g = 2 n / bf blocks per
// axis; the bits are consumed)
void nest_blocks(const HostLevel &L, uint8_t *mark, int n_proper, int bf);
std::vector<Box> merge_block_bits(const int g[3], uint64_t *bits, int bf, int max_grid_size);

// Check boxes of a refined level against its coarser level: 8-alignment,
// inside the index space, disjoint, and proper nesting.  Empty string = ok.
std::string check_nesting(const HostLevel &coarse, const std::vector<Box> &fine, int n_proper);

// coarse-fine interpolation patterns: 0..8 quadratic (printed order),
// 9..12 bilinear, 13 centre only
int select_pattern(uint32_t mask5);
void pattern_window(int pat, int &u0, int &v0, int &np);
// [14][4][9] step-1 weights times 8/15 (see amrmg_kernels.hip)
std::vector<double> cf_weight_table();
// the 25-bit masks of the 9 quadratic windows, built from pattern_window
uint32_t quadratic_mask(int pat);
// the tables the device pattern selection reads: window masks of patterns
// 0..12 and (u0, v0, nodes per axis) of patterns 0..13
void pattern_tables(uint32_t masks13[13], int org14x3[42]);

// Direct solve of the coarsest grid: the cell-centred Laplacian with
// homogeneous boundary ghosts abnd u_c on a full box of n cells is separable;
// along an axis of N cells its 1-D matrix is 2 on the diagonal, 2 - abnd at
// both ends, -1 off the diagonal, times 1/h^2.  For Dirichlet (abnd = -1) it
// has the orthonormal eigenvectors S[i][k] = c_k sin(pi (k+1) (i+1/2) / N),
// c_k = sqrt(2/N) (k < N-1) or sqrt(1/N) (k = N-1), with eigenvalues
// 4 sin^2(pi (k+1) / (2N)) / h^2; otherwise (Robin) they are computed by
// Jacobi rotations.  Layout per axis d (N = n[d]): the forward matrix
// F[k][i] = S[i][k] and the inverse matrix B[i][k] = S[i][k], each N x N,
// output-major; then the three eigenvalue vectors.  Size
// 2 (n0^2 + n1^2 + n2^2) + n0 + n1 + n2 doubles.
std::vector<double> direct_tables(const int n[3], const double h[3], const double abnd[3]);

// One problem (one context): its levels coarsest first; kg = index of AMR
// level 0.
struct Problem {
    double lo[3], hi[3];
    double eps0 = 1.0;
    double robin = 0.0;        // > 0: Robin boundary d phi/dn + phi/robin = 0; 0: Dirichlet
    std::vector<double> mono;  // [n][4] q, x, y, z
    std::vector<HostLevel> lev;
    int kg = 0;
    int namr() const { return (int)lev.size() - kg; }
};

// add the multigrid levels below AMR level 0 (halving while every edge stays
// a multiple of 16 and some edge exceeds 64 cells, so that the coarsest grid
// is small enough for its direct solve); lev[0..] must hold the AMR levels on
// entry
void add_levels_below(Problem &P);

// boundary ghost coefficient per axis of a level of spacing h: u_g = a u_c
// (+ 2 g for Dirichlet data g).  Dirichlet: a = -1.  Robin (Eq. robin_bc,
// central difference across the face): (u_g - u_c)/h + (u_g + u_c)/(2 d) = 0,
// a = (2 d - h) / (2 d + h).
void boundary_ghost(const Problem &P, const double h[3], double a[3]);

// Merged metadata of one or more problems.  Levels are numbered coarsest
// first across problems: level entry (k, i) = level k (counted from each
// problem's coarsest) of problem i, in order k-major; bricks follow the
// level entries.
struct Meta {
    struct Entry {
        int prob, k;      // problem, level index inside it
        int amr;          // AMR level number or -1
        int b0, nb;       // brick range
        int cf0, ncf;     // coarse-fine faces of this level (ids from 0 = first CF face)
        int rf0, nrf;     // reflux list range (bricks of this level with coarse-fine coarse cells)
        double h[3];
    };
    std::vector<Entry> ent;
    std::vector<int> step_ent0;      // per k: first entry of that step (size K+1)
    int K = 0;                       // steps (max levels over problems)
    int nbrick = 0;
    std::vector<int32_t> org;        // [nbrick*4]
    std::vector<int32_t> nbr;        // [nbrick*6]
    std::vector<int32_t> child;      // [nbrick*8]
    std::vector<int32_t> par;        // [nbrick]
    std::vector<uint8_t> cmask;      // [nbrick]
    std::vector<int64_t> ubase;      // [nbrick]
    std::vector<int32_t> ustr;       // [nbrick*2]
    int nbc = 0, ncf = 0;
    std::vector<int32_t> gf_owner;   // [nbc + ncf]
    std::vector<double> gbc;         // [nbc*64]
    std::vector<uint8_t> cf_pat;     // [ncf*16]
    std::vector<int32_t> cf_idx;     // [ncf*16*9]
    std::vector<int32_t> reflux;     // brick ids
    std::vector<int32_t> amr_bricks; // all AMR bricks, in entry order
    std::vector<std::vector<int>> prob_ent;  // per problem: entry index of each level k
    std::vector<std::vector<int64_t>> dof;   // per problem, per AMR level: uncovered cells
    std::string error;                       // non-empty when the hierarchy is inconsistent
};

// The level table only (ent with b0/nb, step_ent0, K, nbrick, prob_ent);
// every other field of M is cleared.  The library builds the brick tables
// from it on the device.
void meta_entries(const std::vector<const Problem *> &probs, Meta &M);
// The whole metadata on the host (meta_entries, then the brick tables, face
// lists, reflux list and composite cell counts).  face_data: also compute
// gbc, cf_pat and cf_idx (the library generates them on the device from
// the same pattern tables).
void build_meta(const std::vector<const Problem *> &probs, Meta &M, bool face_data = true);

}  // namespace amrmg
