// amrmg_internal.hpp -- data layout shared by the host driver and the HIP
// kernels of libamrmg (no torch types, no oracle code).
//
// Internal layout ("bricks"): every level, the user-visible AMR levels and
// the geometric-multigrid levels below level 0 alike, is cut into 8x8x8-cell
// bricks (the blocking factor).  Work arrays of the cycle (e, r, the
// coarse-fine ghost parts) hold one contiguous 512-cell slab per brick, x
// fastest inside the brick.  Bricks of all levels share one global
// numbering, level by level, coarsest first; a kernel works on a contiguous
// range of bricks.  phi, rho and E stay in the caller's box-list layout and
// are reached through each brick's user-layout base and strides; inside a
// solve, phi and rho are copied into brick layout (FP64) and back.
#pragma once
#include <cstdint>

namespace amrmg {

constexpr int BRICK = 8;
constexpr int BRICK_CELLS = 512;

// per-level constants
struct LevelConst {
    double ih2[3];   // 1 / h_d^2
    double h[3];
    double abnd[3];  // boundary ghost u_g = abnd u_c (+ 2 g): -1 for Dirichlet, (2 d - h)/(2 d + h) for Robin
    int amr;         // AMR level number, -1 below level 0
    int pad;
};

// Level ids: every level of every problem in a launch has an id (its entry in
// the level table); bricks carry it in org[].w, and per-level data (spacing,
// user-layout base pointers of phi, rho and E) is looked up by it.

// device view of the hierarchy metadata (all pointers are device pointers)
struct DevMeta {
    const int4 *org;          // [nbrick] brick origin in cells (x, y, z) and level id (w)
    const int32_t *nbr;       // [nbrick*6] face 2d+(s>0): brick id >= 0, or -1-gface
    const int32_t *child;     // [nbrick*8] child brick per octant or -1
    const int32_t *par;       // [nbrick] (parent brick << 3 | octant) or -1
    const uint8_t *cmask;     // [nbrick] covered-octant mask
    const int64_t *ubase;     // [nbrick] user-layout index of the brick's (0,0,0) cell
    const int2 *ustr;         // [nbrick] user-layout strides (y, z)
    const int32_t *gf_owner;  // [ngface] brick << 3 | face
    const double *gbc;        // [nbc*64] Dirichlet values at boundary face centres
    const uint8_t *cf_pat;    // [ncf*16] pattern id per coarse cell of a coarse-fine face
    const int32_t *cf_idx;    // [ncf*16*9] coarse cell (brick*512+local) of each window node
    const LevelConst *lc;     // [nlev]
    int32_t nbc;              // boundary faces are gface [0, nbc)
    int32_t ncf;              // coarse-fine faces are gface [nbc, nbc+ncf)
};

// per level id: what the kernels that build the brick tables and generate
// face data (Dirichlet values of boundary faces, coarse-fine windows) need
// to know about its level
struct EntryDev {
    double lo[3];    // problem domain lower corner
    double h[3];     // cell size
    double eps0;
    int n[3];        // index extent
    int nbk[3];      // brick grid extent
    int amr;         // AMR level number, -1 below level 0
    int crse;        // level id of the next coarser level of the problem, -1 if none
    int bmap_off;    // offset of the brick map (global brick ids, -1 = no brick) in the map pool
    int mono_off;    // first monopole (q, x, y, z) of the problem in the monopole pool
    int mono_n;      // number of monopoles
    int b0, nb;      // its bricks [b0, b0 + nb)
    int amr_pos;     // position of its first brick in the list of AMR bricks (AMR levels)
    int pad;
};

// one box of a level, in bricks: the level's bricks are numbered box by box,
// x fastest inside a box, from g0
struct BoxDev {
    int lo[3];      // first brick (brick index space of the level)
    int ext[3];     // bricks per axis
    int g0;         // global id of its first brick
    int ent;        // level id
    int64_t uoff;   // caller's-layout offset of the box on its level (cells)
    int nx, ny;     // box extent in cells along x and y (caller's-layout strides)
};

}  // namespace amrmg
