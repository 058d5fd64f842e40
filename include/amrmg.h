/*
 * amrmg.h -- C ABI of the MI355X (gfx950) composite-grid AMR multigrid
 * Poisson path for electrostatic particle-in-cell, after Frey, Adelmann &
 * Locans, "On Architecture and Performance of Adaptive Mesh Refinement in an
 * Electrostatics Particle-In-Cell Code" (arXiv:1812.03689).
 *
 * The path (the space-charge workflow of Fig. 2 of the paper):
 * cloud-in-cell charge deposition -> tagging (charge, potential or field)
 * and box generation (Sec. 4.2) -> composite AMR multigrid solve of
 * L_comp phi = -rho / eps0 (Sec. 5.3, Alg. 1-3) with Dirichlet or Robin
 * boundaries (Sec. 5.2) -> E = -grad phi (Alg. 2) -> interpolation of E to
 * the particles; optionally wrapped in the domain transform of Sec. 4.1
 * (particles into computation space, fields rescaled on the grid).  The
 * Lorentz transform of the co-moving frame is the caller's.
 *
 * Conventions shared by every call:
 *   - Domain [lo, hi) with n0 cells per axis on level 0; refinement ratio 2
 *     (Eq. mesh_spacing with r = 2); cell-centred data (Sec. 3).
 *   - A level is a list of disjoint boxes [lo, hi) (hi exclusive) in that
 *     level's index space, every edge a multiple of the blocking factor 8.
 *     Level 0 is one box covering the domain.
 *   - Level arrays ("user layout") concatenate the boxes in box-list order;
 *     each box is stored x-fastest: cell (i,j,k) of box b sits at
 *     offsets[b] + (i-lo_x) + nx*((j-lo_y) + ny*(k-lo_z)).
 *   - All particle and field arrays are DEVICE memory owned by the caller;
 *     the library never frees them.  Host arrays are marked "host".
 *   - Every call enqueues on the stream given to amrmg_create.  deposit and
 *     gather are asynchronous; build_hierarchy, hierarchy_info and solve
 *     synchronise the stream.
 *   - Calls return an amrmg_status; no exception crosses the ABI.  On error
 *     amrmg_last_error() returns a thread-local message.  A context is not
 *     thread-safe.
 */
#ifndef AMRMG_H
#define AMRMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct amrmg_ctx amrmg_ctx;

typedef enum {
    AMRMG_OK = 0,
    AMRMG_E_INVALID = -1,         /* bad argument or parameter */
    AMRMG_E_HIP = -2,             /* a HIP runtime call failed */
    AMRMG_E_NOT_CONVERGED = -3,   /* max_iters reached; phi, E and stats are still written */
    AMRMG_E_NESTING = -4,         /* explicit boxes violate alignment or proper nesting */
    AMRMG_E_OOM = -5,             /* device allocation failed or workspace too small */
    AMRMG_E_STATE = -6,           /* call out of order (e.g. solve before build_hierarchy) */
    AMRMG_E_NOT_IMPLEMENTED = -7
} amrmg_status;

enum { AMRMG_POS_F64 = 0, AMRMG_POS_F32 = 1 };
enum { AMRMG_FP64 = 0, AMRMG_MIXED = 1 };
/* Smoothers: AMRMG_GSRB = red-black Gauss-Seidel inside each 8^3 brick with
 * the brick halo taken from the previous sweep (one pass per sweep, the way a
 * parallel Gauss-Seidel works inside and between subdomains);
 * AMRMG_GSRB_GLOBAL = red-black over the whole level (two passes per sweep);
 * AMRMG_JACOBI = damped Jacobi.  The small levels at the bottom of the cycle
 * always use whole-level red-black inside one workgroup. */
enum { AMRMG_GSRB = 0, AMRMG_JACOBI = 1, AMRMG_GSRB_GLOBAL = 2 };
/* Bottom solvers of the coarsest grid (the multigrid levels below level 0
 * halve the base grid while every edge stays a multiple of 16 and some edge
 * exceeds 64 cells): AMRMG_BOTTOM_AUTO solves it directly (separable
 * eigendecomposition of the Dirichlet Laplacian on its one box) when every
 * edge is at most 64 cells, and by CG to bottom_rtol otherwise;
 * AMRMG_BOTTOM_CG always uses CG. */
enum { AMRMG_BOTTOM_AUTO = 0, AMRMG_BOTTOM_CG = 1 };
enum { AMRMG_MAX_LEVELS = 8 };
/* Refinement criteria of amrmg_build_hierarchy (Sec. 4.2): tag a cell of
 * level l when |rho| > lambda max|rho| (AMRMG_TAG_CHARGE), |phi| > lambda
 * max|phi| (AMRMG_TAG_POTENTIAL), or |E_w| > lambda max|E_w| for some
 * component w (AMRMG_TAG_EFIELD), each maximum taken over level l.  phi and
 * E come from solving the composite problem on the levels built so far
 * (0..l) to a relative residual of AMRMG_TAG_SOLVE_TOL. */
enum { AMRMG_TAG_CHARGE = 0, AMRMG_TAG_POTENTIAL = 1, AMRMG_TAG_EFIELD = 2 };
#define AMRMG_TAG_SOLVE_TOL 1e-10

/* Solver and hierarchy parameters.  amrmg_default_params fills the defaults
 * named in brackets. */
typedef struct amrmg_params {
    double lo[3], hi[3];        /* domain [0,0,0]-[1,1,1] */
    int32_t n0[3];              /* level-0 cells per axis, multiples of 8 [32] */
    int32_t max_level;          /* finest level index allowed, 0..7 [2] */
    int32_t ref_ratio;          /* must be 2 [2] */
    int32_t blocking_factor;    /* must be 8 [8] */
    int32_t max_grid_size;      /* max box edge on refined levels, multiple of 8 [32] */
    int32_t n_buffer;           /* tag dilation in cells [1] */
    int32_t n_proper;           /* proper-nesting margin in coarse cells [2] */
    double eps0;                /* vacuum permittivity [1] */
    int32_t n_monopoles;        /* Dirichlet data g(x) = sum q/(4 pi eps0 |x-x_k|); 0 -> g = 0 */
    const double *monopoles;    /* host [n_monopoles][4] = q, x, y, z; copied by amrmg_create */
    int32_t precision;          /* AMRMG_FP64 or AMRMG_MIXED [MIXED] */
    int32_t smoother;           /* AMRMG_GSRB, AMRMG_JACOBI or AMRMG_GSRB_GLOBAL [GSRB] */
    int32_t nu1, nu2;           /* pre / post smoothing sweeps [2, 4] */
    double omega;               /* damped-Jacobi weight [6/7] */
    int32_t norm_p;             /* residual norm: 1, 2, or 0 for max-norm [2] */
    int32_t max_iters;          /* V-cycle cap i_max [50] */
    double bottom_rtol;         /* CG tolerance on the coarsest grid, relative to its right-hand
                                   side; it bounds only how well each cycle treats the smoothest
                                   modes, not the accuracy of the result [1e-2] */
    int32_t bottom;             /* AMRMG_BOTTOM_AUTO or AMRMG_BOTTOM_CG [AUTO] */
    int32_t tag_policy;         /* AMRMG_TAG_CHARGE, AMRMG_TAG_POTENTIAL or AMRMG_TAG_EFIELD [CHARGE] */
    double robin_d;             /* > 0: open boundary by the Robin condition d phi/dn + phi/robin_d = 0
                                   (Eq. robin_bc, central difference across the boundary face: ghost
                                   (2 d - h)/(2 d + h) phi_in) on every face, with no monopoles;
                                   0: Dirichlet data from the monopoles [0] */
} amrmg_params;

/* Per-solve statistics. */
typedef struct amrmg_solve_stats {
    int32_t iters;              /* V-cycles until every level met the tolerance (the
                                   cycles run when not converged); phi and rel_residual
                                   are those after the last cycle run, which can be a
                                   later one in a batch, or when a cycle queued ahead
                                   of the norms that stopped the solve ran as well */
    int32_t converged;          /* 1 when every level met the tolerance */
    int32_t nlevels;
    int32_t bottom_iters_max;   /* largest CG iteration count of one bottom solve */
    double rel_residual[AMRMG_MAX_LEVELS]; /* final ||r^l||_p / ||b^l||_p */
    double time_ms;             /* device time from the first kernel to the last (events) */
    int64_t dof;                /* composite cells: sum over levels of uncovered cells */
} amrmg_solve_stats;

void amrmg_default_params(amrmg_params *p);

/* Create a context bound to a HIP stream (NULL = the null stream).
 * The parameters are validated and copied; *out receives the context. */
amrmg_status amrmg_create(const amrmg_params *p, void *hip_stream, amrmg_ctx **out);
void amrmg_destroy(amrmg_ctx *ctx);
const char *amrmg_last_error(void);

/* Build the level hierarchy (Sec. 3 and Sec. 4.2 of the paper).  For each
 * level l < max_level in turn: deposit the particles on level l, tag the
 * cells with |rho^l| > tag_rel[l] * max|rho^l| (or, with the potential and
 * field criteria of tag_policy, solve on levels 0..l and tag by |phi^l| or
 * the components of E^l; the solve's status is returned if it fails, with
 * the context left unbuilt), dilate the tags by n_buffer
 * cells, group them into 8-cell blocks of level l+1, drop blocks that break
 * proper nesting, and merge the blocks greedily (x, then y, then z, at most
 * max_grid_size cells per edge) into the boxes of level l+1.  The procedure is
 * pure integer work after the tagging compare and is fully specified, so box
 * lists are reproducible bit for bit.
 *   pos_dtype      AMRMG_POS_F64 or AMRMG_POS_F32 (x, y, z device arrays of n)
 *   q              device [n] charges (FP64)
 *   tag_rel        host [max_level] relative thresholds (may be NULL when
 *                  every refined level is given explicitly)
 *   explicit_boxes host [n_explicit][7] = level, lo[3], hi[3] (level index
 *                  space, hi exclusive) or NULL; a level with explicit boxes
 *                  is not tagged.  Misaligned or badly nested boxes return
 *                  AMRMG_E_NESTING.
 * Levels with no tagged block end the hierarchy early.  Synchronises. */
amrmg_status amrmg_build_hierarchy(amrmg_ctx *ctx, int pos_dtype, const void *x, const void *y,
                                   const void *z, const double *q, int64_t n, const double *tag_rel,
                                   const int32_t *explicit_boxes, int32_t n_explicit);

/* Sizes of the built hierarchy: host outputs, arrays of at least
 * AMRMG_MAX_LEVELS entries (any pointer may be NULL). */
amrmg_status amrmg_hierarchy_info(const amrmg_ctx *ctx, int32_t *nlevels, int32_t *nboxes,
                                  int64_t *ncells, int64_t *ndof);

/* Box list of one level: host boxes[nb][6] = lo[3], hi[3] and offsets[nb+1]
 * (cells, exclusive prefix sums of the box volumes). */
amrmg_status amrmg_get_boxes(const amrmg_ctx *ctx, int32_t level, int32_t *boxes, int64_t *offsets);

/* Coarse-fine ghost faces of a refined level: for every fine cell face that
 * lies on the coarse-fine interface, host out[m][6] = i, j, k (fine cell,
 * level index space), d (normal axis 0..2), s (-1 or +1, side of the face),
 * pattern id (0..8: the quadratic windows of Tab. bit_pattern in the printed
 * order of selection; 9..12: the bilinear windows of the following table;
 * 13: centre value only).  cap bounds the rows written; *count receives the
 * total number of such faces. */
amrmg_status amrmg_cf_faces(const amrmg_ctx *ctx, int32_t level, int32_t *out, int64_t cap,
                            int64_t *count);

/* The brick tables of the built hierarchy, copied to the host for inspection
 * and tests.  Every level (levels below level 0 first, then the AMR levels)
 * is cut into 8^3-cell bricks numbered level by level, box by box, x fastest
 * inside a box.  counts (host [4], required): bricks, boundary faces,
 * coarse-fine faces, bricks with coarse-fine coarse cells (the update list).
 * Each array may be NULL; sizes follow the counts:
 *   org    [bricks][4]: origin (cells, level index space) and level (0 = the
 *          coarsest grid, AMR level l = l + levels below level 0)
 *   nbr    [bricks][6]: per face 2d + (s > 0) the neighbour brick, or
 *          -1 - face id (boundary faces first, then coarse-fine faces, both
 *          in brick and face order)
 *   child  [bricks][8]: child brick per octant (x bit 0, y bit 1, z bit 2) or -1
 *   parent [bricks]: parent << 3 | octant, or -1
 *   cmask  [bricks]: covered octants (AMR levels)
 *   ubase  [bricks], ustr [bricks][2]: caller's-layout index of the brick's
 *          first cell and the y, z strides (AMR levels; 0 below level 0)
 *   owner  [faces]: brick << 3 | face
 *   update [update count]: the bricks with coarse-fine coarse cells
 * Synchronises. */
amrmg_status amrmg_brick_tables(const amrmg_ctx *ctx, int64_t *counts, int32_t *org, int32_t *nbr,
                                int32_t *child, int32_t *parent, uint8_t *cmask, int64_t *ubase,
                                int32_t *ustr, int32_t *owner, int32_t *update);

/* Device workspace for solve: the size needed for the current hierarchy and
 * precision, and an optional caller-owned buffer (device, >= that size,
 * 256-byte aligned) that the context then uses instead of allocating its own.
 * Passing NULL returns to library-owned memory. */
amrmg_status amrmg_workspace_size(const amrmg_ctx *ctx, size_t *bytes);
amrmg_status amrmg_set_workspace(amrmg_ctx *ctx, void *dev, size_t bytes);

/* Cloud-in-cell deposit on every level: rho[l] (device, user layout of level
 * l, overwritten) receives sum_p q_p W(x_p - x_i) / (h_x h_y h_z) with the
 * tensor-product linear (CIC) weights in FP64 (FP32 positions are promoted
 * first).  Stencil indices are clamped to the level's index space; stencil
 * cells outside the level's boxes receive nothing.  Particles outside
 * [lo, hi) are skipped and counted in *n_outside (host, may be NULL; reading
 * it synchronises).  Accumulation uses FP64 atomics, so the rounding order
 * varies run to run. */
amrmg_status amrmg_deposit(amrmg_ctx *ctx, int pos_dtype, const void *x, const void *y,
                           const void *z, const double *q, int64_t n, double *const *rho,
                           int64_t *n_outside);

/* The same cloud-in-cell deposit (same weights, clamping, skipped particles
 * and count) of the particles given to the last amrmg_build_hierarchy,
 * without reading them again: the build keeps the charge of every level it
 * deposited for its tagging passes (each level below the last tagged one)
 * and a copy of the particles in spatial order, from which the other levels
 * (the finest, and levels whose next level was given explicitly) are
 * deposited here.  The deposit a PIC step does anyway after a regrid
 * (Sec. 1's particle-mesh cycle: deposit, solve, gather) then costs little
 * more than copies.  rho and n_outside as in amrmg_deposit.
 * AMRMG_E_STATE when no hierarchy is built, or when the build kept no copy
 * (more than 2^31 - 1 particles).  The particle arrays given to the build
 * may have changed since: the result is that of the build's particles. */
amrmg_status amrmg_deposit_built(amrmg_ctx *ctx, double *const *rho, int64_t *n_outside);

/* Solve the composite problem (Alg. 2 of the paper): A_comp phi = rho/eps0
 * with A = -Laplacian discretised by flux differencing with flux matching at
 * coarse-fine faces (Eqs. lap_flux_differencing, coarse_fluxes,
 * flux_differencing), quadratic two-step Lagrange ghosts (Eq. 2d_lagrange,
 * Tab. bit_pattern) and the Dirichlet data through a linear ghost
 * 2 g - phi_in (or, with robin_d > 0, the Robin ghost of robin_d).  V-cycles (Alg. 3) run until ||r^l||_p <= tol ||b^l||_p on
 * every level, b^l being the uncovered right-hand side including the
 * Dirichlet data, or until max_iters.  In AMRMG_MIXED the cycle works in
 * FP32 on the correction equation of an FP64 outer residual (iterative
 * refinement).  Afterwards phi is averaged down onto covered cells and, if
 * E != NULL, E[3*l + d] = -(phi_{+} - phi_{-}) / (2 h_d) on every cell.
 *   rho  device [L] user-layout charge density (read)
 *   phi  device [L] user layout: initial guess in, solution out
 *   E    device [3L] or NULL
 *   stats host, may be NULL.  Synchronises. */
amrmg_status amrmg_solve(amrmg_ctx *ctx, double *const *rho, double *const *phi, double *const *E,
                         double tol, amrmg_solve_stats *stats);

/* For callers that cannot allocate device memory (code that runs under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * solve of amrmg_solve, same arguments, same results, that allocates no
 * device or pinned host memory and instantiates no graph.  Its workspace is
 * carved from a file-scope device array of AMRMG_NOALLOC_SCRATCH_BYTES
 * (128 MiB) that the library's code object holds on every GPU it runs on
 * until the process ends; the array's address on a device is looked up once,
 * when the first context on that device is created.  The cycle is launched
 * kernel by kernel (no graph replay), with the sweep shapes amrmg_solve has
 * tuned so far or the size rule.  The hierarchy must have been built
 * (amrmg_build_hierarchy allocates); a hierarchy whose workspace
 * (amrmg_workspace_size) exceeds the array gives AMRMG_E_OOM with phi, E
 * and stats untouched.  Every call on a GPU shares that GPU's array and
 * leaves its contents behind (nothing in it is read before the call writes
 * it): calls that overlap in time on one GPU -- contexts on different
 * streams driven from different threads -- race and must not be made.
 * AMRMG_E_HIP when the array's address could not be looked up on the
 * context's device.  Synchronises. */
#define AMRMG_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
amrmg_status amrmg_solve_noalloc(amrmg_ctx *ctx, double *const *rho, double *const *phi, double *const *E,
                                 double tol, amrmg_solve_stats *stats);

/* Interpolate E to particles with the deposit's CIC weights, on the finest
 * level whose boxes hold all 8 stencil cells.  Ex, Ey, Ez device [n];
 * particles outside the domain get 0.  When n equals the particle count of
 * the last build, its spatial visiting order is used (the arrays are taken
 * to hold the same particles, perhaps moved): E is computed in that order
 * into a staging buffer of 32 n bytes, which the context allocates on first
 * use and keeps, and then written in the caller's order; when the buffer
 * cannot be allocated E is written at its places directly (same values). */
amrmg_status amrmg_gather(amrmg_ctx *ctx, int pos_dtype, const void *x, const void *y,
                          const void *z, int64_t n, double *const *E, double *Ex, double *Ey,
                          double *Ez);

/* The same gather (same weights, level choice and result, bit for bit) at
 * the particles given to the last amrmg_build_hierarchy, read from the
 * build's copy of them in spatial order instead of the caller's arrays: the
 * gather of a PIC step at the positions it deposited (Sec. 1's particle-mesh
 * cycle), with coalesced position reads; only the writes of E follow the
 * caller's order (through the staging buffer of amrmg_gather).  Ex, Ey, Ez
 * device [n], n the particle count of that
 * build, in its order.  AMRMG_E_STATE when no hierarchy is built or the
 * build kept no copy (as amrmg_deposit_built).  The particle arrays given to
 * the build may have changed since: the result is that at the build's
 * particles. */
amrmg_status amrmg_gather_built(amrmg_ctx *ctx, double *const *E, double *Ex, double *Ey, double *Ez);

/* The spatial visiting order of the particles given to the last
 * amrmg_build_hierarchy: the order in which the deposit, the tagging passes
 * and the gather of those particles visit them, which keeps the particles of
 * a workgroup in a few neighbouring cells (Sec. 1's particle-mesh cycle
 * gains from it; the order itself is this library's choice).  The particles
 * are sorted by the Morton code of their cell on the finest level's grid
 * (the level-0 grid refined max_level times; beyond 1024 cells per axis,
 * cells merged 2^3 at a time), stably: particles of one cell keep their index
 * order.  A particle outside the domain takes the nearest cell.
 *   perm   device [n]: perm[i] = the index of the i-th particle visited
 *   n      the build's particle count
 * Enqueued on the context's stream.  AMRMG_E_STATE when no hierarchy is
 * built or the build kept no order (no particles, or more than 2^31 - 1);
 * AMRMG_E_INVALID when n differs from the build's count. */
amrmg_status amrmg_visiting_order(amrmg_ctx *ctx, uint32_t *perm, int64_t n);

/* Domain transform (Sec. 4.1 of the paper): map particles from particle
 * space S_p into the computation space S_c = [-l0,l0] x [-l1,l1] x [-l2,l2]
 * around the reference position c.  With Gamma(x, l) = max_d |x_d - c_d| /
 * l_d, the scale is s = max over the n particles of Gamma (the particle
 * farthest out in units of l lands on the boundary of S_c) and
 * x* = (x - c) / s, computed in FP64 (FP32 positions are promoted, the
 * result rounded back).  The mesh domain (lo, hi of the parameters) is then
 * S_c enlarged by the margin the caller chooses.  Solving in S_c with the
 * same charges gives phi* and E*; amrmg_rescale_fields turns them into the
 * particle-space fields.
 *   x, y, z     device [n] (pos_dtype); xs, ys, zs device [n] outputs of the
 *               same type, which may alias x, y, z
 *   center, l   host [3]; l > 0
 *   s           host output; 0 when n == 0 (nothing is written)
 * AMRMG_E_INVALID for a non-finite coordinate or when every particle sits
 * at c (s = 0); then xs, ys, zs are not written.  Synchronises (s is read
 * back); the map itself is enqueued after that. */
amrmg_status amrmg_transform_particles(amrmg_ctx *ctx, int pos_dtype, const void *x, const void *y,
                                       const void *z, int64_t n, const double *center, const double *l,
                                       void *xs, void *ys, void *zs, double *s);

/* Rescale the fields of a solve in computation space to particle space, on
 * the grid (Eqs. potential_transform and efield_transform, three
 * dimensions): phi[l] /= s and E[3l+d] /= s^2 on every level of the built
 * hierarchy (device, user layout; phi or E may be NULL).  s > 0 as returned
 * by amrmg_transform_particles.  Asynchronous. */
amrmg_status amrmg_rescale_fields(amrmg_ctx *ctx, double s, double *const *phi, double *const *E);

/* The FP64 composite residual of Alg. 1 on every level for given rho and phi:
 * r[l] = U^l (rho^l/eps0 - A_comp phi) (user layout, device, zero on covered
 * cells).  Diagnostic entry point; it runs the same kernels as the solve's
 * outer residual. */
amrmg_status amrmg_residual(amrmg_ctx *ctx, double *const *rho, double *const *phi, double *const *r);

/* Solve nb independent problems, each with its own context and hierarchy, as
 * one batch: every kernel of the cycle runs once over the bricks of all
 * problems (level k of every problem, counted from its coarsest grid, in one
 * launch).  The contexts must be distinct, built, and share the stream and
 * the solver settings (precision, smoother, nu1, nu2, omega, norm_p,
 * max_iters, bottom, bottom_rtol, eps0); otherwise AMRMG_E_INVALID.  rho[i],
 * phi[i] as in amrmg_solve (no E).  The iteration runs until every problem
 * meets tol; stats host [nb] or NULL gives each problem the iteration at which
 * it met it.  The merged metadata is kept by ctxs[0] and rebuilt when any
 * context builds a new hierarchy or the context list changes. */
amrmg_status amrmg_solve_batch(amrmg_ctx *const *ctxs, int32_t nb, double *const *const *rho,
                               double *const *const *phi, double tol, amrmg_solve_stats *stats);

/* Kernel classes for amrmg_profile_* (per-launch HIP events on the context's
 * stream; algorithmic bytes per launch as defined in the design notes).  The
 * coarse-fine residual update runs in the restriction's launch and is timed
 * as AMRMG_K_RESTRICT; AMRMG_K_REFLUX records nothing. */
enum {
    AMRMG_K_GSRB = 0, AMRMG_K_JACOBI, AMRMG_K_RESTRICT, AMRMG_K_PROLONG, AMRMG_K_REFLUX, AMRMG_K_CPART,
    AMRMG_K_RESIDUAL, AMRMG_K_PHI_UPDATE, AMRMG_K_BOTTOM, AMRMG_K_EFIELD, AMRMG_K_AVGDOWN, AMRMG_K_DEPOSIT,
    AMRMG_K_GATHER, AMRMG_K_NCLASS
};

/* Enable (mask != 0: bit c = class c) or disable per-launch event timing of
 * the listed kernel classes, and clear the counters.  Off by default.
 * Timing adds two event records per recorded launch. */
amrmg_status amrmg_profile_enable(amrmg_ctx *ctx, uint32_t mask);

/* Totals since the last enable for one class: summed device milliseconds of
 * the recorded launches, their count and their algorithmic bytes (host
 * outputs, any may be NULL).  Synchronises the stream. */
amrmg_status amrmg_profile_read(amrmg_ctx *ctx, int32_t kclass, double *ms, int64_t *launches,
                                double *bytes);

/* The individual launches behind amrmg_profile_read, in launch order: for
 * each of the first min(cap, *count) recorded launches of class kclass since
 * the last enable, its device milliseconds ms[i] and algorithmic bytes
 * bytes[i] (host arrays of cap entries; NULL with cap = 0 to query the
 * count).  *count receives the number recorded (at most 65536 are kept per
 * class; the totals of amrmg_profile_read count every launch).  Synchronises
 * the stream. */
amrmg_status amrmg_profile_launches(amrmg_ctx *ctx, int32_t kclass, double *ms, double *bytes, int64_t cap,
                                    int64_t *count);

#ifdef __cplusplus
}
#endif

#endif /* AMRMG_H */
