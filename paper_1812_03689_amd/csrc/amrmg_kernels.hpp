// amrmg_kernels.hpp -- launchers of the HIP kernels in amrmg_kernels.hip.
#pragma once
#include <hip/hip_runtime.h>

#include "amrmg_internal.hpp"

namespace amrmg {

constexpr int MAX_AMR = 8;

// one AMR level as seen by particle kernels
struct DepLevel {
    double lo[3], hi[3], h[3];
    double ivol;          // 1 / (h_x h_y h_z)
    int n[3];             // index extent of the level
    int nbk[3];           // brick grid extent (n / 8)
    const int32_t *bmap;  // brick grid -> global brick id, or -1
};

// the levels a deposit writes (caller's layout)
struct DepArgs {
    DepLevel lev[MAX_AMR];
    double *rho[MAX_AMR];
    int64_t ncell[MAX_AMR];
    int nlev;
};

struct GatherArgs {
    DepLevel lev[MAX_AMR];
    int nlev;
    const double *E[3 * MAX_AMR];
};

// the small bottom levels of one problem, handled by one workgroup
struct CoarseJob {
    int nlev;
    int b0[8];
    int nb[8];
    int cg_off;
    int direct;  // 1: the coarsest grid is solved by the transform kernels instead
};

// coarsest grid solved directly by its separable eigendecomposition: one box
// of dn cells (each at most DIRECT_DIM), bricks x-fastest from b0
struct DirectJob {
    int b0;
    int dn[3];
    int tab;  // offset of its tables (direct_tables layout) in the table pool
    int w;    // offset of its FP64 scratch (n doubles, x fastest)
    int amr;  // 1 when the grid is an AMR level (phi += e after the solve)
    int pad;
};
constexpr int DIRECT_DIM = 128;
// columns per workgroup of the transform along z
constexpr int DIRECT_COLS = 16;

hipError_t upload_cf_weights(const double *w);
// window masks of patterns 0..12 and (u0, v0, nodes) of patterns 0..13
hipError_t upload_pattern_tables(const uint32_t *masks13, const int *org14x3);
// Device build of the brick tables (org, nbr, child, par, cmask, ubase, ustr,
// gf_owner, reflux list, AMR brick list) from the box table; the per-level
// counts (cf0, ncf, rf0, nrf), composite cell counts and totals (nbc, ncf,
// reflux length, nesting error) reach the host through hout / hdof
// (host-visible), followed by seq at hseq.
struct MetaBuild {
    int nbrick, nbox, nent;
    int64_t npool;
    const BoxDev *boxes;
    const EntryDev *ent;
    int32_t *pool;  // [npool] brick maps of all levels
    int4 *org;
    int64_t *ubase;
    int2 *ustr;
    int32_t *child, *par, *nbr, *gf_owner, *reflux, *amr_list;
    uint8_t *cmask;
    uint64_t *cnt, *off;      // [nbrick + 1]
    uint32_t *flag, *roff;    // [nbrick + 1]
    unsigned long long *dof;  // [nent]
    int *err;
    void *temp;
    size_t temp_bytes;
    int32_t *hout;  // [4 nent + 4]
    int64_t *hdof;  // [nent]
    unsigned *hseq;
    unsigned seq;
};
// exclusive prefix sums out[i] = in[0] + ... + in[i-1] of n values (two
// launches, amrmg_scan.hip); temp: scan_temp_bytes<V>(n) bytes of device
// memory; in and out must not overlap
template <class V>
size_t scan_temp_bytes(int64_t n);
template <class V>
hipError_t exclusive_scan(hipStream_t st, const V *in, V *out, int64_t n, void *temp, size_t temp_bytes);
size_t meta_scan_temp_bytes(int nbrick);
hipError_t launch_meta_build(hipStream_t st, const MetaBuild &B);
// Dirichlet values of the boundary faces (gbc) and the coarse-fine windows
// (cf_pat, cf_idx) of the hierarchy in M; *err is set when a window leaves
// the coarser level
void launch_face_data(hipStream_t st, const DevMeta &M, const EntryDev *ent, const int32_t *pool,
                      const double *mono, double *gbc, uint8_t *cf_pat, int32_t *cf_idx, int *err);
// the next kernel launched by a launcher records kernel-execution timestamps
// into these events (hipExtLaunchKernelGGL); cleared after that launch
void set_launch_timing(hipEvent_t start, hipEvent_t stop);
bool launch_timing_pending();

// Fine sums ffs: per fine brick F, face f and coarse cell m of that face,
// ffs[(F * 6 + f) * 16 + m] = sum over the four fine cells next to the face of
// (u_f/3 + u_in/5 - coarse part of the ghost), written for coarse-fine faces.

// phib, rhob: FP64 phi and rho in brick layout; ffs: fine sums of phib
template <class T>
void launch_outer_residual(hipStream_t st, const DevMeta &M, int b0, int nb, const int32_t *list, const double *phib,
                           const double *rhob, double inv_eps0, const double *cp_phi, T *r_out, double *part,
                           int norm_p, bool zero_phi, double *const *r_user, const double *ffs);
// caller's layout (per-level pointer tables a, bu) <-> brick layout (ab, bb)
void launch_user_brick(hipStream_t st, const DevMeta &M, int b0, int nb, const int32_t *list, bool to_brick,
                       double *const *a, double *ab, double *const *bu, double *bb);
// per-range norms into out (device); with hout, also into host-visible
// memory (at hout + alt when *counter is odd) followed by the sequence number
// *counter + 1 at hseq
void launch_level_norms(hipStream_t st, const int2 *ranges, int n, const double *part, double *out, int norm_p,
                        double *hout = nullptr, int alt = 0, unsigned *hseq = nullptr, unsigned *counter = nullptr);
// coarse parts cp of the ghosts of coarse-fine faces [cf0, cf0 + ncf) from
// the coarse values src; with ffs, also the fine sums from the fine values
template <class T>
void launch_cpart_brick(hipStream_t st, const DevMeta &M, int cf0, int ncf, const T *src, T *cp,
                        const T *fine = nullptr, double *ffs = nullptr);
// fine sums of e (zero coarse parts) of coarse-fine faces [cf0, cf0 + ncf)
template <class T>
void launch_face_sums(hipStream_t st, const DevMeta &M, int cf0, int ncf, const T *e, double *ffs);
template <class T>
void launch_gsrb(hipStream_t st, const DevMeta &M, int b0, int nb, T *e, const T *r, const T *cp, int colour,
                 bool init);
template <class T>
void launch_jacobi(hipStream_t st, const DevMeta &M, int b0, int nb, const T *ein, T *eout, const T *r, const T *cp,
                   double omega, bool init);
// restriction of nb fine bricks from b0 (r -> parents' covered cells) and the
// coarse-fine update of the nrf listed coarse bricks (from the fine sums of
// e), in one launch
template <class T>
void launch_restrict(hipStream_t st, const DevMeta &M, int b0, int nb, const int32_t *rlist, int nrf, const T *e,
                     T *r, const double *ffs);
template <class T>
void launch_prolong(hipStream_t st, const DevMeta &M, int b0, int nb, T *e);
template <class T>
void launch_phi_update(hipStream_t st, const DevMeta &M, int b0, int nb, const int32_t *list, double *phib,
                       const T *e);
void launch_avgdown(hipStream_t st, const DevMeta &M, int b0, int nb, double *phib);
void launch_efield(hipStream_t st, const DevMeta &M, int b0, int nb, const int32_t *list, const double *phib,
                   const double *cp_phi, double *const *E);
template <class T>
void launch_bottom_cg(hipStream_t st, const DevMeta &M, const int4 *jobs, int njobs, const T *rhs, T *e,
                      double *work, double rtol, int maxit, int *iters);
template <class T>
void launch_copy(hipStream_t st, const T *a, T *b, int64_t n);
// brick-hybrid Gauss-Seidel sweep; mode = bits of HG_ZERO 1, HG_PROL 2, HG_CPIN 4, HG_PHI 8,
// HG_FFS 16 (fine sums of the result into ffs)
// one wavefront per brick; nt: threads per workgroup (64, 128 or 256, i.e.
// 1, 2 or 4 bricks per workgroup), or 0 for the size rule hgs_rule_threads
int hgs_rule_threads(int nb);
template <class T>
void launch_hgs(hipStream_t st, const DevMeta &M, int b0, int nb, const T *ein, T *eout, const T *r, T *cp,
                double *phib, double *ffs, int mode, int nt = 0);
// direct solve e = A^-1 r of the coarsest grids of the listed jobs: planes
// (job, z | x-block << 8) for the x/y transforms, column groups (job, first
// column) for the z transform; FP64 scratch W; phi += e on AMR grids when
// phi_update.  one: the only job (host copy), when there is one; the lists
// are then implied by the launch shape.
template <class T>
void launch_direct(hipStream_t st, const DirectJob *jobs, const int2 *planes, int nplanes, const int2 *groups,
                   int ngroups, const double *tab, double *W, const T *r, T *e, double *phib, bool phi_update,
                   int maxdim, const DirectJob *one);
template <class T>
void launch_coarse_cycle(hipStream_t st, const DevMeta &M, const CoarseJob *jobs, int njobs, T *e, T *r,
                         double *work, int nu1, int nu2, double rtol, int maxit, int *iters, double *phib,
                         bool phi_update, int threads_hint);
// with xs != nullptr, also the particles in visiting order (the order perm
// gives; perm required): xs[i] = x[perm[i]], ... (the copy the ordered
// deposits read later, written while the particles pass anyway).
// big_tile: the larger LDS tile, for levels on which a visiting-order
// bucket spans 8 or more cells per axis
void launch_deposit(hipStream_t st, int pos_f32, int64_t n, const void *x, const void *y, const void *z,
                    const double *q, const uint32_t *perm, const DepArgs &A, const int64_t *ubase, const int2 *ustr,
                    unsigned long long *nout,
                    void *xs = nullptr, void *ys = nullptr, void *zs = nullptr, double *qs = nullptr,
                    bool big_tile = false);
void launch_zero_levels(hipStream_t st, const DepArgs &A);
// ordered: x, y, z are already in the order perm gives (x[i] is particle
// perm[i], the build's ordered copy); E is written at perm[i].  With perm,
// its inverse iperm and rec ([n] staging records), E goes to rec in the
// visiting order first and then to the caller's order by a second pass that
// reads rec through iperm (coalesced writes instead of scattered ones).
void launch_gather(hipStream_t st, int pos_f32, int64_t n, const void *x, const void *y, const void *z,
                   const uint32_t *perm, const uint32_t *iperm, const GatherArgs &G, const int64_t *ubase,
                   const int2 *ustr, double *Ex, double *Ey, double *Ez, double4 *rec, bool ordered = false);
void launch_tag(hipStream_t st, const double *v, int64_t n, double lambda, double *scratch, uint8_t *tags);
void launch_fill(hipStream_t st, double *v, int64_t n, double val);
// spatial visiting order of the particles (stable radix sort by the
// Morton code of their cell on a sort grid: the level-0 grid n0 refined
// towards about four particles per cell but at most levels times, at most
// 1024 cells per axis): perm [n] (perm[i] = the i-th particle visited) and
// its inverse iperm [n]; scratch: order_scratch_bytes(n) bytes of device
// memory
size_t order_scratch_bytes(int64_t n);
hipError_t particle_order(hipStream_t st, int pos_f32, int64_t n, const void *x, const void *y, const void *z,
                          const double *lo, const double *hi, const int *n0, int levels, void *scratch,
                          size_t scratch_bytes, uint32_t *perm, uint32_t *iperm);
// log2 of the edge of a sort cell in level-0 cells (negative: finer than level 0)
int order_cell_shift(const double *lo, const double *hi, const int *n0, int levels, int64_t n);
// the particles in the visiting order alone: xs[i] = x[perm[i]], ...
void launch_copy_ordered(hipStream_t st, int pos_f32, int64_t n, const uint32_t *perm, const void *x, const void *y,
                         const void *z, const double *q, void *xs, void *ys, void *zs, double *qs);
// proper nesting of the block marks of the finer level (g blocks per axis,
// total = their product) against the coarse level (index extent cn, brick
// map cbmap over cnbk bricks; half coarse cells per block edge, nesting by np
// cells), packed into bits [(total + 63) / 64] in linear block order
void launch_nest_pack(hipStream_t st, const uint8_t *marks, int64_t total, int3 g, const int32_t *cbmap, int3 cn,
                      int3 cnbk, int half, int np, uint64_t *bits);
void launch_mark_blocks(hipStream_t st, const double *rho, int64_t ncell, const int4 *borg, const int64_t *ubase,
                        const int2 *ustr, int nb, double lambda, int nbuf, int half, int3 n, int3 g, double *scratch,
                        uint8_t *marks);
// domain transform (amrmg_transform.hip): out (one word, zeroed by the
// caller) receives the bits of max_i max_d |x_d - c_d| / l_d (+inf for a NaN
// coordinate); xs = (x - c) / s (may alias x); v[i] = v[i] / div
void launch_domain_scale(hipStream_t st, int pos_f32, int64_t n, const void *x, const void *y, const void *z,
                         const double *c, const double *l, unsigned long long *out);
void launch_to_computation(hipStream_t st, int pos_f32, int64_t n, const void *x, const void *y, const void *z,
                           const double *c, double s, void *xs, void *ys, void *zs);
void launch_divide(hipStream_t st, double *v, int64_t n, double div);

}  // namespace amrmg
