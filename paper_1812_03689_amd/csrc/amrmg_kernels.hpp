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

struct GatherArgs {
    DepLevel lev[MAX_AMR];
    int nlev;
    const double *E[3 * MAX_AMR];
};

hipError_t upload_cf_weights(const double *w);

template <class T>
void launch_outer_residual(hipStream_t st, const DevMeta &M, int b0, int nb, const int32_t *list,
                           double *const *phi, double *const *rho, double inv_eps0, const double *cp_phi, T *r_out,
                           double *part, int norm_p, bool zero_phi, double *const *r_user = nullptr);
void launch_level_norms(hipStream_t st, const int2 *ranges, int n, const double *part, double *out, int norm_p);
void launch_cpart_user(hipStream_t st, const DevMeta &M, int cf0, int ncf, double *const *phi, double *cp);
template <class T>
void launch_cpart_brick(hipStream_t st, const DevMeta &M, int cf0, int ncf, const T *src, T *cp);
template <class T>
void launch_gsrb(hipStream_t st, const DevMeta &M, int b0, int nb, T *e, const T *r, const T *cp, int colour,
                 bool init);
template <class T>
void launch_jacobi(hipStream_t st, const DevMeta &M, int b0, int nb, const T *ein, T *eout, const T *r, const T *cp,
                   double omega, bool init);
template <class T>
void launch_restrict(hipStream_t st, const DevMeta &M, int b0, int nb, const T *e, const T *r, T *rc);
template <class T>
void launch_reflux(hipStream_t st, const DevMeta &M, const int32_t *list, int n, const T *e, T *r);
template <class T>
void launch_prolong(hipStream_t st, const DevMeta &M, int b0, int nb, T *e);
template <class T>
void launch_phi_update(hipStream_t st, const DevMeta &M, int b0, int nb, const int32_t *list, double *const *phi,
                       const T *e);
void launch_avgdown(hipStream_t st, const DevMeta &M, int b0, int nb, double *const *phi);
void launch_efield(hipStream_t st, const DevMeta &M, int b0, int nb, const int32_t *list, double *const *phi,
                   const double *cp_phi, double *const *E);
template <class T>
void launch_bottom_cg(hipStream_t st, const DevMeta &M, const int4 *jobs, int njobs, const T *rhs, T *e,
                      double *work, double rtol, int maxit, int *iters);
template <class T>
void launch_copy(hipStream_t st, const T *a, T *b, int64_t n);
void launch_deposit(hipStream_t st, int pos_f32, int64_t n, const void *x, const void *y, const void *z,
                    const double *q, const DepLevel &D, const int64_t *ubase, const int2 *ustr, double *rho,
                    unsigned long long *nout);
void launch_gather(hipStream_t st, int pos_f32, int64_t n, const void *x, const void *y, const void *z,
                   const GatherArgs &G, const int64_t *ubase, const int2 *ustr, double *Ex, double *Ey, double *Ez);
void launch_tag(hipStream_t st, const double *v, int64_t n, double lambda, double *scratch, uint8_t *tags);
void launch_fill(hipStream_t st, double *v, int64_t n, double val);

}  // namespace amrmg
