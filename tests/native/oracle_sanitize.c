/* Sanitizer driver for the oracle (oracle/amrmg_oracle.c), built with
 * -fsanitize=address,undefined by tests/test_sanitizers.py: one pass through
 * every exported function on small hierarchies (a Gaussian bunch tagged and
 * clustered into two refined levels with Dirichlet monopole data, then the
 * same boxes with the Robin boundary), so that an out-of-bounds access, a
 * leak or undefined behaviour anywhere in the oracle aborts the run.
 * Test infrastructure only; links the oracle and nothing of the product. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int iters, bottom_iters, converged;
    double rel[10];
} OStats;

void *or_new(const double *lo, const double *hi, const int32_t *n0, double eps0, int nmono, const double *mono);
void or_free(void *H);
int or_set_level(void *H, int l, int nb, const int32_t *boxes);
int or_nlev(const void *H);
int or_nboxes(const void *H, int l);
int64_t or_ncells(const void *H, int l);
void or_get_boxes(const void *H, int l, int32_t *boxes, int64_t *off);
int64_t or_cell_index(const void *H, int l, int i, int j, int k);
void or_set_robin(void *H, double d);
int or_cf_pattern(const void *H, int l, int i, int j, int k, int d, int s, uint32_t *mask_out);
void or_apply_composite(const void *H, double *const *phi, double *const *out, int inhom);
void or_apply_nf(const void *H, int l, double *const *u, const double *ucoarse, double *out, int inhom);
void or_relax_point(const void *H, int l, int i, int j, int k, double *e, const double *r);
void or_average_down(const void *H, double *const *phi);
void or_efield(const void *H, double *const *phi, double *const *E);
int or_solve(void *H, double *const *rho, double *const *phi, double *const *E, double tol, int max_iters, int nu1,
             int nu2, int norm_p, double bottom_rtol, OStats *st);
void or_residual(void *H, double *const *rho, double *const *phi, double *const *r);
int64_t or_deposit(const void *H, int l, int64_t n, const double *x, const double *y, const double *z,
                   const double *q, double *rho);
int64_t or_gather(const void *H, int64_t n, const double *x, const double *y, const double *z, double *const *E,
                  double *Ex, double *Ey, double *Ez);
void or_tag(const void *H, int l, const double *rho, double lambda, uint8_t *tags);
int or_cluster(const void *H, int l, const uint8_t *tags, int n_buffer, int n_proper, int bf, int mgs, int32_t *out,
               int max_out);

static uint64_t rng = 88172645463325252ull;
static double unif(void)
{
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (double)(rng >> 11) * (1.0 / 9007199254740992.0);
}
static double gauss(void)
{
    double u = unif() + 1e-300, v = unif();
    return sqrt(-2.0 * log(u)) * cos(6.283185307179586 * v);
}

/* one full pass over hierarchy H with boxes already set */
static int exercise(void *H, int64_t n, const double *x, const double *y, const double *z, const double *q)
{
    int L = or_nlev(H);
    double *rho[10] = {0}, *phi[10] = {0}, *r[10] = {0}, *E[30] = {0};
    for (int l = 0; l < L; ++l) {
        int64_t c = or_ncells(H, l);
        rho[l] = calloc(c, sizeof(double));
        phi[l] = calloc(c, sizeof(double));
        r[l] = calloc(c, sizeof(double));
        for (int d = 0; d < 3; ++d) E[3 * l + d] = calloc(c, sizeof(double));
        if (or_deposit(H, l, n, x, y, z, q, rho[l]) != 1) return 1; /* one particle planted outside */
    }
    OStats st;
    or_solve(H, rho, phi, E, 1e-9, 30, 2, 4, 2, 1e-10, &st);
    if (!st.converged) return 2;
    or_residual(H, rho, phi, r);
    or_apply_composite(H, phi, r, 1);
    or_average_down(H, phi);
    or_efield(H, phi, E);
    for (int l = 0; l < L; ++l) {
        or_apply_nf(H, l, phi, l > 0 ? phi[l - 1] : NULL, r[l], 0);
        if (or_nboxes(H, l) < 1) return 3;
    }
    double *Ex = malloc(n * sizeof(double)), *Ey = malloc(n * sizeof(double)), *Ez = malloc(n * sizeof(double));
    if (or_gather(H, n, x, y, z, E, Ex, Ey, Ez) != 1) return 4;
    /* patterns and point relaxation on every cell of the finest level's first box */
    int32_t *bx = malloc(sizeof(int32_t) * 6 * or_nboxes(H, L - 1));
    int64_t *of = malloc(sizeof(int64_t) * (or_nboxes(H, L - 1) + 1));
    or_get_boxes(H, L - 1, bx, of);
    for (int k = bx[2]; k < bx[5]; ++k)
        for (int j = bx[1]; j < bx[4]; ++j)
            for (int i = bx[0]; i < bx[3]; ++i) {
                for (int d = 0; d < 3; ++d)
                    for (int s = -1; s <= 1; s += 2) {
                        uint32_t m = 0;
                        (void)or_cf_pattern(H, L - 1, i, j, k, d, s, &m);
                    }
                or_relax_point(H, L - 1, i, j, k, phi[L - 1], rho[L - 1]);
                if (or_cell_index(H, L - 1, i, j, k) < 0) return 5;
            }
    free(bx);
    free(of);
    free(Ex);
    free(Ey);
    free(Ez);
    for (int l = 0; l < L; ++l) {
        free(rho[l]);
        free(phi[l]);
        free(r[l]);
        for (int d = 0; d < 3; ++d) free(E[3 * l + d]);
    }
    return 0;
}

int main(void)
{
    const int64_t n = 20001;
    double *x = malloc(n * 8), *y = malloc(n * 8), *z = malloc(n * 8), *q = malloc(n * 8);
    for (int64_t p = 0; p < n; ++p) {
        x[p] = 0.5 + 0.07 * gauss();
        y[p] = 0.45 + 0.06 * gauss();
        z[p] = 0.55 + 0.09 * gauss();
        q[p] = 1.0 / n;
        if (x[p] < 0 || x[p] >= 1 || y[p] < 0 || y[p] >= 1 || z[p] < 0 || z[p] >= 1) x[p] = y[p] = z[p] = 0.5;
    }
    x[n - 1] = 1.5; /* outside the domain */
    const double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1}, mono[4] = {1.0, 0.5, 0.45, 0.55};
    const int32_t n0[3] = {16, 24, 16};
    void *H = or_new(lo, hi, n0, 1.0, 1, mono);
    const int32_t box0[6] = {0, 0, 0, 16, 24, 16};
    if (or_set_level(H, 0, 1, box0) != 0) return 9;
    /* tag and cluster two levels */
    for (int l = 0; l < 2; ++l) {
        int64_t c = or_ncells(H, l);
        double *rho = calloc(c, sizeof(double));
        uint8_t *tags = calloc(c, 1);
        (void)or_deposit(H, l, n, x, y, z, q, rho);
        or_tag(H, l, rho, 1e-2, tags);
        int32_t out[6 * 4096];
        int nb = or_cluster(H, l, tags, 1, 2, 8, 16, out, 4096);
        free(rho);
        free(tags);
        if (nb <= 0) return 10 + l;
        if (or_set_level(H, l + 1, nb, out) != 0) return 20 + l;
    }
    int rc = exercise(H, n, x, y, z, q);
    if (rc) return 30 + rc;
    /* the same hierarchy with the Robin boundary */
    or_set_robin(H, 0.4);
    rc = exercise(H, n, x, y, z, q);
    if (rc) return 40 + rc;
    or_free(H);
    free(x);
    free(y);
    free(z);
    free(q);
    printf("oracle sanitize ok\n");
    return 0;
}
