/*
 * amrmg_oracle.c -- plain, slow FP64 CPU oracle for the composite-grid AMR
 * multigrid Poisson path of Frey, Adelmann & Locans, "On Architecture and
 * Performance of Adaptive Mesh Refinement in an Electrostatics
 * Particle-In-Cell Code" (arXiv:1812.03689).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes, links
 * or calls this file; it shares no code, header or table with the HIP path.
 * Only the test-suite, the smoke check and the CPU-baseline leg of the bench
 * use it.
 *
 * Everything is written cell by cell, face by face, in double precision,
 * without blocking or fusion, so that each function can be checked against
 * the paper by eye.  Conventions:
 *   - cell-centred data; level l has spacing h^l = h^0 / 2^l (ratio 2,
 *     Sec. 3 "The AMReX Library", Eq. mesh_spacing);
 *   - a level is a list of disjoint boxes [lo, hi) in the level's own index
 *     space; its arrays concatenate the boxes in list order, each box stored
 *     x-fastest;
 *   - A := -L_h (the negative discrete Laplacian), b := rho / eps0, residual
 *     r = b - A phi (Sec. 5.3, Alg. 1 writes r = rho - A phi);
 *   - Dirichlet data g on the physical boundary enters through the linear
 *     ghost phi_g = 2 g - phi_in at the boundary face; with an artificial
 *     distance d > 0 the boundary is instead the open (Robin) condition
 *     d phi / dn + phi / d = 0 of Sec. 5.2 (Eq. robin_bc), discretised by
 *     central difference across the boundary face.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXL 10
#define OR_PI 3.14159265358979323846

typedef struct {
    int nb;
    int32_t *box;  /* [nb][6]: lo[3], hi[3] (exclusive) */
    int64_t *off;  /* [nb+1] */
    int n[3];      /* extent of the level index space */
    double h[3];
    int nbk[3];    /* n / 8 : block grid used for cell lookup */
    int32_t *bmap; /* block -> box id, or -1 */
} OLev;

typedef struct {
    int nlev;
    double lo[3], hi[3];
    double eps0;
    double robin; /* artificial distance d of the Robin boundary; 0 = Dirichlet */
    int nmono;
    double *mono; /* [nmono][4] q, x, y, z */
    OLev L[OR_MAXL];
} OHier;

/* ------------------------------------------------------------------------ */
/* hierarchy bookkeeping                                                     */
/* ------------------------------------------------------------------------ */

OHier *or_new(const double *lo, const double *hi, const int32_t *n0, double eps0,
              int nmono, const double *mono)
{
    OHier *H = (OHier *)calloc(1, sizeof(OHier));
    for (int d = 0; d < 3; ++d) {
        H->lo[d] = lo[d];
        H->hi[d] = hi[d];
        H->L[0].n[d] = n0[d];
    }
    H->eps0 = eps0;
    H->nmono = nmono;
    H->mono = (double *)malloc(sizeof(double) * 4 * (nmono > 0 ? nmono : 1));
    if (nmono > 0) memcpy(H->mono, mono, sizeof(double) * 4 * nmono);
    return H;
}

static void lev_clear(OLev *L)
{
    free(L->box);
    free(L->off);
    free(L->bmap);
    L->box = NULL;
    L->off = NULL;
    L->bmap = NULL;
    L->nb = 0;
}

void or_free(OHier *H)
{
    if (!H) return;
    for (int l = 0; l < OR_MAXL; ++l) lev_clear(&H->L[l]);
    free(H->mono);
    free(H);
}

/* Install the box list of level l (levels above l are dropped).  Boxes must be
 * multiples of 8 cells, lie in the level's index space and be disjoint.
 * Returns 0 on success, a negative code otherwise. */
int or_set_level(OHier *H, int l, int nb, const int32_t *boxes)
{
    if (l < 0 || l >= OR_MAXL) return -1;
    if (l > H->nlev) return -2;
    for (int m = l; m < OR_MAXL; ++m) lev_clear(&H->L[m]);
    OLev *L = &H->L[l];
    for (int d = 0; d < 3; ++d) {
        L->n[d] = H->L[0].n[d] << l;
        L->h[d] = (H->hi[d] - H->lo[d]) / L->n[d];
        L->nbk[d] = L->n[d] / 8;
    }
    L->nb = nb;
    L->box = (int32_t *)malloc(sizeof(int32_t) * 6 * (nb > 0 ? nb : 1));
    L->off = (int64_t *)malloc(sizeof(int64_t) * (nb + 1));
    size_t nbm = (size_t)L->nbk[0] * L->nbk[1] * L->nbk[2];
    L->bmap = (int32_t *)malloc(sizeof(int32_t) * nbm);
    for (size_t t = 0; t < nbm; ++t) L->bmap[t] = -1;
    L->off[0] = 0;
    for (int b = 0; b < nb; ++b) {
        const int32_t *B = boxes + 6 * b;
        int64_t vol = 1;
        for (int d = 0; d < 3; ++d) {
            if (B[d] < 0 || B[3 + d] > L->n[d] || B[d] >= B[3 + d]) return -3;
            if (B[d] % 8 || B[3 + d] % 8) return -4;
            vol *= B[3 + d] - B[d];
            L->box[6 * b + d] = B[d];
            L->box[6 * b + 3 + d] = B[3 + d];
        }
        L->off[b + 1] = L->off[b] + vol;
        for (int k = B[2] / 8; k < B[5] / 8; ++k)
            for (int j = B[1] / 8; j < B[4] / 8; ++j)
                for (int i = B[0] / 8; i < B[3] / 8; ++i) {
                    size_t t = (size_t)i + (size_t)L->nbk[0] * (j + (size_t)L->nbk[1] * k);
                    if (L->bmap[t] >= 0) return -5; /* overlap */
                    L->bmap[t] = b;
                }
    }
    H->nlev = l + 1;
    return 0;
}

int or_nlev(const OHier *H) { return H->nlev; }
int or_nboxes(const OHier *H, int l) { return H->L[l].nb; }
int64_t or_ncells(const OHier *H, int l) { return H->L[l].off[H->L[l].nb]; }

void or_get_boxes(const OHier *H, int l, int32_t *boxes, int64_t *off)
{
    const OLev *L = &H->L[l];
    memcpy(boxes, L->box, sizeof(int32_t) * 6 * L->nb);
    memcpy(off, L->off, sizeof(int64_t) * (L->nb + 1));
}

/* arena index of cell (i,j,k) of a level, or -1 when the cell is not part of
 * the level (outside every box or outside the index space) */
static int64_t cidx(const OLev *L, int i, int j, int k)
{
    if (i < 0 || j < 0 || k < 0 || i >= L->n[0] || j >= L->n[1] || k >= L->n[2]) return -1;
    int32_t b = L->bmap[(size_t)(i / 8) + (size_t)L->nbk[0] * ((size_t)(j / 8) + (size_t)L->nbk[1] * (k / 8))];
    if (b < 0) return -1;
    const int32_t *B = L->box + 6 * b;
    int64_t nx = B[3] - B[0], ny = B[4] - B[1];
    return L->off[b] + (i - B[0]) + nx * ((j - B[1]) + ny * (k - B[2]));
}

int64_t or_cell_index(const OHier *H, int l, int i, int j, int k) { return cidx(&H->L[l], i, j, k); }

/* switch the physical boundary to the Robin condition with distance d (d <= 0:
 * back to Dirichlet) */
void or_set_robin(OHier *H, double d) { H->robin = d > 0.0 ? d : 0.0; }

/* cell (i,j,k) of level l is covered when level l+1 holds its children */
static int covered(const OHier *H, int l, int i, int j, int k)
{
    if (l + 1 >= H->nlev) return 0;
    return cidx(&H->L[l + 1], 2 * i, 2 * j, 2 * k) >= 0;
}

/* visit every cell of level l in arena order: box b, level indices (i,j,k),
 * arena index c.  The innermost one-pass loop only declares c. */
#define FOR_CELLS(L, b, i, j, k, c)                                           \
    for (int b = 0; b < (L)->nb; ++b)                                         \
        for (int k = (L)->box[6 * b + 2]; k < (L)->box[6 * b + 5]; ++k)       \
            for (int j = (L)->box[6 * b + 1]; j < (L)->box[6 * b + 4]; ++j)   \
                for (int i = (L)->box[6 * b + 0]; i < (L)->box[6 * b + 3]; ++i) \
                    for (int64_t c = cidx((L), i, j, k), c##_once = 1; c##_once; c##_once = 0)

/* ------------------------------------------------------------------------ */
/* physical boundary data                                                    */
/* ------------------------------------------------------------------------ */

/* Dirichlet value at a point: superposition of point charges,
 * g(x) = sum_k q_k / (4 pi eps0 |x - x_k|)  (zero when there are none) */
static double bc_point(const OHier *H, const double x[3])
{
    double g = 0.0;
    for (int m = 0; m < H->nmono; ++m) {
        const double *M = H->mono + 4 * m;
        double dx = x[0] - M[1], dy = x[1] - M[2], dz = x[2] - M[3];
        g += M[0] / (4.0 * OR_PI * H->eps0 * sqrt(dx * dx + dy * dy + dz * dz));
    }
    return g;
}

/* g at the centre of face (d, s) of cell (i,j,k) of level l */
static double bc_face(const OHier *H, int l, int i, int j, int k, int d, int s)
{
    const OLev *L = &H->L[l];
    int c[3] = {i, j, k};
    double x[3];
    for (int e = 0; e < 3; ++e) x[e] = H->lo[e] + (c[e] + 0.5) * L->h[e];
    x[d] += 0.5 * s * L->h[d];
    return bc_point(H, x);
}

/* ------------------------------------------------------------------------ */
/* coarse-fine ghost interpolation (Sec. 5.1, Eq. 2d_lagrange, Fig. 5,       */
/* Tab. bit_pattern and the linear table that follows it)                    */
/* ------------------------------------------------------------------------ */

/* The nine quadratic windows as printed: bit (i + 5 j) of a 5x5 layer around
 * the coarse cell at the interface, i along the first transverse axis u, j
 * along the second v, centre at (2,2).  Order = the order of selection. */
static const uint32_t QPAT[9] = {473536u, 14798u, 236768u, 15153152u, 947072u,
                                 29596u, 7399u, 7576576u, 30306304u};
/* The four bilinear windows: bit (i + 3 j) of the inner 3x3 layer. */
static const uint32_t LPAT[4] = {27u, 216u, 432u, 54u};

/* transverse axes of an interface with normal d: the two other axes in
 * increasing order (the paper draws a z-normal interface in the xy-plane) */
static void transverse(int d, int *du, int *dv)
{
    *du = (d == 0) ? 1 : 0;
    *dv = (d == 2) ? 1 : 2;
}

/* 5x5 availability mask of the coarse layer through coarse cell C:
 * a bit is set when that coarse cell belongs to level lc and is not covered
 * by level lc+1 */
static uint32_t mask5(const OHier *H, int lc, const int C[3], int d)
{
    int du, dv;
    transverse(d, &du, &dv);
    uint32_t m = 0;
    for (int jv = 0; jv < 5; ++jv)
        for (int iu = 0; iu < 5; ++iu) {
            int p[3] = {C[0], C[1], C[2]};
            p[du] += iu - 2;
            p[dv] += jv - 2;
            if (cidx(&H->L[lc], p[0], p[1], p[2]) >= 0 && !covered(H, lc, p[0], p[1], p[2]))
                m |= 1u << (iu + 5 * jv);
        }
    (void)d;
    return m;
}

static uint32_t mask3_of_mask5(uint32_t m5)
{
    uint32_t m3 = 0;
    for (int j = 0; j < 3; ++j)
        for (int i = 0; i < 3; ++i)
            if (m5 & (1u << ((i + 1) + 5 * (j + 1)))) m3 |= 1u << (i + 3 * j);
    return m3;
}

/* pattern id: 0..8 quadratic (first match in the printed order), 9..12
 * bilinear, 13 = only the centre is usable */
static int select_pattern(uint32_t m5)
{
    for (int k = 0; k < 9; ++k)
        if ((m5 & QPAT[k]) == QPAT[k]) return k;
    uint32_t m3 = mask3_of_mask5(m5);
    for (int k = 0; k < 4; ++k)
        if ((m3 & LPAT[k]) == LPAT[k]) return 9 + k;
    return 13;
}

/* Lagrange basis polynomial for node a of the node set {n0, .., n0+np-1},
 * evaluated at t (Eq. 2d_lagrange, L_i) */
static double lagrange(int a, int n0, int np, double t)
{
    double v = 1.0;
    for (int m = n0; m < n0 + np; ++m)
        if (m != a) v *= (t - m) / (double)(a - m);
    return v;
}

/* Step 1 of the two-step interpolation on a 5x5 layer given as values
 * layer[iu + 5 jv] (centre at (2,2)) with availability mask m5: the value at
 * transverse offset (tu, tv) (in coarse cells, +-1/4) from the centre, using
 * the window that select_pattern picks.  The window's nodes are read off the
 * pattern bits themselves. */
static double step1_layer(uint32_t m5, const double *layer, double tu, double tv, int *pat_out)
{
    int pat = select_pattern(m5);
    if (pat_out) *pat_out = pat;
    int u0 = 5, v0 = 5, np;
    if (pat < 9) {
        uint32_t P = QPAT[pat];
        for (int b = 0; b < 25; ++b)
            if (P & (1u << b)) {
                if (b % 5 - 2 < u0) u0 = b % 5 - 2;
                if (b / 5 - 2 < v0) v0 = b / 5 - 2;
            }
        np = 3;
    } else if (pat < 13) {
        uint32_t P = LPAT[pat - 9];
        for (int b = 0; b < 9; ++b)
            if (P & (1u << b)) {
                if (b % 3 - 1 < u0) u0 = b % 3 - 1;
                if (b / 3 - 1 < v0) v0 = b / 3 - 1;
            }
        np = 2;
    } else {
        return layer[2 + 5 * 2];
    }
    double val = 0.0;
    for (int b = v0; b < v0 + np; ++b)
        for (int a = u0; a < u0 + np; ++a)
            val += lagrange(a, u0, np, tu) * lagrange(b, v0, np, tv) * layer[(a + 2) + 5 * (b + 2)];
    return val;
}

double or_step1_layer(uint32_t m5, const double *layer, double tu, double tv, int *pat_out)
{
    return step1_layer(m5, layer, tu, tv, pat_out);
}

/* step 1 for the coarse layer of level lc through coarse cell C, normal d */
static double cf_step1(const OHier *H, int lc, const int C[3], int d, double tu, double tv,
                       const double *uc, int *pat_out)
{
    int du, dv;
    transverse(d, &du, &dv);
    uint32_t m5 = mask5(H, lc, C, d);
    double layer[25];
    for (int jv = 0; jv < 5; ++jv)
        for (int iu = 0; iu < 5; ++iu) {
            int p[3] = {C[0], C[1], C[2]};
            p[du] += iu - 2;
            p[dv] += jv - 2;
            layer[iu + 5 * jv] = (m5 & (1u << (iu + 5 * jv))) ? uc[cidx(&H->L[lc], p[0], p[1], p[2])] : 0.0;
        }
    return step1_layer(m5, layer, tu, tv, pat_out);
}

/* Value that cell (i,j,k) of level l sees across its face (d, s):
 *   - outside the domain: linear Dirichlet ghost 2 g - u_c (g = 0 unless inhom),
 *     or for the Robin condition the ghost u_g that makes the central
 *     difference (u_g - u_c)/h + (u_g + u_c)/(2 dist) vanish;
 *   - a cell of the same level: its value (covered or not);
 *   - otherwise (l > 0) a coarse-fine ghost: step 1 in the coarse layer
 *     (uc == NULL means the coarse values are zero), step 2 a quadratic along
 *     the normal through the two fine cells inside (-3/2 h, -1/2 h from the
 *     face) and the step-1 point at the coarse centre (+h), evaluated at the
 *     ghost centre (+h/2). */
static double nbval(const OHier *H, int l, int i, int j, int k, int d, int s,
                    const double *ul, const double *uc, int inhom)
{
    const OLev *L = &H->L[l];
    int c[3] = {i, j, k};
    int p[3] = {i, j, k};
    p[d] += s;
    int64_t ic = cidx(L, i, j, k);
    if (p[d] < 0 || p[d] >= L->n[d]) {
        if (H->robin > 0.0) {
            double h = L->h[d], dist = H->robin;
            /* u_g (1/h + 1/(2 dist)) = u_c (1/h - 1/(2 dist)) */
            return ul[ic] * (1.0 / h - 1.0 / (2.0 * dist)) / (1.0 / h + 1.0 / (2.0 * dist));
        }
        double g = inhom ? bc_face(H, l, i, j, k, d, s) : 0.0;
        return 2.0 * g - ul[ic];
    }
    int64_t ip = cidx(L, p[0], p[1], p[2]);
    if (ip >= 0) return ul[ip];
    /* fine side of a coarse-fine interface */
    int in[3] = {c[0], c[1], c[2]};
    in[d] -= s;
    int64_t iin = cidx(L, in[0], in[1], in[2]);
    double P = 0.0;
    if (uc) {
        int du, dv;
        transverse(d, &du, &dv);
        int C[3] = {p[0] >> 1, p[1] >> 1, p[2] >> 1};
        double tu = (p[du] & 1) ? 0.25 : -0.25;
        double tv = (p[dv] & 1) ? 0.25 : -0.25;
        P = cf_step1(H, l - 1, C, d, tu, tv, uc, NULL);
    }
    /* Lagrange weights of the nodes (-3/2, -1/2, +1) fine spacings from the
     * face, evaluated at the ghost centre +1/2 */
    const double xs[3] = {-1.5, -0.5, 1.0};
    double wl[3];
    for (int a = 0; a < 3; ++a) {
        double v = 1.0;
        for (int m = 0; m < 3; ++m)
            if (m != a) v *= (0.5 - xs[m]) / (xs[a] - xs[m]);
        wl[a] = v;
    }
    return wl[0] * ul[iin] + wl[1] * ul[ic] + wl[2] * P;
}

/* pattern id used for the ghost across face (d,s) of fine cell (i,j,k) of
 * level l (l > 0), and the 5x5 mask it was chosen from; -1 if that face is
 * not a coarse-fine face */
int or_cf_pattern(const OHier *H, int l, int i, int j, int k, int d, int s, uint32_t *mask_out)
{
    const OLev *L = &H->L[l];
    int p[3] = {i, j, k};
    p[d] += s;
    if (l == 0 || cidx(L, i, j, k) < 0) return -1;
    if (p[d] < 0 || p[d] >= L->n[d]) return -1;
    if (cidx(L, p[0], p[1], p[2]) >= 0) return -1;
    int C[3] = {p[0] >> 1, p[1] >> 1, p[2] >> 1};
    uint32_t m5 = mask5(H, l - 1, C, d);
    if (mask_out) *mask_out = m5;
    return select_pattern(m5);
}

int or_select_pattern(uint32_t m5) { return select_pattern(m5); }

/* ------------------------------------------------------------------------ */
/* operators (Sec. 5.1 Eqs. lap_flux_differencing, coarse_fluxes,            */
/* flux_differencing)                                                        */
/* ------------------------------------------------------------------------ */

/* (A u)_c for cell (i,j,k) of level l, A = -L:
 *   sum over faces of -(1/h_d) * (outward gradient through the face),
 * the outward gradient being (u_nb - u_c)/h_d with u_nb from nbval, except
 * when composite != 0 and the same-level neighbour is covered by level l+1:
 * then it is the mean of the four fine outward gradients (u_f - u_ghost)/h_f
 * through the fine faces that make up the coarse face.
 * u[l-1], u[l], u[l+1] are the level arrays; ucoarse is the array used for
 * the coarse part of this level's own coarse-fine ghosts (NULL = zero). */
static double apply_cell(const OHier *H, int l, int i, int j, int k, double *const *u,
                         const double *ucoarse, int composite, int inhom)
{
    const OLev *L = &H->L[l];
    const double *ul = u[l];
    int64_t ic = cidx(L, i, j, k);
    double acc = 0.0;
    for (int d = 0; d < 3; ++d)
        for (int s = -1; s <= 1; s += 2) {
            int p[3] = {i, j, k};
            p[d] += s;
            int in_lev = (p[d] >= 0 && p[d] < L->n[d]) && cidx(L, p[0], p[1], p[2]) >= 0;
            if (composite && in_lev && covered(H, l, p[0], p[1], p[2])) {
                const OLev *F = &H->L[l + 1];
                int du, dv;
                transverse(d, &du, &dv);
                double G = 0.0;
                for (int b = 0; b < 2; ++b)
                    for (int a = 0; a < 2; ++a) {
                        int f[3];
                        f[d] = (s > 0) ? 2 * p[d] : 2 * p[d] + 1;
                        f[du] = 2 * p[du] + a;
                        f[dv] = 2 * p[dv] + b;
                        double uf = u[l + 1][cidx(F, f[0], f[1], f[2])];
                        double ug = nbval(H, l + 1, f[0], f[1], f[2], d, -s, u[l + 1], ul, inhom);
                        G += (uf - ug) / F->h[d];
                    }
                G *= 0.25;
                acc += -G / L->h[d];
            } else {
                double v = nbval(H, l, i, j, k, d, s, ul, ucoarse, inhom);
                acc += (ul[ic] - v) / (L->h[d] * L->h[d]);
            }
        }
    return acc;
}

/* diagonal of the no-finer-level operator with homogeneous data: the
 * coefficient of u_c in (A u)_c, face by face (1 - g)/h^2 where g u_c is the
 * part of the value across the face that depends on u_c (nbval):
 *   - a same-level neighbour: g = 0;
 *   - a coarse-fine ghost: g = 2/3, the weight of the cell itself in step 2;
 *   - the physical boundary: g = -1 for the Dirichlet ghost 2 g - u_c, or
 *     g = (1/h - 1/(2 d)) / (1/h + 1/(2 d)) for the Robin ghost. */
static double diag_nf(const OHier *H, int l, int i, int j, int k)
{
    const OLev *L = &H->L[l];
    double a = 0.0;
    for (int d = 0; d < 3; ++d)
        for (int s = -1; s <= 1; s += 2) {
            int p[3] = {i, j, k};
            p[d] += s;
            double h = L->h[d], h2 = h * h, g;
            if (p[d] < 0 || p[d] >= L->n[d]) {
                if (H->robin > 0.0) {
                    double dist = H->robin;
                    g = (1.0 / h - 1.0 / (2.0 * dist)) / (1.0 / h + 1.0 / (2.0 * dist));
                } else {
                    g = -1.0;
                }
            } else if (cidx(L, p[0], p[1], p[2]) >= 0) {
                g = 0.0;
            } else {
                g = 2.0 / 3.0;
            }
            a += (1.0 - g) / h2;
        }
    return a;
}

/* out[l] = A_comp phi on uncovered cells (0 on covered), for every level.
 * inhom selects whether the Dirichlet data g enter. */
void or_apply_composite(const OHier *H, double *const *phi, double *const *out, int inhom)
{
    for (int l = 0; l < H->nlev; ++l) {
        const OLev *L = &H->L[l];
        FOR_CELLS(L, b, i, j, k, c) {
            out[l][c] = covered(H, l, i, j, k)
                            ? 0.0
                            : apply_cell(H, l, i, j, k, phi, l > 0 ? phi[l - 1] : NULL, 1, inhom);
        }
    }
}

/* out = A_nf^l u^l with coarse-fine ghosts from ucoarse (NULL = 0), every cell */
void or_apply_nf(const OHier *H, int l, double *const *u, const double *ucoarse, double *out, int inhom)
{
    const OLev *L = &H->L[l];
    FOR_CELLS(L, b, i, j, k, c) { out[c] = apply_cell(H, l, i, j, k, u, ucoarse, 0, inhom); }
}

/* ------------------------------------------------------------------------ */
/* Alg. 1 (Residual) and helpers                                             */
/* ------------------------------------------------------------------------ */

typedef struct {
    OHier *H;
    int lmax;
    double **phi, **b, **r, **e, **phis, **de, **tmp;
    int nu1, nu2;
    double bottom_rtol;
    int bottom_iters;
} OCtx;

/* Alg. 1: on the finest level r = b - A_nf phi - B_crse phi^{l-1}; below it
 * r = U (b - A_comp phi - B_crse phi^{l-1} - B_fine phi^{l+1}) */
static void residual(OCtx *X, int l)
{
    OHier *H = X->H;
    const OLev *L = &H->L[l];
    FOR_CELLS(L, b, i, j, k, c) {
        if (l < X->lmax && covered(H, l, i, j, k)) {
            X->r[l][c] = 0.0;
        } else {
            X->r[l][c] = X->b[l][c] - apply_cell(H, l, i, j, k, X->phi, l > 0 ? X->phi[l - 1] : NULL,
                                                 l < X->lmax, 1);
        }
    }
}

/* Gauss-Seidel update of one cell of A_nf^l e = r (zero coarse data,
 * homogeneous boundary data): with every other value fixed, the cell's value
 * that makes its own residual vanish (Sec. 5.3, the smoothing of Alg. 3) */
static void relax_point(const OHier *H, int l, int i, int j, int k, double *e, const double *r)
{
    double *u[OR_MAXL] = {0};
    u[l] = e;
    int64_t c = cidx(&H->L[l], i, j, k);
    double Ae = apply_cell(H, l, i, j, k, u, NULL, 0, 0);
    e[c] += (r[c] - Ae) / diag_nf(H, l, i, j, k);
}

void or_relax_point(const OHier *H, int l, int i, int j, int k, double *e, const double *r)
{
    if (cidx(&H->L[l], i, j, k) >= 0) relax_point(H, l, i, j, k, e, r);
}

/* Gauss-Seidel red-black on A_nf^l e = r with zero coarse data and homogeneous
 * boundary data; colour (i+j+k) mod 2 in level indices, even colour first */
static void smooth(OCtx *X, int l, double *e, const double *r, int sweeps)
{
    OHier *H = X->H;
    const OLev *L = &H->L[l];
    for (int it = 0; it < sweeps; ++it)
        for (int colour = 0; colour < 2; ++colour) {
            FOR_CELLS(L, b, i, j, k, c) {
                if (((i + j + k) & 1) != colour) continue;
                relax_point(H, l, i, j, k, e, r);
            }
        }
}

/* CG on A_nf^0 x = rhs with homogeneous Dirichlet data, x0 = 0 */
static int bottom_cg(OCtx *X, double *x, const double *rhs)
{
    OHier *H = X->H;
    const OLev *L = &H->L[0];
    int64_t n = L->off[L->nb];
    double *rr = (double *)malloc(sizeof(double) * n);
    double *p = (double *)malloc(sizeof(double) * n);
    double *q = (double *)malloc(sizeof(double) * n);
    double *u[OR_MAXL] = {0};
    for (int64_t t = 0; t < n; ++t) {
        x[t] = 0.0;
        rr[t] = rhs[t];
        p[t] = rhs[t];
    }
    double rho = 0.0;
    for (int64_t t = 0; t < n; ++t) rho += rr[t] * rr[t];
    double r0 = sqrt(rho);
    int it = 0;
    while (it < 100000 && sqrt(rho) > X->bottom_rtol * r0 && rho > 0.0) {
        u[0] = p;
        or_apply_nf(H, 0, u, NULL, q, 0);
        double pq = 0.0;
        for (int64_t t = 0; t < n; ++t) pq += p[t] * q[t];
        double alpha = rho / pq;
        double rho1 = 0.0;
        for (int64_t t = 0; t < n; ++t) {
            x[t] += alpha * p[t];
            rr[t] -= alpha * q[t];
            rho1 += rr[t] * rr[t];
        }
        double beta = rho1 / rho;
        for (int64_t t = 0; t < n; ++t) p[t] = rr[t] + beta * p[t];
        rho = rho1;
        ++it;
    }
    free(rr);
    free(p);
    free(q);
    return it;
}

/* Alg. 3 (Relax), the residual-correction V-cycle.  Readings:
 *   - the correction e^l starts from zero before the pre-smoothing;
 *   - the prolongation adds to e^l (e^l <- e^l + I e^{l-1});
 *   - the uncovered part of the restricted residual is the composite residual
 *     with the updated phi^l, the covered part keeps the restricted value;
 *   - R is the mean of the 8 children, I injects the parent value. */
static void relax(OCtx *X, int l)
{
    OHier *H = X->H;
    if (l == X->lmax) {
        const OLev *L = &H->L[l];
        FOR_CELLS(L, b, i, j, k, c) {
            X->r[l][c] = X->b[l][c] - apply_cell(H, l, i, j, k, X->phi, l > 0 ? X->phi[l - 1] : NULL, 0, 1);
        }
    }
    if (l > 0) {
        const OLev *L = &H->L[l];
        const OLev *Lc = &H->L[l - 1];
        int64_t n = L->off[L->nb], nc = Lc->off[Lc->nb];
        double *u[OR_MAXL] = {0};
        memcpy(X->phis[l], X->phi[l], sizeof(double) * n);
        for (int64_t t = 0; t < nc; ++t) X->e[l - 1][t] = 0.0;
        for (int64_t t = 0; t < n; ++t) X->e[l][t] = 0.0;
        smooth(X, l, X->e[l], X->r[l], X->nu1);
        for (int64_t t = 0; t < n; ++t) X->phi[l][t] += X->e[l][t];
        /* restrict r^l - A_nf e^l - B_crse e^{l-1} (e^{l-1} = 0) onto covered cells */
        u[l] = X->e[l];
        or_apply_nf(H, l, u, X->e[l - 1], X->tmp[l], 0);
        FOR_CELLS(Lc, b, i, j, k, c) {
            if (covered(H, l - 1, i, j, k)) {
                double s = 0.0;
                for (int dz = 0; dz < 2; ++dz)
                    for (int dy = 0; dy < 2; ++dy)
                        for (int dx = 0; dx < 2; ++dx) {
                            int64_t f = cidx(L, 2 * i + dx, 2 * j + dy, 2 * k + dz);
                            s += X->r[l][f] - X->tmp[l][f];
                        }
                X->r[l - 1][c] = s / 8.0;
            } else {
                X->r[l - 1][c] = X->b[l - 1][c] - apply_cell(H, l - 1, i, j, k, X->phi,
                                                             l - 1 > 0 ? X->phi[l - 2] : NULL, 1, 1);
            }
        }
        relax(X, l - 1);
        /* e^l <- e^l + I e^{l-1} */
        FOR_CELLS(L, b, i, j, k, c) { X->e[l][c] += X->e[l - 1][cidx(Lc, i >> 1, j >> 1, k >> 1)]; }
        /* r^l <- r^l - A_nf e^l - B_crse e^{l-1} */
        u[l] = X->e[l];
        or_apply_nf(H, l, u, X->e[l - 1], X->tmp[l], 0);
        for (int64_t t = 0; t < n; ++t) X->r[l][t] -= X->tmp[l][t];
        for (int64_t t = 0; t < n; ++t) X->de[l][t] = 0.0;
        smooth(X, l, X->de[l], X->r[l], X->nu2);
        for (int64_t t = 0; t < n; ++t) {
            X->e[l][t] += X->de[l][t];
            X->phi[l][t] = X->phis[l][t] + X->e[l][t];
        }
    } else {
        const OLev *L = &H->L[0];
        int64_t n = L->off[L->nb];
        X->bottom_iters += bottom_cg(X, X->e[0], X->r[0]);
        for (int64_t t = 0; t < n; ++t) X->phi[0][t] += X->e[0][t];
    }
}

static double level_norm(const double *v, int64_t n, int p)
{
    double s = 0.0;
    for (int64_t t = 0; t < n; ++t) {
        double a = fabs(v[t]);
        if (p == 1) s += a;
        else if (p == 2) s += a * a;
        else if (a > s) s = a;
    }
    return p == 2 ? sqrt(s) : s;
}

/* Alg. 2 average down: phi^l <- U phi^l + R phi^{l+1}, finest to coarsest */
void or_average_down(const OHier *H, double *const *phi)
{
    for (int l = H->nlev - 2; l >= 0; --l) {
        const OLev *L = &H->L[l];
        const OLev *F = &H->L[l + 1];
        FOR_CELLS(L, b, i, j, k, c) {
            if (!covered(H, l, i, j, k)) continue;
            double s = 0.0;
            for (int dz = 0; dz < 2; ++dz)
                for (int dy = 0; dy < 2; ++dy)
                    for (int dx = 0; dx < 2; ++dx) s += phi[l + 1][cidx(F, 2 * i + dx, 2 * j + dy, 2 * k + dz)];
            phi[l][c] = s / 8.0;
        }
    }
}

/* Alg. 2 field evaluation: E_d = -(u_+ - u_-) / (2 h_d) on every cell of every
 * level, the neighbour values taken as in the operator (same level, coarse-fine
 * ghost from the coarser potential, or the Dirichlet ghost).
 * E is laid out as E[3*l + d]. */
void or_efield(const OHier *H, double *const *phi, double *const *E)
{
    for (int l = 0; l < H->nlev; ++l) {
        const OLev *L = &H->L[l];
        const double *uc = l > 0 ? phi[l - 1] : NULL;
        FOR_CELLS(L, b, i, j, k, c) {
            for (int d = 0; d < 3; ++d) {
                double up = nbval(H, l, i, j, k, d, +1, phi[l], uc, 1);
                double um = nbval(H, l, i, j, k, d, -1, phi[l], uc, 1);
                E[3 * l + d][c] = -(up - um) / (2.0 * L->h[d]);
            }
        }
    }
}

typedef struct {
    int iters;
    int bottom_iters;
    int converged;
    double rel[OR_MAXL]; /* final ||r^l|| / ||b^l|| */
} OStats;

/* residual norms; returns 1 when every level meets tol */
static int converged_all(OCtx *X, const double *bn, int p, double tol, double *rel)
{
    int ok = 1;
    for (int l = 0; l <= X->lmax; ++l) {
        const OLev *L = &X->H->L[l];
        double rn = level_norm(X->r[l], L->off[L->nb], p);
        rel[l] = bn[l] > 0 ? rn / bn[l] : rn;
        if (rn > tol * bn[l]) ok = 0;
    }
    return ok;
}

/* Alg. 2 (Solve).  rho and phi are per-level arrays (phi holds the initial
 * guess); E may be NULL.  Stopping rule: stop when for every level
 * ||r^l||_p <= tol * ||b^l||_p, where b^l is the uncovered right-hand side
 * including the Dirichlet data (the composite residual of phi = 0); a level
 * whose b^l vanishes uses the norm over all levels instead. */
int or_solve(OHier *H, double *const *rho, double *const *phi, double *const *E, double tol,
             int max_iters, int nu1, int nu2, int norm_p, double bottom_rtol, OStats *st)
{
    OCtx X;
    memset(&X, 0, sizeof(X));
    X.H = H;
    X.lmax = H->nlev - 1;
    X.nu1 = nu1;
    X.nu2 = nu2;
    X.bottom_rtol = bottom_rtol;
    int L = H->nlev;
    double *zero[OR_MAXL] = {0};
    X.phi = zero;
    X.b = (double **)calloc(OR_MAXL, sizeof(double *));
    X.r = (double **)calloc(OR_MAXL, sizeof(double *));
    X.e = (double **)calloc(OR_MAXL, sizeof(double *));
    X.phis = (double **)calloc(OR_MAXL, sizeof(double *));
    X.de = (double **)calloc(OR_MAXL, sizeof(double *));
    X.tmp = (double **)calloc(OR_MAXL, sizeof(double *));
    for (int l = 0; l < L; ++l) {
        int64_t n = or_ncells(H, l);
        zero[l] = (double *)calloc(n, sizeof(double));
        X.b[l] = (double *)malloc(sizeof(double) * n);
        for (int64_t t = 0; t < n; ++t) X.b[l][t] = rho[l][t] / H->eps0;
        X.r[l] = (double *)calloc(n, sizeof(double));
        X.e[l] = (double *)calloc(n, sizeof(double));
        X.phis[l] = (double *)calloc(n, sizeof(double));
        X.de[l] = (double *)calloc(n, sizeof(double));
        X.tmp[l] = (double *)calloc(n, sizeof(double));
    }
    /* ||b^l||: the composite residual with phi = 0 */
    double bn[OR_MAXL], rel[OR_MAXL];
    {
        for (int l = 0; l < L; ++l) residual(&X, l);
        double tot = 0.0;
        for (int l = 0; l < L; ++l) {
            bn[l] = level_norm(X.r[l], or_ncells(H, l), norm_p);
            if (norm_p == 2) tot += bn[l] * bn[l];
            else if (norm_p == 1) tot += bn[l];
            else if (bn[l] > tot) tot = bn[l];
        }
        if (norm_p == 2) tot = sqrt(tot);
        for (int l = 0; l < L; ++l)
            if (bn[l] == 0.0) bn[l] = tot;
        for (int l = 0; l < L; ++l) free(zero[l]);
        X.phi = (double **)phi;
    }
    for (int l = 0; l < L; ++l) residual(&X, l);
    int it = 0;
    int ok = converged_all(&X, bn, norm_p, tol, rel);
    while (it < max_iters && !ok) {
        relax(&X, X.lmax);
        for (int l = 0; l < L; ++l) residual(&X, l);
        ++it;
        ok = converged_all(&X, bn, norm_p, tol, rel);
    }
    or_average_down(H, phi);
    if (E) or_efield(H, phi, E);
    if (st) {
        st->iters = it;
        st->bottom_iters = X.bottom_iters;
        st->converged = ok;
        for (int l = 0; l < L; ++l) st->rel[l] = rel[l];
    }
    for (int l = 0; l < L; ++l) {
        free(X.b[l]);
        free(X.r[l]);
        free(X.e[l]);
        free(X.phis[l]);
        free(X.de[l]);
        free(X.tmp[l]);
    }
    free(X.b);
    free(X.r);
    free(X.e);
    free(X.phis);
    free(X.de);
    free(X.tmp);
    return ok ? 0 : 1;
}

/* Alg. 1 on every level for given rho, phi: r[l] (0 on covered cells) */
void or_residual(OHier *H, double *const *rho, double *const *phi, double *const *r)
{
    OCtx X;
    memset(&X, 0, sizeof(X));
    X.H = H;
    X.lmax = H->nlev - 1;
    double *bb[OR_MAXL] = {0};
    for (int l = 0; l < H->nlev; ++l) {
        int64_t n = or_ncells(H, l);
        bb[l] = (double *)malloc(sizeof(double) * n);
        for (int64_t t = 0; t < n; ++t) bb[l][t] = rho[l][t] / H->eps0;
    }
    X.b = bb;
    X.phi = (double **)phi;
    X.r = (double **)r;
    for (int l = 0; l < H->nlev; ++l) residual(&X, l);
    for (int l = 0; l < H->nlev; ++l) free(bb[l]);
}

/* ------------------------------------------------------------------------ */
/* particles: cloud-in-cell deposit and gather, tagging, clustering          */
/* ------------------------------------------------------------------------ */

/* CIC stencil of position x on level l: lower cells i0[d] and weights of the
 * upper cell f[d]; indices are clamped to the index space, so weight that
 * would land outside the domain stays in the boundary cell.  Returns 0 when
 * x lies outside [lo, hi). */
static int cic(const OHier *H, int l, const double x[3], int i0[3], int i1[3], double f[3])
{
    const OLev *L = &H->L[l];
    for (int d = 0; d < 3; ++d) {
        if (!(x[d] >= H->lo[d] && x[d] < H->hi[d])) return 0;
        double s = (x[d] - H->lo[d]) / L->h[d] - 0.5;
        double fl = floor(s);
        int a = (int)fl;
        f[d] = s - fl;
        int b = a + 1;
        if (a < 0) a = 0;
        if (b < 0) b = 0;
        if (a > L->n[d] - 1) a = L->n[d] - 1;
        if (b > L->n[d] - 1) b = L->n[d] - 1;
        i0[d] = a;
        i1[d] = b;
    }
    return 1;
}

/* rho^l += sum_p q_p W(x_p - x_i) / (h_x h_y h_z); stencil cells outside the
 * level's boxes receive nothing.  Returns the number of particles outside
 * the domain. */
int64_t or_deposit(const OHier *H, int l, int64_t n, const double *x, const double *y, const double *z,
                   const double *q, double *rho)
{
    const OLev *L = &H->L[l];
    double vol = L->h[0] * L->h[1] * L->h[2];
    int64_t outside = 0;
    for (int64_t p = 0; p < n; ++p) {
        double X3[3] = {x[p], y[p], z[p]};
        int i0[3], i1[3];
        double f[3];
        if (!cic(H, l, X3, i0, i1, f)) {
            ++outside;
            continue;
        }
        for (int c = 0; c < 8; ++c) {
            int ii = (c & 1) ? i1[0] : i0[0];
            int jj = (c & 2) ? i1[1] : i0[1];
            int kk = (c & 4) ? i1[2] : i0[2];
            double w = ((c & 1) ? f[0] : 1.0 - f[0]) * ((c & 2) ? f[1] : 1.0 - f[1]) *
                       ((c & 4) ? f[2] : 1.0 - f[2]);
            int64_t t = cidx(L, ii, jj, kk);
            if (t >= 0) rho[t] += q[p] * w / vol;
        }
    }
    return outside;
}

/* E at particle positions: interpolate with the same CIC weights on the
 * finest level whose boxes hold all 8 stencil cells (level 0 always does).
 * E is laid out as E[3*l + d].  Particles outside the domain get 0. */
int64_t or_gather(const OHier *H, int64_t n, const double *x, const double *y, const double *z,
                  double *const *E, double *Ex, double *Ey, double *Ez)
{
    int64_t outside = 0;
    for (int64_t p = 0; p < n; ++p) {
        double X3[3] = {x[p], y[p], z[p]};
        Ex[p] = Ey[p] = Ez[p] = 0.0;
        for (int l = H->nlev - 1; l >= 0; --l) {
            const OLev *L = &H->L[l];
            int i0[3], i1[3];
            double f[3];
            if (!cic(H, l, X3, i0, i1, f)) {
                ++outside;
                break;
            }
            int64_t t[8];
            int ok = 1;
            for (int c = 0; c < 8; ++c) {
                t[c] = cidx(L, (c & 1) ? i1[0] : i0[0], (c & 2) ? i1[1] : i0[1], (c & 4) ? i1[2] : i0[2]);
                if (t[c] < 0) ok = 0;
            }
            if (!ok) continue;
            double e[3] = {0, 0, 0};
            for (int c = 0; c < 8; ++c) {
                double w = ((c & 1) ? f[0] : 1.0 - f[0]) * ((c & 2) ? f[1] : 1.0 - f[1]) *
                           ((c & 4) ? f[2] : 1.0 - f[2]);
                for (int d = 0; d < 3; ++d) e[d] += w * E[3 * l + d][t[c]];
            }
            Ex[p] = e[0];
            Ey[p] = e[1];
            Ez[p] = e[2];
            break;
        }
    }
    return outside;
}

/* charge tagging (Sec. 4.2, Eq. tag_charge, in the relative form of the
 * potential and field policies): tag when |rho| > lambda * max |rho^l| */
void or_tag(const OHier *H, int l, const double *rho, double lambda, uint8_t *tags)
{
    int64_t n = or_ncells(H, l);
    double m = 0.0;
    for (int64_t t = 0; t < n; ++t)
        if (fabs(rho[t]) > m) m = fabs(rho[t]);
    for (int64_t t = 0; t < n; ++t) tags[t] = fabs(rho[t]) > lambda * m ? 1 : 0;
}

/* Boxes of level l+1 from the tags of level l.  The paper leaves the box
 * generation to its AMR library; this is a fixed integer procedure:
 *   1. dilate the tags by n_buffer cells (all 26 directions), inside the domain;
 *   2. a block of bf fine cells (bf/2 coarse cells) per direction is tagged
 *      when it holds a dilated tag;
 *   3. a block is kept only when its coarse footprint grown by n_proper cells
 *      (clipped to the domain) lies inside level l;
 *   4. scanning blocks with z slowest and x fastest, an untaken tagged block
 *      starts a box that grows along +x, then +y (whole rows), then +z (whole
 *      slabs) while every block it would add is tagged and untaken and the
 *      edge stays <= max_grid_size cells;
 *   5. boxes are emitted in creation order.
 * Returns the number of boxes written to out (or -1 if more than max_out). */
int or_cluster(const OHier *H, int l, const uint8_t *tags, int n_buffer, int n_proper, int bf, int mgs,
               int32_t *out, int max_out)
{
    const OLev *L = &H->L[l];
    int nf[3], nbk[3];
    for (int d = 0; d < 3; ++d) {
        nf[d] = 2 * L->n[d];
        nbk[d] = nf[d] / bf;
    }
    size_t nblk = (size_t)nbk[0] * nbk[1] * nbk[2];
    uint8_t *tb = (uint8_t *)calloc(nblk, 1);
    uint8_t *taken = (uint8_t *)calloc(nblk, 1);
    FOR_CELLS(L, b, i, j, k, c) {
        if (!tags[c]) continue;
        for (int oz = -n_buffer; oz <= n_buffer; ++oz)
            for (int oy = -n_buffer; oy <= n_buffer; ++oy)
                for (int ox = -n_buffer; ox <= n_buffer; ++ox) {
                    int q[3] = {i + ox, j + oy, k + oz};
                    if (q[0] < 0 || q[1] < 0 || q[2] < 0 || q[0] >= L->n[0] || q[1] >= L->n[1] ||
                        q[2] >= L->n[2])
                        continue;
                    int bx = 2 * q[0] / bf, by = 2 * q[1] / bf, bz = 2 * q[2] / bf;
                    tb[(size_t)bx + (size_t)nbk[0] * (by + (size_t)nbk[1] * bz)] = 1;
                }
    }
    int half = bf / 2;
    for (int bz = 0; bz < nbk[2]; ++bz)
        for (int by = 0; by < nbk[1]; ++by)
            for (int bx = 0; bx < nbk[0]; ++bx) {
                size_t t = (size_t)bx + (size_t)nbk[0] * (by + (size_t)nbk[1] * bz);
                if (!tb[t]) continue;
                int bb[3] = {bx, by, bz};
                int lo[3], hi[3];
                for (int d = 0; d < 3; ++d) {
                    lo[d] = bb[d] * half - n_proper;
                    hi[d] = (bb[d] + 1) * half + n_proper;
                    if (lo[d] < 0) lo[d] = 0;
                    if (hi[d] > L->n[d]) hi[d] = L->n[d];
                }
                int ok = 1;
                for (int k = lo[2]; k < hi[2] && ok; ++k)
                    for (int j = lo[1]; j < hi[1] && ok; ++j)
                        for (int i = lo[0]; i < hi[0] && ok; ++i)
                            if (cidx(L, i, j, k) < 0) ok = 0;
                if (!ok) tb[t] = 0;
            }
    int maxb = mgs / bf;
    int nout = 0;
#define BLK(x, y, z) ((size_t)(x) + (size_t)nbk[0] * ((y) + (size_t)nbk[1] * (z)))
#define FREE_BLK(x, y, z) (tb[BLK(x, y, z)] && !taken[BLK(x, y, z)])
    for (int bz = 0; bz < nbk[2]; ++bz)
        for (int by = 0; by < nbk[1]; ++by)
            for (int bx = 0; bx < nbk[0]; ++bx) {
                if (!FREE_BLK(bx, by, bz)) continue;
                int lx = 1, ly = 1, lz = 1;
                while (bx + lx < nbk[0] && lx + 1 <= maxb && FREE_BLK(bx + lx, by, bz)) ++lx;
                for (;;) {
                    if (by + ly >= nbk[1] || ly + 1 > maxb) break;
                    int ok = 1;
                    for (int x = bx; x < bx + lx; ++x)
                        if (!FREE_BLK(x, by + ly, bz)) ok = 0;
                    if (!ok) break;
                    ++ly;
                }
                for (;;) {
                    if (bz + lz >= nbk[2] || lz + 1 > maxb) break;
                    int ok = 1;
                    for (int y = by; y < by + ly; ++y)
                        for (int x = bx; x < bx + lx; ++x)
                            if (!FREE_BLK(x, y, bz + lz)) ok = 0;
                    if (!ok) break;
                    ++lz;
                }
                for (int z = bz; z < bz + lz; ++z)
                    for (int y = by; y < by + ly; ++y)
                        for (int x = bx; x < bx + lx; ++x) taken[BLK(x, y, z)] = 1;
                if (nout >= max_out) {
                    free(tb);
                    free(taken);
                    return -1;
                }
                int32_t *o = out + 6 * nout;
                o[0] = bx * bf;
                o[1] = by * bf;
                o[2] = bz * bf;
                o[3] = (bx + lx) * bf;
                o[4] = (by + ly) * bf;
                o[5] = (bz + lz) * bf;
                ++nout;
            }
#undef FREE_BLK
#undef BLK
    free(tb);
    free(taken);
    return nout;
}
