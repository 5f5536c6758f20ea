/*
 * Plain FP64 CPU oracle for the multigrid pressure solve of
 * Shin, Chergui & Juric, "A solver for massively parallel direct numerical
 * simulation of three-dimensional multiphase flows" (arXiv:1410.8568), Sec. 2.3.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is loaded by the tests, by the smoke
 * check and by the benchmark's CPU-baseline leg; the product (the HIP library)
 * never links, loads or calls it, and the two share no code.
 *
 * What it computes.  For face coefficients beta > 0 on every interior face and
 * homogeneous Neumann walls, the unique mean-zero p with
 *     L p = b - mean(b),   (L p)_c = sum_{6 faces f} beta_f (p_nb - p_c)
 * i.e. eq. (10) in three dimensions with the h^2 folded into b, beta the face
 * values of alpha = 1/rho (eq. 9).  It gets there with the modified V-cycle the
 * paper describes (features 1-6), step by step and unoptimised:
 *   - coarse operators rediscretised from face averages (R and P not transposes),
 *   - restriction by linear interpolation of the residual (8-child mean),
 *   - flux-conserving prolongation of the error (eqs. 13-14 as flux continuity),
 *   - red-black Gauss-Seidel (SOR with omega = 1) smoothing,
 *   - an exact dense solve on the coarsest grid (the limit of the paper's GMRES),
 *   - the average reduction rate gamma of eq. (15).
 * The FP32-refined mode runs the same V-cycle in float inside an FP64
 * residual/update loop, with the coarsest solve in FP64.
 *
 * Reductions are deterministic (fixed blocks, serial combine), so results do not
 * depend on the OpenMP thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#pragma GCC diagnostic ignored "-Wunused-function"

#define OG_MAX_LEVELS 24

/* Dense factor of the coarsest operator: B = -L + (sigma/n) 1 1^T, sigma = mean diagonal. */
typedef struct {
    int n;
    double *chol; /* lower Cholesky factor of B, row-major n x n */
} coarse_t;

/*
 * Paper-faithful variants of the cycle; the defaults (omega 1, 8-child
 * restriction, exact coarsest solve) give the standard cycle.
 */
typedef struct {
    double omega;          /* SOR factor of the red-black smoother (feature 5); 1 = Gauss-Seidel */
    int restrict64;        /* 1: 64-point restriction (transpose of trilinear interpolation) */
    int gmres_m;           /* > 0: the coarsest grid by restarted GMRES(m) (feature 6) */
    double gmres_tol;      /* GMRES: relative residual reduction on the coarsest grid */
    int gmres_maxit;       /* GMRES: iteration cap */
    const void *coarsest;  /* the coarsest FP64 level (its faces), for GMRES */
} variant_t;

#define R double
#define SFX _d
#include "mg_ops.inc"
#undef R
#undef SFX

#define R float
#define SFX _f
#include "mg_ops.inc"
#undef R
#undef SFX

/* ------------------------------------------------------------------------- */
/* Level planning                                                              */
/* ------------------------------------------------------------------------- */

/*
 * Grids are halved while every dimension is even and the largest exceeds
 * n_coarsest (the paper's hierarchy I_n = 2^(Ng-n), generalised to even sizes).
 * Returns the number of levels; dims receives 3 ints per level.
 */
int og_plan(int nx, int ny, int nz, int n_coarsest, int *dims)
{
    int d[3] = {nx, ny, nz};
    int L = 0;
    for (;;) {
        dims[3 * L + 0] = d[0];
        dims[3 * L + 1] = d[1];
        dims[3 * L + 2] = d[2];
        L++;
        if (L == OG_MAX_LEVELS) break;
        int mx = d[0] > d[1] ? d[0] : d[1];
        mx = mx > d[2] ? mx : d[2];
        if ((d[0] & 1) || (d[1] & 1) || (d[2] & 1) || mx <= n_coarsest) break;
        d[0] /= 2;
        d[1] /= 2;
        d[2] /= 2;
    }
    return L;
}

/* ------------------------------------------------------------------------- */
/* Setup: copy faces with zero walls, coarsen, cell weights                    */
/* ------------------------------------------------------------------------- */

static size_t ncell(int nx, int ny, int nz) { return (size_t)nx * ny * nz; }
static size_t nfx(int nx, int ny, int nz) { return (size_t)(nx + 1) * ny * nz; }
static size_t nfy(int nx, int ny, int nz) { return (size_t)nx * (ny + 1) * nz; }
static size_t nfz(int nx, int ny, int nz) { return (size_t)nx * ny * (nz + 1); }

/* Copy caller faces into L, forcing wall faces to 0 (homogeneous Neumann). */
static void copy_faces_zero_walls(level_d *L, const double *bx, const double *by, const double *bz)
{
    int nx = L->nx, ny = L->ny, nz = L->nz;
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i <= nx; i++)
                L->bx[FXI(L, i, j, k)] = (i == 0 || i == nx) ? 0.0 : bx[FXI(L, i, j, k)];
    for (int k = 0; k < nz; k++)
        for (int j = 0; j <= ny; j++)
            for (int i = 0; i < nx; i++)
                L->by[FYI(L, i, j, k)] = (j == 0 || j == ny) ? 0.0 : by[FYI(L, i, j, k)];
    for (int k = 0; k <= nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++)
                L->bz[FZI(L, i, j, k)] = (k == 0 || k == nz) ? 0.0 : bz[FZI(L, i, j, k)];
}

/*
 * Coarse faces: a coarse face covers 2 x 2 fine faces of the same orientation
 * (the fine faces at the same position m = 2I); its coefficient is their mean
 * (four parallel conductances).  Summation order ((f00 + f10) + (f01 + f11)) / 4,
 * the first index along the first tangential axis.  Fine wall faces are 0, so
 * coarse wall faces are 0.
 */
static void coarsen_faces(const level_d *F, level_d *C)
{
    for (int K = 0; K < C->nz; K++)
        for (int J = 0; J < C->ny; J++)
            for (int I = 0; I <= C->nx; I++) {
                double s0 = F->bx[FXI(F, 2 * I, 2 * J, 2 * K)] + F->bx[FXI(F, 2 * I, 2 * J + 1, 2 * K)];
                double s1 = F->bx[FXI(F, 2 * I, 2 * J, 2 * K + 1)] + F->bx[FXI(F, 2 * I, 2 * J + 1, 2 * K + 1)];
                C->bx[FXI(C, I, J, K)] = 0.25 * (s0 + s1);
            }
    for (int K = 0; K < C->nz; K++)
        for (int J = 0; J <= C->ny; J++)
            for (int I = 0; I < C->nx; I++) {
                double s0 = F->by[FYI(F, 2 * I, 2 * J, 2 * K)] + F->by[FYI(F, 2 * I + 1, 2 * J, 2 * K)];
                double s1 = F->by[FYI(F, 2 * I, 2 * J, 2 * K + 1)] + F->by[FYI(F, 2 * I + 1, 2 * J, 2 * K + 1)];
                C->by[FYI(C, I, J, K)] = 0.25 * (s0 + s1);
            }
    for (int K = 0; K <= C->nz; K++)
        for (int J = 0; J < C->ny; J++)
            for (int I = 0; I < C->nx; I++) {
                double s0 = F->bz[FZI(F, 2 * I, 2 * J, 2 * K)] + F->bz[FZI(F, 2 * I + 1, 2 * J, 2 * K)];
                double s1 = F->bz[FZI(F, 2 * I, 2 * J + 1, 2 * K)] + F->bz[FZI(F, 2 * I + 1, 2 * J + 1, 2 * K)];
                C->bz[FZI(C, I, J, K)] = 0.25 * (s0 + s1);
            }
}

/*
 * Cell weight for the flux-weighted prolongation: the cell's own coefficient
 * alpha is not kept on coarse grids, so it is estimated as the mean of beta over
 * the cell's interior faces (3 to 6 of them), in the order x-, x+, y-, y+, z-, z+.
 */
static void cell_weights(level_d *L)
{
    for (int k = 0; k < L->nz; k++)
        for (int j = 0; j < L->ny; j++)
            for (int i = 0; i < L->nx; i++) {
                double s = 0;
                int cnt = 0;
                if (i > 0) { s += L->bx[FXI(L, i, j, k)]; cnt++; }
                if (i < L->nx - 1) { s += L->bx[FXI(L, i + 1, j, k)]; cnt++; }
                if (j > 0) { s += L->by[FYI(L, i, j, k)]; cnt++; }
                if (j < L->ny - 1) { s += L->by[FYI(L, i, j + 1, k)]; cnt++; }
                if (k > 0) { s += L->bz[FZI(L, i, j, k)]; cnt++; }
                if (k < L->nz - 1) { s += L->bz[FZI(L, i, j, k + 1)]; cnt++; }
                L->a[CELL(L, i, j, k)] = cnt ? s / cnt : 1.0;
            }
}

/* ------------------------------------------------------------------------- */
/* Coarsest level: dense exact solve                                           */
/* ------------------------------------------------------------------------- */

/*
 * Assemble B = -L + (sigma/n) 1 1^T (SPD when the grid is connected with
 * beta > 0) and factor it.  For rhs r: B x = -(r - mean r) gives 1^T x = 0 and
 * L x = r - mean r, the exact mean-zero solution the paper's GMRES approximates.
 */
static int coarse_setup(const level_d *L, coarse_t *C)
{
    int n = (int)ncell(L->nx, L->ny, L->nz);
    double *B = (double *)calloc((size_t)n * n, sizeof(double));
    if (!B) return -1;
    for (int k = 0; k < L->nz; k++)
        for (int j = 0; j < L->ny; j++)
            for (int i = 0; i < L->nx; i++) {
                int c = (int)CELL(L, i, j, k);
                int nb[6];
                double w[6];
                int m = 0;
                if (i > 0) { nb[m] = (int)CELL(L, i - 1, j, k); w[m++] = L->bx[FXI(L, i, j, k)]; }
                if (i < L->nx - 1) { nb[m] = (int)CELL(L, i + 1, j, k); w[m++] = L->bx[FXI(L, i + 1, j, k)]; }
                if (j > 0) { nb[m] = (int)CELL(L, i, j - 1, k); w[m++] = L->by[FYI(L, i, j, k)]; }
                if (j < L->ny - 1) { nb[m] = (int)CELL(L, i, j + 1, k); w[m++] = L->by[FYI(L, i, j + 1, k)]; }
                if (k > 0) { nb[m] = (int)CELL(L, i, j, k - 1); w[m++] = L->bz[FZI(L, i, j, k)]; }
                if (k < L->nz - 1) { nb[m] = (int)CELL(L, i, j, k + 1); w[m++] = L->bz[FZI(L, i, j, k + 1)]; }
                for (int t = 0; t < m; t++) {
                    B[(size_t)c * n + c] += w[t];
                    B[(size_t)c * n + nb[t]] -= w[t];
                }
            }
    double sigma = 0;
    for (int c = 0; c < n; c++) sigma += B[(size_t)c * n + c];
    sigma /= n;
    for (size_t t = 0; t < (size_t)n * n; t++) B[t] += sigma / n;
    /* Cholesky B = G G^T, G lower, stored in place */
    for (int c = 0; c < n; c++) {
        for (int r = c; r < n; r++) {
            double s = B[(size_t)r * n + c];
            for (int t = 0; t < c; t++) s -= B[(size_t)r * n + t] * B[(size_t)c * n + t];
            if (r == c) {
                if (!(s > 0)) { free(B); return -2; }
                B[(size_t)c * n + c] = sqrt(s);
            } else {
                B[(size_t)r * n + c] = s / B[(size_t)c * n + c];
            }
        }
    }
    C->n = n;
    C->chol = B;
    return 0;
}

static void coarse_exact(const coarse_t *C, const double *rhs, double *e)
{
    int n = C->n;
    const double *G = C->chol;
    double mean = 0;
    for (int t = 0; t < n; t++) mean += rhs[t];
    mean /= n;
    double *y = (double *)malloc(sizeof(double) * n);
    for (int r = 0; r < n; r++) { /* G y = -(rhs - mean) */
        double s = -(rhs[r] - mean);
        for (int t = 0; t < r; t++) s -= G[(size_t)r * n + t] * y[t];
        y[r] = s / G[(size_t)r * n + r];
    }
    for (int r = n - 1; r >= 0; r--) { /* G^T e = y */
        double s = y[r];
        for (int t = r + 1; t < n; t++) s -= G[(size_t)t * n + r] * e[t];
        e[r] = s / G[(size_t)r * n + r];
    }
    free(y);
}

/* ------------------------------------------------------------------------- */
/* Hierarchy                                                                   */
/* ------------------------------------------------------------------------- */

typedef struct {
    int nlev;
    level_d d[OG_MAX_LEVELS];
    level_f f[OG_MAX_LEVELS];
    int have_f;
    coarse_t C;
} hier_t;

static void hier_free(hier_t *H)
{
    for (int l = 0; l < H->nlev; l++) {
        level_d *L = &H->d[l];
        free(L->bx); free(L->by); free(L->bz); free(L->a);
        if (l > 0) free(L->e);
        if (l > 0) free(L->rhs);
        free(L->r);
        if (H->have_f) {
            level_f *M = &H->f[l];
            free(M->bx); free(M->by); free(M->bz); free(M->a);
            free(M->e); free(M->rhs); free(M->r);
        }
    }
    free(H->C.chol);
}

/* Build levels 0..nlev-1 (faces, weights, scratch) and the coarsest factor. */
static int hier_build(hier_t *H, int nx, int ny, int nz, const double *bx, const double *by,
                      const double *bz, int n_coarsest, int want_float)
{
    int dims[3 * OG_MAX_LEVELS];
    memset(H, 0, sizeof(*H));
    H->nlev = og_plan(nx, ny, nz, n_coarsest, dims);
    for (int l = 0; l < H->nlev; l++) {
        level_d *L = &H->d[l];
        L->nx = dims[3 * l]; L->ny = dims[3 * l + 1]; L->nz = dims[3 * l + 2];
        L->bx = (double *)calloc(nfx(L->nx, L->ny, L->nz), sizeof(double));
        L->by = (double *)calloc(nfy(L->nx, L->ny, L->nz), sizeof(double));
        L->bz = (double *)calloc(nfz(L->nx, L->ny, L->nz), sizeof(double));
        L->a = (double *)calloc(ncell(L->nx, L->ny, L->nz), sizeof(double));
        L->r = (double *)calloc(ncell(L->nx, L->ny, L->nz), sizeof(double));
        if (l > 0) {
            L->e = (double *)calloc(ncell(L->nx, L->ny, L->nz), sizeof(double));
            L->rhs = (double *)calloc(ncell(L->nx, L->ny, L->nz), sizeof(double));
        }
        if (l == 0)
            copy_faces_zero_walls(L, bx, by, bz);
        else
            coarsen_faces(&H->d[l - 1], L);
        cell_weights(L);
    }
    if (want_float) {
        H->have_f = 1;
        for (int l = 0; l < H->nlev; l++) {
            level_d *L = &H->d[l];
            level_f *M = &H->f[l];
            M->nx = L->nx; M->ny = L->ny; M->nz = L->nz;
            size_t nc = ncell(L->nx, L->ny, L->nz);
            size_t fx = nfx(L->nx, L->ny, L->nz), fy = nfy(L->nx, L->ny, L->nz), fz = nfz(L->nx, L->ny, L->nz);
            M->bx = (float *)malloc(fx * sizeof(float));
            M->by = (float *)malloc(fy * sizeof(float));
            M->bz = (float *)malloc(fz * sizeof(float));
            M->a = (float *)malloc(nc * sizeof(float));
            M->e = (float *)calloc(nc, sizeof(float));
            M->rhs = (float *)calloc(nc, sizeof(float));
            M->r = (float *)calloc(nc, sizeof(float));
            for (size_t t = 0; t < fx; t++) M->bx[t] = (float)L->bx[t];
            for (size_t t = 0; t < fy; t++) M->by[t] = (float)L->by[t];
            for (size_t t = 0; t < fz; t++) M->bz[t] = (float)L->bz[t];
            for (size_t t = 0; t < nc; t++) M->a[t] = (float)L->a[t];
        }
    }
    level_d *Lc = &H->d[H->nlev - 1];
    return coarse_setup(Lc, &H->C);
}

/*
 * Restarted GMRES(m) on one grid (the paper's coarsest-grid solver, feature 6):
 * L e = rhs - mean(rhs) from e = 0, Arnoldi with modified Gram-Schmidt, the
 * least-squares problem kept triangular by Givens rotations, restart every m
 * iterations, stop when ||rhs_bar - L e|| <= tol ||rhs_bar|| or after maxit
 * iterations; e is returned mean-zero.  (On the singular Neumann system the
 * Krylov space of a mean-free residual stays mean-free.)  Returns the number
 * of iterations; *relres gets the final true relative residual.
 */
static int gmres_solve(const level_d *L, const double *rhs, double *e, int m, double tol, int maxit,
                       double *relres)
{
    size_t n = ncell(L->nx, L->ny, L->nz);
    double *bb = (double *)malloc(n * sizeof(double));
    double *r = (double *)malloc(n * sizeof(double));
    double *w = (double *)malloc(n * sizeof(double));
    double *Vb = (double *)malloc((size_t)(m + 1) * n * sizeof(double));
    double *H = (double *)calloc((size_t)(m + 1) * m, sizeof(double));
    double *cs = (double *)malloc(m * sizeof(double)), *sn = (double *)malloc(m * sizeof(double));
    double *g = (double *)malloc((m + 1) * sizeof(double)), *y = (double *)malloc(m * sizeof(double));
    double mb = 0;
    for (size_t t = 0; t < n; t++) mb += rhs[t];
    mb /= (double)n;
    double nb = 0;
    for (size_t t = 0; t < n; t++) {
        bb[t] = rhs[t] - mb;
        nb += bb[t] * bb[t];
        e[t] = 0.0;
    }
    nb = sqrt(nb);
    int it = 0;
    double beta = nb;
    for (size_t t = 0; t < n; t++) r[t] = bb[t];
    while (nb > 0 && beta > tol * nb && it < maxit) {
        for (size_t t = 0; t < n; t++) Vb[t] = r[t] / beta;
        for (int i = 0; i <= m; i++) g[i] = 0;
        g[0] = beta;
        int jj = 0;
        for (int j = 0; j < m && it < maxit; j++) {
            double *vj = Vb + (size_t)j * n;
            apply_d(L, vj, w);
            it++;
            for (int i = 0; i <= j; i++) {
                double *vi = Vb + (size_t)i * n, h = 0;
                for (size_t t = 0; t < n; t++) h += w[t] * vi[t];
                H[i * m + j] = h;
                for (size_t t = 0; t < n; t++) w[t] -= h * vi[t];
            }
            double hn = 0;
            for (size_t t = 0; t < n; t++) hn += w[t] * w[t];
            hn = sqrt(hn);
            H[(j + 1) * m + j] = hn;
            if (hn > 0)
                for (size_t t = 0; t < n; t++) Vb[(size_t)(j + 1) * n + t] = w[t] / hn;
            for (int i = 0; i < j; i++) {   /* earlier rotations on the new column */
                double a = H[i * m + j], b = H[(i + 1) * m + j];
                H[i * m + j] = cs[i] * a + sn[i] * b;
                H[(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
            }
            double a = H[j * m + j], b = H[(j + 1) * m + j], den = sqrt(a * a + b * b);
            cs[j] = den > 0 ? a / den : 1.0;
            sn[j] = den > 0 ? b / den : 0.0;
            H[j * m + j] = den;
            H[(j + 1) * m + j] = 0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            jj = j + 1;
            if (fabs(g[j + 1]) <= tol * nb || hn == 0) break;
        }
        for (int i = jj - 1; i >= 0; i--) {   /* back substitution */
            double t = g[i];
            for (int q = i + 1; q < jj; q++) t -= H[i * m + q] * y[q];
            y[i] = t / H[i * m + i];
        }
        for (int i = 0; i < jj; i++)
            for (size_t t = 0; t < n; t++) e[t] += y[i] * Vb[(size_t)i * n + t];
        residual_d(L, e, bb, r);
        beta = 0;
        for (size_t t = 0; t < n; t++) beta += r[t] * r[t];
        beta = sqrt(beta);
    }
    double me = 0;
    for (size_t t = 0; t < n; t++) me += e[t];
    me /= (double)n;
    for (size_t t = 0; t < n; t++) e[t] -= me;
    if (relres) *relres = nb > 0 ? beta / nb : 0.0;
    free(bb); free(r); free(w); free(Vb); free(H); free(cs); free(sn); free(g); free(y);
    return it;
}

static void coarse_variant(const coarse_t *C, const variant_t *V, const double *rhs, double *e)
{
    if (V && V->gmres_m > 0)
        gmres_solve((const level_d *)V->coarsest, rhs, e, V->gmres_m, V->gmres_tol, V->gmres_maxit, 0);
    else
        coarse_exact(C, rhs, e);
}

/* ------------------------------------------------------------------------- */
/* Exported primitives (for the tests)                                         */
/* ------------------------------------------------------------------------- */

static void wrap(level_d *L, int nx, int ny, int nz, const double *bx, const double *by, const double *bz)
{
    memset(L, 0, sizeof(*L));
    L->nx = nx; L->ny = ny; L->nz = nz;
    L->bx = (double *)bx; L->by = (double *)by; L->bz = (double *)bz;
}

void og_apply(int nx, int ny, int nz, const double *bx, const double *by, const double *bz,
              const double *p, double *out)
{
    level_d L;
    wrap(&L, nx, ny, nz, bx, by, bz);
    apply_d(&L, p, out);
}

void og_residual(int nx, int ny, int nz, const double *bx, const double *by, const double *bz,
                 const double *p, const double *b, double *r)
{
    level_d L;
    wrap(&L, nx, ny, nz, bx, by, bz);
    residual_d(&L, p, b, r);
}

void og_rb_half(int nx, int ny, int nz, const double *bx, const double *by, const double *bz,
                double *p, const double *b, int colour)
{
    level_d L;
    wrap(&L, nx, ny, nz, bx, by, bz);
    rb_half_d(&L, p, b, colour, 1.0);
}

/* One successive over-relaxation half-sweep (factor omega) over one colour. */
void og_rb_half_sor(int nx, int ny, int nz, const double *bx, const double *by, const double *bz,
                    double *p, const double *b, int colour, double omega)
{
    level_d L;
    wrap(&L, nx, ny, nz, bx, by, bz);
    rb_half_d(&L, p, b, colour, omega);
}

void og_restrict(int nx, int ny, int nz, const double *r, double *rc)
{
    level_d F, C;
    wrap(&F, nx, ny, nz, 0, 0, 0);
    wrap(&C, nx / 2, ny / 2, nz / 2, 0, 0, 0);
    restrict8_d(&F, r, &C, rc);
}

void og_restrict64(int nx, int ny, int nz, const double *r, double *rc)
{
    level_d F, C;
    wrap(&F, nx, ny, nz, 0, 0, 0);
    wrap(&C, nx / 2, ny / 2, nz / 2, 0, 0, 0);
    restrict64_d(&F, r, &C, rc);
}

void og_prolong_add(int cnx, int cny, int cnz, const double *a, const double *ec, double *ef)
{
    level_d F, C;
    wrap(&C, cnx, cny, cnz, 0, 0, 0);
    C.a = (double *)a;
    wrap(&F, 2 * cnx, 2 * cny, 2 * cnz, 0, 0, 0);
    prolong_add_d(&C, ec, &F, ef);
}

/* Coarse faces (walls 0) from fine faces; fine walls are taken as 0. */
void og_coarsen_faces(int nx, int ny, int nz, const double *bx, const double *by, const double *bz,
                      double *cbx, double *cby, double *cbz)
{
    level_d F, C;
    wrap(&F, nx, ny, nz, 0, 0, 0);
    F.bx = (double *)malloc(nfx(nx, ny, nz) * sizeof(double));
    F.by = (double *)malloc(nfy(nx, ny, nz) * sizeof(double));
    F.bz = (double *)malloc(nfz(nx, ny, nz) * sizeof(double));
    copy_faces_zero_walls(&F, bx, by, bz);
    wrap(&C, nx / 2, ny / 2, nz / 2, cbx, cby, cbz);
    coarsen_faces(&F, &C);
    free(F.bx); free(F.by); free(F.bz);
}

void og_cell_weights(int nx, int ny, int nz, const double *bx, const double *by, const double *bz,
                     double *a)
{
    level_d L;
    wrap(&L, nx, ny, nz, bx, by, bz);
    L.a = a;
    cell_weights(&L);
}

/* GMRES(m) on one grid (faces in the face layout); returns iterations. */
int og_gmres(int nx, int ny, int nz, const double *bx, const double *by, const double *bz, const double *rhs,
             double *e, int m, double tol, int maxit, double *relres)
{
    level_d L;
    wrap(&L, nx, ny, nz, 0, 0, 0);
    L.bx = (double *)malloc(nfx(nx, ny, nz) * sizeof(double));
    L.by = (double *)malloc(nfy(nx, ny, nz) * sizeof(double));
    L.bz = (double *)malloc(nfz(nx, ny, nz) * sizeof(double));
    copy_faces_zero_walls(&L, bx, by, bz);
    int it = gmres_solve(&L, rhs, e, m, tol, maxit, relres);
    free(L.bx); free(L.by); free(L.bz);
    return it;
}

/* Exact mean-zero solution of L e = rhs - mean(rhs) on one grid (dense). */
int og_dense_solve(int nx, int ny, int nz, const double *bx, const double *by, const double *bz,
                   const double *rhs, double *e)
{
    level_d L;
    wrap(&L, nx, ny, nz, 0, 0, 0);
    L.bx = (double *)malloc(nfx(nx, ny, nz) * sizeof(double));
    L.by = (double *)malloc(nfy(nx, ny, nz) * sizeof(double));
    L.bz = (double *)malloc(nfz(nx, ny, nz) * sizeof(double));
    copy_faces_zero_walls(&L, bx, by, bz);
    coarse_t C;
    int rc = coarse_setup(&L, &C);
    if (rc == 0) coarse_exact(&C, rhs, e);
    free(C.chol);
    free(L.bx); free(L.by); free(L.bz);
    return rc;
}

/* Hierarchy faces and weights for level l (for parity tests of the setup kernels). */
int og_hierarchy_level(int nx, int ny, int nz, const double *bx, const double *by, const double *bz,
                       int n_coarsest, int l, double *obx, double *oby, double *obz, double *oa)
{
    hier_t H;
    hier_build(&H, nx, ny, nz, bx, by, bz, n_coarsest, 0); /* coarse factor not needed here */
    if (l < 0 || l >= H.nlev) {
        hier_free(&H);
        return -1;
    }
    level_d *L = &H.d[l];
    memcpy(obx, L->bx, nfx(L->nx, L->ny, L->nz) * sizeof(double));
    memcpy(oby, L->by, nfy(L->nx, L->ny, L->nz) * sizeof(double));
    memcpy(obz, L->bz, nfz(L->nx, L->ny, L->nz) * sizeof(double));
    memcpy(oa, L->a, ncell(L->nx, L->ny, L->nz) * sizeof(double));
    hier_free(&H);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Projection step around the solve (Sec. 2.2)                                 */
/* ------------------------------------------------------------------------- */
/*
 * The flow solver advances the velocity with Chorin's projection method on the
 * staggered MAC mesh: each velocity component lives on the faces normal to it,
 * the pressure in the cells, and every derivative is a second-order centred
 * difference.  The source of the pressure equation (9) is the divergence of the
 * non-projected velocity u* over the time step, S = div(u*) / dt; with the h^2
 * of eq. (10) folded into the right-hand side,
 *     b_c = h^2 S_c = (h / dt) * sum_d (u_d(upper face of c) - u_d(lower face of c)).
 * The projected velocity is u = u* - dt (1/rho)_f grad p, on each interior face
 * f between cells c- (lower index) and c+:
 *     u_f = u*_f - (dt / h) * beta_f * (p(c+) - p(c-)),
 * with beta_f the face coefficient of eq. (10); its discrete divergence is then
 * (dt / h^2) (b - L p), zero once L p = b.  Wall faces keep their values (the
 * pressure has homogeneous Neumann conditions there).
 *
 * Evaluation order (fixed, so another implementation can reproduce it):
 *     b_c = scale * ((du + dv) + dw),  du = u(i+1) - u(i) etc.;
 *     u_f = u_f - (scale * beta_f) * (p(c+) - p(c-)).
 */
static size_t fx_at(int nx, int ny, int i, int j, int k) { return ((size_t)k * ny + j) * (nx + 1) + i; }
static size_t fy_at(int nx, int ny, int i, int j, int k) { return ((size_t)k * (ny + 1) + j) * nx + i; }
static size_t fz_at(int nx, int ny, int i, int j, int k) { return ((size_t)k * ny + j) * nx + i; }
static size_t c_at(int nx, int ny, int i, int j, int k) { return ((size_t)k * ny + j) * nx + i; }

/* b = scale * (discrete divergence of (u, v, w) times h); scale = h / dt. */
void og_divergence(int nx, int ny, int nz, const double *u, const double *v, const double *w,
                   double scale, double *b)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                double du = u[fx_at(nx, ny, i + 1, j, k)] - u[fx_at(nx, ny, i, j, k)];
                double dv = v[fy_at(nx, ny, i, j + 1, k)] - v[fy_at(nx, ny, i, j, k)];
                double dw = w[fz_at(nx, ny, i, j, k + 1)] - w[fz_at(nx, ny, i, j, k)];
                b[c_at(nx, ny, i, j, k)] = scale * ((du + dv) + dw);
            }
}

/* u -= scale * beta * (pressure difference across the face), interior faces
   only; scale = dt / h.  bx, by, bz in the face layout (walls not read). */
void og_correct_velocity(int nx, int ny, int nz, const double *bx, const double *by, const double *bz,
                         const double *p, double scale, double *u, double *v, double *w)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++) {
            for (int i = 1; i < nx; i++) {
                size_t f = fx_at(nx, ny, i, j, k);
                double dp = p[c_at(nx, ny, i, j, k)] - p[c_at(nx, ny, i - 1, j, k)];
                u[f] = u[f] - (scale * bx[f]) * dp;
            }
            if (j > 0)
                for (int i = 0; i < nx; i++) {
                    size_t f = fy_at(nx, ny, i, j, k);
                    double dp = p[c_at(nx, ny, i, j, k)] - p[c_at(nx, ny, i, j - 1, k)];
                    v[f] = v[f] - (scale * by[f]) * dp;
                }
            if (k > 0)
                for (int i = 0; i < nx; i++) {
                    size_t f = fz_at(nx, ny, i, j, k);
                    double dp = p[c_at(nx, ny, i, j, k)] - p[c_at(nx, ny, i, j, k - 1)];
                    w[f] = w[f] - (scale * bz[f]) * dp;
                }
        }
}

/* ------------------------------------------------------------------------- */
/* Material properties from a level-set field (Sec. 2.2, eq. 8)                */
/* ------------------------------------------------------------------------- */
/*
 * The indicator I is a numerical Heaviside that goes from 0 to 1 over three to
 * four cells; from a level set phi (positive in the liquid) it is the smoothed
 * Heaviside of half-width eps:
 *     I = 0 (phi <= -eps),  1 (phi >= eps),  (1/2)(1 + x + sin(pi x)/pi), x = phi/eps
 * (the band edges take their exact values; the formula would leave a rounding
 * residue of sin(pi) there).
 * Eq. (8) mixes the density linearly, rho = rho_g + (rho_l - rho_g) I, the
 * pressure equation's coefficient is alpha = 1/rho, and each interior face gets
 * the arithmetic mean of its two cells' alpha or, with harmonic = 1, the
 * harmonic mean of eqs. (11)-(12), 2 a b / (a + b).  Wall faces are 0.
 * Evaluation order (fixed): x = phi/eps, I = 0.5 * ((1 + x) + sin(pi * x) / pi),
 * alpha = 1 / (rho_g + (rho_l - rho_g) * I), arithmetic 0.5 * (a + b),
 * harmonic (2 * a * b) / (a + b).
 */
static const double OG_PI = 3.14159265358979323846;

static double cell_alpha(double phi, double rho_l, double rho_g, double eps)
{
    double ind;
    if (phi <= -eps) ind = 0.0;
    else if (phi >= eps) ind = 1.0;
    else {
        double x = phi / eps;
        ind = 0.5 * ((1.0 + x) + sin(OG_PI * x) / OG_PI);
    }
    return 1.0 / (rho_g + (rho_l - rho_g) * ind);
}

static double face_mean(double a, double b, int harmonic)
{
    return harmonic ? (2.0 * a * b) / (a + b) : 0.5 * (a + b);
}

void og_faces_from_levelset(int nx, int ny, int nz, const double *phi, double rho_l, double rho_g, double eps,
                            int harmonic, double *bx, double *by, double *bz)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++) {
            for (int i = 0; i <= nx; i++) {
                size_t f = fx_at(nx, ny, i, j, k);
                bx[f] = (i == 0 || i == nx) ? 0.0
                        : face_mean(cell_alpha(phi[c_at(nx, ny, i - 1, j, k)], rho_l, rho_g, eps),
                                    cell_alpha(phi[c_at(nx, ny, i, j, k)], rho_l, rho_g, eps), harmonic);
            }
        }
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; k++)
        for (int j = 0; j <= ny; j++)
            for (int i = 0; i < nx; i++) {
                size_t f = fy_at(nx, ny, i, j, k);
                by[f] = (j == 0 || j == ny) ? 0.0
                        : face_mean(cell_alpha(phi[c_at(nx, ny, i, j - 1, k)], rho_l, rho_g, eps),
                                    cell_alpha(phi[c_at(nx, ny, i, j, k)], rho_l, rho_g, eps), harmonic);
            }
#pragma omp parallel for schedule(static)
    for (int k = 0; k <= nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                size_t f = fz_at(nx, ny, i, j, k);
                bz[f] = (k == 0 || k == nz) ? 0.0
                        : face_mean(cell_alpha(phi[c_at(nx, ny, i, j, k - 1)], rho_l, rho_g, eps),
                                    cell_alpha(phi[c_at(nx, ny, i, j, k)], rho_l, rho_g, eps), harmonic);
            }
}

/* ------------------------------------------------------------------------- */
/* Driver                                                                      */
/* ------------------------------------------------------------------------- */

typedef struct {
    int nu1, nu2;
    int n_coarsest;
    int max_cycles;  /* V-cycles (FP64) or outer iterations (refined) */
    int precision;   /* 0: FP64 multigrid, 1: FP32 V-cycles inside FP64 refinement */
    int inner_m;     /* FP32 V-cycles per outer iteration */
    double tol;      /* relative residual ||b_bar - L p|| / ||b_bar|| */
    int krylov;      /* FP64 only: 0 V-cycle iteration, 1 flexible CG preconditioned by one
                        V-cycle, 2 unpreconditioned CG (for the tests) */
    double omega;    /* variants, see variant_t */
    int restrict64;
    int gmres_m;
    double gmres_tol;
    int gmres_maxit;
} og_opts;

/*
 * Result codes: 0 converged, 1 not converged within max_cycles, 2 diverged
 * (NaN or growth), -1 invalid input/singular coarse operator.
 */
static double last_setup_s = 0, last_cycles_s = 0;

/* Wall time of the last og_solve: hierarchy setup, and everything after it. */
void og_last_timing(double *setup_s, double *cycles_s)
{
    *setup_s = last_setup_s;
    *cycles_s = last_cycles_s;
}

static double wall(void)
{
#ifdef _OPENMP
    return omp_get_wtime();
#else
    return 0.0;
#endif
}

static double dot_d(const double *a, const double *b, size_t n)
{
    double s = 0.0;
    for (size_t t = 0; t < n; t++) s += a[t] * b[t];
    return s;
}

/*
 * Krylov acceleration of the multigrid solve (FP64): flexible conjugate
 * gradients, FCG(1) of Notay (SIAM J. Sci. Comput. 22, 2000), on A = -L, which
 * is symmetric positive definite on mean-free vectors.  The preconditioner is
 * one V-cycle from a zero guess; since the paper's restriction and
 * prolongation are not transposes of each other the cycle is not a symmetric
 * operator, which the flexible form tolerates: each new direction is made
 * A-orthogonal to the previous one explicitly.  Written with L itself (signs
 * folded in; z = V(r) approximates L^-1 r):
 *     z = V(r);  beta = -(z . q) / (s . q)  (0 on the first iteration);
 *     s = z + beta s;  q = L s;  alpha = (r . z) / (s . q);
 *     p += alpha s;  r = b_bar - L p   (the true residual, every iteration).
 * krylov = 2 replaces the preconditioner by the identity on A (z = -r), which
 * is textbook CG.  p is made mean-zero once, at the end.  Returns the status
 * as og_solve and fills hist / *ncycles with one entry per iteration.
 */
static int krylov_solve(hier_t *H, const double *bbar, double nb, double *p, const og_opts *o,
                        const variant_t *V, double *hist, int *ncycles, double rho0)
{
    level_d *F = &H->d[0];
    size_t n = ncell(F->nx, F->ny, F->nz);
    double *r = (double *)malloc(n * sizeof(double));
    double *z = (double *)calloc(n, sizeof(double));
    double *sd = (double *)calloc(n, sizeof(double));
    double *q = (double *)calloc(n, sizeof(double));
    double sq = 0.0, rho = rho0;
    int status = rho0 <= o->tol ? 0 : 1, it = 0;
    residual_d(F, p, bbar, r);
    while (status == 1 && it < o->max_cycles) {
        if (o->krylov == 1) {
            memset(z, 0, n * sizeof(double));
            F->e = z;
            F->rhs = r;
            vcycle_d(H->d, H->nlev, 0, &H->C, o->nu1, o->nu2, V);
        } else {
            for (size_t t = 0; t < n; t++) z[t] = -r[t];
        }
        double zq = dot_d(z, q, n), rz = dot_d(r, z, n);
        double beta = sq == 0.0 ? 0.0 : -zq / sq;
        for (size_t t = 0; t < n; t++) sd[t] = z[t] + beta * sd[t];
        apply_d(F, sd, q);
        sq = dot_d(sd, q, n);
        double alpha = rz / sq;
        for (size_t t = 0; t < n; t++) p[t] += alpha * sd[t];
        residual_d(F, p, bbar, r);
        rho = sqrt(sumsq_d(r, n)) / nb;
        hist[++it] = rho;
        if (!(rho == rho) || rho > 1e6 * rho0) status = 2;
        else if (rho <= o->tol) status = 0;
    }
    double mp = sum_d(p, n) / (double)n;
    for (size_t t = 0; t < n; t++) p[t] -= mp;
    F->e = 0;
    F->rhs = 0;
    free(r); free(z); free(sd); free(q);
    *ncycles = it;
    return status;
}

int og_solve(int nx, int ny, int nz, const double *bx, const double *by, const double *bz,
             const double *b, double *p, const og_opts *o, double *hist, int *ncycles,
             double *mean_b_out, double *gamma_out)
{
    hier_t H;
    double t0 = wall();
    int rc = hier_build(&H, nx, ny, nz, bx, by, bz, o->n_coarsest, o->precision == 1);
    double t1 = wall();
    last_setup_s = t1 - t0;
    last_cycles_s = 0;
    if (rc != 0) {
        hier_free(&H);
        return -1;
    }
    size_t n = ncell(nx, ny, nz);
    level_d *F = &H.d[0];
    if (!(o->omega > 0 && o->omega < 2) || o->gmres_m < 0 || o->gmres_m > 64 ||
        (o->gmres_m > 0 && (!(o->gmres_tol > 0) || o->gmres_maxit < 1))) {
        hier_free(&H);
        return -1;
    }
    variant_t V = {o->omega, o->restrict64, o->gmres_m, o->gmres_tol, o->gmres_maxit, &H.d[H.nlev - 1]};

    /* right-hand side projected onto the range of L: b_bar = b - mean(b) */
    double mean_b = sum_d(b, n) / (double)n;
    double *bbar = (double *)malloc(n * sizeof(double));
    for (size_t t = 0; t < n; t++) bbar[t] = b[t] - mean_b;
    double nb = sqrt(sumsq_d(bbar, n));
    if (mean_b_out) *mean_b_out = mean_b;
    F->e = p;
    F->rhs = bbar;

    int status = 1, cyc = 0;
    if (nb == 0.0) { /* zero right-hand side: the mean-zero solution is 0 */
        memset(p, 0, n * sizeof(double));
        hist[0] = 0.0;
        *ncycles = 0;
        if (gamma_out) *gamma_out = 0.0;
        free(bbar);
        F->e = 0; F->rhs = 0;
        hier_free(&H);
        return 0;
    }
    residual_d(F, p, bbar, F->r);
    double rho0 = sqrt(sumsq_d(F->r, n)) / nb, rho = rho0;
    hist[0] = rho0;
    if (rho0 <= o->tol) status = 0;

    if (o->precision == 0 && o->krylov != 0) {
        if (o->krylov != 1 && o->krylov != 2) {
            free(bbar);
            F->e = 0; F->rhs = 0;
            hier_free(&H);
            return -1;
        }
        F->e = 0;
        status = krylov_solve(&H, bbar, nb, p, o, &V, hist, &cyc, rho0);
        if (cyc > 0) rho = hist[cyc];
    } else if (o->precision == 0) {
        while (status == 1 && cyc < o->max_cycles) {
            vcycle_d(H.d, H.nlev, 0, &H.C, o->nu1, o->nu2, &V);
            double mp = sum_d(p, n) / (double)n;
            for (size_t t = 0; t < n; t++) p[t] -= mp;
            residual_d(F, p, bbar, F->r);
            rho = sqrt(sumsq_d(F->r, n)) / nb;
            hist[++cyc] = rho;
            if (!(rho == rho) || rho > 1e6 * rho0) status = 2;
            else if (rho <= o->tol) status = 0;
        }
    } else {
        level_f *M = &H.f[0];
        while (status == 1 && cyc < o->max_cycles) {
            /* scale the residual by a power of two near its RMS so the float
               cycles see O(1) values; a power of two leaves every float
               operation's rounding unchanged */
            double rms = sqrt(sumsq_d(F->r, n) / (double)n);
            double s = rms > 0 ? ldexp(1.0, (int)floor(log2(rms))) : 1.0;
            for (size_t t = 0; t < n; t++) M->rhs[t] = (float)(F->r[t] / s);
            memset(M->e, 0, n * sizeof(float));
            for (int it = 0; it < o->inner_m; it++) vcycle_f(H.f, H.nlev, 0, &H.C, o->nu1, o->nu2, &V);
            for (size_t t = 0; t < n; t++) p[t] += s * (double)M->e[t];
            double mp = sum_d(p, n) / (double)n;
            for (size_t t = 0; t < n; t++) p[t] -= mp;
            residual_d(F, p, bbar, F->r);
            rho = sqrt(sumsq_d(F->r, n)) / nb;
            hist[++cyc] = rho;
            if (!(rho == rho) || rho > 1e6 * rho0) status = 2;
            else if (rho <= o->tol) status = 0;
        }
    }
    *ncycles = cyc;
    last_cycles_s = wall() - t1;
    /* average reduction rate, eq. (15) */
    if (gamma_out) *gamma_out = cyc > 0 ? pow(rho / rho0, 1.0 / cyc) : 0.0;
    free(bbar);
    F->e = 0;
    F->rhs = 0;
    hier_free(&H);
    return status;
}

int og_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
