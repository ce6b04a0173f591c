/*
 * FP64 reference implementation ("oracle") of the tensor-product geometric
 * multigrid preconditioned CG solver for the anisotropic pressure-correction
 * equation of Mueller & Scheichl, "Massively parallel solvers for elliptic
 * PDEs in Numerical Weather- and Climate Prediction" (arXiv:1307.2036).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct CPU
 * version that the HIP library is checked against.  It shares no code, header
 * or table with the GPU path; only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.
 *
 * Problem (Sec. 3, eq. ModelEquation, in its Cartesian doubly periodic form):
 *     -omega^2 ( Lap_2d u + d/dz( lambda^2(z) du/dz ) ) + u = f
 * on nx x ny x nz cells, horizontally periodic, homogeneous Neumann at the
 * bottom and top.  Cell-centred finite volumes (Sec. 3.1): every flux through
 * a cell face is a two-point difference, so the stencil has 7 points.
 *
 * Layout: plane-major, idx = (k*ny + j)*nx + i.  Level 0 is the finest grid
 * (the paper numbers levels the other way round, Sec. 4.3).
 *
 * Readings of the paper taken here (each is listed in the design notes):
 *  - operator in flux ("difference") form: A u = V u + sum_faces T (u - u_nbr);
 *    vertical face coefficient by the harmonic rule for lambda^2(z), which
 *    keeps the operator symmetric (Sec. 2, operator D^(z) in divergence form);
 *    faces along a dimension of size 1 join a cell to itself and are omitted;
 *  - coarse operators are re-discretised on h_l = 2^l h (Sec. 4.3.2, 6.2.1);
 *  - block red/black SOR by vertical columns, colour (i+j) mod 2 in level-
 *    local indices (Sec. 4.2 eq. BlockRBSOR, Sec. 6.2.1); pre-smoothing order
 *    (red, black), post-smoothing (black, red);
 *  - the column solve is the Thomas algorithm (Appendix B, Alg. "Tridiagonal
 *    matrix algorithm") with the pivots carried in "excess" form
 *    p_k = T_{k+1/2} + e_k, which is algebraically identical to the printed
 *    recurrence but never forms the huge assembled diagonal;
 *  - restriction sums the four children's integrated residuals (the cell
 *    average of per-volume residuals); prolongation is bilinear 9/3/3/1
 *    (Sec. 6.2.1), or piecewise constant as an option;
 *  - PCG follows Appendix B Alg. "Preconditioned Conjugate Gradient method"
 *    with the residual update written r <- r - alpha q (the printed "+" is a
 *    sign slip); the flexible (Polak-Ribiere) beta is available and default;
 *  - norms are Euclidean norms of the volume-integrated residual b - A u with
 *    b = V f.
 *
 * Horizontally varying vertical coefficients (beyond the paper's lambda^2(r),
 * the next step toward its panel geometry, Sec. 3 and 6.2.1): with a 3D cell
 * field lambda^2(i,j,k) every column has its own vertical face coefficients,
 * by the same harmonic rule; the coarse level's face of a column is the sum of
 * its four children's faces (parallel faces, so the vertical fluxes of a
 * horizontally constant correction are conserved; for a horizontally constant
 * lambda^2 it is exactly the re-discretised face).  The column matrix of the
 * line smoother then differs from column to column.
 *
 * Dots are accumulated sequentially in natural index order.  Build with
 * -ffp-contract=off so that no fused multiply-add changes the rounding.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------------- */
/* public structures (mirrored by the ctypes wrapper oracle/oracle.py)     */
/* ---------------------------------------------------------------------- */
typedef struct {
    int nx, ny, nz;
    double hx, hy;
    double omega2;
    const double *dz;       /* nz cell thicknesses             */
    const double *lambda2;  /* nz cell-centre values of lambda^2 */
    const double *tz3;      /* NULL: vertical faces from lambda2(z); else the
                               per-column vertical face coefficients, (nz+1) x
                               ny x nx, tz3[(k*ny + j)*nx + i] joining cells k-1
                               and k of column (i, j) (faces 0 and nz are 0) */
} orc_geom;

typedef struct {
    orc_geom g;             /* finest level                        */
    int n_levels;           /* 0 = standard depth                  */
    int nu_pre, nu_post, nu_coarse;
    double rho;             /* SOR relaxation factor               */
    int prolong;            /* 0 = bilinear, 1 = piecewise constant */
} orc_mg;

typedef struct {
    double rtol, atol;
    int maxiter;
    int flexible;           /* 1: beta = <z_K, r_K - r_{K-1}>/<z_{K-1}, r_{K-1}> */
    int rel_to_rhs;         /* 1: relative test against ||b|| instead of ||r_0|| */
} orc_opts;

typedef struct {
    int iters;
    double r0_norm, r_norm, true_r_norm, b_norm;
    int status;             /* 0 converged, 1 maxiter reached, -4 non-finite */
} orc_stats;

/* ---------------------------------------------------------------------- */
/* geometry of one level                                                   */
/* ---------------------------------------------------------------------- */
typedef struct {
    int nx, ny, nz;
    double *V;   /* cell volume hx*hy*dz_k                                 */
    double *Tx;  /* x-face coefficient omega^2 * hy*dz_k / hx              */
    double *Ty;  /* y-face coefficient omega^2 * hx*dz_k / hy              */
    double *Tz;  /* nz+1 vertical faces; Tz[k] joins cells k-1 and k;      */
                 /* Tz[0] = Tz[nz] = 0 (homogeneous Neumann)               */
    double *s;   /* column "excess": V_k + (number of x faces) Tx_k + (y faces) Ty_k */
    double *Tz3; /* NULL, or per-column vertical faces, layout as orc_geom.tz3 */
} level_t;

/* Vertical face coefficient joining cells k-1 and k of column (i, j). */
static double tzf(const level_t *L, int i, int j, int k)
{
    return L->Tz3 ? L->Tz3[((size_t)k * L->ny + j) * L->nx + i] : L->Tz[k];
}

static int has_x(const level_t *L) { return L->nx > 1; }
static int has_y(const level_t *L) { return L->ny > 1; }

/* Face coefficients of the finite-volume discretisation (Sec. 3.1):
 * flux through a face = omega^2 * (area / distance) * (u - u_nbr), and for
 * the vertical faces lambda^2 enters through the two half-cell resistances
 * dz_k/(2 lambda^2_k) in series. */
void orc_level_coeffs(int nx, int ny, int nz, double hx, double hy, double omega2,
                      const double *dz, const double *lambda2,
                      double *V, double *Tx, double *Ty, double *Tz, double *s)
{
    for (int k = 0; k < nz; k++) {
        V[k] = hx * hy * dz[k];
        Tx[k] = omega2 * hy * dz[k] / hx;
        Ty[k] = omega2 * hx * dz[k] / hy;
    }
    Tz[0] = 0.0;
    Tz[nz] = 0.0;
    for (int k = 1; k < nz; k++) {
        double resistance = dz[k - 1] / (2.0 * lambda2[k - 1]) + dz[k] / (2.0 * lambda2[k]);
        Tz[k] = omega2 * hx * hy / resistance;
    }
    for (int k = 0; k < nz; k++) {
        double e = V[k];
        if (nx > 1) e += 2.0 * Tx[k];
        if (ny > 1) e += 2.0 * Ty[k];
        s[k] = e;
    }
}

static void level_init(level_t *L, int nx, int ny, int nz, double hx, double hy,
                       double omega2, const double *dz, const double *lambda2)
{
    L->nx = nx; L->ny = ny; L->nz = nz;
    L->V = (double *)malloc(sizeof(double) * nz);
    L->Tx = (double *)malloc(sizeof(double) * nz);
    L->Ty = (double *)malloc(sizeof(double) * nz);
    L->Tz = (double *)malloc(sizeof(double) * (nz + 1));
    L->s = (double *)malloc(sizeof(double) * nz);
    orc_level_coeffs(nx, ny, nz, hx, hy, omega2, dz, lambda2, L->V, L->Tx, L->Ty, L->Tz, L->s);
    L->Tz3 = NULL;
}

/* Per-column faces (copied), layout as orc_geom.tz3. */
static void level_set_tz3(level_t *L, const double *tz3)
{
    size_t n = (size_t)(L->nz + 1) * L->ny * L->nx;
    L->Tz3 = (double *)malloc(sizeof(double) * n);
    memcpy(L->Tz3, tz3, sizeof(double) * n);
}

static void level_free(level_t *L)
{
    free(L->V); free(L->Tx); free(L->Ty); free(L->Tz); free(L->s); free(L->Tz3);
}

/* Per-column vertical faces of a 3D cell field lambda^2 (layout nz x ny x nx,
 * plane-major): the harmonic rule of orc_level_coeffs in every column. */
void orc_tz3_from_lambda2(int nx, int ny, int nz, double hx, double hy, double omega2,
                          const double *dz, const double *lambda2_3d, double *tz3)
{
    size_t plane = (size_t)nx * ny;
    for (size_t c = 0; c < plane; c++) {
        tz3[c] = 0.0;
        tz3[(size_t)nz * plane + c] = 0.0;
        for (int k = 1; k < nz; k++) {
            double resistance = dz[k - 1] / (2.0 * lambda2_3d[(size_t)(k - 1) * plane + c])
                              + dz[k] / (2.0 * lambda2_3d[(size_t)k * plane + c]);
            tz3[(size_t)k * plane + c] = omega2 * hx * hy / resistance;
        }
    }
}

/* Coarse faces: each coarse column's face is the sum of its four children's,
 * added in pairs ((0,0) + (1,0)) + ((0,1) + (1,1)); nx, ny: fine sizes. */
void orc_tz3_coarsen(int nx, int ny, int nz, const double *tz3f, double *tz3c)
{
    int cx = nx / 2, cy = ny / 2;
    for (int k = 0; k <= nz; k++)
        for (int J = 0; J < cy; J++)
            for (int I = 0; I < cx; I++) {
                const double *f = tz3f + (size_t)k * nx * ny;
                double a = f[(size_t)(2 * J) * nx + 2 * I] + f[(size_t)(2 * J) * nx + 2 * I + 1];
                double b = f[(size_t)(2 * J + 1) * nx + 2 * I] + f[(size_t)(2 * J + 1) * nx + 2 * I + 1];
                tz3c[((size_t)k * cy + J) * cx + I] = a + b;
            }
}

static size_t IDX(const level_t *L, int i, int j, int k)
{
    return ((size_t)k * L->ny + j) * L->nx + i;
}

static int wrap(int i, int n) { return (i % n + n) % n; }

/* ---------------------------------------------------------------------- */
/* operator y = A x (eq. ModelEquation integrated over each cell)          */
/* ---------------------------------------------------------------------- */
static void apply_level(const level_t *L, const double *x, double *y)
{
    const int nx = L->nx, ny = L->ny, nz = L->nz;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; k++) {
        for (int j = 0; j < ny; j++) {
            for (int i = 0; i < nx; i++) {
                size_t c = IDX(L, i, j, k);
                double xc = x[c];
                double acc = L->V[k] * xc;
                if (has_x(L)) {
                    acc += L->Tx[k] * (xc - x[IDX(L, wrap(i - 1, nx), j, k)]);
                    acc += L->Tx[k] * (xc - x[IDX(L, wrap(i + 1, nx), j, k)]);
                }
                if (has_y(L)) {
                    acc += L->Ty[k] * (xc - x[IDX(L, i, wrap(j - 1, ny), k)]);
                    acc += L->Ty[k] * (xc - x[IDX(L, i, wrap(j + 1, ny), k)]);
                }
                if (k > 0) acc += tzf(L, i, j, k) * (xc - x[IDX(L, i, j, k - 1)]);
                if (k < nz - 1) acc += tzf(L, i, j, k + 1) * (xc - x[IDX(L, i, j, k + 1)]);
                y[c] = acc;
            }
        }
    }
}

/* Sum of the absolute values of the terms of (A x)_c; a floating-point error
 * scale for comparisons of A x computed in a different order. */
static void apply_abs_level(const level_t *L, const double *x, double *y)
{
    const int nx = L->nx, ny = L->ny, nz = L->nz;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; k++) {
        for (int j = 0; j < ny; j++) {
            for (int i = 0; i < nx; i++) {
                size_t c = IDX(L, i, j, k);
                double xc = x[c];
                double acc = fabs(L->V[k] * xc);
                if (has_x(L)) {
                    acc += L->Tx[k] * (fabs(xc) + fabs(x[IDX(L, wrap(i - 1, nx), j, k)]));
                    acc += L->Tx[k] * (fabs(xc) + fabs(x[IDX(L, wrap(i + 1, nx), j, k)]));
                }
                if (has_y(L)) {
                    acc += L->Ty[k] * (fabs(xc) + fabs(x[IDX(L, i, wrap(j - 1, ny), k)]));
                    acc += L->Ty[k] * (fabs(xc) + fabs(x[IDX(L, i, wrap(j + 1, ny), k)]));
                }
                if (k > 0) acc += tzf(L, i, j, k) * (fabs(xc) + fabs(x[IDX(L, i, j, k - 1)]));
                if (k < nz - 1) acc += tzf(L, i, j, k + 1) * (fabs(xc) + fabs(x[IDX(L, i, j, k + 1)]));
                y[c] = acc;
            }
        }
    }
}

/* ---------------------------------------------------------------------- */
/* tridiagonal solves (Appendix B, Alg. "Tridiagonal matrix algorithm")    */
/* ---------------------------------------------------------------------- */

/* The algorithm as printed, in its own notation: diagonal a, super-diagonal
 * b, sub-diagonal c (c[0] and b[n-1] unused), right-hand side f. */
void orc_thomas_plain(int n, const double *a, const double *b, const double *c,
                      const double *f, double *u)
{
    double *bp = (double *)malloc(sizeof(double) * n);
    double *fp = (double *)malloc(sizeof(double) * n);
    bp[0] = (n > 1) ? b[0] / a[0] : 0.0;
    fp[0] = f[0] / a[0];
    for (int i = 1; i < n; i++) {
        double piv = a[i] - bp[i - 1] * c[i];
        bp[i] = (i < n - 1) ? b[i] / piv : 0.0;
        fp[i] = (f[i] - fp[i - 1] * c[i]) / piv;
    }
    u[n - 1] = fp[n - 1];
    for (int i = n - 2; i >= 0; i--) u[i] = fp[i] - bp[i] * u[i + 1];
    free(bp);
    free(fp);
}

/* The same elimination for the column matrix of the line smoother,
 *   diagonal  d_k = s_k + T_{k-1/2} + T_{k+1/2},  off-diagonals -T_{k+-1/2},
 * with every pivot written as p_k = T_{k+1/2} + e_k, where
 *   e_0 = s_0,   e_k = s_k + T_{k-1/2} e_{k-1} / (T_{k-1/2} + e_{k-1}).
 * (Substituting p_{k-1} = T_{k-1/2} + e_{k-1} into d_k - T_{k-1/2}^2/p_{k-1}
 * gives this.)  All terms are positive, so nothing cancels even when the
 * vertical coefficients exceed the excess s_k by many orders of magnitude.
 * Tz has nz+1 entries, Tz[k] = T_{k-1/2}. */
void orc_column_solve(int nz, const double *s, const double *Tz, const double *g,
                      double *w, double *work)
{
    double *y = work;
    double *p = work + nz;
    double e = s[0];
    for (int k = 0; k < nz; k++) {
        if (k > 0) e = s[k] + Tz[k] * e / (Tz[k] + e);
        p[k] = Tz[k + 1] + e;
        double rhs = g[k];
        if (k > 0) rhs += Tz[k] * y[k - 1];
        y[k] = rhs / p[k];
    }
    w[nz - 1] = y[nz - 1];
    for (int k = nz - 2; k >= 0; k--) w[k] = y[k] + (Tz[k + 1] / p[k]) * w[k + 1];
}

/* ---------------------------------------------------------------------- */
/* block (vertical line) red/black SOR, one colour (Sec. 4.2 eq.          */
/* BlockRBSOR): for each column of the colour, move the couplings to the   */
/* other colour to the right-hand side and solve the column exactly.       */
/* ---------------------------------------------------------------------- */
static void smooth_colour(const level_t *L, int colour, double rho, const double *b, double *u)
{
    const int nx = L->nx, ny = L->ny, nz = L->nz;
#pragma omp parallel
    {
        double *g = (double *)malloc(sizeof(double) * nz);
        double *w = (double *)malloc(sizeof(double) * nz);
        double *work = (double *)malloc(sizeof(double) * 2 * nz);
        double *tcol = (double *)malloc(sizeof(double) * (nz + 1));
#pragma omp for schedule(static)
        for (int j = 0; j < ny; j++) {
            for (int i = 0; i < nx; i++) {
                if (((i + j) & 1) != colour) continue;
                for (int k = 0; k < nz; k++) {
                    double acc = b[IDX(L, i, j, k)];
                    if (has_x(L))
                        acc += L->Tx[k] * (u[IDX(L, wrap(i - 1, nx), j, k)] + u[IDX(L, wrap(i + 1, nx), j, k)]);
                    if (has_y(L))
                        acc += L->Ty[k] * (u[IDX(L, i, wrap(j - 1, ny), k)] + u[IDX(L, i, wrap(j + 1, ny), k)]);
                    g[k] = acc;
                }
                if (L->Tz3) {
                    for (int k = 0; k <= nz; k++) tcol[k] = tzf(L, i, j, k);
                    orc_column_solve(nz, L->s, tcol, g, w, work);
                } else {
                    orc_column_solve(nz, L->s, L->Tz, g, w, work);
                }
                for (int k = 0; k < nz; k++) {
                    size_t c = IDX(L, i, j, k);
                    u[c] = (1.0 - rho) * u[c] + rho * w[k];
                }
            }
        }
        free(g); free(w); free(work); free(tcol);
    }
}

/* ---------------------------------------------------------------------- */
/* inter-grid transfers (Sec. 4.3 and 6.2.1)                              */
/* ---------------------------------------------------------------------- */

/* b_c(I,J,k) = sum over the 2x2 children of r(i,j,k). */
static void restrict_sum(const level_t *F, const level_t *C, const double *r, double *bc)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < C->nz; k++)
        for (int J = 0; J < C->ny; J++)
            for (int I = 0; I < C->nx; I++) {
                double acc = 0.0;
                for (int bb = 0; bb < 2; bb++)
                    for (int aa = 0; aa < 2; aa++)
                        acc += r[IDX(F, 2 * I + aa, 2 * J + bb, k)];
                bc[IDX(C, I, J, k)] = acc;
            }
}

/* u(i,j,k) += interpolated coarse value.  Bilinear for cell-centred data: the
 * fine centre lies a quarter of a coarse cell from its parent's centre, so
 * the parent weighs 3/4 and the nearer neighbour 1/4 in each direction. */
static void prolong_add(const level_t *F, const level_t *C, int mode, const double *uc, double *u)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < F->nz; k++)
        for (int j = 0; j < F->ny; j++)
            for (int i = 0; i < F->nx; i++) {
                int I = i / 2, J = j / 2;
                double e;
                if (mode == 1) {
                    e = uc[IDX(C, I, J, k)];
                } else {
                    int I2 = wrap(I + ((i & 1) ? 1 : -1), C->nx);
                    int J2 = wrap(J + ((j & 1) ? 1 : -1), C->ny);
                    e = (9.0 / 16.0) * uc[IDX(C, I, J, k)]
                      + (3.0 / 16.0) * uc[IDX(C, I2, J, k)]
                      + (3.0 / 16.0) * uc[IDX(C, I, J2, k)]
                      + (1.0 / 16.0) * uc[IDX(C, I2, J2, k)];
                }
                u[IDX(F, i, j, k)] += e;
            }
}

/* ---------------------------------------------------------------------- */
/* hierarchy                                                               */
/* ---------------------------------------------------------------------- */
static int can_halve(int n) { return (n % 2 == 0) && ((n / 2) % 2 == 0 || n / 2 == 1); }

/* Standard depth: halve both horizontal sizes while both are even and each
 * half is even or 1 (red/black colouring needs even periodic sizes). */
int orc_standard_levels(int nx, int ny)
{
    int L = 1;
    while (can_halve(nx) && can_halve(ny)) {
        nx /= 2; ny /= 2; L++;
    }
    return L;
}

static int mg_levels(const orc_mg *mg)
{
    int Ls = orc_standard_levels(mg->g.nx, mg->g.ny);
    if (mg->n_levels <= 0) return Ls;
    return mg->n_levels <= Ls ? mg->n_levels : -1;
}

typedef struct {
    int L;
    level_t *lev;
    double **b, **u, **r;
} hier_t;

static int hier_init(hier_t *H, const orc_mg *mg)
{
    int L = mg_levels(mg);
    if (L <= 0) return -1;
    H->L = L;
    H->lev = (level_t *)calloc(L, sizeof(level_t));
    H->b = (double **)calloc(L, sizeof(double *));
    H->u = (double **)calloc(L, sizeof(double *));
    H->r = (double **)calloc(L, sizeof(double *));
    for (int l = 0; l < L; l++) {
        int f = 1 << l;
        level_init(&H->lev[l], mg->g.nx / f, mg->g.ny / f, mg->g.nz, mg->g.hx * f, mg->g.hy * f,
                   mg->g.omega2, mg->g.dz, mg->g.lambda2);
        if (mg->g.tz3) {
            if (l == 0) {
                level_set_tz3(&H->lev[0], mg->g.tz3);
            } else {
                const level_t *F = &H->lev[l - 1];
                level_t *C = &H->lev[l];
                C->Tz3 = (double *)malloc(sizeof(double) * (size_t)(C->nz + 1) * C->ny * C->nx);
                orc_tz3_coarsen(F->nx, F->ny, F->nz, F->Tz3, C->Tz3);
            }
        }
        size_t n = (size_t)H->lev[l].nx * H->lev[l].ny * H->lev[l].nz;
        H->r[l] = (double *)malloc(sizeof(double) * n);
        if (l > 0) {
            H->b[l] = (double *)malloc(sizeof(double) * n);
            H->u[l] = (double *)malloc(sizeof(double) * n);
        }
    }
    return 0;
}

static void hier_free(hier_t *H)
{
    for (int l = 0; l < H->L; l++) {
        level_free(&H->lev[l]);
        free(H->r[l]);
        if (l > 0) { free(H->b[l]); free(H->u[l]); }
    }
    free(H->lev); free(H->b); free(H->u); free(H->r);
}

static size_t level_n(const level_t *L) { return (size_t)L->nx * L->ny * L->nz; }

static void residual(const level_t *L, const double *b, const double *u, double *r)
{
    size_t n = level_n(L);
    apply_level(L, u, r);
    for (size_t c = 0; c < n; c++) r[c] = b[c] - r[c];
}

static void smooth(const level_t *L, int sweeps, int first, double rho, const double *b, double *u)
{
    for (int s = 0; s < sweeps; s++) {
        smooth_colour(L, first, rho, b, u);
        smooth_colour(L, 1 - first, rho, b, u);
    }
}

/* Multigrid V-cycle (Sec. 4.3, Alg. "Multigrid V-cycle"), started from u = 0. */
static void vcycle_rec(hier_t *H, const orc_mg *mg, int l, const double *b, double *u)
{
    const level_t *Lv = &H->lev[l];
    memset(u, 0, sizeof(double) * level_n(Lv));
    if (l == H->L - 1) {
        if (mg->nu_coarse > 0) {
            smooth(Lv, mg->nu_coarse, 0, mg->rho, b, u);
        } else {
            /* no coarse sweeps: the level is smoothed like a finer one without a
             * coarser correction, red-black then black-red sweeps; on a one-level
             * hierarchy with one sweep each this is the block red/black SSOR
             * line-relaxation preconditioner of the one-level CG solver
             * (Sec. 6.1 and Sec. 7.2, Table 2) */
            smooth(Lv, mg->nu_pre, 0, mg->rho, b, u);
            smooth(Lv, mg->nu_post, 1, mg->rho, b, u);
        }
        return;
    }
    smooth(Lv, mg->nu_pre, 0, mg->rho, b, u);                 /* pre-smoothing   */
    residual(Lv, b, u, H->r[l]);                              /* residual        */
    restrict_sum(Lv, &H->lev[l + 1], H->r[l], H->b[l + 1]);   /* restriction     */
    vcycle_rec(H, mg, l + 1, H->b[l + 1], H->u[l + 1]);       /* coarse problem  */
    prolong_add(Lv, &H->lev[l + 1], mg->prolong, H->u[l + 1], u); /* correction  */
    smooth(Lv, mg->nu_post, 1, mg->rho, b, u);                /* post-smoothing  */
}

/* ---------------------------------------------------------------------- */
/* exported single-level operations (used by the tests)                    */
/* ---------------------------------------------------------------------- */
static void geom_level(level_t *L, const orc_geom *g)
{
    level_init(L, g->nx, g->ny, g->nz, g->hx, g->hy, g->omega2, g->dz, g->lambda2);
    if (g->tz3) level_set_tz3(L, g->tz3);
}

void orc_apply(const orc_geom *g, const double *x, double *y)
{
    level_t L; geom_level(&L, g); apply_level(&L, x, y); level_free(&L);
}

void orc_apply_abs(const orc_geom *g, const double *x, double *y)
{
    level_t L; geom_level(&L, g); apply_abs_level(&L, x, y); level_free(&L);
}

void orc_smooth_colour(const orc_geom *g, int colour, double rho, const double *b, double *u)
{
    level_t L; geom_level(&L, g); smooth_colour(&L, colour, rho, b, u); level_free(&L);
}

void orc_residual(const orc_geom *g, const double *b, const double *u, double *r)
{
    level_t L; geom_level(&L, g); residual(&L, b, u, r); level_free(&L);
}

/* fine geometry g; the coarse grid is nx/2 x ny/2 */
void orc_restrict(const orc_geom *g, const double *r, double *bc)
{
    level_t F, C;
    geom_level(&F, g);
    level_init(&C, g->nx / 2, g->ny / 2, g->nz, 2 * g->hx, 2 * g->hy, g->omega2, g->dz, g->lambda2);
    restrict_sum(&F, &C, r, bc);
    level_free(&F); level_free(&C);
}

void orc_prolong_add(const orc_geom *g, int mode, const double *uc, double *u)
{
    level_t F, C;
    geom_level(&F, g);
    level_init(&C, g->nx / 2, g->ny / 2, g->nz, 2 * g->hx, 2 * g->hy, g->omega2, g->dz, g->lambda2);
    prolong_add(&F, &C, mode, uc, u);
    level_free(&F); level_free(&C);
}

int orc_num_levels(const orc_mg *mg) { return mg_levels(mg); }

/* z = M^{-1} r: one V-cycle from a zero initial guess with b_0 = r. */
int orc_vcycle(const orc_mg *mg, const double *r, double *z)
{
    hier_t H;
    if (hier_init(&H, mg) != 0) return -1;
    vcycle_rec(&H, mg, 0, r, z);
    hier_free(&H);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* preconditioned CG (Appendix B, Alg. "Preconditioned Conjugate Gradient */
/* method"), solving A u = V f                                             */
/* ---------------------------------------------------------------------- */
static double dot(size_t n, const double *x, const double *y)
{
    double s = 0.0;
    for (size_t c = 0; c < n; c++) s += x[c] * y[c];
    return s;
}

int orc_pcg(const orc_mg *mg, const orc_opts *opt, const double *f, double *u, orc_stats *st)
{
    hier_t H;
    if (hier_init(&H, mg) != 0) return -1;
    const level_t *L0 = &H.lev[0];
    const int nx = L0->nx, ny = L0->ny, nz = L0->nz;
    size_t n = level_n(L0);
    double *b = (double *)malloc(sizeof(double) * n);
    double *r = (double *)malloc(sizeof(double) * n);
    double *z = (double *)malloc(sizeof(double) * n);
    double *p = (double *)malloc(sizeof(double) * n);
    double *q = (double *)malloc(sizeof(double) * n);

    /* right-hand side of the integrated equation: b = V f */
    for (int k = 0; k < nz; k++)
        for (size_t c = (size_t)k * nx * ny; c < (size_t)(k + 1) * nx * ny; c++) b[c] = L0->V[k] * f[c];

    memset(st, 0, sizeof(*st));
    residual(L0, b, u, r);                         /* r_0 = b - A u_0 */
    double r0 = sqrt(dot(n, r, r));
    double bn = sqrt(dot(n, b, b));
    st->r0_norm = r0;
    st->b_norm = bn;
    st->r_norm = r0;
    int status = 1;
    int K = 0;
    double ref = opt->rel_to_rhs ? bn : r0;
    if (!isfinite(r0)) {
        status = -4;
    } else if (r0 == 0.0 || r0 < opt->atol || r0 < opt->rtol * ref) {
        status = 0;   /* nothing to do: u_0 already solves the system */
    } else {
        vcycle_rec(&H, mg, 0, r, z);               /* z_0 = M^{-1} r_0 */
        memcpy(p, z, sizeof(double) * n);          /* p_0 = z_0        */
        double kappa_old = dot(n, r, z);
        for (K = 1; K <= opt->maxiter; K++) {
            apply_level(L0, p, q);                 /* q = A p          */
            double alpha = kappa_old / dot(n, p, q);
            if (!isfinite(alpha)) { status = -4; break; }
            for (size_t c = 0; c < n; c++) u[c] += alpha * p[c];
            for (size_t c = 0; c < n; c++) r[c] -= alpha * q[c];
            double rn = sqrt(dot(n, r, r));
            st->r_norm = rn;
            if (!isfinite(rn)) { status = -4; break; }
            if (rn < opt->rtol * ref || rn < opt->atol) { status = 0; break; }
            if (K == opt->maxiter) break;
            vcycle_rec(&H, mg, 0, r, z);           /* z = M^{-1} r     */
            double kappa = dot(n, r, z);
            double beta;
            if (opt->flexible) beta = -alpha * dot(n, z, q) / kappa_old;
            else beta = kappa / kappa_old;
            if (!isfinite(beta)) { status = -4; break; }
            for (size_t c = 0; c < n; c++) p[c] = z[c] + beta * p[c];
            kappa_old = kappa;
        }
        if (K > opt->maxiter) K = opt->maxiter;
    }
    st->iters = K;
    st->status = status;
    residual(L0, b, u, q);                         /* true residual    */
    st->true_r_norm = sqrt(dot(n, q, q));
    free(b); free(r); free(z); free(p); free(q);
    hier_free(&H);
    return 0;
}

/* Stand-alone multigrid (Sec. 4.3, the V-cycle iterated as a solver; Sec. 7.3):
 * u_K = u_{K-1} + z_K, z_K one V-cycle from zero applied to r_{K-1} (the V-cycle
 * is linear in (b, u), so this is the V-cycle started from the current
 * iterate).  The residual is carried by the recurrence r_K = r_{K-1} - A z_K,
 * equal to b - A u_K in exact arithmetic (recomputing b - A u has a rounding
 * floor far above 1e-5 on strongly graded grids).  Stopping as in Alg. PCG. */
int orc_mg_solve(const orc_mg *mg, const orc_opts *opt, const double *f, double *u, orc_stats *st)
{
    hier_t H;
    if (hier_init(&H, mg) != 0) return -1;
    const level_t *L0 = &H.lev[0];
    const int nx = L0->nx, ny = L0->ny, nz = L0->nz;
    size_t n = level_n(L0);
    double *b = (double *)malloc(sizeof(double) * n);
    double *r = (double *)malloc(sizeof(double) * n);
    double *z = (double *)malloc(sizeof(double) * n);
    double *q = (double *)malloc(sizeof(double) * n);
    for (int k = 0; k < nz; k++)
        for (size_t c = (size_t)k * nx * ny; c < (size_t)(k + 1) * nx * ny; c++) b[c] = L0->V[k] * f[c];
    memset(st, 0, sizeof(*st));
    residual(L0, b, u, r);
    double r0 = sqrt(dot(n, r, r));
    double bn = sqrt(dot(n, b, b));
    st->r0_norm = r0;
    st->b_norm = bn;
    st->r_norm = r0;
    int status = 1;
    int K = 0;
    double ref = opt->rel_to_rhs ? bn : r0;
    if (!isfinite(r0)) {
        status = -4;
    } else if (r0 == 0.0 || r0 < opt->atol || r0 < opt->rtol * ref) {
        status = 0;
    } else {
        for (K = 1; K <= opt->maxiter; K++) {
            vcycle_rec(&H, mg, 0, r, z);           /* z = M^{-1} r      */
            apply_level(L0, z, q);                 /* q = A z           */
            for (size_t c = 0; c < n; c++) u[c] += z[c];
            for (size_t c = 0; c < n; c++) r[c] -= q[c];
            double rn = sqrt(dot(n, r, r));
            st->r_norm = rn;
            if (!isfinite(rn)) { status = -4; break; }
            if (rn < opt->rtol * ref || rn < opt->atol) { status = 0; break; }
        }
        if (K > opt->maxiter) K = opt->maxiter;
    }
    st->iters = K;
    st->status = status;
    residual(L0, b, u, q);
    st->true_r_norm = sqrt(dot(n, q, q));
    free(b); free(r); free(z); free(q);
    hier_free(&H);
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
