/*
 * oracle.c -- plain FP64 CPU reference ("the oracle") for the matrix-free
 * two-level deflation preconditioner of Chen, Dwarka & Vuik (arXiv 2308.06152).
 *
 * TEST INFRASTRUCTURE ONLY: tests/, the smoke check and the CPU-baseline leg of
 * the benchmark are the only callers.  Nothing here is shared with, or called
 * by, the HIP product library.
 *
 * Style: plain loops over the (i,j) grid, one step of the method per function,
 * no fusion, no blocking, no caching between calls.  Each function names the
 * passage of the paper it follows.  Readings of passages that are silent or
 * ambiguous are marked "Reading:".
 *
 * Conventions
 *   node (i,j), i = 0..nx-1 (x, fastest), j = 0..ny-1; array index j*nx + i.
 *   Dirichlet boundaries are homogeneous and eliminated: boundary nodes are not
 *   unknowns, every operator writes 0 there and never reads them.
 *   Sommerfeld boundaries: every node is an unknown.
 *   Inner product (a, b) = sum conj(b) a (the paper's h_ij = (w, v_i)).
 */
#include "oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* Loops whose iterations write disjoint outputs (one grid row, or one vector
 * entry, each) may be split over OpenMP threads; the arithmetic of every
 * output is the same either way. */
#ifdef _OPENMP
#include <omp.h>
#define ORA_PARFOR _Pragma("omp parallel for schedule(static)")
#else
#define ORA_PARFOR
#endif

/* the imaginary unit; the single-letter macro of complex.h is released so that
 * I, J can name coarse-grid indices as in the paper */
#define IU _Complex_I
#undef I

#define ORA_OK 0
#define ORA_EINVAL (-1)
#define ORA_EGRID (-2)
#define ORA_ENOMEM (-3)

#define MAXLEV 40

/* ------------------------------------------------------------------------- */
/* Grid levels                                                               */
/* ------------------------------------------------------------------------- */

typedef struct {
    int nx, ny, bc;
    double hx, hy;
    double *k; /* wavenumber per node, owned */
} lvl_t;

typedef struct {
    int nlev;
    lvl_t L[MAXLEV];
} hier_t;

/* A level is coarsened (standard coarsening, h -> 2h, coarse (I,J) sits on fine
 * (2I,2J); Section 4, parallel multigrid) while both point counts are odd and
 * at least 5.  Section 4 stops coarsening at a manually predefined coarsest
 * grid and solves the problem there: levels beyond the first coarse one are
 * only made while the current level has more than coarsest_nodes nodes
 * (0 = coarsen as far as possible).  The deflation coarse grid (level 1) is
 * always made. */
static int coarsenable(int nx, int ny) { return nx >= 5 && ny >= 5 && (nx & 1) && (ny & 1); }

int ora_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void ora_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int ora_num_levels(int nx, int ny, int coarsest_nodes)
{
    int n = 1;
    while (coarsenable(nx, ny) && n < MAXLEV &&
           (n == 1 || (long)nx * (long)ny > (long)coarsest_nodes)) {
        nx = (nx + 1) / 2;
        ny = (ny + 1) / 2;
        n++;
    }
    return n;
}

int ora_level_dims(int nx, int ny, int coarsest_nodes, int l, int *lnx, int *lny)
{
    if (l < 0 || l >= ora_num_levels(nx, ny, coarsest_nodes)) return ORA_EINVAL;
    for (int q = 0; q < l; q++) {
        nx = (nx + 1) / 2;
        ny = (ny + 1) / 2;
    }
    *lnx = nx;
    *lny = ny;
    return ORA_OK;
}

static size_t npts(const lvl_t *g) { return (size_t)g->nx * (size_t)g->ny; }

static int is_bnd(const lvl_t *g, int i, int j)
{
    return i == 0 || j == 0 || i == g->nx - 1 || j == g->ny - 1;
}

static int is_unknown(const lvl_t *g, int i, int j)
{
    return g->bc == ORA_BC_SOMMERFELD || !is_bnd(g, i, j);
}

static void free_hier(hier_t *H)
{
    for (int l = 0; l < H->nlev; l++) free(H->L[l].k);
    H->nlev = 0;
}

/* Coarse-grid parameters follow from the fine grid (Section 4): spacing doubles
 * and the wavenumber is taken from the coincident fine node.
 * Reading: "determined by the fine grid" is read as injection. */
static int build_hier(const ora_problem *p, hier_t *H)
{
    memset(H, 0, sizeof(*H));
    if (!p || p->nx < 3 || p->ny < 3 || !(p->hx > 0) || !(p->hy > 0)) return ORA_EINVAL;
    if (p->bc != ORA_BC_DIRICHLET && p->bc != ORA_BC_SOMMERFELD) return ORA_EINVAL;
    if (p->coarsest_nodes < 0) return ORA_EINVAL;
    H->nlev = ora_num_levels(p->nx, p->ny, p->coarsest_nodes);
    for (int l = 0; l < H->nlev; l++) {
        lvl_t *g = &H->L[l];
        if (l == 0) {
            g->nx = p->nx;
            g->ny = p->ny;
            g->hx = p->hx;
            g->hy = p->hy;
        } else {
            g->nx = (H->L[l - 1].nx + 1) / 2;
            g->ny = (H->L[l - 1].ny + 1) / 2;
            g->hx = 2.0 * H->L[l - 1].hx;
            g->hy = 2.0 * H->L[l - 1].hy;
        }
        g->bc = p->bc;
        g->k = (double *)malloc(npts(g) * sizeof(double));
        if (!g->k) {
            free_hier(H);
            return ORA_ENOMEM;
        }
        for (int j = 0; j < g->ny; j++)
            for (int i = 0; i < g->nx; i++) {
                double kv;
                if (l == 0)
                    kv = p->k ? p->k[(size_t)j * p->nx + i] : p->kconst;
                else
                    kv = H->L[l - 1].k[(size_t)(2 * j) * H->L[l - 1].nx + 2 * i];
                g->k[(size_t)j * g->nx + i] = kv;
            }
    }
    return ORA_OK;
}

/* ------------------------------------------------------------------------- */
/* 5-point operators: A_h (shift 1) and the CSLP M_h (shift beta)            */
/* ------------------------------------------------------------------------- */

/* Multipliers ap, aw, ae, as, an of node (i,j) for  -Lap_h - s*k^2  (the
 * discrete Helmholtz stencil, Section 2.1, and the CSLP stencil, Section 3.1
 * with the matrix-free multipliers of Section 5.1).
 * Sommerfeld: the ghost node outside a boundary node is eliminated with the
 * central-difference radiation condition u_ghost = u_inward + 2 i h k u_bnd
 * (Section 2.1), which gives -2ik/h on the diagonal and doubles the inward
 * coupling; corners do this in both directions.
 * Reading: the CSLP takes the same boundary closure with the unshifted k.
 * Dirichlet: neighbours on the boundary hold 0 and contribute nothing. */
static void stencil5(const lvl_t *g, cplx s, int i, int j, cplx c[5])
{
    const double kk = g->k[(size_t)j * g->nx + i];
    const double ihx2 = 1.0 / (g->hx * g->hx), ihy2 = 1.0 / (g->hy * g->hy);
    cplx ap = 2.0 * ihx2 + 2.0 * ihy2 - s * kk * kk;
    cplx aw = -ihx2, ae = -ihx2, as = -ihy2, an = -ihy2;
    if (g->bc == ORA_BC_SOMMERFELD) {
        if (i == 0) {
            ap += -2.0 * IU * kk / g->hx;
            ae += aw;
            aw = 0;
        }
        if (i == g->nx - 1) {
            ap += -2.0 * IU * kk / g->hx;
            aw += ae;
            ae = 0;
        }
        if (j == 0) {
            ap += -2.0 * IU * kk / g->hy;
            an += as;
            as = 0;
        }
        if (j == g->ny - 1) {
            ap += -2.0 * IU * kk / g->hy;
            as += an;
            an = 0;
        }
    } else {
        if (i - 1 == 0) aw = 0;
        if (i + 1 == g->nx - 1) ae = 0;
        if (j - 1 == 0) as = 0;
        if (j + 1 == g->ny - 1) an = 0;
    }
    c[0] = ap;
    c[1] = aw;
    c[2] = ae;
    c[3] = as;
    c[4] = an;
}

/* y = (-Lap_h - s k^2) x  (the matrix-free matvec of Section 5.1). */
static void op5(const lvl_t *g, cplx s, const cplx *x, cplx *y)
{
    ORA_PARFOR
    for (int j = 0; j < g->ny; j++)
        for (int i = 0; i < g->nx; i++) {
            size_t p = (size_t)j * g->nx + i;
            if (!is_unknown(g, i, j)) {
                y[p] = 0;
                continue;
            }
            cplx c[5];
            stencil5(g, s, i, j, c);
            cplx v = c[0] * x[p];
            if (c[1] != 0) v += c[1] * x[p - 1];
            if (c[2] != 0) v += c[2] * x[p + 1];
            if (c[3] != 0) v += c[3] * x[p - g->nx];
            if (c[4] != 0) v += c[4] * x[p + g->nx];
            y[p] = v;
        }
}

static cplx beta_of(const ora_problem *p) { return p->beta_re + IU * p->beta_im; }

/* ------------------------------------------------------------------------- */
/* Inter-grid transfers                                                      */
/* ------------------------------------------------------------------------- */

/* 1D interpolation weight from coarse node I to fine node i, d = i - 2I.
 * Linear (Section 3.2): even fine nodes copy, odd fine nodes average.
 * Higher order (Bezier, Section 3.2.1): even fine nodes take
 * (u_{I-1} + 6 u_I + u_{I+1})/8, odd ones average the two neighbours. */
static double w_linear(int d)
{
    if (d == 0) return 1.0;
    if (d == 1 || d == -1) return 0.5;
    return 0.0;
}

static double w_bezier(int d)
{
    if (d == 0) return 0.75;
    if (d == 1 || d == -1) return 0.5;
    if (d == 2 || d == -2) return 0.125;
    return 0.0;
}

typedef double (*w1d_t)(int);

/* vf = I_{2h}^h vc with the tensor-product weights w(i-2I) w(j-2J)
 * (2D stencils of Section 3.2 and the matrix-free prolongation of 3.2.1).
 * Coarse nodes outside the grid, and non-unknown coarse nodes, contribute 0;
 * non-unknown fine nodes are 0. */
static void prolong(const lvl_t *gf, const lvl_t *gc, w1d_t w, const cplx *vc, cplx *vf)
{
    ORA_PARFOR
    for (int j = 0; j < gf->ny; j++)
        for (int i = 0; i < gf->nx; i++) {
            size_t p = (size_t)j * gf->nx + i;
            if (!is_unknown(gf, i, j)) {
                vf[p] = 0;
                continue;
            }
            cplx s = 0;
            for (int J = j / 2 - 2; J <= j / 2 + 2; J++) {
                if (J < 0 || J >= gc->ny) continue;
                double wy = w(j - 2 * J);
                if (wy == 0) continue;
                for (int I = i / 2 - 2; I <= i / 2 + 2; I++) {
                    if (I < 0 || I >= gc->nx) continue;
                    if (!is_unknown(gc, I, J)) continue;
                    double wx = w(i - 2 * I);
                    if (wx == 0) continue;
                    s += wx * wy * vc[(size_t)J * gc->nx + I];
                }
            }
            vf[p] = s;
        }
}

/* vc = (I_{2h}^h)^T vf: the exact transpose of prolong() (for the Bezier
 * weights this is the [1 4 6 4 1]/8 tensor restriction of Section 3.2.1; for
 * the linear weights it is 1/2 [1 2 1] per axis). */
static void restrict_t(const lvl_t *gf, const lvl_t *gc, w1d_t w, const cplx *vf, cplx *vc)
{
    ORA_PARFOR
    for (int J = 0; J < gc->ny; J++)
        for (int I = 0; I < gc->nx; I++) {
            size_t P = (size_t)J * gc->nx + I;
            if (!is_unknown(gc, I, J)) {
                vc[P] = 0;
                continue;
            }
            cplx s = 0;
            for (int j = 2 * J - 2; j <= 2 * J + 2; j++) {
                if (j < 0 || j >= gf->ny) continue;
                double wy = w(j - 2 * J);
                if (wy == 0) continue;
                for (int i = 2 * I - 2; i <= 2 * I + 2; i++) {
                    if (i < 0 || i >= gf->nx) continue;
                    if (!is_unknown(gf, i, j)) continue;
                    double wx = w(i - 2 * I);
                    if (wx == 0) continue;
                    s += wx * wy * vf[(size_t)j * gf->nx + i];
                }
            }
            vc[P] = s;
        }
}

/* Full-weighting restriction 1/16 [1 2 1; 2 4 2; 1 2 1] (Section 3.2).
 * Reading: at the boundary it is taken as 1/4 of the transpose of bilinear
 * interpolation, i.e. the same stencil truncated to the grid. */
static void fw_restrict(const lvl_t *gf, const lvl_t *gc, const cplx *vf, cplx *vc)
{
    restrict_t(gf, gc, w_linear, vf, vc);
    ORA_PARFOR
    for (size_t q = 0; q < npts(gc); q++) vc[q] *= 0.25;
}

/* ------------------------------------------------------------------------- */
/* Banded LU with partial pivoting (direct solves)                          */
/* ------------------------------------------------------------------------- */

typedef struct {
    int n, kl, ku, ld;
    cplx *a;  /* row r holds columns r-kl .. r+kl+ku at a[r*ld + (c - r + kl)] */
    int *piv;
} band_t;

static cplx *bel(band_t *B, int r, int c) { return &B->a[(size_t)r * B->ld + (c - r + B->kl)]; }

static int band_alloc(band_t *B, int n, int kl, int ku)
{
    B->n = n;
    B->kl = kl;
    B->ku = ku;
    B->ld = 2 * kl + ku + 1;
    B->a = (cplx *)calloc((size_t)n * B->ld, sizeof(cplx));
    B->piv = (int *)calloc((size_t)n, sizeof(int));
    if (!B->a || !B->piv) {
        free(B->a);
        free(B->piv);
        return ORA_ENOMEM;
    }
    return ORA_OK;
}

static void band_free(band_t *B)
{
    free(B->a);
    free(B->piv);
}

/* Gaussian elimination with row partial pivoting on a band matrix
 * (textbook band LU; the upper bandwidth grows to kl+ku). */
static void band_factor(band_t *B)
{
    const int n = B->n, kl = B->kl, ku = B->ku;
    for (int c = 0; c < n; c++) {
        int last = c + kl < n - 1 ? c + kl : n - 1;
        int p = c;
        double best = cabs(*bel(B, c, c));
        for (int r = c + 1; r <= last; r++) {
            double v = cabs(*bel(B, r, c));
            if (v > best) {
                best = v;
                p = r;
            }
        }
        B->piv[c] = p;
        int cend = c + kl + ku < n - 1 ? c + kl + ku : n - 1;
        if (p != c)
            for (int q = c; q <= cend; q++) {
                cplx t = *bel(B, c, q);
                *bel(B, c, q) = *bel(B, p, q);
                *bel(B, p, q) = t;
            }
        cplx d = *bel(B, c, c);
        if (d == 0) continue; /* singular: leaves a zero pivot, solve yields inf */
        for (int r = c + 1; r <= last; r++) {
            cplx l = *bel(B, r, c) / d;
            *bel(B, r, c) = l;
            if (l == 0) continue;
            for (int q = c + 1; q <= cend; q++) *bel(B, r, q) -= l * *bel(B, c, q);
        }
    }
}

static void band_solve(band_t *B, cplx *x)
{
    const int n = B->n, kl = B->kl, ku = B->ku;
    for (int c = 0; c < n; c++) {
        int p = B->piv[c];
        if (p != c) {
            cplx t = x[c];
            x[c] = x[p];
            x[p] = t;
        }
        int last = c + kl < n - 1 ? c + kl : n - 1;
        for (int r = c + 1; r <= last; r++) x[r] -= *bel(B, r, c) * x[c];
    }
    for (int c = n - 1; c >= 0; c--) {
        int cend = c + kl + ku < n - 1 ? c + kl + ku : n - 1;
        cplx s = x[c];
        for (int q = c + 1; q <= cend; q++) s -= *bel(B, c, q) * x[q];
        x[c] = s / *bel(B, c, c);
    }
}

/* Generic grid operator, for probing into band form. */
typedef void (*gridop_t)(const void *ctx, const cplx *x, cplx *y);

/* Assemble the matrix of a grid operator of stencil reach (rx, ry) by probing
 * it with the (2rx+1)(2ry+1) colour classes of unit vectors, then factor it.
 * Rows of non-unknown nodes (Dirichlet boundary) become identity rows. */
static int band_from_op(const lvl_t *g, int rx, int ry, gridop_t op, const void *ctx, band_t *B)
{
    const int nx = g->nx, ny = g->ny, n = nx * ny;
    const int bw = ry * nx + rx;
    int rc = band_alloc(B, n, bw, bw);
    if (rc) return rc;
    cplx *e = (cplx *)malloc((size_t)n * sizeof(cplx));
    cplx *y = (cplx *)malloc((size_t)n * sizeof(cplx));
    if (!e || !y) {
        free(e);
        free(y);
        band_free(B);
        return ORA_ENOMEM;
    }
    const int px = 2 * rx + 1, py = 2 * ry + 1;
    for (int cy = 0; cy < py; cy++)
        for (int cx = 0; cx < px; cx++) {
            for (int j = 0; j < ny; j++)
                for (int i = 0; i < nx; i++)
                    e[j * nx + i] = (i % px == cx && j % py == cy && is_unknown(g, i, j)) ? 1.0 : 0.0;
            op(ctx, e, y);
            for (int j = 0; j < ny; j++)
                for (int i = 0; i < nx; i++) {
                    if (!is_unknown(g, i, j)) continue;
                    /* the unique column of this colour within reach of (i,j) */
                    int ic = i - ((i - cx) % px + px) % px;
                    if (i - ic > rx) ic += px;
                    int jc = j - ((j - cy) % py + py) % py;
                    if (j - jc > ry) jc += py;
                    if (ic < 0 || ic >= nx || jc < 0 || jc >= ny) continue;
                    if (!is_unknown(g, ic, jc)) continue;
                    *bel(B, j * nx + i, jc * nx + ic) = y[j * nx + i];
                }
        }
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++)
            if (!is_unknown(g, i, j)) *bel(B, j * nx + i, j * nx + i) = 1.0;
    free(e);
    free(y);
    band_factor(B);
    return ORA_OK;
}

typedef struct {
    const lvl_t *g;
    cplx s;
} op5ctx_t;

static void op5_cb(const void *ctx, const cplx *x, cplx *y)
{
    const op5ctx_t *c = (const op5ctx_t *)ctx;
    op5(c->g, c->s, x, y);
}

/* x = (op)^{-1} b on level g; b is copied, non-unknown entries are zeroed. */
static int direct_solve_op(const lvl_t *g, int rx, int ry, gridop_t op, const void *ctx,
                           const cplx *b, cplx *x)
{
    band_t B;
    int rc = band_from_op(g, rx, ry, op, ctx, &B);
    if (rc) return rc;
    for (int j = 0; j < g->ny; j++)
        for (int i = 0; i < g->nx; i++) {
            size_t p = (size_t)j * g->nx + i;
            x[p] = is_unknown(g, i, j) ? b[p] : 0;
        }
    band_solve(&B, x);
    band_free(&B);
    return ORA_OK;
}

/* ------------------------------------------------------------------------- */
/* Multigrid V-cycle for the CSLP (Section 3.1, Section 5.1)                 */
/* ------------------------------------------------------------------------- */

/* One damped-Jacobi sweep x <- x + omega D^{-1} (r - M x), D = diag(M). */
static void jacobi(const lvl_t *g, cplx s, double omega, const cplx *r, cplx *x, cplx *t)
{
    op5(g, s, x, t);
    ORA_PARFOR
    for (int j = 0; j < g->ny; j++)
        for (int i = 0; i < g->nx; i++) {
            size_t p = (size_t)j * g->nx + i;
            if (!is_unknown(g, i, j)) {
                x[p] = 0;
                continue;
            }
            cplx c[5];
            stencil5(g, s, i, j, c);
            x[p] += omega * (r[p] - t[p]) / c[0];
        }
}

/* x = V_l(r): one V-cycle on level l for M re-discretised on every level
 * (Section 5.1): nu_pre damped-Jacobi sweeps from x = 0, residual, full
 * weighting, recursion, bilinear correction, nu_post sweeps.
 * Reading: the coarsest level is solved exactly (the paper runs GMRES to
 * 1e-8 there); x starts from 0 on every level. */
static int vcycle_rec(const hier_t *H, const ora_problem *p, int l, const cplx *r, cplx *x)
{
    const lvl_t *g = &H->L[l];
    const cplx s = beta_of(p);
    const size_t n = npts(g);
    if (l == H->nlev - 1) {
        op5ctx_t c = {g, s};
        return direct_solve_op(g, 1, 1, op5_cb, &c, r, x);
    }
    const lvl_t *gc = &H->L[l + 1];
    const size_t nc = npts(gc);
    cplx *t = (cplx *)malloc(n * sizeof(cplx));
    cplx *rc = (cplx *)malloc(nc * sizeof(cplx));
    cplx *ec = (cplx *)malloc(nc * sizeof(cplx));
    cplx *pe = (cplx *)malloc(n * sizeof(cplx));
    if (!t || !rc || !ec || !pe) {
        free(t);
        free(rc);
        free(ec);
        free(pe);
        return ORA_ENOMEM;
    }
    ORA_PARFOR
    for (size_t q = 0; q < n; q++) x[q] = 0;
    for (int it = 0; it < p->nu_pre; it++) jacobi(g, s, p->omega, r, x, t);
    op5(g, s, x, t);
    ORA_PARFOR
    for (size_t q = 0; q < n; q++) t[q] = r[q] - t[q];
    fw_restrict(g, gc, t, rc);
    int rcode = vcycle_rec(H, p, l + 1, rc, ec);
    if (!rcode) {
        prolong(g, gc, w_linear, ec, pe);
        ORA_PARFOR
        for (size_t q = 0; q < n; q++) x[q] += pe[q];
        for (int it = 0; it < p->nu_post; it++) jacobi(g, s, p->omega, r, x, t);
    }
    free(t);
    free(rc);
    free(ec);
    free(pe);
    return rcode;
}

/* ------------------------------------------------------------------------- */
/* Coarse-grid operators (Section 5.2)                                        */
/* ------------------------------------------------------------------------- */

static w1d_t zweights(const ora_problem *p) { return p->defl_vectors == ORA_Z_LINEAR ? w_linear : w_bezier; }

/* Galerkin Laplacian stencil of the ReD-Glk scheme, as printed in Section
 * 5.2.4: multiply by 1/((2h)^2 * 256). Row index dJ+2 (y), column dI+2 (x);
 * the stencil is symmetric so the orientation does not matter. */
static const double GLK_LAP[5][5] = {
    {-3, -44, -98, -44, -3},
    {-44, -112, 56, -112, -44},
    {-98, 56, 980, 56, -98},
    {-44, -112, 56, -112, -44},
    {-3, -44, -98, -44, -3},
};
/* Galerkin wavenumber stencil of the ReD-Glk scheme (Section 5.2.4):
 * multiply by k^2 / 64^2. */
static const double GLK_K2[5][5] = {
    {1, 28, 70, 28, 1},
    {28, 784, 1960, 784, 28},
    {70, 1960, 4900, 1960, 70},
    {28, 784, 1960, 784, 28},
    {1, 28, 70, 28, 1},
};

typedef struct {
    const hier_t *H;
    const ora_problem *p;
} cctx_t;

/* str-Glk (Section 5.2.1): A_2h x = Z^T (A_h (Z x)), three passes. */
static void coarse_galerkin(const hier_t *H, const ora_problem *p, const cplx *x, cplx *y)
{
    const lvl_t *gf = &H->L[0], *gc = &H->L[1];
    cplx *a = (cplx *)malloc(npts(gf) * sizeof(cplx));
    cplx *b = (cplx *)malloc(npts(gf) * sizeof(cplx));
    if (!a || !b) { /* out of memory: poison the result */
        ORA_PARFOR
        for (size_t q = 0; q < npts(gc); q++) y[q] = NAN;
        free(a);
        free(b);
        return;
    }
    prolong(gf, gc, zweights(p), x, a);
    op5(gf, 1.0, a, b);
    restrict_t(gf, gc, zweights(p), b, y);
    free(a);
    free(b);
}

/* Value of a ghost node (I', J') outside the coarse grid in terms of grid
 * values (ReD-Glk2, Section 5.2.4).  Sommerfeld: u_ghost = u_inward +
 * 2 i H k_bnd u_bnd (Section 2.1 at spacing H); Dirichlet: the boundary value
 * is the mean of the ghost and the inward node, so u_ghost = 2 u_bnd - u_inward.
 * Reading: a ghost outside in both directions (only reached by the node next
 * to a corner) is the mean of its two neighbouring single-direction ghosts. */
static cplx ghost_x(const lvl_t *g, const cplx *u, int Ig, int J)
{
    int Ib = Ig < 0 ? 0 : g->nx - 1;
    int Iin = Ig < 0 ? 1 : g->nx - 2;
    cplx ub = is_unknown(g, Ib, J) ? u[(size_t)J * g->nx + Ib] : 0;
    cplx ui = is_unknown(g, Iin, J) ? u[(size_t)J * g->nx + Iin] : 0;
    if (g->bc == ORA_BC_SOMMERFELD) return ui + 2.0 * IU * g->hx * g->k[(size_t)J * g->nx + Ib] * ub;
    return 2.0 * ub - ui;
}

static cplx ghost_y(const lvl_t *g, const cplx *u, int I0, int Jg)
{
    int Jb = Jg < 0 ? 0 : g->ny - 1;
    int Jin = Jg < 0 ? 1 : g->ny - 2;
    cplx ub = is_unknown(g, I0, Jb) ? u[(size_t)Jb * g->nx + I0] : 0;
    cplx ui = is_unknown(g, I0, Jin) ? u[(size_t)Jin * g->nx + I0] : 0;
    if (g->bc == ORA_BC_SOMMERFELD) return ui + 2.0 * IU * g->hy * g->k[(size_t)Jb * g->nx + I0] * ub;
    return 2.0 * ub - ui;
}

static cplx ghost_value(const lvl_t *g, const cplx *u, int Ig, int Jg)
{
    int outx = Ig < 0 || Ig >= g->nx, outy = Jg < 0 || Jg >= g->ny;
    if (outx && !outy) return ghost_x(g, u, Ig, Jg);
    if (outy && !outx) return ghost_y(g, u, Ig, Jg);
    int Iin = Ig < 0 ? 0 : g->nx - 1; /* neighbour ghost moved inward in x */
    int Jin = Jg < 0 ? 0 : g->ny - 1;
    return 0.5 * (ghost_y(g, u, Iin, Jg) + ghost_x(g, u, Ig, Jin));
}

/* ReD-Glk2 (Section 5.2.4): the Galerkin 5x5 stencils used as a
 * re-discretisation on the coarse grid.  The k^2 weight of each stencil node
 * uses the wavenumber at that coarse node; ghost nodes carry k = 0 and their
 * Laplacian weight is folded in through ghost elimination; the first boundary
 * layer keeps the second-order 5-point stencil (Section 2.1) at spacing 2h,
 * as it is, with no extra factor (the same rows as ReD-O2; with this the outer
 * counts of the paper's Section 6 tables come out within one). */
static cplx row_o2(const lvl_t *g, const cplx *u, int I, int J);

static void coarse_redglk2(const hier_t *H, const cplx *u, cplx *y)
{
    const lvl_t *g = &H->L[1];
    const double H2 = g->hx * g->hx; /* (2h)^2, hx == hy checked by the caller */
    ORA_PARFOR
    for (int J = 0; J < g->ny; J++)
        for (int I0 = 0; I0 < g->nx; I0++) {
            size_t P = (size_t)J * g->nx + I0;
            if (!is_unknown(g, I0, J)) {
                y[P] = 0;
                continue;
            }
            if (is_bnd(g, I0, J)) { /* first layer, Sommerfeld only */
                y[P] = row_o2(g, u, I0, J);
                continue;
            }
            cplx v = 0;
            for (int dJ = -2; dJ <= 2; dJ++)
                for (int dI = -2; dI <= 2; dI++) {
                    int Ii = I0 + dI, Jj = J + dJ;
                    double lap = GLK_LAP[dJ + 2][dI + 2] / (256.0 * H2);
                    double kw = GLK_K2[dJ + 2][dI + 2] / 4096.0;
                    if (Ii >= 0 && Ii < g->nx && Jj >= 0 && Jj < g->ny) {
                        if (!is_unknown(g, Ii, Jj)) continue;
                        double kc = g->k[(size_t)Jj * g->nx + Ii];
                        v += (lap - kw * kc * kc) * u[(size_t)Jj * g->nx + Ii];
                    } else {
                        v += lap * ghost_value(g, u, Ii, Jj);
                    }
                }
            y[P] = v;
        }
}

/* One row of the second-order 5-point Helmholtz stencil at the coarse
 * spacing (Section 2.1, with its Sommerfeld closure) applied to u at (I, J):
 * the rows of ReD-O2, the near-boundary rows of ReD-O4 and ReD-Glk1 and the
 * first-layer rows of ReD-Glk2.  These carry no extra factor: the paper
 * re-discretises with the fine-grid stencil itself, and only without a factor
 * do the variants reproduce the outer iteration counts of its Section 6
 * tables to within one. */
static cplx row_o2(const lvl_t *g, const cplx *u, int I, int J)
{
    size_t P = (size_t)J * g->nx + I;
    cplx c[5];
    stencil5(g, 1.0, I, J, c);
    cplx v = c[0] * u[P];
    if (c[1] != 0) v += c[1] * u[P - 1];
    if (c[2] != 0) v += c[2] * u[P + 1];
    if (c[3] != 0) v += c[3] * u[P - g->nx];
    if (c[4] != 0) v += c[4] * u[P + g->nx];
    return v;
}

/* value of node (I, J), 0 at non-unknowns */
static cplx uval(const lvl_t *g, const cplx *u, int I, int J)
{
    return is_unknown(g, I, J) ? u[(size_t)J * g->nx + I] : 0;
}

/* ReD-O2 (Section 5.2.3): the fine-grid scheme re-discretised at spacing 2h
 * on every row. */
static void coarse_redo2(const hier_t *H, const cplx *u, cplx *y)
{
    const lvl_t *g = &H->L[1];
    ORA_PARFOR
    for (int J = 0; J < g->ny; J++)
        for (int I = 0; I < g->nx; I++)
            y[(size_t)J * g->nx + I] = is_unknown(g, I, J) ? row_o2(g, u, I, J) : 0;
}

/* ReD-O4 (Section 5.2.3): the Laplacian by fourth-order central differences,
 * -u'' ~ (u_{i-2} - 16 u_{i-1} + 30 u_i - 16 u_{i+1} + u_{i+2}) / (12 H^2) per
 * axis, minus k^2 u, at nodes two or more nodes inside the grid; the other
 * rows (where the wide stencil does not fit) use the second-order scheme with
 * the boundary closure.  Reading: the printed centre divides k^2 by 12, taken
 * as a typo for 60/(12 H^2) - k^2 (the consistent fourth-order scheme). */
static void coarse_redo4(const hier_t *H, const cplx *u, cplx *y)
{
    const lvl_t *g = &H->L[1];
    const double ax = 1.0 / (12.0 * g->hx * g->hx), ay = 1.0 / (12.0 * g->hy * g->hy);
    ORA_PARFOR
    for (int J = 0; J < g->ny; J++)
        for (int I = 0; I < g->nx; I++) {
            size_t P = (size_t)J * g->nx + I;
            if (!is_unknown(g, I, J)) {
                y[P] = 0;
                continue;
            }
            if (I < 2 || J < 2 || I > g->nx - 3 || J > g->ny - 3) {
                y[P] = row_o2(g, u, I, J);
                continue;
            }
            double kc = g->k[P];
            cplx lx = uval(g, u, I - 2, J) - 16.0 * uval(g, u, I - 1, J) + 30.0 * u[P] -
                      16.0 * uval(g, u, I + 1, J) + uval(g, u, I + 2, J);
            cplx ly = uval(g, u, I, J - 2) - 16.0 * uval(g, u, I, J - 1) + 30.0 * u[P] -
                      16.0 * uval(g, u, I, J + 1) + uval(g, u, I, J + 2);
            y[P] = ax * lx + ay * ly - kc * kc * u[P];
        }
}

/* ReD-Glk1 (Section 5.2.4): the Galerkin 5x5 stencils of ReD-Glk2 at nodes
 * two or more nodes inside the grid; the two boundary layers use the
 * second-order scheme (ReD-O2 rows) instead of ghost elimination. */
static void coarse_redglk1(const hier_t *H, const cplx *u, cplx *y)
{
    const lvl_t *g = &H->L[1];
    const double H2 = g->hx * g->hx; /* hx == hy checked by the caller */
    ORA_PARFOR
    for (int J = 0; J < g->ny; J++)
        for (int I = 0; I < g->nx; I++) {
            size_t P = (size_t)J * g->nx + I;
            if (!is_unknown(g, I, J)) {
                y[P] = 0;
                continue;
            }
            if (I < 2 || J < 2 || I > g->nx - 3 || J > g->ny - 3) {
                y[P] = row_o2(g, u, I, J);
                continue;
            }
            cplx v = 0;
            for (int dJ = -2; dJ <= 2; dJ++)
                for (int dI = -2; dI <= 2; dI++) {
                    int Ii = I + dI, Jj = J + dJ;
                    if (!is_unknown(g, Ii, Jj)) continue;
                    double lap = GLK_LAP[dJ + 2][dI + 2] / (256.0 * H2);
                    double kw = GLK_K2[dJ + 2][dI + 2] / 4096.0;
                    double kc = g->k[(size_t)Jj * g->nx + Ii];
                    v += (lap - kw * kc * kc) * u[(size_t)Jj * g->nx + Ii];
                }
            y[P] = v;
        }
}

static void coarse_apply_h(const hier_t *H, const ora_problem *p, const cplx *x, cplx *y)
{
    switch (p->coarse_op) {
    case ORA_COARSE_REDGLK2: coarse_redglk2(H, x, y); break;
    case ORA_COARSE_REDO2: coarse_redo2(H, x, y); break;
    case ORA_COARSE_REDO4: coarse_redo4(H, x, y); break;
    case ORA_COARSE_REDGLK1: coarse_redglk1(H, x, y); break;
    default: coarse_galerkin(H, p, x, y);
    }
}

static void coarse_cb(const void *ctx, const cplx *x, cplx *y)
{
    const cctx_t *c = (const cctx_t *)ctx;
    coarse_apply_h(c->H, c->p, x, y);
}

/* ------------------------------------------------------------------------- */
/* Krylov helpers                                                            */
/* ------------------------------------------------------------------------- */

/* Sums over a vector are taken over ORA_NCHUNK fixed contiguous chunks, each
 * summed in index order, then the chunk sums in chunk order: the same
 * rounding whether or not the chunks are summed by several threads. */
#define ORA_NCHUNK 64

static cplx dotc(size_t n, const cplx *a, const cplx *b) /* (a, b) = b^H a */
{
    cplx part[ORA_NCHUNK];
    ORA_PARFOR
    for (int c = 0; c < ORA_NCHUNK; c++) {
        const size_t q0 = n * c / ORA_NCHUNK, q1 = n * (c + 1) / ORA_NCHUNK;
        cplx s = 0;
        for (size_t q = q0; q < q1; q++) s += conj(b[q]) * a[q];
        part[c] = s;
    }
    cplx s = 0;
    for (int c = 0; c < ORA_NCHUNK; c++) s += part[c];
    return s;
}

static double nrm2(size_t n, const cplx *a)
{
    double part[ORA_NCHUNK];
    ORA_PARFOR
    for (int c = 0; c < ORA_NCHUNK; c++) {
        const size_t q0 = n * c / ORA_NCHUNK, q1 = n * (c + 1) / ORA_NCHUNK;
        double s = 0;
        for (size_t q = q0; q < q1; q++) s += creal(a[q]) * creal(a[q]) + cimag(a[q]) * cimag(a[q]);
        part[c] = s;
    }
    double s = 0;
    for (int c = 0; c < ORA_NCHUNK; c++) s += part[c];
    return sqrt(s);
}

/* Complex Givens rotation zeroing b in [a; b]: [c s; -conj(s) c]. */
static void givens(cplx a, cplx b, double *c, cplx *s)
{
    double aa = cabs(a), bb = cabs(b);
    if (bb == 0) {
        *c = 1;
        *s = 0;
        return;
    }
    if (aa == 0) {
        *c = 0;
        *s = conj(b) / bb;
        return;
    }
    double rho = sqrt(aa * aa + bb * bb);
    *c = aa / rho;
    *s = (a / aa) * conj(b) / rho;
}

/* Back substitution of the j x j upper-triangular least-squares system. */
static void backsub(int j, int ldh, const cplx *Hm, const cplx *g, cplx *y)
{
    for (int i = j - 1; i >= 0; i--) {
        cplx s = g[i];
        for (int q = i + 1; q < j; q++) s -= Hm[i * ldh + q] * y[q];
        y[i] = s / Hm[i * ldh + i];
    }
}

/* Linear operator callback on n-vectors. */
typedef int (*vop_t)(void *ctx, const cplx *x, cplx *y);

/* Restarted right-preconditioned GMRES (modified Gram-Schmidt Arnoldi,
 * Givens least squares, x = x0 + M^{-1} V y at the end of each cycle), x0 = 0.
 * fixed > 0: run exactly `fixed` iterations (no tolerance test).
 * fixed == 0: stop once |g_{j+1}| <= tol ||b|| or maxit iterations. */
static int gmres_right(size_t n, vop_t A, void *actx, vop_t Minv, void *mctx, const cplx *b,
                       cplx *x, int m, int fixed, double tol, int maxit, int *iters)
{
    const int ldh = m;
    cplx *V = (cplx *)malloc((size_t)(m + 1) * n * sizeof(cplx));
    cplx *w = (cplx *)malloc(n * sizeof(cplx));
    cplx *z = (cplx *)malloc(n * sizeof(cplx));
    cplx *Hm = (cplx *)calloc((size_t)(m + 1) * m, sizeof(cplx));
    cplx *g = (cplx *)calloc((size_t)m + 1, sizeof(cplx));
    cplx *y = (cplx *)calloc((size_t)m, sizeof(cplx));
    cplx *sn = (cplx *)calloc((size_t)m, sizeof(cplx));
    double *cs = (double *)calloc((size_t)m, sizeof(double));
    int rc = ORA_OK, it = 0;
    if (!V || !w || !z || !Hm || !g || !y || !sn || !cs) {
        rc = ORA_ENOMEM;
        goto done;
    }
    const int cap = fixed > 0 ? fixed : maxit;
    const double bnorm = nrm2(n, b);
    ORA_PARFOR
    for (size_t q = 0; q < n; q++) x[q] = 0;
    if (bnorm == 0) goto done;
    for (;;) {
        /* r = b - A x */
        if ((rc = A(actx, x, w))) goto done;
        ORA_PARFOR
        for (size_t q = 0; q < n; q++) w[q] = b[q] - w[q];
        double beta = nrm2(n, w);
        if (fixed <= 0 && beta <= tol * bnorm) break;
        if (it >= cap || beta == 0) break;
        ORA_PARFOR
        for (size_t q = 0; q < n; q++) V[q] = w[q] / beta;
        memset(g, 0, (size_t)(m + 1) * sizeof(cplx));
        g[0] = beta;
        int j, jend = 0, stop = 0;
        for (j = 0; j < m && it < cap; j++) {
            cplx *vj = V + (size_t)j * n, *vn = V + (size_t)(j + 1) * n;
            if ((rc = Minv(mctx, vj, z))) goto done;
            if ((rc = A(actx, z, w))) goto done;
            for (int i = 0; i <= j; i++) {
                cplx h = dotc(n, w, V + (size_t)i * n);
                Hm[i * ldh + j] = h;
                ORA_PARFOR
                for (size_t q = 0; q < n; q++) w[q] -= h * V[(size_t)i * n + q];
            }
            double hn = nrm2(n, w);
            for (int i = 0; i < j; i++) { /* previous rotations */
                cplx a = Hm[i * ldh + j], bb = Hm[(i + 1) * ldh + j];
                Hm[i * ldh + j] = cs[i] * a + sn[i] * bb;
                Hm[(i + 1) * ldh + j] = -conj(sn[i]) * a + cs[i] * bb;
            }
            givens(Hm[j * ldh + j], hn, &cs[j], &sn[j]);
            Hm[j * ldh + j] = cs[j] * Hm[j * ldh + j] + sn[j] * hn;
            g[j + 1] = -conj(sn[j]) * g[j];
            g[j] = cs[j] * g[j];
            it++;
            jend = j + 1;
            if (hn != 0)
                ORA_PARFOR
                for (size_t q = 0; q < n; q++) vn[q] = w[q] / hn;
            if (fixed <= 0 && cabs(g[j + 1]) <= tol * bnorm) {
                stop = 1;
                break;
            }
            if (hn == 0) {
                stop = 1;
                break;
            }
        }
        backsub(jend, ldh, Hm, g, y);
        ORA_PARFOR
        for (size_t q = 0; q < n; q++) w[q] = 0;
        for (int i = 0; i < jend; i++) {
            ORA_PARFOR
            for (size_t q = 0; q < n; q++) w[q] += y[i] * V[(size_t)i * n + q];
        }
        if ((rc = Minv(mctx, w, z))) goto done;
        ORA_PARFOR
        for (size_t q = 0; q < n; q++) x[q] += z[q];
        if (it >= cap) break;
        if (stop && fixed > 0) break; /* breakdown in fixed mode */
    }
done:
    if (iters) *iters = it;
    free(V);
    free(w);
    free(z);
    free(Hm);
    free(g);
    free(y);
    free(sn);
    free(cs);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Coarse solve and deflation (Section 5.2)                                  */
/* ------------------------------------------------------------------------- */

typedef struct {
    const hier_t *H;
    const ora_problem *p;
} sctx_t;

static int coarse_op_cb(void *ctx, const cplx *x, cplx *y)
{
    sctx_t *c = (sctx_t *)ctx;
    coarse_apply_h(c->H, c->p, x, y);
    return ORA_OK;
}

static int vcycle_l1_cb(void *ctx, const cplx *x, cplx *y)
{
    sctx_t *c = (sctx_t *)ctx;
    return vcycle_rec(c->H, c->p, 1, x, y);
}

static int check_defl(const ora_problem *p, const hier_t *H)
{
    if (H->nlev < 2) return ORA_EGRID; /* no coarse grid for deflation */
    if ((p->coarse_op == ORA_COARSE_REDGLK2 || p->coarse_op == ORA_COARSE_REDGLK1) &&
        p->hx != p->hy)
        return ORA_EINVAL;
    if (p->coarse_op < ORA_COARSE_GALERKIN || p->coarse_op > ORA_COARSE_REDGLK1) return ORA_EINVAL;
    return ORA_OK;
}

/* v2 ~= A_2h^{-1} v1: the coarse-grid problem (Section 5.2), solved by
 * CSLP-preconditioned GMRES whose preconditioner is a V-cycle starting on the
 * coarse grid; or exactly (band LU) for pins and parity. */
static int coarse_solve_h(const hier_t *H, const ora_problem *p, const cplx *v1, cplx *v2, int *iters)
{
    const lvl_t *gc = &H->L[1];
    if (iters) *iters = 0;
    if (p->coarse_mode == ORA_CMODE_EXACT) {
        cctx_t c = {H, p};
        return direct_solve_op(gc, 2, 2, coarse_cb, &c, v1, v2);
    }
    sctx_t c = {H, p};
    int m = p->coarse_restart > 0 ? p->coarse_restart : 30;
    if (p->coarse_mode == ORA_CMODE_FIXED)
        return gmres_right(npts(gc), coarse_op_cb, &c, vcycle_l1_cb, &c, v1, v2, m,
                           p->coarse_iters > 0 ? p->coarse_iters : 1, 0.0, 0, iters);
    return gmres_right(npts(gc), coarse_op_cb, &c, vcycle_l1_cb, &c, v1, v2, m, 0, p->coarse_tol,
                       p->coarse_iters > 0 ? p->coarse_iters : 1000, iters);
}

/* M^{-1} stand-in on the fine grid: one V-cycle, or (test hook) exact A^{-1}. */
static int precond_h(const hier_t *H, const ora_problem *p, const cplx *r, cplx *z)
{
    if (p->precond == ORA_PRECOND_EXACT_A) {
        op5ctx_t c = {&H->L[0], 1.0};
        return direct_solve_op(&H->L[0], 1, 1, op5_cb, &c, r, z);
    }
    return vcycle_rec(H, p, 0, r, z);
}

/* Deflation applied to v (Section 3.2.2 and the step-by-step form of
 * Section 5.2): v1 = Z^T v, v2 = A_2h^{-1} v1, v' = Z v2, then
 *   Q:     w = v'
 *   P:     w = v - A_h v'
 *   ADEF1: w = M^{-1}(v - A_h v') + v'     (P_A-DEF1 = M^{-1} P_h + Q_h).
 * Reading: the expansion printed as v - A v' - gamma v' contradicts
 * P_{h,gamma} = I - A Q + gamma Q two lines above it; the sign of the
 * definition (+Q) is used. */
static int deflate_h(const hier_t *H, const ora_problem *p, int mode, const cplx *v, cplx *w, int *iters)
{
    const lvl_t *gf = &H->L[0], *gc = &H->L[1];
    const size_t n = npts(gf), nc = npts(gc);
    cplx *v1 = (cplx *)malloc(nc * sizeof(cplx));
    cplx *v2 = (cplx *)malloc(nc * sizeof(cplx));
    cplx *vp = (cplx *)malloc(n * sizeof(cplx));
    cplx *t = (cplx *)malloc(n * sizeof(cplx));
    int rc = ORA_OK;
    if (!v1 || !v2 || !vp || !t) {
        rc = ORA_ENOMEM;
        goto done;
    }
    restrict_t(gf, gc, zweights(p), v, v1);
    if ((rc = coarse_solve_h(H, p, v1, v2, iters))) goto done;
    prolong(gf, gc, zweights(p), v2, vp);
    if (mode == ORA_DEFL_Q) {
        memcpy(w, vp, n * sizeof(cplx));
        goto done;
    }
    op5(gf, 1.0, vp, t);
    ORA_PARFOR
    for (size_t q = 0; q < n; q++) t[q] = v[q] - t[q];
    ORA_PARFOR
    for (int j = 0; j < gf->ny; j++) /* v itself carries no boundary value */
        for (int i = 0; i < gf->nx; i++)
            if (!is_unknown(gf, i, j)) t[(size_t)j * gf->nx + i] = 0;
    if (mode == ORA_DEFL_P) {
        memcpy(w, t, n * sizeof(cplx));
        goto done;
    }
    if ((rc = precond_h(H, p, t, w))) goto done;
    ORA_PARFOR
    for (size_t q = 0; q < n; q++) w[q] += vp[q];
done:
    free(v1);
    free(v2);
    free(vp);
    free(t);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Public entry points                                                       */
/* ------------------------------------------------------------------------- */

int ora_helm_apply(const ora_problem *p, const double *x, double *y)
{
    hier_t H;
    int rc = build_hier(p, &H);
    if (rc) return rc;
    op5(&H.L[0], 1.0, (const cplx *)x, (cplx *)y);
    free_hier(&H);
    return ORA_OK;
}

int ora_cslp_apply(const ora_problem *p, const double *x, double *y)
{
    hier_t H;
    int rc = build_hier(p, &H);
    if (rc) return rc;
    op5(&H.L[0], beta_of(p), (const cplx *)x, (cplx *)y);
    free_hier(&H);
    return ORA_OK;
}

int ora_vcycle(const ora_problem *p, int level, const double *r, double *z)
{
    hier_t H;
    int rc = build_hier(p, &H);
    if (rc) return rc;
    if (level < 0 || level >= H.nlev)
        rc = ORA_EINVAL;
    else
        rc = vcycle_rec(&H, p, level, (const cplx *)r, (cplx *)z);
    free_hier(&H);
    return rc;
}

int ora_z_prolong(const ora_problem *p, const double *vc, double *vf)
{
    hier_t H;
    int rc = build_hier(p, &H);
    if (rc) return rc;
    if (H.nlev < 2)
        rc = ORA_EGRID;
    else
        prolong(&H.L[0], &H.L[1], zweights(p), (const cplx *)vc, (cplx *)vf);
    free_hier(&H);
    return rc;
}

int ora_z_restrict(const ora_problem *p, const double *vf, double *vc)
{
    hier_t H;
    int rc = build_hier(p, &H);
    if (rc) return rc;
    if (H.nlev < 2)
        rc = ORA_EGRID;
    else
        restrict_t(&H.L[0], &H.L[1], zweights(p), (const cplx *)vf, (cplx *)vc);
    free_hier(&H);
    return rc;
}

int ora_coarse_apply(const ora_problem *p, const double *x, double *y)
{
    hier_t H;
    int rc = build_hier(p, &H);
    if (rc) return rc;
    if (!(rc = check_defl(p, &H))) coarse_apply_h(&H, p, (const cplx *)x, (cplx *)y);
    free_hier(&H);
    return rc;
}

int ora_coarse_solve(const ora_problem *p, const double *v1, double *v2, int *iters)
{
    hier_t H;
    int rc = build_hier(p, &H);
    if (rc) return rc;
    if (!(rc = check_defl(p, &H))) rc = coarse_solve_h(&H, p, (const cplx *)v1, (cplx *)v2, iters);
    free_hier(&H);
    return rc;
}

int ora_coarse_direct_solve(const ora_problem *p, const double *b, double *x)
{
    hier_t H;
    int rc = build_hier(p, &H);
    if (rc) return rc;
    if (!(rc = check_defl(p, &H))) {
        cctx_t c = {&H, p};
        rc = direct_solve_op(&H.L[1], 2, 2, coarse_cb, &c, (const cplx *)b, (cplx *)x);
    }
    free_hier(&H);
    return rc;
}

int ora_deflate_apply(const ora_problem *p, int mode, const double *v, double *w, int *inner_iters)
{
    hier_t H;
    if (mode != ORA_DEFL_Q && mode != ORA_DEFL_P && mode != ORA_DEFL_ADEF1) return ORA_EINVAL;
    int rc = build_hier(p, &H);
    if (rc) return rc;
    if (!(rc = check_defl(p, &H))) rc = deflate_h(&H, p, mode, (const cplx *)v, (cplx *)w, inner_iters);
    free_hier(&H);
    return rc;
}

int ora_direct_solve(const ora_problem *p, const double *b, double *x)
{
    hier_t H;
    int rc = build_hier(p, &H);
    if (rc) return rc;
    op5ctx_t c = {&H.L[0], 1.0};
    rc = direct_solve_op(&H.L[0], 1, 1, op5_cb, &c, (const cplx *)b, (cplx *)x);
    free_hier(&H);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Adjoint state for the gradient of a misfit with respect to s = k^2/omega^2 */
/* (the model problem of Section 2 with k = omega sqrt(s))                    */
/* ------------------------------------------------------------------------- */

/* y = A_h^H x, the conjugate transpose of the 5-point operator, by scattering
 * each row q of A_h: (A^H x)_p = sum_q conj(A_qp) x_q. */
static void op5_adj(const lvl_t *g, const cplx *x, cplx *y)
{
    const size_t n = npts(g);
    ORA_PARFOR
    for (size_t q = 0; q < n; q++) y[q] = 0;
    for (int j = 0; j < g->ny; j++)
        for (int i = 0; i < g->nx; i++) {
            if (!is_unknown(g, i, j)) continue;
            size_t q = (size_t)j * g->nx + i;
            cplx c[5];
            stencil5(g, 1.0, i, j, c);
            y[q] += conj(c[0]) * x[q];
            if (c[1] != 0) y[q - 1] += conj(c[1]) * x[q];
            if (c[2] != 0) y[q + 1] += conj(c[2]) * x[q];
            if (c[3] != 0) y[q - g->nx] += conj(c[3]) * x[q];
            if (c[4] != 0) y[q + g->nx] += conj(c[4]) * x[q];
        }
}

static void op5_adj_cb(const void *ctx, const cplx *x, cplx *y)
{
    op5_adj((const lvl_t *)ctx, x, y);
}

int ora_helm_apply_adjoint(const ora_problem *p, const double *x, double *y)
{
    hier_t H;
    int rc = build_hier(p, &H);
    if (rc) return rc;
    op5_adj(&H.L[0], (const cplx *)x, (cplx *)y);
    free_hier(&H);
    return ORA_OK;
}

/* lambda = A_h^{-H} f by banded LU of the conjugate transpose. */
int ora_adjoint_solve(const ora_problem *p, const double *f, double *lambda)
{
    hier_t H;
    int rc = build_hier(p, &H);
    if (rc) return rc;
    rc = direct_solve_op(&H.L[0], 1, 1, op5_adj_cb, &H.L[0], (const cplx *)f, (cplx *)lambda);
    free_hier(&H);
    return rc;
}

/* g[p] = -Re(conj(lambda_p) (dA/ds_p) u_p): the gradient of
 * J = 1/2 ||R u - d||^2 with A u = b and A^H lambda = R^T (R u - d).  Only
 * the diagonal of row p depends on s_p: d/ds of -k^2 is -omega^2, and of the
 * Sommerfeld term -2ik/h (per eliminated direction) it is -i omega/(h sqrt s)
 * since k = omega sqrt(s).  Non-unknown (Dirichlet boundary) nodes get 0. */
int ora_grad_s(const ora_problem *p, double omega, const double *uin, const double *lin,
               double *g)
{
    hier_t H;
    int rc = build_hier(p, &H);
    if (rc) return rc;
    const lvl_t *L = &H.L[0];
    const cplx *u = (const cplx *)uin, *lam = (const cplx *)lin;
    ORA_PARFOR
    for (int j = 0; j < L->ny; j++)
        for (int i = 0; i < L->nx; i++) {
            size_t q = (size_t)j * L->nx + i;
            g[q] = 0;
            if (!is_unknown(L, i, j)) continue;
            cplx d = -omega * omega;
            if (L->bc == ORA_BC_SOMMERFELD) {
                double sq = L->k[q] / omega; /* sqrt(s) */
                double w = 0;
                if (i == 0 || i == L->nx - 1) w += 1.0 / L->hx;
                if (j == 0 || j == L->ny - 1) w += 1.0 / L->hy;
                if (w != 0 && sq > 0) d += -IU * omega * w / sq;
            }
            g[q] = -creal(conj(lam[q]) * d * u[q]);
        }
    free_hier(&H);
    return ORA_OK;
}

/* Zero the non-unknown (Dirichlet boundary) entries of a fine vector. */
static void mask_unknowns(const lvl_t *g, cplx *v)
{
    ORA_PARFOR
    for (int j = 0; j < g->ny; j++)
        for (int i = 0; i < g->nx; i++)
            if (!is_unknown(g, i, j)) v[(size_t)j * g->nx + i] = 0;
}

/* Flexible GMRES(m), right preconditioned with P_A-DEF1 (the outer Krylov
 * method; the paper names flexible GMRES as tolerant of a loose coarse-grid
 * tolerance, Section 6.3).  Arnoldi by modified Gram-Schmidt as in
 * Algorithm 1; the preconditioned vectors z_j are stored and x = x0 + Z_m y.
 * After each cycle the true residual ||b - A x|| / ||b|| decides; x0 = 0. */
int ora_fgmres(const ora_problem *p, const double *bin, double *xout, int m, double tol, int maxit,
               int force_iters, ora_info *info)
{
    hier_t H;
    if (m < 1) return ORA_EINVAL;
    int rc = build_hier(p, &H);
    if (rc) return rc;
    if ((rc = check_defl(p, &H)) && p->precond != ORA_PRECOND_EXACT_A) {
        free_hier(&H);
        return rc;
    }
    rc = ORA_OK;
    const lvl_t *g = &H.L[0];
    const size_t n = npts(g);
    const int ldh = m;
    cplx *b = (cplx *)malloc(n * sizeof(cplx));
    cplx *x = (cplx *)xout;
    cplx *V = (cplx *)malloc((size_t)(m + 1) * n * sizeof(cplx));
    cplx *Zs = (cplx *)malloc((size_t)m * n * sizeof(cplx));
    cplx *w = (cplx *)malloc(n * sizeof(cplx));
    cplx *Hm = (cplx *)calloc((size_t)(m + 1) * m, sizeof(cplx));
    cplx *gv = (cplx *)calloc((size_t)m + 1, sizeof(cplx));
    cplx *y = (cplx *)calloc((size_t)m, sizeof(cplx));
    cplx *sn = (cplx *)calloc((size_t)m, sizeof(cplx));
    double *cs = (double *)calloc((size_t)m, sizeof(double));
    ora_info inf = {0, 0, 0, 0, 0.0};
    if (!b || !V || !Zs || !w || !Hm || !gv || !y || !sn || !cs) {
        rc = ORA_ENOMEM;
        goto done;
    }
    memcpy(b, bin, n * sizeof(cplx));
    mask_unknowns(g, b);
    ORA_PARFOR
    for (size_t q = 0; q < n; q++) x[q] = 0;
    const double bnorm = nrm2(n, b);
    const int cap = force_iters > 0 ? force_iters : maxit;
    if (bnorm == 0) {
        inf.converged = 1;
        goto done;
    }
    for (;;) {
        op5(g, 1.0, x, w);
        ORA_PARFOR
        for (size_t q = 0; q < n; q++) w[q] = b[q] - w[q];
        double beta = nrm2(n, w);
        inf.relres = beta / bnorm;
        if (force_iters <= 0 && inf.relres <= tol) {
            inf.converged = 1;
            break;
        }
        if (inf.iters >= cap || beta == 0) break;
        ORA_PARFOR
        for (size_t q = 0; q < n; q++) V[q] = w[q] / beta;
        memset(gv, 0, (size_t)(m + 1) * sizeof(cplx));
        gv[0] = beta;
        int jend = 0;
        for (int j = 0; j < m && inf.iters < cap; j++) {
            cplx *vj = V + (size_t)j * n, *vn = V + (size_t)(j + 1) * n, *zj = Zs + (size_t)j * n;
            int inner = 0;
            if (p->precond == ORA_PRECOND_EXACT_A) {
                op5ctx_t c = {g, 1.0};
                rc = direct_solve_op(g, 1, 1, op5_cb, &c, vj, zj);
            } else {
                rc = deflate_h(&H, p, ORA_DEFL_ADEF1, vj, zj, &inner);
            }
            if (rc) goto done;
            inf.inner_total += inner;
            if (inner > inf.inner_max) inf.inner_max = inner;
            op5(g, 1.0, zj, w);
            for (int i = 0; i <= j; i++) {
                cplx h = dotc(n, w, V + (size_t)i * n);
                Hm[i * ldh + j] = h;
                ORA_PARFOR
                for (size_t q = 0; q < n; q++) w[q] -= h * V[(size_t)i * n + q];
            }
            double hn = nrm2(n, w);
            for (int i = 0; i < j; i++) {
                cplx a = Hm[i * ldh + j], bb = Hm[(i + 1) * ldh + j];
                Hm[i * ldh + j] = cs[i] * a + sn[i] * bb;
                Hm[(i + 1) * ldh + j] = -conj(sn[i]) * a + cs[i] * bb;
            }
            givens(Hm[j * ldh + j], hn, &cs[j], &sn[j]);
            Hm[j * ldh + j] = cs[j] * Hm[j * ldh + j] + sn[j] * hn;
            gv[j + 1] = -conj(sn[j]) * gv[j];
            gv[j] = cs[j] * gv[j];
            inf.iters++;
            jend = j + 1;
            if (hn != 0)
                ORA_PARFOR
                for (size_t q = 0; q < n; q++) vn[q] = w[q] / hn;
            if (force_iters <= 0 && cabs(gv[j + 1]) <= tol * bnorm) break;
            if (hn == 0) break;
        }
        backsub(jend, ldh, Hm, gv, y);
        for (int i = 0; i < jend; i++) {
            ORA_PARFOR
            for (size_t q = 0; q < n; q++) x[q] += y[i] * Zs[(size_t)i * n + q];
        }
        if (force_iters > 0 && inf.iters >= cap) {
            op5(g, 1.0, x, w);
            ORA_PARFOR
            for (size_t q = 0; q < n; q++) w[q] = b[q] - w[q];
            inf.relres = nrm2(n, w) / bnorm;
            inf.converged = inf.relres <= tol;
            break;
        }
    }
done:
    if (info) *info = inf;
    free(b);
    free(V);
    free(Zs);
    free(w);
    free(Hm);
    free(gv);
    free(y);
    free(sn);
    free(cs);
    free_hier(&H);
    return rc;
}

/* Right-preconditioned GCR(m) with the A-DEF1 preconditioner: the outer
 * method of Section 6.3 (Eisenstat, Elman and Schultz), which admits a
 * preconditioner that changes from step to step.  Step j: z = P r,
 * w = A z; w is made orthogonal to the earlier w_i by modified Gram-Schmidt,
 * the same combination is applied to z (so w = A z still holds), and both are
 * divided by ||w||; then alpha = (r, w), x += alpha z, r -= alpha w.  After m
 * steps the stored pairs are dropped (restart).  When the updated residual
 * reaches tol ||b|| the true residual is recomputed; the method stops if it
 * is below tol and otherwise restarts from it.  force_iters > 0 runs exactly
 * that many steps.  x0 = 0. */
int ora_gcr(const ora_problem *p, const double *bin, double *xout, int m, double tol, int maxit,
            int force_iters, ora_info *info)
{
    hier_t H;
    if (m < 1 || maxit < 1) return ORA_EINVAL;
    int rc = build_hier(p, &H);
    if (rc) return rc;
    if ((rc = check_defl(p, &H))) {
        free_hier(&H);
        return rc;
    }
    const lvl_t *g = &H.L[0];
    const size_t n = npts(g);
    cplx *b = (cplx *)malloc(n * sizeof(cplx));
    cplx *x = (cplx *)xout;
    cplx *r = (cplx *)malloc(n * sizeof(cplx));
    cplx *Zs = (cplx *)malloc((size_t)m * n * sizeof(cplx));
    cplx *Ws = (cplx *)malloc((size_t)m * n * sizeof(cplx));
    ora_info inf = {0, 0, 0, 0, 0.0};
    if (!b || !r || !Zs || !Ws) {
        rc = ORA_ENOMEM;
        goto done;
    }
    memcpy(b, bin, n * sizeof(cplx));
    mask_unknowns(g, b);
    ORA_PARFOR
    for (size_t q = 0; q < n; q++) x[q] = 0;
    const double bnorm = nrm2(n, b);
    const int cap = force_iters > 0 ? force_iters : maxit;
    if (bnorm == 0) {
        inf.converged = 1;
        goto done;
    }
    for (;;) {
        /* (re)start from the true residual */
        op5(g, 1.0, x, r);
        ORA_PARFOR
        for (size_t q = 0; q < n; q++) r[q] = b[q] - r[q];
        inf.relres = nrm2(n, r) / bnorm;
        if (force_iters <= 0 && inf.relres <= tol) {
            inf.converged = 1;
            break;
        }
        if (inf.iters >= cap || inf.relres == 0) break;
        for (int j = 0; j < m && inf.iters < cap; j++) {
            cplx *zj = Zs + (size_t)j * n, *wj = Ws + (size_t)j * n;
            int inner = 0;
            if (p->precond == ORA_PRECOND_EXACT_A) {
                op5ctx_t c = {g, 1.0};
                rc = direct_solve_op(g, 1, 1, op5_cb, &c, r, zj);
            } else {
                rc = deflate_h(&H, p, ORA_DEFL_ADEF1, r, zj, &inner);
            }
            if (rc) goto done;
            inf.inner_total += inner;
            if (inner > inf.inner_max) inf.inner_max = inner;
            op5(g, 1.0, zj, wj);
            for (int i = 0; i < j; i++) {
                const cplx *wi = Ws + (size_t)i * n, *zi = Zs + (size_t)i * n;
                cplx beta = dotc(n, wj, wi);
                ORA_PARFOR
                for (size_t q = 0; q < n; q++) {
                    wj[q] -= beta * wi[q];
                    zj[q] -= beta * zi[q];
                }
            }
            double nu = nrm2(n, wj);
            inf.iters++;
            if (nu == 0) break; /* breakdown: A P r lies in the span already searched */
            ORA_PARFOR
            for (size_t q = 0; q < n; q++) {
                wj[q] /= nu;
                zj[q] /= nu;
            }
            cplx alpha = dotc(n, r, wj);
            ORA_PARFOR
            for (size_t q = 0; q < n; q++) {
                x[q] += alpha * zj[q];
                r[q] -= alpha * wj[q];
            }
            if (force_iters <= 0 && nrm2(n, r) <= tol * bnorm) break;
        }
        if (force_iters > 0 && inf.iters >= cap) {
            op5(g, 1.0, x, r);
            ORA_PARFOR
            for (size_t q = 0; q < n; q++) r[q] = b[q] - r[q];
            inf.relres = nrm2(n, r) / bnorm;
            inf.converged = inf.relres <= tol;
            break;
        }
    }
done:
    if (info) *info = inf;
    free(b);
    free(r);
    free(Zs);
    free(Ws);
    free_hier(&H);
    return rc;
}

/* The paper's preconditioned deflated GMRES (Algorithm 1) for the A-DEF1
 * system P A u = P b (left preconditioning, full GMRES, modified Gram-Schmidt),
 * stopping once the preconditioned residual drops below tol relative to the
 * preconditioned initial residual.  u0 = 0.
 * Reading: A-DEF1 is non-singular, so the final projection step printed for
 * the singular deflated system is not applied, and V holds the orthonormal
 * basis v_j. */
int ora_gmres_left(const ora_problem *p, const double *bin, double *xout, double tol, int maxit,
                   ora_info *info)
{
    hier_t H;
    if (maxit < 1) return ORA_EINVAL;
    int rc = build_hier(p, &H);
    if (rc) return rc;
    if ((rc = check_defl(p, &H))) {
        free_hier(&H);
        return rc;
    }
    const lvl_t *g = &H.L[0];
    const size_t n = npts(g);
    const int m = maxit, ldh = maxit;
    cplx *b = (cplx *)malloc(n * sizeof(cplx));
    cplx *x = (cplx *)xout;
    cplx *V = (cplx *)malloc((size_t)(m + 1) * n * sizeof(cplx));
    cplx *w = (cplx *)malloc(n * sizeof(cplx));
    cplx *t = (cplx *)malloc(n * sizeof(cplx));
    cplx *Hm = (cplx *)calloc((size_t)(m + 1) * m, sizeof(cplx));
    cplx *gv = (cplx *)calloc((size_t)m + 1, sizeof(cplx));
    cplx *y = (cplx *)calloc((size_t)m, sizeof(cplx));
    cplx *sn = (cplx *)calloc((size_t)m, sizeof(cplx));
    double *cs = (double *)calloc((size_t)m, sizeof(double));
    ora_info inf = {0, 0, 0, 0, 0.0};
    int inner = 0;
    if (!b || !V || !w || !t || !Hm || !gv || !y || !sn || !cs) {
        rc = ORA_ENOMEM;
        goto done;
    }
    memcpy(b, bin, n * sizeof(cplx));
    mask_unknowns(g, b);
    ORA_PARFOR
    for (size_t q = 0; q < n; q++) x[q] = 0;
    /* r0 = P (b - A u0) with u0 = 0 */
    if ((rc = deflate_h(&H, p, ORA_DEFL_ADEF1, b, w, &inner))) goto done;
    inf.inner_total += inner;
    inf.inner_max = inner;
    double beta = nrm2(n, w);
    if (beta == 0) {
        inf.converged = 1;
        goto done;
    }
    ORA_PARFOR
    for (size_t q = 0; q < n; q++) V[q] = w[q] / beta;
    gv[0] = beta;
    int jend = 0;
    for (int j = 0; j < m; j++) {
        cplx *vj = V + (size_t)j * n, *vn = V + (size_t)(j + 1) * n;
        op5(g, 1.0, vj, t);                                        /* v~ = A v_j */
        if ((rc = deflate_h(&H, p, ORA_DEFL_ADEF1, t, w, &inner))) goto done; /* w = P v~ */
        inf.inner_total += inner;
        if (inner > inf.inner_max) inf.inner_max = inner;
        for (int i = 0; i <= j; i++) {
            cplx h = dotc(n, w, V + (size_t)i * n);
            Hm[i * ldh + j] = h;
            ORA_PARFOR
            for (size_t q = 0; q < n; q++) w[q] -= h * V[(size_t)i * n + q];
        }
        double hn = nrm2(n, w);
        for (int i = 0; i < j; i++) {
            cplx a = Hm[i * ldh + j], bb = Hm[(i + 1) * ldh + j];
            Hm[i * ldh + j] = cs[i] * a + sn[i] * bb;
            Hm[(i + 1) * ldh + j] = -conj(sn[i]) * a + cs[i] * bb;
        }
        givens(Hm[j * ldh + j], hn, &cs[j], &sn[j]);
        Hm[j * ldh + j] = cs[j] * Hm[j * ldh + j] + sn[j] * hn;
        gv[j + 1] = -conj(sn[j]) * gv[j];
        gv[j] = cs[j] * gv[j];
        inf.iters++;
        jend = j + 1;
        if (hn != 0)
            ORA_PARFOR
            for (size_t q = 0; q < n; q++) vn[q] = w[q] / hn;
        if (cabs(gv[j + 1]) <= tol * beta) {
            inf.converged = 1;
            break;
        }
        if (hn == 0) break;
    }
    backsub(jend, ldh, Hm, gv, y);
    for (int i = 0; i < jend; i++) {
        ORA_PARFOR
        for (size_t q = 0; q < n; q++) x[q] += y[i] * V[(size_t)i * n + q];
    }
    op5(g, 1.0, x, w);
    ORA_PARFOR
    for (size_t q = 0; q < n; q++) w[q] = b[q] - w[q];
    inf.relres = nrm2(n, w) / nrm2(n, b);
done:
    if (info) *info = inf;
    free(b);
    free(V);
    free(w);
    free(t);
    free(Hm);
    free(gv);
    free(y);
    free(sn);
    free(cs);
    free_hier(&H);
    return rc;
}
