/*
 * oracle.h -- plain FP64 CPU reference ("the oracle") for the matrix-free
 * two-level deflation Helmholtz solver of Chen, Dwarka & Vuik,
 * "A matrix-free parallel two-level deflation preconditioner for the
 * two-dimensional Helmholtz problems" (arXiv 2308.06152).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline
 * leg of the benchmark may load or call this library.  It shares no code,
 * header, table or helper with the HIP product library, and the product never
 * calls it.
 *
 * Every routine follows the paper's definitions step by step in plain loops,
 * in the paper's order, with no blocking or fusion.  Vectors are complex128,
 * stored as [ny][nx] with x fastest; node (i,j) is the vertex i*hx, j*hy.
 *
 * Parity status per routine (the pins live in tests/test_oracle.py):
 *   ora_helm_apply     pinned: Dirichlet sine-mode eigenvalues (Appendix B
 *                      eigenvalue formula), manufactured O(h^2) convergence
 *                      (Dirichlet and Sommerfeld), complex symmetry of D*A.
 *   ora_z_prolong /    pinned: printed Galerkin stencils (ReD-Glk section),
 *   ora_z_restrict     exact transpose identity, Z(x^2) = x^2 + H^2/4.
 *   ora_coarse_apply   pinned: interior rows equal the printed Galerkin
 *                      Laplacian and k^2 stencils; ReD-Glk2 boundary-band rows
 *                      (variable k, both boundary types, corner rows) equal the
 *                      coefficients derived from the printed stencils and the
 *                      ghost rules (Sections 2.1, 5.2.4, 5.2.5).
 *   ora_vcycle         pinned: exact on a 3x3 grid, transpose-symmetric for
 *                      Dirichlet, textbook multigrid contraction for k = 0.
 *   ora_coarse_solve   pinned: EXACT mode residual; TOL/FIXED against EXACT.
 *   ora_deflate_apply  pinned: A-DEF1 identities (Z y reproduced, P^2 = P,
 *                      exact-M case equals A^{-1}).
 *   ora_fgmres         pinned: banded direct solve; exact-M case = 1 iteration.
 *   ora_gmres_left     soft pin: iteration counts of the paper's tables.
 */
#ifndef HELM_ORACLE_H
#define HELM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORA_BC_DIRICHLET = 0, ORA_BC_SOMMERFELD = 1 };
enum { ORA_Z_LINEAR = 0, ORA_Z_HIGH = 1 };
enum {
    ORA_COARSE_GALERKIN = 0, /* str-Glk: Z^T A_h Z                       */
    ORA_COARSE_REDGLK2 = 1,  /* Galerkin 5x5 stencils, ghost-point band     */
    ORA_COARSE_REDO2 = 2,    /* second-order re-discretisation            */
    ORA_COARSE_REDO4 = 3,    /* fourth-order re-discretisation            */
    ORA_COARSE_REDGLK1 = 4   /* Galerkin 5x5 stencils, second-order band    */
};
enum { ORA_CMODE_EXACT = 0, ORA_CMODE_FIXED = 1, ORA_CMODE_TOL = 2 };
enum { ORA_DEFL_Q = 0, ORA_DEFL_P = 1, ORA_DEFL_ADEF1 = 2 };
enum { ORA_PRECOND_VCYCLE = 0, ORA_PRECOND_EXACT_A = 1 };

typedef struct {
    int nx, ny;               /* vertex nodes including the boundary          */
    double hx, hy;            /* mesh widths                                  */
    int bc;                   /* ORA_BC_*                                     */
    const double *k;          /* wavenumber [ny][nx], or NULL for kconst      */
    double kconst;
    double beta_re, beta_im;  /* CSLP shift: M = -Lap - (beta_re + i beta_im) k^2 */
    double omega;             /* damped-Jacobi relaxation                      */
    int nu_pre, nu_post;      /* smoothing sweeps                              */
    int defl_vectors;         /* ORA_Z_*                                       */
    int coarse_op;            /* ORA_COARSE_*                                  */
    int coarse_mode;          /* ORA_CMODE_*                                   */
    int coarse_iters;         /* FIXED: exact count; TOL: iteration cap        */
    int coarse_restart;       /* restart length of the inner GMRES             */
    double coarse_tol;        /* TOL: relative residual target                 */
    int precond;              /* ORA_PRECOND_*: what stands for M^{-1}          */
    int coarsest_nodes;       /* predefined coarsest grid: stop coarsening below
                                 level 1 once a level has <= this many nodes
                                 (0 = coarsen down to 3 x 3)                   */
} ora_problem;

typedef struct {
    int iters;                /* preconditioner applications (outer iterations) */
    int converged;
    int inner_total;          /* inner coarse-solve iterations, summed          */
    int inner_max;
    double relres;            /* true ||b - A x|| / ||b|| at exit               */
} ora_info;

/* Level hierarchy of the V-cycle: number of levels and the dims of level l. */
/* Threads the element-wise loops and chunked sums use (1 in the serial
 * build); results do not depend on it. */
int ora_threads(void);
void ora_set_threads(int n);

int ora_num_levels(int nx, int ny, int coarsest_nodes);
int ora_level_dims(int nx, int ny, int coarsest_nodes, int l, int *lnx, int *lny);

/* y = A_h x (5-point Helmholtz operator with the boundary closure). */
int ora_helm_apply(const ora_problem *p, const double *x, double *y);
/* y = M_h x (CSLP operator on level 0). */
int ora_cslp_apply(const ora_problem *p, const double *x, double *y);
/* z = one V-cycle for M applied to r, starting at level `level`
 * (r, z have that level's dims). */
int ora_vcycle(const ora_problem *p, int level, const double *r, double *z);
/* Deflation vectors: vf = Z vc (coarse -> fine), vc = Z^T vf (fine -> coarse). */
int ora_z_prolong(const ora_problem *p, const double *vc, double *vf);
int ora_z_restrict(const ora_problem *p, const double *vf, double *vc);
/* y = A_2h x on the deflation coarse grid. */
int ora_coarse_apply(const ora_problem *p, const double *x, double *y);
/* v2 ~= A_2h^{-1} v1 (EXACT / FIXED / TOL per p->coarse_mode). */
int ora_coarse_solve(const ora_problem *p, const double *v1, double *v2, int *iters);
/* w = Q v, (I - A Q) v or the A-DEF1 preconditioner applied to v. */
int ora_deflate_apply(const ora_problem *p, int mode, const double *v, double *w,
                      int *inner_iters);
/* Right-preconditioned flexible GMRES(restart) with the A-DEF1 preconditioner.
 * force_iters > 0 runs exactly that many iterations (no tolerance test). */
int ora_fgmres(const ora_problem *p, const double *b, double *x, int restart,
               double tol, int maxit, int force_iters, ora_info *info);
/* Right-preconditioned GCR(restart) with the A-DEF1 preconditioner (the
 * variable-preconditioner outer method of Section 6.3). */
int ora_gcr(const ora_problem *p, const double *b, double *x, int restart, double tol,
            int maxit, int force_iters, ora_info *info);
/* The paper's left-preconditioned full GMRES (Algorithm 1, no restart),
 * stopping on the preconditioned relative residual. */
int ora_gmres_left(const ora_problem *p, const double *b, double *x, double tol,
                   int maxit, ora_info *info);
/* y = A_h^H x (conjugate transpose); lambda = A_h^{-H} f (banded LU). */
int ora_helm_apply_adjoint(const ora_problem *p, const double *x, double *y);
int ora_adjoint_solve(const ora_problem *p, const double *f, double *lambda);
/* g = -Re(conj(lambda) (dA/ds) u) per node, s = (k/omega)^2: the adjoint-state
 * gradient of 1/2 ||R u - d||^2 for A u = b, A^H lambda = R^T (R u - d). */
int ora_grad_s(const ora_problem *p, double omega, const double *u, const double *lambda,
               double *g);
/* x = A_h^{-1} b by banded LU with partial pivoting. */
int ora_direct_solve(const ora_problem *p, const double *b, double *x);
/* Same for A_2h (the coarse operator) and for M on level `level`. */
int ora_coarse_direct_solve(const ora_problem *p, const double *b, double *x);

#ifdef __cplusplus
}
#endif
#endif
