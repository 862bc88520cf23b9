/*
 * Driver for the sanitizer build of the oracle (AddressSanitizer and
 * UndefinedBehaviorSanitizer, host code only): every entry point of
 * oracle/oracle.h on small grids, both boundary conditions, constant and
 * variable wavenumber, every coarse operator and outer method.  Exits 0 when
 * every call returned 0 and every result is finite; the sanitizers abort the
 * process on the first invalid access or undefined operation.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static int fails = 0;

static void check(int rc, const char *what, const double *v, size_t n)
{
    if (rc != 0) {
        printf("FAIL %s rc=%d\n", what, rc);
        fails++;
        return;
    }
    for (size_t q = 0; q < n; q++)
        if (!isfinite(v[q])) {
            printf("FAIL %s: non-finite output at %zu\n", what, q);
            fails++;
            return;
        }
}

/* deterministic pseudo-random values in [-1, 1] */
static double rnd(unsigned *s)
{
    *s = *s * 1664525u + 1013904223u;
    return ((*s >> 8) / 8388608.0) - 1.0;
}

static void run(int nx, int ny, int bc, int vark, int cop, unsigned seed)
{
    const double h = 1.0 / (nx > ny ? nx - 1 : ny - 1);
    const size_t n = (size_t)nx * ny;
    double *k = NULL;
    if (vark) {
        k = malloc(n * sizeof(double));
        for (size_t q = 0; q < n; q++) k[q] = 12.0 + 4.0 * rnd(&seed);
    }
    ora_problem p;
    memset(&p, 0, sizeof p);
    p.nx = nx;
    p.ny = ny;
    p.hx = p.hy = h;
    p.bc = bc;
    p.k = k;
    p.kconst = 10.0;
    p.beta_re = 1.0;
    p.beta_im = 0.5;
    p.omega = 0.8;
    p.nu_pre = p.nu_post = 1;
    p.defl_vectors = ORA_Z_HIGH;
    p.coarse_op = cop;
    p.coarse_mode = ORA_CMODE_FIXED;
    p.coarse_iters = 4;
    p.coarse_restart = 3;
    p.coarse_tol = 0.1;
    p.precond = ORA_PRECOND_VCYCLE;
    p.coarsest_nodes = 0;
    const int nxc = (nx + 1) / 2, nyc = (ny + 1) / 2;
    const size_t nc = (size_t)nxc * nyc;
    double *x = malloc(2 * n * sizeof(double)), *y = malloc(2 * n * sizeof(double));
    double *xc = malloc(2 * nc * sizeof(double)), *yc = malloc(2 * nc * sizeof(double));
    double *g = malloc(n * sizeof(double));
    for (size_t q = 0; q < 2 * n; q++) x[q] = rnd(&seed);
    for (size_t q = 0; q < 2 * nc; q++) xc[q] = rnd(&seed);
    char tag[96];
    snprintf(tag, sizeof tag, "%dx%d bc=%d vark=%d op=%d", nx, ny, bc, vark, cop);
    int it = 0;
    check(ora_helm_apply(&p, x, y), tag, y, 2 * n);
    check(ora_cslp_apply(&p, x, y), tag, y, 2 * n);
    check(ora_vcycle(&p, 0, x, y), tag, y, 2 * n);
    check(ora_vcycle(&p, 1, xc, yc), tag, yc, 2 * nc);
    check(ora_z_prolong(&p, xc, y), tag, y, 2 * n);
    check(ora_z_restrict(&p, x, yc), tag, yc, 2 * nc);
    check(ora_coarse_apply(&p, xc, yc), tag, yc, 2 * nc);
    check(ora_coarse_solve(&p, xc, yc, &it), tag, yc, 2 * nc);
    for (int mode = 0; mode < 3; mode++) check(ora_deflate_apply(&p, mode, x, y, &it), tag, y, 2 * n);
    p.coarse_mode = ORA_CMODE_EXACT;
    check(ora_deflate_apply(&p, ORA_DEFL_ADEF1, x, y, &it), tag, y, 2 * n);
    check(ora_coarse_direct_solve(&p, xc, yc), tag, yc, 2 * nc);
    check(ora_direct_solve(&p, x, y), tag, y, 2 * n);
    p.coarse_mode = ORA_CMODE_TOL;
    p.coarse_iters = 50;
    ora_info inf;
    check(ora_fgmres(&p, x, y, 10, 1e-6, 60, 0, &inf), tag, y, 2 * n);
    check(ora_gcr(&p, x, y, 5, 1e-6, 60, 0, &inf), tag, y, 2 * n);
    check(ora_gmres_left(&p, x, y, 1e-6, 60, &inf), tag, y, 2 * n);
    check(ora_fgmres(&p, x, y, 10, 1e-6, 60, 3, &inf), tag, y, 2 * n);
    check(ora_helm_apply_adjoint(&p, x, y), tag, y, 2 * n);
    check(ora_adjoint_solve(&p, x, y), tag, y, 2 * n);
    if (vark) check(ora_grad_s(&p, 10.0, x, y, g), tag, g, n);
    printf("ok %s\n", tag);
    free(x);
    free(y);
    free(xc);
    free(yc);
    free(g);
    free(k);
}

int main(void)
{
    unsigned seed = 230806152u;
    const int cops[5] = {ORA_COARSE_GALERKIN, ORA_COARSE_REDGLK2, ORA_COARSE_REDO2,
                         ORA_COARSE_REDO4, ORA_COARSE_REDGLK1};
    for (int c = 0; c < 5; c++) {
        run(17, 17, ORA_BC_DIRICHLET, 0, cops[c], seed + c);
        run(17, 25, ORA_BC_SOMMERFELD, 1, cops[c], seed + 10 + c);
        run(5, 5, ORA_BC_SOMMERFELD, 0, cops[c], seed + 20 + c);
        run(9, 7, ORA_BC_DIRICHLET, 1, cops[c], seed + 30 + c);
    }
    printf("%s: %d failed calls\n", fails ? "FAIL" : "PASS", fails);
    return fails ? 1 : 0;
}
