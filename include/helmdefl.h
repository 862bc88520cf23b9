/*
 * helmdefl.h -- C-ABI of libhelmdefl.so, an MI355X (gfx950) solver for the 2D
 * finite-difference Helmholtz problem with the matrix-free two-level deflation
 * preconditioner of Chen, Dwarka & Vuik (arXiv 2308.06152).
 *
 * The problem (Section 2): -Lap u - k(x,y)^2 u = b on a rectangle, with
 * homogeneous Dirichlet or first-order Sommerfeld (du/dn - i k u = 0)
 * boundaries, discretised by the 5-point stencil on a vertex-centred grid
 * (Section 2.1).  The preconditioner (Section 3) is A-DEF1 / APD:
 *     P = M^{-1} (I - A Q) + Q,   Q = Z A_2h^{-1} Z^T,
 * with M^{-1} one multigrid V-cycle for the complex shifted Laplacian
 * M = -Lap - (beta_re + i beta_im) k^2 (damped Jacobi, full weighting, bilinear
 * interpolation), Z the linear or higher-order (Bezier) deflation vectors, and
 * A_2h the Galerkin (str-Glk) or re-discretised (ReD-Glk2) coarse operator,
 * inverted by CSLP-preconditioned GMRES (Section 5.2).
 *
 * Conventions shared by every entry point
 *  - Vectors are complex128, real/imaginary interleaved (the memory layout of
 *    torch.complex128 / std::complex<double>), stored [ny][nx] with x fastest;
 *    node (i,j) is at (i*hx, j*hy), boundary nodes included.  With nrhs > 1 the
 *    right-hand sides are nrhs contiguous [ny][nx] blocks.
 *  - Every vector argument is a DEVICE pointer on the current HIP device, owned
 *    by the caller, at least 16-byte aligned.  Inputs and outputs must not
 *    overlap.  The library keeps no pointer after a call returns.
 *  - Homogeneous Dirichlet boundary nodes are not unknowns: every operator
 *    writes 0 there and ignores the values it is given there.
 *  - Calls are asynchronous on the handle's stream, except helm_solve and
 *    helm_coarse_solve, which synchronise that stream (they read Krylov scalars
 *    back to the host every iteration) and fill their info before returning.
 *  - Return value: HELM_OK (0) or a negative helm_status.  No C++ exception
 *    crosses the ABI.  On an error the output buffers are unspecified, except
 *    for HELM_ENOCONV (see helm_solve).
 */
#ifndef HELMDEFL_H
#define HELMDEFL_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HELM_OK = 0,
    HELM_EINVAL = -1,     /* null pointer, bad size or option                    */
    HELM_EGRID = -2,      /* grid cannot be coarsened as deflation/multigrid need */
    HELM_ENONFINITE = -3, /* NaN or Inf in k or in a right-hand side              */
    HELM_ENOMEM = -4,     /* device or host allocation failed                    */
    HELM_EHIP = -5,       /* a HIP runtime call or kernel launch failed          */
    HELM_ENOCONV = -6,    /* solver stopped at maxit above the tolerance         */
    HELM_ESCRATCH = -7    /* cslp_vcycle_noalloc: levels exceed its fixed scratch */
} helm_status;

enum { HELM_BC_DIRICHLET = 0, HELM_BC_SOMMERFELD = 1 };
enum { HELM_DEFL_Q = 0, HELM_DEFL_P = 1, HELM_DEFL_ADEF1 = 2 };
enum { HELM_Z_LINEAR = 0, HELM_Z_HIGH = 1 };
/* Coarse-grid operators A_2h (Section 5.2): str-Glk (Z^T A_h Z, Section
 * 5.2.1); ReD-Glk2 and ReD-Glk1 (the Galerkin 5x5 stencils re-used as a
 * coarse discretisation, with ghost-point or second-order boundary rows,
 * Section 5.2.4); ReD-O2 and ReD-O4 (second- and fourth-order
 * re-discretisation, Section 5.2.3).  ReD-Glk* need hx == hy. */
enum {
    HELM_COARSE_GALERKIN = 0,
    HELM_COARSE_REDGLK2 = 1,
    HELM_COARSE_REDO2 = 2,
    HELM_COARSE_REDO4 = 3,
    HELM_COARSE_REDGLK1 = 4
};
/* Outer Krylov methods: flexible GMRES (right preconditioning, true residual
 * test; the default), GCR (right preconditioning, Section 6.3), and the
 * paper's left-preconditioned GMRES of Algorithm 1 (restarted after
 * `restart` steps; stops on the preconditioned residual relative to ||P b||). */
enum { HELM_OUTER_FGMRES = 0, HELM_OUTER_GCR = 1, HELM_OUTER_GMRES_LEFT = 2 };
enum { HELM_CMODE_FIXED = 1, HELM_CMODE_TOL = 2 };
enum { HELM_PREC_FP64 = 0, HELM_PREC_MIXED = 1, HELM_PREC_MIXED_C64BASIS = 2 };

/* The grid: nx x ny vertex nodes including the boundary, spacings hx, hy
 * (Section 2.1 takes hx = hy = h; ReD-Glk2 requires hx == hy). */
typedef struct {
    int nx, ny;
    double hx, hy;
    int bc; /* HELM_BC_* on all four sides */
} helm_grid;

/* Method options; helm_opts_default() fills the paper's values. */
typedef struct {
    double beta_re, beta_im; /* CSLP shift, default (1, 0.5) (Section 3.1)      */
    double omega;            /* damped-Jacobi relaxation, default 0.8           */
    int nu_pre, nu_post;     /* smoothing sweeps; only 1/1 is supported         */
    int defl_vectors;        /* HELM_Z_*, default HELM_Z_HIGH (APD)             */
    int coarse_op;           /* HELM_COARSE_*, default HELM_COARSE_GALERKIN     */
    int coarse_mode;         /* HELM_CMODE_*, default HELM_CMODE_TOL            */
    int coarse_iters;        /* FIXED: iteration count; TOL: cap (default 300)  */
    int coarse_restart;      /* inner GMRES restart length (default 30)         */
    double coarse_tol;       /* TOL: relative residual target (default 1e-1)    */
    int restart;             /* outer FGMRES restart length (default 50)        */
    int maxit;               /* outer iteration cap (default 1000)              */
    double tol;              /* outer relative residual target (default 1e-6)   */
    int x0_given;            /* helm_solve: 1 = x holds the initial guess       */
    int force_iters;         /* >0: run exactly this many outer iterations      */
    int coarsest_nodes;      /* predefined coarsest multigrid grid (Section 4):
                                below level 1, stop coarsening once a level has
                                <= this many nodes; that level is solved exactly
                                (default 1089 = 33 x 33; 0 = down to 3 x 3;
                                at most 2048) */
    int precision;           /* HELM_PREC_FP64 (default): everything in FP64.
                                HELM_PREC_MIXED: the fine-grid CSLP V-cycle
                                and its smoother (cslp_vcycle, and M^{-1}
                                inside A-DEF1) run in complex64 on every
                                level: the cycle reads r in FP64, stores the
                                levels in FP32 and writes z in FP64.  The
                                outer Krylov method, A_h, Z, Z^T, the
                                deflation coarse solve (its basis, its V-cycle
                                and A_2h) and the residual test stay FP64;
                                FGMRES absorbs the perturbed preconditioner
                                (Sections 3.1, 6.3).
                                HELM_PREC_MIXED_C64BASIS: as HELM_PREC_MIXED,
                                and the coarse GMRES also stores its Krylov
                                basis in complex64 (when its V-cycle has a
                                level below level 1), with A_2h, that V-cycle,
                                the products and the updates in FP64. */
    int outer;               /* HELM_OUTER_* (default HELM_OUTER_FGMRES)       */
    int batch;               /* nrhs > 1: 1 (default) = all right-hand sides
                                in one batched pass (one launch per kernel for
                                all of them; helm_solve runs one FGMRES per
                                right-hand side in lockstep, masking converged
                                ones out), in FP64 or HELM_PREC_MIXED; 0 = one
                                after another.  GCR, left GMRES and
                                HELM_PREC_MIXED_C64BASIS always go one after
                                another. */
    int graphs;              /* 0 (default): every kernel is launched directly.
                                1: the steps of the coarse GMRES (V-cycle, A_2h,
                                Gram-Schmidt kernels) are captured into HIP
                                graphs on first use and replayed: one graph per
                                basis index for a single right-hand side, one
                                per chunk of 4 steps (with their read-backs) in
                                the batched path, which then checks
                                convergence per chunk (steps computed past a
                                convergence are not used).  Not while kernel
                                timing is enabled.  Results are identical
                                either way. */
    int vc_tail;             /* >0 (default 300000): in the FP64 V-cycle of a
                                single right-hand side, the levels below the
                                cycle's top level run fused: the downward passes
                                of the last three levels above the coarsest in
                                one launch, and the upward passes of the levels
                                with at most this many nodes (6 at most) in
                                another, each keeping the intermediate levels
                                on-chip (at least two levels each, else one
                                launch per level); 0 = one launch per level.
                                Both evaluate the same expressions in the same
                                order (bit-identical results with a constant k;
                                with a variable k the per-node coefficients may
                                differ in the last bit). */
} helm_opts;

/* Per right-hand side result of helm_solve. */
typedef struct {
    int outer_iters;       /* preconditioner applications, over all restarts     */
    int inner_iters_total; /* coarse-grid GMRES iterations, summed               */
    int inner_iters_max;   /* largest single coarse solve                        */
    int converged;         /* relres <= tol (GMRES_LEFT: the preconditioned
                              residual test of Algorithm 1 was met)             */
    double relres;         /* ||b - A x|| / ||b|| recomputed in FP64 at exit     */
    double t_solve_ms;     /* wall time of this right-hand side (of the batch)   */
    double t_setup_ms;     /* wall time of helm_create for this handle           */
    double t_coarse_ms;    /* GPU time of the coarse-grid solves (HIP events on
                              the handle's stream; of the whole batch in a
                              batched solve)                                    */
    double t_vcycle_ms;    /* GPU time of the fine-grid CSLP V-cycles (as above) */
    int reorth_steps;      /* Arnoldi steps (outer and inner) that took a second
                              Gram-Schmidt pass (the cancellation test fired)  */
} helm_solve_info;

typedef struct helm_ctx helm_ctx;

/* Fill *o with the defaults listed above.  HELM_EINVAL if o is NULL. */
int helm_opts_default(helm_opts *o);

/* Create a solver handle.
 *  g        grid; nx, ny >= 5 and odd (the deflation coarse grid is
 *           ((nx+1)/2) x ((ny+1)/2), Section 4), else HELM_EGRID.  Multigrid
 *           levels coarsen while both counts are odd and >= 5 and (below level
 *           1) the level has more than opts.coarsest_nodes nodes; the coarsest
 *           level (at most 2048 nodes, else HELM_EGRID) is solved exactly.
 *  k_dev    device pointer to the real FP64 wavenumber field [ny][nx]
 *           (k = 2 pi f / c, Section 2), or NULL to use k_const everywhere.
 *           Copied at create; not retained.
 *  opts     options, or NULL for the defaults.
 *  stream   hipStream_t for every call on this handle (NULL = null stream).
 * Allocates the level hierarchy and the coarse-solve workspace on the device.
 * HELM_ENONFINITE if k has a non-finite or negative value. */
int helm_create(const helm_grid *g, const double *k_dev, double k_const, const helm_opts *opts,
                void *stream, helm_ctx **out);

/* y = A_h x: the 5-point Helmholtz operator with the boundary closure of
 * Section 2.1 (Sommerfeld ghost nodes eliminated: -2ik/h on the diagonal per
 * boundary direction, inward neighbour -2/h^2), the matrix-free matvec of
 * Section 5.1. */
int helm_apply(helm_ctx *h, const void *x, void *y, int nrhs);

/* z = V(r): one CSLP multigrid V-cycle (Sections 3.1 and 5.1) for
 * M = -Lap - (beta_re + i beta_im) k^2, re-discretised on every level with the
 * injected wavenumber; 1 damped-Jacobi pre- and post-sweep from x = 0, full
 * weighting, bilinear interpolation, exact solve on the coarsest level.
 * With opts.precision == HELM_PREC_MIXED the cycle computes in complex64
 * (r and z stay complex128 in memory). */
int cslp_vcycle(helm_ctx *h, const void *r, void *z, int nrhs);

/* cslp_vcycle (one right-hand side after another) for callers that cannot
 * allocate device memory, e.g. code under HIP graph capture or a serving loop
 * that forbids hipMalloc.  The V-cycle's level buffers (levels >= 1) live in a
 * fixed device array of 64 MiB per GPU, held until the process ends, instead
 * of the handle's buffers; the call allocates nothing and creates no events
 * (kernel timing is suspended inside it).  The levels take 2 n_l complex128
 * values each (complex64 with a mixed-precision handle), rounded up to 256
 * bytes, about 10.7 bytes per fine-grid node in FP64: a 2049 x 2049 grid takes
 * 45 MB; 4097 x 4097 does not fit.  HELM_ESCRATCH, before anything is
 * launched, if they do not fit.
 * Every call on one GPU shares that array: calls that may overlap in time on
 * one GPU (different streams, or different host threads) race and must be
 * serialised by the caller.  Arguments and results as for cslp_vcycle. */
int cslp_vcycle_noalloc(helm_ctx *h, const void *r, void *z, int nrhs);

/* Deflation applied to v (Sections 3.2.2 and 5.2): with v1 = Z^T v,
 * v2 ~= A_2h^{-1} v1 (per coarse_mode), v' = Z v2:
 *   HELM_DEFL_Q:     w = v'
 *   HELM_DEFL_P:     w = v - A_h v'
 *   HELM_DEFL_ADEF1: w = V(v - A_h v') + v'   (the preconditioner P_A-DEF1) */
int deflate_apply(helm_ctx *h, int mode, const void *v, void *w, int nrhs);

/* Solve A_h x = b by flexible GMRES(restart), right-preconditioned with
 * P_A-DEF1, to ||b - A x|| / ||b|| <= tol (true residual, checked at every
 * restart); or by GCR(restart) or the left-preconditioned GMRES of
 * Algorithm 1, per opts.outer.  x: output, and input when opts.x0_given.  info: array of nrhs
 * entries, may be NULL.  HELM_ENOCONV when maxit was reached above tol; x then
 * holds the last iterate and info is filled.  HELM_ENONFINITE if b is not
 * finite. */
int helm_solve(helm_ctx *h, const void *b, void *x, int nrhs, helm_solve_info *info);

/* ---- Adjoint state: gradient of a misfit with respect to s = 1/c^2 -------
 * For k = omega sqrt(s) (Section 2) and J = 1/2 sum ||R u - d||^2 with
 * A_h u = b, the gradient is g = -Re(conj(lambda) (dA_h/ds) u) summed over the
 * sources, with A_h^H lambda = R^T (R u - d). */

/* lambda = A_h^{-H} f for nrhs right-hand sides ([nrhs][ny][nx], device).
 * D A_h is complex symmetric for the diagonal D that halves each
 * Sommerfeld-eliminated direction, so the adjoint solve is the forward solve
 * (helm_solve with the handle's options, x0 = 0) of conj(D^{-1} f), mapped back
 * by lambda = D conj(.).  info as for helm_solve (may be NULL); returns
 * HELM_ENOCONV like helm_solve.  Synchronises. */
int helm_adjoint_solve(helm_ctx *h, const void *f, void *lambda, int nrhs, helm_solve_info *info);

/* g[p] += sum over the nrhs right-hand sides of -Re(conj(lambda_p) d_p u_p),
 * d_p = dA_pp/ds_p = -omega^2 (- i omega^2 / k_p per Sommerfeld-eliminated
 * direction, divided by hx or hy; omitted where k_p = 0).  u, lambda:
 * [nrhs][ny][nx] complex128; g: real FP64 [ny][nx], device, accumulated.
 * omega > 0 is the angular frequency with which the handle's k was formed. */
int helm_gradient_s(helm_ctx *h, double omega, const void *u, const void *lambda, int nrhs,
                    double *g);

/* Receiver residuals for nrhs wavefields: res[b][r] = u_b[rec[r]] - d[b][r],
 * f_b = R^T res_b (zero away from the receivers: the adjoint source) and
 * J[b] = 1/2 ||res_b||^2.  rec: device int array of nrec distinct node indices
 * j*nx + i (HELM_EINVAL otherwise); d, res: device complex128 [nrhs][nrec];
 * f: device [nrhs][ny][nx]; J: device double [nrhs]. */
int helm_receivers(helm_ctx *h, const int *rec, int nrec, const void *u, const void *d, int nrhs,
                   void *res, void *f, double *J);

/* Free the handle and its device memory (after synchronising its stream). */
int helm_destroy(helm_ctx *h);

/* Static text for a helm_status code. */
const char *helm_strerror(int code);

/* ---- Steps of the path, exported for step-by-step parity checks ---------- */

/* Dimensions of the deflation coarse grid (= multigrid level 1). */
int helm_coarse_dims(helm_ctx *h, int *nxc, int *nyc);
/* Number of multigrid levels (level 0 is the fine grid). */
int helm_num_levels(helm_ctx *h, int *nlev);
/* Dimensions of multigrid level l, 0 <= l < nlev. */
int helm_level_dims(helm_ctx *h, int l, int *nx, int *ny);
/* vc = Z^T vf (fine -> coarse): [1 4 6 4 1]/8 (higher order) or 1/2 [1 2 1]
 * (linear) per axis, truncated at the boundary (Sections 3.2, 3.2.1). */
int helm_z_restrict(helm_ctx *h, const void *vf, void *vc);
/* vf = Z vc (coarse -> fine), the transpose of helm_z_restrict. */
int helm_z_prolong(helm_ctx *h, const void *vc, void *vf);
/* y = A_2h x on the coarse grid: Z^T A_h Z (str-Glk, Section 5.2.1) or the
 * ReD-Glk2 re-discretisation (Section 5.2.4). */
int helm_coarse_apply(helm_ctx *h, const void *x, void *y);
/* v2 ~= A_2h^{-1} v1 by right-preconditioned GMRES(coarse_restart) with a
 * V-cycle starting on the coarse grid, x0 = 0 (FIXED or TOL mode).
 * *iters receives the iteration count (may be NULL).  Synchronises. */
int helm_coarse_solve(helm_ctx *h, const void *v1, void *v2, int *iters);

/* ---- Kernel timing (HIP events on the handle's stream) ------------------- */

/* Kernel classes that can be timed. */
enum {
    HELM_K_APPLY = 0,     /* 5-point operator                      */
    HELM_K_VC_DOWN = 1,   /* fused pre-smooth/residual/restriction */
    HELM_K_VC_UP = 2,     /* fused interpolation/post-smooth       */
    HELM_K_ZT = 3,        /* Z^T restriction                       */
    HELM_K_DRESID = 4,    /* t = v - A_h Z v2                      */
    HELM_K_COARSE = 5,    /* coarse operator A_2h                  */
    HELM_K_DOT = 6,       /* block dot products V^H w              */
    HELM_K_UPDATE = 7,    /* w -= V c                              */
    HELM_K_NCLASSES = 8
};
/* Start timing launches of kernel class `kclass` on multigrid level `level`
 * (-1 = any level).  Resets the accumulators.  kclass < 0 disables timing.
 * A fused V-cycle tail (opts.vc_tail) is one launch of HELM_K_VC_DOWN or
 * HELM_K_VC_UP, filed under the highest level it covers. */
int helm_timing_enable(helm_ctx *h, int kclass, int level);
/* Read the accumulated launch count, summed event time (ms) and the summed
 * algorithmic HBM bytes of the timed launches (synchronises the stream). */
int helm_timing_read(helm_ctx *h, long long *launches, double *total_ms, double *alg_bytes);

#ifdef __cplusplus
}
#endif
#endif
