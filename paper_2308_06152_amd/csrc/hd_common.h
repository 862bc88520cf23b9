// hd_common.h -- types and launch wrappers shared by the HIP kernels and the
// host driver of libhelmdefl.so (gfx950).  Complex128 values are double2
// (x = real, y = imaginary), 16-byte aligned, interleaved as in the C-ABI;
// complex64 values (the mixed-precision V-cycle) are float2.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace hd {

typedef double2 cd;
typedef float2 cf;

enum { BC_DIR = 0, BC_SOM = 1 };

// Partial-sum stride of the block reductions: at most 63 dot products plus one
// norm slot per block.
constexpr int PSTRIDE = 64;
constexpr int MAX_RESTART = 60;

// Batched launches (several right-hand sides of one operator).  Grid y is the
// right-hand side.  A right-hand side's vectors are contiguous and follow each
// other at the level's node count (or at an explicit stride for Krylov
// bases); its small device arrays (projections, norms, scales, coefficients)
// follow each other at SB entries.  act: per right-hand side 1 = active,
// 0 = skip (nullptr: all active).
constexpr int SB = 256;
struct Batch {
    int B = 1;
    const int *act = nullptr;
};

// One grid level as the kernels see it (passed by value).
struct Lev {
    int nx, ny;
    double hx, hy;
    double ihx2, ihy2;  // 1/hx^2, 1/hy^2
    int bc;
    const double *k;    // wavenumber [ny][nx] on this level, or nullptr
    double kc;          // constant wavenumber when k == nullptr
};

inline Lev make_lev(int nx, int ny, double hx, double hy, int bc, const double *k, double kc)
{
    Lev L;
    L.nx = nx;
    L.ny = ny;
    L.hx = hx;
    L.hy = hy;
    L.ihx2 = 1.0 / (hx * hx);
    L.ihy2 = 1.0 / (hy * hy);
    L.bc = bc;
    L.k = k;
    L.kc = kc;
    return L;
}

__host__ __device__ inline double kat(const Lev &L, int i, int j)
{
    return L.k ? L.k[(size_t)j * L.nx + i] : L.kc;
}

__host__ __device__ inline bool unknown(const Lev &L, int i, int j)
{
    return L.bc == BC_SOM || (i > 0 && j > 0 && i < L.nx - 1 && j < L.ny - 1);
}

// Multipliers of the 5-point operator -Lap - s k^2 at node (i,j) (Section 2.1
// stencil; Section 5.1 names them ap, aw, ae, as, an).  Sommerfeld: the ghost
// node beyond a boundary node is eliminated (u_ghost = u_inward + 2ikh u_bnd),
// adding -2ik/h to ap and doubling the inward coupling, per direction.
// Dirichlet: boundary nodes are not unknowns (returns false); couplings to
// them are dropped.  (i,j) must lie inside the grid; k is the wavenumber
// there (coef5 reads it from the level).
__host__ __device__ inline bool coef5k(const Lev &L, cd s, int i, int j, double k, cd &ap,
                                       double &aw, double &ae, double &as, double &an)
{
    const double k2 = k * k;
    ap = make_double2(2.0 * L.ihx2 + 2.0 * L.ihy2 - s.x * k2, -s.y * k2);
    aw = -L.ihx2;
    ae = -L.ihx2;
    as = -L.ihy2;
    an = -L.ihy2;
    if (L.bc == BC_SOM) {
        if (i == 0) {
            ap.y -= 2.0 * k / L.hx;
            ae += aw;
            aw = 0.0;
        }
        if (i == L.nx - 1) {
            ap.y -= 2.0 * k / L.hx;
            aw += ae;
            ae = 0.0;
        }
        if (j == 0) {
            ap.y -= 2.0 * k / L.hy;
            an += as;
            as = 0.0;
        }
        if (j == L.ny - 1) {
            ap.y -= 2.0 * k / L.hy;
            as += an;
            an = 0.0;
        }
        return true;
    }
    if (i == 0 || j == 0 || i == L.nx - 1 || j == L.ny - 1) return false;
    if (i == 1) aw = 0.0;
    if (i == L.nx - 2) ae = 0.0;
    if (j == 1) as = 0.0;
    if (j == L.ny - 2) an = 0.0;
    return true;
}

__host__ __device__ inline bool coef5(const Lev &L, cd s, int i, int j, cd &ap, double &aw,
                                      double &ae, double &as, double &an)
{
    return coef5k(L, s, i, j, kat(L, i, j), ap, aw, ae, as, an);
}

// ---- launch wrappers (kernels.hip); all return the launch's hipError_t ----

// y = (-Lap - s k^2) x, or y = b - (-Lap - s k^2) x when b != nullptr.
hipError_t launch_apply5(const Lev &L, cd s, const cd *x, const cd *b, cd *y, hipStream_t st,
                         Batch bt = Batch{});
// rc = FW( r - M (omega D^-1 r) ): pre-smooth from zero, residual, restriction.
// The right-hand side is rs[0].x * r when rs != nullptr (a lazily normalised
// Krylov vector).
hipError_t launch_vc_down(const Lev &Lf, const Lev &Lc, cd s, double omega, const cd *r,
                          const cd *rs, cd *rc, hipStream_t st, Batch bt = Batch{});
// out (+)= x2 + omega D^-1 (r - M x2), x2 = omega D^-1 r + P ec  [+ Z v2];
// right-hand side scaled by rs[0].x as above.
hipError_t launch_vc_up(const Lev &Lf, const Lev &Lc, cd s, double omega, const cd *r,
                        const cd *rs, const cd *ec, cd *out, int accumulate, const cd *v2, int zho,
                        hipStream_t st, Batch bt = Batch{});
// Mixed-precision V-cycle (complex64 arithmetic and level storage): the top
// level reads r in FP64 and writes rc in FP32, and its upward pass reads r in
// FP64, ec in FP32 and writes out in FP64 (adding Z v2 in FP64); levels below
// are FP32 throughout.
hipError_t launch_vc_down(const Lev &Lf, const Lev &Lc, cd s, double omega, const cd *r, cf *rc,
                          hipStream_t st, Batch bt = Batch{});
hipError_t launch_vc_down(const Lev &Lf, const Lev &Lc, cd s, double omega, const cf *r, cf *rc,
                          hipStream_t st, Batch bt = Batch{});
hipError_t launch_vc_up(const Lev &Lf, const Lev &Lc, cd s, double omega, const cd *r,
                        const cf *ec, cd *out, int accumulate, const cd *v2, int zho,
                        hipStream_t st, Batch bt = Batch{});
hipError_t launch_vc_up(const Lev &Lf, const Lev &Lc, cd s, double omega, const cf *r,
                        const cf *ec, cf *out, hipStream_t st, Batch bt = Batch{});
// The top level of a cycle whose right-hand side is a complex64 vector (the
// mixed-precision inner Krylov basis), scaled by rs[0].x, with FP64 arithmetic
// and FP64 levels below.
hipError_t launch_vc_down(const Lev &Lf, const Lev &Lc, cd s, double omega, const cf *r,
                          const cd *rs, cd *rc, hipStream_t st);
hipError_t launch_vc_up(const Lev &Lf, const Lev &Lc, cd s, double omega, const cf *r,
                        const cd *rs, const cd *ec, cd *out, int accumulate, hipStream_t st);
// The upward passes of levels l .. l + nt - 1 (the last one above the
// coarsest) in one launch, FP64: levs[k] = level l + k, levs[nt] = the
// coarsest; r[k] = level l + k's right-hand side, xc = the coarsest solution;
// out = the correction of level l.  Equal to nt launches of launch_vc_up with
// no scale, accumulation or Z v2.  1 <= nt <= VC_TAIL_MAXLEV.
constexpr int VC_TAIL_MAXLEV = 6;
// The downward passes of the last nd levels above the coarsest in one launch,
// FP64: levs[j] = level Lc - j (levs[0] the coarsest), r = level Lc - nd's
// right-hand side; out[j] = the right-hand side of level Lc - j, for j < nd
// (out[0]: the coarsest).  Equal to nd launches of launch_vc_down with no
// scale.  1 <= nd <= VC_DTAIL_MAXLEV.
constexpr int VC_DTAIL_MAXLEV = 3;
hipError_t launch_vc_down_tail(int nd, const Lev *levs, const cd *r, cd *const *out, cd s,
                               double omega, hipStream_t st);
hipError_t launch_vc_up_tail(int nt, const Lev *levs, const cd *const *r, const cd *xc, cd *out,
                             cd s, double omega, hipStream_t st);
// x = Minv r on the coarsest level (dense inverse, n x n, row major).
hipError_t launch_coarsest(int n, const cd *Minv, const cd *r, cd *x, hipStream_t st,
                           Batch bt = Batch{});
hipError_t launch_coarsest(int n, const cf *Minv, const cf *r, cf *x, hipStream_t st,
                           Batch bt = Batch{});
// vc = Z^T vf, or vc = b - Z^T vf when b != nullptr.
hipError_t launch_zt(const Lev &Lf, const Lev &Lc, int zho, const cd *vf, const cd *b, cd *vc,
                     hipStream_t st, Batch bt = Batch{});
// vf = Z vc.
hipError_t launch_z(const Lev &Lf, const Lev &Lc, int zho, const cd *vc, cd *vf, hipStream_t st,
                    Batch bt = Batch{});
// y = Z^T A_h Z x, or y = b - Z^T A_h Z x (the Galerkin coarse operator, one
// launch; the fine-grid intermediates stay in LDS).
hipError_t launch_glk(const Lev &Lf, const Lev &Lc, int zho, const cd *x, const cd *b, cd *y,
                      hipStream_t st, Batch bt = Batch{});
// t = v - A_h (Z v2).
hipError_t launch_dresid(const Lev &Lf, const Lev &Lc, int zho, const cd *v, const cd *v2,
                         cd *t, hipStream_t st, Batch bt = Batch{});
// y = A_2h x (ReD-Glk2, or ReD-Glk1 when glk1) or y = b - A_2h x; interior
// and boundary band.
hipError_t launch_redglk2(const Lev &Lc, const cd *x, const cd *b, cd *y, int glk1,
                          hipStream_t st, Batch bt = Batch{});
// y = A_2h x (ReD-O4) or y = b - A_2h x.
hipError_t launch_redo4(const Lev &Lc, const cd *x, const cd *b, cd *y, hipStream_t st,
                        Batch bt = Batch{});

// ---- adjoint state ----
// mode 0: out = conj(in / D), mode 1: out = D conj(in), D = 1/2 per
// Sommerfeld-eliminated direction (B contiguous vectors).
hipError_t launch_adj_map(const Lev &L, const cd *in, cd *out, int mode, int B, hipStream_t st);
// g += sum_b -Re(conj(lam_b) (dA/ds) u_b), s = (k/omega)^2.
hipError_t launch_grad_s(const Lev &L, double omega, const cd *u, const cd *lam, int B, double *g,
                         hipStream_t st);
// res = R u - d, f = R^T res (f pre-zeroed), J = 1/2 ||res||^2 per right-hand side.
hipError_t launch_receivers(const int *rec, int nrec, const cd *u, const cd *d, size_t n, int B,
                            cd *res, cd *f, double *J, hipStream_t st);

// ---- Krylov kernels ----
// Number of partial-sum blocks per vector that the Krylov kernel `kind` uses
// for B vectors of length n each (every launch of that kernel, and the
// reduction of its partial sums, use this count); the partial-sum buffers
// need krylov_blocks_max blocks per vector.
enum { KB_DOT = 0, KB_UPDATE = 1, KB_DOT32 = 2, KB_UPDATE32 = 3, KB_NKINDS = 4 };
int krylov_blocks(size_t n, int B = 1, int kind = KB_DOT);
int krylov_blocks_max(size_t n, int B = 1);
// part[blk][i] = sum conj(V_i) w over the block, i < m; slot m = |w|^2 if
// with_norm.  cond != nullptr: second Gram-Schmidt pass, a no-op unless the
// reorthogonalisation test on cond (projections, then ||w||^2 at [jcond]) fires.
// Batched: V and w of right-hand side b start vbs / wbs entries after b-1's.
hipError_t launch_mdot(const cd *V, size_t ld, int m, const cd *w, size_t n, cd *part,
                       int with_norm, const cd *cond, int jcond, hipStream_t st,
                       Batch bt = Batch{}, size_t vbs = 0, size_t wbs = 0);
// w -= sum_i c_i sig_i V_i (sig_i = 1 if sig == nullptr); partn[blk] =
// |w_new|^2 partial if partn != nullptr.
hipError_t launch_mupdate(cd *w, const cd *V, size_t ld, int m, const cd *c, size_t n, cd *partn,
                          const cd *cond, int jcond, const cd *sig, hipStream_t st,
                          Batch bt = Batch{}, size_t vbs = 0, size_t wbs = 0);
// The same two kernels on a complex64 basis V (mixed precision): products and
// updates are formed in FP64; w is read as complex128 or complex64, and the
// update writes complex64 (in place, or from a complex128 w into wout), with
// partn the norm of the stored entries.
hipError_t launch_mdot32(const cf *V, size_t ld, int m, const cd *w, size_t n, cd *part,
                         int with_norm, const cd *cond, int jcond, hipStream_t st);
hipError_t launch_mdot32(const cf *V, size_t ld, int m, const cf *w, size_t n, cd *part,
                         int with_norm, const cd *cond, int jcond, hipStream_t st);
hipError_t launch_mupdate32(const cd *win, cf *wout, const cf *V, size_t ld, int m, const cd *c,
                            size_t n, cd *partn, const cd *cond, int jcond, const cd *sig,
                            hipStream_t st);
hipError_t launch_mupdate32(cf *w, const cf *V, size_t ld, int m, const cd *c, size_t n,
                            cd *partn, const cd *cond, int jcond, const cd *sig, hipStream_t st);
// out[i] (=|+=) sum_blk part[blk][i], i < m (mode 0: times sig[i] for
// i < nsig); mode 2: out[0] = (sqrt(sum re), 0) and sig_out[0] = its
// reciprocal.  cond: as above; writes zeros when the second pass is skipped.
hipError_t launch_reduce(const cd *part, int nblk, int m, cd *out, int mode, const cd *cond,
                         int jcond, const cd *sig, int nsig, cd *sig_out, hipStream_t st,
                         Batch bt = Batch{});
// The mode-2 reduction of one vector's norm partials (out[0], sig_out[0] as
// above), then pub_dst[0, pub_n) = pub_src[0, pub_n) with a system-scope fence:
// pub_dst is host memory the device can write (the scalars of a Krylov step
// reach the host without a copy launch).
hipError_t launch_norm_publish(const cd *part, int nblk, cd *out, cd *sig_out,
                               const cd *pub_src, int pub_n, cd *pub_dst, hipStream_t st);
// v = w / nrm[0].x (v = 0 if the norm is 0).
hipError_t launch_scale(const cd *w, const cd *nrm, cd *v, size_t n, hipStream_t st,
                        Batch bt = Batch{}, size_t wbs = 0, size_t vbs = 0);
// out (+)= sum_i y_i V_i.
hipError_t launch_lincomb(const cd *V, size_t ld, int m, const cd *y, cd *out, size_t n,
                          int accumulate, hipStream_t st, Batch bt = Batch{}, size_t vbs = 0,
                          size_t obs = 0);
// p[0..n) = 0.
hipError_t launch_zero(cd *p, size_t n, hipStream_t st);
// out = in with the non-unknown (Dirichlet boundary) entries set to zero.
hipError_t launch_mask_copy(const Lev &L, const cd *in, cd *out, hipStream_t st, int B = 1);

}  // namespace hd
