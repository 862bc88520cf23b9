// kernels.hip -- HIP kernels for gfx950 (MI355X, wave64) of the matrix-free
// two-level deflation Helmholtz solver (arXiv 2308.06152).
//
// Every kernel here is bandwidth-bound (<= ~4 flop/byte in FP64), so none uses
// MFMA.  Design rules:
//  * complex128 is one 16-byte load/store per node (double2), rows are
//    contiguous in x so a wave touches 1 KB of consecutive memory per row;
//  * stencil kernels stage a tile plus halo in LDS and fuse the steps of the
//    method that share the tile (smoothing + residual + restriction in one
//    pass, interpolation + correction + smoothing in another);
//  * the block -> tile map is XCD-aware: consecutive block ids go to different
//    XCDs, so tiles are renumbered to give every XCD a contiguous band of the
//    grid, keeping vertical halos in that XCD's L2;
//  * reductions are deterministic: fixed per-block partial sums, then a fixed
//    tree in a second kernel.
#include "hd_common.h"

#include <type_traits>


namespace hd {

#define HD_LAUNCH_CHECK() return hipGetLastError()

// ------------------------------------------------------------------------
// small complex helpers
// ------------------------------------------------------------------------
__device__ __forceinline__ cd czero() { return make_double2(0.0, 0.0); }
__device__ __forceinline__ cd cadd(cd a, cd b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ cd csub(cd a, cd b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ cd cscal(double s, cd a) { return make_double2(s * a.x, s * a.y); }
__device__ __forceinline__ cd cmul(cd a, cd b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ cd cinv(cd a)
{
    const double d = 1.0 / (a.x * a.x + a.y * a.y);
    return make_double2(a.x * d, -a.y * d);
}
// a += s * b  (s real)
__device__ __forceinline__ void caxpy(cd &a, double s, cd b)
{
    a.x = fma(s, b.x, a.x);
    a.y = fma(s, b.y, a.y);
}

// The same helpers for complex64 (float2), and the precision-generic names
// used by the kernels templated on the real type R (double or float).
__device__ __forceinline__ cf cadd(cf a, cf b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ cf csub(cf a, cf b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ cf cscal(float s, cf a) { return make_float2(s * a.x, s * a.y); }
__device__ __forceinline__ cf cmul(cf a, cf b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ void caxpy(cf &a, float s, cf b)
{
    a.x = fmaf(s, b.x, a.x);
    a.y = fmaf(s, b.y, a.y);
}
template <class R> struct CxT;
template <> struct CxT<double> { typedef cd T; };
template <> struct CxT<float> { typedef cf T; };
template <class R> using cx = typename CxT<R>::T;
template <class R> __device__ __forceinline__ cx<R> mkc(R a, R b);
template <> __device__ __forceinline__ cd mkc<double>(double a, double b) { return make_double2(a, b); }
template <> __device__ __forceinline__ cf mkc<float>(float a, float b) { return make_float2(a, b); }
template <class R> __device__ __forceinline__ cx<R> zc() { return mkc<R>((R)0, (R)0); }
// conversion (rounding to nearest) between the two complex types
template <class R> __device__ __forceinline__ cx<R> cvt(cd a) { return mkc<R>((R)a.x, (R)a.y); }
template <class R> __device__ __forceinline__ cx<R> cvt(cf a) { return mkc<R>((R)a.x, (R)a.y); }

// Wave-wide lane shifts (DPP wave_shr:1 / wave_shl:1): lane i receives the
// value of lane i-1 (west) or lane i+1 (east); lane 0 resp. 63 receives 0.
// Every lane of the wave must be active.
__device__ __forceinline__ int lane_from(int v, bool west)
{
    return west ? __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, false)
                : __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, false);
}
__device__ __forceinline__ float lane_from(float v, bool west)
{
    return __int_as_float(lane_from(__float_as_int(v), west));
}
__device__ __forceinline__ double lane_from(double v, bool west)
{
    const long long u = __double_as_longlong(v);
    const int lo = lane_from((int)u, west), hi = lane_from((int)(u >> 32), west);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ cd lane_from(cd v, bool west)
{
    return make_double2(lane_from(v.x, west), lane_from(v.y, west));
}
__device__ __forceinline__ cf lane_from(cf v, bool west)
{
    return make_float2(lane_from(v.x, west), lane_from(v.y, west));
}

// Map hardware block id to a logical tile id so that each of the 8 XCDs
// (which receive block ids round-robin) works on a contiguous range of tiles.
__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    const int X = 8;
    const int xcd = b % X, q = b / X, full = nb / X, rem = nb % X;
    return xcd < rem ? xcd * (full + 1) + q : rem * (full + 1) + (xcd - rem) * full + q;
}

static inline int cdiv(int a, int b) { return (a + b - 1) / b; }

// Batched launches: blockIdx.y is the right-hand side; a block of an inactive
// right-hand side exits at once.
__device__ __forceinline__ bool skip_rhs(const Batch &bt) { return bt.act && !bt.act[blockIdx.y]; }

// 1D interpolation rule from the coarse grid to fine index i: returns the
// number of coarse neighbours and fills their indices and weights.
// zho = 1: Bezier vectors (even i: (1, 6, 1)/8 on I-1, I, I+1; odd: 1/2, 1/2);
// zho = 0: linear (even i: 1 on I; odd: 1/2, 1/2).
__device__ __forceinline__ int zrule(int i, int zho, int *I, double *w)
{
    if (i & 1) {
        I[0] = (i - 1) >> 1;
        I[1] = (i + 1) >> 1;
        w[0] = 0.5;
        w[1] = 0.5;
        return 2;
    }
    if (zho) {
        I[0] = (i >> 1) - 1;
        I[1] = i >> 1;
        I[2] = (i >> 1) + 1;
        w[0] = 0.125;
        w[1] = 0.75;
        w[2] = 0.125;
        return 3;
    }
    I[0] = i >> 1;
    w[0] = 1.0;
    return 1;
}

// (I_{2h}^h vc) at fine node (i,j); coarse nodes outside the grid or not
// unknowns contribute nothing.
__device__ __forceinline__ cd prolong_at(const Lev &Lc, const cd *__restrict__ vc, int i, int j,
                                         int zho)
{
    int Ix[3], Jy[3];
    double wx[3], wy[3];
    const int nxw = zrule(i, zho, Ix, wx), nyw = zrule(j, zho, Jy, wy);
    cd s = czero();
    for (int b = 0; b < nyw; b++) {
        const int J = Jy[b];
        if (J < 0 || J >= Lc.ny) continue;
        for (int a = 0; a < nxw; a++) {
            const int I = Ix[a];
            if (I < 0 || I >= Lc.nx || !unknown(Lc, I, J)) continue;
            caxpy(s, wx[a] * wy[b], vc[(size_t)J * Lc.nx + I]);
        }
    }
    return s;
}

// (Z v) at a fine node from an LDS tile of the coarse values around it, whose
// entries outside the grid or at non-unknowns hold 0: (a, b) is the fine node
// relative to the tile origin's fine image, so its coarse node (a >> 1,
// b >> 1) must have a tile neighbour on each side.  Each axis takes 3 taps,
// relative to that coarse node, with weights
//   even fine index: (w2, w0, w2) = (1, 6, 1)/8 Bezier, (0, 1, 0) linear;
//   odd  fine index: (0, 1/2, 1/2);
// no per-node index arrays, so nothing is kept in scratch memory.
template <int W>
__device__ __forceinline__ cd zv2_tile(const cd (*t)[W], int a, int b, int zho)
{
    const int A = a >> 1, B = b >> 1;
    const double w0 = zho ? 0.75 : 1.0, w2 = zho ? 0.125 : 0.0;
    const double xm = (a & 1) ? 0.0 : w2, x0 = (a & 1) ? 0.5 : w0, xp = (a & 1) ? 0.5 : w2;
    const double ym = (b & 1) ? 0.0 : w2, y0 = (b & 1) ? 0.5 : w0, yp = (b & 1) ? 0.5 : w2;
    cd r[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const cd *row = t[B - 1 + d];
        cd v = cscal(x0, row[A]);
        caxpy(v, xm, row[A - 1]);
        caxpy(v, xp, row[A + 1]);
        r[d] = v;
    }
    cd z = cscal(y0, r[1]);
    caxpy(z, ym, r[0]);
    caxpy(z, yp, r[2]);
    return z;
}

// ------------------------------------------------------------------------
// 5-point operator: y = op x  or  y = b - op x
// Each wave streams a strip of A5_RPW rows of 64 consecutive columns and
// writes the 62 in the middle (lanes 1..62): every row is one 1 KB load, the
// west/east neighbours come from the adjacent lanes by DPP shifts, and the
// north/south ones from the rows before and after in registers.  A block is
// 4 waves stacked over 4 * A5_RPW rows; rows are loaded unconditionally from
// a clamped address A5_AHEAD rows ahead of their use and zeroed outside the
// grid (and at Dirichlet nodes) by a 0/1 factor, so each wave keeps many rows
// in flight.
// ------------------------------------------------------------------------
constexpr int A5_TX = 62, A5_RPW = 16, A5_AHEAD = 12;

template <bool RESID, bool VARK>
__global__ __launch_bounds__(256) void k_apply5(Lev L, cd s, const cd *__restrict__ x,
                                                const cd *__restrict__ b, cd *__restrict__ y,
                                                int tiles_x, Batch bt)
{
    if (skip_rhs(bt)) return;
    {
        const size_t off = (size_t)blockIdx.y * L.nx * L.ny;
        x += off;
        if (RESID) b += off;
        y += off;
    }
    const int lane = threadIdx.x & 63;
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int i = (t % tiles_x) * A5_TX - 1 + lane;
    const int j0 = (t / tiles_x) * (4 * A5_RPW) + (threadIdx.x >> 6) * A5_RPW;
    const int nx = L.nx, ny = L.ny;
    if (j0 >= ny) return;  // the whole wave: no row here
    const bool colin = i >= 0 && i < nx;
    const int ic = i < 0 ? 0 : (i >= nx ? nx - 1 : i);
    const bool outc = lane >= 1 && lane <= A5_TX && colin;
    constexpr int NR = A5_RPW + 2;  // rows j0-1 .. j0+A5_RPW
    cd xb[NR], bb[RESID ? A5_RPW : 1];
    double kb[VARK ? A5_RPW : 1];
    auto load_row = [&](int q) {
        const int jj = j0 - 1 + q;
        const size_t p = (size_t)(jj < 0 ? 0 : (jj >= ny ? ny - 1 : jj)) * nx + ic;
        xb[q] = x[p];
        if (q >= 1 && q <= A5_RPW) {
            if (VARK) kb[q - 1] = L.k[p];
            if (RESID) bb[q - 1] = b[p];
        }
    };
#pragma unroll
    for (int q = 0; q < A5_AHEAD && q < NR; q++) load_row(q);
    // keep the loads above ahead of the arithmetic below
    __builtin_amdgcn_sched_barrier(0);
    cd xs = czero(), xc = czero();
#pragma unroll
    for (int q = 0; q < NR; q++) {
        if (q + A5_AHEAD < NR) load_row(q + A5_AHEAD);
        const int jj = j0 - 1 + q;
        const double m = colin && jj >= 0 && jj < ny && unknown(L, ic, jj) ? 1.0 : 0.0;
        const cd xn = cscal(m, xb[q]);
        if (q >= 2) {
            // output row j = jj - 1: south xs, centre xc, north xn
            const int j = jj - 1;
            const cd xw = lane_from(xc, true), xe = lane_from(xc, false);
            if (outc && j < ny) {
                cd ap;
                double aw, ae, as, an;
                cd v = czero();
                const double kv = VARK ? kb[q - 2] : L.kc;
                if (coef5k(L, s, i, j, kv, ap, aw, ae, as, an)) {
                    v = cmul(ap, xc);
                    caxpy(v, aw, xw);
                    caxpy(v, ae, xe);
                    caxpy(v, as, xs);
                    caxpy(v, an, xn);
                    if (RESID) v = csub(bb[q - 2], v);
                }
                y[(size_t)j * nx + i] = v;
            }
        }
        xs = xc;
        xc = xn;
    }
}

hipError_t launch_apply5(const Lev &L, cd s, const cd *x, const cd *b, cd *y, hipStream_t st,
                         Batch bt)
{
    const int tx = cdiv(L.nx, A5_TX), ty = cdiv(L.ny, 4 * A5_RPW);
    const dim3 g(tx * ty, bt.B);
    if (L.k) {
        if (b)
            k_apply5<true, true><<<g, 256, 0, st>>>(L, s, x, b, y, tx, bt);
        else
            k_apply5<false, true><<<g, 256, 0, st>>>(L, s, x, b, y, tx, bt);
    } else {
        if (b)
            k_apply5<true, false><<<g, 256, 0, st>>>(L, s, x, b, y, tx, bt);
        else
            k_apply5<false, false><<<g, 256, 0, st>>>(L, s, x, b, y, tx, bt);
    }
    HD_LAUNCH_CHECK();
}

// ------------------------------------------------------------------------
// Per-node smoother coefficients.  With a constant wavenumber every node that
// is not on the grid boundary has the same diagonal, so the kernels take
// ap and omega/ap for those nodes as launch constants (no division per node);
// boundary nodes (Sommerfeld closure) and variable-k levels use coef5, always
// evaluated in FP64 and then rounded to the working precision R.
// Dirichlet boundary nodes are not unknowns and hold 0 in the LDS tiles, so
// the interior constants are exact for their unknown neighbours too.
// ------------------------------------------------------------------------
template <class R>
struct Smooth {
    R apr, api;  // interior diagonal (constant k)
    R wr, wi;    // omega / diagonal
    R ax, ay;    // interior off-diagonals -1/hx^2, -1/hy^2
};

template <class R>
Smooth<R> smooth_consts(const Lev &L, cd s, double omega)
{
    const double k2 = L.kc * L.kc;
    const double apr = 2.0 * L.ihx2 + 2.0 * L.ihy2 - s.x * k2, api = -s.y * k2;
    const double d = omega / (apr * apr + api * api);
    Smooth<R> c;
    c.apr = (R)apr;
    c.api = (R)api;
    c.wr = (R)(apr * d);
    c.wi = (R)(-api * d);
    c.ax = (R)(-L.ihx2);
    c.ay = (R)(-L.ihy2);
    return c;
}

// Coefficients of node (i,j) (inside the grid) in precision R, k being the
// wavenumber there (read only on variable-k levels and at boundary nodes).
// Returns false for a non-unknown node.  winv = omega / ap.
template <bool VARK, class R>
__device__ __forceinline__ bool node_coef_k(const Lev &L, cd s, double omega, const Smooth<R> &c,
                                            int i, int j, double k, cx<R> &ap, cx<R> &winv,
                                            R &aw, R &ae, R &as, R &an)
{
    const bool edge = i == 0 || j == 0 || i == L.nx - 1 || j == L.ny - 1;
    if (!VARK && !edge) {
        ap = mkc<R>(c.apr, c.api);
        winv = mkc<R>(c.wr, c.wi);
        aw = ae = c.ax;
        as = an = c.ay;
        return true;
    }
    if constexpr (std::is_same<R, double>::value) {
        if (!coef5k(L, s, i, j, k, ap, aw, ae, as, an)) return false;
        winv = cscal(omega, cinv(ap));
    } else {
        cd apd;
        double awd, aed, asd, and_;
        if (!coef5k(L, s, i, j, k, apd, awd, aed, asd, and_)) return false;
        ap = cvt<R>(apd);
        winv = cvt<R>(cscal(omega, cinv(apd)));
        aw = (R)awd;
        ae = (R)aed;
        as = (R)asd;
        an = (R)and_;
    }
    return true;
}

template <bool VARK, class R>
__device__ __forceinline__ bool node_coef(const Lev &L, cd s, double omega, const Smooth<R> &c,
                                          int i, int j, cx<R> &ap, cx<R> &winv, R &aw, R &ae,
                                          R &as, R &an)
{
    // a constant-k level (VARK false) has no k array: no load
    const double k = VARK ? kat(L, i, j) : L.kc;
    return node_coef_k<VARK, R>(L, s, omega, c, i, j, k, ap, winv, aw, ae, as, an);
}

// ------------------------------------------------------------------------
// V-cycle, downward pass on a level (fused):
//   x1 = omega D^{-1} r            (one damped-Jacobi sweep from x = 0)
//   r1 = r - M x1                  (residual)
//   rc = full weighting of r1      (1/16 [1 2 1; 2 4 2; 1 2 1], truncated)
// One block computes a 32 x 8 tile of coarse nodes from the 67 x 19 fine
// region it needs: r and x1 live in LDS, r1 overwrites r in place.
// Types: r is read in precision RI, everything is computed and rc stored in
// precision R (RI = R = double for the FP64 cycle; RI = double, R = float on
// the top level of the mixed-precision cycle; float, float below it).
// ------------------------------------------------------------------------
constexpr int VD_CX = 32, VD_CY = 8;
constexpr int VD_X1W = 2 * VD_CX + 3, VD_X1H = 2 * VD_CY + 3;  // 67 x 19

template <bool VARK, class RI, class R>
__global__ __launch_bounds__(256) void k_vc_down(Lev Lf, Lev Lc, cd s, double omega,
                                                 Smooth<R> c, const cx<RI> *__restrict__ r,
                                                 const cd *__restrict__ rs,
                                                 cx<R> *__restrict__ rc, int tiles_x, Batch bt)
{
    if (skip_rhs(bt)) return;
    r += (size_t)blockIdx.y * Lf.nx * Lf.ny;
    rc += (size_t)blockIdx.y * Lc.nx * Lc.ny;
    if (rs) rs += (size_t)blockIdx.y * SB;
    // Thread t owns the fine nodes of local column 2 + (t & 63), rows
    // 2 + 4 (t >> 6) .. + 3 (consecutive threads touch consecutive LDS
    // entries), keeping r and then r1 there in registers, and computes coarse
    // node (I0 + cx, J0 + cy), cx = t % 32, cy = t / 32, in the last phase.
    // One LDS tile (67 x 19, local (a, b) = fine (2*I0-2+a, 2*J0-2+b)) holds
    // x1, then is reused for r1.  The 249 halo nodes of the tile are spread
    // one per thread; those on the r1 ring (a == 1 or b == 1) also get r1.
    typedef cx<R> C;
    const R rsc = rs ? (R)rs[0].x : (R)1;  // right-hand side = rsc * r
    __shared__ C st[VD_X1H][VD_X1W];
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int I0 = (t % tiles_x) * VD_CX, J0 = (t / tiles_x) * VD_CY;
    const int fi0 = 2 * I0 - 2, fj0 = 2 * J0 - 2;
    const int cx_ = threadIdx.x % VD_CX, cy = threadIdx.x / VD_CX;
    const int ox = 2 + (threadIdx.x & 63), oy = 2 + (threadIdx.x >> 6) * 4;  // owned column/rows
    // halo node of this thread
    int ha = -1, hb = -1;
    {
        const int q = threadIdx.x;
        if (q < 3 * VD_X1H) {
            const int col = q / VD_X1H;
            ha = col == 0 ? 0 : (col == 1 ? 1 : VD_X1W - 1);
            hb = q % VD_X1H;
        } else if (q < 3 * VD_X1H + 3 * 2 * VD_CX) {
            const int qq = q - 3 * VD_X1H, row = qq / (2 * VD_CX);
            hb = row == 0 ? 0 : (row == 1 ? 1 : VD_X1H - 1);
            ha = 2 + qq % (2 * VD_CX);
        }
    }
    // ---- global loads (unconditional, from a valid address); r is taken
    // as 0 at non-unknown nodes (Dirichlet boundary) and outside the grid
    // (zeroing by a 0/1 factor rather than a select keeps the loads
    // unconditional: a select lets the compiler sink each load into a branch
    // that waits for it before the next one is issued)
    // On a variable-k level the wavenumber of the same nodes is loaded with r
    // (the coefficients of a node are used only where it is an unknown).
    C rown[4], rhalo;
    R mown[4], mhalo;
    double kown[4], khalo = 0.0;
#pragma unroll
    for (int d = 0; d < 4; d++) {
        const int fi = fi0 + ox, fj = fj0 + oy + d;
        const bool in = fi < Lf.nx && fj < Lf.ny && unknown(Lf, fi, fj);
        const size_t p = in ? (size_t)fj * Lf.nx + fi : 0;
        rown[d] = cvt<R>(r[p]);
        mown[d] = in ? (R)1 : (R)0;
        kown[d] = VARK ? Lf.k[p] : Lf.kc;
    }
    {
        const int fi = fi0 + ha, fj = fj0 + hb;
        const bool in = ha >= 0 && fi >= 0 && fi < Lf.nx && fj >= 0 && fj < Lf.ny &&
                        unknown(Lf, fi, fj);
        const size_t p = in ? (size_t)fj * Lf.nx + fi : 0;
        rhalo = cvt<R>(r[p]);
        mhalo = in ? (R)1 : (R)0;
        if (VARK) khalo = Lf.k[p];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int d = 0; d < 4; d++) rown[d] = cscal(mown[d], rs ? cscal(rsc, rown[d]) : rown[d]);
    rhalo = cscal(mhalo, rs ? cscal(rsc, rhalo) : rhalo);
    if (!VARK) khalo = Lf.kc;
    auto x1_at = [&](int fi, int fj, C rv, double kv) -> C {
        C ap, wv;
        R aw, ae, as, an;
        if (fi < 0 || fi >= Lf.nx || fj < 0 || fj >= Lf.ny ||
            !node_coef_k<VARK, R>(Lf, s, omega, c, fi, fj, kv, ap, wv, aw, ae, as, an))
            return zc<R>();
        return cmul(wv, rv);
    };
#pragma unroll
    for (int d = 0; d < 4; d++)
        st[oy + d][ox] = x1_at(fi0 + ox, fj0 + oy + d, rown[d], kown[d]);
    if (ha >= 0) st[hb][ha] = x1_at(fi0 + ha, fj0 + hb, rhalo, khalo);
    __syncthreads();
    // ---- r1 = r - M x1 at the owned nodes and the r1 ring
    auto r1_at = [&](int a, int b, C rv, double kv) -> C {
        const int fi = fi0 + a, fj = fj0 + b;
        C ap, wv;
        R aw, ae, as, an;
        if (fi < 0 || fi >= Lf.nx || fj < 0 || fj >= Lf.ny ||
            !node_coef_k<VARK, R>(Lf, s, omega, c, fi, fj, kv, ap, wv, aw, ae, as, an))
            return zc<R>();
        C m = cmul(ap, st[b][a]);
        caxpy(m, aw, st[b][a - 1]);
        caxpy(m, ae, st[b][a + 1]);
        caxpy(m, as, st[b - 1][a]);
        caxpy(m, an, st[b + 1][a]);
        return csub(rv, m);
    };
    C r1own[4], r1halo = zc<R>();
#pragma unroll
    for (int d = 0; d < 4; d++) r1own[d] = r1_at(ox, oy + d, rown[d], kown[d]);
    const bool ring = ha >= 1 && ha <= VD_X1W - 2 && hb >= 1 && hb <= VD_X1H - 2;
    if (ring) r1halo = r1_at(ha, hb, rhalo, khalo);
    __syncthreads();
#pragma unroll
    for (int d = 0; d < 4; d++) st[oy + d][ox] = r1own[d];
    if (ring) st[hb][ha] = r1halo;
    __syncthreads();
    // ---- full weighting around fine node (2I, 2J) = local (2cx+2, 2cy+2)
    const int I = I0 + cx_, J = J0 + cy;
    if (I >= Lc.nx || J >= Lc.ny) return;
    C v = zc<R>();
    if (unknown(Lc, I, J)) {
        const int a = 2 * cx_ + 2, bb = 2 * cy + 2;
        C ce = cscal((R)4, st[bb][a]);
        C e = cadd(cadd(st[bb][a - 1], st[bb][a + 1]), cadd(st[bb - 1][a], st[bb + 1][a]));
        C d = cadd(cadd(st[bb - 1][a - 1], st[bb - 1][a + 1]),
                   cadd(st[bb + 1][a - 1], st[bb + 1][a + 1]));
        v = cscal((R)(1.0 / 16.0), cadd(cadd(ce, cscal((R)2, e)), d));
    }
    rc[(size_t)J * Lc.nx + I] = v;
}

template <class RI, class R>
static hipError_t vc_down_t(const Lev &Lf, const Lev &Lc, cd s, double omega, const cx<RI> *r,
                            const cd *rs, cx<R> *rc, hipStream_t st, Batch bt)
{
    const int tx = cdiv(Lc.nx, VD_CX), ty = cdiv(Lc.ny, VD_CY);
    const Smooth<R> c = smooth_consts<R>(Lf, s, omega);
    const dim3 g(tx * ty, bt.B);
    if (Lf.k)
        k_vc_down<true, RI, R><<<g, 256, 0, st>>>(Lf, Lc, s, omega, c, r, rs, rc, tx, bt);
    else
        k_vc_down<false, RI, R><<<g, 256, 0, st>>>(Lf, Lc, s, omega, c, r, rs, rc, tx, bt);
    HD_LAUNCH_CHECK();
}

hipError_t launch_vc_down(const Lev &Lf, const Lev &Lc, cd s, double omega, const cd *r,
                          const cd *rs, cd *rc, hipStream_t st, Batch bt)
{
    return vc_down_t<double, double>(Lf, Lc, s, omega, r, rs, rc, st, bt);
}

hipError_t launch_vc_down(const Lev &Lf, const Lev &Lc, cd s, double omega, const cd *r, cf *rc,
                          hipStream_t st, Batch bt)
{
    return vc_down_t<double, float>(Lf, Lc, s, omega, r, nullptr, rc, st, bt);
}

hipError_t launch_vc_down(const Lev &Lf, const Lev &Lc, cd s, double omega, const cf *r, cf *rc,
                          hipStream_t st, Batch bt)
{
    return vc_down_t<float, float>(Lf, Lc, s, omega, r, nullptr, rc, st, bt);
}

hipError_t launch_vc_down(const Lev &Lf, const Lev &Lc, cd s, double omega, const cf *r,
                          const cd *rs, cd *rc, hipStream_t st)
{
    return vc_down_t<float, double>(Lf, Lc, s, omega, r, rs, rc, st, Batch{});
}

// (q / w, q % w) for 0 <= q < 2^12, 0 < w < 2^8 by a float reciprocal: the
// quotient's fraction is at least 1/(2w) from an integer, far above the error
struct Div {
    float rw;
    int w;
    __device__ explicit Div(int w_) : rw(1.0f / (float)w_), w(w_) {}
    __device__ int quo(int q) const { return (int)(((float)q + 0.5f) * rw); }
};

// ------------------------------------------------------------------------
// The downward passes of the last nd <= 3 levels above the coarsest fused
// into one launch.  A block owns a DT_C x DT_C tile [A, B] of the coarsest
// level and computes its right-hand side from level Lc - nd's: the tile needs
// r1 of level Lc - 1 on [2A-1, 2B+1], hence x1 and r there grown by one node,
// so level Lc - j contributes its r on G_j = [2^j A - (2^(j+1) - 2),
// 2^j B + (2^(j+1) - 2)] (37 x 37 nodes at j = 3).  The block loads r on G_nd
// once and computes every stage in LDS: x1 on G_j, r1 on G_j shrunk by one
// node, full weighting on G_(j-1), each in k_vc_down's expressions and order
// (no right-hand side scale), with 0 outside the grid and at nodes that are
// not unknowns, as k_vc_down's tile and output hold.  Level Lc - j + 1's
// right-hand side is also needed by the upward pass: each block writes the
// nodes it owns there, [2^(j-1) A, 2^(j-1) (B+1) - 1] per axis (a partition of
// the level; the last tile's range runs past the grid's end).
// ------------------------------------------------------------------------
constexpr int DT_C = 2;                        // coarsest nodes per tile side
constexpr int DT_G = 8 * (DT_C - 1) + 29;      // side of G_3 (37)
constexpr int DT_N = DT_G * DT_G;              // nodes of G_3
constexpr int DT_T = 512;                      // threads per block
constexpr int DT_S = (DT_N + DT_T - 1) / DT_T;  // r loads per thread

struct DTailArgs {
    int nd;                         // fused levels Lc - nd .. Lc - 1
    int tiles_x;                    // tiles per row of the coarsest level
    Lev L[VC_DTAIL_MAXLEV + 1];     // L[j]: level Lc - j (L[0]: the coarsest)
    Smooth<double> c[VC_DTAIL_MAXLEV + 1];  // c[j]: level Lc - j, j >= 1
    const cd *r;                    // right-hand side of level Lc - nd
    cd *out[VC_DTAIL_MAXLEV];       // out[j]: right-hand side of level Lc - j, j < nd
};

template <bool VARK>
__global__ __launch_bounds__(DT_T) void k_vc_down_tail(DTailArgs a, cd s, double omega)
{
    __shared__ cd rb[DT_N];    // r on G_j
    __shared__ cd x1b[DT_N];   // x1 on G_j, then r1 on G_j shrunk by one node
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int nd = a.nd;
    const int A = (t % a.tiles_x) * DT_C, Ay = (t / a.tiles_x) * DT_C;
    // ---- r of level Lc - nd on G_nd (masked like k_vc_down's loads)
    {
        const Lev &L = a.L[nd];
        const int lox = (A << nd) - ((2 << nd) - 2), loy = (Ay << nd) - ((2 << nd) - 2);
        const int w = (DT_C - 1) * (1 << nd) + (4 << nd) - 3;
        const Div d(w);
        cd v[DT_S];
        double m[DT_S];
#pragma unroll
        for (int sl = 0; sl < DT_S; sl++) {
            const int q = threadIdx.x + DT_T * sl;
            const int qy = d.quo(q);
            const int fi = lox + q - qy * w, fj = loy + qy;
            const bool in = q < w * w && fi >= 0 && fi < L.nx && fj >= 0 && fj < L.ny &&
                            unknown(L, fi, fj);
            v[sl] = a.r[in ? (size_t)fj * L.nx + fi : 0];
            m[sl] = in ? 1.0 : 0.0;
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int sl = 0; sl < DT_S; sl++) {
            const int q = threadIdx.x + DT_T * sl;
            if (q < w * w) rb[q] = cscal(m[sl], v[sl]);
        }
    }
    __syncthreads();
    for (int j = nd; j >= 1; j--) {
        const Lev &L = a.L[j];
        const Lev &Lc = a.L[j - 1];
        const Smooth<double> &c = a.c[j];
        const int lox = (A << j) - ((2 << j) - 2), loy = (Ay << j) - ((2 << j) - 2);
        const int w = (DT_C - 1) * (1 << j) + (4 << j) - 3;
        // x1 = omega D^-1 r on G_j
        {
            const Div d(w);
            for (int q = threadIdx.x; q < w * w; q += DT_T) {
                const int qy = d.quo(q);
                const int fi = lox + q - qy * w, fj = loy + qy;
                cd x = czero();
                cd ap, wv;
                double aw, ae, as, an;
                if (fi >= 0 && fi < L.nx && fj >= 0 && fj < L.ny &&
                    node_coef<VARK, double>(L, s, omega, c, fi, fj, ap, wv, aw, ae, as, an))
                    x = cmul(wv, rb[q]);
                x1b[q] = x;
            }
        }
        __syncthreads();
        // r1 = r - M x1 on G_j shrunk by one node (kept in registers until
        // every thread has read x1)
        const int w1 = w - 2;
        constexpr int NR = (DT_G - 2) * (DT_G - 2) / DT_T + 1;
        cd r1[NR];
        {
            const Div d(w1);
#pragma unroll
            for (int sl = 0; sl < NR; sl++) {
                const int q = threadIdx.x + DT_T * sl;
                r1[sl] = czero();
                if (q >= w1 * w1) continue;
                const int qy = d.quo(q);
                const int ii = q - qy * w1 + 1, jj = qy + 1;
                const int fi = lox + ii, fj = loy + jj;
                const int cxy = jj * w + ii;
                cd ap, wv;
                double aw, ae, as, an;
                if (fi >= 0 && fi < L.nx && fj >= 0 && fj < L.ny &&
                    node_coef<VARK, double>(L, s, omega, c, fi, fj, ap, wv, aw, ae, as, an)) {
                    cd mm = cmul(ap, x1b[cxy]);
                    caxpy(mm, aw, x1b[cxy - 1]);
                    caxpy(mm, ae, x1b[cxy + 1]);
                    caxpy(mm, as, x1b[cxy - w]);
                    caxpy(mm, an, x1b[cxy + w]);
                    r1[sl] = csub(rb[cxy], mm);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int sl = 0; sl < NR; sl++) {
            const int q = threadIdx.x + DT_T * sl;
            if (q < w1 * w1) x1b[q] = r1[sl];
        }
        __syncthreads();
        // full weighting on G_(j-1) = [lox/2 + 1, ...]: coarse node (I, J) sits
        // at fine (2I, 2J) = r1 entry (2(I - clo) + 1, 2(J - cloy) + 1)
        {
            const int clox = (lox + 2) >> 1, cloy = (loy + 2) >> 1;
            const int cw = (w - 3) >> 1;
            const int ox = A << (j - 1), oy = Ay << (j - 1);  // owned range
            const int on = DT_C << (j - 1);
            const Div d(cw);
            for (int q = threadIdx.x; q < cw * cw; q += DT_T) {
                const int qy = d.quo(q);
                const int I = clox + q - qy * cw, J = cloy + qy;
                const bool ing = I >= 0 && I < Lc.nx && J >= 0 && J < Lc.ny;
                cd v = czero();
                if (ing && unknown(Lc, I, J)) {
                    const int aa = 2 * (I - clox) + 1, bb = 2 * (J - cloy) + 1;
                    const cd *rr = x1b + bb * w1 + aa;
                    cd ce = cscal(4.0, rr[0]);
                    cd e = cadd(cadd(rr[-1], rr[1]), cadd(rr[-w1], rr[w1]));
                    cd dd = cadd(cadd(rr[-w1 - 1], rr[-w1 + 1]), cadd(rr[w1 - 1], rr[w1 + 1]));
                    v = cscal(1.0 / 16.0, cadd(cadd(ce, cscal(2.0, e)), dd));
                }
                rb[q] = v;
                if (ing && I >= ox && I < ox + on && J >= oy && J < oy + on)
                    a.out[j - 1][(size_t)J * Lc.nx + I] = v;
            }
        }
        __syncthreads();
    }
}

hipError_t launch_vc_down_tail(int nd, const Lev *levs, const cd *r, cd *const *out, cd s,
                               double omega, hipStream_t st)
{
    if (nd < 1 || nd > VC_DTAIL_MAXLEV) return hipErrorInvalidValue;
    DTailArgs a;
    a.nd = nd;
    a.tiles_x = cdiv(levs[0].nx, DT_C);
    bool vark = false;
    for (int j = 0; j <= nd; j++) {
        a.L[j] = levs[j];
        vark |= levs[j].k != nullptr;
        a.c[j] = j ? smooth_consts<double>(levs[j], s, omega) : Smooth<double>{};
    }
    for (int j = 0; j < nd; j++) a.out[j] = out[j];
    a.r = r;
    const int g = a.tiles_x * cdiv(levs[0].ny, DT_C);
    if (vark)
        k_vc_down_tail<true><<<g, DT_T, 0, st>>>(a, s, omega);
    else
        k_vc_down_tail<false><<<g, DT_T, 0, st>>>(a, s, omega);
    HD_LAUNCH_CHECK();
}

// ------------------------------------------------------------------------
// V-cycle, upward pass on a level (fused):
//   x2 = omega D^{-1} r + P ec      (the pre-smoothed iterate, recomputed,
//                                    plus the bilinear coarse correction)
//   x3 = x2 + omega D^{-1} (r - M x2)   (post-smoothing sweep)
//   out = x3 [+ Z v2] [+ out]
// One block writes a 64 x 16 fine tile.  r (66 x 18), the coarse correction
// tile (34 x 10) and x2 (66 x 18) live in LDS.
// Types: r is read in precision RI, ec and the arithmetic are in R, out is
// stored in RO; Z v2 (always FP64, level-0 deflation term) is added in FP64
// when RO is double.
// ------------------------------------------------------------------------
constexpr int VU_TX = 64, VU_TY = 16;
constexpr int VU_W = VU_TX + 2, VU_H = VU_TY + 2;
constexpr int VU_CW = VU_TX / 2 + 2, VU_CH = VU_TY / 2 + 2;  // 34 x 10

template <bool VARK, class RI, class R, class RO, bool V2>
__global__ __launch_bounds__(256) void k_vc_up(Lev Lf, Lev Lc, cd s, double omega, Smooth<R> c,
                                               const cx<RI> *__restrict__ r,
                                               const cd *__restrict__ rs,
                                               const cx<R> *__restrict__ ec,
                                               cx<RO> *__restrict__ out, int accumulate,
                                               const cd *__restrict__ v2, int zho, int tiles_x,
                                               Batch bt)
{
    if (skip_rhs(bt)) return;
    {
        const size_t nf = (size_t)Lf.nx * Lf.ny, nc = (size_t)Lc.nx * Lc.ny;
        r += blockIdx.y * nf;
        out += blockIdx.y * nf;
        ec += blockIdx.y * nc;
        if (v2) v2 += blockIdx.y * nc;
        if (rs) rs += (size_t)blockIdx.y * SB;
    }
    // Thread (tx, ty) owns output column tx and rows 4*ty .. 4*ty+3 of the
    // 64 x 16 tile and keeps r there in registers; x2 (66 x 18 with its
    // one-node halo) and the coarse correction tile (34 x 10) live in LDS.
    typedef cx<R> C;
    const R rsc = rs ? (R)rs[0].x : (R)1;  // right-hand side = rsc * r
    __shared__ C sx2[VU_H][VU_W];
    __shared__ C se[VU_CH][VU_CW];
    // Z v2 term (level 0 only, V2): v2 on the coarse tile
    __shared__ cd sv2[V2 ? VU_CH : 1][V2 ? VU_CW : 1];
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int i0 = (t % tiles_x) * VU_TX, j0 = (t / tiles_x) * VU_TY;
    const int ci0 = i0 / 2 - 1, cj0 = j0 / 2 - 1;  // coarse tile origin
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    constexpr int NC = VU_CW * VU_CH, NKC = (NC + 255) / 256;
    constexpr int NHALO = 2 * VU_H + 2 * VU_TX;  // 164 halo nodes of the x2 tile
    // the halo node of this thread (threads >= NHALO have none)
    int ha = -1, hb = -1;
    {
        const int q = threadIdx.x;
        if (q < VU_H) {
            ha = 0;
            hb = q;
        } else if (q < 2 * VU_H) {
            ha = VU_W - 1;
            hb = q - VU_H;
        } else if (q < 2 * VU_H + VU_TX) {
            ha = q - 2 * VU_H + 1;
            hb = 0;
        } else if (q < NHALO) {
            ha = q - 2 * VU_H - VU_TX + 1;
            hb = VU_H - 1;
        }
    }
    // ---- all global loads first (unconditional, from a valid address)
    // (zeroing by a 0/1 factor rather than a select keeps the loads
    // unconditional, see k_vc_down)
    // (on a variable-k level the wavenumber of the same nodes comes with r;
    // when accumulating, the old output of the owned nodes too)
    C el[NKC], rown[4], rhalo;
    R mel[NKC], mown[4], mhalo;
    double kown[4], khalo = 0.0;
    cx<RO> oold[4];
#pragma unroll
    for (int kq = 0; kq < NKC; kq++) {
        const int q = threadIdx.x + 256 * kq;
        const int I = ci0 + q % VU_CW, J = cj0 + q / VU_CW;
        const bool in = q < NC && I >= 0 && I < Lc.nx && J >= 0 && J < Lc.ny && unknown(Lc, I, J);
        el[kq] = ec[in ? (size_t)J * Lc.nx + I : 0];
        mel[kq] = in ? (R)1 : (R)0;
    }
    const int i = i0 + tx;
#pragma unroll
    for (int rr = 0; rr < 4; rr++) {
        const int j = j0 + 4 * ty + rr;
        const bool in = i < Lf.nx && j < Lf.ny && unknown(Lf, i, j);
        const size_t p = in ? (size_t)j * Lf.nx + i : 0;
        rown[rr] = cvt<R>(r[p]);
        mown[rr] = in ? (R)1 : (R)0;
        kown[rr] = VARK ? Lf.k[p] : Lf.kc;
    }
    if (accumulate) {
#pragma unroll
        for (int rr = 0; rr < 4; rr++) {
            const int j = j0 + 4 * ty + rr;
            oold[rr] = out[i < Lf.nx && j < Lf.ny ? (size_t)j * Lf.nx + i : 0];
        }
    }
    // v2 on the same coarse tile as ec: every coarse node the Z rule reaches
    // from the owned fine nodes; nodes outside the grid or not unknowns hold
    // 0, as the rule leaves them out (zeroed by a 0/1 factor, see above)
    cd v2l[V2 ? NKC : 1];
    double mv2[V2 ? NKC : 1];
    if constexpr (V2) {
#pragma unroll
        for (int kq = 0; kq < NKC; kq++) {
            const int q = threadIdx.x + 256 * kq;
            const int I = ci0 + q % VU_CW, J = cj0 + q / VU_CW;
            const bool in = q < NC && I >= 0 && I < Lc.nx && J >= 0 && J < Lc.ny &&
                            unknown(Lc, I, J);
            v2l[kq] = v2[in ? (size_t)J * Lc.nx + I : 0];
            mv2[kq] = in ? 1.0 : 0.0;
        }
    }
    {
        const int fi = i0 - 1 + ha, fj = j0 - 1 + hb;
        const bool in = ha >= 0 && fi >= 0 && fi < Lf.nx && fj >= 0 && fj < Lf.ny &&
                        unknown(Lf, fi, fj);
        const size_t p = in ? (size_t)fj * Lf.nx + fi : 0;
        rhalo = cvt<R>(r[p]);
        mhalo = in ? (R)1 : (R)0;
        if (VARK) khalo = Lf.k[p];
    }
    __builtin_amdgcn_sched_barrier(0);
    if (!VARK) khalo = Lf.kc;
#pragma unroll
    for (int kq = 0; kq < NKC; kq++) el[kq] = cscal(mel[kq], el[kq]);
#pragma unroll
    for (int rr = 0; rr < 4; rr++)
        rown[rr] = cscal(mown[rr], rs ? cscal(rsc, rown[rr]) : rown[rr]);
    rhalo = cscal(mhalo, rs ? cscal(rsc, rhalo) : rhalo);
#pragma unroll
    for (int kq = 0; kq < NKC; kq++) {
        const int q = threadIdx.x + 256 * kq;
        if (q < NC) se[q / VU_CW][q % VU_CW] = el[kq];
        if constexpr (V2)
            if (q < NC) sv2[q / VU_CW][q % VU_CW] = cscal(mv2[kq], v2l[kq]);
    }
    __syncthreads();
    // ---- x2 = omega D^-1 r + P ec at the owned nodes and the halo node
    auto x2_at = [&](int fi, int fj, C rv, double kv) -> C {
        C ap, wv;
        R aw, ae, as, an;
        if (fi < 0 || fi >= Lf.nx || fj < 0 || fj >= Lf.ny ||
            !node_coef_k<VARK, R>(Lf, s, omega, c, fi, fj, kv, ap, wv, aw, ae, as, an))
            return zc<R>();
        // bilinear interpolation from the coarse tile: coarse node
        // (fi >> 1, fj >> 1) sits at se[(fj >> 1) - cj0][(fi >> 1) - ci0]
        const int ca = (fi >> 1) - ci0, cb = (fj >> 1) - cj0;
        C p = se[cb][ca];
        if (fi & 1) p = cscal((R)0.5, cadd(p, se[cb][ca + 1]));
        if (fj & 1) {
            C p2 = se[cb + 1][ca];
            if (fi & 1) p2 = cscal((R)0.5, cadd(p2, se[cb + 1][ca + 1]));
            p = cscal((R)0.5, cadd(p, p2));
        }
        return cadd(cmul(wv, rv), p);
    };
#pragma unroll
    for (int rr = 0; rr < 4; rr++) {
        const int jl = 4 * ty + rr;
        sx2[jl + 1][tx + 1] = x2_at(i, j0 + jl, rown[rr], kown[rr]);
    }
    if (ha >= 0) sx2[hb][ha] = x2_at(i0 - 1 + ha, j0 - 1 + hb, rhalo, khalo);
    __syncthreads();
    // ---- post-smoothing at the owned nodes
    if (i >= Lf.nx) return;
#pragma unroll
    for (int rr = 0; rr < 4; rr++) {
        const int jl = 4 * ty + rr;
        const int j = j0 + jl;
        if (j >= Lf.ny) break;
        const int a = tx + 1, bb = jl + 1;
        const size_t p = (size_t)j * Lf.nx + i;
        C ap, wv;
        R aw, ae, as, an;
        cx<RO> v = zc<RO>();
        if (node_coef_k<VARK, R>(Lf, s, omega, c, i, j, kown[rr], ap, wv, aw, ae, as, an)) {
            C m = cmul(ap, sx2[bb][a]);
            caxpy(m, aw, sx2[bb][a - 1]);
            caxpy(m, ae, sx2[bb][a + 1]);
            caxpy(m, as, sx2[bb - 1][a]);
            caxpy(m, an, sx2[bb + 1][a]);
            v = cvt<RO>(cadd(sx2[bb][a], cmul(wv, csub(rown[rr], m))));
            if constexpr (V2) v = cadd(v, cvt<RO>(zv2_tile(sv2, i - 2 * ci0, j - 2 * cj0, zho)));
        }
        if (accumulate) v = cadd(v, oold[rr]);
        out[p] = v;
    }
}

// ------------------------------------------------------------------------
// The upward passes of the small levels fused into one launch: a block owns a
// VT_TX x VT_TY tile of level lt and computes the corrections of every level
// from the coarsest up to lt on the nodes its tile needs, in LDS.  Level k's
// output region R_k (k = 0 is level lt) needs x2 on R_k grown by one node, so
// the correction of level k+1 on R_{k+1} = [floor((a-1)/2), ceil((b+1)/2)]
// per axis; the regions shrink by about half per level (32 x 16, 18 x 10,
// 11 x 7, 7 x 5, ...), so the redundant work below level lt is small.  Each
// stage is k_vc_up's arithmetic, in its order (r from the level's buffer, no
// right-hand side scale, no accumulation, no Z v2), and nodes outside the grid
// or not unknowns hold 0, as k_vc_up's output there and its masked ec tile do.
// The kernel is latency bound (a few thousand nodes per block over several
// dependent stages), so the loads are pipelined: thread q of a stage's grown
// region loads r (and k) there into registers one stage ahead, uses them for
// x2 and leaves them in LDS for the smoothing of the same nodes.
// ------------------------------------------------------------------------
constexpr int VT_TX = 32, VT_TY = 16;                       // tile of level lt
constexpr int VT_E = (VT_TX / 2 + 2) * (VT_TY / 2 + 2);     // largest region below lt
constexpr int VT_X = (VT_TX + 2) * (VT_TY + 2);             // largest x2 region (level lt)
constexpr int VT_T = 256;                                   // threads per block
constexpr int VT_S = (VT_X + VT_T - 1) / VT_T;              // x2 nodes per thread

struct TailArgs {
    int nt;                         // levels lt .. lt + nt - 1 (the last is above the coarsest)
    int tiles_x;
    Lev L[VC_TAIL_MAXLEV + 1];      // L[k]: level lt + k; L[nt]: the coarsest level
    Smooth<double> c[VC_TAIL_MAXLEV];
    const cd *r[VC_TAIL_MAXLEV];    // right-hand side of level lt + k
    const cd *xc;                   // coarsest solution
    cd *out;                        // correction of level lt
};


template <bool VARK>
__global__ __launch_bounds__(VT_T) void k_vc_up_tail(TailArgs a, cd s, double omega)
{
    __shared__ cd x2b[VT_X];
    __shared__ cd rbuf[VT_X];                 // r on the stage's grown region
    __shared__ double kbuf[VARK ? VT_X : 1];  // k there (variable k)
    __shared__ cd eb[2][VT_E];
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int nt = a.nt;
    int ia[VC_TAIL_MAXLEV + 1], ib[VC_TAIL_MAXLEV + 1], ja[VC_TAIL_MAXLEV + 1],
        jb[VC_TAIL_MAXLEV + 1];
    ia[0] = (t % a.tiles_x) * VT_TX;
    ib[0] = ia[0] + VT_TX - 1;
    ja[0] = (t / a.tiles_x) * VT_TY;
    jb[0] = ja[0] + VT_TY - 1;
#pragma unroll
    for (int k = 0; k < VC_TAIL_MAXLEV; k++) {
        ia[k + 1] = (ia[k] - 1) >> 1;
        ib[k + 1] = (ib[k] + 2) >> 1;
        ja[k + 1] = (ja[k] - 1) >> 1;
        jb[k + 1] = (jb[k] + 2) >> 1;
    }
    // r (and k) of level k's grown region at this thread's nodes q = tid + VT_T sl,
    // masked to 0 outside the grid (loads unconditional, from a valid address)
    cd rn[VT_S];
    double kn[VT_S], mn[VT_S];
    auto load_level = [&](int k) {
        const Lev &L = a.L[k];
        const cd *__restrict__ r = a.r[k];
        const int xw = ib[k] - ia[k] + 3, xh = jb[k] - ja[k] + 3;
        const Div d(xw);
#pragma unroll
        for (int sl = 0; sl < VT_S; sl++) {
            const int q = threadIdx.x + VT_T * sl;
            const int qy = d.quo(q);
            const int fi = ia[k] - 1 + q - qy * xw, fj = ja[k] - 1 + qy;
            const bool in = q < xw * xh && fi >= 0 && fi < L.nx && fj >= 0 && fj < L.ny;
            const size_t p = in ? (size_t)fj * L.nx + fi : 0;
            rn[sl] = r[p];
            if (VARK) kn[sl] = L.k[p];
            mn[sl] = in ? 1.0 : 0.0;
        }
    };
    {  // the coarsest solution on R_nt, with the first stage's r
        const Lev &Lc = a.L[nt];
        const int w = ib[nt] - ia[nt] + 1, hh = jb[nt] - ja[nt] + 1;
        const Div d(w);
        constexpr int NE = (VT_E + VT_T - 1) / VT_T;
        cd ce[NE];
        double cm[NE];
#pragma unroll
        for (int sl = 0; sl < NE; sl++) {
            const int q = threadIdx.x + VT_T * sl;
            const int qy = d.quo(q);
            const int I = ia[nt] + q - qy * w, J = ja[nt] + qy;
            const bool in = q < w * hh && I >= 0 && I < Lc.nx && J >= 0 && J < Lc.ny &&
                            unknown(Lc, I, J);
            ce[sl] = a.xc[in ? (size_t)J * Lc.nx + I : 0];
            cm[sl] = in ? 1.0 : 0.0;
        }
        load_level(nt - 1);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int sl = 0; sl < NE; sl++) {
            const int q = threadIdx.x + VT_T * sl;
            if (q < w * hh) eb[nt & 1][q] = cscal(cm[sl], ce[sl]);
        }
    }
    __syncthreads();
    for (int k = nt - 1; k >= 0; k--) {
        const Lev &L = a.L[k];
        const Smooth<double> &c = a.c[k];
        const cd *ec = eb[(k + 1) & 1];
        const int ew = ib[k + 1] - ia[k + 1] + 1;
        const int xw = ib[k] - ia[k] + 3, xh = jb[k] - ja[k] + 3;
        // x2 = omega D^-1 r + P e on R_k grown by one node (this thread's nodes)
        {
            const Div d(xw);
#pragma unroll
            for (int sl = 0; sl < VT_S; sl++) {
                const int q = threadIdx.x + VT_T * sl;
                if (q >= xw * xh) break;
                const int qy = d.quo(q);
                const int fi = ia[k] - 1 + q - qy * xw, fj = ja[k] - 1 + qy;
                const cd rv = cscal(mn[sl], rn[sl]);
                cd x = czero();
                cd ap, wv;
                double aw, ae, as, an;
                if (fi >= 0 && fi < L.nx && fj >= 0 && fj < L.ny &&
                    node_coef_k<VARK, double>(L, s, omega, c, fi, fj, VARK ? kn[sl] : L.kc, ap,
                                              wv, aw, ae, as, an)) {
                    const int ca = (fi >> 1) - ia[k + 1], cb = (fj >> 1) - ja[k + 1];
                    cd p = ec[cb * ew + ca];
                    if (fi & 1) p = cscal(0.5, cadd(p, ec[cb * ew + ca + 1]));
                    if (fj & 1) {
                        cd p2 = ec[(cb + 1) * ew + ca];
                        if (fi & 1) p2 = cscal(0.5, cadd(p2, ec[(cb + 1) * ew + ca + 1]));
                        p = cscal(0.5, cadd(p, p2));
                    }
                    x = cadd(cmul(wv, rv), p);
                }
                x2b[q] = x;
                rbuf[q] = rv;
                if (VARK) kbuf[q] = kn[sl];
            }
        }
        // the next stage's loads fly during this stage's smoothing
        if (k > 0) load_level(k - 1);
        __syncthreads();
        // post-smoothing on R_k: the correction of level k
        const int ow = xw - 2, oh = xh - 2;
        const Div d(ow);
        for (int q = threadIdx.x; q < ow * oh; q += VT_T) {
            const int jj = d.quo(q), ii = q - jj * ow;
            const int fi = ia[k] + ii, fj = ja[k] + jj;
            const int cxy = (jj + 1) * xw + ii + 1;
            const bool ing = fi >= 0 && fi < L.nx && fj >= 0 && fj < L.ny;
            cd x = czero();
            cd ap, wv;
            double aw, ae, as, an;
            if (ing && node_coef_k<VARK, double>(L, s, omega, c, fi, fj,
                                                 VARK ? kbuf[cxy] : L.kc, ap, wv, aw, ae, as,
                                                 an)) {
                cd m = cmul(ap, x2b[cxy]);
                caxpy(m, aw, x2b[cxy - 1]);
                caxpy(m, ae, x2b[cxy + 1]);
                caxpy(m, as, x2b[cxy - xw]);
                caxpy(m, an, x2b[cxy + xw]);
                x = cadd(x2b[cxy], cmul(wv, csub(rbuf[cxy], m)));
            }
            if (k == 0) {
                if (ing) a.out[(size_t)fj * L.nx + fi] = x;
            } else {
                eb[k & 1][q] = x;
            }
        }
        __syncthreads();
    }
}

hipError_t launch_vc_up_tail(int nt, const Lev *levs, const cd *const *r, const cd *xc, cd *out,
                             cd s, double omega, hipStream_t st)
{
    if (nt < 1 || nt > VC_TAIL_MAXLEV) return hipErrorInvalidValue;
    TailArgs a;
    a.nt = nt;
    a.tiles_x = cdiv(levs[0].nx, VT_TX);
    bool vark = false;
    for (int k = 0; k <= nt; k++) {
        a.L[k] = levs[k];
        vark |= levs[k].k != nullptr;
    }
    for (int k = 0; k < nt; k++) {
        a.c[k] = smooth_consts<double>(levs[k], s, omega);
        a.r[k] = r[k];
    }
    a.xc = xc;
    a.out = out;
    const int g = a.tiles_x * cdiv(levs[0].ny, VT_TY);
    if (vark)
        k_vc_up_tail<true><<<g, VT_T, 0, st>>>(a, s, omega);
    else
        k_vc_up_tail<false><<<g, VT_T, 0, st>>>(a, s, omega);
    HD_LAUNCH_CHECK();
}

template <class RI, class R, class RO>
static hipError_t vc_up_t(const Lev &Lf, const Lev &Lc, cd s, double omega, const cx<RI> *r,
                          const cd *rs, const cx<R> *ec, cx<RO> *out, int accumulate,
                          const cd *v2, int zho, hipStream_t st, Batch bt)
{
    const int tx = cdiv(Lf.nx, VU_TX), ty = cdiv(Lf.ny, VU_TY);
    const Smooth<R> c = smooth_consts<R>(Lf, s, omega);
    const dim3 g(tx * ty, bt.B);
#define VU_LAUNCH(VK, V2)                                                                      \
    k_vc_up<VK, RI, R, RO, V2><<<g, 256, 0, st>>>(Lf, Lc, s, omega, c, r, rs, ec, out, accumulate, \
                                                  v2, zho, tx, bt)
    if (Lf.k) {
        if (v2)
            VU_LAUNCH(true, true);
        else
            VU_LAUNCH(true, false);
    } else {
        if (v2)
            VU_LAUNCH(false, true);
        else
            VU_LAUNCH(false, false);
    }
#undef VU_LAUNCH
    HD_LAUNCH_CHECK();
}

hipError_t launch_vc_up(const Lev &Lf, const Lev &Lc, cd s, double omega, const cd *r,
                        const cd *rs, const cd *ec, cd *out, int accumulate, const cd *v2, int zho,
                        hipStream_t st, Batch bt)
{
    return vc_up_t<double, double, double>(Lf, Lc, s, omega, r, rs, ec, out, accumulate, v2, zho,
                                           st, bt);
}

hipError_t launch_vc_up(const Lev &Lf, const Lev &Lc, cd s, double omega, const cd *r,
                        const cf *ec, cd *out, int accumulate, const cd *v2, int zho,
                        hipStream_t st, Batch bt)
{
    return vc_up_t<double, float, double>(Lf, Lc, s, omega, r, nullptr, ec, out, accumulate, v2,
                                          zho, st, bt);
}

hipError_t launch_vc_up(const Lev &Lf, const Lev &Lc, cd s, double omega, const cf *r,
                        const cf *ec, cf *out, hipStream_t st, Batch bt)
{
    return vc_up_t<float, float, float>(Lf, Lc, s, omega, r, nullptr, ec, out, 0, nullptr, 0, st,
                                        bt);
}

hipError_t launch_vc_up(const Lev &Lf, const Lev &Lc, cd s, double omega, const cf *r,
                        const cd *rs, const cd *ec, cd *out, int accumulate, hipStream_t st)
{
    return vc_up_t<float, double, double>(Lf, Lc, s, omega, r, rs, ec, out, accumulate, nullptr, 0,
                                          st, Batch{});
}

// ------------------------------------------------------------------------
// Coarsest level: x = Minv r with the precomputed dense inverse (FP64, or its
// FP32 rounding for the mixed-precision cycle).  One wave per row: the lanes
// stride along the row (coalesced) and reduce by shuffles.
// ------------------------------------------------------------------------
__device__ __forceinline__ double shfl_xor64(double v, int o) { return __shfl_xor(v, o, 64); }
__device__ __forceinline__ float shfl_xor64(float v, int o) { return __shfl_xor(v, o, 64); }

template <class R>
__device__ __forceinline__ cx<R> wave_sum64(cx<R> v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        v.x += shfl_xor64(v.x, o);
        v.y += shfl_xor64(v.y, o);
    }
    return v;
}

template <class R>
__global__ __launch_bounds__(256) void k_coarsest(int n, const cx<R> *__restrict__ Minv,
                                                  const cx<R> *__restrict__ r,
                                                  cx<R> *__restrict__ x, Batch bt)
{
    if (skip_rhs(bt)) return;
    r += (size_t)blockIdx.y * n;
    x += (size_t)blockIdx.y * n;
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    cx<R> s0 = zc<R>(), s1 = zc<R>(), s2 = zc<R>(), s3 = zc<R>();
    const cx<R> *m = Minv + (size_t)row * n;
    int c = lane;
    for (; c + 192 < n; c += 256) {
        s0 = cadd(s0, cmul(m[c], r[c]));
        s1 = cadd(s1, cmul(m[c + 64], r[c + 64]));
        s2 = cadd(s2, cmul(m[c + 128], r[c + 128]));
        s3 = cadd(s3, cmul(m[c + 192], r[c + 192]));
    }
    for (; c < n; c += 64) s0 = cadd(s0, cmul(m[c], r[c]));
    cx<R> s = wave_sum64<R>(cadd(cadd(s0, s1), cadd(s2, s3)));
    if (lane == 0) x[row] = s;
}

hipError_t launch_coarsest(int n, const cd *Minv, const cd *r, cd *x, hipStream_t st, Batch bt)
{
    k_coarsest<double><<<dim3(cdiv(n, 4), bt.B), 256, 0, st>>>(n, Minv, r, x, bt);
    HD_LAUNCH_CHECK();
}

hipError_t launch_coarsest(int n, const cf *Minv, const cf *r, cf *x, hipStream_t st, Batch bt)
{
    k_coarsest<float><<<dim3(cdiv(n, 4), bt.B), 256, 0, st>>>(n, Minv, r, x, bt);
    HD_LAUNCH_CHECK();
}

// ------------------------------------------------------------------------
// Deflation restriction vc = Z^T vf (or b - Z^T vf): [1 4 6 4 1]/8 (Bezier)
// or 1/2 [1 2 1] (linear) per axis, centred on fine node (2I, 2J); the x pass
// first, then the y pass.
// (ZT_CX x ZT_CY is the coarse tile of the one-launch Galerkin operator
// below, which computes a 67 x 19 fine region per block.)
// ------------------------------------------------------------------------
constexpr int ZT_CX = 32, ZT_CY = 8;
constexpr int ZT_W = 2 * ZT_CX + 3, ZT_H = 2 * ZT_CY + 3;

// Streaming form: lane l of a wave holds fine column i = c0 + l (c0 even) of
// 19 consecutive fine rows, loaded A5_AHEAD rows ahead; each row is filtered
// along x with the neighbours at distance 1 and 2 from adjacent lanes (DPP
// shifts), a rolling window of 5 filtered rows gives the y filter, and the
// lanes on even fine columns 2..61 write coarse columns I = i / 2 (30 per
// wave) of 8 coarse rows.  A block is 4 waves stacked over 32 coarse rows.
constexpr int ZS_CX = 30, ZS_RPW = 8;

template <bool RESID>
__global__ __launch_bounds__(256) void k_zt(Lev Lf, Lev Lc, int zho, const cd *__restrict__ vf,
                                            const cd *__restrict__ b, cd *__restrict__ vc,
                                            int tiles_x, Batch bt)
{
    if (skip_rhs(bt)) return;
    {
        const size_t nf = (size_t)Lf.nx * Lf.ny, nc = (size_t)Lc.nx * Lc.ny;
        vf += blockIdx.y * nf;
        if (RESID) b += blockIdx.y * nc;
        vc += blockIdx.y * nc;
    }
    const int lane = threadIdx.x & 63;
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int i = (t % tiles_x) * (2 * ZS_CX) - 2 + lane;
    const int J0 = (t / tiles_x) * (4 * ZS_RPW) + (threadIdx.x >> 6) * ZS_RPW;
    const int nx = Lf.nx, ny = Lf.ny;
    if (J0 >= Lc.ny) return;  // the whole wave: no coarse row here
    const bool colin = i >= 0 && i < nx;
    const int ic = i < 0 ? 0 : (i >= nx ? nx - 1 : i);
    const int I = i >> 1;
    const bool outc = lane >= 2 && lane <= 2 * ZS_CX + 1 && !(i & 1) && I < Lc.nx;
    constexpr int NR = 2 * ZS_RPW + 3;  // fine rows 2 J0 - 2 .. 2 J0 + 2 ZS_RPW
    cd vb[NR];
    auto load_row = [&](int q) {
        const int jj = 2 * J0 - 2 + q;
        vb[q] = vf[(size_t)(jj < 0 ? 0 : (jj >= ny ? ny - 1 : jj)) * nx + ic];
    };
#pragma unroll
    for (int q = 0; q < A5_AHEAD && q < NR; q++) load_row(q);
    __builtin_amdgcn_sched_barrier(0);
    const double w0 = zho ? 0.75 : 1.0, w1 = 0.5, w2 = zho ? 0.125 : 0.0;
    cd X[5];
#pragma unroll
    for (int q = 0; q < NR; q++) {
        if (q + A5_AHEAD < NR) load_row(q + A5_AHEAD);
        const int jj = 2 * J0 - 2 + q;
        const double m = colin && jj >= 0 && jj < ny && unknown(Lf, ic, jj) ? 1.0 : 0.0;
        const cd c = cscal(m, vb[q]);
        const cd l1 = lane_from(c, true), r1 = lane_from(c, false);
        const cd l2 = lane_from(l1, true), r2 = lane_from(r1, false);
        cd xv = cscal(w0, c);
        caxpy(xv, w1, cadd(l1, r1));
        if (zho) caxpy(xv, w2, cadd(l2, r2));
#pragma unroll
        for (int d = 0; d < 4; d++) X[d] = X[d + 1];
        X[4] = xv;
        if (q >= 4 && !(q & 1)) {
            const int J = J0 + (q - 4) / 2;
            if (outc && J < Lc.ny) {
                cd v = czero();
                if (unknown(Lc, I, J)) {
                    v = cscal(w0, X[2]);
                    caxpy(v, w1, cadd(X[1], X[3]));
                    if (zho) caxpy(v, w2, cadd(X[0], X[4]));
                    if (RESID) v = csub(b[(size_t)J * Lc.nx + I], v);
                }
                vc[(size_t)J * Lc.nx + I] = v;
            }
        }
    }
}

hipError_t launch_zt(const Lev &Lf, const Lev &Lc, int zho, const cd *vf, const cd *b, cd *vc,
                     hipStream_t st, Batch bt)
{
    const int tx = cdiv(Lc.nx, ZS_CX), ty = cdiv(Lc.ny, 4 * ZS_RPW);
    const dim3 g(tx * ty, bt.B);
    if (b)
        k_zt<true><<<g, 256, 0, st>>>(Lf, Lc, zho, vf, b, vc, tx, bt);
    else
        k_zt<false><<<g, 256, 0, st>>>(Lf, Lc, zho, vf, b, vc, tx, bt);
    HD_LAUNCH_CHECK();
}

// ------------------------------------------------------------------------
// Deflation prolongation vf = Z vc (thread per fine node, 64 x 4 blocks).
// ------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_z(Lev Lf, Lev Lc, int zho, const cd *__restrict__ vc,
                                           cd *__restrict__ vf, int tiles_x, Batch bt)
{
    if (skip_rhs(bt)) return;
    vc += (size_t)blockIdx.y * Lc.nx * Lc.ny;
    vf += (size_t)blockIdx.y * Lf.nx * Lf.ny;
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int i = (t % tiles_x) * 64 + (threadIdx.x & 63);
    const int j = (t / tiles_x) * 4 + (threadIdx.x >> 6);
    if (i >= Lf.nx || j >= Lf.ny) return;
    cd v = czero();
    if (unknown(Lf, i, j)) v = prolong_at(Lc, vc, i, j, zho);
    vf[(size_t)j * Lf.nx + i] = v;
}

hipError_t launch_z(const Lev &Lf, const Lev &Lc, int zho, const cd *vc, cd *vf, hipStream_t st,
                    Batch bt)
{
    const int tx = cdiv(Lf.nx, 64), ty = cdiv(Lf.ny, 4);
    k_z<<<dim3(tx * ty, bt.B), 256, 0, st>>>(Lf, Lc, zho, vc, vf, tx, bt);
    HD_LAUNCH_CHECK();
}

// ------------------------------------------------------------------------
// Galerkin coarse operator y = Z^T A_h Z x (or y = b - Z^T A_h Z x) in one
// launch (Section 5.2.1): a block owns a ZT_CX x ZT_CY coarse tile and
// computes, in LDS, x on the coarse nodes around it, Z x on the fine nodes
// the tile's Z^T needs plus one more ring, A_h (Z x) on the former, and Z^T
// of that, so the fine-grid vectors Z x and A_h Z x never reach memory.  Each
// step is the arithmetic, in its order, of k_z, k_apply5 and k_zt above.
// ------------------------------------------------------------------------
constexpr int GK_CW = ZT_CX + 4, GK_CH = ZT_CY + 4;  // coarse x: I0-2 .. I0+CX+1
constexpr int GK_1W = 2 * ZT_CX + 5, GK_1H = 2 * ZT_CY + 5;  // Z x: fi0-1 .. fi0+2CX+3
constexpr int GK_2W = ZT_W, GK_2H = ZT_H;  // A_h Z x: fi0 .. fi0+2CX+2 (fi0 = 2 I0 - 2)

// (Z x) at fine node (i,j) from the LDS coarse tile sc (origin I0-2, J0-2):
// prolong_at with the coarse values read from the tile.
__device__ __forceinline__ cd prolong_lds(const Lev &Lc, const cd (*sc)[GK_CW], int ci0, int cj0,
                                          int i, int j, int zho)
{
    int Ix[3], Jy[3];
    double wx[3], wy[3];
    const int nxw = zrule(i, zho, Ix, wx), nyw = zrule(j, zho, Jy, wy);
    cd s = czero();
    for (int b = 0; b < nyw; b++) {
        const int J = Jy[b];
        if (J < 0 || J >= Lc.ny) continue;
        for (int a = 0; a < nxw; a++) {
            const int I = Ix[a];
            if (I < 0 || I >= Lc.nx || !unknown(Lc, I, J)) continue;
            caxpy(s, wx[a] * wy[b], sc[J - cj0][I - ci0]);
        }
    }
    return s;
}

template <bool RESID, bool VARK>
__global__ __launch_bounds__(256) void k_glk(Lev Lf, Lev Lc, int zho, const cd *__restrict__ x,
                                             const cd *__restrict__ b, cd *__restrict__ y,
                                             int tiles_x, Batch bt)
{
    if (skip_rhs(bt)) return;
    {
        const size_t nc = (size_t)Lc.nx * Lc.ny;
        x += blockIdx.y * nc;
        if (RESID) b += blockIdx.y * nc;
        y += blockIdx.y * nc;
    }
    __shared__ cd sc[GK_CH][GK_CW];
    __shared__ cd s1[GK_1H * GK_1W];  // Z x, later the horizontal Z^T sums
    __shared__ cd s2[GK_2H][GK_2W];
    __shared__ double sk[VARK ? GK_2H : 1][VARK ? GK_2W : 1];
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int I0 = (t % tiles_x) * ZT_CX, J0 = (t / tiles_x) * ZT_CY;
    const int ci0 = I0 - 2, cj0 = J0 - 2, fi0 = 2 * I0 - 2, fj0 = 2 * J0 - 2;
    // ---- loads: coarse x (0 outside the grid or at non-unknowns; those
    // nodes are skipped by prolong_lds anyway), k on the A_h nodes
    constexpr int NC = GK_CW * GK_CH, NK = GK_2W * GK_2H;
    cd xv[(NC + 255) / 256];
    double mx[(NC + 255) / 256], kv[VARK ? (NK + 255) / 256 : 1];
#pragma unroll
    for (int kq = 0; kq < (NC + 255) / 256; kq++) {
        const int q = threadIdx.x + 256 * kq;
        const int I = ci0 + q % GK_CW, J = cj0 + q / GK_CW;
        const bool in = q < NC && I >= 0 && I < Lc.nx && J >= 0 && J < Lc.ny && unknown(Lc, I, J);
        xv[kq] = x[in ? (size_t)J * Lc.nx + I : 0];
        mx[kq] = in ? 1.0 : 0.0;
    }
    if (VARK) {
#pragma unroll
        for (int kq = 0; kq < (NK + 255) / 256; kq++) {
            const int q = threadIdx.x + 256 * kq;
            const int i = fi0 + q % GK_2W, j = fj0 + q / GK_2W;
            const bool in = q < NK && i >= 0 && i < Lf.nx && j >= 0 && j < Lf.ny;
            kv[kq] = Lf.k[in ? (size_t)j * Lf.nx + i : 0];
        }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int kq = 0; kq < (NC + 255) / 256; kq++) {
        const int q = threadIdx.x + 256 * kq;
        if (q < NC) sc[q / GK_CW][q % GK_CW] = cscal(mx[kq], xv[kq]);
    }
    if (VARK) {
#pragma unroll
        for (int kq = 0; kq < (NK + 255) / 256; kq++) {
            const int q = threadIdx.x + 256 * kq;
            if (q < NK) sk[q / GK_2W][q % GK_2W] = kv[kq];
        }
    }
    __syncthreads();
    // ---- Z x on fine nodes fi0-1 .. fi0+2CX+3 (k_z: 0 at non-unknowns),
    // separably: along x into s2 (GK_CH coarse rows x GK_1W fine columns;
    // coarse nodes outside the grid or not unknowns hold 0 in sc), then along
    // y into s1
    cd *sh = &s2[0][0];  // GK_CH * GK_1W <= GK_2H * GK_2W entries
    const double zw0 = zho ? 0.75 : 1.0, zw1 = zho ? 0.125 : 0.0;
    for (int q = threadIdx.x; q < GK_CH * GK_1W; q += 256) {
        const int r = q / GK_1W, a1 = q % GK_1W;
        const int i = fi0 - 1 + a1, ci = (i >> 1) - ci0;  // coarse I = floor(i / 2)
        cd v;
        if (i & 1) {
            v = cscal(0.5, cadd(sc[r][ci], sc[r][ci + 1]));
        } else {
            v = cscal(zw0, sc[r][ci]);
            if (zho) caxpy(v, zw1, cadd(sc[r][ci - 1], sc[r][ci + 1]));
        }
        sh[q] = v;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < GK_1W * GK_1H; q += 256) {
        const int a1 = q % GK_1W, b1 = q / GK_1W;
        const int i = fi0 - 1 + a1, j = fj0 - 1 + b1, cj = (j >> 1) - cj0;
        cd v = czero();
        if (i >= 0 && i < Lf.nx && j >= 0 && j < Lf.ny && unknown(Lf, i, j)) {
            if (j & 1) {
                v = cscal(0.5, cadd(sh[cj * GK_1W + a1], sh[(cj + 1) * GK_1W + a1]));
            } else {
                v = cscal(zw0, sh[cj * GK_1W + a1]);
                if (zho) caxpy(v, zw1, cadd(sh[(cj - 1) * GK_1W + a1], sh[(cj + 1) * GK_1W + a1]));
            }
        }
        s1[q] = v;
    }
    __syncthreads();
    // ---- A_h (Z x) on fine nodes fi0 .. fi0+2CX+2 (k_apply5; 0 outside the
    // grid and at non-unknowns, as k_zt reads it).  Away from the grid edge
    // the stencil is the interior one (Z x is 0 at Dirichlet boundary nodes,
    // so their dropped couplings add nothing).
    const bool som = Lf.bc == BC_SOM;
    for (int q = threadIdx.x; q < GK_2W * GK_2H; q += 256) {
        const int a = q % GK_2W, bb = q / GK_2W;
        const int i = fi0 + a, j = fj0 + bb;
        const int c = (bb + 1) * GK_1W + a + 1;  // (i,j) in s1
        cd v = czero();
        const bool inner = i > 0 && j > 0 && i < Lf.nx - 1 && j < Lf.ny - 1;
        if (inner) {
            const double k = VARK ? sk[bb][a] : Lf.kc;
            const cd ap = make_double2(2.0 * Lf.ihx2 + 2.0 * Lf.ihy2 - k * k, -0.0 * (k * k));
            v = cmul(ap, s1[c]);
            caxpy(v, -Lf.ihx2, s1[c - 1]);
            caxpy(v, -Lf.ihx2, s1[c + 1]);
            caxpy(v, -Lf.ihy2, s1[c - GK_1W]);
            caxpy(v, -Lf.ihy2, s1[c + GK_1W]);
        } else if (som && i >= 0 && i < Lf.nx && j >= 0 && j < Lf.ny) {
            cd ap;
            double aw, ae, as, an;
            coef5k(Lf, make_double2(1.0, 0.0), i, j, VARK ? sk[bb][a] : Lf.kc, ap, aw, ae, as, an);
            v = cmul(ap, s1[c]);
            if (aw != 0.0) caxpy(v, aw, s1[c - 1]);
            if (ae != 0.0) caxpy(v, ae, s1[c + 1]);
            if (as != 0.0) caxpy(v, as, s1[c - GK_1W]);
            if (an != 0.0) caxpy(v, an, s1[c + GK_1W]);
        }
        s2[bb][a] = v;
    }
    __syncthreads();
    // ---- Z^T (k_zt): rows first, into s1 as sx[GK_2H][ZT_CX]
    const double w0 = zho ? 0.75 : 1.0, w1 = 0.5, w2 = zho ? 0.125 : 0.0;
    for (int q = threadIdx.x; q < ZT_CX * GK_2H; q += 256) {
        const int c = q % ZT_CX, bb = q / ZT_CX;
        const int a = 2 * c + 2;
        cd v = cscal(w0, s2[bb][a]);
        caxpy(v, w1, cadd(s2[bb][a - 1], s2[bb][a + 1]));
        if (zho) caxpy(v, w2, cadd(s2[bb][a - 2], s2[bb][a + 2]));
        s1[bb * ZT_CX + c] = v;
    }
    __syncthreads();
    const int c = threadIdx.x % ZT_CX, rl = threadIdx.x / ZT_CX;
    const int I = I0 + c, J = J0 + rl;
    if (I >= Lc.nx || J >= Lc.ny) return;
    cd v = czero();
    if (unknown(Lc, I, J)) {
        const int bb = 2 * rl + 2;
        v = cscal(w0, s1[bb * ZT_CX + c]);
        caxpy(v, w1, cadd(s1[(bb - 1) * ZT_CX + c], s1[(bb + 1) * ZT_CX + c]));
        if (zho) caxpy(v, w2, cadd(s1[(bb - 2) * ZT_CX + c], s1[(bb + 2) * ZT_CX + c]));
        if (RESID) v = csub(b[(size_t)J * Lc.nx + I], v);
    }
    y[(size_t)J * Lc.nx + I] = v;
}

hipError_t launch_glk(const Lev &Lf, const Lev &Lc, int zho, const cd *x, const cd *b, cd *y,
                      hipStream_t st, Batch bt)
{
    const int tx = cdiv(Lc.nx, ZT_CX), ty = cdiv(Lc.ny, ZT_CY);
    const dim3 g(tx * ty, bt.B);
    if (Lf.k) {
        if (b)
            k_glk<true, true><<<g, 256, 0, st>>>(Lf, Lc, zho, x, b, y, tx, bt);
        else
            k_glk<false, true><<<g, 256, 0, st>>>(Lf, Lc, zho, x, b, y, tx, bt);
    } else {
        if (b)
            k_glk<true, false><<<g, 256, 0, st>>>(Lf, Lc, zho, x, b, y, tx, bt);
        else
            k_glk<false, false><<<g, 256, 0, st>>>(Lf, Lc, zho, x, b, y, tx, bt);
    }
    HD_LAUNCH_CHECK();
}

// ------------------------------------------------------------------------
// Deflated residual t = v - A_h (Z v2); Z v2 is formed in registers and never
// written to memory.
// A wave streams 64 consecutive fine columns i = c0 + lane (c0 even) and
// writes the 58 of lanes 2..59 on DR_RPW rows.  Lane l loads v2 at coarse
// column i >> 1 of every coarse row the strip needs; the Z rule's x part then
// takes its coarse neighbours from the adjacent lanes (DPP shifts: an even
// column i = 2I needs I - 1 from lane l - 1 and I + 1 from lane l + 2, an odd
// one (i + 1) / 2 from lane l + 1), its y part combines the x-filtered coarse
// rows, and the 5-point operator takes the west/east values of Z v2 from the
// adjacent lanes and north/south from the rows before and after.  Coarse
// values outside the grid or not unknowns count as 0, and so does Z v2 at a
// fine node that is not an unknown.  A block is 4 waves stacked over
// 4 * DR_RPW rows; every load is issued before the arithmetic.
// ------------------------------------------------------------------------
constexpr int DR_TX = 58, DR_RPW = 16, DR_NC = DR_RPW / 2 + 3;

template <bool VARK>
__global__ __launch_bounds__(256) void k_dresid(Lev Lf, Lev Lc, int zho,
                                                const cd *__restrict__ v,
                                                const cd *__restrict__ v2, cd *__restrict__ tout,
                                                int tiles_x, Batch bt)
{
    if (skip_rhs(bt)) return;
    {
        const size_t nf = (size_t)Lf.nx * Lf.ny, nc = (size_t)Lc.nx * Lc.ny;
        v += blockIdx.y * nf;
        tout += blockIdx.y * nf;
        v2 += blockIdx.y * nc;
    }
    const int lane = threadIdx.x & 63;
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int i = (t % tiles_x) * DR_TX - 2 + lane;
    const int j0 = (t / tiles_x) * (4 * DR_RPW) + (threadIdx.x >> 6) * DR_RPW;  // even
    const int nx = Lf.nx, ny = Lf.ny;
    if (j0 >= ny) return;  // the whole wave: no row here
    const bool colin = i >= 0 && i < nx;
    const int ic = i < 0 ? 0 : (i >= nx ? nx - 1 : i);
    const bool outc = lane >= 2 && lane <= DR_TX + 1 && colin;
    // coarse rows Jb .. Jb + DR_NC - 1 cover fine rows j0 - 1 .. j0 + DR_RPW
    const int Jb = j0 / 2 - 1;
    const int Iv = i >= 0 ? i >> 1 : -1;
    const bool cin = Iv >= 0 && Iv < Lc.nx;
    const int Ivc = Iv < 0 ? 0 : (Iv >= Lc.nx ? Lc.nx - 1 : Iv);
    cd cr[DR_NC], vr[DR_RPW];
    double kr[VARK ? DR_RPW : 1];
#pragma unroll
    for (int q = 0; q < DR_NC; q++) {
        const int J = Jb + q;
        cr[q] = v2[(size_t)(J < 0 ? 0 : (J >= Lc.ny ? Lc.ny - 1 : J)) * Lc.nx + Ivc];
    }
#pragma unroll
    for (int r = 0; r < DR_RPW; r++) {
        const int j = j0 + r;
        const size_t p = (size_t)(j < ny ? j : ny - 1) * nx + ic;
        vr[r] = v[p];
        if (VARK) kr[r] = Lf.k[p];
    }
    __builtin_amdgcn_sched_barrier(0);
    // x part of the Z rule on every coarse row (in place)
    const double w0 = zho ? 0.75 : 1.0, w2 = zho ? 0.125 : 0.0;
#pragma unroll
    for (int q = 0; q < DR_NC; q++) {
        const int J = Jb + q;
        const double m = cin && J >= 0 && J < Lc.ny && unknown(Lc, Ivc, J) ? 1.0 : 0.0;
        const cd c = cscal(m, cr[q]);
        const cd cw = lane_from(c, true), ce = lane_from(c, false);
        const cd ce2 = lane_from(ce, false);
        // even i: w0 v(I) + w2 (v(I-1) + v(I+1)); odd i: (v(I) + v(I+1)) / 2
        cd xe = cscal(w0, c);
        caxpy(xe, w2, cadd(cw, ce2));
        cr[q] = (i & 1) ? cscal(0.5, cadd(c, ce)) : xe;
    }
    // Z v2 on fine row j0 + rr, -1 <= rr <= DR_RPW (rr is a compile-time
    // constant in the unrolled loop; j0 is even): coarse row j0 / 2 + rr / 2
    // is cr[rr / 2 + 1] for even rr, and an odd rr lies between cr[(rr+1)/2]
    // and the next one
    auto zrow = [&](int rr) -> cd {
        cd z;
        if (rr & 1) {
            const int q = (rr + 1) / 2;
            z = cscal(0.5, cadd(cr[q], cr[q + 1]));
        } else {
            const int q = rr / 2 + 1;
            z = cscal(w0, cr[q]);
            caxpy(z, w2, cadd(cr[q - 1], cr[q + 1]));
        }
        const int j = j0 + rr;
        const double m = colin && j >= 0 && j < ny && unknown(Lf, ic, j) ? 1.0 : 0.0;
        return cscal(m, z);
    };
    const cd one = make_double2(1.0, 0.0);
    cd zs = zrow(-1);
    cd zc = zrow(0);
#pragma unroll
    for (int r = 0; r < DR_RPW; r++) {
        const int j = j0 + r;
        const cd zn = zrow(r + 1);
        const cd zw = lane_from(zc, true), ze = lane_from(zc, false);
        if (outc && j < ny) {
            cd ap;
            double aw, ae, as, an;
            cd o = czero();
            const double kv = VARK ? kr[r] : Lf.kc;
            if (coef5k(Lf, one, i, j, kv, ap, aw, ae, as, an)) {
                cd m = cmul(ap, zc);
                caxpy(m, aw, zw);
                caxpy(m, ae, ze);
                caxpy(m, as, zs);
                caxpy(m, an, zn);
                o = csub(vr[r], m);
            }
            tout[(size_t)j * nx + i] = o;
        }
        zs = zc;
        zc = zn;
    }
}

hipError_t launch_dresid(const Lev &Lf, const Lev &Lc, int zho, const cd *v, const cd *v2,
                         cd *t, hipStream_t st, Batch bt)
{
    const int tx = cdiv(Lf.nx, DR_TX), ty = cdiv(Lf.ny, 4 * DR_RPW);
    const dim3 g(tx * ty, bt.B);
    if (Lf.k)
        k_dresid<true><<<g, 256, 0, st>>>(Lf, Lc, zho, v, v2, t, tx, bt);
    else
        k_dresid<false><<<g, 256, 0, st>>>(Lf, Lc, zho, v, v2, t, tx, bt);
    HD_LAUNCH_CHECK();
}

// ------------------------------------------------------------------------
// ReD-Glk2 coarse operator (Section 5.2.4).
// Interior nodes (2 <= I <= nx-3, 2 <= J <= ny-3) take the Galerkin 5x5
// stencils, written as tensor products of 1D factors:
//   Laplacian  = (1/H^2) [LX (x) WY + WX (x) LY],
//                LX = LY = [-6 -8 28 -8 -6]/16,  WX = WY = [1 28 70 28 1]/64,
//   (1D Galerkin products of the Bezier vectors with [-1 2 -1]/h^2 and with
//   the identity, H = 2h);
//   k^2 part   = WX (x) WY applied to (k^2 u), k taken at each stencil node;
// these reproduce the printed stencils (1/256)[...]/(2h)^2 and k^2/64^2 [...].
// Each thread streams one column over RG_RPW rows, keeping the x-filtered rows
// in registers.  Boundary rows are done by redglk2_band in the same launch.
// ------------------------------------------------------------------------
__constant__ double c_L1[5] = {-6.0 / 16, -8.0 / 16, 28.0 / 16, -8.0 / 16, -6.0 / 16};
__constant__ double c_W1[5] = {1.0 / 64, 28.0 / 64, 70.0 / 64, 28.0 / 64, 1.0 / 64};

// Interior tiling: a wave loads 64 consecutive columns and writes the 60 in
// the middle (lanes 2..61); the west/east neighbours at distance 1 and 2 come
// from the adjacent lanes by wave-wide DPP shifts, so each node is loaded once
// per row it touches.  A block is 4 waves stacked over 4 x RG_RPW output rows.
// Rows are loaded unconditionally from a clamped (valid) address and RG_AHEAD
// rows ahead of their use, so a wave keeps several rows in flight instead of
// waiting on each; values outside the grid or at Dirichlet nodes are then
// replaced by zero.
constexpr int RG_TX = 60, RG_RPW = 8, RG_AHEAD = 12;

template <bool RESID, bool VARK>
__device__ __forceinline__ void redglk2_interior(const Lev &L, const cd *__restrict__ u,
                                                 const cd *__restrict__ b, cd *__restrict__ y,
                                                 int tiles_x, int nb_int, int blk)
{
    const int lane = threadIdx.x & 63;
    const int t = xcd_tile(blk, nb_int);
    const int I = (t % tiles_x) * RG_TX + lane;
    const int J0 = (t / tiles_x) * (4 * RG_RPW) + (threadIdx.x >> 6) * RG_RPW;
    if (J0 > L.ny - 3) return;  // the whole wave: no output row here
    const int nx = L.nx, ny = L.ny;
    const bool dir = L.bc == BC_DIR;
    const bool colok = I < nx && !(dir && (I == 0 || I == nx - 1));
    const int Ic = I < nx ? I : nx - 1;
    const bool outc = lane >= 2 && lane <= 61 && I >= 2 && I <= nx - 3;
    const double iH2 = L.ihx2;  // hx == hy on this path
    const double kc2 = L.kc * L.kc;
    constexpr int NR = RG_RPW + 4;
    cd ub[NR], bb[RG_RPW];
    double kb[NR];
    auto load_row = [&](int q) {
        const int jj = J0 - 2 + q;
        const int jc = jj < 0 ? 0 : (jj >= ny ? ny - 1 : jj);
        ub[q] = u[(size_t)jc * nx + Ic];
        if (VARK) kb[q] = L.k[(size_t)jc * nx + Ic];
        if (RESID && q >= 4) {
            const int J = jj - 2;
            bb[q - 4] = b[(size_t)(J < ny ? J : ny - 1) * nx + Ic];
        }
    };
#pragma unroll
    for (int q = 0; q < RG_AHEAD && q < NR; q++) load_row(q);
    // keep the loads above ahead of the arithmetic below
    __builtin_amdgcn_sched_barrier(0);
    // rolling window of x-filtered rows: P = (LX/H^2 - k^2 WX) u  (constant k)
    //                                    or LX/H^2 u  (variable k, with R = WX (k^2 u)),
    //                                    Q = WX u / H^2
    cd P[5], Q[5], R[5];
#pragma unroll
    for (int q = 0; q < NR; q++) {
        if (q + RG_AHEAD < NR) load_row(q + RG_AHEAD);
        const int jj = J0 - 2 + q;
        // Dirichlet boundary rows/columns are not unknowns: read as zero
        const bool ok = colok && jj >= 0 && jj < ny && (!dir || (jj > 0 && jj < ny - 1));
        // zeroing by a 0/1 factor rather than a select, so that the compiler
        // keeps the load unconditional (a select lets it sink the load into a
        // branch whose wait drains every row already in flight)
        const double m = ok ? 1.0 : 0.0;
        cd uv[5];
        uv[2] = make_double2(ub[q].x * m, ub[q].y * m);
        uv[1] = lane_from(uv[2], true);
        uv[0] = lane_from(uv[1], true);
        uv[3] = lane_from(uv[2], false);
        uv[4] = lane_from(uv[3], false);
        double kv[5];
        if (VARK) {
            kv[2] = kb[q];
            kv[1] = lane_from(kv[2], true);
            kv[0] = lane_from(kv[1], true);
            kv[3] = lane_from(kv[2], false);
            kv[4] = lane_from(kv[3], false);
        }
        cd pv = czero(), qv = czero(), rv = czero();
#pragma unroll
        for (int d = 0; d < 5; d++) {
            if (VARK) {
                caxpy(pv, c_L1[d] * iH2, uv[d]);
                caxpy(rv, c_W1[d] * kv[d] * kv[d], uv[d]);
            } else {
                caxpy(pv, c_L1[d] * iH2 - kc2 * c_W1[d], uv[d]);
            }
            caxpy(qv, c_W1[d] * iH2, uv[d]);
        }
#pragma unroll
        for (int d = 0; d < 4; d++) {
            P[d] = P[d + 1];
            Q[d] = Q[d + 1];
            if (VARK) R[d] = R[d + 1];
        }
        P[4] = pv;
        Q[4] = qv;
        if (VARK) R[4] = rv;
        if (q >= 4) {
            const int J = jj - 2;
            if (outc && J >= 2 && J <= ny - 3) {
                cd o = czero();
#pragma unroll
                for (int d = 0; d < 5; d++) {
                    caxpy(o, c_W1[d], P[d]);
                    caxpy(o, c_L1[d], Q[d]);
                    if (VARK) caxpy(o, -c_W1[d], R[d]);
                }
                const size_t p = (size_t)J * nx + I;
                if (RESID) o = csub(bb[q - 4], o);
                y[p] = o;
            }
        }
    }
}

// The 5x5 printed-stencil weight at offset (dI, dJ): Laplacian / H^2 part and
// the k^2 part.
__device__ __forceinline__ double glk_lap(int dI, int dJ, double iH2)
{
    return (c_L1[dI + 2] * c_W1[dJ + 2] + c_W1[dI + 2] * c_L1[dJ + 2]) * iH2;
}
__device__ __forceinline__ double glk_k2w(int dI, int dJ) { return c_W1[dI + 2] * c_W1[dJ + 2]; }

// value of grid node (I,J), 0 for non-unknowns
__device__ __forceinline__ cd uat(const Lev &L, const cd *u, int I, int J)
{
    return unknown(L, I, J) ? u[(size_t)J * L.nx + I] : czero();
}

// Ghost value beyond the x-boundary in row J (Ig = -1 or nx): Sommerfeld
// u_g = u_inward + 2 i H k_bnd u_bnd; Dirichlet u_g = 2 u_bnd - u_inward.
__device__ __forceinline__ cd ghost_x(const Lev &L, const cd *u, int Ig, int J)
{
    const int Ib = Ig < 0 ? 0 : L.nx - 1, Ii = Ig < 0 ? 1 : L.nx - 2;
    const cd ub = uat(L, u, Ib, J), ui = uat(L, u, Ii, J);
    if (L.bc == BC_SOM) {
        const double c = 2.0 * L.hx * kat(L, Ib, J);
        return make_double2(ui.x - c * ub.y, ui.y + c * ub.x);
    }
    return make_double2(2.0 * ub.x - ui.x, 2.0 * ub.y - ui.y);
}
__device__ __forceinline__ cd ghost_y(const Lev &L, const cd *u, int I, int Jg)
{
    const int Jb = Jg < 0 ? 0 : L.ny - 1, Ji = Jg < 0 ? 1 : L.ny - 2;
    const cd ub = uat(L, u, I, Jb), ui = uat(L, u, I, Ji);
    if (L.bc == BC_SOM) {
        const double c = 2.0 * L.hy * kat(L, I, Jb);
        return make_double2(ui.x - c * ub.y, ui.y + c * ub.x);
    }
    return make_double2(2.0 * ub.x - ui.x, 2.0 * ub.y - ui.y);
}

// Boundary band of ReD-Glk2: first layer (boundary nodes) = the 5-point
// second-order operator at spacing H with the Sommerfeld closure; second layer
// = the 5x5 stencil with ghost nodes eliminated (k = 0 at ghosts; a ghost
// outside in both directions is the mean of its two single-direction
// neighbours).  Dirichlet boundary nodes are not unknowns.
// ReD-Glk1 (GLK1): both layers are the second-order 5-point rows.
// Band layout: nR boundary-band rows (0, 1, ny-2, ny-1 without repeats; all
// rows when ny < 5) cover every column; then nC band columns cover the rows
// 2..ny-3 in between.  Band row k is k for k < 2, else ny - nR + k (columns
// alike).  blk numbers the band's own blocks.
template <bool RESID, bool GLK1>
__device__ __forceinline__ void redglk2_band(const Lev &L, const cd *__restrict__ u,
                                             const cd *__restrict__ b, cd *__restrict__ y,
                                             int nR, int nC, int count, int blk)
{
    const int idx = blk * 256 + threadIdx.x;
    if (idx >= count) return;
    int I, J;
    if (idx < nR * L.nx) {
        const int k = idx / L.nx;
        J = k < 2 ? k : L.ny - nR + k;
        I = idx - k * L.nx;
    } else {
        const int q = idx - nR * L.nx;
        const int c = q % nC;
        I = c < 2 ? c : L.nx - nC + c;
        J = 2 + q / nC;
    }
    const size_t p = (size_t)J * L.nx + I;
    cd o = czero();
    if (unknown(L, I, J)) {
        const bool bnd = GLK1 || I == 0 || J == 0 || I == L.nx - 1 || J == L.ny - 1;
        if (bnd) {
            cd ap;
            double aw, ae, as, an;
            coef5(L, make_double2(1.0, 0.0), I, J, ap, aw, ae, as, an);
            o = cmul(ap, u[p]);
            if (aw != 0.0) caxpy(o, aw, u[p - 1]);
            if (ae != 0.0) caxpy(o, ae, u[p + 1]);
            if (as != 0.0) caxpy(o, as, u[p - L.nx]);
            if (an != 0.0) caxpy(o, an, u[p + L.nx]);
        } else {
            const double iH2 = L.ihx2;
            for (int dJ = -2; dJ <= 2; dJ++)
                for (int dI = -2; dI <= 2; dI++) {
                    const int Ii = I + dI, Jj = J + dJ;
                    const double lw = glk_lap(dI, dJ, iH2);
                    const bool inx = Ii >= 0 && Ii < L.nx, iny = Jj >= 0 && Jj < L.ny;
                    if (inx && iny) {
                        const double kk = kat(L, Ii, Jj);
                        caxpy(o, lw - glk_k2w(dI, dJ) * kk * kk, uat(L, u, Ii, Jj));
                    } else if (!inx && iny) {
                        caxpy(o, lw, ghost_x(L, u, Ii, Jj));
                    } else if (inx && !iny) {
                        caxpy(o, lw, ghost_y(L, u, Ii, Jj));
                    } else {
                        const int In = Ii < 0 ? 0 : L.nx - 1, Jn = Jj < 0 ? 0 : L.ny - 1;
                        const cd g = cadd(ghost_y(L, u, In, Jj), ghost_x(L, u, Ii, Jn));
                        caxpy(o, 0.5 * lw, g);
                    }
                }
        }
        if (RESID) o = csub(b[p], o);
    }
    y[p] = o;
}

// One launch for the whole coarse operator: blocks [0, nb_band) do the
// boundary band, the blocks after them the interior tiles, so both run
// concurrently.  The band goes first: its nodes take long dependent chains of
// reads, which then overlap the interior instead of trailing it.  nb_band is a
// multiple of 8, so block ids keep their XCD in the interior's tile map.
template <bool RESID, bool VARK, bool GLK1>
__global__ __launch_bounds__(256) void k_redglk2(Lev L, const cd *__restrict__ u,
                                                 const cd *__restrict__ b, cd *__restrict__ y,
                                                 int tiles_x, int nb_int, int nb_band, int nR,
                                                 int nC, int count, Batch bt)
{
    if (skip_rhs(bt)) return;
    {
        const size_t off = (size_t)blockIdx.y * L.nx * L.ny;
        u += off;
        if (RESID) b += off;
        y += off;
    }
    if ((int)blockIdx.x < nb_band)
        redglk2_band<RESID, GLK1>(L, u, b, y, nR, nC, count, blockIdx.x);
    else
        redglk2_interior<RESID, VARK>(L, u, b, y, tiles_x, nb_int, blockIdx.x - nb_band);
}

template <bool GLK1>
static hipError_t redglk_t(const Lev &L, const cd *x, const cd *b, cd *y, hipStream_t st, Batch bt)
{
    int tx = 0, nb_int = 0;
    if (L.nx >= 5 && L.ny >= 5) {
        tx = cdiv(L.nx - 4, RG_TX);
        nb_int = tx * cdiv(L.ny, 4 * RG_RPW);
    }
    // band: rows {0,1,ny-2,ny-1} and columns {0,1,nx-2,nx-1} without repeats
    const int nR = L.ny < 4 ? L.ny : 4, nC = L.nx < 4 ? L.nx : 4;
    const int inner_rows = L.ny - nR;  // rows 2..ny-3 when ny >= 5, else 0
    const int count = nR * L.nx + nC * inner_rows;
    const int nb_band = cdiv(cdiv(count, 256), 8) * 8;
    const dim3 g(nb_band + nb_int, bt.B);
#define RG_LAUNCH(RES, VK)                                                                   \
    k_redglk2<RES, VK, GLK1><<<g, 256, 0, st>>>(L, x, b, y, tx, nb_int, nb_band, nR, nC, count, \
                                                bt)
    if (L.k) {
        if (b)
            RG_LAUNCH(true, true);
        else
            RG_LAUNCH(false, true);
    } else {
        if (b)
            RG_LAUNCH(true, false);
        else
            RG_LAUNCH(false, false);
    }
#undef RG_LAUNCH
    HD_LAUNCH_CHECK();
}

hipError_t launch_redglk2(const Lev &L, const cd *x, const cd *b, cd *y, int glk1, hipStream_t st,
                          Batch bt)
{
    return glk1 ? redglk_t<true>(L, x, b, y, st, bt) : redglk_t<false>(L, x, b, y, st, bt);
}

// ------------------------------------------------------------------------
// ReD-O4 coarse operator (Section 5.2.3): fourth-order central differences
// for the Laplacian, (u_{i-2} - 16 u_{i-1} + 30 u_i - 16 u_{i+1} + u_{i+2}) /
// (12 H^2) per axis, minus k^2 u, at nodes two or more nodes inside the
// grid; the other rows are the second-order 5-point rows with the boundary
// closure.  One thread per node; the 9 reads of a row come through L1/L2.
// ------------------------------------------------------------------------
template <bool RESID>
__global__ __launch_bounds__(256) void k_redo4(Lev L, const cd *__restrict__ u,
                                               const cd *__restrict__ b, cd *__restrict__ y,
                                               int tiles_x, Batch bt)
{
    if (skip_rhs(bt)) return;
    {
        const size_t off = (size_t)blockIdx.y * L.nx * L.ny;
        u += off;
        if (RESID) b += off;
        y += off;
    }
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int I = (t % tiles_x) * 64 + (threadIdx.x & 63);
    const int J = (t / tiles_x) * 4 + (threadIdx.x >> 6);
    if (I >= L.nx || J >= L.ny) return;
    const size_t p = (size_t)J * L.nx + I;
    cd o = czero();
    if (unknown(L, I, J)) {
        if (I < 2 || J < 2 || I > L.nx - 3 || J > L.ny - 3) {
            cd ap;
            double aw, ae, as, an;
            coef5(L, make_double2(1.0, 0.0), I, J, ap, aw, ae, as, an);
            o = cmul(ap, u[p]);
            if (aw != 0.0) caxpy(o, aw, u[p - 1]);
            if (ae != 0.0) caxpy(o, ae, u[p + 1]);
            if (as != 0.0) caxpy(o, as, u[p - L.nx]);
            if (an != 0.0) caxpy(o, an, u[p + L.nx]);
        } else {
            const double ax = L.ihx2 / 12.0, ay = L.ihy2 / 12.0;
            const double k = kat(L, I, J);
            const cd uc = u[p];
            // Dirichlet boundary nodes are not unknowns: they read as zero
            const cd lx = cadd(cadd(uat(L, u, I - 2, J), uat(L, u, I + 2, J)),
                               cadd(cscal(-16.0, cadd(uat(L, u, I - 1, J), uat(L, u, I + 1, J))),
                                    cscal(30.0, uc)));
            const cd ly = cadd(cadd(uat(L, u, I, J - 2), uat(L, u, I, J + 2)),
                               cadd(cscal(-16.0, cadd(uat(L, u, I, J - 1), uat(L, u, I, J + 1))),
                                    cscal(30.0, uc)));
            o = cadd(cadd(cscal(ax, lx), cscal(ay, ly)), cscal(-k * k, uc));
        }
        if (RESID) o = csub(b[p], o);
    }
    y[p] = o;
}

hipError_t launch_redo4(const Lev &L, const cd *x, const cd *b, cd *y, hipStream_t st, Batch bt)
{
    const int tx = cdiv(L.nx, 64), ty = cdiv(L.ny, 4);
    const dim3 g(tx * ty, bt.B);
    if (b)
        k_redo4<true><<<g, 256, 0, st>>>(L, x, b, y, tx, bt);
    else
        k_redo4<false><<<g, 256, 0, st>>>(L, x, b, y, tx, bt);
    HD_LAUNCH_CHECK();
}

// ------------------------------------------------------------------------
// Adjoint state.  D A_h is complex symmetric for the D that halves each
// Sommerfeld-eliminated direction (the ghost closure doubles the inward
// coupling), so A_h^H = D conj(A_h) D^{-1} and A_h^{-H} f = D conj(A_h^{-1}
// conj(D^{-1} f)): the adjoint solve is a forward solve between two
// element-wise maps.  mode 0: out = conj(in / D); mode 1: out = D conj(in).
// Dirichlet boundary nodes are not unknowns (D = 1 elsewhere): out = 0 there.
// ------------------------------------------------------------------------
__device__ __forceinline__ double dscale(const Lev &L, int i, int j)
{
    if (L.bc != BC_SOM) return 1.0;
    double d = 1.0;
    if (i == 0 || i == L.nx - 1) d *= 0.5;
    if (j == 0 || j == L.ny - 1) d *= 0.5;
    return d;
}

__global__ __launch_bounds__(256) void k_adj_map(Lev L, const cd *in, cd *out, int mode)
{
    const size_t n = (size_t)L.nx * L.ny;
    in += blockIdx.y * n;
    out += blockIdx.y * n;
    const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= n) return;
    const int i = (int)(q % L.nx), j = (int)(q / L.nx);
    cd o = czero();
    if (unknown(L, i, j)) {
        const double d = dscale(L, i, j);
        const cd v = in[q];
        const double c = mode == 0 ? 1.0 / d : d;
        o = make_double2(c * v.x, -c * v.y);
    }
    out[q] = o;
}

hipError_t launch_adj_map(const Lev &L, const cd *in, cd *out, int mode, int B, hipStream_t st)
{
    const size_t n = (size_t)L.nx * L.ny;
    k_adj_map<<<dim3((unsigned)((n + 255) / 256), B), 256, 0, st>>>(L, in, out, mode);
    HD_LAUNCH_CHECK();
}

// g[p] += sum over the B right-hand sides of -Re(conj(lambda_p) (dA/ds)_pp u_p)
// with s = (k/omega)^2: (dA/ds)_pp = -omega^2, plus -i omega^2 / k_p times
// (1/hx per eliminated x direction + 1/hy per y direction) on Sommerfeld
// boundary nodes (the derivative of -2ik/h through k = omega sqrt(s); dropped
// where k_p = 0).  One thread per node, looping over the right-hand sides.
__global__ __launch_bounds__(256) void k_grad_s(Lev L, double omega, const cd *__restrict__ u,
                                                const cd *__restrict__ lam, int B,
                                                double *__restrict__ g)
{
    const size_t n = (size_t)L.nx * L.ny;
    const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= n) return;
    const int i = (int)(q % L.nx), j = (int)(q / L.nx);
    if (!unknown(L, i, j)) return;
    double dr = -omega * omega, di = 0.0;
    if (L.bc == BC_SOM) {
        double w = 0.0;
        if (i == 0 || i == L.nx - 1) w += 1.0 / L.hx;
        if (j == 0 || j == L.ny - 1) w += 1.0 / L.hy;
        const double k = kat(L, i, j);
        if (w != 0.0 && k > 0.0) di = -omega * omega * w / k;
    }
    double acc = 0.0;
    for (int b = 0; b < B; b++) {
        const cd uv = u[(size_t)b * n + q], lv = lam[(size_t)b * n + q];
        // t = d * u; contribution -Re(conj(lambda) t)
        const double tr = dr * uv.x - di * uv.y, ti = dr * uv.y + di * uv.x;
        acc -= lv.x * tr + lv.y * ti;
    }
    g[q] += acc;
}

hipError_t launch_grad_s(const Lev &L, double omega, const cd *u, const cd *lam, int B, double *g,
                         hipStream_t st)
{
    const size_t n = (size_t)L.nx * L.ny;
    k_grad_s<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(L, omega, u, lam, B, g);
    HD_LAUNCH_CHECK();
}

// Receivers: res[b][r] = u_b[rec[r]] - d[b][r]; f_b[rec[r]] = res[b][r] (f must
// hold zeros; receiver nodes are distinct); J[b] = 1/2 sum_r |res[b][r]|^2.
// One block per right-hand side.
__global__ __launch_bounds__(256) void k_receivers(const int *__restrict__ rec, int nrec,
                                                   const cd *__restrict__ u,
                                                   const cd *__restrict__ d, size_t n,
                                                   cd *__restrict__ res, cd *__restrict__ f,
                                                   double *__restrict__ J)
{
    __shared__ double red[256];
    const size_t b = blockIdx.x;
    double acc = 0.0;
    for (int r = threadIdx.x; r < nrec; r += 256) {
        const size_t node = (size_t)rec[r];
        const cd v = csub(u[b * n + node], d[b * nrec + r]);
        res[b * nrec + r] = v;
        f[b * n + node] = v;
        acc = fma(v.x, v.x, fma(v.y, v.y, acc));
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) J[b] = 0.5 * red[0];
}

hipError_t launch_receivers(const int *rec, int nrec, const cd *u, const cd *d, size_t n, int B,
                            cd *res, cd *f, double *J, hipStream_t st)
{
    k_receivers<<<B, 256, 0, st>>>(rec, nrec, u, d, n, res, f, J);
    HD_LAUNCH_CHECK();
}

// ------------------------------------------------------------------------
// Krylov kernels.  Vectors of length n; a basis V holds m vectors at stride
// ld.  The grid is sized to the number of blocks the chip holds at once
// (times a whole number of rounds), and each block owns one contiguous chunk
// of the vector, so every block does the same work and no tail round is left.
// Each thread keeps up to KR_S entries of w (or of its update) in registers.
// ------------------------------------------------------------------------
constexpr int KR_S = 16;

// Krylov blocks of each kind resident on the device at once
static int g_resident[KB_NKINDS] = {0, 0, 0, 0};

template <class TV, class TW>
__global__ __launch_bounds__(256, 3) void k_mdot(const TV *__restrict__ V, size_t ld, int m,
                                              const TW *__restrict__ w, size_t n, size_t chunk,
                                              cd *__restrict__ part, int with_norm,
                                              const cd *__restrict__ cond, int jcond, size_t vbs,
                                              size_t wbs, Batch bt);
template <class TV, class TW, class TO>
__global__ __launch_bounds__(256) void k_mupdate(const TW *win, TO *wout,
                                                 const TV *__restrict__ V, size_t ld, int m,
                                                 const cd *__restrict__ c, size_t n, size_t chunk,
                                                 cd *__restrict__ partn,
                                                 const cd *__restrict__ cond, int jcond,
                                                 const cd *__restrict__ sig, size_t vbs,
                                                 size_t wbs, Batch bt);

static int resident_blocks(int kind)
{
    if (g_resident[kind] > 0) return g_resident[kind];
    int dev = 0, ncu = 0, bk = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        ncu = 256;
    (void)hipGetLastError();
    const void *k = kind == KB_DOT      ? (const void *)k_mdot<cd, cd>
                    : kind == KB_UPDATE ? (const void *)k_mupdate<cd, cd, cd>
                    : kind == KB_DOT32  ? (const void *)k_mdot<cf, cd>
                                        : (const void *)k_mupdate<cf, cd, cf>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&bk, k, 256, 0) != hipSuccess) bk = 4;
    (void)hipGetLastError();
    if (bk < 1) bk = 1;
    g_resident[kind] = ncu * bk;
    return g_resident[kind];
}

int krylov_blocks(size_t n, int B, int kind)
{
    // Whole rounds of resident blocks over the B vectors together, split
    // evenly between them; a block never takes more than 256 * KR_S entries
    // nor fewer than 256.  Vectors that fit in one round of the less occupied
    // kernel of the dot/update pair use that round for both (fewer, fuller
    // blocks: 3% faster on a 577 x 961 solve); past that, each kernel takes
    // whole rounds of its own occupancy, which leaves no partial last round
    // (the update kernel on 2049^2 vectors: 7% faster).
    const size_t b = B > 1 ? (size_t)B : 1;
    const bool k32 = kind == KB_DOT32 || kind == KB_UPDATE32;
    const size_t r0 = (size_t)resident_blocks(k32 ? KB_DOT32 : KB_DOT),
                 r1 = (size_t)resident_blocks(k32 ? KB_UPDATE32 : KB_UPDATE);
    const size_t rmin = r0 < r1 ? r0 : r1;
    const size_t res = n * b <= rmin * 256 * KR_S ? rmin : (size_t)resident_blocks(kind);
    const size_t per_round = res * 256 * KR_S;
    const size_t rounds = (n * b + per_round - 1) / per_round;
    size_t nb = (res * (rounds > 0 ? rounds : 1) + b - 1) / b;
    const size_t minb = (n + 256 * KR_S - 1) / (256 * KR_S);
    if (nb < minb) nb = minb;
    const size_t maxb = (n + 255) / 256;
    if (nb > maxb) nb = maxb > 0 ? maxb : 1;
    return (int)nb;
}

int krylov_blocks_max(size_t n, int B)
{
    int m = 0;
    for (int k = 0; k < KB_NKINDS; k++) {
        const int v = krylov_blocks(n, B, k);
        if (v > m) m = v;
    }
    return m;
}

static size_t krylov_chunk(size_t n, int nb) { return (n + nb - 1) / nb; }

// Basis vectors are streamed once per pass: non-temporal 16-byte loads keep
// them from displacing w and the partial sums in the caches.
typedef double d2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ cd ldnt(const cd *p)
{
    const d2v v = __builtin_nontemporal_load((const d2v *)p);
    return make_double2(v.x, v.y);
}
typedef float f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ cd ldnt(const cf *p)
{
    const f2v v = __builtin_nontemporal_load((const f2v *)p);
    return make_double2(v.x, v.y);
}
// An entry of w (either storage type) as complex128.
__device__ __forceinline__ cd ldc(const cd *p) { return *p; }
__device__ __forceinline__ cd ldc(const cf *p)
{
    const cf v = *p;
    return make_double2(v.x, v.y);
}
// Store v; return the value as stored (rounded to complex64 for cf).
// (complex128 entries are stored non-temporally: the updated vector is the
// new basis vector, streamed past the caches like the rest of the basis)
__device__ __forceinline__ cd stc(cd *p, cd v)
{
    d2v t;
    t.x = v.x;
    t.y = v.y;
    __builtin_nontemporal_store(t, (d2v *)p);
    return v;
}
__device__ __forceinline__ cd stc(cf *p, cd v)
{
    const cf r = make_float2((float)v.x, (float)v.y);
    *p = r;
    return make_double2(r.x, r.y);
}

__device__ __forceinline__ cd wave_sum(cd v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        v.x += __shfl_xor(v.x, o, 64);
        v.y += __shfl_xor(v.y, o, 64);
    }
    return v;
}

// Reorthogonalisation test of the DGKS kind on the first Gram-Schmidt pass:
// hb[0..j1) are the projections h_i, hb[j1].x = ||w||^2 before projection.
// With ||w'||^2 = ||w||^2 - sum |h_i|^2, a second pass is needed when
// ||w'|| < ||w|| / sqrt(2).  Every kernel of the second pass evaluates this
// same expression in the same order, so they agree.
__device__ __forceinline__ bool need_reorth(const cd *__restrict__ hb, int j1)
{
    double s = 0.0;
    for (int i = 0; i < j1; i++) s = fma(hb[i].x, hb[i].x, fma(hb[i].y, hb[i].y, s));
    const double w2 = hb[j1].x;
    return !(w2 - s > 0.5 * w2);
}

// (At least 3 waves per SIMD: the complex64 basis passes otherwise take
// enough registers to drop to 2, measured 10% slower.)
// part[blk][i] = sum over the block's chunk of conj(V_i) w, i < m; slot m gets
// |w|^2 when with_norm.  If cond != nullptr the kernel is the second
// Gram-Schmidt pass and exits at once unless need_reorth(cond, jcond).
// NV basis vectors V[i..i+NV) against the thread's KR_S entries of w: the
// block's partial products go to red[wave][i + u].
template <int NV, class TV>
__device__ __forceinline__ void mdot_pass(const TV *__restrict__ V, size_t ld, int i,
                                          const cd (&wv)[KR_S], size_t base, size_t end,
                                          cd (&red)[4][PSTRIDE], int lane, int wave)
{
    cd a[NV];
#pragma unroll
    for (int u = 0; u < NV; u++) a[u] = czero();
#pragma unroll
    for (int s = 0; s < KR_S; s++) {
        const size_t p = base + threadIdx.x + (size_t)s * 256;
        if (p < end) {
            cd x[NV];
#pragma unroll
            for (int u = 0; u < NV; u++) x[u] = ldnt(V + (size_t)(i + u) * ld + p);
#pragma unroll
            for (int u = 0; u < NV; u++) {
                a[u].x = fma(x[u].x, wv[s].x, fma(x[u].y, wv[s].y, a[u].x));
                a[u].y = fma(x[u].x, wv[s].y, fma(-x[u].y, wv[s].x, a[u].y));
            }
        }
    }
#pragma unroll
    for (int u = 0; u < NV; u++) {
        a[u] = wave_sum(a[u]);
        if (lane == 0) red[wave][i + u] = a[u];
    }
}

template <class TV, class TW>
__global__ __launch_bounds__(256, 3) void k_mdot(const TV *__restrict__ V, size_t ld, int m,
                                              const TW *__restrict__ w, size_t n, size_t chunk,
                                              cd *__restrict__ part, int with_norm,
                                              const cd *__restrict__ cond, int jcond, size_t vbs,
                                              size_t wbs, Batch bt)
{
    if (skip_rhs(bt)) return;
    {
        const size_t rb = blockIdx.y;
        if (V) V += rb * vbs;
        w += rb * wbs;
        part += rb * gridDim.x * PSTRIDE;
        if (cond) cond += rb * SB;
    }
    if (cond && !need_reorth(cond, jcond)) return;
    __shared__ cd red[4][PSTRIDE];
    const size_t base = (size_t)blockIdx.x * chunk;
    size_t end = base + chunk;
    if (end > n) end = n;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    cd wv[KR_S];
#pragma unroll
    for (int s = 0; s < KR_S; s++) {
        const size_t p = base + threadIdx.x + (size_t)s * 256;
        wv[s] = p < end ? ldc(w + p) : czero();
    }
    // Basis vectors per pass: 2 of complex128, 8 of complex64 (measured best
    // for 8-byte entries); each product sums over s in order.
    int i = 0;
    if constexpr (sizeof(TV) == 16) {
        for (; i + 1 < m; i += 2) {
            const TV *v0 = V + (size_t)i * ld, *v1 = V + (size_t)(i + 1) * ld;
            cd a0 = czero(), a1 = czero();
#pragma unroll
            for (int s = 0; s < KR_S; s++) {
                const size_t p = base + threadIdx.x + (size_t)s * 256;
                if (p < end) {
                    const cd x0 = ldnt(v0 + p), x1 = ldnt(v1 + p);
                    a0.x = fma(x0.x, wv[s].x, fma(x0.y, wv[s].y, a0.x));
                    a0.y = fma(x0.x, wv[s].y, fma(-x0.y, wv[s].x, a0.y));
                    a1.x = fma(x1.x, wv[s].x, fma(x1.y, wv[s].y, a1.x));
                    a1.y = fma(x1.x, wv[s].y, fma(-x1.y, wv[s].x, a1.y));
                }
            }
            a0 = wave_sum(a0);
            a1 = wave_sum(a1);
            if (lane == 0) {
                red[wave][i] = a0;
                red[wave][i + 1] = a1;
            }
        }
    }
    if constexpr (sizeof(TV) == 8) {
        for (; i + 8 <= m; i += 8) mdot_pass<8>(V, ld, i, wv, base, end, red, lane, wave);
        if (i + 4 <= m) {
            mdot_pass<4>(V, ld, i, wv, base, end, red, lane, wave);
            i += 4;
        }
        if (i + 2 <= m) {
            mdot_pass<2>(V, ld, i, wv, base, end, red, lane, wave);
            i += 2;
        }
        if (i < m) mdot_pass<1>(V, ld, i, wv, base, end, red, lane, wave);
    } else if (i < m) {
        const TV *v0 = V + (size_t)i * ld;
        cd a0 = czero();
#pragma unroll
        for (int s = 0; s < KR_S; s++) {
            const size_t p = base + threadIdx.x + (size_t)s * 256;
            if (p < end) {
                const cd x0 = ldnt(v0 + p);
                a0.x = fma(x0.x, wv[s].x, fma(x0.y, wv[s].y, a0.x));
                a0.y = fma(x0.x, wv[s].y, fma(-x0.y, wv[s].x, a0.y));
            }
        }
        a0 = wave_sum(a0);
        if (lane == 0) red[wave][i] = a0;
    }
    if (with_norm) {
        cd acc = czero();
#pragma unroll
        for (int s = 0; s < KR_S; s++) acc.x = fma(wv[s].x, wv[s].x, fma(wv[s].y, wv[s].y, acc.x));
        acc = wave_sum(acc);
        if (lane == 0) red[wave][m] = acc;
    }
    __syncthreads();
    const int tot = m + (with_norm ? 1 : 0);
    if ((int)threadIdx.x < tot) {
        const int q = threadIdx.x;
        part[(size_t)blockIdx.x * PSTRIDE + q] =
            cadd(cadd(red[0][q], red[1][q]), cadd(red[2][q], red[3][q]));
    }
}

hipError_t launch_mdot(const cd *V, size_t ld, int m, const cd *w, size_t n, cd *part,
                       int with_norm, const cd *cond, int jcond, hipStream_t st, Batch bt,
                       size_t vbs, size_t wbs)
{
    const int nb = krylov_blocks(n, bt.B, KB_DOT);
    k_mdot<cd, cd><<<dim3(nb, bt.B), 256, 0, st>>>(V, ld, m, w, n, krylov_chunk(n, nb), part,
                                                   with_norm, cond, jcond, vbs, wbs, bt);
    HD_LAUNCH_CHECK();
}

hipError_t launch_mdot32(const cf *V, size_t ld, int m, const cd *w, size_t n, cd *part,
                         int with_norm, const cd *cond, int jcond, hipStream_t st)
{
    const int nb = krylov_blocks(n, 1, KB_DOT32);
    k_mdot<cf, cd><<<nb, 256, 0, st>>>(V, ld, m, w, n, krylov_chunk(n, nb), part, with_norm,
                                       cond, jcond, 0, 0, Batch{});
    HD_LAUNCH_CHECK();
}

hipError_t launch_mdot32(const cf *V, size_t ld, int m, const cf *w, size_t n, cd *part,
                         int with_norm, const cd *cond, int jcond, hipStream_t st)
{
    const int nb = krylov_blocks(n, 1, KB_DOT32);
    k_mdot<cf, cf><<<nb, 256, 0, st>>>(V, ld, m, w, n, krylov_chunk(n, nb), part, with_norm,
                                       cond, jcond, 0, 0, Batch{});
    HD_LAUNCH_CHECK();
}

// w -= sum_i c_i sig_i V_i over the block's chunk (sig_i = 1 without sig);
// partn[blk] = |w_new|^2 partial (if partn).  cond: second pass, skipped
// unless need_reorth(cond, jcond).
// acc -= sum_{u < NV} c_{i+u} sig_{i+u} V[i+u] over the thread's KR_S entries
// (sig_i = 1 without sig), the vectors taken in the order of i.
template <int NV, class TV>
__device__ __forceinline__ void mupdate_pass(const TV *__restrict__ V, size_t ld, int i,
                                             const cd *__restrict__ c,
                                             const cd *__restrict__ sig, cd (&acc)[KR_S],
                                             size_t base, size_t end)
{
    cd cc[NV];
#pragma unroll
    for (int u = 0; u < NV; u++) cc[u] = sig ? cscal(sig[i + u].x, c[i + u]) : c[i + u];
#pragma unroll
    for (int s = 0; s < KR_S; s++) {
        const size_t p = base + threadIdx.x + (size_t)s * 256;
        if (p < end) {
            cd x[NV];
#pragma unroll
            for (int u = 0; u < NV; u++) x[u] = ldnt(V + (size_t)(i + u) * ld + p);
#pragma unroll
            for (int u = 0; u < NV; u++) {
                acc[s].x = fma(-cc[u].x, x[u].x, fma(cc[u].y, x[u].y, acc[s].x));
                acc[s].y = fma(-cc[u].x, x[u].y, fma(-cc[u].y, x[u].x, acc[s].y));
            }
        }
    }
}

// win and wout may be the same vector (in-place update, same entry type).
template <class TV, class TW, class TO>
__global__ __launch_bounds__(256) void k_mupdate(const TW *win, TO *wout,
                                                 const TV *__restrict__ V,
                                                 size_t ld, int m, const cd *__restrict__ c,
                                                 size_t n, size_t chunk, cd *__restrict__ partn,
                                                 const cd *__restrict__ cond, int jcond,
                                                 const cd *__restrict__ sig, size_t vbs,
                                                 size_t wbs, Batch bt)
{
    if (skip_rhs(bt)) return;
    {
        const size_t rb = blockIdx.y;
        win += rb * wbs;
        wout += rb * wbs;
        V += rb * vbs;
        c += rb * SB;
        if (partn) partn += rb * gridDim.x * PSTRIDE;
        if (cond) cond += rb * SB;
        if (sig) sig += rb * SB;
    }
    if (cond && !need_reorth(cond, jcond)) return;
    __shared__ cd red[4];
    const size_t base = (size_t)blockIdx.x * chunk;
    size_t end = base + chunk;
    if (end > n) end = n;
    // acc = w - sum_i c_i V_i, started from w so that its loads overlap the
    // first basis loads instead of waiting for the end
    cd acc[KR_S];
#pragma unroll
    for (int s = 0; s < KR_S; s++) {
        const size_t p = base + threadIdx.x + (size_t)s * 256;
        acc[s] = p < end ? ldc(win + p) : czero();
    }
    // Basis vectors per pass: 2 of complex128 (this form measured 7% faster
    // than a hand-written pair loop), up to 8 of complex64; the updates of an
    // entry are applied in the order of i.
    int i = 0;
    if constexpr (sizeof(TV) == 8) {
        for (; i + 8 <= m; i += 8) mupdate_pass<8>(V, ld, i, c, sig, acc, base, end);
        if (i + 4 <= m) {
            mupdate_pass<4>(V, ld, i, c, sig, acc, base, end);
            i += 4;
        }
    }
    for (; i + 2 <= m; i += 2) mupdate_pass<2>(V, ld, i, c, sig, acc, base, end);
    if (i < m) mupdate_pass<1>(V, ld, i, c, sig, acc, base, end);
    cd nrm = czero();
#pragma unroll
    for (int s = 0; s < KR_S; s++) {
        const size_t p = base + threadIdx.x + (size_t)s * 256;
        if (p < end) {
            // the norm is that of the stored (possibly rounded) entries
            const cd o = stc(wout + p, acc[s]);
            nrm.x = fma(o.x, o.x, fma(o.y, o.y, nrm.x));
        }
    }
    if (partn) {
        nrm = wave_sum(nrm);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nrm;
        __syncthreads();
        if (threadIdx.x == 0)
            partn[(size_t)blockIdx.x * PSTRIDE] = cadd(cadd(red[0], red[1]), cadd(red[2], red[3]));
    }
}

hipError_t launch_mupdate(cd *w, const cd *V, size_t ld, int m, const cd *c, size_t n, cd *partn,
                          const cd *cond, int jcond, const cd *sig, hipStream_t st, Batch bt,
                          size_t vbs, size_t wbs)
{
    const int nb = krylov_blocks(n, bt.B, KB_UPDATE);
    k_mupdate<cd, cd, cd><<<dim3(nb, bt.B), 256, 0, st>>>(w, w, V, ld, m, c, n,
                                                          krylov_chunk(n, nb), partn, cond, jcond,
                                                          sig, vbs, wbs, bt);
    HD_LAUNCH_CHECK();
}

hipError_t launch_mupdate32(const cd *win, cf *wout, const cf *V, size_t ld, int m, const cd *c,
                            size_t n, cd *partn, const cd *cond, int jcond, const cd *sig,
                            hipStream_t st)
{
    const int nb = krylov_blocks(n, 1, KB_UPDATE32);
    k_mupdate<cf, cd, cf><<<nb, 256, 0, st>>>(win, wout, V, ld, m, c, n, krylov_chunk(n, nb),
                                              partn, cond, jcond, sig, 0, 0, Batch{});
    HD_LAUNCH_CHECK();
}

hipError_t launch_mupdate32(cf *w, const cf *V, size_t ld, int m, const cd *c, size_t n,
                            cd *partn, const cd *cond, int jcond, const cd *sig, hipStream_t st)
{
    const int nb = krylov_blocks(n, 1, KB_UPDATE32);
    k_mupdate<cf, cf, cf><<<nb, 256, 0, st>>>(w, w, V, ld, m, c, n, krylov_chunk(n, nb), partn,
                                              cond, jcond, sig, 0, 0, Batch{});
    HD_LAUNCH_CHECK();
}

// out[i] = sum over blocks of part[blk][i] (fixed tree order); mode 0 store
// (times sig[i] for i < nsig when sig is given), 1 accumulate, 2 store
// sqrt(real part) into out[0] and, if sig_out, its reciprocal (0 for a zero
// norm) into sig_out[0].  cond: second-pass reduction, which stores zeros
// unless need_reorth(cond, jcond).
__global__ __launch_bounds__(256) void k_reduce(const cd *__restrict__ part, int nblk,
                                                cd *out, int mode,
                                                const cd *__restrict__ cond, int jcond,
                                                const cd *__restrict__ sig, int nsig,
                                                cd *__restrict__ sig_out, Batch bt,
                                                const cd *pub_src, int pub_n, cd *pub_dst)
{
    if (skip_rhs(bt)) return;
    {
        const size_t rb = blockIdx.y;
        part += rb * nblk * PSTRIDE;
        out += rb * SB;
        if (cond) cond += rb * SB;
        if (sig) sig += rb * SB;
        if (sig_out) sig_out += rb * SB;
    }
    __shared__ cd red[256];
    const int i = blockIdx.x;
    if (cond && !need_reorth(cond, jcond)) {
        if (threadIdx.x == 0) out[i] = czero();
        return;
    }
    cd s = czero();
    for (int b = threadIdx.x; b < nblk; b += 256) s = cadd(s, part[(size_t)b * PSTRIDE + i]);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        cd v = red[0];
        if (mode == 0) {
            if (sig && i < nsig) v = cscal(sig[i].x, v);
            out[i] = v;
        } else if (mode == 1) {
            out[i] = cadd(out[i], v);
        } else {
            const double nr = sqrt(v.x);
            out[i] = make_double2(nr, 0.0);
            if (sig_out) sig_out[0] = make_double2(nr > 0.0 ? 1.0 / nr : 0.0, 0.0);
        }
    }
    if (pub_dst) {
        // publish pub_src[0, pub_n) (written by earlier kernels, and out[i]
        // just above: out may lie inside pub_src, so neither is restrict) to
        // host-visible memory
        __syncthreads();
        for (int q = threadIdx.x; q < pub_n; q += 256) pub_dst[q] = pub_src[q];
        __threadfence_system();
    }
}

hipError_t launch_reduce(const cd *part, int nblk, int m, cd *out, int mode, const cd *cond,
                         int jcond, const cd *sig, int nsig, cd *sig_out, hipStream_t st,
                         Batch bt)
{
    k_reduce<<<dim3(m, bt.B), 256, 0, st>>>(part, nblk, out, mode, cond, jcond, sig, nsig, sig_out,
                                            bt, nullptr, 0, nullptr);
    HD_LAUNCH_CHECK();
}

hipError_t launch_norm_publish(const cd *part, int nblk, cd *out, cd *sig_out,
                               const cd *pub_src, int pub_n, cd *pub_dst, hipStream_t st)
{
    k_reduce<<<1, 256, 0, st>>>(part, nblk, out, 2, nullptr, 0, nullptr, 0, sig_out, Batch{},
                                pub_src, pub_n, pub_dst);
    HD_LAUNCH_CHECK();
}

__global__ __launch_bounds__(256) void k_scale(const cd *__restrict__ w, const cd *__restrict__ nrm,
                                               cd *__restrict__ v, size_t n, size_t wbs,
                                               size_t vbs, Batch bt)
{
    if (skip_rhs(bt)) return;
    w += blockIdx.y * wbs;
    v += blockIdx.y * vbs;
    nrm += (size_t)blockIdx.y * SB;
    const size_t p = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    const double h = nrm[0].x;
    v[p] = h > 0.0 ? cscal(1.0 / h, w[p]) : czero();
}

hipError_t launch_scale(const cd *w, const cd *nrm, cd *v, size_t n, hipStream_t st, Batch bt,
                        size_t wbs, size_t vbs)
{
    k_scale<<<dim3((unsigned)((n + 255) / 256), bt.B), 256, 0, st>>>(w, nrm, v, n, wbs, vbs, bt);
    HD_LAUNCH_CHECK();
}

template <class TV>
__global__ __launch_bounds__(256) void k_lincomb(const TV *__restrict__ V, size_t ld, int m,
                                                 const cd *__restrict__ y, cd *__restrict__ out,
                                                 size_t n, int accumulate, size_t vbs,
                                                 size_t obs, Batch bt)
{
    if (skip_rhs(bt)) return;
    V += blockIdx.y * vbs;
    out += blockIdx.y * obs;
    y += (size_t)blockIdx.y * SB;
    const size_t p = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    cd s = accumulate ? out[p] : czero();
    // a zero weight skips its vector: slots past a right-hand side's last
    // step (padded with zeros) never enter the sum, whatever they hold
    for (int i = 0; i < m; i++)
        if (y[i].x != 0.0 || y[i].y != 0.0) s = cadd(s, cmul(y[i], ldc(V + (size_t)i * ld + p)));
    out[p] = s;
}

hipError_t launch_lincomb(const cd *V, size_t ld, int m, const cd *y, cd *out, size_t n,
                          int accumulate, hipStream_t st, Batch bt, size_t vbs, size_t obs)
{
    k_lincomb<cd><<<dim3((unsigned)((n + 255) / 256), bt.B), 256, 0, st>>>(V, ld, m, y, out, n,
                                                                           accumulate, vbs, obs,
                                                                           bt);
    HD_LAUNCH_CHECK();
}

__global__ __launch_bounds__(256) void k_zero(cd *__restrict__ p, size_t n)
{
    const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (q < n) p[q] = czero();
}

hipError_t launch_zero(cd *p, size_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    k_zero<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(p, n);
    HD_LAUNCH_CHECK();
}

// in and out may be the same buffer (each thread touches one entry)
__global__ __launch_bounds__(256) void k_mask_copy(Lev L, const cd *in, cd *out)
{
    in += (size_t)blockIdx.y * L.nx * L.ny;
    out += (size_t)blockIdx.y * L.nx * L.ny;
    const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= (size_t)L.nx * L.ny) return;
    const int i = (int)(q % L.nx), j = (int)(q / L.nx);
    out[q] = unknown(L, i, j) ? in[q] : czero();
}

hipError_t launch_mask_copy(const Lev &L, const cd *in, cd *out, hipStream_t st, int B)
{
    const size_t n = (size_t)L.nx * L.ny;
    k_mask_copy<<<dim3((unsigned)((n + 255) / 256), B), 256, 0, st>>>(L, in, out);
    HD_LAUNCH_CHECK();
}

}  // namespace hd
