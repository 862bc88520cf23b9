// helmdefl.cpp -- host side of libhelmdefl.so: the solver handle, the level
// hierarchy, the V-cycle / deflation / Krylov drivers that sequence the HIP
// kernels, and the C-ABI of include/helmdefl.h.
//
// Every arithmetic step of the solve runs in the kernels of kernels.hip; the
// host only launches them, reads the Krylov scalars back (one small copy per
// Arnoldi step), does the O(m^2) Givens / least-squares work of GMRES and,
// on the single-source inner path, evaluates the Gram-Schmidt cancellation
// test on the scalars it has read, to queue the rare second pass.
#include "helmdefl.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "hd_common.h"

using namespace hd;
typedef std::complex<double> zc;

// Fixed device scratch of cslp_vcycle_noalloc: the level buffers (r and x on
// levels >= 1, FP64 or complex64) of such a call live here instead of in the
// handle.  Every GPU that loads the library holds its own copy until the
// process ends.  In host code `scratch` names a host-side stand-in: kernels
// are given the device address that hipGetSymbolAddress returns for it, kept
// per device in g_scratch_dev.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) double2 scratch[NOALLOC_SCRATCH_BYTES / sizeof(double2)];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[MAX_DEVICES] = {};

// Device address of `scratch` on device `dev` (the current device), looked up
// once per device.
int scratch_init(int dev)
{
    if (dev < 0 || dev >= MAX_DEVICES) return HELM_EHIP;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_dev[dev]) return HELM_OK;
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
        (void)hipGetLastError();
        return HELM_EHIP;
    }
    g_scratch_dev[dev] = p;
    return HELM_OK;
}
}  // namespace

namespace {

constexpr int MAXLEV = 40;
constexpr int MAX_COARSEST = 2048;  // nodes of the coarsest multigrid level
// device scalars of the inner solve: h1[64], h2[64], norm, the constant 1, and
// the norm of a restart's residual (published with the cycle's first step)
constexpr int HBUF = 2 * PSTRIDE + 3;
constexpr int HB_BETA = 2 * PSTRIDE + 2;

#define HCHK(call)                                   \
    do {                                             \
        hipError_t e_ = (call);                      \
        if (e_ != hipSuccess) return HELM_EHIP;      \
    } while (0)
#define RCHK(call)                    \
    do {                              \
        int r_ = (call);              \
        if (r_ != HELM_OK) return r_; \
    } while (0)

struct LevelH {
    int nx = 0, ny = 0;
    double hx = 0, hy = 0;
    double *kdev = nullptr;  // per-level wavenumber (nullptr: constant)
    cd *r = nullptr;         // V-cycle right-hand side on this level (l >= 1)
    cd *x = nullptr;         // V-cycle correction on this level (l >= 1)
    cf *rf = nullptr;        // complex64 twins for the mixed-precision cycle
    cf *xf = nullptr;
    size_t n() const { return (size_t)nx * (size_t)ny; }
};

// Host-side GMRES least-squares state: Hessenberg columns reduced by complex
// Givens rotations.
struct Givens {
    int m;
    std::vector<zc> H, g, sn;
    std::vector<double> cs;
    explicit Givens(int m_) : m(m_), H((size_t)(m_ + 1) * m_), g(m_ + 1), sn(m_), cs(m_) {}
    void start(double beta)
    {
        std::fill(g.begin(), g.end(), zc(0));
        g[0] = beta;
    }
    zc &h(int i, int j) { return H[(size_t)i * m + j]; }
    // column j holds h(0..j, j); hn = h(j+1, j) >= 0.  Returns |g_{j+1}|.
    double add_column(int j, const zc *col, double hn)
    {
        for (int i = 0; i <= j; i++) h(i, j) = col[i];
        for (int i = 0; i < j; i++) {
            const zc a = h(i, j), b = h(i + 1, j);
            h(i, j) = cs[i] * a + sn[i] * b;
            h(i + 1, j) = -std::conj(sn[i]) * a + cs[i] * b;
        }
        const zc a = h(j, j);
        const double aa = std::abs(a);
        if (hn == 0.0) {
            cs[j] = 1.0;
            sn[j] = 0.0;
        } else if (aa == 0.0) {
            cs[j] = 0.0;
            sn[j] = 1.0;
        } else {
            const double rho = std::sqrt(aa * aa + hn * hn);
            cs[j] = aa / rho;
            sn[j] = (a / aa) * hn / rho;
        }
        h(j, j) = cs[j] * a + sn[j] * hn;
        g[j + 1] = -std::conj(sn[j]) * g[j];
        g[j] = cs[j] * g[j];
        return std::abs(g[j + 1]);
    }
    void solve(int jend, std::vector<zc> &y)
    {
        y.assign(jend, zc(0));
        for (int i = jend - 1; i >= 0; i--) {
            zc s = g[i];
            for (int q = i + 1; q < jend; q++) s -= h(i, q) * y[q];
            y[i] = s / h(i, i);
        }
    }
};

// Workspace of batched solves: B right-hand sides of one operator in
// lockstep.  Level buffers are [B][n_l]; Krylov bases are stored j-major,
// [j][B][n], so basis slot j of every right-hand side is one contiguous block
// (the input of a batched V-cycle or operator) and vector j of right-hand side
// b sits at (j*B + b)*n.  Small per-right-hand-side device arrays (projections,
// norms, 1/||u||, least-squares solutions) are SB entries apart.
constexpr int HB = 2 * PSTRIDE + 1;  // scalars read back per right-hand side
constexpr int NMASK = 64;            // rotating active-mask buffers
constexpr int GCHUNK = 4;            // inner steps per captured graph (batched path)
constexpr int NSLOT = 2 * GCHUNK;    // read-back slots of the batched inner steps

struct BatchWS {
    int B = 0;
    cd *lr[MAXLEV] = {}, *lx[MAXLEV] = {};
    cf *lrf[MAXLEV] = {}, *lxf[MAXLEV] = {};  // complex64 levels (mixed precision)
    cd *v1 = nullptr, *v2 = nullptr, *tf = nullptr;
    cd *Vc = nullptr, *Zc = nullptr;  // inner basis V and Z = M^-1 V (slot-major, B per slot)
    cd *part = nullptr, *partn = nullptr;
    cd *hbuf = nullptr, *sig = nullptr, *ydev = nullptr;
    cd *V = nullptr, *Z = nullptr, *w = nullptr, *bm = nullptr;  // outer FGMRES
    int *dmask = nullptr;  // NMASK device masks of B entries
    int *hmask = nullptr;  // their pinned staging
    int next_mask = 0;
    cd *hpin = nullptr;    // pinned: NSLOT read-back slots of B x HB, then y staging B x SB
    hipEvent_t ev[2] = {nullptr, nullptr};
    // captured chunks of inner steps (opts.graphs): one graph per (first step,
    // length), reading the active mask from gmask
    int *gmask = nullptr;
    std::vector<std::pair<int, hipGraphExec_t>> gchunk;
    bool graph_off = false;
    std::vector<int> reo;  // per right-hand side: Arnoldi steps with a second pass
};

}  // namespace

struct helm_ctx {
    helm_grid g{};
    helm_opts o{};
    hipStream_t st = nullptr;
    int dev = 0;  // the HIP device current at helm_create
    double kconst = 0;
    int nlev = 0;
    LevelH L[MAXLEV];
    cd shift = make_double2(1.0, 0.5);
    int zho = 1;

    // coarsest level dense inverse
    cd *cinv = nullptr;
    cf *cinvf = nullptr;  // its FP32 rounding (mixed precision)
    int ncoarsest = 0;

    // deflation workspace (coarse grid = level 1)
    cd *v1 = nullptr, *v2 = nullptr, *tf = nullptr;
    // inner GMRES: basis V (mc + 1 vectors) and Z (mc vectors), z_j = M^-1 v_j
    int mc = 0;
    cd *Vc = nullptr, *Zc = nullptr, *xin = nullptr;
    // mixed precision: the inner basis in complex64 (FP64 A_2h output in wtmp)
    bool basis32 = false;
    cf *Vc32 = nullptr;
    cd *wtmp = nullptr;
    // reductions
    cd *part = nullptr, *partn = nullptr;
    int part_blocks = 0;
    long long n_arnoldi = 0, n_reorth = 0;  // Arnoldi steps, and those with a second pass
    cd *hbuf = nullptr, *ydev = nullptr;
    cd *sig = nullptr;   // 1/||u_i|| of the lazily normalised inner basis
    cd *hpin = nullptr;  // pinned: two Arnoldi read-back slots, y staging, norm
    // pinned, coherent and device-mapped: the inner steps' scalars, two slots
    // (written by the device; hpub_dev is the device's address of hpub)
    cd *hpub = nullptr, *hpub_dev = nullptr;
    hipEvent_t ev_slot[2] = {nullptr, nullptr};
    hipEvent_t ev_y = nullptr;  // the last upload of y from its pinned staging
    // outer FGMRES (allocated on first solve)
    int m = 0;
    cd *V = nullptr, *Z = nullptr, *w = nullptr, *bm = nullptr;
    cd *w2 = nullptr, *r = nullptr;  // GCR / left GMRES work vectors
    BatchWS *bw = nullptr;           // batched solves (allocated on first use)
    cd *adjb = nullptr;              // adjoint solve right-hand sides
    size_t adjb_n = 0;

    // captured coarse-GMRES steps, one per basis index (null until first use),
    // without and with the device-side second Gram-Schmidt pass; graph_off
    // after a capture failed
    std::vector<hipGraphExec_t> gstep, gstep2;
    bool graph_off = false;
    // moving average of how often an inner step's cancellation test fires
    // (0.9 old + 0.1 new): from 1/8 on, the steps launch the second pass
    // themselves (decided on the device) rather than leave it to the host;
    // both give the same iterates
    double reo_rate = 0.0;

    // kernel timing
    int t_cls = -1, t_lev = -1;
    std::vector<hipEvent_t> ev_free;
    struct Pend {
        hipEvent_t a, b;
        double bytes;
    };
    std::vector<Pend> pend;
    long long t_count = 0;
    double t_ms = 0, t_bytes = 0;

    // phase timing of helm_solve: events around the coarse solves (phase 0)
    // and the fine-grid V-cycles (phase 1) of the solve in progress
    bool ph_on = false;
    std::vector<hipEvent_t> ph_free;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ph_pend[2];
    double t_setup_ms = 0;  // wall time of helm_create

    Lev lev(int l) const
    {
        const LevelH &q = L[l];
        return make_lev(q.nx, q.ny, q.hx, q.hy, g.bc, q.kdev, kconst);
    }
};

namespace {

// ---------------------------------------------------------------------------
// kernel timing: events around launches of one kernel class / level
// ---------------------------------------------------------------------------
int timing_flush(helm_ctx *h)
{
    if (h->pend.empty()) return HELM_OK;
    HCHK(hipStreamSynchronize(h->st));
    for (auto &p : h->pend) {
        float ms = 0;
        HCHK(hipEventElapsedTime(&ms, p.a, p.b));
        h->t_ms += ms;
        h->t_bytes += p.bytes;
        h->t_count++;
        h->ev_free.push_back(p.a);
        h->ev_free.push_back(p.b);
    }
    h->pend.clear();
    return HELM_OK;
}

struct Timed {
    helm_ctx *h;
    bool on;
    hipEvent_t a{}, b{};
    double bytes;
    Timed(helm_ctx *h_, int cls, int level, double bytes_) : h(h_), on(false), bytes(bytes_)
    {
        if (h->t_cls != cls || (h->t_lev >= 0 && h->t_lev != level)) return;
        if (h->pend.size() >= 4096 && timing_flush(h) != HELM_OK) return;
        for (int q = 0; q < 2; q++) {
            hipEvent_t e;
            if (!h->ev_free.empty()) {
                e = h->ev_free.back();
                h->ev_free.pop_back();
            } else if (hipEventCreate(&e) != hipSuccess) {
                return;
            }
            (q == 0 ? a : b) = e;
        }
        on = hipEventRecord(a, h->st) == hipSuccess;
    }
    ~Timed()
    {
        if (!on) return;
        (void)hipEventRecord(b, h->st);
        h->pend.push_back({a, b, bytes});
    }
};

// Events bracketing one phase of a solve (no-op unless h->ph_on).
struct Phase {
    helm_ctx *h;
    int k;
    hipEvent_t a{}, b{};
    bool on = false;
    Phase(helm_ctx *h_, int k_) : h(h_), k(k_)
    {
        if (!h->ph_on) return;
        for (int q = 0; q < 2; q++) {
            hipEvent_t e;
            if (!h->ph_free.empty()) {
                e = h->ph_free.back();
                h->ph_free.pop_back();
            } else if (hipEventCreate(&e) != hipSuccess) {
                (void)hipGetLastError();
                return;
            }
            (q == 0 ? a : b) = e;
        }
        on = hipEventRecord(a, h->st) == hipSuccess;
    }
    ~Phase()
    {
        if (!on) return;
        (void)hipEventRecord(b, h->st);
        h->ph_pend[k].push_back({a, b});
    }
};

// Start phase timing for a solve.
void phase_begin(helm_ctx *h)
{
    h->ph_on = true;
    for (auto &v : h->ph_pend) v.clear();
}

// Stop phase timing (after the stream has been synchronised) and return the
// summed times in ms of the coarse solves and of the fine V-cycles.
void phase_end(helm_ctx *h, double *t_coarse, double *t_vcycle)
{
    double t[2] = {0, 0};
    for (int k = 0; k < 2; k++) {
        for (auto &p : h->ph_pend[k]) {
            float ms = 0;
            if (hipEventElapsedTime(&ms, p.first, p.second) == hipSuccess) t[k] += ms;
            h->ph_free.push_back(p.first);
            h->ph_free.push_back(p.second);
        }
        h->ph_pend[k].clear();
    }
    (void)hipGetLastError();
    h->ph_on = false;
    *t_coarse = t[0];
    *t_vcycle = t[1];
}

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
template <class T>
int dalloc(T **p, size_t count)
{
    *p = nullptr;
    if (count == 0) return HELM_OK;
    if (hipMalloc((void **)p, count * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return HELM_ENOMEM;
    }
    return HELM_OK;
}

void dfree(void *p)
{
    if (p) (void)hipFree(p);
}

bool coarsenable(int nx, int ny) { return nx >= 5 && ny >= 5 && (nx & 1) && (ny & 1); }

// Pinned read-back layout: slot q of the Arnoldi scalars at q*HBUF, the
// least-squares solution staging at 2*HBUF, the norm read-back at 3*HBUF.
constexpr int PIN_Y = 2 * HBUF, PIN_NORM = 3 * HBUF, PIN_TOTAL = 4 * HBUF;

// ||v|| of a device vector into out_dev[0] (device), and 1/||v|| into
// sig_out[0] when given; nothing is read back.
int vnorm_enqueue(helm_ctx *h, const cd *v, size_t n, cd *out_dev, cd *sig_out)
{
    const int nb = krylov_blocks(n);
    HCHK(launch_mdot(nullptr, 0, 0, v, n, h->part, 1, nullptr, 0, h->st));
    HCHK(launch_reduce(h->part, nb, 1, out_dev, 2, nullptr, 0, nullptr, 0, sig_out, h->st));
    return HELM_OK;
}

// ||v|| of a device vector (synchronises); also stores 1/||v|| in sig_out[0]
// when given.
int vnorm(helm_ctx *h, const cd *v, size_t n, double *out, cd *sig_out = nullptr)
{
    RCHK(vnorm_enqueue(h, v, n, h->hbuf + 2 * PSTRIDE, sig_out));
    HCHK(hipMemcpyAsync(h->hpin + PIN_NORM, h->hbuf + 2 * PSTRIDE, sizeof(cd),
                        hipMemcpyDeviceToHost, h->st));
    HCHK(hipStreamSynchronize(h->st));
    *out = h->hpin[PIN_NORM].x;
    return HELM_OK;
}

// Arnoldi step by classical Gram-Schmidt with conditional reorthogonalisation:
// w is projected against V[0..j1-1] in one pass; a second pass runs only when
// the device-side test of the DGKS kind finds cancellation (||w'|| below
// ||w||/sqrt(2)); the kernels of the second pass read the first pass's
// projections and decide by themselves, so the host never waits in between.
// Then V[j1] = w / ||w||; col[0..j1-1] receives the projections (both passes
// summed), *hn the norm.  One device->host copy, then sync.
int arnoldi_step(helm_ctx *h, cd *V, size_t ld, int j1, cd *w, size_t n, zc *col, double *hn,
                 int lev)
{
    const int nb = krylov_blocks(n), nbu = krylov_blocks(n, 1, KB_UPDATE);
    cd *h1 = h->hbuf, *h2 = h->hbuf + PSTRIDE, *nr = h->hbuf + 2 * PSTRIDE;
    {
        Timed tm(h, HELM_K_DOT, lev, 16.0 * (j1 + 1) * n);
        HCHK(launch_mdot(V, ld, j1, w, n, h->part, 1, nullptr, 0, h->st));
    }
    HCHK(launch_reduce(h->part, nb, j1 + 1, h1, 0, nullptr, 0, nullptr, 0, nullptr,
                       h->st));  // h1[j1] = ||w||^2
    {
        Timed tm(h, HELM_K_UPDATE, lev, 16.0 * (j1 + 2) * n);
        HCHK(launch_mupdate(w, V, ld, j1, h1, n, h->partn, nullptr, 0, nullptr, h->st));
    }
    HCHK(launch_mdot(V, ld, j1, w, n, h->part, 0, h1, j1, h->st));
    HCHK(launch_reduce(h->part, nb, j1, h2, 0, h1, j1, nullptr, 0, nullptr, h->st));
    HCHK(launch_mupdate(w, V, ld, j1, h2, n, h->partn, h1, j1, nullptr, h->st));
    HCHK(launch_reduce(h->partn, nbu, 1, nr, 2, nullptr, 0, nullptr, 0, nullptr, h->st));
    HCHK(launch_scale(w, nr, V + (size_t)j1 * ld, n, h->st));
    HCHK(hipMemcpyAsync(h->hpin, h->hbuf, (2 * PSTRIDE + 1) * sizeof(cd), hipMemcpyDeviceToHost,
                        h->st));
    HCHK(hipStreamSynchronize(h->st));
    bool reorth = false;
    for (int i = 0; i < j1; i++) {
        col[i] = zc(h->hpin[i].x + h->hpin[PSTRIDE + i].x, h->hpin[i].y + h->hpin[PSTRIDE + i].y);
        reorth |= h->hpin[PSTRIDE + i].x != 0.0 || h->hpin[PSTRIDE + i].y != 0.0;
    }
    h->n_arnoldi++;
    h->n_reorth += reorth;
    *hn = h->hpin[2 * PSTRIDE].x;
    return HELM_OK;
}

// Record slot `slot`'s event after an inner step: the step's last kernel has
// written its scalars (projections, second-pass projections, norm) to the
// host-visible slot hpub + slot * HBUF.
int step_readback(helm_ctx *h, int slot)
{
    HCHK(hipEventRecord(h->ev_slot[slot], h->st));
    return HELM_OK;
}

// Arnoldi step of the inner solve on a lazily normalised basis: V[i] holds
// u_i with v_i = sig[i] u_i.  The new vector w = A z already sits in V[j1];
// it is orthogonalised in place by one classical Gram-Schmidt pass and
// sig[j1] = 1/||w'|| is stored, so no scaling pass is needed.  Everything is
// enqueued; the norm reduction also writes the step's scalars to the host
// slot hpub + slot * HBUF, and (with readback) ev_slot[slot] is recorded.
// arnoldi_finish() waits for that event and evaluates the cancellation test;
// the second pass is then arnoldi_repair(), queued by the host.  With dev2
// the step launches the second pass itself, each kernel of it returning at
// once unless the same test, evaluated on the device, fires (h2 = 0 then).
int arnoldi_lazy_enqueue(helm_ctx *h, cd *V, size_t ld, int j1, size_t n, int lev, int slot,
                         bool readback = true, bool dev2 = false)
{
    const int nb = krylov_blocks(n), nbu = krylov_blocks(n, 1, KB_UPDATE);
    cd *w = V + (size_t)j1 * ld;
    cd *h1 = h->hbuf, *h2 = h->hbuf + PSTRIDE, *nr = h->hbuf + 2 * PSTRIDE;
    {
        Timed tm(h, HELM_K_DOT, lev, 16.0 * (j1 + 1) * n);
        HCHK(launch_mdot(V, ld, j1, w, n, h->part, 1, nullptr, 0, h->st));
    }
    HCHK(launch_reduce(h->part, nb, j1 + 1, h1, 0, nullptr, 0, h->sig, j1, nullptr, h->st));
    {
        Timed tm(h, HELM_K_UPDATE, lev, 16.0 * (j1 + 2) * n);
        HCHK(launch_mupdate(w, V, ld, j1, h1, n, h->partn, nullptr, 0, h->sig, h->st));
    }
    if (dev2) {
        HCHK(launch_mdot(V, ld, j1, w, n, h->part, 0, h1, j1, h->st));
        HCHK(launch_reduce(h->part, nb, j1, h2, 0, h1, j1, h->sig, j1, nullptr, h->st));
        HCHK(launch_mupdate(w, V, ld, j1, h2, n, h->partn, h1, j1, h->sig, h->st));
    }
    HCHK(launch_norm_publish(h->partn, nbu, nr, h->sig + j1, h->hbuf, HBUF,
                             h->hpub_dev + slot * HBUF, h->st));
    if (readback) RCHK(step_readback(h, slot));
    return HELM_OK;
}

// The cancellation test of the first pass, from the published projections
// hb[0..j1) and hb[j1].x = ||w||^2: a second pass is needed when
// ||w'||^2 = ||w||^2 - sum |h_i|^2 falls to half of ||w||^2 or below (the
// expression and order of need_reorth on the device, with explicit FMAs).
bool need_reorth_host(const cd *hb, int j1)
{
    double s = 0.0;
    for (int i = 0; i < j1; i++) s = std::fma(hb[i].x, hb[i].x, std::fma(hb[i].y, hb[i].y, s));
    const double w2 = hb[j1].x;
    return !(w2 - s > 0.5 * w2);
}

// Wait for an inner step's scalars (slot `slot`).  col[0..j1) = the
// projections, *hn = ||w'||.  With `lazy` (a step of arnoldi_lazy_enqueue
// without its second pass) *repair tells whether the cancellation test asks
// for one; otherwise the step's own second pass (h2) is added in, and *fired
// tells whether it ran.
int arnoldi_finish(helm_ctx *h, int j1, int slot, zc *col, double *hn, bool lazy = false,
                   bool *repair = nullptr, bool *fired = nullptr)
{
    HCHK(hipEventSynchronize(h->ev_slot[slot]));
    const cd *hp = h->hpub + slot * HBUF;
    bool reorth = false;
    for (int i = 0; i < j1; i++) {
        if (lazy) {
            col[i] = zc(hp[i].x, hp[i].y);
        } else {
            col[i] = zc(hp[i].x + hp[PSTRIDE + i].x, hp[i].y + hp[PSTRIDE + i].y);
            reorth |= hp[PSTRIDE + i].x != 0.0 || hp[PSTRIDE + i].y != 0.0;
        }
    }
    h->n_arnoldi++;
    h->n_reorth += reorth;
    *hn = hp[2 * PSTRIDE].x;
    if (repair) *repair = lazy && need_reorth_host(hp, j1);
    if (fired) *fired = reorth;
    return HELM_OK;
}

// The second Gram-Schmidt pass of the inner step that produced V[j1], queued
// by the host after arnoldi_finish() asked for it (behind whatever step was
// already queued): h2 = V^H w', w'' = w' - V h2 in place, sig[j1] =
// 1/||w''||, and the slot republished (its h2 and norm; its h1 part then
// holds the later step's projections and is not read).  Waits for the slot;
// col[0..j1) += h2, *hn = ||w''||.
int arnoldi_repair(helm_ctx *h, int j1, int slot, zc *col, double *hn)
{
    const size_t n = h->L[1].n(), ld = n;
    const int nb = krylov_blocks(n), nbu = krylov_blocks(n, 1, KB_UPDATE);
    cd *V = h->Vc, *w = h->Vc + (size_t)j1 * ld;
    cd *h2 = h->hbuf + PSTRIDE, *nr = h->hbuf + 2 * PSTRIDE;
    HCHK(launch_mdot(V, ld, j1, w, n, h->part, 0, nullptr, 0, h->st));
    HCHK(launch_reduce(h->part, nb, j1, h2, 0, nullptr, 0, h->sig, j1, nullptr, h->st));
    HCHK(launch_mupdate(w, V, ld, j1, h2, n, h->partn, nullptr, 0, h->sig, h->st));
    HCHK(launch_norm_publish(h->partn, nbu, nr, h->sig + j1, h->hbuf, HBUF,
                             h->hpub_dev + slot * HBUF, h->st));
    RCHK(step_readback(h, slot));
    HCHK(hipEventSynchronize(h->ev_slot[slot]));
    const cd *hp = h->hpub + slot * HBUF;
    for (int i = 0; i < j1; i++) col[i] += zc(hp[PSTRIDE + i].x, hp[PSTRIDE + i].y);
    h->n_reorth++;
    *hn = hp[2 * PSTRIDE].x;
    return HELM_OK;
}

int upload_y(helm_ctx *h, const std::vector<zc> &y)
{
    // the staging buffer may still be read by the previous upload's copy
    // (in practice long done: the host has waited on later work since)
    HCHK(hipEventSynchronize(h->ev_y));
    for (size_t i = 0; i < y.size(); i++)
        h->hpin[PIN_Y + i] = make_double2(y[i].real(), y[i].imag());
    HCHK(hipMemcpyAsync(h->ydev, h->hpin + PIN_Y, y.size() * sizeof(cd), hipMemcpyHostToDevice,
                        h->st));
    HCHK(hipEventRecord(h->ev_y, h->st));
    return HELM_OK;
}

// ---------------------------------------------------------------------------
// operators
// ---------------------------------------------------------------------------
int apply_A(helm_ctx *h, int l, const cd *x, const cd *b, cd *y)
{
    const Lev Lv = h->lev(l);
    Timed tm(h, HELM_K_APPLY, l, (b ? 48.0 : 32.0) * h->L[l].n());
    HCHK(launch_apply5(Lv, make_double2(1.0, 0.0), x, b, y, h->st));
    return HELM_OK;
}

// z (+)= V-cycle(r) from level 0 in complex64: FP64 r in, FP32 levels, FP64 z
// out (with Z v2 added in FP64).
int vcycle_mixed(helm_ctx *h, const cd *r, cd *z, int accumulate, const cd *v2)
{
    const int Lc = h->nlev - 1;
    for (int l = 0; l < Lc; l++) {
        const double by = (l == 0 ? 16.0 : 8.0) * h->L[l].n() + 8.0 * h->L[l + 1].n();
        Timed tm(h, HELM_K_VC_DOWN, l, by);
        if (l == 0)
            HCHK(launch_vc_down(h->lev(0), h->lev(1), h->shift, h->o.omega, r, h->L[1].rf, h->st));
        else
            HCHK(launch_vc_down(h->lev(l), h->lev(l + 1), h->shift, h->o.omega, h->L[l].rf,
                                h->L[l + 1].rf, h->st));
    }
    HCHK(launch_coarsest(h->ncoarsest, h->cinvf, h->L[Lc].rf, h->L[Lc].xf, h->st));
    for (int l = Lc - 1; l >= 0; l--) {
        if (l == 0) {
            const double by = (32.0 + 16.0 * accumulate) * h->L[0].n() + 8.0 * h->L[1].n() +
                              (v2 ? 16.0 * h->L[1].n() : 0.0);
            Timed tm(h, HELM_K_VC_UP, 0, by);
            HCHK(launch_vc_up(h->lev(0), h->lev(1), h->shift, h->o.omega, r, h->L[1].xf, z,
                              accumulate, v2, h->zho, h->st));
        } else {
            Timed tm(h, HELM_K_VC_UP, l, 16.0 * h->L[l].n() + 8.0 * h->L[l + 1].n());
            HCHK(launch_vc_up(h->lev(l), h->lev(l + 1), h->shift, h->o.omega, h->L[l].rf,
                              h->L[l + 1].xf, h->L[l].xf, h->st));
        }
    }
    return HELM_OK;
}

// The downward passes of the levels below level `top`: the last ones above
// the coarsest (VC_DTAIL_MAXLEV at most, two at least, with opts.vc_tail > 0)
// in one fused launch.  Returns the first level whose downward pass is fused
// (its right-hand side must be in place before vc_down_tail), or the
// coarsest level when none is.
int dtail_start(const helm_ctx *h, int top)
{
    const int Lc = h->nlev - 1;
    if (h->o.vc_tail <= 0) return Lc;
    const int nd = std::min(VC_DTAIL_MAXLEV, Lc - top - 1);
    if (nd < 2 || (double)h->L[Lc - nd].n() > (double)h->o.vc_tail) return Lc;
    return Lc - nd;
}

// The fused downward passes from level ld (as dtail_start chose it) to the
// coarsest: reads level ld's right-hand side, writes those of levels
// ld + 1 .. Lc.
int vc_down_tail(helm_ctx *h, int ld)
{
    const int Lc = h->nlev - 1, nd = Lc - ld;
    Lev levs[VC_DTAIL_MAXLEV + 1];
    cd *out[VC_DTAIL_MAXLEV];
    double by = 16.0 * h->L[ld].n();
    for (int j = 0; j <= nd; j++) levs[j] = h->lev(Lc - j);
    for (int j = 0; j < nd; j++) {
        out[j] = h->L[Lc - j].r;
        by += 16.0 * h->L[Lc - j].n();
    }
    Timed tm(h, HELM_K_VC_DOWN, ld, by);
    HCHK(launch_vc_down_tail(nd, levs, h->L[ld].r, out, h->shift, h->o.omega, h->st));
    return HELM_OK;
}

// The upward passes of the levels below level `top`, from the coarsest up:
// the small ones (at most opts.vc_tail nodes each, VC_TAIL_MAXLEV at most,
// two at least) in one fused launch.  *next = the highest level whose upward
// pass is still to run, level by level.
int vc_up_tail(helm_ctx *h, int top, int *next)
{
    const int Lc = h->nlev - 1;
    *next = Lc - 1;
    if (h->o.vc_tail <= 0) return HELM_OK;
    int lt = top + 1;
    while (lt < Lc && (double)h->L[lt].n() > (double)h->o.vc_tail) lt++;
    lt = std::max(lt, Lc - VC_TAIL_MAXLEV);
    const int nt = Lc - lt;
    if (nt < 2) return HELM_OK;
    Lev levs[VC_TAIL_MAXLEV + 1];
    const cd *rr[VC_TAIL_MAXLEV];
    double by = 16.0 * h->L[lt].n() + 16.0 * h->L[Lc].n();
    for (int k = 0; k <= nt; k++) levs[k] = h->lev(lt + k);
    for (int k = 0; k < nt; k++) {
        rr[k] = h->L[lt + k].r;
        by += 16.0 * h->L[lt + k].n();
    }
    Timed tm(h, HELM_K_VC_UP, lt, by);
    HCHK(launch_vc_up_tail(nt, levs, rr, h->L[Lc].x, h->L[lt].x, h->shift, h->o.omega, h->st));
    *next = lt - 1;
    return HELM_OK;
}

// z (+)= V-cycle(r) starting on level l0; on level 0 the last pass may add
// Z v2 (v2 on level 1).  From level 0 with the mixed-precision option the
// cycle runs in complex64.
int vcycle(helm_ctx *h, int l0, const cd *r, cd *z, int accumulate, const cd *v2,
           const cd *rs = nullptr)
{
    const int Lc = h->nlev - 1;
    if (l0 == 0 && h->o.precision != HELM_PREC_FP64 && !rs)
        return vcycle_mixed(h, r, z, accumulate, v2);
    if (l0 == Lc) {
        // the cycle is the exact coarsest solve; it is linear, so a right-hand
        // side scale is applied to the result
        if (!accumulate && !rs) {
            HCHK(launch_coarsest(h->ncoarsest, h->cinv, r, z, h->st));
            return HELM_OK;
        }
        HCHK(launch_coarsest(h->ncoarsest, h->cinv, r, h->L[Lc].x, h->st));
        HCHK(launch_lincomb(h->L[Lc].x, 0, 1, rs ? rs : h->hbuf + 2 * PSTRIDE + 1, z,
                            h->L[Lc].n(), accumulate, h->st));
        return HELM_OK;
    }
    const cd *rin = r;
    const int ld = dtail_start(h, l0);
    for (int l = l0; l < ld; l++) {
        Timed tm(h, HELM_K_VC_DOWN, l, 16.0 * h->L[l].n() + 16.0 * h->L[l + 1].n());
        HCHK(launch_vc_down(h->lev(l), h->lev(l + 1), h->shift, h->o.omega, rin,
                            l == l0 ? rs : nullptr, h->L[l + 1].r, h->st));
        rin = h->L[l + 1].r;
    }
    if (ld < Lc) RCHK(vc_down_tail(h, ld));
    HCHK(launch_coarsest(h->ncoarsest, h->cinv, h->L[Lc].r, h->L[Lc].x, h->st));
    int lup;
    RCHK(vc_up_tail(h, l0, &lup));
    for (int l = lup; l >= l0; l--) {
        const bool top = l == l0;
        const cd *rl = top ? r : h->L[l].r;
        cd *out = top ? z : h->L[l].x;
        const int acc = top ? accumulate : 0;
        const cd *vv = top ? v2 : nullptr;
        const double by = (32.0 + 16.0 * acc) * h->L[l].n() + 16.0 * h->L[l + 1].n() * (vv ? 2 : 1);
        Timed tm(h, HELM_K_VC_UP, l, by);
        HCHK(launch_vc_up(h->lev(l), h->lev(l + 1), h->shift, h->o.omega, rl,
                          top ? rs : nullptr, h->L[l + 1].x, out, acc, vv, h->zho, h->st));
    }
    return HELM_OK;
}

// z = V-cycle(rs[0].x r) from level 1 for a complex64 r (an entry of the
// mixed-precision inner basis): the top level reads r in complex64, the
// arithmetic and the levels below are FP64.  Needs a level below level 1.
int vcycle32(helm_ctx *h, const cf *r, cd *z, const cd *rs)
{
    const int Lc = h->nlev - 1;
    {
        Timed tm(h, HELM_K_VC_DOWN, 1, 8.0 * h->L[1].n() + 16.0 * h->L[2].n());
        HCHK(launch_vc_down(h->lev(1), h->lev(2), h->shift, h->o.omega, r, rs, h->L[2].r, h->st));
    }
    const int ld = dtail_start(h, 1);
    for (int l = 2; l < ld; l++) {
        Timed tm(h, HELM_K_VC_DOWN, l, 16.0 * h->L[l].n() + 16.0 * h->L[l + 1].n());
        HCHK(launch_vc_down(h->lev(l), h->lev(l + 1), h->shift, h->o.omega, h->L[l].r, nullptr,
                            h->L[l + 1].r, h->st));
    }
    if (ld < Lc) RCHK(vc_down_tail(h, ld));
    HCHK(launch_coarsest(h->ncoarsest, h->cinv, h->L[Lc].r, h->L[Lc].x, h->st));
    int lup;
    RCHK(vc_up_tail(h, 1, &lup));
    for (int l = lup; l >= 2; l--) {
        Timed tm(h, HELM_K_VC_UP, l, 32.0 * h->L[l].n() + 16.0 * h->L[l + 1].n());
        HCHK(launch_vc_up(h->lev(l), h->lev(l + 1), h->shift, h->o.omega, h->L[l].r, nullptr,
                          h->L[l + 1].x, h->L[l].x, 0, nullptr, h->zho, h->st));
    }
    Timed tm(h, HELM_K_VC_UP, 1, 24.0 * h->L[1].n() + 16.0 * h->L[2].n());
    HCHK(launch_vc_up(h->lev(1), h->lev(2), h->shift, h->o.omega, r, rs, h->L[2].x, z, 0, h->st));
    return HELM_OK;
}

// y = A_2h x  or  y = b - A_2h x
int coarse_apply(helm_ctx *h, const cd *x, const cd *b, cd *y)
{
    const Lev Lf = h->lev(0), Lc = h->lev(1);
    const size_t nc = h->L[1].n(), nf = h->L[0].n();
    if (h->o.coarse_op != HELM_COARSE_GALERKIN) {
        Timed tm(h, HELM_K_COARSE, 1, (b ? 48.0 : 32.0) * nc);
        switch (h->o.coarse_op) {
        case HELM_COARSE_REDGLK2: HCHK(launch_redglk2(Lc, x, b, y, 0, h->st)); break;
        case HELM_COARSE_REDGLK1: HCHK(launch_redglk2(Lc, x, b, y, 1, h->st)); break;
        case HELM_COARSE_REDO4: HCHK(launch_redo4(Lc, x, b, y, h->st)); break;
        default: HCHK(launch_apply5(Lc, make_double2(1.0, 0.0), x, b, y, h->st));  // ReD-O2
        }
        return HELM_OK;
    }
    // Galerkin: Z^T A_h Z in one launch (coarse vectors in and out, plus the
    // fine wavenumber on a variable-k grid)
    Timed tm(h, HELM_K_COARSE, 1, (b ? 48.0 : 32.0) * nc + (Lf.k ? 8.0 * nf : 0.0));
    HCHK(launch_glk(Lf, Lc, h->zho, x, b, y, h->st));
    return HELM_OK;
}

// One inner Arnoldi step j, enqueued: z = V(v_j), w = A_2h z written into
// basis slot j+1, then the lazily normalised orthogonalisation, whose last
// kernel writes the step's scalars to host slot `slot` (and, with readback,
// the slot's event).
int inner_step_enqueue(helm_ctx *h, int j, int slot, bool readback = true, bool dev2 = false)
{
    const size_t nc = h->L[1].n();
    cd *z = h->Zc + (size_t)j * nc;
    RCHK(vcycle(h, 1, h->Vc + (size_t)j * nc, z, 0, nullptr, h->sig + j));
    RCHK(coarse_apply(h, z, nullptr, h->Vc + (size_t)(j + 1) * nc));
    return arnoldi_lazy_enqueue(h, h->Vc, nc, j + 1, nc, 1, slot, readback, dev2);
}

// The same step on the complex64 basis (mixed precision): A_2h z is formed
// in FP64 in wtmp; the first Gram-Schmidt pass reads it and writes the
// orthogonalised vector, rounded, into basis slot j1; a second pass (when
// needed) works in place on that slot.  Products and norms are FP64.
int arnoldi_lazy_enqueue32(helm_ctx *h, size_t n, int j1, int slot, bool readback = true)
{
    const int nb = krylov_blocks(n, 1, KB_DOT32), nbu = krylov_blocks(n, 1, KB_UPDATE32);
    const size_t ld = n;
    const cf *V = h->Vc32;
    cf *w = h->Vc32 + (size_t)j1 * ld;
    cd *h1 = h->hbuf, *h2 = h->hbuf + PSTRIDE, *nr = h->hbuf + 2 * PSTRIDE;
    {
        Timed tm(h, HELM_K_DOT, 1, 8.0 * j1 * n + 16.0 * n);
        HCHK(launch_mdot32(V, ld, j1, h->wtmp, n, h->part, 1, nullptr, 0, h->st));
    }
    HCHK(launch_reduce(h->part, nb, j1 + 1, h1, 0, nullptr, 0, h->sig, j1, nullptr, h->st));
    {
        Timed tm(h, HELM_K_UPDATE, 1, 8.0 * j1 * n + 24.0 * n);
        HCHK(launch_mupdate32(h->wtmp, w, V, ld, j1, h1, n, h->partn, nullptr, 0, h->sig, h->st));
    }
    HCHK(launch_mdot32(V, ld, j1, w, n, h->part, 0, h1, j1, h->st));
    HCHK(launch_reduce(h->part, nb, j1, h2, 0, h1, j1, h->sig, j1, nullptr, h->st));
    HCHK(launch_mupdate32(w, V, ld, j1, h2, n, h->partn, h1, j1, h->sig, h->st));
    HCHK(launch_norm_publish(h->partn, nbu, nr, h->sig + j1, h->hbuf, HBUF,
                             h->hpub_dev + slot * HBUF, h->st));
    if (readback) RCHK(step_readback(h, slot));
    return HELM_OK;
}

int inner_step_enqueue32(helm_ctx *h, int j, int slot, bool readback = true)
{
    const size_t nc = h->L[1].n();
    cd *z = h->Zc + (size_t)j * nc;
    RCHK(vcycle32(h, h->Vc32 + (size_t)j * nc, z, h->sig + j));
    RCHK(coarse_apply(h, z, nullptr, h->wtmp));
    return arnoldi_lazy_enqueue32(h, nc, j + 1, slot, readback);
}

// Inner step j through a HIP graph: its kernels (they depend on j only: the
// basis slots, the Gram-Schmidt length) are captured on first use and
// replayed from then on, one launch instead of about twenty.  The slot's
// event stays ordinary stream work (the scalars reach the host slot from the
// step's last kernel), so the graph holds kernel nodes only.  Off while
// kernel timing is on; a failed capture turns graphs off for this context and
// the step is launched directly.
int inner_step_run(helm_ctx *h, int j, int slot, bool dev2)
{
    const bool b32 = h->basis32;
    auto direct = [&](bool rb) {
        return b32 ? inner_step_enqueue32(h, j, slot, rb)
                   : inner_step_enqueue(h, j, slot, rb, dev2);
    };
    if (!h->o.graphs || h->graph_off || h->t_cls >= 0) return direct(true);
    std::vector<hipGraphExec_t> &gs = dev2 && !b32 ? h->gstep2 : h->gstep;
    if ((int)gs.size() <= j) gs.resize(j + 1, nullptr);
    if (!gs[j]) {
        if (hipStreamBeginCapture(h->st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            (void)hipGetLastError();
            h->graph_off = true;
            return direct(true);
        }
        const int rc = direct(false);
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(h->st, &g);
        hipGraphExec_t ex = nullptr;
        if (rc == HELM_OK && ec == hipSuccess && g &&
            hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess) {
            gs[j] = ex;
        } else {
            (void)hipGetLastError();
            h->graph_off = true;
        }
        if (g) (void)hipGraphDestroy(g);
        if (h->graph_off) return direct(true);
    }
    HCHK(hipGraphLaunch(gs[j], h->st));
    return step_readback(h, slot);
}

// Basis slot 0 (complex64) = u (FP64), rounded.
int basis32_set0(helm_ctx *h, const cd *u)
{
    const size_t nc = h->L[1].n();
    HCHK(launch_mupdate32(u, h->Vc32, h->Vc32, nc, 0, h->hbuf, nc, h->partn, nullptr, 0, nullptr,
                          h->st));
    return HELM_OK;
}

// x ~= A_2h^{-1} b: right-preconditioned restarted GMRES, preconditioner = a
// V-cycle starting on level 1, x0 = 0.  FIXED mode runs exactly coarse_iters
// iterations; TOL mode stops at |g_{j+1}| <= coarse_tol ||b|| (checked on the
// true residual at every restart) or at coarse_iters.
// The host needs each step's Hessenberg column only to test convergence, so
// step j+1 is enqueued before the host waits for step j: the GPU never idles
// on the read-back.  A converged cycle leaves one speculative step, whose
// results are not used.  Each step keeps z_j = M^-1 v_j (the V-cycle output
// that A_2h is applied to), so the end of a cycle adds sum_i y_i z_i to x
// without another V-cycle: with an exact coarsest solve the V-cycle is a fixed
// linear operator, and this equals M^-1 (V y) up to rounding.  With the
// complex64-basis option V is stored in complex64 (Z, and all arithmetic,
// stay FP64).
int coarse_solve(helm_ctx *h, const cd *b, cd *x, int *iters)
{
    const size_t nc = h->L[1].n();
    const int m = h->mc;
    const bool fixed = h->o.coarse_mode == HELM_CMODE_FIXED;
    const int cap = h->o.coarse_iters;
    const double tol = h->o.coarse_tol;
    const bool b32 = h->basis32;
    int it = 0;
    if (iters) *iters = 0;
    double bnorm;
    RCHK(vnorm(h, b, nc, &bnorm, h->sig));
    HCHK(launch_zero(x, nc, h->st));
    if (!std::isfinite(bnorm)) return HELM_ENONFINITE;
    if (bnorm == 0.0) return HELM_OK;
    Givens gv(m);
    std::vector<zc> col(m + 1), y;
    bool first = true, stop = false;
    for (;;) {
        // A cycle that ended at its restart length (its estimate still above
        // the tolerance) restarts without reading the residual norm back: the
        // norm stays on the device (hbuf[HB_BETA], 1/beta in sig[0]) and
        // reaches the host with the next cycle's first step, which is queued
        // at once; the tests on it are made then, and a cycle found not to be
        // needed is dropped (its queued steps write nothing read afterwards).
        // After a cycle whose estimate met the tolerance, the true residual is
        // read back first, as that restart usually ends the solve.
        const bool late_beta = !first && !stop;
        double beta = bnorm;  // first cycle: sig[0] = 1/||b|| was stored by vnorm
        if (first) {
            if (b32)
                RCHK(basis32_set0(h, b));
            else
                HCHK(hipMemcpyAsync(h->Vc, b, nc * sizeof(cd), hipMemcpyDeviceToDevice, h->st));
        } else {
            cd *r0 = b32 ? h->wtmp : h->Vc;
            RCHK(coarse_apply(h, x, b, r0));
            if (late_beta)
                RCHK(vnorm_enqueue(h, r0, nc, h->hbuf + HB_BETA, h->sig));
            else
                RCHK(vnorm(h, r0, nc, &beta, h->sig));
            if (b32) RCHK(basis32_set0(h, r0));
        }
        if (!late_beta) {
            if (!fixed && beta <= tol * bnorm) break;
            if (it >= cap || beta == 0.0) break;
            gv.start(beta);
        }
        const int steps = std::min(m, cap - it);
        int jend = 0;
        stop = false;
        bool dropped = false;
        // per slot: whether its step launched the second pass itself
        bool dev2[2] = {true, true};
        auto step = [&](int j, int slot) {
            dev2[slot] = b32 || h->reo_rate >= 0.125;
            return inner_step_run(h, j, slot, dev2[slot]);
        };
        RCHK(step(0, 0));
        for (int j = 0; j < steps; j++) {
            if (j + 1 < steps) RCHK(step(j + 1, (j + 1) & 1));
            if (j == 0 && late_beta) {
                HCHK(hipEventSynchronize(h->ev_slot[0]));
                beta = h->hpub[HB_BETA].x;
                if ((!fixed && beta <= tol * bnorm) || beta == 0.0) {
                    dropped = true;
                    break;
                }
                gv.start(beta);
            }
            double hn;
            bool repair = false, fired = false;
            RCHK(arnoldi_finish(h, j + 1, j & 1, col.data(), &hn, !dev2[j & 1], &repair,
                                &fired));
            h->reo_rate = 0.9 * h->reo_rate + ((repair || fired) ? 0.1 : 0.0);
            if (repair) {
                // second pass on v_{j+1}, queued behind the speculative step
                // j + 1, which read the vector before it; that step is then
                // queued again on the repaired vector
                RCHK(arnoldi_repair(h, j + 1, j & 1, col.data(), &hn));
                if (j + 1 < steps) RCHK(step(j + 1, (j + 1) & 1));
            }
            const double res = gv.add_column(j, col.data(), hn);
            it++;
            jend = j + 1;
            if ((!fixed && res <= tol * bnorm) || hn == 0.0) {
                stop = true;
                break;
            }
        }
        if (dropped) break;
        // x += sum_i y_i M^-1 v_i, from the z_i the steps kept, by the
        // Gram-Schmidt update kernel (x -= sum_i c_i z_i with c = -y), which
        // streams the z_i faster than the plain combination kernel
        gv.solve(jend, y);
        for (zc &v : y) v = -v;
        RCHK(upload_y(h, y));
        HCHK(launch_mupdate(x, h->Zc, nc, jend, h->ydev, nc, nullptr, nullptr, 0, nullptr, h->st));
        if (it >= cap) break;
        if (stop && fixed) break;
        first = false;
    }
    if (iters) *iters = it;
    return HELM_OK;
}

// w = Q v, (I - A Q) v or P_A-DEF1 v for one vector on level 0.
int deflate_one(helm_ctx *h, int mode, const cd *v, cd *w, int *inner)
{
    const Lev Lf = h->lev(0), Lc = h->lev(1);
    const size_t nf = h->L[0].n(), nc = h->L[1].n();
    {
        Timed tm(h, HELM_K_ZT, 0, 16.0 * nf + 16.0 * nc);
        HCHK(launch_zt(Lf, Lc, h->zho, v, nullptr, h->v1, h->st));
    }
    {
        Phase ph(h, 0);
        RCHK(coarse_solve(h, h->v1, h->v2, inner));
    }
    if (mode == HELM_DEFL_Q) {
        HCHK(launch_z(Lf, Lc, h->zho, h->v2, w, h->st));
        return HELM_OK;
    }
    cd *t = mode == HELM_DEFL_P ? w : h->tf;
    {
        Timed tm(h, HELM_K_DRESID, 0, 32.0 * nf + 16.0 * nc);
        HCHK(launch_dresid(Lf, Lc, h->zho, v, h->v2, t, h->st));
    }
    if (mode == HELM_DEFL_P) return HELM_OK;
    Phase ph(h, 1);
    return vcycle(h, 0, t, w, 0, h->v2);
}

int ensure_outer(helm_ctx *h)
{
    if (h->V) return HELM_OK;
    const size_t n = h->L[0].n();
    const int m = h->o.restart;
    const bool extra = h->o.outer != HELM_OUTER_FGMRES;
    int rc;
    if ((rc = dalloc(&h->V, (size_t)(m + 1) * n)) || (rc = dalloc(&h->Z, (size_t)m * n)) ||
        (rc = dalloc(&h->w, n)) || (rc = dalloc(&h->bm, n)) ||
        (extra && ((rc = dalloc(&h->w2, n)) || (rc = dalloc(&h->r, n))))) {
        dfree(h->V);
        dfree(h->Z);
        dfree(h->w);
        dfree(h->bm);
        dfree(h->w2);
        dfree(h->r);
        h->V = h->Z = h->w = h->bm = h->w2 = h->r = nullptr;
        return rc;
    }
    h->m = m;
    return HELM_OK;
}

// Flexible GMRES(m) for one right-hand side, right-preconditioned by
// P_A-DEF1 (z_j stored), true residual at every restart.
int solve_one(helm_ctx *h, const cd *b, cd *x, helm_solve_info *info)
{
    const auto t0 = std::chrono::steady_clock::now();
    const size_t n = h->L[0].n();
    const int m = h->m;
    const Lev L0 = h->lev(0);
    const int force = h->o.force_iters;
    const int cap = force > 0 ? force : h->o.maxit;
    helm_solve_info inf{};
    HCHK(launch_mask_copy(L0, b, h->bm, h->st));
    double bnorm;
    RCHK(vnorm(h, h->bm, n, &bnorm));
    if (!std::isfinite(bnorm)) return HELM_ENONFINITE;
    if (h->o.x0_given)
        HCHK(launch_mask_copy(L0, x, x, h->st));
    else
        HCHK(launch_zero(x, n, h->st));
    int rc = HELM_OK;
    if (bnorm == 0.0) {
        HCHK(launch_zero(x, n, h->st));
        inf.converged = 1;
    } else {
        Givens gv(m);
        std::vector<zc> col(m + 1), y;
        for (;;) {
            RCHK(apply_A(h, 0, x, h->bm, h->w));
            double beta;
            RCHK(vnorm(h, h->w, n, &beta));
            inf.relres = beta / bnorm;
            if (force <= 0 && inf.relres <= h->o.tol) {
                inf.converged = 1;
                break;
            }
            if (inf.outer_iters >= cap || beta == 0.0) break;
            HCHK(launch_scale(h->w, h->hbuf + 2 * PSTRIDE, h->V, n, h->st));
            gv.start(beta);
            int jend = 0;
            for (int j = 0; j < m && inf.outer_iters < cap; j++) {
                cd *vj = h->V + (size_t)j * n, *zj = h->Z + (size_t)j * n;
                int inner = 0;
                RCHK(deflate_one(h, HELM_DEFL_ADEF1, vj, zj, &inner));
                inf.inner_iters_total += inner;
                if (inner > inf.inner_iters_max) inf.inner_iters_max = inner;
                RCHK(apply_A(h, 0, zj, nullptr, h->w));
                double hn;
                RCHK(arnoldi_step(h, h->V, n, j + 1, h->w, n, col.data(), &hn, 0));
                const double res = gv.add_column(j, col.data(), hn);
                inf.outer_iters++;
                jend = j + 1;
                if (std::getenv("HELMDEFL_LOG"))
                    std::fprintf(stderr, "helmdefl: it %d  est relres %.3e  inner %d\n",
                                 inf.outer_iters, res / bnorm, inner);
                if (force <= 0 && res <= h->o.tol * bnorm) break;
                if (hn == 0.0) break;
            }
            gv.solve(jend, y);
            RCHK(upload_y(h, y));
            HCHK(launch_lincomb(h->Z, n, jend, h->ydev, x, n, 1, h->st));
            if (force > 0 && inf.outer_iters >= cap) {
                RCHK(apply_A(h, 0, x, h->bm, h->w));
                double r2;
                RCHK(vnorm(h, h->w, n, &r2));
                inf.relres = r2 / bnorm;
                inf.converged = inf.relres <= h->o.tol;
                break;
            }
        }
        if (!inf.converged && force <= 0) rc = HELM_ENOCONV;
    }
    HCHK(hipStreamSynchronize(h->st));
    inf.t_solve_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = inf;
    return rc;
}

// Read back the norm left by a mode-2 reduction in hbuf[2*PSTRIDE] (sync).
int read_norm(helm_ctx *h, double *out)
{
    HCHK(hipMemcpyAsync(h->hpin + PIN_NORM, h->hbuf + 2 * PSTRIDE, sizeof(cd),
                        hipMemcpyDeviceToHost, h->st));
    HCHK(hipStreamSynchronize(h->st));
    *out = h->hpin[PIN_NORM].x;
    return HELM_OK;
}

// Right-preconditioned GCR(m) (Section 6.3; the method of Eisenstat, Elman
// and Schultz), preconditioner P_A-DEF1.  Step j: z = P r, w = A z; w is
// orthogonalised against W[0..j-1] (the same Gram-Schmidt pass as the Arnoldi
// steps, with its conditional second pass) and the same coefficients are
// applied to z, so w = A z is kept; both are divided by ||w|| into W[j], Z[j];
// then alpha = W[j]^H r, x += alpha Z[j], r -= alpha W[j].  The pairs are
// dropped after m steps (restart from the true residual); when the updated
// residual reaches tol ||b|| the true residual decides.
int solve_gcr(helm_ctx *h, const cd *b, cd *x, helm_solve_info *info)
{
    const auto t0 = std::chrono::steady_clock::now();
    const size_t n = h->L[0].n();
    const int m = h->m, nb = krylov_blocks(n), nbu = krylov_blocks(n, 1, KB_UPDATE);
    const Lev L0 = h->lev(0);
    const int force = h->o.force_iters;
    const int cap = force > 0 ? force : h->o.maxit;
    cd *W = h->V, *Zs = h->Z, *r = h->r, *z = h->w2, *w = h->w;
    cd *h1 = h->hbuf, *h2 = h->hbuf + PSTRIDE, *nr = h->hbuf + 2 * PSTRIDE;
    helm_solve_info inf{};
    HCHK(launch_mask_copy(L0, b, h->bm, h->st));
    double bnorm;
    RCHK(vnorm(h, h->bm, n, &bnorm));
    if (!std::isfinite(bnorm)) return HELM_ENONFINITE;
    if (h->o.x0_given)
        HCHK(launch_mask_copy(L0, x, x, h->st));
    else
        HCHK(launch_zero(x, n, h->st));
    int rc = HELM_OK;
    std::vector<zc> col(m + 1);
    if (bnorm == 0.0) {
        HCHK(launch_zero(x, n, h->st));
        inf.converged = 1;
    } else {
        for (;;) {
            RCHK(apply_A(h, 0, x, h->bm, r));
            double rn;
            RCHK(vnorm(h, r, n, &rn));
            inf.relres = rn / bnorm;
            if (force <= 0 && inf.relres <= h->o.tol) {
                inf.converged = 1;
                break;
            }
            if (inf.outer_iters >= cap || rn == 0.0) break;
            for (int j = 0; j < m && inf.outer_iters < cap; j++) {
                int inner = 0;
                RCHK(deflate_one(h, HELM_DEFL_ADEF1, r, z, &inner));
                inf.inner_iters_total += inner;
                if (inner > inf.inner_iters_max) inf.inner_iters_max = inner;
                RCHK(apply_A(h, 0, z, nullptr, w));
                double nu;
                if (j == 0) {
                    RCHK(vnorm(h, w, n, &nu));
                    HCHK(launch_scale(w, nr, W, n, h->st));
                } else {
                    RCHK(arnoldi_step(h, W, n, j, w, n, col.data(), &nu, 0));
                    HCHK(launch_mupdate(z, Zs, n, j, h1, n, nullptr, nullptr, 0, nullptr, h->st));
                    HCHK(launch_mupdate(z, Zs, n, j, h2, n, nullptr, h1, j, nullptr, h->st));
                }
                HCHK(launch_scale(z, nr, Zs + (size_t)j * n, n, h->st));
                inf.outer_iters++;
                if (nu == 0.0) break;  // A P r already lies in the searched space
                cd *Wj = W + (size_t)j * n, *Zj = Zs + (size_t)j * n;
                HCHK(launch_mdot(Wj, n, 1, r, n, h->part, 0, nullptr, 0, h->st));
                HCHK(launch_reduce(h->part, nb, 1, h->ydev, 0, nullptr, 0, nullptr, 0, nullptr,
                                   h->st));
                HCHK(launch_lincomb(Zj, n, 1, h->ydev, x, n, 1, h->st));
                HCHK(launch_mupdate(r, Wj, n, 1, h->ydev, n, h->partn, nullptr, 0, nullptr,
                                    h->st));
                HCHK(launch_reduce(h->partn, nbu, 1, nr, 2, nullptr, 0, nullptr, 0, nullptr,
                                   h->st));
                RCHK(read_norm(h, &rn));
                if (std::getenv("HELMDEFL_LOG"))
                    std::fprintf(stderr, "helmdefl: gcr it %d  relres %.3e  inner %d\n",
                                 inf.outer_iters, rn / bnorm, inner);
                if (force <= 0 && rn <= h->o.tol * bnorm) break;
            }
            if (force > 0 && inf.outer_iters >= cap) {
                RCHK(apply_A(h, 0, x, h->bm, r));
                RCHK(vnorm(h, r, n, &rn));
                inf.relres = rn / bnorm;
                inf.converged = inf.relres <= h->o.tol;
                break;
            }
        }
        if (!inf.converged && force <= 0) rc = HELM_ENOCONV;
    }
    HCHK(hipStreamSynchronize(h->st));
    inf.t_solve_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = inf;
    return rc;
}

// The paper's left-preconditioned deflated GMRES (Algorithm 1) on
// P A x = P b, P = P_A-DEF1: v_1 = P (b - A x0) / ||.||, each step w = P (A v_j)
// orthogonalised against V (the Arnoldi step above), stopping when the
// preconditioned residual |g_{j+1}| drops to tol ||P b||.  Restarted after
// `restart` steps from the current x.  The non-singular A-DEF1 needs no final
// projection.  info.relres is the true residual at exit.
int solve_left(helm_ctx *h, const cd *b, cd *x, helm_solve_info *info)
{
    const auto t0 = std::chrono::steady_clock::now();
    const size_t n = h->L[0].n();
    const int m = h->m;
    const Lev L0 = h->lev(0);
    const int cap = h->o.maxit;
    cd *nr = h->hbuf + 2 * PSTRIDE;
    helm_solve_info inf{};
    HCHK(launch_mask_copy(L0, b, h->bm, h->st));
    double bnorm;
    RCHK(vnorm(h, h->bm, n, &bnorm));
    if (!std::isfinite(bnorm)) return HELM_ENONFINITE;
    if (h->o.x0_given)
        HCHK(launch_mask_copy(L0, x, x, h->st));
    else
        HCHK(launch_zero(x, n, h->st));
    int rc = HELM_OK;
    if (bnorm == 0.0) {
        HCHK(launch_zero(x, n, h->st));
        inf.converged = 1;
    } else {
        Givens gv(m);
        std::vector<zc> col(m + 1), y;
        double beta0 = -1.0;
        for (;;) {
            int inner = 0;
            RCHK(apply_A(h, 0, x, h->bm, h->w));
            RCHK(deflate_one(h, HELM_DEFL_ADEF1, h->w, h->w2, &inner));
            inf.inner_iters_total += inner;
            if (inner > inf.inner_iters_max) inf.inner_iters_max = inner;
            double beta;
            RCHK(vnorm(h, h->w2, n, &beta));
            if (beta0 < 0) beta0 = beta;
            if (beta <= h->o.tol * beta0 || beta == 0.0) {
                inf.converged = 1;
                break;
            }
            if (inf.outer_iters >= cap) break;
            HCHK(launch_scale(h->w2, nr, h->V, n, h->st));
            gv.start(beta);
            int jend = 0;
            bool done = false;
            for (int j = 0; j < m && inf.outer_iters < cap; j++) {
                RCHK(apply_A(h, 0, h->V + (size_t)j * n, nullptr, h->w));
                RCHK(deflate_one(h, HELM_DEFL_ADEF1, h->w, h->w2, &inner));
                inf.inner_iters_total += inner;
                if (inner > inf.inner_iters_max) inf.inner_iters_max = inner;
                double hn;
                RCHK(arnoldi_step(h, h->V, n, j + 1, h->w2, n, col.data(), &hn, 0));
                const double res = gv.add_column(j, col.data(), hn);
                inf.outer_iters++;
                jend = j + 1;
                if (std::getenv("HELMDEFL_LOG"))
                    std::fprintf(stderr, "helmdefl: left it %d  prec relres %.3e  inner %d\n",
                                 inf.outer_iters, res / beta0, inner);
                if (res <= h->o.tol * beta0) {
                    done = true;
                    break;
                }
                if (hn == 0.0) break;
            }
            gv.solve(jend, y);
            RCHK(upload_y(h, y));
            HCHK(launch_lincomb(h->V, n, jend, h->ydev, x, n, 1, h->st));
            if (done) {
                inf.converged = 1;
                break;
            }
        }
        RCHK(apply_A(h, 0, x, h->bm, h->w));
        double rn;
        RCHK(vnorm(h, h->w, n, &rn));
        inf.relres = rn / bnorm;
        if (!inf.converged) rc = HELM_ENOCONV;
    }
    HCHK(hipStreamSynchronize(h->st));
    inf.t_solve_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = inf;
    return rc;
}

// ---------------------------------------------------------------------------
// Batched solves (B right-hand sides of one operator, in lockstep).  Every
// right-hand side keeps its own Krylov basis, Hessenberg matrix and
// convergence test; the kernels of one step run for all of them in one launch
// each, and right-hand sides that have converged are masked out on the device.
// ---------------------------------------------------------------------------
void free_batch(BatchWS *W)
{
    if (!W) return;
    for (int l = 0; l < MAXLEV; l++) {
        dfree(W->lr[l]);
        dfree(W->lx[l]);
        dfree(W->lrf[l]);
        dfree(W->lxf[l]);
    }
    for (void *p : {(void *)W->v1, (void *)W->v2, (void *)W->tf,
                    (void *)W->Vc, (void *)W->Zc, (void *)W->part,
                    (void *)W->partn, (void *)W->hbuf, (void *)W->sig, (void *)W->ydev,
                    (void *)W->V, (void *)W->Z, (void *)W->w, (void *)W->bm, (void *)W->dmask})
        dfree(p);
    if (W->hmask) (void)hipHostFree(W->hmask);
    if (W->hpin) (void)hipHostFree(W->hpin);
    dfree(W->gmask);
    for (auto &g : W->gchunk)
        if (g.second) (void)hipGraphExecDestroy(g.second);
    for (auto e : W->ev)
        if (e) (void)hipEventDestroy(e);
    delete W;
}

// Batch workspace for exactly B right-hand sides (the layouts depend on B);
// the outer FGMRES bases only when `outer`.
int ensure_batch(helm_ctx *h, int B, bool outer)
{
    if (h->bw && h->bw->B != B) {
        HCHK(hipStreamSynchronize(h->st));
        free_batch(h->bw);
        h->bw = nullptr;
    }
    if (!h->bw) {
        BatchWS *W = new (std::nothrow) BatchWS();
        if (!W) return HELM_ENOMEM;
        W->B = B;
        const size_t nf = h->L[0].n(), nc = h->L[1].n(), b = (size_t)B;
        int rc = HELM_OK;
        for (int l = 1; l < h->nlev && !rc; l++) {
            rc = dalloc(&W->lr[l], b * h->L[l].n());
            if (!rc) rc = dalloc(&W->lx[l], b * h->L[l].n());
            if (!rc && h->o.precision != HELM_PREC_FP64) {
                rc = dalloc(&W->lrf[l], b * h->L[l].n());
                if (!rc) rc = dalloc(&W->lxf[l], b * h->L[l].n());
            }
        }
        if (!rc) rc = dalloc(&W->v1, b * nc);
        if (!rc) rc = dalloc(&W->v2, b * nc);
        if (!rc) rc = dalloc(&W->tf, b * nf);
        if (!rc) rc = dalloc(&W->Vc, (size_t)(h->mc + 1) * b * nc);
        if (!rc) rc = dalloc(&W->Zc, (size_t)h->mc * b * nc);
        // slots past a right-hand side's last step are read with weight 0
        // at the end of a cycle: keep them finite
        if (!rc && hipMemset(W->Zc, 0, (size_t)h->mc * b * nc * sizeof(cd)) != hipSuccess)
            rc = HELM_EHIP;
        if (!rc) rc = dalloc(&W->part, b * krylov_blocks_max(nf) * PSTRIDE);
        if (!rc) rc = dalloc(&W->partn, b * krylov_blocks_max(nf) * PSTRIDE);
        if (!rc) rc = dalloc(&W->hbuf, b * SB);
        if (!rc) rc = dalloc(&W->sig, b * SB);
        if (!rc) rc = dalloc(&W->ydev, b * SB);
        if (!rc) rc = dalloc(&W->dmask, (size_t)NMASK * b);
        if (!rc && hipHostMalloc((void **)&W->hmask, (size_t)NMASK * b * sizeof(int)) !=
                       hipSuccess) {
            W->hmask = nullptr;
            rc = HELM_ENOMEM;
        }
        if (!rc) rc = dalloc(&W->gmask, b);
        if (!rc && hipHostMalloc((void **)&W->hpin, (NSLOT * HB + SB) * b * sizeof(cd)) !=
                       hipSuccess) {
            W->hpin = nullptr;
            rc = HELM_ENOMEM;
        }
        for (int q = 0; q < 2 && !rc; q++)
            if (hipEventCreateWithFlags(&W->ev[q], hipEventDisableTiming) != hipSuccess) {
                W->ev[q] = nullptr;
                rc = HELM_EHIP;
            }
        if (!rc) {
            // slot 2*PSTRIDE+1 of every right-hand side holds the constant 1
            std::vector<cd> init(b * SB, make_double2(0.0, 0.0));
            for (int q = 0; q < B; q++) init[(size_t)q * SB + 2 * PSTRIDE + 1] = make_double2(1.0, 0.0);
            if (hipMemcpy(W->hbuf, init.data(), init.size() * sizeof(cd), hipMemcpyHostToDevice) !=
                hipSuccess)
                rc = HELM_EHIP;
        }
        if (rc) {
            free_batch(W);
            return rc;
        }
        h->bw = W;
    }
    BatchWS *W = h->bw;
    if (outer && !W->V) {
        const size_t nf = h->L[0].n(), b = (size_t)B;
        const int m = h->o.restart;
        int rc;
        if ((rc = dalloc(&W->V, (size_t)(m + 1) * b * nf)) ||
            (rc = dalloc(&W->Z, (size_t)m * b * nf)) || (rc = dalloc(&W->w, b * nf)) ||
            (rc = dalloc(&W->bm, b * nf))) {
            dfree(W->V);
            dfree(W->Z);
            dfree(W->w);
            dfree(W->bm);
            W->V = W->Z = W->w = W->bm = nullptr;
            return rc;
        }
    }
    return HELM_OK;
}

// Upload an active mask (host flags) into the next rotating device buffer and
// return it.  Buffers are reused only after NMASK uploads, and the stream is
// drained before the first reuse, so no buffer changes under a queued kernel.
const int *upload_mask(helm_ctx *h, const std::vector<char> &act)
{
    BatchWS *W = h->bw;
    if (W->next_mask == NMASK) {
        if (hipStreamSynchronize(h->st) != hipSuccess) return nullptr;
        W->next_mask = 0;
    }
    const int q = W->next_mask++;
    int *hm = W->hmask + (size_t)q * W->B;
    int *dm = W->dmask + (size_t)q * W->B;
    for (int b = 0; b < W->B; b++) hm[b] = act[b] ? 1 : 0;
    if (hipMemcpyAsync(dm, hm, W->B * sizeof(int), hipMemcpyHostToDevice, h->st) != hipSuccess)
        return nullptr;
    return dm;
}

#define MCHK(ptr)                                \
    do {                                         \
        if (!(ptr)) return HELM_EHIP;            \
    } while (0)

// Norms of B vectors (length n each, contiguous) for the active ones; when
// sig_out is given its entry 0 per right-hand side receives 1/||v||.
int vnorm_b(helm_ctx *h, const cd *v, size_t n, std::vector<double> &out, cd *sig_out,
            const int *dm)
{
    BatchWS *W = h->bw;
    const Batch bt{W->B, dm};
    const int nb = krylov_blocks(n, W->B);
    HCHK(launch_mdot(nullptr, 0, 0, v, n, W->part, 1, nullptr, 0, h->st, bt, 0, n));
    HCHK(launch_reduce(W->part, nb, 1, W->hbuf + 2 * PSTRIDE, 2, nullptr, 0, nullptr, 0, sig_out,
                       h->st, bt));
    HCHK(hipMemcpy2DAsync(W->hpin, sizeof(cd), W->hbuf + 2 * PSTRIDE, SB * sizeof(cd), sizeof(cd),
                          W->B, hipMemcpyDeviceToHost, h->st));
    HCHK(hipStreamSynchronize(h->st));
    out.resize(W->B);
    for (int b = 0; b < W->B; b++) out[b] = W->hpin[b].x;
    return HELM_OK;
}

// Batched V-cycle from level l0 (see vcycle); r, z: B contiguous vectors of
// level l0; rs: per-right-hand-side scale (SB apart) or nullptr.
// Batched V-cycle from level 0 in complex64 (as vcycle_mixed for every
// active right-hand side): FP64 r in, FP32 levels, FP64 z out with Z v2.
int vcycle_mixed_b(helm_ctx *h, const cd *r, cd *z, int accumulate, const cd *v2, const int *dm)
{
    BatchWS *W = h->bw;
    const Batch bt{W->B, dm};
    const int Lc = h->nlev - 1;
    for (int l = 0; l < Lc; l++) {
        if (l == 0)
            HCHK(launch_vc_down(h->lev(0), h->lev(1), h->shift, h->o.omega, r, W->lrf[1], h->st,
                                bt));
        else
            HCHK(launch_vc_down(h->lev(l), h->lev(l + 1), h->shift, h->o.omega, W->lrf[l],
                                W->lrf[l + 1], h->st, bt));
    }
    HCHK(launch_coarsest(h->ncoarsest, h->cinvf, W->lrf[Lc], W->lxf[Lc], h->st, bt));
    for (int l = Lc - 1; l >= 1; l--)
        HCHK(launch_vc_up(h->lev(l), h->lev(l + 1), h->shift, h->o.omega, W->lrf[l],
                          W->lxf[l + 1], W->lxf[l], h->st, bt));
    HCHK(launch_vc_up(h->lev(0), h->lev(1), h->shift, h->o.omega, r, W->lxf[1], z, accumulate, v2,
                      h->zho, h->st, bt));
    return HELM_OK;
}

int vcycle_b(helm_ctx *h, int l0, const cd *r, cd *z, int accumulate, const cd *v2,
             const cd *rs, const int *dm)
{
    BatchWS *W = h->bw;
    const Batch bt{W->B, dm};
    const int Lc = h->nlev - 1;
    if (l0 == 0 && h->o.precision != HELM_PREC_FP64 && !rs)
        return vcycle_mixed_b(h, r, z, accumulate, v2, dm);
    if (l0 == Lc) {
        const size_t n = h->L[Lc].n();
        if (!accumulate && !rs) {
            HCHK(launch_coarsest(h->ncoarsest, h->cinv, r, z, h->st, bt));
            return HELM_OK;
        }
        HCHK(launch_coarsest(h->ncoarsest, h->cinv, r, W->lx[Lc], h->st, bt));
        HCHK(launch_lincomb(W->lx[Lc], 0, 1, rs ? rs : W->hbuf + 2 * PSTRIDE + 1, z, n, accumulate,
                            h->st, bt, n, n));
        return HELM_OK;
    }
    const cd *rin = r;
    for (int l = l0; l < Lc; l++) {
        HCHK(launch_vc_down(h->lev(l), h->lev(l + 1), h->shift, h->o.omega, rin,
                            l == l0 ? rs : nullptr, W->lr[l + 1], h->st, bt));
        rin = W->lr[l + 1];
    }
    HCHK(launch_coarsest(h->ncoarsest, h->cinv, W->lr[Lc], W->lx[Lc], h->st, bt));
    for (int l = Lc - 1; l >= l0; l--) {
        const bool top = l == l0;
        HCHK(launch_vc_up(h->lev(l), h->lev(l + 1), h->shift, h->o.omega, top ? r : W->lr[l],
                          top ? rs : nullptr, W->lx[l + 1], top ? z : W->lx[l],
                          top ? accumulate : 0, top ? v2 : nullptr, h->zho, h->st, bt));
    }
    return HELM_OK;
}

// y = A_2h x or b - A_2h x for B coarse vectors.
int coarse_apply_b(helm_ctx *h, const cd *x, const cd *b, cd *y, const int *dm)
{
    BatchWS *W = h->bw;
    const Batch bt{W->B, dm};
    const Lev Lf = h->lev(0), Lc = h->lev(1);
    switch (h->o.coarse_op) {
    case HELM_COARSE_REDGLK2: HCHK(launch_redglk2(Lc, x, b, y, 0, h->st, bt)); break;
    case HELM_COARSE_REDGLK1: HCHK(launch_redglk2(Lc, x, b, y, 1, h->st, bt)); break;
    case HELM_COARSE_REDO4: HCHK(launch_redo4(Lc, x, b, y, h->st, bt)); break;
    case HELM_COARSE_REDO2: HCHK(launch_apply5(Lc, make_double2(1.0, 0.0), x, b, y, h->st, bt)); break;
    default: HCHK(launch_glk(Lf, Lc, h->zho, x, b, y, h->st, bt));
    }
    return HELM_OK;
}

// Lazily normalised Arnoldi step of the batched inner GMRES (as
// arnoldi_lazy_enqueue, for every active right-hand side): basis slot j1
// already holds A z; projections and the norm go to read-back slot `slot`.
// Copy every right-hand side's step scalars (projections of both passes and
// the norm) into read-back slot `slot` of the pinned buffer.
int readback_b(helm_ctx *h, int slot)
{
    BatchWS *W = h->bw;
    HCHK(hipMemcpy2DAsync(W->hpin + (size_t)slot * HB * W->B, HB * sizeof(cd), W->hbuf,
                          SB * sizeof(cd), HB * sizeof(cd), W->B, hipMemcpyDeviceToHost, h->st));
    return HELM_OK;
}

int arnoldi_lazy_b(helm_ctx *h, int j1, int slot, const int *dm, int nact)
{
    BatchWS *W = h->bw;
    const Batch bt{W->B, dm};
    const size_t n = h->L[1].n(), ld = (size_t)W->B * n;
    const int nb = krylov_blocks(n, W->B), nbu = krylov_blocks(n, W->B, KB_UPDATE);
    cd *w = W->Vc + (size_t)j1 * ld;
    cd *h1 = W->hbuf, *h2 = W->hbuf + PSTRIDE, *nr = W->hbuf + 2 * PSTRIDE;
    {
        Timed tm(h, HELM_K_DOT, 1, 16.0 * (j1 + 1) * n * nact);
        HCHK(launch_mdot(W->Vc, ld, j1, w, n, W->part, 1, nullptr, 0, h->st, bt, n, n));
    }
    HCHK(launch_reduce(W->part, nb, j1 + 1, h1, 0, nullptr, 0, W->sig, j1, nullptr, h->st, bt));
    {
        Timed tm(h, HELM_K_UPDATE, 1, 16.0 * (j1 + 2) * n * nact);
        HCHK(launch_mupdate(w, W->Vc, ld, j1, h1, n, W->partn, nullptr, 0, W->sig, h->st, bt, n,
                            n));
    }
    HCHK(launch_mdot(W->Vc, ld, j1, w, n, W->part, 0, h1, j1, h->st, bt, n, n));
    HCHK(launch_reduce(W->part, nb, j1, h2, 0, h1, j1, W->sig, j1, nullptr, h->st, bt));
    HCHK(launch_mupdate(w, W->Vc, ld, j1, h2, n, W->partn, h1, j1, W->sig, h->st, bt, n, n));
    HCHK(launch_reduce(W->partn, nbu, 1, nr, 2, nullptr, 0, nullptr, 0, W->sig + j1, h->st, bt));
    return readback_b(h, slot);
}

// Projections (both passes summed) and norm of right-hand side b from a
// read-back slot.
double read_col(BatchWS *W, int slot, int b, int j1, zc *col)
{
    const cd *hp = W->hpin + ((size_t)slot * W->B + b) * HB;
    bool reorth = false;
    for (int i = 0; i < j1; i++) {
        col[i] = zc(hp[i].x + hp[PSTRIDE + i].x, hp[i].y + hp[PSTRIDE + i].y);
        reorth |= hp[PSTRIDE + i].x != 0.0 || hp[PSTRIDE + i].y != 0.0;
    }
    if (reorth && (int)W->reo.size() > b) W->reo[b]++;
    return hp[2 * PSTRIDE].x;
}

int inner_step_b(helm_ctx *h, int j, int slot, const int *dm, int nact)
{
    BatchWS *W = h->bw;
    const size_t ld = (size_t)W->B * h->L[1].n();
    cd *z = W->Zc + (size_t)j * ld;
    RCHK(vcycle_b(h, 1, W->Vc + (size_t)j * ld, z, 0, nullptr, W->sig + j, dm));
    RCHK(coarse_apply_b(h, z, nullptr, W->Vc + (size_t)(j + 1) * ld, dm));
    return arnoldi_lazy_b(h, j + 1, slot, dm, nact);
}

// Copy an active mask into the fixed device mask the captured chunks read
// (through the rotating pinned staging of upload_mask).
int upload_gmask(helm_ctx *h, const std::vector<char> &act)
{
    BatchWS *W = h->bw;
    if (W->next_mask == NMASK) {
        HCHK(hipStreamSynchronize(h->st));
        W->next_mask = 0;
    }
    int *hm = W->hmask + (size_t)(W->next_mask++) * W->B;
    for (int b = 0; b < W->B; b++) hm[b] = act[b] ? 1 : 0;
    HCHK(hipMemcpyAsync(W->gmask, hm, W->B * sizeof(int), hipMemcpyHostToDevice, h->st));
    return HELM_OK;
}

// Inner steps j0 .. j0 + len - 1 of the batched coarse GMRES as one graph
// (captured on first use, then replayed): each step's kernels for the
// right-hand sides that W->gmask marks active, and its read-back into slot
// sbase + (step - j0).  The chunk's event is recorded after it as stream work.
// Returns HELM_EHIP with W->graph_off set when capture is not possible; the
// caller then launches the steps directly.
int chunk_b(helm_ctx *h, int j0, int len, int sbase, int par)
{
    BatchWS *W = h->bw;
    const int key = j0 * 64 + len * 2 + (sbase ? 1 : 0);
    hipGraphExec_t ex = nullptr;
    for (auto &g : W->gchunk)
        if (g.first == key) ex = g.second;
    if (!ex) {
        if (hipStreamBeginCapture(h->st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            (void)hipGetLastError();
            W->graph_off = true;
            return HELM_EHIP;
        }
        int rc = HELM_OK;
        for (int s = 0; s < len && rc == HELM_OK; s++)
            rc = inner_step_b(h, j0 + s, sbase + s, W->gmask, W->B);
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(h->st, &g);
        if (rc == HELM_OK && ec == hipSuccess && g &&
            hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess) {
            W->gchunk.push_back({key, ex});
        } else {
            (void)hipGetLastError();
            ex = nullptr;
            W->graph_off = true;
        }
        if (g) (void)hipGraphDestroy(g);
        if (!ex) return HELM_EHIP;
    }
    HCHK(hipGraphLaunch(ex, h->st));
    HCHK(hipEventRecord(W->ev[par], h->st));
    return HELM_OK;
}

// Upload per-right-hand-side least-squares solutions (y[b], zero-padded to
// jmax) into W->ydev.
int upload_y_b(helm_ctx *h, const std::vector<std::vector<zc>> &y, int jmax)
{
    BatchWS *W = h->bw;
    cd *stg = W->hpin + (size_t)NSLOT * HB * W->B;
    for (int b = 0; b < W->B; b++)
        for (int i = 0; i < jmax; i++) {
            const zc v = i < (int)y[b].size() ? y[b][i] : zc(0);
            stg[(size_t)b * SB + i] = make_double2(v.real(), v.imag());
        }
    HCHK(hipMemcpyAsync(W->ydev, stg, (size_t)W->B * SB * sizeof(cd), hipMemcpyHostToDevice,
                        h->st));
    HCHK(hipStreamSynchronize(h->st));  // the staging buffer is reused next time
    return HELM_OK;
}

// Batched coarse solve (coarse_solve for every right-hand side with
// act[b]): b, x are B contiguous coarse vectors.  Each right-hand side runs
// its own restarted GMRES; all active ones step together and those that meet
// their tolerance leave the active mask.  iters[b] receives the counts.
int coarse_solve_b(helm_ctx *h, const cd *bvec, cd *x, const std::vector<char> &act,
                   std::vector<int> &iters)
{
    BatchWS *W = h->bw;
    const int B = W->B;
    const size_t n = h->L[1].n(), ld = (size_t)B * n;
    const int m = h->mc;
    const bool fixed = h->o.coarse_mode == HELM_CMODE_FIXED;
    const int cap = h->o.coarse_iters;
    const double tol = h->o.coarse_tol;
    iters.assign(B, 0);
    std::vector<char> live(act);
    const int *dm = upload_mask(h, live);
    MCHK(dm);
    std::vector<double> bn, beta;
    RCHK(vnorm_b(h, bvec, n, bn, W->sig, dm));
    HCHK(launch_zero(x, (size_t)B * n, h->st));
    for (int b = 0; b < B; b++) {
        if (!live[b]) continue;
        if (!std::isfinite(bn[b])) return HELM_ENONFINITE;
        if (bn[b] == 0.0) live[b] = 0;
    }
    std::vector<Givens> gv(B, Givens(m));
    std::vector<std::vector<zc>> y(B);
    std::vector<int> jend(B);
    std::vector<char> stop(B), cyc(B), stepm(B);
    std::vector<zc> col(m + 1);
    bool first = true;
    for (;;) {
        if (first) {
            HCHK(hipMemcpyAsync(W->Vc, bvec, ld * sizeof(cd), hipMemcpyDeviceToDevice, h->st));
            beta = bn;  // sig[.][0] = 1/||b|| was stored by vnorm_b
        } else {
            dm = upload_mask(h, live);
            MCHK(dm);
            RCHK(coarse_apply_b(h, x, bvec, W->Vc, dm));
            RCHK(vnorm_b(h, W->Vc, n, beta, W->sig, dm));
            for (int b = 0; b < B; b++)
                if (live[b] && ((!fixed && beta[b] <= tol * bn[b]) || beta[b] == 0.0)) live[b] = 0;
        }
        int nlive = 0, itmin = cap;
        for (int b = 0; b < B; b++)
            if (live[b] && iters[b] < cap) {
                nlive++;
                itmin = std::min(itmin, iters[b]);
            } else {
                live[b] = 0;
            }
        if (nlive == 0) break;
        cyc = live;
        stepm = live;
        dm = upload_mask(h, stepm);
        MCHK(dm);
        for (int b = 0; b < B; b++) {
            stop[b] = 0;
            jend[b] = 0;
            if (!cyc[b]) continue;
            gv[b].start(beta[b]);
        }
        const int steps = std::min(m, cap - itmin);
        int nact = nlive;
        // the columns of step j (read-back slot `slot`) for every stepping
        // right-hand side; returns the number still stepping
        bool changed = false;
        auto take_step = [&](int j, int slot) {
            int nstep = 0;
            for (int b = 0; b < B; b++) {
                if (!stepm[b]) continue;
                const double hn = read_col(W, slot, b, j + 1, col.data());
                const double res = gv[b].add_column(j, col.data(), hn);
                iters[b]++;
                jend[b] = j + 1;
                if ((!fixed && res <= tol * bn[b]) || hn == 0.0 || iters[b] >= cap) {
                    stop[b] = 1;
                    stepm[b] = 0;
                    changed = true;
                } else {
                    nstep++;
                }
            }
            return nstep;
        };
        bool graphs = h->o.graphs && !W->graph_off && h->t_cls < 0;
        int rc = HELM_OK;
        if (graphs) {
            RCHK(upload_gmask(h, stepm));
            rc = chunk_b(h, 0, std::min(GCHUNK, steps), 0, 0);
            // a chunk that cannot be captured: this and later cycles launch
            // their steps directly
            if (rc != HELM_OK && W->graph_off) graphs = false;
        }
        if (graphs) {
            // chunks of GCHUNK steps replayed from graphs; chunk c + 1 is
            // queued before the host reads chunk c (its steps past a
            // convergence are not used), and a new mask reaches the chunks
            // queued after it
            for (int c0 = 0; rc == HELM_OK && c0 < steps; c0 += GCHUNK) {
                const int len = std::min(GCHUNK, steps - c0), par = (c0 / GCHUNK) & 1;
                if (c0 + GCHUNK < steps) {
                    if (changed) {
                        RCHK(upload_gmask(h, stepm));
                        changed = false;
                    }
                    rc = chunk_b(h, c0 + GCHUNK, std::min(GCHUNK, steps - c0 - GCHUNK),
                                 (par ^ 1) * GCHUNK, par ^ 1);
                    if (rc != HELM_OK) break;
                }
                HCHK(hipEventSynchronize(W->ev[par]));
                int nstep = 1;
                for (int q = 0; q < len && nstep > 0; q++) nstep = take_step(c0 + q, par * GCHUNK + q);
                if (nstep == 0) break;
            }
            if (rc != HELM_OK) return rc;
        } else {
            if (h->o.graphs) HCHK(hipStreamSynchronize(h->st));  // after a failed capture
            RCHK(inner_step_b(h, 0, 0, dm, nact));
            HCHK(hipEventRecord(W->ev[0], h->st));
            for (int j = 0; j < steps; j++) {
                if (j + 1 < steps) {
                    RCHK(inner_step_b(h, j + 1, (j + 1) & 1, dm, nact));
                    HCHK(hipEventRecord(W->ev[(j + 1) & 1], h->st));
                }
                HCHK(hipEventSynchronize(W->ev[j & 1]));
                changed = false;
                const int nstep = take_step(j, j & 1);
                if (nstep == 0) break;
                if (changed) {
                    dm = upload_mask(h, stepm);
                    MCHK(dm);
                    nact = nstep;
                }
            }
        }
        // x += sum_i y_i M^-1 v_i for every right-hand side of the cycle, from
        // the z_i its steps kept (a shorter cycle's y is padded with zeros)
        int jmax = 0;
        for (int b = 0; b < B; b++) {
            y[b].clear();
            if (!cyc[b]) continue;
            gv[b].solve(jend[b], y[b]);
            jmax = std::max(jmax, jend[b]);
        }
        RCHK(upload_y_b(h, y, jmax));
        dm = upload_mask(h, cyc);
        MCHK(dm);
        HCHK(launch_lincomb(W->Zc, ld, jmax, W->ydev, x, n, 1, h->st, Batch{B, dm}, n, n));
        for (int b = 0; b < B; b++)
            if (cyc[b] && ((fixed && stop[b]) || iters[b] >= cap)) live[b] = 0;
        first = false;
    }
    return HELM_OK;
}

// Batched A-DEF1 (or Q, P) applied to B fine vectors v -> w for act[b].
int deflate_b(helm_ctx *h, int mode, const cd *v, cd *w, const std::vector<char> &act,
              std::vector<int> &inner)
{
    BatchWS *W = h->bw;
    const Lev Lf = h->lev(0), Lc = h->lev(1);
    const int *dm = upload_mask(h, act);
    MCHK(dm);
    const Batch bt{W->B, dm};
    HCHK(launch_zt(Lf, Lc, h->zho, v, nullptr, W->v1, h->st, bt));
    {
        Phase ph(h, 0);
        RCHK(coarse_solve_b(h, W->v1, W->v2, act, inner));
    }
    dm = upload_mask(h, act);
    MCHK(dm);
    const Batch bt2{W->B, dm};
    if (mode == HELM_DEFL_Q) {
        HCHK(launch_z(Lf, Lc, h->zho, W->v2, w, h->st, bt2));
        return HELM_OK;
    }
    cd *t = mode == HELM_DEFL_P ? w : W->tf;
    HCHK(launch_dresid(Lf, Lc, h->zho, v, W->v2, t, h->st, bt2));
    if (mode == HELM_DEFL_P) return HELM_OK;
    Phase ph(h, 1);
    return vcycle_b(h, 0, W->tf, w, 0, W->v2, nullptr, dm);
}

// Arnoldi step of the batched outer FGMRES (as arnoldi_step): W->w holds
// A z_j of every right-hand side; V is [m+1][B][n].
int arnoldi_b(helm_ctx *h, int j1, const int *dm)
{
    BatchWS *W = h->bw;
    const Batch bt{W->B, dm};
    const size_t n = h->L[0].n(), ld = (size_t)W->B * n;
    const int nb = krylov_blocks(n, W->B), nbu = krylov_blocks(n, W->B, KB_UPDATE);
    cd *h1 = W->hbuf, *h2 = W->hbuf + PSTRIDE, *nr = W->hbuf + 2 * PSTRIDE;
    HCHK(launch_mdot(W->V, ld, j1, W->w, n, W->part, 1, nullptr, 0, h->st, bt, n, n));
    HCHK(launch_reduce(W->part, nb, j1 + 1, h1, 0, nullptr, 0, nullptr, 0, nullptr, h->st, bt));
    HCHK(launch_mupdate(W->w, W->V, ld, j1, h1, n, W->partn, nullptr, 0, nullptr, h->st, bt, n,
                        n));
    HCHK(launch_mdot(W->V, ld, j1, W->w, n, W->part, 0, h1, j1, h->st, bt, n, n));
    HCHK(launch_reduce(W->part, nb, j1, h2, 0, h1, j1, nullptr, 0, nullptr, h->st, bt));
    HCHK(launch_mupdate(W->w, W->V, ld, j1, h2, n, W->partn, h1, j1, nullptr, h->st, bt, n, n));
    HCHK(launch_reduce(W->partn, nbu, 1, nr, 2, nullptr, 0, nullptr, 0, nullptr, h->st, bt));
    HCHK(launch_scale(W->w, nr, W->V + (size_t)j1 * ld, n, h->st, bt, n, n));
    HCHK(hipMemcpy2DAsync(W->hpin, HB * sizeof(cd), W->hbuf, SB * sizeof(cd), HB * sizeof(cd),
                          W->B, hipMemcpyDeviceToHost, h->st));
    HCHK(hipStreamSynchronize(h->st));
    return HELM_OK;
}

// Flexible GMRES(m) for B right-hand sides of one operator in lockstep (as
// solve_one for each): b, x are [B][ny][nx].
int solve_b(helm_ctx *h, const cd *b, cd *x, int B, helm_solve_info *info)
{
    const auto t0 = std::chrono::steady_clock::now();
    RCHK(ensure_batch(h, B, true));
    BatchWS *W = h->bw;
    W->reo.assign(B, 0);
    const size_t n = h->L[0].n(), ld = (size_t)B * n;
    const int m = h->o.restart;
    const Lev L0 = h->lev(0);
    const int force = h->o.force_iters;
    const int cap = force > 0 ? force : h->o.maxit;
    std::vector<helm_solve_info> inf(B);
    HCHK(launch_mask_copy(L0, b, W->bm, h->st, B));
    std::vector<char> all(B, 1);
    const int *dm = upload_mask(h, all);
    MCHK(dm);
    std::vector<double> bn, beta;
    RCHK(vnorm_b(h, W->bm, n, bn, nullptr, dm));
    for (int q = 0; q < B; q++)
        if (!std::isfinite(bn[q])) return HELM_ENONFINITE;
    if (h->o.x0_given)
        HCHK(launch_mask_copy(L0, x, x, h->st, B));
    else
        HCHK(launch_zero(x, ld, h->st));
    std::vector<char> live(B), cyc(B), stepm(B);
    for (int q = 0; q < B; q++) {
        live[q] = bn[q] > 0.0;
        if (!live[q]) inf[q].converged = 1;
    }
    std::vector<Givens> gv(B, Givens(m));
    std::vector<std::vector<zc>> y(B);
    std::vector<int> jend(B), inner;
    std::vector<zc> col(m + 1);
    for (;;) {
        // true residual of every live right-hand side
        dm = upload_mask(h, live);
        MCHK(dm);
        HCHK(launch_apply5(L0, make_double2(1.0, 0.0), x, W->bm, W->w, h->st, Batch{B, dm}));
        RCHK(vnorm_b(h, W->w, n, beta, nullptr, dm));
        int nlive = 0;
        for (int q = 0; q < B; q++) {
            if (!live[q]) continue;
            inf[q].relres = beta[q] / bn[q];
            if (force > 0 && inf[q].outer_iters >= cap) {
                inf[q].converged = inf[q].relres <= h->o.tol;
                live[q] = 0;
            } else if (force <= 0 && inf[q].relres <= h->o.tol) {
                inf[q].converged = 1;
                live[q] = 0;
            } else if (inf[q].outer_iters >= cap || beta[q] == 0.0) {
                live[q] = 0;
            } else {
                nlive++;
            }
        }
        if (nlive == 0) break;
        cyc = live;
        stepm = live;
        dm = upload_mask(h, stepm);
        MCHK(dm);
        // v_0 = r / ||r|| (the norms sit in hbuf[2*PSTRIDE] of each right-hand side)
        HCHK(launch_scale(W->w, W->hbuf + 2 * PSTRIDE, W->V, n, h->st, Batch{B, dm}, n, n));
        for (int q = 0; q < B; q++) {
            jend[q] = 0;
            if (cyc[q]) gv[q].start(beta[q]);
        }
        for (int j = 0; j < m; j++) {
            RCHK(deflate_b(h, HELM_DEFL_ADEF1, W->V + (size_t)j * ld, W->Z + (size_t)j * ld,
                           stepm, inner));
            dm = upload_mask(h, stepm);
            MCHK(dm);
            HCHK(launch_apply5(L0, make_double2(1.0, 0.0), W->Z + (size_t)j * ld, nullptr, W->w,
                               h->st, Batch{B, dm}));
            RCHK(arnoldi_b(h, j + 1, dm));
            int nstep = 0;
            for (int q = 0; q < B; q++) {
                if (!stepm[q]) continue;
                const double hn = read_col(W, 0, q, j + 1, col.data());
                const double res = gv[q].add_column(j, col.data(), hn);
                inf[q].outer_iters++;
                inf[q].inner_iters_total += inner[q];
                inf[q].inner_iters_max = std::max(inf[q].inner_iters_max, inner[q]);
                jend[q] = j + 1;
                if ((force <= 0 && res <= h->o.tol * bn[q]) || hn == 0.0 ||
                    inf[q].outer_iters >= cap)
                    stepm[q] = 0;
                else
                    nstep++;
            }
            if (std::getenv("HELMDEFL_LOG"))
                std::fprintf(stderr, "helmdefl: batch outer step %d, %d right-hand sides active\n",
                             j + 1, nstep);
            if (nstep == 0) break;
        }
        int jmax = 0;
        for (int q = 0; q < B; q++) {
            y[q].clear();
            if (!cyc[q]) continue;
            gv[q].solve(jend[q], y[q]);
            jmax = std::max(jmax, jend[q]);
        }
        RCHK(upload_y_b(h, y, jmax));
        dm = upload_mask(h, cyc);
        MCHK(dm);
        HCHK(launch_lincomb(W->Z, ld, jmax, W->ydev, x, n, 1, h->st, Batch{B, dm}, n, n));
    }
    HCHK(hipStreamSynchronize(h->st));
    const double ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    int rc = HELM_OK;
    for (int q = 0; q < B; q++) {
        inf[q].t_solve_ms = ms;
        if (!inf[q].converged && force <= 0) rc = HELM_ENOCONV;
        inf[q].reorth_steps = W->reo[q];
        if (info) info[q] = inf[q];
    }
    return rc;
}

// ---------------------------------------------------------------------------
// setup
// ---------------------------------------------------------------------------

// Dense inverse of M on the coarsest level (Gauss-Jordan, partial pivoting).
// Non-unknown nodes get zero rows and columns, so they read and write 0.
int setup_coarsest(helm_ctx *h, const std::vector<std::vector<double>> &khost)
{
    const int l = h->nlev - 1;
    const int nx = h->L[l].nx, ny = h->L[l].ny, n = nx * ny;
    if (n > MAX_COARSEST) return HELM_EGRID;
    Lev Lv = make_lev(nx, ny, h->L[l].hx, h->L[l].hy, h->g.bc,
                      khost[l].empty() ? nullptr : khost[l].data(), h->kconst);
    std::vector<zc> A((size_t)n * n, zc(0)), B((size_t)n * n, zc(0));
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            const int p = j * nx + i;
            B[(size_t)p * n + p] = 1.0;
            cd ap;
            double aw, ae, as, an;
            if (!coef5(Lv, h->shift, i, j, ap, aw, ae, as, an)) {
                A[(size_t)p * n + p] = 1.0;
                continue;
            }
            A[(size_t)p * n + p] = zc(ap.x, ap.y);
            if (aw != 0.0) A[(size_t)p * n + p - 1] += aw;
            if (ae != 0.0) A[(size_t)p * n + p + 1] += ae;
            if (as != 0.0) A[(size_t)p * n + p - nx] += as;
            if (an != 0.0) A[(size_t)p * n + p + nx] += an;
        }
    for (int c = 0; c < n; c++) {
        int piv = c;
        double best = std::abs(A[(size_t)c * n + c]);
        for (int r = c + 1; r < n; r++)
            if (std::abs(A[(size_t)r * n + c]) > best) {
                best = std::abs(A[(size_t)r * n + c]);
                piv = r;
            }
        if (best == 0.0) return HELM_EGRID;  // singular coarsest operator
        if (piv != c)
            for (int q = 0; q < n; q++) {
                std::swap(A[(size_t)c * n + q], A[(size_t)piv * n + q]);
                std::swap(B[(size_t)c * n + q], B[(size_t)piv * n + q]);
            }
        const zc d = 1.0 / A[(size_t)c * n + c];
        for (int q = 0; q < n; q++) {
            A[(size_t)c * n + q] *= d;
            B[(size_t)c * n + q] *= d;
        }
        for (int r = 0; r < n; r++) {
            if (r == c) continue;
            const zc f = A[(size_t)r * n + c];
            if (f == 0.0) continue;
            for (int q = 0; q < n; q++) {
                A[(size_t)r * n + q] -= f * A[(size_t)c * n + q];
                B[(size_t)r * n + q] -= f * B[(size_t)c * n + q];
            }
        }
    }
    std::vector<cd> inv((size_t)n * n);
    for (int r = 0; r < n; r++)
        for (int c = 0; c < n; c++) {
            const bool keep = unknown(Lv, r % nx, r / nx) && unknown(Lv, c % nx, c / nx);
            const zc v = keep ? B[(size_t)r * n + c] : zc(0);
            inv[(size_t)r * n + c] = make_double2(v.real(), v.imag());
        }
    RCHK(dalloc(&h->cinv, (size_t)n * n));
    HCHK(hipMemcpy(h->cinv, inv.data(), inv.size() * sizeof(cd), hipMemcpyHostToDevice));
    if (h->o.precision != HELM_PREC_FP64) {
        std::vector<cf> invf(inv.size());
        for (size_t q = 0; q < inv.size(); q++)
            invf[q] = make_float2((float)inv[q].x, (float)inv[q].y);
        RCHK(dalloc(&h->cinvf, invf.size()));
        HCHK(hipMemcpy(h->cinvf, invf.data(), invf.size() * sizeof(cf), hipMemcpyHostToDevice));
    }
    h->ncoarsest = n;
    return HELM_OK;
}

void release(helm_ctx *h)
{
    if (!h) return;
    for (auto *gs : {&h->gstep, &h->gstep2}) {
        for (hipGraphExec_t &e : *gs)
            if (e) (void)hipGraphExecDestroy(e);
        gs->clear();
    }
    if (h->st) (void)hipStreamSynchronize(h->st);
    for (int l = 0; l < h->nlev; l++) {
        dfree(h->L[l].kdev);
        dfree(h->L[l].r);
        dfree(h->L[l].x);
        dfree(h->L[l].rf);
        dfree(h->L[l].xf);
    }
    dfree(h->cinv);
    dfree(h->cinvf);
    dfree(h->v1);
    dfree(h->v2);
    dfree(h->tf);
    dfree(h->Vc);
    dfree(h->Zc);
    dfree(h->xin);
    dfree(h->Vc32);
    dfree(h->wtmp);
    dfree(h->part);
    dfree(h->partn);
    dfree(h->hbuf);
    dfree(h->ydev);
    dfree(h->V);
    dfree(h->Z);
    dfree(h->w);
    dfree(h->bm);
    dfree(h->w2);
    dfree(h->r);
    if (h->hpin) (void)hipHostFree(h->hpin);
    if (h->hpub) (void)hipHostFree(h->hpub);
    dfree(h->sig);
    for (auto e : h->ev_slot)
        if (e) (void)hipEventDestroy(e);
    if (h->ev_y) (void)hipEventDestroy(h->ev_y);
    for (auto &p : h->pend) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : h->ev_free) (void)hipEventDestroy(e);
    for (auto e : h->ph_free) (void)hipEventDestroy(e);
    for (auto &v : h->ph_pend)
        for (auto &p : v) {
            (void)hipEventDestroy(p.first);
            (void)hipEventDestroy(p.second);
        }
    free_batch(h->bw);
    dfree(h->adjb);
    delete h;
}

int create_impl(const helm_grid *g, const double *k_dev, double k_const, const helm_opts *opts,
                void *stream, helm_ctx **out)
{
    if (!g || !out) return HELM_EINVAL;
    *out = nullptr;
    if (!(g->hx > 0) || !(g->hy > 0) || !std::isfinite(g->hx) || !std::isfinite(g->hy))
        return HELM_EINVAL;
    if (g->bc != HELM_BC_DIRICHLET && g->bc != HELM_BC_SOMMERFELD) return HELM_EINVAL;
    if (!coarsenable(g->nx, g->ny)) return HELM_EGRID;
    helm_opts o;
    helm_opts_default(&o);
    if (opts) o = *opts;
    if (o.nu_pre != 1 || o.nu_post != 1) return HELM_EINVAL;
    if (!(o.omega > 0) || !std::isfinite(o.beta_re) || !std::isfinite(o.beta_im)) return HELM_EINVAL;
    if (o.defl_vectors != HELM_Z_LINEAR && o.defl_vectors != HELM_Z_HIGH) return HELM_EINVAL;
    if (o.coarse_op < HELM_COARSE_GALERKIN || o.coarse_op > HELM_COARSE_REDGLK1)
        return HELM_EINVAL;
    if ((o.coarse_op == HELM_COARSE_REDGLK2 || o.coarse_op == HELM_COARSE_REDGLK1) &&
        g->hx != g->hy)
        return HELM_EINVAL;
    if (o.outer < HELM_OUTER_FGMRES || o.outer > HELM_OUTER_GMRES_LEFT) return HELM_EINVAL;
    if (o.batch != 0 && o.batch != 1) return HELM_EINVAL;
    if (o.graphs != 0 && o.graphs != 1) return HELM_EINVAL;
    if (o.vc_tail < 0) return HELM_EINVAL;
    if (o.coarse_mode != HELM_CMODE_FIXED && o.coarse_mode != HELM_CMODE_TOL) return HELM_EINVAL;
    if (o.coarse_iters < 1 || o.coarse_restart < 1 || o.coarse_restart > MAX_RESTART)
        return HELM_EINVAL;
    if (o.restart < 1 || o.restart > MAX_RESTART || o.maxit < 1) return HELM_EINVAL;
    if (!(o.tol >= 0) || !(o.coarse_tol >= 0)) return HELM_EINVAL;
    if (o.coarsest_nodes < 0 || o.coarsest_nodes > MAX_COARSEST) return HELM_EINVAL;
    if (o.precision != HELM_PREC_FP64 && o.precision != HELM_PREC_MIXED &&
        o.precision != HELM_PREC_MIXED_C64BASIS)
        return HELM_EINVAL;
    if (!k_dev && (!std::isfinite(k_const) || k_const < 0)) return HELM_ENONFINITE;
    const auto t_start = std::chrono::steady_clock::now();

    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return HELM_EHIP;
    RCHK(scratch_init(dev));
    helm_ctx *h = new (std::nothrow) helm_ctx();
    if (!h) return HELM_ENOMEM;
    h->dev = dev;
    h->g = *g;
    h->o = o;
    h->st = (hipStream_t)stream;
    h->kconst = k_const;
    h->shift = make_double2(o.beta_re, o.beta_im);
    h->zho = o.defl_vectors == HELM_Z_HIGH;
    int rc = HELM_OK;

    // level dims
    int nx = g->nx, ny = g->ny;
    double hx = g->hx, hy = g->hy;
    h->nlev = 0;
    for (;;) {
        LevelH &q = h->L[h->nlev++];
        q.nx = nx;
        q.ny = ny;
        q.hx = hx;
        q.hy = hy;
        if (!coarsenable(nx, ny) || h->nlev == MAXLEV) break;
        if (h->nlev > 1 && (long)nx * (long)ny <= (long)o.coarsest_nodes) break;
        nx = (nx + 1) / 2;
        ny = (ny + 1) / 2;
        hx *= 2;
        hy *= 2;
    }
    // wavenumber per level: copy, validate, inject
    std::vector<std::vector<double>> kh(h->nlev);
    if (k_dev) {
        kh[0].resize(h->L[0].n());
        if (hipMemcpy(kh[0].data(), k_dev, kh[0].size() * sizeof(double), hipMemcpyDeviceToHost) !=
            hipSuccess) {
            release(h);
            return HELM_EHIP;
        }
        for (double v : kh[0])
            if (!std::isfinite(v) || v < 0) {
                release(h);
                return HELM_ENONFINITE;
            }
        for (int l = 1; l < h->nlev; l++) {
            kh[l].resize(h->L[l].n());
            const int fnx = h->L[l - 1].nx;
            for (int j = 0; j < h->L[l].ny; j++)
                for (int i = 0; i < h->L[l].nx; i++)
                    kh[l][(size_t)j * h->L[l].nx + i] = kh[l - 1][(size_t)(2 * j) * fnx + 2 * i];
        }
        for (int l = 0; l < h->nlev && !rc; l++) {
            rc = dalloc(&h->L[l].kdev, h->L[l].n());
            if (!rc && hipMemcpy(h->L[l].kdev, kh[l].data(), kh[l].size() * sizeof(double),
                                 hipMemcpyHostToDevice) != hipSuccess)
                rc = HELM_EHIP;
        }
    }
    // V-cycle buffers on levels >= 1
    for (int l = 1; l < h->nlev && !rc; l++) {
        rc = dalloc(&h->L[l].r, h->L[l].n());
        if (!rc) rc = dalloc(&h->L[l].x, h->L[l].n());
        if (!rc && o.precision != HELM_PREC_FP64) rc = dalloc(&h->L[l].rf, h->L[l].n());
        if (!rc && o.precision != HELM_PREC_FP64) rc = dalloc(&h->L[l].xf, h->L[l].n());
    }
    if (!rc) rc = setup_coarsest(h, kh);
    // deflation and inner-GMRES workspace
    const size_t nf = h->L[0].n(), nc = h->L[1].n();
    h->mc = o.coarse_restart;
    if (!rc) rc = dalloc(&h->v1, nc);
    if (!rc) rc = dalloc(&h->v2, nc);
    if (!rc) rc = dalloc(&h->tf, nf);
    if (!rc) rc = dalloc(&h->Vc, (size_t)(h->mc + 1) * nc);
    if (!rc) rc = dalloc(&h->Zc, (size_t)h->mc * nc);
    if (!rc) rc = dalloc(&h->xin, nc);
    // with HELM_PREC_MIXED_C64BASIS the inner basis is complex64 (when the
    // inner V-cycle has a level below level 1)
    h->basis32 = o.precision == HELM_PREC_MIXED_C64BASIS && h->nlev > 2;
    if (!rc && h->basis32) rc = dalloc(&h->Vc32, (size_t)(h->mc + 1) * nc);
    if (!rc && h->basis32) rc = dalloc(&h->wtmp, nc);
    h->part_blocks = krylov_blocks_max(nf);
    if (!rc) rc = dalloc(&h->part, (size_t)h->part_blocks * PSTRIDE);
    if (!rc) rc = dalloc(&h->partn, (size_t)h->part_blocks * PSTRIDE);
    if (!rc) rc = dalloc(&h->hbuf, (size_t)HBUF);
    if (!rc) rc = dalloc(&h->ydev, (size_t)PSTRIDE);
    if (!rc) rc = dalloc(&h->sig, (size_t)PSTRIDE);
    if (!rc && hipHostMalloc((void **)&h->hpin, PIN_TOTAL * sizeof(cd)) != hipSuccess) {
        h->hpin = nullptr;
        rc = HELM_ENOMEM;
    }
    if (!rc && hipHostMalloc((void **)&h->hpub, 2 * HBUF * sizeof(cd),
                             hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
        h->hpub = nullptr;
        rc = HELM_ENOMEM;
    }
    if (!rc && hipHostGetDevicePointer((void **)&h->hpub_dev, h->hpub, 0) != hipSuccess) {
        h->hpub_dev = nullptr;
        rc = HELM_EHIP;
    }
    for (int q = 0; q < 2 && !rc; q++)
        if (hipEventCreateWithFlags(&h->ev_slot[q], hipEventDisableTiming) != hipSuccess) {
            h->ev_slot[q] = nullptr;
            rc = HELM_EHIP;
        }
    if (!rc && hipEventCreateWithFlags(&h->ev_y, hipEventDisableTiming) != hipSuccess) {
        h->ev_y = nullptr;
        rc = HELM_EHIP;
    }
    // record it once, so that the first upload's wait has an event to wait on
    if (!rc && hipEventRecord(h->ev_y, h->st) != hipSuccess) rc = HELM_EHIP;
    if (!rc) {
        // slot 2*PSTRIDE+1 holds the constant 1 used to accumulate on the
        // coarsest level
        cd one = make_double2(1.0, 0.0);
        if (hipMemcpy(h->hbuf + 2 * PSTRIDE + 1, &one, sizeof(cd), hipMemcpyHostToDevice) !=
            hipSuccess)
            rc = HELM_EHIP;
    }
    if (!rc && hipStreamSynchronize(h->st) != hipSuccess) rc = HELM_EHIP;
    if (rc) {
        release(h);
        return rc;
    }
    h->t_setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() -
                                                              t_start)
                        .count();
    *out = h;
    return HELM_OK;
}

bool valid(helm_ctx *h) { return h != nullptr; }

// The handle's V-cycle level buffers pointed into the fixed scratch for the
// length of one call (restored, with kernel timing, on scope exit).
struct ScratchLevels {
    helm_ctx *h;
    cd *r[MAXLEV] = {}, *x[MAXLEV] = {};
    cf *rf[MAXLEV] = {}, *xf[MAXLEV] = {};
    int t_cls;
    explicit ScratchLevels(helm_ctx *h_) : h(h_), t_cls(h_->t_cls)
    {
        for (int l = 0; l < h->nlev; l++) {
            r[l] = h->L[l].r;
            x[l] = h->L[l].x;
            rf[l] = h->L[l].rf;
            xf[l] = h->L[l].xf;
        }
    }
    // Lay levels 1..nlev-1 out in `base` (16-node aligned); false if they do
    // not fit in NOALLOC_SCRATCH_BYTES.
    bool place(char *base)
    {
        const bool fp32 = h->o.precision != HELM_PREC_FP64;
        const size_t node = fp32 ? sizeof(cf) : sizeof(cd);
        size_t off = 0;
        for (int l = 1; l < h->nlev; l++) {
            const size_t b = ((h->L[l].n() * node + 255) / 256) * 256;
            if (off + 2 * b > NOALLOC_SCRATCH_BYTES) return false;
            if (fp32) {
                h->L[l].rf = (cf *)(base + off);
                h->L[l].xf = (cf *)(base + off + b);
            } else {
                h->L[l].r = (cd *)(base + off);
                h->L[l].x = (cd *)(base + off + b);
            }
            off += 2 * b;
        }
        h->t_cls = -1;  // no timing events are created inside the call
        return true;
    }
    ~ScratchLevels()
    {
        for (int l = 0; l < h->nlev; l++) {
            h->L[l].r = r[l];
            h->L[l].x = x[l];
            h->L[l].rf = rf[l];
            h->L[l].xf = xf[l];
        }
        h->t_cls = t_cls;
    }
};

}  // namespace

// ===========================================================================
// C-ABI
// ===========================================================================
extern "C" {

int helm_opts_default(helm_opts *o)
{
    if (!o) return HELM_EINVAL;
    o->beta_re = 1.0;
    o->beta_im = 0.5;
    o->omega = 0.8;
    o->nu_pre = 1;
    o->nu_post = 1;
    o->defl_vectors = HELM_Z_HIGH;
    o->coarse_op = HELM_COARSE_GALERKIN;
    o->coarse_mode = HELM_CMODE_TOL;
    o->coarse_iters = 300;
    o->coarse_restart = 30;
    o->coarse_tol = 1e-1;
    o->restart = 50;
    o->maxit = 1000;
    o->tol = 1e-6;
    o->x0_given = 0;
    o->force_iters = 0;
    o->coarsest_nodes = 1089;
    o->precision = HELM_PREC_FP64;
    o->outer = HELM_OUTER_FGMRES;
    o->batch = 1;
    o->graphs = 0;
    o->vc_tail = 300000;
    return HELM_OK;
}

int helm_create(const helm_grid *g, const double *k_dev, double k_const, const helm_opts *opts,
                void *stream, helm_ctx **out)
{
    try {
        return create_impl(g, k_dev, k_const, opts, stream, out);
    } catch (...) {
        return HELM_ENOMEM;
    }
}

int helm_destroy(helm_ctx *h)
{
    if (!h) return HELM_EINVAL;
    release(h);
    return HELM_OK;
}

int helm_apply(helm_ctx *h, const void *x, void *y, int nrhs)
{
    if (!valid(h) || !x || !y || nrhs < 1) return HELM_EINVAL;
    if (nrhs > 1) {
        // one launch for all right-hand sides
        HCHK(launch_apply5(h->lev(0), make_double2(1.0, 0.0), (const cd *)x, nullptr, (cd *)y,
                           h->st, Batch{nrhs, nullptr}));
        return HELM_OK;
    }
    return apply_A(h, 0, (const cd *)x, nullptr, (cd *)y);
}

// Several right-hand sides go through the batched kernels when the option
// asks for it (FP64, or the complex64 fine-grid V-cycle of HELM_PREC_MIXED).
static bool batched(const helm_ctx *h, int nrhs)
{
    return nrhs > 1 && h->o.batch && h->o.precision != HELM_PREC_MIXED_C64BASIS;
}

int cslp_vcycle(helm_ctx *h, const void *r, void *z, int nrhs)
{
    if (!valid(h) || !r || !z || nrhs < 1) return HELM_EINVAL;
    const size_t n = h->L[0].n();
    try {
        if (batched(h, nrhs)) {
            RCHK(ensure_batch(h, nrhs, false));
            return vcycle_b(h, 0, (const cd *)r, (cd *)z, 0, nullptr, nullptr, nullptr);
        }
        for (int q = 0; q < nrhs; q++)
            RCHK(vcycle(h, 0, (const cd *)r + q * n, (cd *)z + q * n, 0, nullptr));
    } catch (...) {
        return HELM_ENOMEM;
    }
    return HELM_OK;
}

int cslp_vcycle_noalloc(helm_ctx *h, const void *r, void *z, int nrhs)
{
    if (!valid(h) || !r || !z || nrhs < 1) return HELM_EINVAL;
    if (h->dev < 0 || h->dev >= MAX_DEVICES || !g_scratch_dev[h->dev]) return HELM_EHIP;
    ScratchLevels sl(h);
    if (!sl.place((char *)g_scratch_dev[h->dev])) return HELM_ESCRATCH;
    const size_t n = h->L[0].n();
    for (int q = 0; q < nrhs; q++)
        RCHK(vcycle(h, 0, (const cd *)r + q * n, (cd *)z + q * n, 0, nullptr));
    return HELM_OK;
}

int deflate_apply(helm_ctx *h, int mode, const void *v, void *w, int nrhs)
{
    if (!valid(h) || !v || !w || nrhs < 1) return HELM_EINVAL;
    if (mode != HELM_DEFL_Q && mode != HELM_DEFL_P && mode != HELM_DEFL_ADEF1) return HELM_EINVAL;
    const size_t n = h->L[0].n();
    try {
        if (batched(h, nrhs)) {
            RCHK(ensure_batch(h, nrhs, false));
            std::vector<char> all(nrhs, 1);
            std::vector<int> inner;
            return deflate_b(h, mode, (const cd *)v, (cd *)w, all, inner);
        }
        for (int q = 0; q < nrhs; q++)
            RCHK(deflate_one(h, mode, (const cd *)v + q * n, (cd *)w + q * n, nullptr));
    } catch (...) {
        return HELM_ENOMEM;
    }
    return HELM_OK;
}

// The phase times of a solve (or of a batched solve, shared by its right-hand
// sides) into info[0..cnt).
static void set_phases(helm_ctx *h, helm_solve_info *info, int cnt)
{
    double tc = 0, tv = 0;
    phase_end(h, &tc, &tv);
    if (!info) return;
    for (int q = 0; q < cnt; q++) {
        info[q].t_setup_ms = h->t_setup_ms;
        info[q].t_coarse_ms = tc;
        info[q].t_vcycle_ms = tv;
    }
}

static int solve_dispatch(helm_ctx *h, const void *b, void *x, int nrhs, helm_solve_info *info)
{
    const size_t n = h->L[0].n();
    int worst = HELM_OK;
    try {
        if (batched(h, nrhs) && h->o.outer == HELM_OUTER_FGMRES) {
            phase_begin(h);
            const int rc = solve_b(h, (const cd *)b, (cd *)x, nrhs, info);
            set_phases(h, info, nrhs);
            return rc;
        }
        RCHK(ensure_outer(h));
        for (int q = 0; q < nrhs; q++) {
            const cd *bq = (const cd *)b + q * n;
            cd *xq = (cd *)x + q * n;
            helm_solve_info *iq = info ? info + q : nullptr;
            phase_begin(h);
            const long long r0 = h->n_reorth;
            const int rc = h->o.outer == HELM_OUTER_GCR         ? solve_gcr(h, bq, xq, iq)
                           : h->o.outer == HELM_OUTER_GMRES_LEFT ? solve_left(h, bq, xq, iq)
                                                                 : solve_one(h, bq, xq, iq);
            set_phases(h, iq, 1);
            if (iq) iq->reorth_steps = (int)(h->n_reorth - r0);
            if (rc != HELM_OK && rc != HELM_ENOCONV) return rc;
            if (rc == HELM_ENOCONV) worst = rc;
        }
    } catch (...) {
        h->ph_on = false;
        return HELM_ENOMEM;
    }
    return worst;
}

int helm_solve(helm_ctx *h, const void *b, void *x, int nrhs, helm_solve_info *info)
{
    if (!valid(h) || !b || !x || nrhs < 1) return HELM_EINVAL;
    return solve_dispatch(h, b, x, nrhs, info);
}

int helm_adjoint_solve(helm_ctx *h, const void *f, void *lambda, int nrhs, helm_solve_info *info)
{
    if (!valid(h) || !f || !lambda || nrhs < 1) return HELM_EINVAL;
    const size_t n = h->L[0].n(), need = (size_t)nrhs * n;
    if (h->adjb_n < need) {
        HCHK(hipStreamSynchronize(h->st));
        dfree(h->adjb);
        h->adjb = nullptr;
        h->adjb_n = 0;
        RCHK(dalloc(&h->adjb, need));
        h->adjb_n = need;
    }
    const Lev L0 = h->lev(0);
    HCHK(launch_adj_map(L0, (const cd *)f, h->adjb, 0, nrhs, h->st));
    const int x0 = h->o.x0_given;
    h->o.x0_given = 0;
    const int rc = solve_dispatch(h, h->adjb, lambda, nrhs, info);
    h->o.x0_given = x0;
    if (rc != HELM_OK && rc != HELM_ENOCONV) return rc;
    HCHK(launch_adj_map(L0, (const cd *)lambda, (cd *)lambda, 1, nrhs, h->st));
    HCHK(hipStreamSynchronize(h->st));
    return rc;
}

int helm_gradient_s(helm_ctx *h, double omega, const void *u, const void *lambda, int nrhs,
                    double *g)
{
    if (!valid(h) || !u || !lambda || !g || nrhs < 1) return HELM_EINVAL;
    if (!(omega > 0) || !std::isfinite(omega)) return HELM_EINVAL;
    HCHK(launch_grad_s(h->lev(0), omega, (const cd *)u, (const cd *)lambda, nrhs, g, h->st));
    return HELM_OK;
}

int helm_receivers(helm_ctx *h, const int *rec, int nrec, const void *u, const void *d, int nrhs,
                   void *res, void *f, double *J)
{
    if (!valid(h) || !rec || !u || !d || !res || !f || !J || nrhs < 1 || nrec < 1)
        return HELM_EINVAL;
    const size_t n = h->L[0].n();
    // receiver nodes: inside the grid and distinct (f = R^T res is a scatter)
    std::vector<int> hr(nrec);
    HCHK(hipMemcpyAsync(hr.data(), rec, nrec * sizeof(int), hipMemcpyDeviceToHost, h->st));
    HCHK(hipStreamSynchronize(h->st));
    for (int v : hr)
        if (v < 0 || (size_t)v >= n) return HELM_EINVAL;
    std::sort(hr.begin(), hr.end());
    if (std::adjacent_find(hr.begin(), hr.end()) != hr.end()) return HELM_EINVAL;
    HCHK(launch_zero((cd *)f, (size_t)nrhs * n, h->st));
    HCHK(launch_receivers(rec, nrec, (const cd *)u, (const cd *)d, n, nrhs, (cd *)res, (cd *)f, J,
                          h->st));
    return HELM_OK;
}

const char *helm_strerror(int code)
{
    switch (code) {
    case HELM_OK: return "success";
    case HELM_EINVAL: return "invalid argument";
    case HELM_EGRID: return "grid cannot be coarsened (need odd nx, ny >= 5)";
    case HELM_ENONFINITE: return "non-finite value in k or right-hand side";
    case HELM_ENOMEM: return "out of memory";
    case HELM_EHIP: return "HIP runtime error";
    case HELM_ENOCONV: return "no convergence within maxit";
    case HELM_ESCRATCH:
        return "the V-cycle levels exceed the fixed 64 MiB scratch of cslp_vcycle_noalloc";
    default: return "unknown error";
    }
}

int helm_coarse_dims(helm_ctx *h, int *nxc, int *nyc)
{
    if (!valid(h) || !nxc || !nyc) return HELM_EINVAL;
    *nxc = h->L[1].nx;
    *nyc = h->L[1].ny;
    return HELM_OK;
}

int helm_num_levels(helm_ctx *h, int *nlev)
{
    if (!valid(h) || !nlev) return HELM_EINVAL;
    *nlev = h->nlev;
    return HELM_OK;
}

int helm_level_dims(helm_ctx *h, int l, int *nx, int *ny)
{
    if (!valid(h) || !nx || !ny || l < 0 || l >= h->nlev) return HELM_EINVAL;
    *nx = h->L[l].nx;
    *ny = h->L[l].ny;
    return HELM_OK;
}

int helm_z_restrict(helm_ctx *h, const void *vf, void *vc)
{
    if (!valid(h) || !vf || !vc) return HELM_EINVAL;
    HCHK(launch_zt(h->lev(0), h->lev(1), h->zho, (const cd *)vf, nullptr, (cd *)vc, h->st));
    return HELM_OK;
}

int helm_z_prolong(helm_ctx *h, const void *vc, void *vf)
{
    if (!valid(h) || !vf || !vc) return HELM_EINVAL;
    HCHK(launch_z(h->lev(0), h->lev(1), h->zho, (const cd *)vc, (cd *)vf, h->st));
    return HELM_OK;
}

int helm_coarse_apply(helm_ctx *h, const void *x, void *y)
{
    if (!valid(h) || !x || !y) return HELM_EINVAL;
    return coarse_apply(h, (const cd *)x, nullptr, (cd *)y);
}

int helm_coarse_solve(helm_ctx *h, const void *v1, void *v2, int *iters)
{
    if (!valid(h) || !v1 || !v2) return HELM_EINVAL;
    try {
        RCHK(coarse_solve(h, (const cd *)v1, (cd *)v2, iters));
    } catch (...) {
        return HELM_ENOMEM;
    }
    HCHK(hipStreamSynchronize(h->st));
    return HELM_OK;
}

int helm_timing_enable(helm_ctx *h, int kclass, int level)
{
    if (!valid(h) || kclass >= HELM_K_NCLASSES) return HELM_EINVAL;
    RCHK(timing_flush(h));
    h->t_cls = kclass < 0 ? -1 : kclass;
    h->t_lev = level;
    h->t_count = 0;
    h->t_ms = 0;
    h->t_bytes = 0;
    return HELM_OK;
}

int helm_timing_read(helm_ctx *h, long long *launches, double *total_ms, double *alg_bytes)
{
    if (!valid(h)) return HELM_EINVAL;
    RCHK(timing_flush(h));
    if (launches) *launches = h->t_count;
    if (total_ms) *total_ms = h->t_ms;
    if (alg_bytes) *alg_bytes = h->t_bytes;
    return HELM_OK;
}

}  // extern "C"
