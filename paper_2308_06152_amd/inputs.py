"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only builds input data (grids, wavenumber fields, right-hand sides,
random vectors).  It holds none of the solver's arithmetic, and it imports
neither the HIP binding nor the CPU oracle, so both sides can be fed the same
arrays.

Workloads follow the paper's model problems (Section 2): the unit square with a
constant wavenumber and a point source at the centre, with Dirichlet (MP-2a) or
first-order Sommerfeld (MP-2b) boundaries.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED = 230806152

BC_DIRICHLET, BC_SOMMERFELD = 0, 1
COARSE_GALERKIN, COARSE_REDGLK2 = 0, 1


@dataclasses.dataclass(frozen=True)
class Workload:
    """One problem instance: grid, wavenumber, boundary, source and method options."""
    name: str
    nx: int
    ny: int
    hx: float
    hy: float
    bc: int
    kconst: float
    source: str              # "point" or "gauss"
    coarse_op: int
    restart: int = 50
    tol: float = 1e-6
    coarse_restart: int = 30
    coarse_tol: float = 1e-1
    coarse_maxit: int = 300
    model: str = "const"     # "const" (k = kconst), "wedge" or "layered" (k from a velocity model)
    freq: float = 0.0        # frequency in Hz for a velocity model
    nsrc: int = 1            # sources of a multi-source workload

    @property
    def npts(self) -> int:
        return self.nx * self.ny

    def kfield(self):
        """The wavenumber field [ny][nx] (None for a constant k)."""
        if self.model == "wedge":
            return 2.0 * math.pi * self.freq / wedge_velocity(self.nx, self.ny, self.hx, self.hy)
        if self.model == "layered":
            return 2.0 * math.pi * self.freq / layered_velocity(self.nx, self.ny, self.hx)
        return None

    def sources(self) -> np.ndarray:
        """All right-hand sides of a multi-source workload, [nsrc][ny][nx]."""
        if self.model != "layered":
            return self.rhs()[None]
        return layered_sources(self.nx, self.ny, self.hx, self.nsrc)

    def rhs(self) -> np.ndarray:
        if self.model == "wedge":
            # source at (300 m, 0 m): the middle of the top edge
            return point_source(self.nx, self.ny, self.hx, self.hy, (self.nx - 1) // 2,
                                self.ny - 1)
        ic, jc = (self.nx - 1) // 2, (self.ny - 1) // 2
        if self.source == "point":
            return point_source(self.nx, self.ny, self.hx, self.hy, ic, jc)
        return gaussian_source(self.nx, self.ny, self.hx, self.hy, ic, jc, 2.0 * self.hx)


def unit_square(n: int) -> tuple[int, int, float, float]:
    """n x n vertex grid on [0,1]^2 including the boundary; h = 1/(n-1)."""
    h = 1.0 / (n - 1)
    return n, n, h, h


def point_source(nx: int, ny: int, hx: float, hy: float, i: int, j: int) -> np.ndarray:
    """Discrete unit point source: 1/(hx*hy) at node (i, j), so that the source
    integrates to one over the cell (the delta of the model problems)."""
    b = np.zeros((ny, nx), np.complex128)
    b[j, i] = 1.0 / (hx * hy)
    return b


def gaussian_source(nx: int, ny: int, hx: float, hy: float, i: int, j: int,
                    sigma: float) -> np.ndarray:
    """Gaussian-smoothed point source of width sigma centred on node (i, j):
    exp(-r^2 / 2 sigma^2) / (2 pi sigma^2) on nodes with r <= 8 sigma, zero
    elsewhere, renormalised so that sum(b) * hx * hy = 1."""
    b = np.zeros((ny, nx), np.complex128)
    ri = int(math.ceil(8 * sigma / hx))
    rj = int(math.ceil(8 * sigma / hy))
    i0, i1 = max(0, i - ri), min(nx - 1, i + ri)
    j0, j1 = max(0, j - rj), min(ny - 1, j + rj)
    xs = (np.arange(i0, i1 + 1) - i) * hx
    ys = (np.arange(j0, j1 + 1) - j) * hy
    r2 = ys[:, None] ** 2 + xs[None, :] ** 2
    g = np.exp(-r2 / (2 * sigma * sigma)) / (2 * math.pi * sigma * sigma)
    g[r2 > (8 * sigma) ** 2] = 0.0
    g /= g.sum() * hx * hy
    b[j0:j1 + 1, i0:i1 + 1] = g
    return b


def random_complex(shape, seed: int = SEED) -> np.ndarray:
    """Standard complex normal entries (real and imaginary parts N(0,1))."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def random_field(ny: int, nx: int, lo: float, hi: float, seed: int = SEED) -> np.ndarray:
    """Smoothly varying positive field in [lo, hi] (a sum of a few seeded
    Gaussian bumps on a linear trend), used as a variable wavenumber."""
    rng = np.random.default_rng(seed)
    y, x = np.meshgrid(np.linspace(0, 1, ny), np.linspace(0, 1, nx), indexing="ij")
    f = 0.5 + 0.3 * (x - 0.5) + 0.2 * (y - 0.5)
    for _ in range(3):
        cx, cy = rng.uniform(0.2, 0.8, 2)
        s = rng.uniform(0.08, 0.2)
        f += rng.uniform(-0.3, 0.3) * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2 * s * s))
    f = (f - f.min()) / (f.max() - f.min())
    return lo + (hi - lo) * f


# The two plain-method workloads.  The small one is the oracle-sized case
# (MP-2a, Dirichlet, 129^2, k = 20, Galerkin coarse operator); the large one is
# the throughput case (MP-2b-like, Sommerfeld, 4097^2, k = 800, re-discretised
# higher-order coarse operator ReD-Glk2, Gaussian source of width 2h).
def small_plain() -> Workload:
    nx, ny, hx, hy = unit_square(129)
    return Workload("mp2a_129_k20_galerkin", nx, ny, hx, hy, BC_DIRICHLET, 20.0, "point",
                    COARSE_GALERKIN)


def large_plain() -> Workload:
    # inner GMRES restart 15: the fastest at a coarse tolerance of 0.1 on this
    # problem (restart 10..30 all converge in 10 outer iterations)
    nx, ny, hx, hy = unit_square(4097)
    return Workload("mp2b_4097_k800_redglk2", nx, ny, hx, hy, BC_SOMMERFELD, 800.0, "gauss",
                    COARSE_REDGLK2, coarse_restart=15)


def scaled_plain(n: int, k: float, bc: int = BC_SOMMERFELD,
                 coarse_op: int = COARSE_REDGLK2, source: str = "gauss") -> Workload:
    """A plain-method workload on an n x n unit-square grid."""
    nx, ny, hx, hy = unit_square(n)
    return Workload(f"unit_{n}_k{k:g}_bc{bc}_c{coarse_op}", nx, ny, hx, hy, bc, k, source,
                    coarse_op)


# The wedge model (the paper's layered test, Section 2): x in [0, 600] m,
# y in [-1000, 0] m (node row j = 0 at the bottom), three layers of 2000, 1500
# and 3000 m/s from the top down, split by two sloping planar interfaces.  The
# paper's figure of the geometry is not available; the interfaces used here are
#   upper: y = -400 + 100 * x / 600   (from -400 m at x = 0 to -300 m at 600)
#   lower: y = -750 + 250 * x / 600   (from -750 m to -500 m; they never meet).
WEDGE_X, WEDGE_Y = 600.0, 1000.0
WEDGE_C = (2000.0, 1500.0, 3000.0)


def wedge_interfaces(x):
    return -400.0 + 100.0 * x / WEDGE_X, -750.0 + 250.0 * x / WEDGE_X


def wedge_velocity(nx: int, ny: int, hx: float, hy: float) -> np.ndarray:
    x = np.arange(nx) * hx
    y = -WEDGE_Y + np.arange(ny) * hy
    up, lo = wedge_interfaces(x)
    Y = y[:, None]
    return np.where(Y >= up[None, :], WEDGE_C[0],
                    np.where(Y >= lo[None, :], WEDGE_C[1], WEDGE_C[2])).astype(np.float64)


def wedge(nx: int = 1153, ny: int = 1921, freq: float | None = None) -> Workload:
    """The wedge on an nx x ny grid (h = 600/(nx-1) = 1000/(ny-1) for the
    paper's 9*2^q+1 x 15*2^q+1 grids).  The frequency defaults to 40 Hz on the
    1153 x 1921 grid and scales with 1/h below it (same points per wavelength,
    kh <= 0.087).  Sommerfeld boundary, point source at the top centre,
    Galerkin (str-Glk) coarse operator, coarse GMRES(30) to 0.1."""
    hx, hy = WEDGE_X / (nx - 1), WEDGE_Y / (ny - 1)
    if freq is None:
        freq = 40.0 * (nx - 1) / 1152.0
    return Workload(f"wedge_{nx}x{ny}_f{freq:g}", nx, ny, hx, hy, BC_SOMMERFELD, 0.0, "point",
                    COARSE_GALERKIN, model="wedge", freq=freq)


# A layered multi-source model for batched solves: 2049 x 1025 nodes at
# h = 5 m (10240 m x 5120 m), 8 horizontal layers of equal thickness with
# seeded velocities in [1500, 4500] m/s, and 3 seeded Gaussian anomalies of
# +-15% (centres in the middle 80% of the domain, widths 200..600 m), so
# c >= 1275 m/s and kh <= 0.49 at 20 Hz.  Sources: 1/h^2 at i = 16 + 32 s,
# five nodes below the top edge (row ny - 1 - 5), s = 0 .. nsrc-1.
def layered_velocity(nx: int, ny: int, h: float, seed: int = SEED) -> np.ndarray:
    rng = np.random.default_rng(seed)
    c_layers = rng.uniform(1500.0, 4500.0, 8)
    depth = (ny - 1 - np.arange(ny)) / (ny - 1)            # 0 at the top row, 1 at the bottom
    layer = np.minimum((depth * 8).astype(int), 7)
    c = np.repeat(c_layers[layer][:, None], nx, axis=1)
    X, Y = np.meshgrid(np.arange(nx) * h, np.arange(ny) * h)
    Lx, Ly = (nx - 1) * h, (ny - 1) * h
    pert = np.zeros_like(c)
    for _ in range(3):
        amp = 0.15 * rng.choice([-1.0, 1.0])
        cx, cy = rng.uniform(0.1, 0.9) * Lx, rng.uniform(0.1, 0.9) * Ly
        sig = rng.uniform(200.0, 600.0)
        pert += amp * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2 * sig * sig))
    return c * (1.0 + np.clip(pert, -0.15, 0.15))


def layered_sources(nx: int, ny: int, h: float, nsrc: int) -> np.ndarray:
    b = np.zeros((nsrc, ny, nx), np.complex128)
    for s in range(nsrc):
        i = 16 + 32 * s
        if i >= nx:
            raise ValueError(f"source {s} at column {i} is outside the {nx}-node grid")
        b[s, ny - 1 - 5, i] = 1.0 / (h * h)
    return b


def layered(nx: int = 2049, ny: int = 1025, h: float = 5.0, freq: float = 10.0,
            nsrc: int = 64) -> Workload:
    """The layered model at one frequency with nsrc sources (one operator, nsrc
    right-hand sides): Sommerfeld boundary, ReD-Glk2 coarse operator, FGMRES(20)
    (the outer bases of 64 right-hand sides then take about 90 GB), coarse
    GMRES(15) to 0.1."""
    return Workload(f"layered_{nx}x{ny}_f{freq:g}_x{nsrc}", nx, ny, h, h, BC_SOMMERFELD, 0.0,
                    "point", COARSE_REDGLK2, restart=20, coarse_restart=15, model="layered",
                    freq=freq, nsrc=nsrc)


# The adjoint-gradient case: the layered model's physical domain (10240 m x
# 5120 m) on an nx x ny grid (1025 x 513 at h = 10 m), one frequency (10 Hz
# there; scaled with 1/h on coarser grids to keep kh), nshot sources at
# i = 32 + 64 s and nrec receivers spread evenly over i = 2 .. 1022 (i = 2 + 4 r
# for 256 of them) on the row five nodes below the top edge (positions scaled
# with the grid).  The "true" model adds one
# seeded +10% Gaussian anomaly (width 400 m) to the layered model; the initial
# model is the layered model itself.
def adjoint_case(nx: int = 1025, ny: int = 513, nshot: int = 16, nrec: int = 256,
                 seed: int = SEED + 1):
    h = 10240.0 / (nx - 1)
    if abs(h * (ny - 1) - 5120.0) > 1e-9:
        raise ValueError("the grid must span 10240 m x 5120 m")
    freq = 10.0 * 10.0 / h
    c0 = layered_velocity(nx, ny, h)
    rng = np.random.default_rng(seed)
    X, Y = np.meshgrid(np.arange(nx) * h, np.arange(ny) * h)
    cx, cy = rng.uniform(0.3, 0.7) * 10240.0, rng.uniform(0.3, 0.7) * 5120.0
    c_true = c0 * (1.0 + 0.10 * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2 * 400.0 ** 2)))
    scale = (nx - 1) / 1024.0
    jrow = ny - 1 - 5
    src_i = [int(round((32 + 64 * q) * scale)) for q in range(nshot)]
    rec_i = [int(round((2 + r * 1020.0 / max(nrec - 1, 1)) * scale)) for r in range(nrec)]
    if len(set(rec_i)) != nrec or max(src_i + rec_i) >= nx:
        raise ValueError("sources/receivers do not fit this grid")
    sources = np.zeros((nshot, ny, nx), np.complex128)
    for q, i in enumerate(src_i):
        sources[q, jrow, i] = 1.0 / (h * h)
    rec = np.array([jrow * nx + i for i in rec_i], np.int32)
    return dict(nx=nx, ny=ny, h=h, freq=freq, s_true=1.0 / c_true ** 2, s_init=1.0 / c0 ** 2,
                sources=sources, rec=rec)
