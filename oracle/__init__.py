"""Python access to the plain FP64 CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check and the benchmark's
CPU-baseline leg import this module.  The product library never does, and this
module imports nothing from the product package.

Every function takes and returns numpy ``complex128`` arrays shaped ``(ny, nx)``
(x fastest), matching the layout of the C code.  The C source says, per routine,
which passage of the paper it follows and how it is pinned.
"""
from __future__ import annotations

import contextlib
import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")

BC_DIRICHLET, BC_SOMMERFELD = 0, 1
Z_LINEAR, Z_HIGH = 0, 1
COARSE_GALERKIN, COARSE_REDGLK2, COARSE_REDO2, COARSE_REDO4, COARSE_REDGLK1 = 0, 1, 2, 3, 4
CMODE_EXACT, CMODE_FIXED, CMODE_TOL = 0, 1, 2
DEFL_Q, DEFL_P, DEFL_ADEF1 = 0, 1, 2
PRECOND_VCYCLE, PRECOND_EXACT_A = 0, 1


_SO_SERIAL = os.path.join(_HERE, "liboracle_serial.so")
# Plain optimisation for any x86-64 host with AVX2 and FMA (the build host and
# the GPU host may differ, so no -march=native).  -fopenmp splits the
# element-wise grid loops and the fixed-chunk sums over threads; the serial
# build (same flags without -fopenmp) gives bit-identical results.
_CFLAGS = ["-O3", "-march=x86-64-v3", "-std=c99", "-Wall", "-Wextra", "-fPIC", "-shared"]


def build(force: bool = True, serial: bool = False) -> str:
    """Compile oracle.c into liboracle.so (OpenMP) or liboracle_serial.so."""
    so = _SO_SERIAL if serial else _SO
    if force or not os.path.exists(so):
        cmd = ["gcc", *_CFLAGS, *([] if serial else ["-fopenmp"]), "-o", so + ".tmp",
               os.path.join(_HERE, "oracle.c"), "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(so + ".tmp", so)
    return so


class _Problem(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("hx", ctypes.c_double), ("hy", ctypes.c_double),
        ("bc", ctypes.c_int),
        ("k", ctypes.POINTER(ctypes.c_double)), ("kconst", ctypes.c_double),
        ("beta_re", ctypes.c_double), ("beta_im", ctypes.c_double),
        ("omega", ctypes.c_double),
        ("nu_pre", ctypes.c_int), ("nu_post", ctypes.c_int),
        ("defl_vectors", ctypes.c_int), ("coarse_op", ctypes.c_int),
        ("coarse_mode", ctypes.c_int), ("coarse_iters", ctypes.c_int),
        ("coarse_restart", ctypes.c_int), ("coarse_tol", ctypes.c_double),
        ("precond", ctypes.c_int),
        ("coarsest_nodes", ctypes.c_int),
    ]


class _Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("converged", ctypes.c_int),
                ("inner_total", ctypes.c_int), ("inner_max", ctypes.c_int),
                ("relres", ctypes.c_double)]


@dataclasses.dataclass
class Problem:
    """The discrete problem and method options, mirroring ``ora_problem``."""
    nx: int
    ny: int
    hx: float
    hy: float
    bc: int = BC_DIRICHLET
    k: np.ndarray | None = None      # real (ny, nx) wavenumber field, or None
    kconst: float = 0.0
    beta_re: float = 1.0
    beta_im: float = 0.5
    omega: float = 0.8
    nu_pre: int = 1
    nu_post: int = 1
    defl_vectors: int = Z_HIGH
    coarse_op: int = COARSE_GALERKIN
    coarse_mode: int = CMODE_EXACT
    coarse_iters: int = 300
    coarse_restart: int = 30
    coarse_tol: float = 1e-1
    precond: int = PRECOND_VCYCLE
    coarsest_nodes: int = 0           # predefined coarsest grid (0 = down to 3x3)

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)

    def _c(self):
        p = _Problem()
        p.nx, p.ny, p.hx, p.hy, p.bc = self.nx, self.ny, self.hx, self.hy, self.bc
        keep = None
        if self.k is not None:
            keep = np.ascontiguousarray(self.k, dtype=np.float64)
            assert keep.shape == (self.ny, self.nx)
            p.k = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        p.kconst = self.kconst
        p.beta_re, p.beta_im, p.omega = self.beta_re, self.beta_im, self.omega
        p.nu_pre, p.nu_post = self.nu_pre, self.nu_post
        p.defl_vectors, p.coarse_op = self.defl_vectors, self.coarse_op
        p.coarse_mode, p.coarse_iters = self.coarse_mode, self.coarse_iters
        p.coarse_restart, p.coarse_tol = self.coarse_restart, self.coarse_tol
        p.precond = self.precond
        p.coarsest_nodes = self.coarsest_nodes
        return p, keep


_lib = None
_libs = {}


@contextlib.contextmanager
def serial_build():
    """Run the calls inside the block on the serial (no OpenMP) build."""
    global _lib
    saved = lib()
    _lib = _load(_SO_SERIAL, serial=True)
    try:
        yield
    finally:
        _lib = saved


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        _lib = _load(_SO, serial=False)
    return _lib


def _load(path: str, serial: bool) -> ctypes.CDLL:
    if path not in _libs:
        if not os.path.exists(path):
            build(force=False, serial=serial)
        L = ctypes.CDLL(path)
        P = ctypes.POINTER(_Problem)
        D = ctypes.POINTER(ctypes.c_double)
        IP = ctypes.POINTER(ctypes.c_int)
        L.ora_set_threads.argtypes = [ctypes.c_int]
        L.ora_set_threads.restype = None
        L.ora_num_levels.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.ora_level_dims.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, IP,
                                     IP]
        for name in ("ora_helm_apply", "ora_cslp_apply", "ora_z_prolong", "ora_z_restrict",
                     "ora_coarse_apply", "ora_direct_solve", "ora_coarse_direct_solve"):
            getattr(L, name).argtypes = [P, D, D]
        L.ora_vcycle.argtypes = [P, ctypes.c_int, D, D]
        L.ora_coarse_solve.argtypes = [P, D, D, IP]
        L.ora_deflate_apply.argtypes = [P, ctypes.c_int, D, D, IP]
        L.ora_fgmres.argtypes = [P, D, D, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                 ctypes.c_int, ctypes.POINTER(_Info)]
        L.ora_gmres_left.argtypes = [P, D, D, ctypes.c_double, ctypes.c_int,
                                     ctypes.POINTER(_Info)]
        L.ora_gcr.argtypes = [P, D, D, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                              ctypes.c_int, ctypes.POINTER(_Info)]
        L.ora_helm_apply_adjoint.argtypes = [P, D, D]
        L.ora_adjoint_solve.argtypes = [P, D, D]
        L.ora_grad_s.argtypes = [P, ctypes.c_double, D, D, D]
        _libs[path] = L
    return _libs[path]


class OracleError(RuntimeError):
    pass


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _cin(a, shape) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.complex128)
    if a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _check(rc: int, what: str):
    if rc != 0:
        raise OracleError(f"{what} failed with code {rc}")


def threads() -> int:
    """OpenMP threads the oracle's loops use (results do not depend on it)."""
    return int(lib().ora_threads())


def set_threads(n: int) -> None:
    lib().ora_set_threads(int(n))


def num_levels(nx: int, ny: int, coarsest_nodes: int = 0) -> int:
    return lib().ora_num_levels(nx, ny, coarsest_nodes)


def level_dims(nx: int, ny: int, level: int, coarsest_nodes: int = 0) -> tuple[int, int]:
    a, b = ctypes.c_int(), ctypes.c_int()
    _check(lib().ora_level_dims(nx, ny, coarsest_nodes, level, ctypes.byref(a),
                                ctypes.byref(b)), "level_dims")
    return a.value, b.value


def coarse_dims(p: Problem) -> tuple[int, int]:
    return level_dims(p.nx, p.ny, 1, p.coarsest_nodes)


def _unary(name, p: Problem, x, in_shape, out_shape):
    c, keep = p._c()
    x = _cin(x, in_shape)
    y = np.empty(out_shape, np.complex128)
    _check(getattr(lib(), name)(ctypes.byref(c), _ptr(x), _ptr(y)), name)
    del keep
    return y


def helm_apply(p: Problem, x):
    """y = A_h x."""
    s = (p.ny, p.nx)
    return _unary("ora_helm_apply", p, x, s, s)


def cslp_apply(p: Problem, x):
    """y = M_h x (CSLP on the fine grid)."""
    s = (p.ny, p.nx)
    return _unary("ora_cslp_apply", p, x, s, s)


def z_prolong(p: Problem, vc):
    """v_f = Z v_c (deflation vectors, coarse -> fine)."""
    return _unary("ora_z_prolong", p, vc, coarse_dims(p)[::-1], (p.ny, p.nx))


def z_restrict(p: Problem, vf):
    """v_c = Z^T v_f."""
    return _unary("ora_z_restrict", p, vf, (p.ny, p.nx), coarse_dims(p)[::-1])


def coarse_apply(p: Problem, x):
    """y = A_2h x."""
    s = coarse_dims(p)[::-1]
    return _unary("ora_coarse_apply", p, x, s, s)


def direct_solve(p: Problem, b):
    """x = A_h^{-1} b by banded LU."""
    s = (p.ny, p.nx)
    return _unary("ora_direct_solve", p, b, s, s)


def coarse_direct_solve(p: Problem, b):
    """x = A_2h^{-1} b by banded LU."""
    s = coarse_dims(p)[::-1]
    return _unary("ora_coarse_direct_solve", p, b, s, s)


def vcycle(p: Problem, r, level: int = 0):
    """z = one CSLP V-cycle applied to r, starting at `level`."""
    nx, ny = level_dims(p.nx, p.ny, level, p.coarsest_nodes)
    c, keep = p._c()
    r = _cin(r, (ny, nx))
    z = np.empty((ny, nx), np.complex128)
    _check(lib().ora_vcycle(ctypes.byref(c), level, _ptr(r), _ptr(z)), "vcycle")
    del keep
    return z


def coarse_solve(p: Problem, v1):
    """(v2, inner_iterations) with v2 ~= A_2h^{-1} v1."""
    s = coarse_dims(p)[::-1]
    c, keep = p._c()
    v1 = _cin(v1, s)
    v2 = np.empty(s, np.complex128)
    it = ctypes.c_int()
    _check(lib().ora_coarse_solve(ctypes.byref(c), _ptr(v1), _ptr(v2), ctypes.byref(it)),
           "coarse_solve")
    del keep
    return v2, it.value


def deflate_apply(p: Problem, v, mode: int = DEFL_ADEF1):
    """(w, inner_iterations): w = Q v, (I - A Q) v, or P_A-DEF1 v."""
    s = (p.ny, p.nx)
    c, keep = p._c()
    v = _cin(v, s)
    w = np.empty(s, np.complex128)
    it = ctypes.c_int()
    _check(lib().ora_deflate_apply(ctypes.byref(c), mode, _ptr(v), _ptr(w), ctypes.byref(it)),
           "deflate_apply")
    del keep
    return w, it.value


@dataclasses.dataclass
class Info:
    iters: int
    converged: bool
    inner_total: int
    inner_max: int
    relres: float


def fgmres(p: Problem, b, restart: int = 50, tol: float = 1e-6, maxit: int = 500,
           force_iters: int = 0):
    """(x, Info): right-preconditioned FGMRES(restart) with P_A-DEF1."""
    s = (p.ny, p.nx)
    c, keep = p._c()
    b = _cin(b, s)
    x = np.empty(s, np.complex128)
    inf = _Info()
    _check(lib().ora_fgmres(ctypes.byref(c), _ptr(b), _ptr(x), restart, tol, maxit,
                            force_iters, ctypes.byref(inf)), "fgmres")
    del keep
    return x, Info(inf.iters, bool(inf.converged), inf.inner_total, inf.inner_max, inf.relres)


def gcr(p: Problem, b, restart: int = 50, tol: float = 1e-6, maxit: int = 500,
        force_iters: int = 0):
    """(x, Info): right-preconditioned GCR(restart) with P_A-DEF1."""
    s = (p.ny, p.nx)
    c, keep = p._c()
    b = _cin(b, s)
    x = np.empty(s, np.complex128)
    inf = _Info()
    _check(lib().ora_gcr(ctypes.byref(c), _ptr(b), _ptr(x), restart, tol, maxit, force_iters,
                         ctypes.byref(inf)), "gcr")
    del keep
    return x, Info(inf.iters, bool(inf.converged), inf.inner_total, inf.inner_max, inf.relres)


def gmres_left(p: Problem, b, tol: float = 1e-6, maxit: int = 200):
    """(x, Info): the paper's left-preconditioned full GMRES with P_A-DEF1."""
    s = (p.ny, p.nx)
    c, keep = p._c()
    b = _cin(b, s)
    x = np.empty(s, np.complex128)
    inf = _Info()
    _check(lib().ora_gmres_left(ctypes.byref(c), _ptr(b), _ptr(x), tol, maxit,
                                ctypes.byref(inf)), "gmres_left")
    del keep
    return x, Info(inf.iters, bool(inf.converged), inf.inner_total, inf.inner_max, inf.relres)


def helm_apply_adjoint(p: Problem, x):
    """y = A_h^H x."""
    s = (p.ny, p.nx)
    c, keep = p._c()
    x = _cin(x, s)
    y = np.empty(s, np.complex128)
    _check(lib().ora_helm_apply_adjoint(ctypes.byref(c), _ptr(x), _ptr(y)), "helm_apply_adjoint")
    del keep
    return y


def adjoint_solve(p: Problem, f):
    """lambda = A_h^{-H} f (direct)."""
    s = (p.ny, p.nx)
    c, keep = p._c()
    f = _cin(f, s)
    lam = np.empty(s, np.complex128)
    _check(lib().ora_adjoint_solve(ctypes.byref(c), _ptr(f), _ptr(lam)), "adjoint_solve")
    del keep
    return lam


def grad_s(p: Problem, omega: float, u, lam):
    """Per-node -Re(conj(lambda) dA/ds u), s = (k/omega)^2."""
    s = (p.ny, p.nx)
    c, keep = p._c()
    u = _cin(u, s)
    lam = _cin(lam, s)
    g = np.empty(s, np.float64)
    _check(lib().ora_grad_s(ctypes.byref(c), float(omega), _ptr(u), _ptr(lam),
                            g.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "grad_s")
    del keep
    return g
