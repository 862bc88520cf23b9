"""Thin ctypes binding of libhelmdefl.so (include/helmdefl.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  Tensors are ``torch.complex128`` on the GPU (PyTorch supplies device
memory and the stream); the binding passes their data pointers.  Importing this
module fails loudly if the compiled library is missing -- there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(HERE, "libhelmdefl.so")

HELM_OK, HELM_EINVAL, HELM_EGRID, HELM_ENONFINITE = 0, -1, -2, -3
HELM_ENOMEM, HELM_EHIP, HELM_ENOCONV, HELM_ESCRATCH = -4, -5, -6, -7
BC_DIRICHLET, BC_SOMMERFELD = 0, 1
DEFL_Q, DEFL_P, DEFL_ADEF1 = 0, 1, 2
Z_LINEAR, Z_HIGH = 0, 1
COARSE_GALERKIN, COARSE_REDGLK2, COARSE_REDO2, COARSE_REDO4, COARSE_REDGLK1 = 0, 1, 2, 3, 4
CMODE_FIXED, CMODE_TOL = 1, 2
PREC_FP64, PREC_MIXED, PREC_MIXED_C64BASIS = 0, 1, 2
OUTER_FGMRES, OUTER_GCR, OUTER_GMRES_LEFT = 0, 1, 2
K_APPLY, K_VC_DOWN, K_VC_UP, K_ZT, K_DRESID, K_COARSE, K_DOT, K_UPDATE = range(8)
KERNEL_CLASS_NAMES = ["apply5", "vc_down", "vc_up", "zt", "dresid", "coarse_op", "mdot",
                      "mupdate"]

EXPORTED = [
    "helm_opts_default", "helm_create", "helm_apply", "cslp_vcycle", "deflate_apply",
    "helm_solve", "helm_destroy", "helm_strerror", "helm_coarse_dims", "helm_num_levels",
    "helm_level_dims", "helm_z_restrict", "helm_z_prolong", "helm_coarse_apply",
    "helm_coarse_solve", "helm_timing_enable", "helm_timing_read", "helm_adjoint_solve",
    "helm_gradient_s", "helm_receivers", "cslp_vcycle_noalloc",
]


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("hx", ctypes.c_double),
                ("hy", ctypes.c_double), ("bc", ctypes.c_int)]


class Opts(ctypes.Structure):
    _fields_ = [("beta_re", ctypes.c_double), ("beta_im", ctypes.c_double),
                ("omega", ctypes.c_double), ("nu_pre", ctypes.c_int), ("nu_post", ctypes.c_int),
                ("defl_vectors", ctypes.c_int), ("coarse_op", ctypes.c_int),
                ("coarse_mode", ctypes.c_int), ("coarse_iters", ctypes.c_int),
                ("coarse_restart", ctypes.c_int), ("coarse_tol", ctypes.c_double),
                ("restart", ctypes.c_int), ("maxit", ctypes.c_int), ("tol", ctypes.c_double),
                ("x0_given", ctypes.c_int), ("force_iters", ctypes.c_int),
                ("coarsest_nodes", ctypes.c_int), ("precision", ctypes.c_int),
                ("outer", ctypes.c_int), ("batch", ctypes.c_int),
                ("graphs", ctypes.c_int), ("vc_tail", ctypes.c_int)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int), ("inner_iters_total", ctypes.c_int),
                ("inner_iters_max", ctypes.c_int), ("converged", ctypes.c_int),
                ("relres", ctypes.c_double), ("t_solve_ms", ctypes.c_double),
                ("t_setup_ms", ctypes.c_double), ("t_coarse_ms", ctypes.c_double),
                ("t_vcycle_ms", ctypes.c_double), ("reorth_steps", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def load() -> ctypes.CDLL:
    """Load libhelmdefl.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(SO_PATH):
        raise ImportError(f"{SO_PATH} is missing: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`")
    L = ctypes.CDLL(SO_PATH)
    vp, ip, cint = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.c_int
    L.helm_opts_default.argtypes = [ctypes.POINTER(Opts)]
    L.helm_create.argtypes = [ctypes.POINTER(Grid), vp, ctypes.c_double, ctypes.POINTER(Opts),
                              vp, ctypes.POINTER(vp)]
    L.helm_apply.argtypes = [vp, vp, vp, cint]
    L.cslp_vcycle.argtypes = [vp, vp, vp, cint]
    L.cslp_vcycle_noalloc.argtypes = [vp, vp, vp, cint]
    L.deflate_apply.argtypes = [vp, cint, vp, vp, cint]
    L.helm_solve.argtypes = [vp, vp, vp, cint, ctypes.POINTER(SolveInfo)]
    L.helm_destroy.argtypes = [vp]
    L.helm_strerror.argtypes = [cint]
    L.helm_strerror.restype = ctypes.c_char_p
    L.helm_coarse_dims.argtypes = [vp, ip, ip]
    L.helm_num_levels.argtypes = [vp, ip]
    L.helm_level_dims.argtypes = [vp, cint, ip, ip]
    L.helm_z_restrict.argtypes = [vp, vp, vp]
    L.helm_z_prolong.argtypes = [vp, vp, vp]
    L.helm_coarse_apply.argtypes = [vp, vp, vp]
    L.helm_coarse_solve.argtypes = [vp, vp, vp, ip]
    L.helm_timing_enable.argtypes = [vp, cint, cint]
    L.helm_timing_read.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong),
                                   ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double)]
    L.helm_adjoint_solve.argtypes = [vp, vp, vp, cint, ctypes.POINTER(SolveInfo)]
    L.helm_gradient_s.argtypes = [vp, ctypes.c_double, vp, vp, cint, vp]
    L.helm_receivers.argtypes = [vp, vp, cint, vp, vp, cint, vp, vp, vp]
    _lib = L
    return L


class HelmError(RuntimeError):
    def __init__(self, code: int, what: str):
        msg = load().helm_strerror(code).decode()
        super().__init__(f"{what}: {msg} ({code})")
        self.code = code


def check(code: int, what: str) -> int:
    if code != HELM_OK:
        raise HelmError(code, what)
    return code


def default_opts(**kw) -> Opts:
    o = Opts()
    check(load().helm_opts_default(ctypes.byref(o)), "helm_opts_default")
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def _ptr(t) -> int:
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.complex128:
        raise TypeError("expected a CUDA complex128 tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


class Solver:
    """A helm_ctx handle: the grid, wavenumber and method options of one problem."""

    def __init__(self, nx: int, ny: int, hx: float, hy: float, bc: int, k=None,
                 kconst: float = 0.0, stream=None, **opts):
        import torch
        L = load()
        self.grid = Grid(nx, ny, hx, hy, bc)
        self.opts = default_opts(**opts)
        self.nx, self.ny = nx, ny
        kp = None
        if k is not None:
            if not (k.is_cuda and k.dtype == torch.float64 and k.shape == (ny, nx)):
                raise TypeError("k must be a CUDA float64 tensor of shape (ny, nx)")
            kp = k.contiguous().data_ptr()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        check(L.helm_create(ctypes.byref(self.grid), kp, float(kconst), ctypes.byref(self.opts),
                            ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
              "helm_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            load().helm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # shapes -------------------------------------------------------------
    def coarse_dims(self) -> tuple[int, int]:
        a, b = ctypes.c_int(), ctypes.c_int()
        check(load().helm_coarse_dims(self.h, ctypes.byref(a), ctypes.byref(b)), "coarse_dims")
        return a.value, b.value

    def num_levels(self) -> int:
        n = ctypes.c_int()
        check(load().helm_num_levels(self.h, ctypes.byref(n)), "num_levels")
        return n.value

    def level_dims(self, level: int) -> tuple[int, int]:
        a, b = ctypes.c_int(), ctypes.c_int()
        check(load().helm_level_dims(self.h, level, ctypes.byref(a), ctypes.byref(b)),
              "level_dims")
        return a.value, b.value

    def _nrhs(self, t, shape) -> int:
        if tuple(t.shape[-2:]) != shape:
            raise ValueError(f"expected trailing shape {shape}, got {tuple(t.shape)}")
        return 1 if t.dim() == 2 else int(t.numel() // (shape[0] * shape[1]))

    # operators ----------------------------------------------------------
    def apply(self, x, out=None):
        import torch
        out = torch.empty_like(x) if out is None else out
        n = self._nrhs(x, (self.ny, self.nx))
        check(load().helm_apply(self.h, _ptr(x), _ptr(out), n), "helm_apply")
        return out

    def vcycle(self, r, out=None):
        import torch
        out = torch.empty_like(r) if out is None else out
        n = self._nrhs(r, (self.ny, self.nx))
        check(load().cslp_vcycle(self.h, _ptr(r), _ptr(out), n), "cslp_vcycle")
        return out

    def vcycle_noalloc(self, r, out):
        """cslp_vcycle through the entry point that allocates nothing (the
        level buffers live in the library's fixed device scratch); `out` must
        be given."""
        n = self._nrhs(r, (self.ny, self.nx))
        check(load().cslp_vcycle_noalloc(self.h, _ptr(r), _ptr(out), n), "cslp_vcycle_noalloc")
        return out

    def deflate(self, v, mode: int = DEFL_ADEF1, out=None):
        import torch
        out = torch.empty_like(v) if out is None else out
        n = self._nrhs(v, (self.ny, self.nx))
        check(load().deflate_apply(self.h, mode, _ptr(v), _ptr(out), n), "deflate_apply")
        return out

    def solve(self, b, x=None, raise_on_noconv: bool = False):
        """Returns (x, [info dict per right-hand side])."""
        import torch
        x = torch.zeros_like(b) if x is None else x
        n = self._nrhs(b, (self.ny, self.nx))
        infos = (SolveInfo * n)()
        rc = load().helm_solve(self.h, _ptr(b), _ptr(x), n, infos)
        if rc != HELM_OK and (rc != HELM_ENOCONV or raise_on_noconv):
            raise HelmError(rc, "helm_solve")
        return x, [i.as_dict() for i in infos]

    def z_restrict(self, vf, out=None):
        import torch
        nxc, nyc = self.coarse_dims()
        out = torch.empty((nyc, nxc), dtype=vf.dtype, device=vf.device) if out is None else out
        check(load().helm_z_restrict(self.h, _ptr(vf), _ptr(out)), "helm_z_restrict")
        return out

    def z_prolong(self, vc, out=None):
        import torch
        out = torch.empty((self.ny, self.nx), dtype=vc.dtype, device=vc.device) \
            if out is None else out
        check(load().helm_z_prolong(self.h, _ptr(vc), _ptr(out)), "helm_z_prolong")
        return out

    def coarse_apply(self, x, out=None):
        import torch
        out = torch.empty_like(x) if out is None else out
        check(load().helm_coarse_apply(self.h, _ptr(x), _ptr(out)), "helm_coarse_apply")
        return out

    def coarse_solve(self, v1, out=None):
        import torch
        out = torch.empty_like(v1) if out is None else out
        it = ctypes.c_int()
        check(load().helm_coarse_solve(self.h, _ptr(v1), _ptr(out), ctypes.byref(it)),
              "helm_coarse_solve")
        return out, it.value

    # adjoint state ------------------------------------------------------
    def adjoint_solve(self, f, out=None, raise_on_noconv: bool = False):
        """(lambda, [info per right-hand side]): lambda = A_h^{-H} f."""
        import torch
        out = torch.empty_like(f) if out is None else out
        n = self._nrhs(f, (self.ny, self.nx))
        infos = (SolveInfo * n)()
        rc = load().helm_adjoint_solve(self.h, _ptr(f), _ptr(out), n, infos)
        if rc != HELM_OK and (rc != HELM_ENOCONV or raise_on_noconv):
            raise HelmError(rc, "helm_adjoint_solve")
        return out, [i.as_dict() for i in infos]

    def gradient_s(self, omega: float, u, lam, g=None):
        """g (+)= -Re(conj(lambda) dA/ds u) summed over right-hand sides, as a
        float64 [ny][nx] tensor."""
        import torch
        if g is None:
            g = torch.zeros((self.ny, self.nx), dtype=torch.float64, device=u.device)
        if not (g.is_cuda and g.dtype == torch.float64 and g.is_contiguous()
                and tuple(g.shape) == (self.ny, self.nx)):
            raise TypeError("g must be a contiguous CUDA float64 (ny, nx) tensor")
        n = self._nrhs(u, (self.ny, self.nx))
        if self._nrhs(lam, (self.ny, self.nx)) != n:
            raise ValueError("u and lambda hold different numbers of right-hand sides")
        check(load().helm_gradient_s(self.h, float(omega), _ptr(u), _ptr(lam), n,
                                     g.data_ptr()), "helm_gradient_s")
        return g

    def receivers(self, rec, u, d):
        """(res, f, J): res = R u - d, f = R^T res, J = 1/2 ||res||^2 per
        right-hand side.  rec: CUDA int32 node indices j*nx + i; d: [nrhs][nrec]."""
        import torch
        if not (rec.is_cuda and rec.dtype == torch.int32 and rec.is_contiguous()):
            raise TypeError("rec must be a contiguous CUDA int32 tensor")
        n = self._nrhs(u, (self.ny, self.nx))
        nrec = int(rec.numel())
        if int(d.numel()) != n * nrec:
            raise ValueError(f"d must hold nrhs x nrec = {n} x {nrec} values")
        res = torch.empty((n, nrec), dtype=torch.complex128, device=u.device)
        f = torch.empty((n, self.ny, self.nx), dtype=torch.complex128, device=u.device)
        J = torch.empty(n, dtype=torch.float64, device=u.device)
        check(load().helm_receivers(self.h, rec.data_ptr(), nrec, _ptr(u), _ptr(d), n,
                                    _ptr(res), _ptr(f), J.data_ptr()), "helm_receivers")
        return res, f, J

    # timing -------------------------------------------------------------
    def timing_enable(self, kclass: int, level: int = -1):
        check(load().helm_timing_enable(self.h, kclass, level), "helm_timing_enable")

    def timing_read(self):
        n, ms, by = ctypes.c_longlong(), ctypes.c_double(), ctypes.c_double()
        check(load().helm_timing_read(self.h, ctypes.byref(n), ctypes.byref(ms),
                                      ctypes.byref(by)), "helm_timing_read")
        return n.value, ms.value, by.value
