"""C-ABI checks that need no GPU: the library loads, exports every entry point
that include/helmdefl.h declares, and rejects bad arguments before touching the
device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "helmdefl.h")


@pytest.fixture(scope="module")
def H():
    from paper_2308_06152_amd import helmdefl
    if not os.path.exists(helmdefl.SO_PATH):
        pytest.skip("libhelmdefl.so not built")
    helmdefl.load()
    return helmdefl


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_the_path_entry_points():
    names = declared_functions()
    for n in ("helm_apply", "cslp_vcycle", "deflate_apply", "helm_solve", "helm_create",
              "helm_destroy", "helm_strerror", "helm_opts_default"):
        assert n in names


def test_library_exports_every_declared_symbol(H):
    lib = ctypes.CDLL(H.SO_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing
    assert sorted(H.EXPORTED) == declared_functions()


def test_defaults_and_strerror(H):
    o = H.default_opts()
    assert (o.beta_re, o.beta_im, o.omega, o.nu_pre, o.nu_post) == (1.0, 0.5, 0.8, 1, 1)
    assert (o.restart, o.tol, o.coarse_tol, o.coarse_restart) == (50, 1e-6, 0.1, 30)
    assert o.defl_vectors == H.Z_HIGH
    assert o.coarsest_nodes == 1089
    assert o.precision == H.PREC_FP64
    assert o.outer == H.OUTER_FGMRES
    assert o.batch == 1
    assert o.graphs == 0
    assert o.vc_tail == 300000
    L = H.load()
    assert L.helm_strerror(0) == b"success"
    assert b"coarsen" in L.helm_strerror(H.HELM_EGRID)
    assert b"scratch" in L.helm_strerror(H.HELM_ESCRATCH)
    assert L.helm_strerror(12345) == b"unknown error"
    assert L.helm_opts_default(None) == H.HELM_EINVAL


def _create(H, nx, ny, hx=0.1, hy=0.1, bc=1, kconst=1.0, **opts):
    L = H.load()
    g = H.Grid(nx, ny, hx, hy, bc)
    o = H.default_opts(**opts)
    h = ctypes.c_void_p()
    return L.helm_create(ctypes.byref(g), None, kconst, ctypes.byref(o), None, ctypes.byref(h))


@pytest.mark.parametrize("nx,ny", [(4, 9), (9, 4), (3, 3), (8, 8), (65, 64)])
def test_create_rejects_uncoarsenable_grids(H, nx, ny):
    assert _create(H, nx, ny) == H.HELM_EGRID


@pytest.mark.parametrize("kw", [dict(nu_pre=2), dict(nu_post=0), dict(restart=0),
                                dict(restart=61), dict(coarse_restart=0), dict(coarse_iters=0),
                                dict(coarse_mode=0), dict(coarse_op=7), dict(defl_vectors=3),
                                dict(omega=0.0), dict(tol=-1.0), dict(coarsest_nodes=-1),
                                dict(coarsest_nodes=5000), dict(precision=3),
                                dict(precision=-1), dict(coarse_op=5), dict(coarse_op=-1),
                                dict(outer=3), dict(outer=-1), dict(batch=2),
                                dict(graphs=2), dict(graphs=-1), dict(vc_tail=-1)])
def test_create_rejects_bad_options(H, kw):
    assert _create(H, 9, 9, **kw) == H.HELM_EINVAL


def test_create_rejects_bad_grid_values(H):
    assert _create(H, 9, 9, hx=0.0) == H.HELM_EINVAL
    assert _create(H, 9, 9, hx=float("nan")) == H.HELM_EINVAL
    assert _create(H, 9, 9, bc=5) == H.HELM_EINVAL
    # ReD-Glk2 and ReD-Glk1 are defined for hx == hy only
    assert _create(H, 9, 9, hx=0.1, hy=0.2, coarse_op=1) == H.HELM_EINVAL
    assert _create(H, 9, 9, hx=0.1, hy=0.2, coarse_op=4) == H.HELM_EINVAL
    assert _create(H, 9, 9, kconst=float("inf")) == H.HELM_ENONFINITE
    assert _create(H, 9, 9, kconst=-1.0) == H.HELM_ENONFINITE


def test_null_arguments(H):
    L = H.load()
    h = ctypes.c_void_p()
    assert L.helm_create(None, None, 1.0, None, None, ctypes.byref(h)) == H.HELM_EINVAL
    assert L.helm_apply(None, None, None, 1) == H.HELM_EINVAL
    assert L.cslp_vcycle(None, None, None, 1) == H.HELM_EINVAL
    assert L.cslp_vcycle_noalloc(None, None, None, 1) == H.HELM_EINVAL
    assert L.deflate_apply(None, 2, None, None, 1) == H.HELM_EINVAL
    assert L.helm_solve(None, None, None, 1, None) == H.HELM_EINVAL
    assert L.helm_destroy(None) == H.HELM_EINVAL
