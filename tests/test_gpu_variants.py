"""GPU parity of the paper's variants: the ReD-O2, ReD-O4 and ReD-Glk1
coarse operators (Sections 5.2.3, 5.2.4), the GCR outer method (Section 6.3)
and the left-preconditioned GMRES of Algorithm 1, against the CPU oracle.
Bars as for the plain path: 1e-12 per operator, 1e-11 for A-DEF1 with a fixed
inner count, outer counts within one and true residuals below tolerance for
solves, 1e-5 between iterates at an equal iteration count."""
import numpy as np
import pytest

from paper_2308_06152_amd import inputs

from test_gpu_parity import CASES, H, dev, host, make_pair, rel  # noqa: F401

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

VARIANTS = [2, 3, 4]  # ReD-O2, ReD-O4, ReD-Glk1


@pytest.mark.parametrize("cop", VARIANTS)
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_variant_coarse_operator_parity(H, ora, case, cop):
    S, P = make_pair(H, ora, case[:6] + (cop,))
    nxc, nyc = S.coarse_dims()
    x = inputs.random_complex((nyc, nxc), 141)
    got = host(S.coarse_apply(dev(x)))
    assert rel(got, ora.coarse_apply(P, x)) <= 1e-12


@pytest.mark.parametrize("cop", VARIANTS)
@pytest.mark.parametrize("case", CASES[:6], ids=[c[0] for c in CASES[:6]])
def test_variant_deflate_apply_parity(H, ora, case, cop):
    n_it = 8
    S, P = make_pair(H, ora, case[:6] + (cop,), coarse_mode=1, coarse_iters=n_it,
                     coarse_restart=30)
    Po = P.replace(coarse_mode=ora.CMODE_FIXED, coarse_iters=n_it, coarse_restart=30)
    v = inputs.random_complex((P.ny, P.nx), 142)
    got = host(S.deflate(dev(v), 2))
    want, _ = ora.deflate_apply(Po, v, 2)
    assert rel(got, want) <= 1e-11


def _pair(H, ora, n, k, bc, cop, **kw):
    w = inputs.scaled_plain(n, k, bc=bc, coarse_op=cop, source="point")
    okw = dict(coarse_op=cop, coarse_mode=2, coarse_tol=0.1, coarse_iters=300,
               coarse_restart=30, restart=50, tol=1e-6)
    okw.update(kw)
    S = H.Solver(w.nx, w.ny, w.hx, w.hy, w.bc, kconst=w.kconst, **okw)
    P = ora.Problem(w.nx, w.ny, w.hx, w.hy, bc=w.bc, kconst=w.kconst, coarse_op=cop,
                    coarsest_nodes=S.opts.coarsest_nodes,
                    coarse_mode=ora.CMODE_TOL if okw["coarse_mode"] == 2 else ora.CMODE_FIXED,
                    coarse_tol=okw["coarse_tol"], coarse_iters=okw["coarse_iters"],
                    coarse_restart=okw["coarse_restart"])
    return w, S, P


@pytest.mark.parametrize("bc,cop", [(1, 1), (0, 0), (1, 3)])
def test_gcr_solve_matches_oracle(H, ora, bc, cop):
    w, S, P = _pair(H, ora, 129, 30.0, bc, cop, outer=H.OUTER_GCR)
    b = w.rhs()
    x, info = S.solve(dev(b))
    xo, io = ora.gcr(P, b, restart=50, tol=1e-6, maxit=300)
    assert info[0]["converged"] and io.converged
    assert abs(info[0]["outer_iters"] - io.iters) <= 1
    r = ora.helm_apply(P, host(x)) - b  # the point source is off the boundary
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-6


def test_gcr_equal_iterations_match(H, ora):
    w, S, P = _pair(H, ora, 65, 20.0, 1, 1, outer=H.OUTER_GCR, coarse_mode=1, coarse_iters=10,
                    force_iters=6)
    Po = P.replace(coarse_mode=ora.CMODE_FIXED, coarse_iters=10)
    b = w.rhs()
    x, info = S.solve(dev(b))
    xo, io = ora.gcr(Po, b, restart=50, tol=1e-6, maxit=200, force_iters=6)
    assert info[0]["outer_iters"] == io.iters == 6
    assert rel(host(x), xo) <= 1e-5
    assert abs(info[0]["relres"] - io.relres) <= 1e-6 * max(io.relres, 1e-3)


def test_gcr_restart_and_tolerance(H, ora):
    """Restarted GCR(5) still reaches the FP64 tolerance on the true residual."""
    w, S, P = _pair(H, ora, 129, 30.0, 1, 1, outer=H.OUTER_GCR, restart=5)
    b = w.rhs()
    x, info = S.solve(dev(b))
    assert info[0]["converged"]
    r = ora.helm_apply(P, host(x)) - b
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-6


@pytest.mark.parametrize("cop", [0, 1, 2, 3, 4])
def test_left_gmres_matches_oracle_fixed_inner(H, ora, cop):
    """Algorithm 1 with a fixed inner count on both sides: the same outer
    count (within one) and the same true residual level."""
    w, S, P = _pair(H, ora, 65, 40.0, 1, cop, outer=H.OUTER_GMRES_LEFT, coarse_mode=1,
                    coarse_iters=25, restart=60, maxit=60)
    Po = P.replace(coarse_mode=ora.CMODE_FIXED, coarse_iters=25)
    b = w.rhs()
    x, info = S.solve(dev(b))
    xo, io = ora.gmres_left(Po, b, tol=1e-6, maxit=60)
    assert info[0]["converged"] and io.converged
    assert abs(info[0]["outer_iters"] - io.iters) <= 1


PAPER_65_K40 = {0: 7, 1: 9, 2: 20, 3: 17, 4: 12}  # MP-2b table, APD, 65 x 65, k = 40


@pytest.mark.parametrize("cop", [0, 1, 2, 3, 4])
def test_left_gmres_paper_counts_on_gpu(H, ora, cop):
    """The paper's setting for its coarse-operator table (left GMRES, coarse
    problem solved to 1e-12): the GPU path lands within two outer iterations
    of the printed counts (the oracle, with an exact coarse solve, within one)."""
    w, S, P = _pair(H, ora, 65, 40.0, 1, cop, outer=H.OUTER_GMRES_LEFT, coarse_mode=2,
                    coarse_tol=1e-12, coarse_iters=3000, coarse_restart=60, restart=60,
                    maxit=60)
    x, info = S.solve(dev(w.rhs()))
    assert info[0]["converged"]
    assert abs(info[0]["outer_iters"] - PAPER_65_K40[cop]) <= 2, info[0]


# The paper's coarse-tolerance experiments (Section 6.3): APD (higher-order
# vectors) with ReD-Glk2, point source at the centre of the unit square,
# Sommerfeld boundary; outer GMRES of Algorithm 1 (left preconditioning,
# preconditioned residual to 1e-6) or GCR; coarse problem solved by
# CSLP-preconditioned GMRES to the given tolerance.
PAPER_COARSE_TOL = [  # (n, k, coarse tolerance, outer method, printed count)
    (513, 320.0, 1e-2, "left", 10),
    (513, 320.0, 1e-6, "left", 10),
    (513, 320.0, 1e-10, "left", 10),
    (1025, 320.0, 1e-2, "left", 7),
    (1025, 320.0, 1e-6, "left", 6),
    (513, 320.0, 1e-1, "gcr", 12),
    (513, 320.0, 1e-2, "gcr", 11),
    (513, 320.0, 1e-6, "gcr", 11),
]


@pytest.mark.parametrize("n,k,ctol,outer,paper", PAPER_COARSE_TOL,
                         ids=[f"{c[0]}-k{c[1]:g}-{c[2]:g}-{c[3]}" for c in PAPER_COARSE_TOL])
def test_paper_coarse_tolerance_table(H, ora, n, k, ctol, outer, paper):
    """Outer iteration counts of the paper's coarse-tolerance table and its GCR
    runs, within one."""
    w = inputs.scaled_plain(n, k, bc=1, coarse_op=1, source="point")
    S = H.Solver(w.nx, w.ny, w.hx, w.hy, w.bc, kconst=w.kconst, coarse_op=1, coarse_mode=2,
                 coarse_tol=ctol, coarse_iters=5000, coarse_restart=60, restart=60, maxit=60,
                 tol=1e-6,
                 outer=H.OUTER_GMRES_LEFT if outer == "left" else H.OUTER_GCR)
    x, info = S.solve(dev(w.rhs()))
    print(f"{n}^2 k={k:g} coarse tol {ctol:g} {outer}: {info[0]['outer_iters']} outer "
          f"(paper {paper}), {info[0]['inner_iters_total']} inner, relres {info[0]['relres']:.2e}")
    assert info[0]["converged"]
    assert abs(info[0]["outer_iters"] - paper) <= 1


def test_paper_wedge_coarse_tolerance(H, ora):
    """The wedge row of the same table (289 x 481, 40 Hz, 9 outer iterations for
    every coarse tolerance).  The wedge geometry here is this build's own (the
    paper's figure is not available), so the count is checked within two."""
    w = inputs.wedge(289, 481, freq=40.0)
    for ctol in (1e-2, 1e-6):
        S = H.Solver(w.nx, w.ny, w.hx, w.hy, w.bc, k=dev(w.kfield()), coarse_op=1, coarse_mode=2,
                     coarse_tol=ctol, coarse_iters=5000, coarse_restart=60, restart=60,
                     maxit=60, tol=1e-6, outer=H.OUTER_GMRES_LEFT)
        b = inputs.point_source(w.nx, w.ny, w.hx, w.hy, (w.nx - 1) // 2, w.ny - 1)
        x, info = S.solve(dev(b))
        print(f"wedge 289x481 40 Hz coarse tol {ctol:g}: {info[0]['outer_iters']} outer (paper 9)")
        assert info[0]["converged"]
        assert abs(info[0]["outer_iters"] - 9) <= 2
