"""The fused tails of the V-cycle (opts.vc_tail > 0: the downward passes of
the last levels above the coarsest in one launch, the upward passes of the
small levels in another) against one launch per level (vc_tail = 0).
Both evaluate the same expressions in the same order at every node.  With a
constant k the smoother's coefficients of the interior come from the host and
the results agree bit for bit; with a variable k each kernel computes them per
node and the compiler may fuse their multiply-adds differently, so the bar is
rounding (1e-14 relative for a cycle, 1e-12 after a fixed number of GMRES
steps).  The oracle parity tests cover the fused path against the oracle (it
is on by default)."""
import numpy as np
import pytest
import torch

from paper_2308_06152_amd import inputs

from test_gpu_parity import H, dev, host, make_pair  # noqa: F401

pytestmark = pytest.mark.gpu

# (name, nx, ny, bc, kind of k, k value / range, coarse operator), coarsest nodes
TCASES = [
    (("dir129_k20", 129, 129, 0, "const", 20.0, 0), 0),        # 5 fused levels
    (("som257_k40", 257, 257, 1, "const", 40.0, 1), 0),        # 6 fused levels
    (("som257_k40_c1089", 257, 257, 1, "const", 40.0, 1), 1089),  # 2 fused levels
    (("som161_vark", 161, 161, 1, "var", (20.0, 60.0), 1), 0),  # variable k
    (("som97x161", 97, 161, 1, "const", 30.0, 0), 0),           # rectangular
    (("dir65x97_vark", 65, 97, 0, "var", (5.0, 25.0), 0), 0),   # ragged, Dirichlet, var k
]


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def same(got, want, case, bar):
    if case[4] == "var":
        assert rel(got, want) <= bar
    else:
        assert np.array_equal(got, want), np.abs(got - want).max()


def _pair(H, ora, case, coarsest, **kw):
    Sf, P = make_pair(H, ora, case, coarsest_nodes=coarsest, vc_tail=300000, **kw)
    Sl, _ = make_pair(H, ora, case, coarsest_nodes=coarsest, vc_tail=0, **kw)
    return Sf, Sl, P


@pytest.mark.parametrize("case,coarsest", TCASES, ids=[c[0][0] for c in TCASES])
def test_vcycle_fused_tail_matches_per_level(H, ora, case, coarsest):
    Sf, Sl, P = _pair(H, ora, case, coarsest)
    r = inputs.random_complex((P.ny, P.nx), 301)
    want = host(Sl.vcycle(dev(r)))
    for rep in range(2):
        same(host(Sf.vcycle(dev(r))), want, case, 1e-14)


@pytest.mark.parametrize("case,coarsest", TCASES, ids=[c[0][0] for c in TCASES])
def test_fused_tails_run(H, ora, case, coarsest):
    """The fused kernels really run for every case above: a cycle launches
    fewer downward and upward passes with the tails on (the timing hooks file
    a fused tail as one launch)."""
    Sf, Sl, P = _pair(H, ora, case, coarsest)
    r = dev(inputs.random_complex((P.ny, P.nx), 304))
    counts = {}
    for name, S in (("fused", Sf), ("per_level", Sl)):
        for kc in (H.K_VC_DOWN, H.K_VC_UP):
            S.timing_enable(kc, -1)
            S.vcycle(r)
            counts[name, kc] = S.timing_read()[0]
            S.timing_enable(-1, -1)
    nlev = Sl.num_levels()
    assert counts["per_level", H.K_VC_DOWN] == nlev - 1
    assert counts["per_level", H.K_VC_UP] == nlev - 1
    assert counts["fused", H.K_VC_DOWN] < nlev - 1
    assert counts["fused", H.K_VC_UP] < nlev - 1


@pytest.mark.parametrize("limit", [1, 100, 4225, 20000])
def test_vcycle_fused_tail_level_limits(H, ora, limit):
    case = ("som257_k40", 257, 257, 1, "const", 40.0, 1)
    Sf, P = make_pair(H, ora, case, coarsest_nodes=0, vc_tail=limit)
    Sl, _ = make_pair(H, ora, case, coarsest_nodes=0, vc_tail=0)
    r = inputs.random_complex((P.ny, P.nx), 302)
    assert np.array_equal(host(Sf.vcycle(dev(r))), host(Sl.vcycle(dev(r))))


@pytest.mark.parametrize("precision", [0, 1, 2])
@pytest.mark.parametrize("case,coarsest", TCASES[:2] + TCASES[3:4], ids=["dir129", "som257",
                                                                          "som161_vark"])
def test_coarse_solve_fused_tail_matches_per_level(H, ora, case, coarsest, precision):
    kw = dict(coarse_mode=1, coarse_iters=10, coarse_restart=6, precision=precision)
    Sf, Sl, _ = _pair(H, ora, case, coarsest, **kw)
    nxc, nyc = Sf.coarse_dims()
    v1 = inputs.random_complex((nyc, nxc), 303)
    want, itl = Sl.coarse_solve(dev(v1))
    got, itf = Sf.coarse_solve(dev(v1))
    assert itf == itl
    same(host(got), host(want), case, 1e-12)


def test_solve_fused_tail_matches_per_level(H, ora):
    case = ("som257_k40", 257, 257, 1, "const", 40.0, 1)
    Sf, Sl, _ = _pair(H, ora, case, 0)
    nx, ny, hx, hy = inputs.unit_square(257)
    b = inputs.point_source(nx, ny, hx, hy, 128, 128)
    xl, il = Sl.solve(dev(b))
    xf, iff = Sf.solve(dev(b))
    assert iff[0]["outer_iters"] == il[0]["outer_iters"]
    assert iff[0]["inner_iters_total"] == il[0]["inner_iters_total"]
    assert iff[0]["converged"]
    assert np.array_equal(host(xf), host(xl))


def test_vcycle_fused_tail_large_grid(H):
    """1025 x 1025 with the default coarsest grid: levels 513^2 .. 65^2 fused."""
    kc = 80.0
    Sf = H.Solver(1025, 1025, 1 / 1024, 1 / 1024, 1, kconst=kc, vc_tail=300000)
    Sl = H.Solver(1025, 1025, 1 / 1024, 1 / 1024, 1, kconst=kc, vc_tail=0)
    assert Sf.num_levels() == 6
    r = dev(inputs.random_complex((1025, 1025), 304))
    a = Sf.vcycle(r)
    b = Sl.vcycle(r)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
