"""Captured coarse-GMRES steps (opts.graphs = 1) against direct launches
(graphs = 0): every replay must give the direct result bit for bit, since the
graph holds the same kernels, with the same arguments, in the same order."""
import numpy as np
import pytest
import torch

from paper_2308_06152_amd import inputs

from test_gpu_parity import H, dev, host, make_pair  # noqa: F401

pytestmark = pytest.mark.gpu

# (name, nx, ny, bc, kind of k, k value / range, coarse operator)
GCASES = [
    ("som129_redglk2", 129, 129, 1, "const", 25.0, 1),
    ("dir129_galerkin", 129, 129, 0, "const", 20.0, 0),
    ("som133x69_vark_galerkin", 133, 69, 1, "var", (10.0, 40.0), 0),
    ("som97x161_redo4", 97, 161, 1, "const", 30.0, 3),
]


@pytest.mark.parametrize("case", GCASES, ids=[c[0] for c in GCASES])
def test_graph_coarse_solve_replays_match_direct(H, ora, case):
    kw = dict(coarse_mode=1, coarse_iters=12, coarse_restart=5)
    Sg, _ = make_pair(H, ora, case, graphs=1, **kw)
    Sd, _ = make_pair(H, ora, case, graphs=0, **kw)
    nxc, nyc = Sg.coarse_dims()
    v1 = inputs.random_complex((nyc, nxc), 211)
    want, itd = Sd.coarse_solve(dev(v1))
    want = host(want)
    for rep in range(3):
        got, itg = Sg.coarse_solve(dev(v1))
        assert itg == itd
        assert np.array_equal(host(got), want), rep
        # eager work and a synchronisation between replays
        x = dev(inputs.random_complex((Sg.grid.ny, Sg.grid.nx), 212 + rep))
        Sg.apply(x)
        torch.cuda.synchronize()


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_graph_solve_matches_direct(H, ora, precision):
    case = ("som129", 129, 129, 1, "const", 30.0, 1)
    kw = dict(coarse_mode=2, coarse_tol=0.1, coarse_iters=300, coarse_restart=15,
              precision=precision)
    Sg, _ = make_pair(H, ora, case, graphs=1, **kw)
    Sd, _ = make_pair(H, ora, case, graphs=0, **kw)
    nx, ny, hx, hy = inputs.unit_square(129)
    b = inputs.point_source(nx, ny, hx, hy, 64, 64)
    xd, idd = Sd.solve(dev(b))
    for rep in range(2):
        xg, ig = Sg.solve(dev(b))
        assert ig[0]["outer_iters"] == idd[0]["outer_iters"]
        assert ig[0]["inner_iters_total"] == idd[0]["inner_iters_total"]
        assert ig[0]["converged"] and ig[0]["relres"] <= 1e-6
        assert np.array_equal(host(xg), host(xd)), rep


@pytest.mark.parametrize("case", GCASES[:3], ids=[c[0] for c in GCASES[:3]])
def test_batched_graph_chunks_match_direct(H, ora, case):
    """Batched solves with the coarse GMRES steps replayed in captured chunks
    against direct launches: right-hand sides that converge at different
    inner and outer iterations (the chunks run on past a convergence, and a
    new active mask reaches later chunks), three replays with eager work and
    synchronisations in between, each bit for bit equal to the direct solve."""
    kw = dict(coarse_mode=2, coarse_tol=0.1, coarse_iters=300, coarse_restart=11, restart=30)
    Sg, P = make_pair(H, ora, case, graphs=1, **kw)
    Sd, _ = make_pair(H, ora, case, graphs=0, **kw)
    nx, ny = P.nx, P.ny
    b = np.stack([inputs.point_source(nx, ny, P.hx, P.hy, nx // 2, ny // 2),
                  inputs.random_complex((ny, nx), 215),
                  inputs.point_source(nx, ny, P.hx, P.hy, 3, ny // 3),
                  np.zeros((ny, nx), complex)])
    xd, idd = Sd.solve(dev(b))
    xd = host(xd)
    assert len({i["inner_iters_total"] for i in idd[:3]}) > 1
    for rep in range(3):
        xg, ig = Sg.solve(dev(b))
        for q in range(len(b)):
            assert ig[q]["outer_iters"] == idd[q]["outer_iters"]
            assert ig[q]["inner_iters_total"] == idd[q]["inner_iters_total"]
        assert np.array_equal(host(xg), xd), rep
        # eager work and a synchronisation between replays
        Sg.apply(dev(b[1]))
        torch.cuda.synchronize()
    # batched deflation with a fixed inner count, replayed
    Sgf, _ = make_pair(H, ora, case, graphs=1, coarse_mode=1, coarse_iters=9, coarse_restart=4)
    Sdf, _ = make_pair(H, ora, case, graphs=0, coarse_mode=1, coarse_iters=9, coarse_restart=4)
    v = np.stack([inputs.random_complex((ny, nx), 216 + q) for q in range(3)])
    want = host(Sdf.deflate(dev(v), 2))
    for rep in range(2):
        assert np.array_equal(host(Sgf.deflate(dev(v), 2)), want), rep
