"""Failure handling and the solve's phase timers, through the C-ABI.

* A Dirichlet system made singular by putting k^2 on a discrete eigenvalue
  (the sine-mode eigenvalues of the 5-point Laplacian): the solve must stop at
  maxit with HELM_ENOCONV and a finite last iterate, not with NaN.
* A 5 x 5 grid (9 unknowns) with tolerance 0: the Krylov space is exhausted
  within 9 steps, the Arnoldi norms fall to rounding level (the breakdown
  region), and the solve must still end with a finite x whose true residual is
  at rounding level.
* HELM_ENOMEM from helm_create when the first device buffer cannot exist (a
  1.1 TB level, refused by hipMalloc at once), with nothing left allocated.
* helm_solve_info's phase times: setup, coarse solves and fine V-cycles.
"""
import math

import numpy as np
import pytest

from paper_2308_06152_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def H():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2308_06152_amd import helmdefl
    helmdefl.load()
    return helmdefl


def test_singular_dirichlet_system_reports_noconv(H, ora):
    n = 33
    h = 1.0 / (n - 1)
    # lambda_11 of -Lap_h on the interior nodes (the Appendix B formula)
    k = math.sqrt(4.0 / h**2 * (2.0 * math.sin(math.pi * h / 2) ** 2))
    P = ora.Problem(n, n, h, h, bc=ora.BC_DIRICHLET, kconst=k)
    phi = np.outer(np.sin(np.pi * np.arange(n) * h), np.sin(np.pi * np.arange(n) * h))
    Aphi = ora.helm_apply(P, phi.astype(np.complex128))
    assert np.linalg.norm(Aphi) <= 1e-9 * np.linalg.norm(phi) / h**2  # singular indeed
    S = H.Solver(n, n, h, h, H.BC_DIRICHLET, kconst=k, maxit=25, restart=10)
    b = inputs.point_source(n, n, h, h, 10, 20)
    x = torch.zeros_like(torch.from_numpy(b)).cuda()
    with pytest.raises(H.HelmError) as e:
        S.solve(torch.from_numpy(b).cuda(), x, raise_on_noconv=True)
    assert e.value.code == H.HELM_ENOCONV
    xs, info = S.solve(torch.from_numpy(b).cuda())
    assert not info[0]["converged"] and info[0]["outer_iters"] == 25
    assert torch.isfinite(xs).all()
    assert math.isfinite(info[0]["relres"]) and info[0]["relres"] > 1e-6
    S.close()


@pytest.mark.parametrize("bc", [0, 1])
def test_tiny_grid_runs_into_breakdown_finitely(H, ora, bc):
    n, k = 5, 3.0
    h = 1.0 / (n - 1)
    S = H.Solver(n, n, h, h, bc, kconst=k, tol=0.0, maxit=30, restart=30,
                 coarse_mode=H.CMODE_FIXED, coarse_iters=3)
    b = inputs.random_complex((n, n), 17)
    x, info = S.solve(torch.from_numpy(b).cuda())
    assert torch.isfinite(x).all()
    P = ora.Problem(n, n, h, h, bc=bc, kconst=k)
    xg = x.cpu().numpy()
    bm = b * (ora.helm_apply(P, np.ones_like(b)) != 0) if bc == 0 else b
    r = ora.helm_apply(P, xg) - bm
    assert np.linalg.norm(r) / np.linalg.norm(bm) <= 1e-10
    assert info[0]["outer_iters"] <= 30
    S.close()


def test_create_reports_enomem(H):
    n = 524289  # level 1 alone would take 1.1 TB
    with pytest.raises(H.HelmError) as e:
        H.Solver(n, n, 1.0 / (n - 1), 1.0 / (n - 1), H.BC_SOMMERFELD, kconst=1.0)
    assert e.value.code == H.HELM_ENOMEM
    # the device is still usable
    S = H.Solver(65, 65, 1 / 64, 1 / 64, H.BC_SOMMERFELD, kconst=10.0)
    y = S.apply(torch.ones((65, 65), dtype=torch.complex128, device="cuda"))
    torch.cuda.synchronize()
    assert torch.isfinite(y).all()
    S.close()


def test_solve_info_phase_times(H):
    w = inputs.scaled_plain(129, 40.0)
    S = H.Solver(w.nx, w.ny, w.hx, w.hy, w.bc, kconst=w.kconst, coarse_op=w.coarse_op,
                 coarse_mode=H.CMODE_TOL, coarse_tol=0.1, coarse_iters=300)
    b = torch.from_numpy(np.stack([w.rhs(), 2 * w.rhs()])).cuda()
    for batch in (0, 1):
        S2 = H.Solver(w.nx, w.ny, w.hx, w.hy, w.bc, kconst=w.kconst, coarse_op=w.coarse_op,
                      coarse_mode=H.CMODE_TOL, coarse_tol=0.1, coarse_iters=300, batch=batch)
        _, info = S2.solve(b)
        for i in info:
            assert i["converged"]
            assert i["t_setup_ms"] > 0
            assert i["t_coarse_ms"] > 0 and i["t_vcycle_ms"] > 0
            assert i["t_vcycle_ms"] < i["t_coarse_ms"]  # the inner solves dominate
            assert i["t_coarse_ms"] + i["t_vcycle_ms"] <= 1.05 * i["t_solve_ms"] + 0.5
        S2.close()
    S.close()
