"""Adjoint state on the GPU against the oracle: receiver residuals, the
adjoint solve (complex-symmetric scaling + forward solve), the gradient
kernel, and the whole misfit gradient through torch.autograd, checked against
the oracle's direct-solve gradient and against central differences."""
import numpy as np
import pytest

from paper_2308_06152_amd import inputs

from test_gpu_parity import H, dev, host, rel  # noqa: F401

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TIGHT = dict(coarse_mode=2, coarse_tol=0.1, coarse_iters=300, coarse_restart=15, restart=50,
             tol=1e-11, maxit=400)


def _solver(H, nx, ny, h, bc, k, **kw):
    o = dict(TIGHT)
    o.update(kw)
    return H.Solver(nx, ny, h, h, bc, k=dev(k), coarse_op=1, **o)


@pytest.mark.parametrize("bc", [0, 1])
def test_receivers_match_definition(H, ora, bc):
    nx, ny, h = 65, 33, 1 / 64
    k = inputs.random_field(ny, nx, 5.0, 9.0, seed=40)
    S = _solver(H, nx, ny, h, bc, k)
    B = 3
    u = np.stack([inputs.random_complex((ny, nx), 41 + q) for q in range(B)])
    rec = np.array([j * nx + i for i, j in ((3, 30), (10, 30), (40, 2), (64, 16))], np.int32)
    d = inputs.random_complex((B, len(rec)), 44)
    res, f, J = S.receivers(torch.from_numpy(rec).cuda(), dev(u), dev(d))
    res, f, J = host(res), host(f), host(J)
    want = u.reshape(B, -1)[:, rec] - d
    assert np.array_equal(res, want)
    fw = np.zeros((B, ny * nx), complex)
    fw[:, rec] = want
    assert np.array_equal(f.reshape(B, -1), fw)
    assert np.allclose(J, 0.5 * (np.abs(want) ** 2).sum(axis=1), rtol=1e-14, atol=0)
    # duplicates and out-of-range nodes are rejected before any launch
    for bad in (np.array([5, 5], np.int32), np.array([-1], np.int32),
                np.array([nx * ny], np.int32)):
        with pytest.raises(H.HelmError) as e:
            S.receivers(torch.from_numpy(bad).cuda(), dev(u), dev(d[:, :len(bad)]))
        assert e.value.code == H.HELM_EINVAL


@pytest.mark.parametrize("bc", [0, 1])
def test_gradient_kernel_parity(H, ora, bc):
    nx, ny, h, omega = 97, 49, 1 / 96, 7.0
    s = inputs.random_field(ny, nx, 0.4, 2.5, seed=45)
    k = omega * np.sqrt(s)
    S = _solver(H, nx, ny, h, bc, k)
    P = ora.Problem(nx, ny, h, h, bc=bc, k=k)
    B = 2
    u = np.stack([inputs.random_complex((ny, nx), 46 + q) for q in range(B)])
    lam = np.stack([inputs.random_complex((ny, nx), 48 + q) for q in range(B)])
    g = host(S.gradient_s(omega, dev(u), dev(lam)))
    want = sum(ora.grad_s(P, omega, u[q], lam[q]) for q in range(B))
    assert rel(g, want) <= 1e-12
    # accumulation into an existing gradient
    g2 = host(S.gradient_s(omega, dev(u), dev(lam), g=dev(g)))
    assert rel(g2, 2 * want) <= 1e-12


@pytest.mark.parametrize("bc,nrhs", [(1, 1), (1, 3), (0, 2)])
def test_adjoint_solve_parity(H, ora, bc, nrhs):
    nx, ny, h = 129, 65, 1 / 128
    k = inputs.random_field(ny, nx, 10.0, 30.0, seed=50)
    S = _solver(H, nx, ny, h, bc, k)
    P = ora.Problem(nx, ny, h, h, bc=bc, k=k)
    f = np.stack([inputs.random_complex((ny, nx), 51 + q) for q in range(nrhs)])
    if bc == 0:
        f[:, 0, :] = f[:, -1, :] = f[:, :, 0] = f[:, :, -1] = 0
    lam, info = S.adjoint_solve(dev(f))
    lam = host(lam)
    assert all(i["converged"] for i in info)
    for q in range(nrhs):
        want = ora.adjoint_solve(P, f[q])
        assert rel(lam[q], want) <= 1e-8
        r = ora.helm_apply_adjoint(P, lam[q]) - f[q]
        assert np.linalg.norm(r) <= 1e-9 * np.linalg.norm(f[q])


def _case(n=129):
    c = inputs.adjoint_case(n, (n - 1) // 2 + 1, nshot=4, nrec=32)
    c["omega"] = 2 * np.pi * c["freq"]
    return c


def _oracle_misfit_gradient(ora, c, s):
    nx, ny, h, omega = c["nx"], c["ny"], c["h"], c["omega"]
    P = ora.Problem(nx, ny, h, h, bc=1, k=omega * np.sqrt(s))
    Pt = ora.Problem(nx, ny, h, h, bc=1, k=omega * np.sqrt(c["s_true"]))
    J, g = 0.0, np.zeros((ny, nx))
    for q in range(len(c["sources"])):
        u = ora.direct_solve(P, c["sources"][q])
        d = ora.direct_solve(Pt, c["sources"][q]).ravel()[c["rec"]]
        r = u.ravel()[c["rec"]] - d
        J += 0.5 * np.vdot(r, r).real
        f = np.zeros(nx * ny, complex)
        f[c["rec"]] = r
        g += ora.grad_s(P, omega, u, ora.adjoint_solve(P, f.reshape(ny, nx)))
    return J, g


def _observed(H, c):
    """d_obs = R u_true from a tight GPU solve with the true model."""
    nx, ny, h = c["nx"], c["ny"], c["h"]
    S = _solver(H, nx, ny, h, 1, c["omega"] * np.sqrt(c["s_true"]))
    u, _ = S.solve(dev(c["sources"]))
    return u.reshape(len(c["sources"]), -1)[:, torch.from_numpy(c["rec"]).long().cuda()]


def test_autograd_gradient_matches_oracle(H, ora):
    from paper_2308_06152_amd import adjoint
    c = _case()
    d_obs = _observed(H, c).contiguous()
    s = dev(c["s_init"]).requires_grad_(True)
    J = adjoint.misfit(s, c["omega"], (c["nx"], c["ny"], c["h"], c["h"], 1),
                       dev(c["sources"]), torch.from_numpy(c["rec"]).cuda(), d_obs,
                       coarse_op=1, **TIGHT)
    J.backward()
    Jo, go = _oracle_misfit_gradient(ora, c, c["s_init"])
    assert abs(J.item() - Jo) <= 1e-7 * Jo
    assert rel(host(s.grad), go) <= 1e-6


def test_autograd_gradient_matches_central_differences(H, ora):
    from paper_2308_06152_amd import adjoint
    c = _case()
    d_obs = _observed(H, c).contiguous()
    grid = (c["nx"], c["ny"], c["h"], c["h"], 1)
    src, rec = dev(c["sources"]), torch.from_numpy(c["rec"]).cuda()

    def J(sv, grad=False):
        s = dev(sv).requires_grad_(grad)
        val = adjoint.misfit(s, c["omega"], grid, src, rec, d_obs, coarse_op=1, **TIGHT)
        if grad:
            val.backward()
            return val.item(), host(s.grad)
        return val.item()

    J0, g = J(c["s_init"], grad=True)
    rng = np.random.default_rng(52)
    cells = [(int(rng.integers(0, c["nx"])), int(rng.integers(0, c["ny"]))) for _ in range(5)]
    cells += [(0, 10), (c["nx"] - 1, c["ny"] - 1), (40, c["ny"] - 7)]
    gscale = np.abs(g).max()
    for i, j in cells:
        eps = 1e-4 * c["s_init"][j, i]
        sp, sm = c["s_init"].copy(), c["s_init"].copy()
        sp[j, i] += eps
        sm[j, i] -= eps
        fd = (J(sp) - J(sm)) / (2 * eps)
        assert abs(fd - g[j, i]) <= 1e-4 * max(abs(fd), 1e-2 * gscale), (i, j, fd, g[j, i])


def test_recomputed_fields_give_the_stored_gradient(H, ora):
    """The recompute path (wavefields not kept, solved again in the backward
    pass): with the sources in one group the same batched solves run, so J and
    the gradient equal the stored-field ones bit for bit; in groups of one or
    two sources the Krylov sums are split differently, which moves them by
    rounding only."""
    from paper_2308_06152_amd import adjoint
    c = _case()
    d_obs = _observed(H, c).contiguous()
    grid = (c["nx"], c["ny"], c["h"], c["h"], 1)
    src, rec = dev(c["sources"]), torch.from_numpy(c["rec"]).cuda()

    def run(**kw):
        s = dev(c["s_init"]).requires_grad_(True)
        J = adjoint.misfit(s, c["omega"], grid, src, rec, d_obs, coarse_op=1, **TIGHT, **kw)
        J.backward()
        return J.item(), host(s.grad)

    J0, g0 = run()
    J1, g1 = run(max_field_bytes=0)
    assert J1 == J0 and np.array_equal(g1, g0)
    for group in (1, 2):
        Jg, gg = run(max_field_bytes=0, shot_group=group)
        assert abs(Jg - J0) <= 1e-9 * J0
        assert rel(gg, g0) <= 1e-8


def test_full_size_gradient_central_differences(H, ora):
    """The adjoint workload at full size: 1025 x 513 (h = 10 m), 16 shots and
    256 receivers at 10 Hz.  The autograd gradient against central differences
    of J at 20 seeded cells (each a pair of batched 16-shot solves)."""
    from paper_2308_06152_amd import adjoint
    c = inputs.adjoint_case()
    assert (c["nx"], c["ny"], len(c["sources"]), len(c["rec"])) == (1025, 513, 16, 256)
    assert abs(c["freq"] - 10.0) < 1e-12
    c["omega"] = 2 * np.pi * c["freq"]
    d_obs = _observed(H, c).contiguous()
    grid = (c["nx"], c["ny"], c["h"], c["h"], 1)
    src, rec = dev(c["sources"]), torch.from_numpy(c["rec"]).cuda()
    opts = dict(TIGHT)

    def J(sv, grad=False):
        s = dev(sv).requires_grad_(grad)
        val = adjoint.misfit(s, c["omega"], grid, src, rec, d_obs, coarse_op=1, **opts)
        if grad:
            val.backward()
            return val.item(), host(s.grad)
        return val.item()

    J0, g = J(c["s_init"], grad=True)
    assert np.all(np.isfinite(g)) and J0 > 0
    rng = np.random.default_rng(230806152 + 5)
    cells = [(int(rng.integers(0, c["nx"])), int(rng.integers(0, c["ny"]))) for _ in range(20)]
    gscale = np.abs(g).max()
    for n, (i, j) in enumerate(cells):
        eps = 1e-4 * c["s_init"][j, i]
        sp, sm = c["s_init"].copy(), c["s_init"].copy()
        sp[j, i] += eps
        sm[j, i] -= eps
        fd = (J(sp) - J(sm)) / (2 * eps)
        print(f"cell {n} ({i},{j}): fd {fd:.6e} adjoint {g[j, i]:.6e}", flush=True)
        assert abs(fd - g[j, i]) <= 1e-4 * max(abs(fd), 1e-2 * gscale), (i, j, fd, g[j, i])


def _dscale(nx, ny):
    """D of the complex-symmetric scaling (Sommerfeld grid): 1/2 per direction
    in which a boundary ghost was eliminated (edges 1/2, corners 1/4)."""
    dx = np.ones(nx)
    dy = np.ones(ny)
    dx[[0, -1]] = 0.5
    dy[[0, -1]] = 0.5
    return dy[:, None] * dx[None, :]


def _oracle_adjoint_iterative(ora, P, f, **kw):
    """lambda = A^-H f from the oracle's FGMRES: A^H = D conj(A) D^-1, so
    lambda = D conj(A^-1 conj(D^-1 f))."""
    D = _dscale(P.nx, P.ny)
    y, info = ora.fgmres(P, np.conj(f / D), **kw)
    assert info.converged
    return D * np.conj(y)


def test_full_size_gradient_against_oracle(H, ora):
    """The adjoint workload at full size (1025 x 513, 256 receivers, 10 Hz),
    two of its shots: the autograd misfit and gradient against the oracle's,
    whose forward and adjoint solves are the oracle's own FGMRES to the same
    tolerance (its direct adjoint solve is meant for small grids; the
    iterative form is first checked against it on a small grid).  Measured:
    J equal to 11 digits, gradients equal to 3e-11."""
    from paper_2308_06152_amd import adjoint
    # the iterative adjoint against the direct one (129 x 65)
    cs = _case()
    Ps = ora.Problem(cs["nx"], cs["ny"], cs["h"], cs["h"], bc=1,
                     k=cs["omega"] * np.sqrt(cs["s_init"]), coarse_op=1,
                     coarse_mode=ora.CMODE_TOL, coarse_tol=0.1, coarse_restart=15)
    f = inputs.random_complex((cs["ny"], cs["nx"]), 77)
    lam_it = _oracle_adjoint_iterative(ora, Ps, f, restart=50, tol=1e-12, maxit=400)
    assert rel(lam_it, ora.adjoint_solve(Ps, f)) <= 1e-9
    # full size, shots 0 and 1
    c = inputs.adjoint_case()
    c["omega"] = 2 * np.pi * c["freq"]
    nsh = 2
    d_obs = _observed(H, c)[:nsh].contiguous()
    grid = (c["nx"], c["ny"], c["h"], c["h"], 1)
    src, rec = dev(c["sources"][:nsh]), torch.from_numpy(c["rec"]).cuda()
    s = dev(c["s_init"]).requires_grad_(True)
    J = adjoint.misfit(s, c["omega"], grid, src, rec, d_obs, coarse_op=1, **TIGHT)
    J.backward()
    g = host(s.grad)
    P = ora.Problem(c["nx"], c["ny"], c["h"], c["h"], bc=1, k=c["omega"] * np.sqrt(c["s_init"]),
                    coarse_op=1, coarse_mode=ora.CMODE_TOL, coarse_tol=0.1, coarse_restart=15)
    d = host(d_obs)
    Jo, go = 0.0, np.zeros((c["ny"], c["nx"]))
    for q in range(nsh):
        u, info = ora.fgmres(P, c["sources"][q], restart=50, tol=1e-11, maxit=400)
        assert info.converged
        r = u.ravel()[c["rec"]] - d[q]
        Jo += 0.5 * np.vdot(r, r).real
        fq = np.zeros(c["nx"] * c["ny"], complex)
        fq[c["rec"]] = r
        lam = _oracle_adjoint_iterative(ora, P, fq.reshape(c["ny"], c["nx"]), restart=50,
                                        tol=1e-11, maxit=400)
        go += ora.grad_s(P, c["omega"], u, lam)
        print(f"full-size adjoint, shot {q}: oracle forward {info.iters} outer", flush=True)
    dg = rel(g, go)
    print(f"full-size adjoint (2 shots): J GPU {J.item():.10e} oracle {Jo:.10e}; "
          f"||g - g_oracle|| / ||g_oracle|| = {dg:.3e}")
    assert abs(J.item() - Jo) <= 1e-7 * Jo
    assert dg <= 1e-6
