"""cslp_vcycle_noalloc (the V-cycle entry point that allocates nothing: its
level buffers live in the library's fixed device scratch) against cslp_vcycle
on the same handle, through the C-ABI.

Two calls in a row share the scratch: the first on a larger grid, the second
on a smaller one (whose levels then sit on memory the first call left
written), then the larger again.  Each must match cslp_vcycle's result within
the 1e-12 FP64 bar, and equal its single-right-hand-side cycle bit for bit
(the same kernels on other buffers), in FP64 and in the mixed-precision form;
a grid whose levels exceed the scratch is refused before anything is
launched.
"""
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


def solver(H, nx, ny, bc, prec, kvar):
    h = 1.0 / (max(nx, ny) - 1)
    if kvar:
        k = torch.from_numpy(inputs.random_field(ny, nx, 10.0, 40.0, seed=nx + 3 * ny)).cuda()
        return H.Solver(nx, ny, h, h, bc, k=k, precision=prec)
    return H.Solver(nx, ny, h, h, bc, kconst=25.0, precision=prec)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
def test_noalloc_vcycle_matches_cslp_vcycle(H, prec):
    cases = [(513, 385, 1, True), (97, 161, 0, False), (513, 385, 1, True)]
    handles = {}
    for q, (nx, ny, bc, kvar) in enumerate(cases):
        print(f"noalloc case {q}: {nx}x{ny} bc={bc} vark={kvar} prec={prec}", flush=True)
        key = (nx, ny)
        if key not in handles:
            handles[key] = solver(H, nx, ny, bc, prec, kvar)
        S = handles[key]
        r = torch.from_numpy(inputs.random_complex((2, ny, nx), 500 + q)).cuda()
        # two right-hand sides: cslp_vcycle takes them in one batched pass,
        # the no-allocation variant one after another
        want = S.vcycle(r)
        want1 = torch.stack([S.vcycle(r[0].contiguous()), S.vcycle(r[1].contiguous())])
        got = torch.full_like(r, complex(float("nan"), float("nan")))
        S.vcycle_noalloc(r, got)
        torch.cuda.synchronize()
        w, w1, g = want.cpu().numpy(), want1.cpu().numpy(), got.cpu().numpy()
        assert np.all(np.isfinite(g))
        for b in range(2):
            err = np.linalg.norm(g[b] - w[b]) / np.linalg.norm(w[b])
            assert err <= 1e-12, (b, err)
        # the single-right-hand-side cycle on the handle's own buffers: the
        # same kernels, bit for bit
        assert np.array_equal(g, w1)
    for S in handles.values():
        S.close()


def test_noalloc_rejects_levels_beyond_the_scratch(H):
    n = 4097
    S = H.Solver(n, n, 1.0 / (n - 1), 1.0 / (n - 1), H.BC_SOMMERFELD, kconst=100.0)
    r = torch.zeros((n, n), dtype=torch.complex128, device="cuda")
    z = torch.zeros_like(r)
    with pytest.raises(H.HelmError) as e:
        S.vcycle_noalloc(r, z)
    assert e.value.code == H.HELM_ESCRATCH
    torch.cuda.synchronize()
    assert float(z.abs().max()) == 0.0  # nothing was launched
    S.close()
