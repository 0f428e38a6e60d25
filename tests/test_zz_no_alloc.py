"""dg_vjp_noalloc, the reverse product for callers that cannot allocate
device memory, against dg_vjp through the C ABI: bitwise equal (the same
kernels with the buffers carved from the library's fixed device scratch), on
two calls in a row with the second on a smaller mesh (the scratch keeps the
first call's contents), for Navier-Stokes, blended Euler and blended
Navier-Stokes; a mesh whose buffers exceed the scratch is refused."""
import ctypes

import numpy as np
import pytest

from paper_2306_12891_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _noalloc(op, U, lam, out):
    P = ctypes.c_void_p
    return op.raw_call("dg_vjp_noalloc", P(U.data_ptr()), P(lam.data_ptr()), P(out.data_ptr()))


def _case(torch, dg, N, nelem, eq, blending, seed):
    lo, hi = (0.0, 0.0, 0.0), (1.0, 0.25, 0.25)
    if blending:
        op = dg.DG(nelem, N, gamma=1.4, mu=2e-3 if eq else 0.0, lo=lo, hi=hi, equations=eq, vol_flux=dg.KG,
                   surf_flux=dg.LLF, blending=1, fv_recon=dg.FV_MINMOD)
        # density and pressure jump inside an element, so the indicator fires
        X, _, _ = I.node_coordinates(N, nelem, lo, hi)
        left = X < 0.53
        one = np.ones_like(X)
        U = I.from_primitive(np.where(left, 1.0, 0.125), 0 * one, 0 * one, 0 * one, np.where(left, 1.0, 0.1), 1.4)
        U = U * (1.0 + 1e-3 * I.random_directions(U.shape, seed))
    else:
        op = dg.DG(nelem, N, gamma=1.4, mu=2e-2, equations=eq, vol_flux=dg.PI, surf_flux=dg.ROE)
        U = I.random_smooth(N, nelem, seed=seed, noise=0.02)
    Ud = torch.from_numpy(U).cuda()
    lam = torch.from_numpy(I.random_directions(U.shape, seed + 1)).cuda()
    return op, Ud, lam


@pytest.mark.parametrize("eq,blending", [(1, 0), (0, 1), (1, 1)])
def test_noalloc_equals_vjp_on_two_calls(torch_cuda, eq, blending):
    import torch

    from paper_2306_12891_amd import dg
    for N, nelem, seed in ((5, (6, 3, 2), 31), (3, (4, 2, 1), 33)):  # the second call: a smaller mesh
        op, U, lam = _case(torch, dg, N, nelem, eq, blending, seed)
        if blending:
            assert float((op.alpha(U) > 0).double().sum().item()) >= 1
        out = torch.full_like(U, float("nan"))
        assert _noalloc(op, U, lam, out) == dg.DG_OK
        ref = op.vjp(U, lam)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (N, nelem)
        # the binding's method is the same call
        out2 = torch.empty_like(U)
        assert torch.equal(op.vjp_noalloc(U, lam, out2), ref)
        op.close()


def test_noalloc_refuses_meshes_beyond_the_scratch(torch_cuda):
    import torch

    from paper_2306_12891_amd import dg
    N, nelem = 7, (16, 16, 24)  # face buffer 6144 x 6 x 4 x 64 doubles = 75 MB > 64 MiB
    op = dg.DG(nelem, N, gamma=1.4, mu=1e-3, equations=dg.NS, vol_flux=dg.PI, surf_flux=dg.ROE)
    U = torch.from_numpy(I.freestream(N, nelem)).cuda()
    out = torch.empty_like(U)
    assert _noalloc(op, U, U.clone(), out) == dg.DG_EINVAL
    assert "scratch" in op.last_error()
    op.close()
