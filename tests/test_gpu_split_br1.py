"""Split BR1 lifting (options lifting = LIFT_SPLIT) against the FP64 oracle.

The split scheme evaluates the same Navier-Stokes operator as the two-pass
lifting, with the interface values q* = (q- + q+)/2 of the BR1 gradient (the
standard lifting, which the paper leaves open) taken apart into each element's
own half and the rest, so
it must meet the same bar: single evaluations per variable to 1e-12 of
max(max |U_t|, S_v), rollouts to 1e-12 of max |U_v| (the helpers of the
parity tests).  The rest is added by the stage kernel from the face states
and, at the edges of a face, from the diagonal elements, whose coordinates
wrap around the periodic box: meshes with one or two elements along a
direction, anisotropic cells and every degree cover those index paths.
Within a Runge-Kutta step the stage kernel writes the own part of its output
for the next stage, so a step lifts once; n steps in one call equal n calls
of one step bitwise, and rk_step_record equals rk_step bitwise.
"""
import numpy as np
import pytest

from paper_2306_12891_amd import inputs as I
from test_gpu_parity import G, TWO_PI, assert_state_close, assert_ut_close, gpu_ut

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def make_split(orc, N, nelem, lo, hi, vf, sf, mu, lifting=1):
    from paper_2306_12891_amd import dg
    s = orc.Setup(N=N, nelem=nelem, lo=lo, hi=hi, equations=1, vol_flux=vf, surf_flux=sf, mu=mu)
    op = dg.DG(nelem, N, gamma=G, mu=mu, lo=lo, hi=hi, equations=dg.NS, vol_flux=vf, surf_flux=sf,
               lifting=lifting)
    return s, op


@pytest.mark.parametrize("vf,sf", [(1, 1), (0, 0), (3, 2), (2, 1)])
@pytest.mark.parametrize("N", range(1, 8))
def test_split_time_derivative(orc, torch_cuda, N, vf, sf):
    nelem, lo, hi = (3, 2, 2), (0.0, 0.0, 0.0), (2.0, 1.5, 1.0)
    s, op = make_split(orc, N, nelem, lo, hi, vf, sf, 2e-2)
    U = I.random_smooth(N, nelem, lo, hi, seed=150 + N + 11 * vf, noise=0.02)
    assert_ut_close(gpu_ut(torch_cuda, op, U), orc.time_derivative(s, U), U, N, nelem, lo, hi)


@pytest.mark.parametrize("nelem", [(1, 1, 1), (1, 2, 3), (2, 1, 2), (4, 3, 1)])
def test_split_thin_periodic_meshes(orc, torch_cuda, nelem):
    """One or two elements along a direction: the neighbour and the diagonal
    element are the element itself or coincide."""
    N, lo, hi = 4, (0.0, -1.0, 0.5), (1.5, 1.0, 2.0)
    s, op = make_split(orc, N, nelem, lo, hi, 1, 1, 5e-2)
    U = I.random_smooth(N, nelem, lo, hi, seed=sum(nelem), noise=0.03)
    assert_ut_close(gpu_ut(torch_cuda, op, U), orc.time_derivative(s, U), U, N, nelem, lo, hi)


@pytest.mark.parametrize("N", [2, 3, 5, 7])
def test_split_rollout(orc, torch_cuda, N):
    """Runge-Kutta steps (the chained own parts) against the oracle, and the
    two-pass lifting on the GPU to the same bar."""
    import torch
    nelem, lo, hi = (3, 2, 3), (0.0, 0.0, 0.0), (TWO_PI, 1.5 * TWO_PI, TWO_PI)
    mu = 2e-2
    s, op = make_split(orc, N, nelem, lo, hi, 1, 1, mu)
    _, op2 = make_split(orc, N, nelem, lo, hi, 1, 1, mu, lifting=0)
    U0 = I.random_smooth(N, nelem, lo, hi, seed=40 + N, noise=0.01)
    Ud = torch.from_numpy(U0).cuda()
    dt = op.max_dt(Ud, 0.5)
    V = Ud.clone()
    op.rk_steps(Ud, dt, 3)
    op2.rk_steps(V, dt, 3)
    ref = orc.rk_steps(s, U0, dt, 3)
    got = Ud.cpu().numpy()
    assert_state_close(got, ref)
    assert_state_close(got, V.cpu().numpy())
    assert np.max(np.abs(ref - U0)) > 1e3 * 1e-12 * np.max(np.abs(U0))


def test_split_step_calls_agree_bitwise(orc, torch_cuda):
    """n steps in one call equal n calls of one step; rk_step_record advances
    U as rk_step does and records Y_0 = U_n; rk_step_vjp on the recomputed
    stages equals rk_step_vjp_recorded on the recorded ones."""
    import torch
    N, nelem = 5, (2, 3, 2)
    _, op = make_split(orc, N, nelem, (0, 0, 0), (TWO_PI,) * 3, 1, 1, 1e-2)
    U0 = torch.from_numpy(I.random_smooth(N, nelem, seed=12, noise=0.02)).cuda()
    dt = op.max_dt(U0, 0.5)
    a, b = U0.clone(), U0.clone()
    op.rk_steps(a, dt, 3)
    for _ in range(3):
        op.rk_step(b, dt)
    assert torch.equal(a, b)
    c = U0.clone()
    Y = torch.empty((5,) + tuple(U0.shape), dtype=torch.float64, device="cuda")
    op.rk_step_record(c, dt, Y)
    d = U0.clone()
    op.rk_step(d, dt)
    assert torch.equal(c, d) and torch.equal(Y[0], U0)
    w = torch.from_numpy(I.random_directions(U0.shape, 3)).cuda()
    assert torch.equal(op.rk_step_vjp(U0, dt, w), op.rk_step_vjp_recorded(Y, dt, w))


def test_split_switch_between_calls(orc, torch_cuda):
    """Switching the lifting scheme between calls of one context: each call
    starts from a lifting of its own state, so the results do not depend on
    what ran before."""
    import torch
    N, nelem = 3, (2, 2, 3)
    s, op = make_split(orc, N, nelem, (0, 0, 0), (TWO_PI,) * 3, 1, 1, 1e-2)
    U0 = torch.from_numpy(I.random_smooth(N, nelem, seed=21, noise=0.02)).cuda()
    dt = op.max_dt(U0, 0.5)
    a = U0.clone()
    op.rk_steps(a, dt, 2)
    op.set_options(lifting=0)
    b = U0.clone()
    op.rk_steps(b, dt, 2)
    op.set_options(lifting=1)
    c = U0.clone()
    op.rk_step(c, dt)
    op.time_derivative(U0 * 1.01)  # an unrelated evaluation between the steps
    op.rk_step(c, dt)
    assert torch.equal(a, c)
    assert_state_close(a.cpu().numpy(), b.cpu().numpy())


def test_split_not_used_where_unsupported(orc, torch_cuda):
    """The split option leaves the Euler operator, the eddy viscosity and
    the mixed operator on their usual path: bitwise the two-pass results."""
    import torch

    from paper_2306_12891_amd import dg
    N, nelem = 4, (2, 2, 2)
    U = torch.from_numpy(I.random_smooth(N, nelem, seed=8, noise=0.02)).cuda()
    for kw in ({"equations": dg.EULER}, {"equations": dg.NS, "Cs": 0.17},
               {"equations": dg.NS, "precision": dg.MIXED, "vol_flux": dg.PI}):
        a = dg.DG(nelem, N, gamma=G, mu=1e-2, lifting=1, **kw)
        b = dg.DG(nelem, N, gamma=G, mu=1e-2, lifting=0, **kw)
        assert torch.equal(a.time_derivative(U), b.time_derivative(U)), kw
