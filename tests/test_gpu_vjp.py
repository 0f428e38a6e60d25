"""Reverse mode of the HIP operator (dg_vjp, rk_step_vjp, the torch autograd
functions and the checkpointed rollout) against the oracle's forward-mode
dual numbers (the oracle has no transpose: the identity <w, J v> = <J^T w, v>
checks one against the other), a full Jacobian on a one-element mesh, and
central finite differences of a rollout functional."""
import ctypes
import math

import numpy as np
import pytest

from paper_2306_12891_amd import inputs as I

pytestmark = pytest.mark.gpu

G = 1.4
TWO_PI = 2 * math.pi


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def make(orc, N, nelem, eq, vf, sf, mu=2e-2, lo=(0, 0, 0), hi=(TWO_PI,) * 3):
    from paper_2306_12891_amd import dg
    s = orc.Setup(N=N, nelem=nelem, lo=lo, hi=hi, equations=eq, vol_flux=vf, surf_flux=sf, mu=mu)
    op = dg.DG(nelem, N, gamma=G, mu=mu, lo=lo, hi=hi, equations=eq, vol_flux=vf, surf_flux=sf)
    return s, op


def dot_check(a, b, scale, tol):
    assert abs(a - b) <= tol * scale, (a, b, abs(a - b) / scale)


@pytest.mark.parametrize("eq,vf,sf", [(0, 0, 0), (0, 1, 1), (0, 3, 2), (0, 0, 1), (1, 1, 1), (1, 0, 0), (1, 3, 2)])
@pytest.mark.parametrize("N", [2, 3, 5])
def test_vjp_dot_product(orc, torch_cuda, eq, vf, sf, N):
    nelem = (3, 2, 2)
    s, op = make(orc, N, nelem, eq, vf, sf)
    U = I.random_smooth(N, nelem, seed=400 + N, noise=0.02)
    v = I.random_directions(U.shape, 0)
    w = I.random_directions(U.shape, 1)
    _, Jv = orc.jvp(s, U, v)
    JTw = op.vjp(torch_cuda.from_numpy(U).cuda(), torch_cuda.from_numpy(w).cuda()).cpu().numpy()
    a, b = np.sum(w * Jv), np.sum(JTw * v)
    dot_check(a, b, np.sum(np.abs(w * Jv)), 1e-12)


@pytest.mark.parametrize("eq,vf,sf", [(0, 1, 1), (1, 1, 1), (1, 0, 0)])
def test_full_jacobian_one_element(orc, torch_cuda, eq, vf, sf):
    """N = 2 on a self-periodic element: all 135 columns J e_k from the oracle's
    dual numbers against all 135 products J^T e_k (the rows of J) from the GPU."""
    import torch
    N, nelem = 2, (1, 1, 1)
    s, op = make(orc, N, nelem, eq, vf, sf, mu=5e-2)
    U = I.random_smooth(N, nelem, seed=11, noise=0.05)
    n = U.size
    J = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        J[:, k] = orc.jvp(s, U, e.reshape(U.shape))[1].ravel()
    Ud = torch.from_numpy(U).cuda()
    JT = np.zeros((n, n))
    for k in range(n):
        e = torch.zeros(U.shape, dtype=torch.float64, device="cuda")
        e.view(-1)[k] = 1.0
        JT[k] = op.vjp(Ud, e).cpu().numpy().ravel()  # J^T e_k = row k of J
    assert np.max(np.abs(JT - J)) <= 1e-12 * np.max(np.abs(J))


@pytest.mark.parametrize("eq,vf,sf", [(1, 1, 1), (0, 0, 0)])
def test_rk_step_vjp_dot_product(orc, torch_cuda, eq, vf, sf):
    import torch
    N, nelem = 3, (2, 3, 2)
    s, op = make(orc, N, nelem, eq, vf, sf)
    U = I.random_smooth(N, nelem, seed=21, noise=0.01)
    v = I.random_directions(U.shape, 2)
    w = I.random_directions(U.shape, 3)
    dt = 0.5 * orc.max_dt(s, U, 0.5)
    _, Jv = orc.rk_jvp(s, U, v, dt, 1)
    Ud, wd = torch.from_numpy(U).cuda(), torch.from_numpy(w).cuda()
    JTw = op.rk_step_vjp(Ud, dt, wd).cpu().numpy()
    dot_check(np.sum(w * Jv), np.sum(JTw * v), np.sum(np.abs(w * Jv)), 1e-12)
    # in-place form (U_bar_n aliasing U_bar_np1) gives the same result
    op.rk_step_vjp(Ud, dt, wd, out=wd)
    assert np.array_equal(wd.cpu().numpy(), JTw)


@pytest.mark.parametrize("eq,vf,sf", [(0, 0, 0), (1, 1, 1)])
def test_recorded_stages(orc, torch_cuda, eq, vf, sf):
    """rk_step_record advances U bitwise as rk_step, starts its stage record
    with U_n, and rk_step_vjp_recorded on that record equals rk_step_vjp
    bitwise (the same stage states, not recomputed)."""
    import torch

    from paper_2306_12891_amd import dg
    N, nelem = 3, (2, 3, 2)
    s, op = make(orc, N, nelem, eq, vf, sf)
    U0 = torch.from_numpy(I.random_smooth(N, nelem, seed=23, noise=0.01)).cuda()
    w = torch.from_numpy(I.random_directions(U0.shape, 6)).cuda()
    dt = 0.5 * orc.max_dt(s, U0.cpu().numpy(), 0.5)
    Y = torch.empty((5,) + tuple(U0.shape), dtype=torch.float64, device="cuda")
    Ua, Ub = U0.clone(), U0.clone()
    op.rk_step(Ua, dt)
    op.rk_step_record(Ub, dt, Y)
    assert torch.equal(Ua, Ub)
    assert torch.equal(Y[0], U0)
    assert not torch.equal(Y[1], Y[0]) and not torch.equal(Y[4], Ua)
    ref = op.rk_step_vjp(U0, dt, w)
    got = op.rk_step_vjp_recorded(Y, dt, w)
    assert torch.equal(ref, got)
    # errors: Y overlapping U or the output
    Yb = torch.empty((5,) + tuple(U0.shape), dtype=torch.float64, device="cuda")
    assert op.raw_call("rk_step_record", ctypes.c_void_p(Yb[2].data_ptr()), ctypes.c_double(dt),
                       ctypes.c_void_p(Yb.data_ptr())) == dg.DG_EINVAL
    assert op.raw_call("rk_step_vjp_recorded", ctypes.c_void_p(Y.data_ptr()), ctypes.c_double(dt),
                       ctypes.c_void_p(w.data_ptr()), ctypes.c_void_p(Y[3].data_ptr())) == dg.DG_EINVAL


def test_rollout_forward_is_rk_steps(orc, torch_cuda):
    """The checkpointed rollout's forward (one library call per segment, with
    checkpoints) gives bitwise the state of plain rk_steps and of rk_step
    called step by step."""
    import torch

    from paper_2306_12891_amd import dg
    N, nelem = 3, (2, 2, 2)
    s, op = make(orc, N, nelem, 1, 1, 1)
    U0 = torch.from_numpy(I.random_smooth(N, nelem, seed=27, noise=0.01)).cuda()
    dt = 0.5 * orc.max_dt(s, U0.cpu().numpy(), 0.5)
    a = dg.rollout(op, U0, dt, 7, checkpoint_every=3)
    b = U0.clone()
    op.rk_steps(b, dt, 7)
    c = U0.clone()
    for _ in range(7):
        op.rk_step(c, dt)
    assert torch.equal(a, b) and torch.equal(b, c)


def test_autograd_functions(orc, torch_cuda):
    import torch

    from paper_2306_12891_amd import dg
    N, nelem = 3, (2, 2, 2)
    s, op = make(orc, N, nelem, 1, 1, 1)
    U = torch.from_numpy(I.random_smooth(N, nelem, seed=5, noise=0.01)).cuda().requires_grad_(True)
    w = torch.from_numpy(I.random_directions(U.shape, 4)).cuda()
    (dg.DGOperator.apply(U, op) * w).sum().backward()
    assert torch.equal(U.grad, op.vjp(U.detach(), w))
    U.grad = None
    (dg.RKStep.apply(U, op, 1e-3) * w).sum().backward()
    assert torch.equal(U.grad, op.rk_step_vjp(U.detach(), 1e-3, w))


def kinetic_energy(op, U, weights):
    import torch
    vol = np.prod([op.hi[d] - op.lo[d] for d in range(3)])
    m = U[:, 1:4]
    return torch.sum(weights * 0.5 * torch.sum(m * m, 1) / U[:, 0]) / vol


def test_rollout_gradient_matches_finite_differences(orc, torch_cuda):
    """Gradient of the volume-averaged kinetic energy after 12 steps with
    respect to the initial state (checkpoints every 5 steps) against central
    differences (eps = 1e-6) in three seeded directions."""
    import torch

    from paper_2306_12891_amd import dg
    N, nelem = 3, (3, 3, 3)
    _, op = make(orc, N, nelem, 1, 1, 1, mu=1.0 / 1600)
    U0 = torch.from_numpy(I.tgv(N, nelem, symmetry_break=True)).cuda()
    W = op.node_weights("cuda")
    dt = op.max_dt(U0, 0.5)
    nsteps = 12
    x = U0.clone().requires_grad_(True)
    kinetic_energy(op, dg.rollout(op, x, dt, nsteps, checkpoint_every=5), W).backward()
    grad = x.grad.detach()

    def J(U):
        V = U.clone()
        op.rk_steps(V, dt, nsteps)
        return kinetic_energy(op, V, W).item()

    eps = 1e-6
    for k in range(3):
        v = torch.from_numpy(I.random_directions(tuple(U0.shape), 1000 + k)).cuda()
        fd = (J(U0 + eps * v) - J(U0 - eps * v)) / (2 * eps)
        ad = torch.sum(grad * v).item()
        assert abs(fd - ad) <= 1e-6 * abs(ad), (k, fd, ad)


def test_vjp_errors(orc, torch_cuda):
    import ctypes

    import torch

    from paper_2306_12891_amd import dg
    op = dg.DG((2, 2, 2), 3, vol_flux=dg.CH)
    U = torch.from_numpy(I.density_wave(3, (2, 2, 2))).cuda()
    with pytest.raises(dg.DGError) as ei:
        op.vjp(U, U.clone())
    assert ei.value.code == dg.DG_EUNSUPPORTED
    op.set_options(vol_flux=dg.KG)
    W = U.clone()
    P = ctypes.c_void_p
    assert op.raw_call("dg_vjp", P(U.data_ptr()), P(W.data_ptr()), P(W.data_ptr())) == dg.DG_EINVAL
    assert op.raw_call("rk_step_vjp", P(U.data_ptr()), ctypes.c_double(1e-3), P(W.data_ptr()),
                       P(U.data_ptr())) == dg.DG_EINVAL


@pytest.mark.parametrize("N", [2, 3, 5, 7])
def test_recorded_stages_blended_euler(orc, torch_cuda, N):
    """Blended Euler: rk_step (whose stage kernel computes the next stage's
    indicator in its epilogue) and rk_step_record (separate indicator launch
    per stage) advance U bitwise alike; the reverse products on recomputed and
    recorded stages agree bitwise; blended elements are present."""
    import torch

    from paper_2306_12891_amd import dg
    nelem, lo, hi = (8, 2, 1), (0.0, 0.0, 0.0), (1.0, 0.25, 0.125)
    op = dg.DG(nelem, N, gamma=G, lo=lo, hi=hi, vol_flux=dg.KG, surf_flux=dg.LLF, blending=1,
               fv_recon=dg.FV_MINMOD)
    # a density and pressure jump inside element 4 (at x = 0.53), so that its
    # modal indicator fires at every degree, with 1e-3 noise against ties
    X, _, _ = I.node_coordinates(N, nelem, lo, hi)
    left = X < 0.53
    one = np.ones_like(X)
    U0n = I.from_primitive(np.where(left, 1.0, 0.125), 0 * one, 0 * one, 0 * one, np.where(left, 1.0, 0.1), G)
    U0n = U0n * (1.0 + 1e-3 * I.random_directions(U0n.shape, 8))
    U0 = torch.from_numpy(U0n).cuda()
    assert float((op.alpha(U0) > 0).double().sum().item()) >= 2
    dt = 0.5 * op.max_dt(U0, 0.5)
    w = torch.from_numpy(I.random_directions(U0.shape, 9)).cuda()
    Y = torch.empty((5,) + tuple(U0.shape), dtype=torch.float64, device="cuda")
    Ua, Ub, Uc = U0.clone(), U0.clone(), U0.clone()
    op.rk_step(Ua, dt)
    op.rk_step_record(Ub, dt, Y)
    op.rk_steps(Uc, dt, 1)
    assert torch.equal(Ua, Ub) and torch.equal(Ua, Uc)
    assert torch.equal(op.rk_step_vjp(U0, dt, w), op.rk_step_vjp_recorded(Y, dt, w))


@pytest.mark.parametrize("eq,vf,sf", [(1, 1, 1), (0, 0, 0), (1, 0, 0)])
@pytest.mark.parametrize("N", [5, 7])
def test_vjp_sampled_entries(orc, torch_cuda, eq, vf, sf, N):
    """Entry by entry: (J^T w)_j = w . (J e_j) for sampled inputs j of one GPU
    reverse product on a 12-element mesh, each against the oracle's
    dual-number column J e_j.  The samples cover corner, edge, face and
    interior nodes of several elements and all five variables, so the own and
    the neighbour's face contributions (interface flux, BR1 lifting of both
    passes) are checked separately, not only through a dot product."""
    import torch
    nelem = (3, 2, 2)
    s, op = make(orc, N, nelem, eq, vf, sf, mu=2e-2)
    U = I.random_smooth(N, nelem, seed=610 + N, noise=0.02)
    w = I.random_directions(U.shape, 13)
    JTw = op.vjp(torch.from_numpy(U).cuda(), torch.from_numpy(w).cuda()).cpu().numpy()
    n1 = N + 1
    picks = [(0, 0, 0, 0), (N, 0, 0, 1), (N, N, N, 2), (0, N, 1, 3), (1, 2, N, 4), (2, 1, 3, 0),
             (N, 3, 2, 4), (0, 0, N, 1), (3, N, 0, 2), (2, 2, 2, 4)]
    rng = np.random.default_rng(77 + N)
    cnt = 0
    for e in (0, 4, 7, 11):
        for (i, j, k, v) in picks:
            i, j, k = (min(x, N) for x in (i, j, k))
            if rng.random() < 0.3:
                continue
            col = np.zeros_like(U)
            col[e, v, k, j, i] = 1.0
            _, Jej = orc.jvp(s, U, col)
            ref = np.sum(w * Jej)
            scale = np.sum(np.abs(w * Jej))
            got = JTw[e, v, k, j, i]
            assert abs(got - ref) <= 1e-12 * scale, (e, v, k, j, i, got, ref, scale)
            cnt += 1
    assert cnt >= 20
