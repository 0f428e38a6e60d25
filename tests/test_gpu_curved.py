"""Curved elements on the GPU (dg_set_geometry) against the FP64 oracle,
through the C ABI: single evaluations on a warped periodic mesh for every
degree and flux pair to 1e-12 of the term scale (Euler and Navier-Stokes),
free-stream preservation, conservation, a Runge-Kutta rollout, the time step
and integrals, the Cartesian box given as coordinates, a full-size TGV at
N = 5 on 32^3 warped elements, and the error paths."""
import ctypes
import math

import numpy as np
import pytest

from paper_2306_12891_amd import inputs as I
from test_gpu_parity import G, TWO_PI, assert_state_close, assert_ut_close, phys_flux_scale

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def make(orc, torch, N, nelem, xn, eq=0, vf=0, sf=0, mu=0.0):
    from paper_2306_12891_amd import dg
    s = orc.Setup(N=N, nelem=nelem, equations=eq, vol_flux=vf, surf_flux=sf, mu=mu, xnodes=xn)
    op = dg.DG(nelem, N, gamma=G, mu=mu, equations=eq, vol_flux=vf, surf_flux=sf)
    op.set_geometry(torch.from_numpy(xn).cuda())
    return s, op


def gpu_ut(torch, op, U):
    return op.time_derivative(torch.from_numpy(U).cuda()).cpu().numpy()


def assert_curved_close(orc, s, got, ref, U, tol=1e-12):
    """Per variable to tol of max(max |U_t|, S_v): S_v the scale of the terms
    that cancel, N(N+1)/2 max |F| times the largest |Ja^i|/J of the mesh (the
    curved counterpart of 2/dx)."""
    Ja, J = orc.metrics(s)
    h = max(np.max(np.sqrt(np.sum(Ja[:, i] ** 2, axis=1)) / J) for i in range(3))
    S = phys_flux_scale(U, s.N, [h, h, h])
    for v in range(5):
        scale = max(np.max(np.abs(ref[:, v])), S[v])
        err = np.max(np.abs(got[:, v] - ref[:, v]))
        assert err <= tol * scale, f"var {v}: err {err:.3e} scale {scale:.3e} rel {err / scale:.3e}"


BOX = ((0.0, 0.0, 0.0), (TWO_PI,) * 3)


@pytest.mark.parametrize("N", range(1, 8))
def test_euler_all_degrees(orc, torch_cuda, N):
    ne = (3, 2, 2)
    xn = I.warped_coordinates(N, ne, amp=0.05)
    s, op = make(orc, torch_cuda, N, ne, xn, vf=0, sf=0)
    U = I.random_smooth(N, ne, seed=80 + N, noise=0.02, xnodes=xn)
    assert_curved_close(orc, s, gpu_ut(torch_cuda, op, U), orc.time_derivative(s, U), U)


@pytest.mark.parametrize("vf,sf", [(1, 1), (3, 2), (0, 1), (1, 0), (3, 0)])
@pytest.mark.parametrize("N", [3, 5])
def test_euler_flux_pairs(orc, torch_cuda, N, vf, sf):
    ne = (2, 3, 2)
    xn = I.warped_coordinates(N, ne, amp=0.05)
    s, op = make(orc, torch_cuda, N, ne, xn, vf=vf, sf=sf)
    U = I.random_smooth(N, ne, seed=90 + N + 7 * vf, noise=0.02, xnodes=xn)
    assert_curved_close(orc, s, gpu_ut(torch_cuda, op, U), orc.time_derivative(s, U), U)


@pytest.mark.parametrize("vf,sf", [(1, 1), (0, 0), (3, 2)])
@pytest.mark.parametrize("N", [2, 3, 4, 5, 6, 7])
def test_navier_stokes(orc, torch_cuda, N, vf, sf):
    ne = (2, 2, 3)
    xn = I.warped_coordinates(N, ne, amp=0.05)
    s, op = make(orc, torch_cuda, N, ne, xn, eq=1, vf=vf, sf=sf, mu=2e-2)
    U = I.random_smooth(N, ne, seed=100 + N, noise=0.02, xnodes=xn)
    ref = orc.time_derivative(s, U)
    assert_curved_close(orc, s, gpu_ut(torch_cuda, op, U), ref, U)


@pytest.mark.parametrize("eq", [0, 1])
def test_freestream_and_conservation(orc, torch_cuda, eq):
    import torch
    N, ne = 4, (3, 3, 2)
    xn = I.warped_coordinates(N, ne, amp=0.06)
    s, op = make(orc, torch_cuda, N, ne, xn, eq=eq, vf=1, sf=1, mu=1e-2)
    U = I.freestream(N, ne, u=(0.4, -0.3, 0.2))
    Ut = gpu_ut(torch_cuda, op, U)
    scale = np.max(np.abs(U)) * (2.0 / (TWO_PI / 3)) * N * (N + 1) / 2
    assert np.max(np.abs(Ut)) <= 1e-12 * scale
    U = I.random_smooth(N, ne, seed=7, noise=0.02, xnodes=xn)
    Utd = op.time_derivative(torch.from_numpy(U).cuda())
    tot = np.array(op.integrals(Utd))
    mag = np.array(op.integrals(Utd.abs()))
    assert np.all(np.abs(tot) <= 1e-13 * mag), (tot, mag)


def test_rollout(orc, torch_cuda):
    import torch
    N, ne = 3, (3, 3, 3)
    xn = I.warped_coordinates(N, ne, amp=0.04)
    s, op = make(orc, torch_cuda, N, ne, xn, eq=1, vf=1, sf=1, mu=1.0 / 1600)
    U0 = I.tgv(N, ne, symmetry_break=True, xnodes=xn)
    Ud = torch.from_numpy(U0).cuda()
    dt = op.max_dt(Ud, 0.5)
    assert abs(dt - orc.max_dt(s, U0, 0.5)) <= 1e-12 * dt
    op.rk_steps(Ud, dt, 5)
    assert_state_close(Ud.cpu().numpy(), orc.rk_steps(s, U0, dt, 5))


def test_integrals_and_dt(orc, torch_cuda):
    import torch
    N, ne = 5, (2, 3, 2)
    xn = I.warped_coordinates(N, ne, amp=0.06)
    s, op = make(orc, torch_cuda, N, ne, xn, eq=1, vf=1, sf=1, mu=3e-2)
    U = I.random_smooth(N, ne, seed=12, xnodes=xn)
    Ud = torch.from_numpy(U).cuda()
    assert np.allclose(op.integrals(Ud), orc.integrals(s, U), rtol=1e-13, atol=0)
    assert abs(op.max_dt(Ud, 0.5) - orc.max_dt(s, U, 0.5)) <= 1e-12 * orc.max_dt(s, U, 0.5)


def test_box_coordinates_and_reset(orc, torch_cuda):
    """The Cartesian box given as coordinates gives the Cartesian operator, and
    set_geometry(None) returns to it."""
    import torch

    from paper_2306_12891_amd import dg
    N, ne = 4, (3, 2, 2)
    X, Y, Z = I.node_coordinates(N, ne, *BOX)
    xc = np.ascontiguousarray(np.stack([X, Y, Z], axis=1))
    U = I.random_smooth(N, ne, seed=13, noise=0.02)
    Ud = torch.from_numpy(U).cuda()
    op = dg.DG(ne, N, gamma=G, mu=2e-2, equations=dg.NS, vol_flux=dg.PI, surf_flux=dg.ROE)
    box = op.time_derivative(Ud).cpu().numpy()
    op.set_geometry(torch.from_numpy(xc).cuda())
    cur = op.time_derivative(Ud).cpu().numpy()
    assert_ut_close(cur, box, U, N, ne, *BOX)
    op.set_geometry(None)
    assert np.array_equal(op.time_derivative(Ud).cpu().numpy(), box)


def test_full_size_tgv_n5_32(orc, torch_cuda):
    """TGV at N = 5 on 32^3 warped elements (7 M DOF): whole-mesh U_t."""
    N, ne = 5, (32, 32, 32)
    xn = I.warped_coordinates(N, ne, amp=0.04)
    s, op = make(orc, torch_cuda, N, ne, xn, eq=1, vf=1, sf=1, mu=1.0 / 1600)
    U = I.tgv(N, ne, xnodes=xn)
    assert_curved_close(orc, s, gpu_ut(torch_cuda, op, U), orc.time_derivative(s, U), U)


def test_error_paths(orc, torch_cuda):
    import torch

    from paper_2306_12891_amd import dg
    N, ne = 3, (2, 2, 2)
    xn = I.warped_coordinates(N, ne, amp=0.05)
    op = dg.DG(ne, N, gamma=G, mu=1e-2, equations=dg.NS, vol_flux=dg.PI, surf_flux=dg.ROE)
    assert op.raw_call("dg_set_geometry", ctypes.c_void_p(xn.ctypes.data)) == dg.DG_EINVAL  # host pointer
    # an inverted element: its x coordinates mirrored
    bad = xn.copy()
    bad[0, 0] = bad[0, 0, :, :, ::-1]
    with pytest.raises(dg.DGError) as ei:
        op.set_geometry(torch.from_numpy(np.ascontiguousarray(bad)).cuda())
    assert ei.value.code == dg.DG_EINVAL
    U = torch.from_numpy(I.random_smooth(N, ne, seed=3)).cuda()
    box = op.time_derivative(U).cpu().numpy()  # still the box
    s_box = orc.Setup(N=N, nelem=ne, equations=1, vol_flux=1, surf_flux=1, mu=1e-2)
    assert_ut_close(box, orc.time_derivative(s_box, U.cpu().numpy()), U.cpu().numpy(), N, ne, *BOX)
    op.set_geometry(torch.from_numpy(xn).cuda())
    for kw in (dict(precision=dg.MIXED), dict(vol_flux=dg.CH), dict(equations=dg.EULER, blending=1)):
        with pytest.raises(dg.DGError) as ei:
            op.set_options(**kw)
        assert ei.value.code == dg.DG_EUNSUPPORTED, kw
    op.vjp(U, U.clone())  # the reverse mode covers curved meshes
    op.set_cs_field(torch.full((8,), 0.1, dtype=torch.float64, device="cuda"))  # the model and its adjoint too
    op.vjp(U, U.clone())
    op.set_cs_field(None)
    op2 = dg.DG(ne, N, gamma=G, mu=1e-2, equations=dg.NS, vol_flux=dg.PI, surf_flux=dg.ROE, precision=dg.MIXED)
    with pytest.raises(dg.DGError) as ei:
        op2.set_geometry(torch.from_numpy(xn).cuda())
    assert ei.value.code == dg.DG_EUNSUPPORTED


# ---------------------------------------------------------------------------
# General connectivity (dg_set_connectivity): the warped periodic mesh with
# every element's reference axes relabelled by a seeded cube rotation (all 8
# face orientations occur).
# ---------------------------------------------------------------------------
def make_rotated(orc, torch, N, ne, seed, eq=0, vf=0, sf=0, mu=0.0, amp=0.05):
    from paper_2306_12891_amd import dg
    xn = I.warped_coordinates(N, ne, amp=amp)
    perm, conn = I.rotated_elements(N, ne, seed=seed)
    xr = I.relabel(xn, perm)
    s = orc.Setup(N=N, nelem=ne, equations=eq, vol_flux=vf, surf_flux=sf, mu=mu, xnodes=xr, conn=conn)
    op = dg.DG(ne, N, gamma=G, mu=mu, equations=eq, vol_flux=vf, surf_flux=sf)
    op.set_connectivity(conn)
    op.set_geometry(torch.from_numpy(xr).cuda())
    return s, op, xn, perm


@pytest.mark.parametrize("eq,vf,sf", [(0, 0, 0), (0, 1, 1), (1, 1, 1), (1, 3, 2), (1, 0, 0)])
@pytest.mark.parametrize("N", [2, 3, 5])
def test_rotated_elements(orc, torch_cuda, N, eq, vf, sf):
    ne = (3, 2, 2)
    s, op, xn, perm = make_rotated(orc, torch_cuda, N, ne, seed=N + 3, eq=eq, vf=vf, sf=sf, mu=2e-2)
    U = I.relabel(I.random_smooth(N, ne, seed=110 + N, noise=0.02, xnodes=xn), perm)
    assert_curved_close(orc, s, gpu_ut(torch_cuda, op, U), orc.time_derivative(s, U), U)


def test_rotated_equals_structured_on_gpu(orc, torch_cuda):
    """The relabelled mesh gives the relabelled U_t of the structured mesh."""
    N, ne = 4, (2, 3, 2)
    s, op, xn, perm = make_rotated(orc, torch_cuda, N, ne, seed=5, eq=1, vf=1, sf=1, mu=2e-2)
    _, op0 = make(orc, torch_cuda, N, ne, xn, eq=1, vf=1, sf=1, mu=2e-2)
    U = I.random_smooth(N, ne, seed=17, noise=0.02, xnodes=xn)
    a = gpu_ut(torch_cuda, op0, U)
    b = I.unlabel(gpu_ut(torch_cuda, op, I.relabel(U, perm)), perm)
    assert_curved_close(orc, s, b, a, U)


def test_rotated_rollout_and_conservation(orc, torch_cuda):
    import torch
    N, ne = 3, (3, 3, 2)
    s, op, xn, perm = make_rotated(orc, torch_cuda, N, ne, seed=11, eq=1, vf=1, sf=1, mu=1.0 / 1600, amp=0.04)
    U0 = I.relabel(I.random_smooth(N, ne, seed=23, xnodes=xn), perm)
    Ud = torch.from_numpy(U0).cuda()
    Utd = op.time_derivative(Ud)
    tot, mag = np.array(op.integrals(Utd)), np.array(op.integrals(Utd.abs()))
    assert np.all(np.abs(tot) <= 1e-13 * mag), (tot, mag)
    dt = op.max_dt(Ud, 0.5)
    op.rk_steps(Ud, dt, 4)
    assert_state_close(Ud.cpu().numpy(), orc.rk_steps(s, U0, dt, 4))


def test_connectivity_error_paths(orc, torch_cuda):
    import torch

    from paper_2306_12891_amd import dg
    N, ne = 2, (2, 2, 2)
    perm, conn = I.rotated_elements(N, ne, seed=2)
    op = dg.DG(ne, N, gamma=G, equations=dg.EULER)
    bad = conn.copy()
    bad[3, 2, 2] = (bad[3, 2, 2] + 3) % 8
    with pytest.raises(dg.DGError) as ei:
        op.set_connectivity(bad)
    assert ei.value.code == dg.DG_EINVAL
    bad = conn.copy()
    bad[1, 0, 0] = 99
    with pytest.raises(dg.DGError) as ei:
        op.set_connectivity(bad)
    assert ei.value.code == dg.DG_EINVAL
    U = torch.from_numpy(I.random_smooth(N, ne, seed=1)).cuda()
    ref = op.time_derivative(U).cpu().numpy()  # rejected connectivity left the box unchanged
    op.set_connectivity(conn)
    with pytest.raises(dg.DGError) as ei:  # general connectivity without curved elements
        op.time_derivative(U)
    assert ei.value.code == dg.DG_ESTATE
    op.set_connectivity(None)
    assert np.array_equal(op.time_derivative(U).cpu().numpy(), ref)


def test_failed_calls_keep_the_previous_mesh(orc, torch_cuda):
    """A rejected geometry or connectivity leaves the context as it was."""
    import torch

    from paper_2306_12891_amd import dg
    N, ne = 3, (2, 2, 2)
    s, op = make(orc, torch_cuda, N, ne, I.warped_coordinates(N, ne, amp=0.05), eq=1, vf=1, sf=1, mu=1e-2)
    U = torch.from_numpy(I.random_smooth(N, ne, seed=4, xnodes=I.warped_coordinates(N, ne, amp=0.05))).cuda()
    before = op.time_derivative(U).cpu().numpy()
    bad = I.warped_coordinates(N, ne, amp=0.05)
    bad[1, 1] = bad[1, 1, :, ::-1, :]  # element 1 inverted
    with pytest.raises(dg.DGError):
        op.set_geometry(torch.from_numpy(np.ascontiguousarray(bad)).cuda())
    _, conn = I.rotated_elements(N, ne, seed=1)
    conn[0, 0, 1] = (conn[0, 0, 1] + 1) % 6
    with pytest.raises(dg.DGError):
        op.set_connectivity(conn)
    assert np.array_equal(op.time_derivative(U).cpu().numpy(), before)


# ---------------------------------------------------------------------------
# Smagorinsky eddy viscosity on curved elements (filter width from the element
# volume), constant and per-element C_s, structured and rotated-element meshes.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("vf,sf,field", [(1, 1, False), (0, 0, True), (3, 2, False)])
@pytest.mark.parametrize("N", [2, 3, 5])
def test_les_on_warped_mesh(orc, torch_cuda, N, vf, sf, field):
    from paper_2306_12891_amd import dg
    ne = (3, 2, 2)
    xn = I.warped_coordinates(N, ne, amp=0.05)
    cs = np.random.default_rng(120 + N).uniform(0.1, 0.4, 12) if field else None
    s = orc.Setup(N=N, nelem=ne, equations=1, vol_flux=vf, surf_flux=sf, mu=2e-3, Cs=0.0 if field else 0.3,
                  cs_elem=cs, xnodes=xn)
    op = dg.DG(ne, N, gamma=G, mu=2e-3, equations=dg.NS, vol_flux=vf, surf_flux=sf, Cs=0.0 if field else 0.3)
    op.set_geometry(torch_cuda.from_numpy(xn).cuda())
    if field:
        op.set_cs_field(torch_cuda.from_numpy(cs).cuda())
    U = I.random_smooth(N, ne, seed=130 + N, noise=0.02, xnodes=xn)
    ref = orc.time_derivative(s, U)
    assert_curved_close(orc, s, gpu_ut(torch_cuda, op, U), ref, U)
    plain = orc.time_derivative(orc.Setup(N=N, nelem=ne, equations=1, vol_flux=vf, surf_flux=sf, mu=2e-3,
                                          xnodes=xn), U)
    assert np.max(np.abs(plain - ref)) > 1e-4 * np.max(np.abs(ref))


def test_les_on_rotated_elements_and_rollout(orc, torch_cuda):
    import torch
    N, ne = 3, (3, 2, 2)
    s, op, xn, perm = make_rotated(orc, torch_cuda, N, ne, seed=9, eq=1, vf=1, sf=1, mu=2e-3)
    op.set_options(Cs=0.25)
    s = orc.Setup(N=N, nelem=ne, equations=1, vol_flux=1, surf_flux=1, mu=2e-3, Cs=0.25, xnodes=s.xnodes,
                  conn=s.conn)
    U = I.relabel(I.random_smooth(N, ne, seed=140, noise=0.02, xnodes=xn), perm)
    assert_curved_close(orc, s, gpu_ut(torch_cuda, op, U), orc.time_derivative(s, U), U)
    dt = 0.5 * orc.max_dt(s, U, 0.5)
    Ud = torch.from_numpy(U).cuda()
    op.rk_steps(Ud, dt, 3)
    assert_state_close(Ud.cpu().numpy(), orc.rk_steps(s, U, dt, 3))


def test_les_box_coordinates_match_cartesian_gpu(orc, torch_cuda):
    """The box given as node coordinates: the curved kernels with the element
    filter width reproduce the Cartesian LES kernels."""
    from paper_2306_12891_amd import dg
    N, ne, lo, hi = 3, (3, 2, 2), (0.0, 0.0, 0.0), (6.0, 1.0, 2.0)
    X, Y, Z = I.node_coordinates(N, ne, lo, hi)
    xn = np.ascontiguousarray(np.stack([X, Y, Z], axis=1))
    U = I.random_smooth(N, ne, lo, hi, seed=150, noise=0.02)
    kw = dict(gamma=G, mu=2e-3, lo=lo, hi=hi, equations=dg.NS, vol_flux=dg.PI, surf_flux=dg.ROE, Cs=0.3)
    box = dg.DG(ne, N, **kw)
    cur = dg.DG(ne, N, **kw)
    cur.set_geometry(torch_cuda.from_numpy(xn).cuda())
    a, b = gpu_ut(torch_cuda, box, U), gpu_ut(torch_cuda, cur, U)
    assert_ut_close(b, a, U, N, ne, lo, hi)
