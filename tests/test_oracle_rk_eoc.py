"""Pins of the time integrator and of design-order convergence.

The 5-stage 2N-storage scheme is converted to Butcher form here and checked
against the eight order-4 conditions, the published abscissae c_k and its
stability polynomial; the oracle's integration loop is checked on a linear
system against R(dt A).  Convergence is checked on the exact density wave."""
import numpy as np
import pytest

from paper_2306_12891_amd import inputs as I

# Published abscissae of the Carpenter-Kennedy (5,4) scheme.
C_PUBLISHED = np.array([0.0, 1432997174477 / 9575080441755, 2526269341429 / 6820363962896,
                        2006345519317 / 3224310063776, 2802321613138 / 2924317926251])


def butcher(A, B):
    s = len(A)
    Gc = np.zeros((s, s))  # G_k = sum_j Gc[k, j] F_j
    for k in range(s):
        if k > 0:
            Gc[k, :k] = A[k] * Gc[k - 1, :k]
        Gc[k, k] = 1.0
    a = np.zeros((s, s))
    for i in range(1, s):  # stage i evaluates F at Y_{i-1} = Y_0 + dt sum_{m<i} B_m G_m
        for j in range(i):
            a[i, j] = sum(B[m] * Gc[m, j] for m in range(j, i))
    b = np.array([sum(B[m] * Gc[m, j] for m in range(j, s)) for j in range(s)])
    return a, b


def test_order_conditions(orc):
    A, B = orc.rk_coefficients()
    assert A[0] == 0.0
    a, b = butcher(A, B)
    c = a.sum(1)
    assert np.allclose(c, C_PUBLISHED, rtol=0, atol=1e-14)
    conds = [(b.sum(), 1), (b @ c, 1 / 2), (b @ c ** 2, 1 / 3), (b @ a @ c, 1 / 6), (b @ c ** 3, 1 / 4),
             (b @ (c * (a @ c)), 1 / 8), (b @ a @ c ** 2, 1 / 12), (b @ a @ a @ c, 1 / 24)]
    for got, want in conds:
        assert abs(got - want) < 1e-14
    # stability polynomial R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24 + z^5/200
    e = np.ones(5)
    assert abs(b @ np.linalg.matrix_power(a, 4) @ e - 1 / 200) < 1e-10


def test_linear_system_matches_stability_polynomial(orc):
    rng = np.random.default_rng(1)
    n = 6
    A = rng.standard_normal((n, n))
    A = A - A.T - 0.5 * np.eye(n)
    u0 = rng.standard_normal(n)
    dt = 0.05
    Z = dt * A
    R = np.eye(n) + Z + Z @ Z / 2 + Z @ Z @ Z / 6 + np.linalg.matrix_power(Z, 4) / 24 + np.linalg.matrix_power(Z, 5) / 200
    u1 = orc.lserk4_linear(A, u0, dt, 1)
    assert np.allclose(u1, R @ u0, rtol=0, atol=1e-14)
    u3 = orc.lserk4_linear(A, u0, dt, 3)
    assert np.allclose(u3, np.linalg.matrix_power(R, 3) @ u0, rtol=0, atol=1e-13)


def _dw_error(orc, N, nelem, tend=0.2, cfl=0.5, oned=False):
    if oned:
        X, _, _ = I.node_coordinates(N, nelem, (0, 0, 0), (2 * np.pi,) * 3)
        mk = lambda t: I.from_primitive(1 + 0.2 * np.sin(X - t), np.ones_like(X), 0 * X, 0 * X, np.ones_like(X), 1.4)
    else:
        mk = lambda t: I.density_wave(N, nelem, t=t)
    s = orc.Setup(N=N, nelem=nelem)
    U = mk(0.0)
    dt = orc.max_dt(s, U, cfl)
    ns = int(np.ceil(tend / dt))
    U1 = orc.rk_steps(s, U, tend / ns, ns)
    return np.sqrt(orc.integrals(s, (U1 - mk(tend)) ** 2)[0])


def test_eoc_density_wave_1d(orc):
    """Density wave along x, N = 3: the L2 error converges at close to N + 1."""
    e = [_dw_error(orc, 3, (n, 1, 1), tend=1.0, oned=True) for n in (8, 16, 32)]
    eoc = np.log2(np.array(e[:-1]) / np.array(e[1:]))
    assert np.all(eoc > 3.7), eoc


@pytest.mark.slow
def test_eoc_density_wave_3d(orc):
    """The 3-D density wave (speed (1,1,1)) on 4^3, 8^3, 16^3 elements at N = 3.
    On these coarse meshes the rate is still pre-asymptotic (about 3.2 then 3.35);
    the pin requires it above 3.1 and rising."""
    e = [_dw_error(orc, 3, (n, n, n)) for n in (4, 8, 16)]
    eoc = np.log2(np.array(e[:-1]) / np.array(e[1:]))
    assert np.all(eoc > 3.1) and eoc[1] > eoc[0], eoc
    # C1 time step: dt = 0.5 / (4 * max sum (|u|+c)/dx) ~ 2.818e-2 on 4^3 elements
    s = orc.Setup(N=3, nelem=(4, 4, 4))
    assert abs(orc.max_dt(s, I.density_wave(3, (4, 4, 4)), 0.5) - 2.818e-2) < 5e-5
