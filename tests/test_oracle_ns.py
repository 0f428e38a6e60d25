"""Pins of the Navier-Stokes terms (BR1 lifting, viscous and heat fluxes) and
of the dual-number Jacobian-vector products."""
import numpy as np
import pytest

from paper_2306_12891_amd import inputs as I

G = 1.4
PR = 0.72


def lagrange_D(x):
    n = len(x)
    lam = np.array([1.0 / np.prod([x[j] - x[k] for k in range(n) if k != j]) for j in range(n)])
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                D[i, j] = lam[j] / lam[i] / (x[i] - x[j])
        D[i, i] = -np.sum(D[i])
    return D


def test_gradient_continuous_data_is_local_derivative(orc):
    """Globally smooth nodal data is continuous across faces, so the BR1
    corrections vanish and the lifted gradient is the local D q; sin x lifts
    spectrally to cos x."""
    N, ne = 7, (4, 4, 2)
    X, Y, Z = I.node_coordinates(N, ne, (0, 0, 0), (2 * np.pi,) * 3)
    rho = 1 + 0.2 * np.cos(Y)
    u, v, w = np.sin(X), np.cos(Z) * 0.5, np.sin(Y) * np.cos(X) * 0.3
    p = 1.0 + 0.1 * np.sin(Z)
    U = I.from_primitive(rho, u, v, w, p, G)
    s = orc.Setup(N=N, nelem=ne, equations=1, mu=1e-3)
    g = orc.gradient(s, U)  # (e, d, c, k, j, i)
    D = lagrange_D(I.lgl_points(N))
    theta = p / rho
    for d, ax in ((0, 3), (1, 2), (2, 1)):
        invJ = 2.0 / (2 * np.pi / ne[d])
        for c, q in enumerate((u, v, w, theta)):
            local = invJ * np.moveaxis(np.tensordot(D, np.moveaxis(q, ax, 0), axes=([1], [0])), 0, ax)
            assert np.max(np.abs(g[:, d, c] - local)) < 1e-12
    assert np.max(np.abs(g[:, 0, 0] - np.cos(X))) < 1e-5
    assert np.max(np.abs(g[:, 1, 3] + 0.2 * np.sin(Y) * (-(p / rho ** 2)))) < 1e-4


@pytest.mark.parametrize("vf,sf", [(1, 1), (0, 0)])
def test_shear_wave_viscous_terms(orc, vf, sf):
    """u = A sin y, rho = 1, p = const: the advective terms vanish and the
    viscous operator gives m_x,t = -mu A sin y and E_t = mu A^2 cos 2y."""
    N, ne, mu, A = 7, (1, 8, 1), 0.05, 0.3
    X, Y, Z = I.node_coordinates(N, ne, (0, 0, 0), (2 * np.pi,) * 3)
    one = np.ones_like(X)
    U = I.from_primitive(one, A * np.sin(Y), 0 * X, 0 * X, 2.0 * one, G)
    s = orc.Setup(N=N, nelem=ne, equations=1, vol_flux=vf, surf_flux=sf, mu=mu, Pr=PR)
    Ut = orc.time_derivative(s, U)
    assert np.max(np.abs(Ut[:, 0])) < 1e-13
    assert np.max(np.abs(Ut[:, 1] + mu * A * np.sin(Y))) < 1e-8
    assert np.max(np.abs(Ut[:, 2:4])) < 1e-12
    assert np.max(np.abs(Ut[:, 4] - mu * A * A * np.cos(2 * Y))) < 1e-8


def test_heat_conduction(orc):
    """u = 0, p = 1, theta = p/rho = 1 + eps sin x: only E changes, with
    E_t = kappa' theta_xx, kappa' = mu gamma / ((gamma - 1) Pr)."""
    N, ne, mu, eps = 6, (4, 1, 2), 0.02, 0.1
    X, Y, Z = I.node_coordinates(N, ne, (0, 0, 0), (2 * np.pi,) * 3)
    theta = 1 + eps * np.sin(X)
    U = I.from_primitive(1.0 / theta, 0 * X, 0 * X, 0 * X, np.ones_like(X), G)
    s = orc.Setup(N=N, nelem=ne, equations=1, vol_flux=1, surf_flux=1, mu=mu, Pr=PR)
    Ut = orc.time_derivative(s, U)
    kap = mu * G / ((G - 1) * PR)
    assert np.max(np.abs(Ut[:, :4])) < 1e-12
    assert np.max(np.abs(Ut[:, 4] - kap * (-eps * np.sin(X)))) < 1e-5


@pytest.mark.slow
def test_tgv_initial_kinetic_energy_and_dissipation(orc):
    """TGV at Ma 0.1, Re 1600: KE(0) = 1/8 (rho close to 1) and
    dKE/dt(0) = -mu <|grad u|^2> = -(3/4) mu within about 1 %."""
    N, n = 5, 8
    mu = 1.0 / 1600
    U = I.tgv(N, (n, n, n))
    s = orc.Setup(N=N, nelem=(n, n, n), equations=1, vol_flux=1, surf_flux=1, mu=mu, Pr=PR)
    vol = (2 * np.pi) ** 3
    rho, m = U[:, 0], U[:, 1:4]
    X = np.zeros_like(U)
    X[:, 0] = 0.5 * np.sum(m * m, 1) / rho
    ke0 = orc.integrals(s, X)[0] / vol
    assert abs(ke0 - 0.125) < 2e-4
    Ut = orc.time_derivative(s, U)
    u = m / rho[:, None]
    X[:, 0] = np.einsum("evkji,evkji->ekji", u, Ut[:, 1:4]) - 0.5 * np.sum(u * u, 1) * Ut[:, 0]
    dke = orc.integrals(s, X)[0] / vol
    assert abs(dke / (-0.75 * mu) - 1.0) < 0.01, dke
    mom = orc.integrals(s, U)[1:4]
    assert np.max(np.abs(mom)) < 1e-12


@pytest.mark.parametrize("eq,vf,sf", [(0, 0, 0), (0, 1, 1), (1, 1, 1), (1, 0, 0), (0, 2, 1)])
def test_jvp_matches_central_differences(orc, eq, vf, sf):
    N, ne = 3, (2, 2, 1)
    s = orc.Setup(N=N, nelem=ne, equations=eq, vol_flux=vf, surf_flux=sf, mu=2e-2)
    U = I.random_smooth(N, ne, seed=31, noise=0.02)
    V = I.random_directions(U.shape, 0)
    Ut, JV = orc.jvp(s, U, V)
    assert np.array_equal(Ut, orc.time_derivative(s, U))
    eps = 1e-6
    fd = (orc.time_derivative(s, U + eps * V) - orc.time_derivative(s, U - eps * V)) / (2 * eps)
    assert np.max(np.abs(JV - fd)) < 1e-6 * np.max(np.abs(JV))


def test_rollout_jvp_matches_central_differences(orc):
    N, ne = 3, (2, 1, 2)
    s = orc.Setup(N=N, nelem=ne, equations=1, vol_flux=1, surf_flux=1, mu=2e-2)
    U = I.random_smooth(N, ne, seed=32, noise=0.01)
    V = I.random_directions(U.shape, 1)
    dt, n = 0.01, 3
    U1, JV = orc.rk_jvp(s, U, V, dt, n)
    assert np.array_equal(U1, orc.rk_steps(s, U, dt, n))
    eps = 1e-6
    fd = (orc.rk_steps(s, U + eps * V, dt, n) - orc.rk_steps(s, U - eps * V, dt, n)) / (2 * eps)
    assert np.max(np.abs(JV - fd)) < 1e-7 * np.max(np.abs(JV))
