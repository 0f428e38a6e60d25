"""Pins of the oracle's Smagorinsky eddy viscosity (standard model with constant
C_s and per-element C_s; paper Sec. 5).

Model (reading): mu_t = rho (C_s Delta)^2 |S|, |S| = sqrt(2 S_ij S_ij),
kappa'_t = mu_t gamma / ((gamma - 1) Pr_t), Delta = (dx dy dz)^(1/3) / (N + 1).

* C_s = 0, and a per-element field equal to a constant, reproduce the plain
  Navier-Stokes operator / the constant-coefficient operator bitwise.
* One-dimensional shear and temperature profiles: the exact U_t is the
  derivative of the analytic viscous flux (velocity gradient, strain rate and
  temperature gradient of the profile in closed form), differentiated here by
  a sixth-order central difference.  The DG operator converges to it.  |S|
  has kinks where the shear changes sign; they lie on element interfaces, and
  the nodes on them (where the exact energy U_t jumps) are left out.
* A per-element coefficient acts locally: changing C_s in one element leaves
  U_t bitwise unchanged outside that element and its six face neighbours.
* Forward-mode derivatives through the model (|S| and the density factor;
  reading: |S|' = 0 where |S| = 0, as |x|' = 0 at 0) agree with central
  differences of the operator and of a two-step rollout.
"""
import math

import numpy as np
import pytest

from paper_2306_12891_amd import inputs as I

G = 1.4
TWO_PI = 2 * math.pi


def delta_of(N, nelem, lo=(0, 0, 0), hi=(TWO_PI,) * 3):
    dx = [(hi[d] - lo[d]) / nelem[d] for d in range(3)]
    return (dx[0] * dx[1] * dx[2]) ** (1.0 / 3.0) / (N + 1)


def test_zero_coefficient_is_navier_stokes(orc):
    N, nelem = 3, (2, 3, 2)
    U = I.random_smooth(N, nelem, seed=41, noise=0.01)
    base = dict(N=N, nelem=nelem, equations=orc.NS, vol_flux=orc.PI, surf_flux=orc.ROE, mu=0.02)
    a = orc.time_derivative(orc.Setup(**base), U)
    b = orc.time_derivative(orc.Setup(**base, Cs=0.0), U)
    assert np.array_equal(a, b)
    c = orc.time_derivative(orc.Setup(**base, Cs=0.3), U)
    d = orc.time_derivative(orc.Setup(**base, cs_elem=np.full(12, 0.3)), U)
    assert np.array_equal(c, d)
    assert np.max(np.abs(c - a)) > 1e-3 * np.max(np.abs(a))  # the model acts


def shear_profile(y, A, B, th0, p0):
    """u = A sin y (x-velocity), theta = th0 + B cos y, p = p0: rho = p0 / theta."""
    th = th0 + B * np.cos(y)
    return p0 / th, A * np.sin(y), th


def exact_viscous_flux_y(y, A, B, th0, p0, mu, Pr, cd2, Prt):
    """y-components of the viscous flux of the profile (momentum x, energy)."""
    rho, u, th = shear_profile(y, A, B, th0, p0)
    dudy = A * np.cos(y)
    dthdy = -B * np.sin(y)
    S = np.abs(dudy)  # only S_xy = S_yx = du/dy / 2 is non-zero: sqrt(2 S:S) = |du/dy|
    mut = rho * cd2 * S
    kap = mu * G / ((G - 1) * Pr) + mut * G / ((G - 1) * Prt)
    tau_xy = (mu + mut) * dudy
    return tau_xy, u * tau_xy + kap * dthdy


def exact_ut(y, *args):
    h = 1e-3
    w = [(-3, -1 / 60), (-2, 3 / 20), (-1, -3 / 4), (1, 3 / 4), (2, -3 / 20), (3, 1 / 60)]
    m = sum(c * exact_viscous_flux_y(y + k * h, *args)[0] for k, c in w) / h
    E = sum(c * exact_viscous_flux_y(y + k * h, *args)[1] for k, c in w) / h
    return m, E


@pytest.mark.parametrize("Cs", [0.0, 0.4])
def test_shear_profile_converges_to_exact(orc, Cs):
    N, mu, Pr, Prt = 5, 0.01, 0.72, 0.9
    A, B, th0 = 0.5, 0.2, 1.0
    p0 = 1.0 / G
    errs = []
    for ny in (8, 16):
        nelem = (1, ny, 1)
        X, Y, Z = I.node_coordinates(N, nelem, (0, 0, 0), (TWO_PI,) * 3)
        rho, u, th = shear_profile(Y, A, B, th0, p0)
        zero = np.zeros_like(Y)
        U = I.from_primitive(rho, u, zero, zero, p0 + zero, G)
        s = orc.Setup(N=N, nelem=nelem, equations=orc.NS, vol_flux=orc.PI, surf_flux=orc.ROE, mu=mu, Pr=Pr,
                      Cs=Cs, Prt=Prt)
        Ut = orc.time_derivative(s, U)
        cd2 = (Cs * delta_of(N, nelem)) ** 2
        m_ex, E_ex = exact_ut(Y, A, B, th0, p0, mu, Pr, cd2, Prt)
        scale = max(np.max(np.abs(m_ex)), np.max(np.abs(E_ex)))
        assert np.max(np.abs(Ut[:, 0])) <= 1e-12 * scale  # mass: no viscous part, no advection
        assert np.max(np.abs(Ut[:, 2:4])) <= 1e-11 * scale  # y, z momentum: constant p, no shear there
        ok = np.abs(np.cos(Y)) > 1e-6
        errs.append(max(np.max(np.abs(Ut[:, 1] - m_ex)[ok]), np.max(np.abs(Ut[:, 4] - E_ex)[ok])) / scale)
    # smooth inside every element: high-order convergence (measured EOC about 5 at N = 5)
    assert errs[1] < 5e-5 and errs[1] < errs[0] / 16, errs


def test_shear_in_other_directions(orc):
    """The same profile along x with the velocity in z (w = A sin x): exercises
    other strain-tensor components."""
    N, mu, Pr, Prt, Cs = 5, 0.01, 0.72, 0.9, 0.4
    A, B, th0 = 0.5, 0.2, 1.0
    p0 = 1.0 / G
    nelem = (16, 1, 1)
    X, Y, Z = I.node_coordinates(N, nelem, (0, 0, 0), (TWO_PI,) * 3)
    rho, w, th = shear_profile(X, A, B, th0, p0)
    zero = np.zeros_like(X)
    U = I.from_primitive(rho, zero, zero, w, p0 + zero, G)
    s = orc.Setup(N=N, nelem=nelem, equations=orc.NS, vol_flux=orc.PI, surf_flux=orc.ROE, mu=mu, Pr=Pr, Cs=Cs,
                  Prt=Prt)
    Ut = orc.time_derivative(s, U)
    cd2 = (Cs * delta_of(N, nelem)) ** 2
    m_ex, E_ex = exact_ut(X, A, B, th0, p0, mu, Pr, cd2, Prt)
    scale = max(np.max(np.abs(m_ex)), np.max(np.abs(E_ex)))
    ok = np.abs(np.cos(X)) > 1e-6
    assert np.max(np.abs(Ut[:, 3] - m_ex)[ok]) <= 5e-5 * scale
    assert np.max(np.abs(Ut[:, 4] - E_ex)[ok]) <= 5e-5 * scale
    assert np.max(np.abs(Ut[:, 1:3])) <= 1e-11 * scale


def test_per_element_coefficient_is_local(orc):
    N, nelem = 3, (4, 4, 4)
    U = I.random_smooth(N, nelem, seed=43, noise=0.01)
    cs = np.full(64, 0.2)
    base = dict(N=N, nelem=nelem, equations=orc.NS, vol_flux=orc.PI, surf_flux=orc.ROE, mu=0.02)
    a = orc.time_derivative(orc.Setup(**base, cs_elem=cs), U)
    e = 1 + 4 * (2 + 4 * 1)
    cs2 = cs.copy()
    cs2[e] = 0.5
    b = orc.time_derivative(orc.Setup(**base, cs_elem=cs2), U)
    touched = {e, *orc.neighbors(orc.Setup(**base))[e].tolist()}
    for k in range(64):
        same = np.array_equal(a[k], b[k])
        assert same == (k not in touched), k


@pytest.mark.parametrize("vf,sf,field", [(1, 1, False), (0, 0, True), (3, 2, False)])
def test_jvp_through_the_model_matches_central_differences(orc, vf, sf, field):
    """Dual numbers through the eddy viscosity (|S| and the density factor)
    against central differences of the operator, constant and per-element
    C_s; a state with |S| > 0 at every node (away from the convention at
    |S| = 0)."""
    N, nelem = 3, (2, 3, 2)
    cs = np.random.default_rng(3).uniform(0.1, 0.4, 12) if field else None
    s = orc.Setup(N=N, nelem=nelem, equations=orc.NS, vol_flux=vf, surf_flux=sf, mu=5e-3, Cs=0.0 if field else 0.3,
                  cs_elem=cs)
    U = I.random_smooth(N, nelem, seed=51, noise=0.02)
    V = I.random_directions(U.shape, 8)
    Ut, JV = orc.jvp(s, U, V)
    assert np.array_equal(Ut, orc.time_derivative(s, U))
    h = 1e-6
    fd = (orc.time_derivative(s, U + h * V) - orc.time_derivative(s, U - h * V)) / (2 * h)
    assert np.max(np.abs(JV - fd)) <= 1e-6 * np.max(np.abs(JV))
    # the model's share of the derivative is well above that tolerance
    s0 = orc.Setup(N=N, nelem=nelem, equations=orc.NS, vol_flux=vf, surf_flux=sf, mu=5e-3)
    assert np.max(np.abs(orc.jvp(s0, U, V)[1] - JV)) > 1e-3 * np.max(np.abs(JV))


def test_rollout_jvp_through_the_model(orc):
    N, nelem = 2, (2, 2, 2)
    s = orc.Setup(N=N, nelem=nelem, equations=orc.NS, vol_flux=1, surf_flux=1, mu=5e-3, Cs=0.2)
    U = I.random_smooth(N, nelem, seed=52, noise=0.02)
    V = I.random_directions(U.shape, 9)
    dt = 0.5 * orc.max_dt(s, U, 0.5)
    _, JV = orc.rk_jvp(s, U, V, dt, 2)
    h = 1e-6
    fd = (orc.rk_steps(s, U + h * V, dt, 2) - orc.rk_steps(s, U - h * V, dt, 2)) / (2 * h)
    assert np.max(np.abs(JV - fd)) <= 1e-6 * np.max(np.abs(JV))
