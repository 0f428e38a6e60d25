"""Flux-level pins of the oracle: consistency and symmetry of the two-point
fluxes, the Roe property (full upwinding for supersonic states), the LLF
dissipation form and f*(U, U) = F(U)."""
import numpy as np
import pytest

from paper_2306_12891_amd.inputs import from_primitive

G = 1.4


def state(rho, u, v, w, p):
    return from_primitive(np.array([rho]), np.array([u]), np.array([v]), np.array([w]), np.array([p]), G)[0]


def euler_flux(U, d):
    """Physical flux written out here, independently of the oracle."""
    rho, m, E = U[0], U[1:4], U[4]
    u = m / rho
    p = (G - 1) * (E - 0.5 * rho * u @ u)
    F = np.zeros(5)
    F[0] = m[d]
    F[1:4] = m * u[d]
    F[1 + d] += p
    F[4] = (E + p) * u[d]
    return F


rng = np.random.default_rng(3)
STATES = [state(1.0 + 0.5 * rng.random(), *(rng.standard_normal(3)), 0.5 + rng.random()) for _ in range(6)]


@pytest.mark.parametrize("vf", [0, 1, 2, 3])
@pytest.mark.parametrize("d", [0, 1, 2])
def test_two_point_consistent_symmetric(orc, vf, d):
    s = orc.Setup(N=3, vol_flux=vf)
    for a in STATES:
        assert np.allclose(orc.two_point_flux(s, d, a, a), euler_flux(a, d), rtol=1e-14, atol=1e-14)
        assert np.allclose(orc.physical_flux(s, d, a), euler_flux(a, d), rtol=1e-15, atol=1e-15)
    for a, b in zip(STATES[:-1], STATES[1:]):
        fab, fba = orc.two_point_flux(s, d, a, b), orc.two_point_flux(s, d, b, a)
        assert np.allclose(fab, fba, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("sf", [0, 1, 2])
@pytest.mark.parametrize("vf", [0, 1, 3])
def test_surface_consistent(orc, sf, vf):
    s = orc.Setup(N=3, vol_flux=vf, surf_flux=sf)
    for d in range(3):
        for a in STATES:
            assert np.allclose(orc.surface_flux(s, d, a, a), euler_flux(a, d), rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("d", [0, 1, 2])
@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_roe_supersonic_upwind(orc, d, sign):
    """All Roe waves travel one way when |u_n| > c on both sides; then the Roe
    property (dissipation = F(R) - F(L)) turns f* into the upwind flux.  This
    holds only if the Roe averages, wave strengths and eigenvectors are all right."""
    s = orc.Setup(N=3, vol_flux=3, surf_flux=1)
    for k in range(5):
        uL = np.array(rng.standard_normal(3)) * 0.3
        uR = np.array(rng.standard_normal(3)) * 0.3
        uL[d] = sign * (3.0 + rng.random())
        uR[d] = sign * (3.0 + rng.random())
        L = state(1.0 + 0.3 * rng.random(), *uL, 0.6 + 0.3 * rng.random())
        R = state(0.7 + 0.3 * rng.random(), *uR, 0.5 + 0.3 * rng.random())
        f = orc.surface_flux(s, d, L, R)
        ref = euler_flux(L, d) if sign > 0 else euler_flux(R, d)
        assert np.allclose(f, ref, rtol=1e-12, atol=1e-12), (f, ref)


@pytest.mark.parametrize("d", [0, 1, 2])
def test_roe_dissipation_annihilates_shear_only_when_un_zero(orc, d):
    """A pure tangential-velocity jump with u_n = 0 is a contact/shear wave of
    speed 0: the Roe flux then equals its central part."""
    s = orc.Setup(N=3, vol_flux=3, surf_flux=1)
    ut = np.zeros(3)
    ut[(d + 1) % 3] = 0.7
    L = state(1.0, *np.zeros(3), 1.0)
    R = state(1.0, *ut, 1.0)
    f = orc.surface_flux(s, d, L, R)
    central = 0.5 * (euler_flux(L, d) + euler_flux(R, d))
    assert np.allclose(f, central, atol=1e-14)


@pytest.mark.parametrize("vf", [0, 1])
def test_llf_form(orc, vf):
    s = orc.Setup(N=3, vol_flux=vf, surf_flux=0)
    sc = orc.Setup(N=3, vol_flux=vf, surf_flux=2)
    for d in range(3):
        for L, R in zip(STATES[:-1], STATES[1:]):
            def speed(U):
                u = U[1:4] / U[0]
                p = (G - 1) * (U[4] - 0.5 * U[0] * u @ u)
                return abs(u[d]) + np.sqrt(G * p / U[0])
            lam = max(speed(L), speed(R))
            f = orc.surface_flux(s, d, L, R)
            ref = orc.surface_flux(sc, d, L, R) - 0.5 * lam * (R - L)
            assert np.allclose(f, ref, rtol=1e-14, atol=1e-14)
