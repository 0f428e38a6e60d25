"""Pins of the indicator, the blending coefficient, the FV subcell operator and
the blended scheme (paper Sec. 4.1 and 4.2)."""
import numpy as np
import pytest
from numpy.polynomial import legendre as leg

from paper_2306_12891_amd import inputs as I

G = 1.4
S_SHARP = np.log(9999.0)  # alpha0(E = 0) = 1e-4


def T_paper(N):
    # threshold printed with the blending sigmoid (paper Sec. 4.1)
    return 0.5 * 10 ** (-1.8 * (N + 1) ** 0.25)


def state_from_q(q, N, ne):
    """u = 0, rho = 1, p = q: the indicator quantity rho*p equals q."""
    n1 = N + 1
    q = np.broadcast_to(q, (ne, n1, n1, n1))
    one = np.ones_like(q)
    return I.from_primitive(one, 0 * q, 0 * q, 0 * q, q, G)


def modal_energy_fraction(q, N):
    """(E_N, E_{N-1}) from an independent numpy modal transform."""
    x = I.lgl_points(N)
    V = np.stack([np.sqrt((2 * j + 1) / 2) * leg.legval(x, np.eye(N + 1)[j]) for j in range(N + 1)], 1)
    Vi = np.linalg.inv(V)
    qh = np.einsum("ck,bj,ai,kji->cba", Vi, Vi, Vi, q)
    a = np.arange(N + 1)
    m = np.maximum(np.maximum(a[:, None, None], a[None, :, None]), a[None, None, :])
    S = [np.sum(qh ** 2 * (m <= k)) for k in (N, N - 1, N - 2)]
    return (S[0] - S[1]) / S[0], (S[1] - S[2]) / S[1]


def test_threshold_values(orc):
    for N in range(2, 9):
        assert abs(orc.threshold(N) - T_paper(N)) < 1e-18
    assert abs(T_paper(3) - 1.4236e-3) < 1e-7 and abs(T_paper(5) - 7.6176e-4) < 1e-8


@pytest.mark.parametrize("N", [3, 5])
def test_indicator_special_cases(orc, N):
    x = I.lgl_points(N)
    X = x[None, None, :] * np.ones((N + 1, N + 1, 1))
    Y = x[None, :, None] * np.ones((N + 1, 1, N + 1))
    s = orc.Setup(N=N, nelem=(1, 1, 1), blending=1)
    # degree <= N-2 in every direction: no top-mode energy, alpha0 = 1e-4 -> alpha = 0
    q = 1.0 + 0.3 * X ** (N - 2) * Y + 0.1 * Y ** (N - 2)
    E, a1, al = orc.alpha(s, state_from_q(q, N, 1))
    assert E[0] < 1e-25 and a1[0] == 0.0 and al[0] == 0.0
    # pure top mode in x: E = 1 -> alpha clipped at alpha_max
    q = leg.legval(X, np.eye(N + 1)[N])
    E, a1, al = orc.alpha(s, state_from_q(q, N, 1))
    assert abs(E[0] - 1.0) < 1e-13 and abs(al[0] - 0.7) < 1e-15
    # E = T(N): the sigmoid sits at 1/2 (independent modal energies confirm E)
    T = T_paper(N)
    c0 = 1.0
    a = np.sqrt(2 * T * c0 ** 2 / (1 - T))
    q = c0 + a * np.sqrt((2 * N + 1) / 2) * leg.legval(X, np.eye(N + 1)[N])
    EN, EN1 = modal_energy_fraction(q, N)
    assert abs(EN - T) < 1e-14 and EN1 < 1e-25
    E, a1, al = orc.alpha(s, state_from_q(q, N, 1))
    assert abs(E[0] - T) < 1e-14 and abs(a1[0] - 0.5) < 1e-9


def test_indicator_matches_independent_modal_energy(orc):
    N = 4
    ne = 4
    U = I.random_smooth(N, (ne, 1, 1), seed=3, noise=0.05)
    rho = U[:, 0]
    u = U[:, 1:4] / rho[:, None]
    p = (G - 1) * (U[:, 4] - 0.5 * rho * np.sum(u * u, 1))
    s = orc.Setup(N=N, nelem=(ne, 1, 1), blending=1)
    E, a1, al = orc.alpha(s, U)
    for e in range(ne):
        EN, EN1 = modal_energy_fraction(rho[e] * p[e], N)
        assert abs(E[e] - max(EN, EN1)) < 1e-13
        a0 = 1 / (1 + np.exp(-(S_SHARP / T_paper(N)) * (E[e] - T_paper(N))))
        ref = min(a0, 0.7)
        ref = 0.0 if ref < 0.01 else ref
        assert abs(a1[e] - ref) < 1e-13
    sp = orc.Setup(N=N, nelem=(ne, 1, 1), blending=1, indicator=1)
    Ep, _, _ = orc.alpha(sp, U)
    for e in range(ne):
        assert abs(Ep[e] - modal_energy_fraction(rho[e] * p[e], N)[0]) < 1e-13


def _hot_mesh(N, hot_q):
    n = 3
    ne = n ** 3
    x = I.lgl_points(N)
    X = x[None, None, :] * np.ones((N + 1, N + 1, 1))
    q = np.ones((ne, N + 1, N + 1, N + 1))
    centre = 1 + n * (1 + n * 1)
    q[centre] = hot_q(X)
    return state_from_q(q, N, ne), centre


def test_spread_to_face_neighbours(orc):
    N = 3
    U, c = _hot_mesh(N, lambda X: leg.legval(X, np.eye(N + 1)[N]))
    s = orc.Setup(N=N, nelem=(3, 3, 3), blending=1)
    nbr = orc.neighbors(s)
    _, a1, al = orc.alpha(s, U)
    assert a1[c] == 0.7 and np.count_nonzero(a1) == 1
    want = np.zeros(27)
    want[c] = 0.7
    want[nbr[c]] = 0.35
    assert np.array_equal(al, want)
    assert len(set(nbr[c])) == 6


def test_spread_below_alpha_min_is_dropped(orc):
    """A hot element with alpha1 = 0.015: its neighbours would get 0.0075 < 0.01
    and stay pure DG; the values lie in {0} U [0.01, 0.7]."""
    N = 3
    T = T_paper(N)
    target = 0.015
    E = T + (T / S_SHARP) * np.log(target / (1 - target))
    a = np.sqrt(2 * E / (1 - E))
    U, c = _hot_mesh(N, lambda X: 1.0 + a * np.sqrt((2 * N + 1) / 2) * leg.legval(X, np.eye(N + 1)[N]))
    s = orc.Setup(N=N, nelem=(3, 3, 3), blending=1)
    _, a1, al = orc.alpha(s, U)
    assert abs(a1[c] - target) < 1e-9
    assert np.count_nonzero(al) == 1 and al[c] == a1[c]


def test_alpha_zero_is_pure_dg_bitwise(orc):
    N = 4
    s = orc.Setup(N=N, nelem=(2, 2, 1), blending=1)
    U = I.random_smooth(N, (2, 2, 1), seed=8, noise=0.02)
    Ut, Udg, Ufv, al = orc.time_derivative(s, U, alpha=np.zeros(4), parts=True)
    assert np.array_equal(Ut, Udg)
    s0 = orc.Setup(N=N, nelem=(2, 2, 1), blending=0)
    assert np.array_equal(Ut, orc.time_derivative(s0, U))


def fv_first_order_numpy(U, N, nelem, lo, hi):
    """Independent first-order FV on the LGL subcell grid (subcell widths w_i),
    arithmetic-mean central flux with LLF (Davis) dissipation, periodic."""
    x = I.lgl_points(N)
    w = 2.0 / (N * (N + 1) * leg.legval(x, np.eye(N + 1)[N]) ** 2)
    nx, ny, nz = nelem
    n1 = N + 1
    # global structured grid of subcells: (5, Z, Y, X)
    Ug = U.reshape(nz, ny, nx, 5, n1, n1, n1).transpose(3, 0, 4, 1, 5, 2, 6).reshape(5, nz * n1, ny * n1, nx * n1)

    def flux(Us, d):
        rho = Us[0]
        u = Us[1:4] / rho
        p = (G - 1) * (Us[4] - 0.5 * rho * np.sum(u * u, 0))
        F = np.empty_like(Us)
        F[0] = Us[1 + d]
        F[1:4] = Us[1:4] * u[d]
        F[1 + d] += p
        F[4] = (Us[4] + p) * u[d]
        return F, np.abs(u[d]) + np.sqrt(G * p / rho)

    Ut = np.zeros_like(Ug)
    for d in range(3):
        ax = 3 - d
        dxd = (hi[d] - lo[d]) / nelem[d]
        width = np.tile(w, nelem[d]) * dxd / 2
        UL = Ug
        UR = np.roll(Ug, -1, axis=ax)
        FL, lL = flux(UL, d)
        FR, lR = flux(UR, d)
        Fh = 0.5 * (FL + FR) - 0.5 * np.maximum(lL, lR) * (UR - UL)  # flux at right edge of each subcell
        shape = [1, 1, 1, 1]
        shape[ax] = -1
        Ut -= (Fh - np.roll(Fh, 1, axis=ax)) / width.reshape(shape)
    return Ut.reshape(5, nz, n1, ny, n1, nx, n1).transpose(1, 3, 5, 0, 2, 4, 6).reshape(U.shape)


@pytest.mark.parametrize("N", [2, 4])
def test_alpha_one_first_order_is_plain_fv(orc, N):
    nelem, lo, hi = (3, 2, 2), (0.0, 0.0, 0.0), (1.0, 0.5, 0.7)
    s = orc.Setup(N=N, nelem=nelem, lo=lo, hi=hi, vol_flux=3, surf_flux=0, blending=1, fv_recon=0)
    U = I.random_smooth(N, nelem, lo, hi, seed=9, noise=0.05)
    ne = int(np.prod(nelem))
    Ut = orc.time_derivative(s, U, alpha=np.ones(ne))
    ref = fv_first_order_numpy(U, N, nelem, lo, hi)
    scale = np.max(np.abs(ref), axis=(0, 2, 3, 4))
    assert np.all(np.max(np.abs(Ut - ref), axis=(0, 2, 3, 4)) < 1e-13 * scale)


def fv_muscl_numpy(U, N, nelem, lo, hi, slope="minmod"):
    """Independent second-order FV on the LGL subcell grid, periodic: the
    primitive variables are reconstructed linearly in each subcell with a
    limited slope built from the divided differences a, b to the two
    neighbouring nodes; the first and last subcell of every element stay
    first order; arithmetic-mean flux with LLF (Davis) dissipation.
    slope: "minmod" (the textbook (sgn a + sgn b)/2 min(|a|, |b|)), or, to
    show that the comparison can tell limiters apart, "larger" (the other
    one-sided slope where a and b agree in sign) and "central" ((a + b)/2,
    unlimited)."""
    x = I.lgl_points(N)
    w = 2.0 / (N * (N + 1) * leg.legval(x, np.eye(N + 1)[N]) ** 2)
    edges = -1.0 + np.concatenate([[0.0], np.cumsum(w)])
    nx, ny, nz = nelem
    n1 = N + 1
    Ug = U.reshape(nz, ny, nx, 5, n1, n1, n1).transpose(3, 0, 4, 1, 5, 2, 6).reshape(5, nz * n1, ny * n1, nx * n1)

    def prim(Us):
        u = Us[1:4] / Us[0]
        return np.concatenate([Us[:1], u, (G - 1) * (Us[4:] - 0.5 * Us[0] * np.sum(u * u, 0))])

    def flux(W, d):
        rho, u, p = W[0], W[1:4], W[4]
        Us = np.concatenate([W[:1], rho * u, (p / (G - 1) + 0.5 * rho * np.sum(u * u, 0))[None]])
        F = Us * u[d]
        F[1 + d] += p
        F[4] += p * u[d]
        return F, Us, np.abs(u[d]) + np.sqrt(G * p / rho)

    W = prim(Ug)
    Ut = np.zeros_like(Ug)
    for d in range(3):
        ax, ne = 3 - d, nelem[d]
        dxd = (hi[d] - lo[d]) / ne
        shape = [1, 1, 1, 1]
        shape[ax] = -1
        at = lambda ref: ((2.0 * np.arange(ne)[:, None] + 1.0 + ref[None, :]) * dxd / 2).reshape(shape)
        xn, xl, xr = at(x), at(edges[:-1]), at(edges[1:])  # nodes, left and right subcell edges
        with np.errstate(divide="ignore", invalid="ignore"):  # element ends: masked below
            a = (W - np.roll(W, 1, axis=ax)) / (xn - np.roll(xn, 1, axis=ax))
            b = (np.roll(W, -1, axis=ax) - W) / (np.roll(xn, -1, axis=ax) - xn)
            agree = 0.5 * (np.sign(a) + np.sign(b))
            if slope == "minmod":
                sig = agree * np.minimum(np.abs(a), np.abs(b))
            elif slope == "larger":
                sig = agree * np.maximum(np.abs(a), np.abs(b))
            else:
                sig = 0.5 * (a + b)
        inner = np.tile((np.arange(n1) > 0) & (np.arange(n1) < N), ne).reshape(shape)
        sig = np.where(inner, sig, 0.0)
        FL, UL, lL = flux(W + sig * (xr - xn), d)  # right-edge value of each subcell
        FR, UR, lR = flux(np.roll(W + sig * (xl - xn), -1, axis=ax), d)  # left-edge value of the next
        Fh = 0.5 * (FL + FR) - 0.5 * np.maximum(lL, lR) * (UR - UL)
        Ut -= (Fh - np.roll(Fh, 1, axis=ax)) / (np.tile(w, ne) * dxd / 2).reshape(shape)
    return Ut.reshape(5, nz, n1, ny, n1, nx, n1).transpose(1, 3, 5, 0, 2, 4, 6).reshape(U.shape)


@pytest.mark.parametrize("N", [2, 3, 4, 6])
def test_alpha_one_minmod_is_independent_muscl_fv(orc, N):
    """The minmod subcell reconstruction on non-linear data (extrema, where
    the slope is zero, and monotone stretches with unequal one-sided slopes,
    where the smaller one is kept) equals an independent numpy MUSCL scheme;
    the same scheme with the larger slope or the unlimited central slope is
    far off, so the comparison fixes the limiter's choice."""
    nelem, lo, hi = (3, 2, 2), (0.0, 0.0, 0.0), (1.0, 0.5, 0.7)
    s = orc.Setup(N=N, nelem=nelem, lo=lo, hi=hi, vol_flux=3, surf_flux=0, blending=1, fv_recon=1)
    U = I.random_smooth(N, nelem, lo, hi, seed=9 + N, noise=0.05)
    ne = int(np.prod(nelem))
    Ut = orc.time_derivative(s, U, alpha=np.ones(ne))
    ref = fv_muscl_numpy(U, N, nelem, lo, hi)
    scale = np.max(np.abs(ref), axis=(0, 2, 3, 4))
    err = lambda v: np.max(np.abs(Ut - v), axis=(0, 2, 3, 4)) / scale
    assert np.all(err(ref) < 1e-13)
    assert np.all(err(fv_muscl_numpy(U, N, nelem, lo, hi, "larger")) > 1e-3)
    assert np.all(err(fv_muscl_numpy(U, N, nelem, lo, hi, "central")) > 1e-3)
    assert np.all(err(fv_first_order_numpy(U, N, nelem, lo, hi)) > 1e-3)


@pytest.mark.parametrize("N", range(1, 8))
def test_subcell_edges_interlace_nodes(N):
    """Each interior subcell edge (the edges sit at the cumulative quadrature
    weights) lies strictly between the two LGL nodes it separates.  So a minmod face value w_m + s (x_edge - x_m), with
    |s| at most the one-sided divided difference towards that edge and of its
    sign, lies between w_m and the neighbouring node's value: for states with
    positive density and pressure at every node the reconstruction never
    produces a non-positive face state, and the first-order fallback the
    subcell scheme keeps for that case is reached only by states that are
    invalid already at a node."""
    x = I.lgl_points(N)
    w = 2.0 / (N * (N + 1) * leg.legval(x, np.eye(N + 1)[N]) ** 2)
    edges = -1.0 + np.concatenate([[0.0], np.cumsum(w)])
    assert abs(edges[-1] - 1.0) < 1e-14
    assert edges[0] == x[0] == -1.0 and x[-1] == 1.0
    assert np.all(edges[1:-1] > x[:-1]) and np.all(edges[1:-1] < x[1:])


def test_minmod_exact_on_linear_data(orc):
    """rho linear inside each element, u = 0, p = 1: minmod reconstructs the
    interior subcell interfaces exactly, so only subcells touching a first-order
    interface see a density change; first-order reconstruction changes all."""
    N = 5
    x = I.lgl_points(N)
    ne = 2
    rho = np.empty((ne, N + 1, N + 1, N + 1))
    rho[0] = 1.0 + 0.1 * x[None, None, :]
    rho[1] = 1.3 - 0.2 * x[None, None, :]
    z = np.zeros_like(rho)
    U = I.from_primitive(rho, z, z, z, np.ones_like(rho), G)
    for recon in (1, 0):
        s = orc.Setup(N=N, nelem=(ne, 1, 1), lo=(0, 0, 0), hi=(1, 1, 1), blending=1, fv_recon=recon)
        Ut = orc.time_derivative(s, U, alpha=np.ones(ne))
        r = np.abs(Ut[:, 0]).max(axis=(1, 2))  # per element, per x-subcell
        if recon == 1:
            assert np.all(r[:, 2:N - 1] < 1e-14) and np.all(r[:, [0, 1, N - 1, N]] > 1e-6)
        else:
            assert np.all(r > 1e-6)


# ---------------------------------------------------------------------------
# Sod shock tube (periodic in x: the jump at x = 0.5 and its mirror at x = 0).
# ---------------------------------------------------------------------------
def exact_riemann(WL, WR, xi_arr):
    """Exact ideal-gas Riemann solution (rho, u, p) at similarity coordinates xi = x/t."""
    rl, ul, pl = WL
    rr, ur, pr = WR
    cl, cr = np.sqrt(G * pl / rl), np.sqrt(G * pr / rr)

    def f(p, r, pk, ck):
        if p > pk:
            A, B = 2 / ((G + 1) * r), (G - 1) / (G + 1) * pk
            return (p - pk) * np.sqrt(A / (p + B))
        return 2 * ck / (G - 1) * ((p / pk) ** ((G - 1) / (2 * G)) - 1)

    from scipy.optimize import brentq
    ps = brentq(lambda p: f(p, rl, pl, cl) + f(p, rr, pr, cr) + ur - ul, 1e-10, 100.0, xtol=1e-15)
    us = 0.5 * (ul + ur) + 0.5 * (f(ps, rr, pr, cr) - f(ps, rl, pl, cl))
    out = np.zeros((3, len(xi_arr)))
    for n, s in enumerate(xi_arr):
        if s < us:  # left of contact
            r, u, p, ck = rl, ul, pl, cl
            if ps > p:
                S = u - ck * np.sqrt((G + 1) / (2 * G) * ps / p + (G - 1) / (2 * G))
                out[:, n] = (r * (ps / p + (G - 1) / (G + 1)) / ((G - 1) / (G + 1) * ps / p + 1), us, ps) if s > S else (r, u, p)
            else:
                cs = ck * (ps / p) ** ((G - 1) / (2 * G))
                if s < u - ck:
                    out[:, n] = (r, u, p)
                elif s > us - cs:
                    out[:, n] = (r * (ps / p) ** (1 / G), us, ps)
                else:
                    uf = 2 / (G + 1) * (ck + (G - 1) / 2 * u + s)
                    cf = 2 / (G + 1) * (ck + (G - 1) / 2 * (u - s))
                    out[:, n] = (r * (cf / ck) ** (2 / (G - 1)), uf, p * (cf / ck) ** (2 * G / (G - 1)))
        else:
            r, u, p, ck = rr, ur, pr, cr
            if ps > p:
                S = u + ck * np.sqrt((G + 1) / (2 * G) * ps / p + (G - 1) / (2 * G))
                out[:, n] = (r * (ps / p + (G - 1) / (G + 1)) / ((G - 1) / (G + 1) * ps / p + 1), us, ps) if s < S else (r, u, p)
            else:
                cs = ck * (ps / p) ** ((G - 1) / (2 * G))
                if s > u + ck:
                    out[:, n] = (r, u, p)
                elif s < us + cs:
                    out[:, n] = (r * (ps / p) ** (1 / G), us, ps)
                else:
                    uf = 2 / (G + 1) * (-ck + (G - 1) / 2 * u + s)
                    cf = 2 / (G + 1) * (ck - (G - 1) / 2 * (u - s))
                    out[:, n] = (r * (cf / ck) ** (2 / (G - 1)), uf, p * (cf / ck) ** (2 * G / (G - 1)))
    return out, ps, us


def sod_exact_rho(x, t):
    """Both non-interacting Riemann problems of the periodic tube (t < 0.1427)."""
    L, R = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    xc = np.where(x > 0.75, x - 1.0, x)  # nearest jump: 0.5, or 0 == 1
    out = np.empty_like(x)
    near_half = np.abs(x - 0.5) < 0.25
    a, _, _ = exact_riemann(L, R, (x[near_half] - 0.5) / t)
    out[near_half] = a[0]
    b, _, _ = exact_riemann(R, L, xc[~near_half] / t)
    out[~near_half] = b[0]
    return out


def test_sod_star_state():
    _, ps, us = exact_riemann((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), np.array([0.0]))
    assert abs(ps - 0.30313) < 1e-5 and abs(us - 0.92745) < 1e-5


@pytest.mark.slow
def test_sod_blended_converges(orc):
    """Blended KG/LLF with minmod subcells on the quasi-1-D Sod tube at N = 5
    (cells as long in y and z as in x, so the time step is that of the 3-D
    tube): the L1 density error against the exact solution shrinks under
    refinement and the solution stays free of large over/undershoots."""
    N, t_end = 5, 0.1
    errs = []
    for nx in (32, 64):
        nelem, lo, hi = (nx, 1, 1), (0, 0, 0), (1.0, 1.0 / nx, 1.0 / nx)
        s = orc.Setup(N=N, nelem=nelem, lo=lo, hi=hi, blending=1, fv_recon=1)
        U = I.sod(N, nelem, lo, hi)
        dt = orc.max_dt(s, U, 0.5)
        ns = int(np.ceil(t_end / dt))
        U1 = orc.rk_steps(s, U, t_end / ns, ns)
        X, _, _ = I.node_coordinates(N, nelem, lo, hi)
        rho = U1[:, 0]
        ex = sod_exact_rho(X.ravel(), t_end).reshape(X.shape)
        wq = orc.integrals(s, np.repeat(np.abs(rho - ex)[:, None], 5, 1))[0] * nx * nx
        errs.append(wq)
        assert rho.min() > 0.125 - 0.02 and rho.max() < 1.0 + 0.02
    assert errs[1] < 0.75 * errs[0], errs


def blended_noisy_state(N=3, nelem=(3, 3, 2)):
    """Smooth state with element-wise scaled node noise: blending coefficients
    strictly inside (alpha_min, alpha_max), from the elements' own indicator
    and from the neighbour spread, with no ties."""
    base = I.random_smooth(N, nelem, seed=12, amp=0.1)
    ne = int(np.prod(nelem))
    fac = np.random.default_rng(5).uniform(0.2, 1.0, ne)[:, None, None, None, None]
    return base * (1 + np.random.default_rng(99).standard_normal(base.shape) * 0.05 * fac)


def test_jvp_through_blending_matches_central_differences(orc):
    """The dual-number JVP of the blended operator includes the derivative of
    the blending coefficient (indicator sigmoid, clip, spread) and of the
    minmod reconstruction; central differences (eps = 1e-6) agree to 1e-7 of
    max |J v|.  With alpha held fixed the result differs by the alpha part."""
    N, nelem = 3, (3, 3, 2)
    s = orc.Setup(N=N, nelem=nelem, blending=1, fv_recon=orc.FV_MINMOD, vol_flux=orc.KG, surf_flux=orc.LLF)
    U = blended_noisy_state(N, nelem)
    _, _, al = orc.alpha(s, U)
    assert np.sum((al > 0.02) & (al < 0.69)) >= 6
    eps = 1e-6
    for k in range(2):
        v = I.random_directions(U.shape, k)
        _, Jv = orc.jvp(s, U, v)
        fd = (orc.time_derivative(s, U + eps * v) - orc.time_derivative(s, U - eps * v)) / (2 * eps)
        scale = np.max(np.abs(Jv))
        assert np.max(np.abs(fd - Jv)) <= 1e-7 * scale
        fixed = (orc.time_derivative(s, U + eps * v, alpha=al) - orc.time_derivative(s, U - eps * v, alpha=al)) / (
            2 * eps)
        assert np.max(np.abs(fixed - Jv)) > 1e-2 * scale


# ---------------------------------------------------------------------------
# Navier-Stokes with blending.  Reading: only the advective operator is
# blended (the FV subcell scheme carries no viscous terms); the BR1 viscous
# terms enter with weight one in every element.
# ---------------------------------------------------------------------------
def _ns(orc, N, nelem, blending, eq=1, mu=2e-2, **kw):
    return orc.Setup(N=N, nelem=nelem, equations=eq, mu=mu, blending=blending, fv_recon=orc.FV_MINMOD,
                     vol_flux=orc.KG, surf_flux=orc.LLF, **kw)


def test_ns_blending_leaves_viscous_terms_unweighted(orc):
    """For any fixed alpha field, NS-blended minus Euler-blended equals the
    unblended NS minus Euler operator: the viscous terms do not depend on
    alpha."""
    N, nelem = 3, (3, 2, 2)
    U = I.random_smooth(N, nelem, seed=21, noise=0.03)
    visc = orc.time_derivative(_ns(orc, N, nelem, 0), U) - orc.time_derivative(_ns(orc, N, nelem, 0, eq=0), U)
    assert np.max(np.abs(visc)) > 1e-3 * np.max(np.abs(orc.time_derivative(_ns(orc, N, nelem, 0), U)))
    rng = np.random.default_rng(3)
    for alpha in (np.zeros(12), np.ones(12), rng.uniform(0, 1, 12)):
        d = orc.time_derivative(_ns(orc, N, nelem, 1), U, alpha=alpha) - orc.time_derivative(
            _ns(orc, N, nelem, 1, eq=0), U, alpha=alpha)
        assert np.max(np.abs(d - visc)) <= 1e-13 * np.max(np.abs(visc)) * 100


def test_ns_alpha_zero_is_unblended_bitwise(orc):
    N, nelem = 4, (2, 2, 1)
    U = I.random_smooth(N, nelem, seed=22, noise=0.02)
    Ut = orc.time_derivative(_ns(orc, N, nelem, 1), U, alpha=np.zeros(4))
    assert np.array_equal(Ut, orc.time_derivative(_ns(orc, N, nelem, 0), U))


@pytest.mark.parametrize("N", [2, 4])
def test_ns_alpha_one_is_plain_fv_plus_viscous(orc, N):
    """alpha = 1 with first-order subcells: the independent numpy FV scheme
    plus the unblended viscous terms."""
    nelem, lo, hi = (3, 2, 2), (0.0, 0.0, 0.0), (1.0, 0.5, 0.7)
    U = I.random_smooth(N, nelem, lo, hi, seed=23, noise=0.02)
    mk = lambda eq, b: orc.Setup(N=N, nelem=nelem, lo=lo, hi=hi, equations=eq, mu=1e-2, vol_flux=3, surf_flux=0,
                                 blending=b, fv_recon=0)
    visc = orc.time_derivative(mk(1, 0), U) - orc.time_derivative(mk(0, 0), U)
    Ut = orc.time_derivative(mk(1, 1), U, alpha=np.ones(12))
    ref = fv_first_order_numpy(U, N, nelem, lo, hi) + visc
    assert np.max(np.abs(Ut - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_ns_blended_freestream_and_conservation(orc):
    N, nelem = 4, (3, 2, 2)
    rng = np.random.default_rng(4)
    alpha = rng.uniform(0, 1, 12)
    s = _ns(orc, N, nelem, 1)
    Uf = I.freestream(N, nelem, u=(0.4, -0.3, 0.2))
    assert np.max(np.abs(orc.time_derivative(s, Uf, alpha=alpha))) <= 1e-13 * 10 * N * N
    U = I.random_smooth(N, nelem, seed=24, noise=0.05)
    Ut = orc.time_derivative(s, U, alpha=alpha)
    I_ = orc.integrals(s, Ut)
    scale = orc.integrals(s, np.abs(Ut))
    assert np.all(np.abs(I_) < 1e-13 * scale)


@pytest.mark.parametrize("eq", [1, 2])
def test_ns_jvp_through_blending_matches_central_differences(orc, eq):
    """Indicator-driven alpha with Navier-Stokes (eq 2: with the Smagorinsky
    model): dual numbers against central differences to 1e-7 of max |J v|."""
    N, nelem = 3, (3, 3, 2)
    s = _ns(orc, N, nelem, 1, eq=1, mu=5e-3, Cs=0.2 if eq == 2 else 0.0)
    U = blended_noisy_state(N, nelem)
    _, _, al = orc.alpha(s, U)
    assert np.sum((al > 0.02) & (al < 0.69)) >= 6
    eps = 1e-6
    for k in range(2):  # directions whose +-eps segment crosses no minmod switch
        v = I.random_directions(U.shape, k)
        _, Jv = orc.jvp(s, U, v)
        fd = (orc.time_derivative(s, U + eps * v) - orc.time_derivative(s, U - eps * v)) / (2 * eps)
        assert np.max(np.abs(fd - Jv)) <= 1e-7 * np.max(np.abs(Jv))


@pytest.mark.parametrize("N", [3, 5])
def test_sharpness_reading(orc, N):
    """The sharpness s of the sigmoid is a reading (the paper does not print
    it): s = ln(9999), so that the raw coefficient of a state without top-mode
    energy is 1e-4.  With alpha_min = 0 and alpha_max = 1 (no cut-off, no
    clip) the raw sigmoid is observable: E = 0 gives 1e-4, E = T/2 gives
    1/(1 + 9999^(1/2)), E = T gives 1/2 (E from the independent numpy modal
    transform)."""
    x = I.lgl_points(N)
    X = x[None, None, :] * np.ones((N + 1, N + 1, 1))
    Y = x[None, :, None] * np.ones((N + 1, 1, N + 1))
    s = orc.Setup(N=N, nelem=(1, 1, 1), blending=1, alpha_min=0.0, alpha_max=1.0)
    q = 1.0 + 0.3 * X ** (N - 2) * Y + 0.1 * Y ** (N - 2)
    E, a1, _ = orc.alpha(s, state_from_q(q, N, 1))
    assert E[0] < 1e-25 and abs(a1[0] - 1e-4) < 1e-15
    T = T_paper(N)
    for frac, expect in ((0.5, 1.0 / (1.0 + 9999.0 ** 0.5)), (1.0, 0.5)):
        Et = frac * T
        a = np.sqrt(2 * Et / (1 - Et))
        q = 1.0 + a * np.sqrt((2 * N + 1) / 2) * leg.legval(X, np.eye(N + 1)[N])
        EN, _ = modal_energy_fraction(q, N)
        assert abs(EN - Et) < 1e-14
        E, a1, _ = orc.alpha(s, state_from_q(q, N, 1))
        assert abs(E[0] - Et) < 1e-14
        # the sigmoid's slope s/T turns the 1e-14 error of E into ~s/T * 1e-14 * a(1-a)
        assert abs(a1[0] - expect) < 1e-9, (frac, a1[0], expect)
