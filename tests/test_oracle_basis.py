"""Pins of the oracle's LGL basis: closed-form nodes/weights, exactness of D,
the summation-by-parts property and the orthonormal Legendre Vandermonde."""
import numpy as np
import pytest
from numpy.polynomial import legendre as leg

CLOSED = {
    1: ([-1.0, 1.0], [1.0, 1.0]),
    2: ([-1.0, 0.0, 1.0], [1 / 3, 4 / 3, 1 / 3]),
    3: ([-1.0, -1 / np.sqrt(5), 1 / np.sqrt(5), 1.0], [1 / 6, 5 / 6, 5 / 6, 1 / 6]),
    4: ([-1.0, -np.sqrt(3 / 7), 0.0, np.sqrt(3 / 7), 1.0], [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10]),
}


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_closed_form_nodes_weights(orc, N):
    b = orc.basis(N)
    xi, w = CLOSED[N]
    assert np.allclose(b["xi"], xi, rtol=0, atol=1e-15)
    assert np.allclose(b["w"], w, rtol=0, atol=1e-15)


@pytest.mark.parametrize("N", range(1, 9))
def test_weights_nodes_D(orc, N):
    b = orc.basis(N)
    xi, w, D = b["xi"], b["w"], b["D"]
    assert abs(w.sum() - 2.0) < 1e-14
    # LGL quadrature is exact up to degree 2N-1
    for k in range(2 * N):
        exact = (1 - (-1) ** (k + 1)) / (k + 1)
        assert abs(np.dot(w, xi ** k) - exact) < 1e-13
    # D differentiates polynomials of degree <= N exactly
    for k in range(N + 1):
        d = k * xi ** (k - 1) if k > 0 else np.zeros_like(xi)
        assert np.max(np.abs(D @ xi ** k - d)) < 1e-12 * max(1, k * N)
    # SBP: W D + (W D)^T = diag(-1, 0, ..., 0, 1)
    Q = np.diag(w) @ D
    B = np.zeros_like(Q)
    B[0, 0], B[-1, -1] = -1.0, 1.0
    assert np.max(np.abs(Q + Q.T - B)) < 1e-14 * max(1, N)


@pytest.mark.parametrize("N", range(1, 9))
def test_dhat_and_edges(orc, N):
    b = orc.basis(N)
    D, Dh, w, xi, edge = b["D"], b["Dhat"], b["w"], b["xi"], b["edge"]
    R = 2 * D.copy()
    R[0, 0] += 1 / w[0]
    R[-1, -1] -= 1 / w[-1]
    assert np.max(np.abs(Dh - R)) < 1e-13 * N * N
    assert Dh[0, 0] == 0.0 and Dh[N, N] == 0.0
    # split-form skew property: w_i Dhat_il + w_l Dhat_li = 0 except at the two corners
    S = np.diag(w) @ Dh
    assert np.max(np.abs(S + S.T)) < 1e-13 * N * N
    # subcell edges enclose the nodes and have width w_i
    assert abs(edge[0] + 1) < 1e-16 and abs(edge[-1] - 1) < 1e-14
    assert np.all(edge[:-1] <= xi + 1e-15) and np.all(xi <= edge[1:] + 1e-15)
    assert np.allclose(np.diff(edge), w, atol=1e-15)


@pytest.mark.parametrize("N", [2, 5, 7])
def test_vandermonde_inverse(orc, N):
    """Vinv inverts the orthonormal Legendre Vandermonde evaluated by numpy."""
    b = orc.basis(N)
    xi = b["xi"]
    V = np.stack([np.sqrt((2 * j + 1) / 2) * leg.legval(xi, np.eye(N + 1)[j]) for j in range(N + 1)], axis=1)
    assert np.max(np.abs(b["Vinv"] @ V - np.eye(N + 1))) < 1e-13
    # the nodes are the roots of (1 - x^2) L_N'
    c = np.zeros(N + 1)
    c[N] = 1
    assert np.max(np.abs((1 - xi ** 2) * leg.legval(xi, leg.legder(c)))) < 1e-13
