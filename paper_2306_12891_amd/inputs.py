"""Seeded, synthetic initial states shared by the tests, the benchmark and the
oracle-side checks.

This module holds no part of the discretisation: it only samples closed-form
initial conditions at the interpolation nodes and draws seeded random numbers.
It imports nothing else from the package, so the oracle side can use it
without touching the GPU library.

Layout of every state: float64, shape (nElems, 5, N+1, N+1, N+1), variables
(rho, rho*u, rho*v, rho*w, E), x index fastest, elements e = ex + nx*(ey + ny*ez).
Node positions inside an element are the Legendre-Gauss-Lobatto points
(paper Sec. 2, split form on LGL nodes), computed here with numpy's Legendre
polynomials.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as _leg

TWO_PI = 2.0 * np.pi


def lgl_points(N: int) -> np.ndarray:
    """Legendre-Gauss-Lobatto points on [-1, 1]: +-1 and the roots of L_N'."""
    c = np.zeros(N + 1)
    c[N] = 1.0
    inner = np.sort(np.real(_leg.legroots(_leg.legder(c)))) if N > 1 else np.zeros(0)
    return np.concatenate([[-1.0], inner, [1.0]])


def node_coordinates(N: int, nelem, lo, hi):
    """x, y, z arrays of shape (nElems, N+1, N+1, N+1) (index order k, j, i)."""
    nx, ny, nz = nelem
    xi = lgl_points(N)
    dx = [(hi[d] - lo[d]) / nelem[d] for d in range(3)]
    ex = np.arange(nx)
    ey = np.arange(ny)
    ez = np.arange(nz)
    # element index e = ex + nx (ey + ny ez)
    EZ, EY, EX = np.meshgrid(ez, ey, ex, indexing="ij")
    EX, EY, EZ = EX.ravel(), EY.ravel(), EZ.ravel()
    r = (xi + 1.0) / 2.0
    x = lo[0] + (EX[:, None] + r[None, :]) * dx[0]  # (nE, n1) along i
    y = lo[1] + (EY[:, None] + r[None, :]) * dx[1]
    z = lo[2] + (EZ[:, None] + r[None, :]) * dx[2]
    n1 = N + 1
    X = np.broadcast_to(x[:, None, None, :], (len(EX), n1, n1, n1))
    Y = np.broadcast_to(y[:, None, :, None], (len(EX), n1, n1, n1))
    Z = np.broadcast_to(z[:, :, None, None], (len(EX), n1, n1, n1))
    return X, Y, Z


def warped_coordinates(N: int, nelem, lo=(0.0, 0.0, 0.0), hi=(TWO_PI,) * 3, amp: float = 0.04) -> np.ndarray:
    """Node coordinates of a curved periodic mesh, shape (nElems, 3, N+1, N+1, N+1).

    Every Cartesian node (X, Y, Z) of the box is displaced by a smooth periodic
    field, component d by amp * min(L) * sin(2pi(Xt + a_d)) sin(2pi(Yt + b_d))
    sin(2pi(Zt + c_d)) with Xt = (X - lo_x)/L_x etc. and fixed phase offsets, so
    all nine metric terms are non-zero; amp * 2pi < 1 keeps the mapping one to
    one.  Faces shared by two elements get the same physical points.
    """
    X, Y, Z = node_coordinates(N, nelem, lo, hi)
    L = [hi[d] - lo[d] for d in range(3)]
    A = amp * min(L)
    t = [(X - lo[0]) / L[0], (Y - lo[1]) / L[1], (Z - lo[2]) / L[2]]
    ph = [(0.0, 0.1, 0.2), (0.3, 0.0, 0.4), (0.5, 0.6, 0.0)]
    out = []
    for d, base in enumerate((X, Y, Z)):
        a, b, c = ph[d]
        out.append(base + A * np.sin(TWO_PI * (t[0] + a)) * np.sin(TWO_PI * (t[1] + b)) * np.sin(TWO_PI * (t[2] + c)))
    return np.ascontiguousarray(np.stack(out, axis=1), dtype=np.float64)


def _xyz(N, nelem, lo, hi, xnodes):
    if xnodes is None:
        return node_coordinates(N, nelem, lo, hi)
    return xnodes[:, 0], xnodes[:, 1], xnodes[:, 2]


def element_centres(nelem, lo, hi):
    nx, ny, nz = nelem
    dx = [(hi[d] - lo[d]) / nelem[d] for d in range(3)]
    EZ, EY, EX = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return (lo[0] + (EX.ravel() + 0.5) * dx[0], lo[1] + (EY.ravel() + 0.5) * dx[1],
            lo[2] + (EZ.ravel() + 0.5) * dx[2])


def from_primitive(rho, u, v, w, p, gamma: float) -> np.ndarray:
    rho, u, v, w, p = np.broadcast_arrays(rho, u, v, w, p)
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.ascontiguousarray(np.stack([rho, rho * u, rho * v, rho * w, E], axis=1), dtype=np.float64)


def density_wave(N: int, nelem=(4, 4, 4), lo=(0.0, 0.0, 0.0), hi=(TWO_PI,) * 3, gamma: float = 1.4,
                 t: float = 0.0, amp: float = 0.2, xnodes=None) -> np.ndarray:
    """rho = 1 + amp sin(x + y + z - 3t), u = (1, 1, 1), p = 1 (exact Euler solution).
    xnodes: sample at these node coordinates (curved mesh) instead of the box's."""
    X, Y, Z = _xyz(N, nelem, lo, hi, xnodes)
    rho = 1.0 + amp * np.sin(X + Y + Z - 3.0 * t)
    one = np.ones_like(rho)
    return from_primitive(rho, one, one, one, one, gamma)


def tgv(N: int, nelem=(32, 32, 32), Ma: float = 0.1, gamma: float = 1.4, symmetry_break: bool = False,
        seed: int = 7, eps: float = 1e-3, xnodes=None) -> np.ndarray:
    """Taylor-Green vortex on [0, 2pi]^3 with rho0 = U0 = L = 1.

    p0 = 1/(gamma Ma^2); u = sin x cos y cos z, v = -cos x sin y cos z, w = 0;
    p = p0 + (cos 2x + cos 2y)(cos 2z + 2)/16; rho = p / p0 (isothermal start).
    symmetry_break adds eps sin(x+f1) sin(2y+f2) cos(z+f3) to w, phases f ~ U(0, 2pi)
    drawn from numpy's default_rng(seed).  xnodes: sample at these node
    coordinates (curved mesh of the same box).
    """
    X, Y, Z = _xyz(N, nelem, (0.0, 0.0, 0.0), (TWO_PI,) * 3, xnodes)
    p0 = 1.0 / (gamma * Ma * Ma)
    u = np.sin(X) * np.cos(Y) * np.cos(Z)
    v = -np.cos(X) * np.sin(Y) * np.cos(Z)
    w = np.zeros_like(u)
    if symmetry_break:
        ph = np.random.default_rng(seed).uniform(0.0, TWO_PI, size=3)
        w = w + eps * np.sin(X + ph[0]) * np.sin(2.0 * Y + ph[1]) * np.cos(Z + ph[2])
    p = p0 + (np.cos(2.0 * X) + np.cos(2.0 * Y)) * (np.cos(2.0 * Z) + 2.0) / 16.0
    rho = p / p0
    return from_primitive(rho, u, v, w, p, gamma)


def channel(N: int, nelem=(32, 32, 32), lo=(0.0, 0.0, 0.0), hi=(TWO_PI, 2.0, np.pi), Ma: float = 0.7,
            gamma: float = 1.4, seed: int = 11, amp: float = 0.1, modes: int = 4) -> np.ndarray:
    """Channel between walls normal to y (half height h = (hi_y - lo_y)/2,
    centre-line velocity 1, density 1, centre-line Mach number Ma):
    u = 1 - eta^8 (eta = (y - y_c)/h, a flat turbulent-like profile) plus seeded
    smooth perturbations of all three velocity components, amp (1 - eta^2)
    times a sum of periodic Fourier modes in x and z with random phases;
    p = 1/(gamma Ma^2), rho = 1."""
    rng = np.random.default_rng(seed)
    X, Y, Z = _xyz(N, nelem, lo, hi, None)
    Lx, Lz = hi[0] - lo[0], hi[2] - lo[2]
    yc, h = 0.5 * (lo[1] + hi[1]), 0.5 * (hi[1] - lo[1])
    eta = (Y - yc) / h
    env = amp * (1.0 - eta * eta)

    def pert():
        f = np.zeros_like(X)
        for _ in range(modes):
            kx, kz = rng.integers(1, 4, size=2)
            ky = rng.uniform(0.5, 2.0)
            ph = rng.uniform(0, TWO_PI, size=3)
            f = f + np.sin(TWO_PI * kx * (X - lo[0]) / Lx + ph[0]) * np.cos(np.pi * ky * eta + ph[1]) \
                * np.sin(TWO_PI * kz * (Z - lo[2]) / Lz + ph[2])
        return env * f / modes

    u = 1.0 - eta ** 8 + pert()
    v = pert()
    w = pert()
    rho = np.ones_like(u)
    p = np.full_like(u, 1.0 / (gamma * Ma * Ma))
    return from_primitive(rho, u, v, w, p, gamma)


def sod(N: int, nelem=(64, 8, 8), lo=(0.0, 0.0, 0.0), hi=(1.0, 0.125, 0.125), gamma: float = 1.4,
        x0: float = 0.5) -> np.ndarray:
    """Extruded Sod states chosen by element centre: (1, 0, 1) left of x0, (0.125, 0, 0.1) right."""
    n1 = N + 1
    xc, _, _ = element_centres(nelem, lo, hi)
    left = (xc < x0)[:, None, None, None]
    shape = (len(xc), n1, n1, n1)
    rho = np.where(left, 1.0, 0.125) * np.ones(shape)
    p = np.where(left, 1.0, 0.1) * np.ones(shape)
    z = np.zeros(shape)
    return from_primitive(rho, z, z, z, p, gamma)


def freestream(N: int, nelem=(4, 4, 4), lo=(0.0, 0.0, 0.0), hi=(TWO_PI,) * 3, gamma: float = 1.4,
               rho: float = 1.0, u=(0.5, 0.0, 0.0), p=None) -> np.ndarray:
    """Constant state (default Ma 0.5: rho = 1, u = (0.5, 0, 0), p = 1/gamma)."""
    n1 = N + 1
    ne = int(np.prod(nelem))
    if p is None:
        p = 1.0 / gamma
    one = np.ones((ne, n1, n1, n1))
    return from_primitive(rho * one, u[0] * one, u[1] * one, u[2] * one, p * one, gamma)


def random_smooth(N: int, nelem=(3, 2, 2), lo=(0.0, 0.0, 0.0), hi=(TWO_PI,) * 3, gamma: float = 1.4,
                  seed: int = 0, amp: float = 0.1, modes: int = 3, mach: float = 0.5,
                  noise: float = 0.0, xnodes=None) -> np.ndarray:
    """Seeded smooth positive state: sums of low Fourier modes with random phases.

    noise > 0 adds i.i.d. node noise (relative) so that element interfaces are
    discontinuous and every code path of the surface terms is exercised.
    """
    rng = np.random.default_rng(seed)
    X, Y, Z = _xyz(N, nelem, lo, hi, xnodes)
    L = [hi[d] - lo[d] for d in range(3)]

    def field():
        f = np.zeros_like(X)
        for _ in range(modes):
            k = rng.integers(1, 3, size=3)
            ph = rng.uniform(0, TWO_PI, size=3)
            a = rng.uniform(-1.0, 1.0)
            f = f + a * np.sin(TWO_PI * k[0] * X / L[0] + ph[0]) * np.cos(TWO_PI * k[1] * Y / L[1] + ph[1]) \
                * np.sin(TWO_PI * k[2] * Z / L[2] + ph[2])
        return f / modes

    rho = 1.0 + amp * field()
    p = 1.0 / gamma + amp * field() / gamma
    u = mach * (0.5 + field())
    v = mach * field()
    w = mach * field()
    if noise > 0:
        rho = rho * (1.0 + noise * rng.standard_normal(rho.shape))
        p = p * (1.0 + noise * rng.standard_normal(p.shape))
        u = u + noise * rng.standard_normal(u.shape)
    return from_primitive(rho, u, v, w, p, gamma)


def random_directions(shape, k: int, base_seed: int = 1000) -> np.ndarray:
    """Direction k of an i.i.d. N(0, 1) family, seed base_seed + k."""
    return np.random.default_rng(base_seed + k).standard_normal(shape)


def structured_neighbors(nelem) -> np.ndarray:
    """Face neighbours (-x, +x, -y, +y, -z, +z) of the periodic structured mesh."""
    nx, ny, nz = nelem
    e = np.arange(nx * ny * nz)
    ex, ey, ez = e % nx, (e // nx) % ny, e // (nx * ny)
    idx = lambda x, y, z: (x % nx) + nx * ((y % ny) + ny * (z % nz))
    return np.stack([idx(ex - 1, ey, ez), idx(ex + 1, ey, ez), idx(ex, ey - 1, ez), idx(ex, ey + 1, ez),
                     idx(ex, ey, ez - 1), idx(ex, ey, ez + 1)], axis=1)


def cube_rotations():
    """The 24 rotations of the reference cube: signed permutation matrices P
    with det P = +1 (new reference coordinates xi' = P xi)."""
    import itertools
    out = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            P = np.zeros((3, 3), dtype=int)
            for a in range(3):
                P[a, perm[a]] = signs[a]
            if round(np.linalg.det(P)) == 1:
                out.append(P)
    return out


def _face_local(N, d, i, j, k):
    n1 = N + 1
    return (j + n1 * k) if d == 0 else ((i + n1 * k) if d == 1 else (i + n1 * j))


def _face_node_ijk(N, d, l, a):
    n1 = N + 1
    t1, t2 = a % n1, a // n1
    return (l, t1, t2) if d == 0 else ((t1, l, t2) if d == 1 else (t1, t2, l))


def _orient(N, o, a):
    n1 = N + 1
    t1, t2 = a % n1, a // n1
    u, v = (t2, t1) if o & 1 else (t1, t2)
    if o & 2:
        u = N - u
    if o & 4:
        v = N - v
    return u + n1 * v


def rotated_elements(N: int, nelem, seed: int = 0):
    """Unstructured-mesh test case from the periodic structured mesh: the
    reference axes of every element are relabelled by a seeded cube rotation.

    Returns (perm, conn): perm[e][n'] is the node of the structured labelling
    that is node n' after the relabelling (apply as X_new[e][..., n'] =
    X_old[e][..., perm[e][n']] on flattened nodes), and conn[e][f] = (neighbour,
    neighbour's local face, orientation) in the new labelling, orientation o:
    bit 0 swaps the face-local indices (t1, t2), bit 1 reverses the first and
    bit 2 the second of the result (t1 along the lower remaining axis).
    """
    n1 = N + 1
    nn = n1 ** 3
    ne = int(np.prod(nelem))
    rots = cube_rotations()
    rng = np.random.default_rng(seed)
    P = [rots[k] for k in rng.integers(0, len(rots), size=ne)]
    perm = np.zeros((ne, nn), dtype=np.int64)
    new_of_old = np.zeros((ne, nn), dtype=np.int64)
    old_face = np.zeros((ne, 6), dtype=np.int64)  # new face -> old face
    for e in range(ne):
        Pe = P[e]
        src = [int(np.nonzero(Pe[a])[0][0]) for a in range(3)]  # new axis a <- old axis src[a]
        sg = [int(Pe[a, src[a]]) for a in range(3)]
        for np_ in range(nn):
            inew = (np_ % n1, (np_ // n1) % n1, np_ // (n1 * n1))
            iold = [0, 0, 0]
            for a in range(3):
                iold[src[a]] = inew[a] if sg[a] > 0 else N - inew[a]
            o = iold[0] + n1 * (iold[1] + n1 * iold[2])
            perm[e, np_] = o
            new_of_old[e, o] = np_
        for a in range(3):
            for side in range(2):
                old_side = side if sg[a] > 0 else 1 - side
                old_face[e, 2 * a + side] = 2 * src[a] + old_side
    nbr = structured_neighbors(nelem)
    conn = np.zeros((ne, 6, 3), dtype=np.int32)
    for e in range(ne):
        for f in range(6):
            fo = int(old_face[e, f])
            nb = int(nbr[e, fo])
            fo_nb = fo ^ 1
            fnew_nb = int(np.nonzero(old_face[nb] == fo_nb)[0][0])
            # face-local indices: own new face -> old node -> matching node of nb -> nb's new face index
            d, dn = f >> 1, fnew_nb >> 1
            lo_, ln_ = (N if f & 1 else 0), (N if fnew_nb & 1 else 0)
            target = []
            for a in range(n1 * n1):
                i, j, k = _face_node_ijk(N, d, lo_, a)
                old = perm[e, i + n1 * (j + n1 * k)]
                oi = [old % n1, (old // n1) % n1, old // (n1 * n1)]
                ax = fo >> 1
                oi[ax] = N - oi[ax]  # the matching node of the structured neighbour across that face
                nbnew = new_of_old[nb, oi[0] + n1 * (oi[1] + n1 * oi[2])]
                ii, jj, kk = nbnew % n1, (nbnew // n1) % n1, nbnew // (n1 * n1)
                assert (ii, jj, kk)[dn] == ln_
                target.append(_face_local(N, dn, ii, jj, kk))
            o = [o for o in range(8) if all(_orient(N, o, a) == target[a] for a in range(n1 * n1))]
            assert len(o) >= 1
            conn[e, f] = (nb, fnew_nb, o[0])
    return perm, conn


def relabel(arr, perm) -> np.ndarray:
    """Apply rotated_elements' node relabelling to nodal data (nElems, ..., N+1, N+1, N+1)."""
    ne = arr.shape[0]
    flat = arr.reshape(ne, -1, perm.shape[1])
    out = np.take_along_axis(flat, perm[:, None, :], axis=2)
    return np.ascontiguousarray(out.reshape(arr.shape))


def unlabel(arr, perm) -> np.ndarray:
    """Inverse of relabel."""
    ne = arr.shape[0]
    flat = arr.reshape(ne, -1, perm.shape[1])
    out = np.empty_like(flat)
    np.put_along_axis(out, np.broadcast_to(perm[:, None, :], flat.shape), flat, axis=2)
    return np.ascontiguousarray(out.reshape(arr.shape))
