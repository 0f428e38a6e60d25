"""ctypes binding of the plain FP64 CPU oracle (oracle/dg_oracle.cpp).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
CPU-baseline leg of bench.py.  The product library never imports it, and it
imports nothing from the product.

State arrays are numpy float64, C-contiguous, shape (nElems, 5, N+1, N+1, N+1)
with the x index fastest; elements are ordered e = ex + nx*(ey + ny*ez).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dg_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

EULER, NS = 0, 1
KG, PI, CH, STD = 0, 1, 2, 3
LLF, ROE, CENTRAL = 0, 1, 2
HENNEMANN, PERSSON = 0, 1
FV_FIRST, FV_MINMOD = 0, 1


def build(verbose: bool = False) -> str:
    """Compile the oracle with g++ (FP64, no FMA contraction, OpenMP)."""
    cmd = ["g++", "-O3", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-shared", "-fPIC", "-o", LIB + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def sanitize_check(timeout: float = 300.0):
    """Builds oracle/sanitize_check.cpp (the oracle source with a driver that
    calls every entry point on small cases) with g++'s address and
    undefined-behaviour sanitizers and runs it; returns (exit status, output)."""
    exe = os.path.join(HERE, "_sanitize_check")
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-o", exe, os.path.join(HERE, "sanitize_check.cpp")]
    subprocess.check_call(cmd)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", OMP_NUM_THREADS="2")
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, env=env, timeout=timeout)
    return r.returncode, r.stdout


class _Setup(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("equations", ctypes.c_int32), ("vol_flux", ctypes.c_int32), ("surf_flux", ctypes.c_int32),
                ("blending", ctypes.c_int32), ("indicator", ctypes.c_int32), ("fv_recon", ctypes.c_int32),
                ("pad0", ctypes.c_int32), ("pad1", ctypes.c_int32),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("gamma", ctypes.c_double), ("mu", ctypes.c_double), ("Pr", ctypes.c_double),
                ("alpha_min", ctypes.c_double), ("alpha_max", ctypes.c_double),
                ("alpha_spread", ctypes.c_double), ("Cs", ctypes.c_double), ("Prt", ctypes.c_double),
                ("cs_elem", ctypes.c_void_p), ("xnodes", ctypes.c_void_p), ("conn", ctypes.c_void_p),
                ("wall_dir", ctypes.c_int32), ("pad2", ctypes.c_int32), ("wm_uinf", ctypes.c_double),
                ("wm_mainf", ctypes.c_double)]


@dataclass
class Setup:
    N: int
    nelem: tuple = (1, 1, 1)
    lo: tuple = (0.0, 0.0, 0.0)
    hi: tuple = (2 * np.pi, 2 * np.pi, 2 * np.pi)
    gamma: float = 1.4
    mu: float = 0.0
    Pr: float = 0.72
    equations: int = EULER
    vol_flux: int = KG
    surf_flux: int = LLF
    blending: int = 0
    indicator: int = HENNEMANN
    fv_recon: int = FV_MINMOD
    alpha_min: float = 0.01
    alpha_max: float = 0.7
    alpha_spread: float = 0.5
    Cs: float = 0.0          # Smagorinsky coefficient (0: no eddy viscosity)
    Prt: float = 0.9         # turbulent Prandtl number
    cs_elem: object = None   # optional per-element coefficients (numpy, n_elems)
    xnodes: object = None    # curved mesh: node coordinates (n_elems, 3, N+1, N+1, N+1), x index fastest
    conn: object = None      # curved mesh, general connectivity: int32 (n_elems, 6, 3) (neighbour, face, orientation)
    wall_dir: int = -1       # wall-modelled boundaries normal to this direction (-1: periodic)
    wm_uinf: float = 1.0     # van Driest freestream velocity
    wm_mainf: float = 0.0    # van Driest freestream Mach number (0: untransformed Spalding)
    _c: object = field(default=None, repr=False, compare=False)
    _keep: object = field(default=None, repr=False, compare=False)
    _keepx: object = field(default=None, repr=False, compare=False)
    _keepc: object = field(default=None, repr=False, compare=False)

    @property
    def n1(self) -> int:
        return self.N + 1

    @property
    def n_elems(self) -> int:
        return int(np.prod(self.nelem))

    @property
    def shape(self) -> tuple:
        n1 = self.N + 1
        return (self.n_elems, 5, n1, n1, n1)

    def c(self) -> _Setup:
        s = _Setup()
        s.N = self.N
        s.nx, s.ny, s.nz = self.nelem
        s.equations, s.vol_flux, s.surf_flux = self.equations, self.vol_flux, self.surf_flux
        s.blending, s.indicator, s.fv_recon = self.blending, self.indicator, self.fv_recon
        for d in range(3):
            s.lo[d] = self.lo[d]
            s.hi[d] = self.hi[d]
        s.gamma, s.mu, s.Pr = self.gamma, self.mu, self.Pr
        s.alpha_min, s.alpha_max, s.alpha_spread = self.alpha_min, self.alpha_max, self.alpha_spread
        s.Cs, s.Prt = self.Cs, self.Prt
        s.wall_dir, s.wm_uinf, s.wm_mainf = self.wall_dir, self.wm_uinf, self.wm_mainf
        if self.cs_elem is not None:
            self._keep = np.ascontiguousarray(self.cs_elem, dtype=np.float64)
            assert self._keep.shape == (self.n_elems,)
            s.cs_elem = self._keep.ctypes.data
        else:
            s.cs_elem = None
        if self.xnodes is not None:
            self._keepx = np.ascontiguousarray(self.xnodes, dtype=np.float64)
            n1 = self.N + 1
            assert self._keepx.shape == (self.n_elems, 3, n1, n1, n1), self._keepx.shape
            s.xnodes = self._keepx.ctypes.data
        else:
            s.xnodes = None
        if self.conn is not None:
            self._keepc = np.ascontiguousarray(self.conn, dtype=np.int32)
            assert self._keepc.shape == (self.n_elems, 6, 3), self._keepc.shape
            s.conn = self._keepc.ctypes.data
        else:
            s.conn = None
        return s


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        for name, args, res in [
            ("or_set_threads", [ctypes.c_int], ctypes.c_int),
            ("or_basis", [ctypes.c_int, P, P, P, P, P, P], ctypes.c_int),
            ("or_neighbors", [P, P], ctypes.c_int),
            ("or_two_point_flux", [P, ctypes.c_int, P, P, P], ctypes.c_int),
            ("or_surface_flux", [P, ctypes.c_int, P, P, P], ctypes.c_int),
            ("or_physical_flux", [P, ctypes.c_int, P, P], ctypes.c_int),
            ("or_time_derivative", [P, P, P, P, P, P, P], ctypes.c_int),
            ("or_dense_time_derivative", [P, P, P], ctypes.c_int),
            ("or_time_derivative_elems", [P, P, P, ctypes.c_int, P], ctypes.c_int),
            ("or_alpha", [P, P, P, P, P], ctypes.c_int),
            ("or_threshold", [ctypes.c_int], ctypes.c_double),
            ("or_gradient", [P, P, P], ctypes.c_int),
            ("or_rk_steps", [P, P, ctypes.c_double, ctypes.c_int], ctypes.c_int),
            ("or_lserk4_linear", [ctypes.c_int, P, P, ctypes.c_double, ctypes.c_int], ctypes.c_int),
            ("or_jvp", [P, P, P, P, P], ctypes.c_int),
            ("or_rk_jvp", [P, P, P, ctypes.c_double, ctypes.c_int], ctypes.c_int),
            ("or_integrals", [P, P, P], ctypes.c_int),
            ("or_max_dt", [P, P, ctypes.c_double], ctypes.c_double),
            ("or_rk_coefficients", [P, P], None),
            ("or_metrics", [P, P, P], ctypes.c_int),
            ("or_surface_flux_n", [P, P, P, P, P], ctypes.c_int),
            ("or_wall_friction_velocity", [P, ctypes.c_double, ctypes.c_double, ctypes.c_double], ctypes.c_double),
            ("or_spalding", [ctypes.c_double], ctypes.c_double),
        ]:
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ref(s: Setup):
    cs = s.c()
    s._c = cs  # keep alive
    return ctypes.byref(cs)


def _check(rc):
    if rc != 0:
        raise ValueError("oracle rejected the setup")


def set_threads(n: int) -> int:
    return lib().or_set_threads(int(n))


def basis(N: int):
    n1 = N + 1
    xi, w, edge = np.zeros(n1), np.zeros(n1), np.zeros(n1 + 1)
    D, Dhat, Vinv = np.zeros((n1, n1)), np.zeros((n1, n1)), np.zeros((n1, n1))
    _check(lib().or_basis(N, _p(xi), _p(w), _p(D), _p(Dhat), _p(Vinv), _p(edge)))
    return dict(xi=xi, w=w, D=D, Dhat=Dhat, Vinv=Vinv, edge=edge)


def neighbors(s: Setup) -> np.ndarray:
    out = np.zeros((s.n_elems, 6), dtype=np.int32)
    _check(lib().or_neighbors(_ref(s), _p(out)))
    return out


def two_point_flux(s: Setup, d: int, a, b):
    f = np.zeros(5)
    lib().or_two_point_flux(_ref(s), d, _p(_f64(a)), _p(_f64(b)), _p(f))
    return f


def surface_flux(s: Setup, d: int, L, R):
    f = np.zeros(5)
    lib().or_surface_flux(_ref(s), d, _p(_f64(L)), _p(_f64(R)), _p(f))
    return f


def physical_flux(s: Setup, d: int, U):
    f = np.zeros(5)
    lib().or_physical_flux(_ref(s), d, _p(_f64(U)), _p(f))
    return f


def time_derivative(s: Setup, U, alpha=None, parts: bool = False):
    """U_t of the full operator.  parts=True also returns (Ut_dg_adv, Ut_fv, alpha)."""
    U = _f64(U)
    assert U.shape == s.shape, (U.shape, s.shape)
    Ut = np.zeros_like(U)
    a_in = None if alpha is None else _f64(alpha)
    if parts:
        Udg, Ufv, al = np.zeros_like(U), np.zeros_like(U), np.zeros(s.n_elems)
    else:
        Udg = Ufv = al = None
    _check(lib().or_time_derivative(_ref(s), _p(U), _p(Ut), _p(a_in), _p(Udg), _p(Ufv), _p(al)))
    return (Ut, Udg, Ufv, al) if parts else Ut


def time_derivative_elems(s: Setup, U, elems):
    """U_t of the listed elements only (no blending): shape (len(elems), 5, n1, n1, n1)."""
    U = _f64(U)
    el = np.ascontiguousarray(elems, dtype=np.int32)
    n1 = s.N + 1
    out = np.zeros((len(el), 5, n1, n1, n1))
    _check(lib().or_time_derivative_elems(_ref(s), _p(U), _p(el), len(el), _p(out)))
    return out


def dense_time_derivative(s: Setup, U):
    U = _f64(U)
    Ut = np.zeros_like(U)
    _check(lib().or_dense_time_derivative(_ref(s), _p(U), _p(Ut)))
    return Ut


def alpha(s: Setup, U):
    """(E, a1 before spreading, final alpha) per element."""
    U = _f64(U)
    E, a1, al = np.zeros(s.n_elems), np.zeros(s.n_elems), np.zeros(s.n_elems)
    _check(lib().or_alpha(_ref(s), _p(U), _p(E), _p(a1), _p(al)))
    return E, a1, al


def threshold(N: int) -> float:
    return lib().or_threshold(N)


def gradient(s: Setup, U):
    U = _f64(U)
    n1 = s.N + 1
    g = np.zeros((s.n_elems, 3, 4, n1, n1, n1))
    _check(lib().or_gradient(_ref(s), _p(U), _p(g)))
    return g


def rk_steps(s: Setup, U, dt: float, nsteps: int):
    U = _f64(U).copy()
    _check(lib().or_rk_steps(_ref(s), _p(U), float(dt), int(nsteps)))
    return U


def lserk4_linear(A, u, dt: float, nsteps: int):
    A = _f64(A)
    u = _f64(u).copy()
    lib().or_lserk4_linear(len(u), _p(A), _p(u), float(dt), int(nsteps))
    return u


def jvp(s: Setup, U, V):
    U, V = _f64(U), _f64(V)
    Ut, JV = np.zeros_like(U), np.zeros_like(U)
    _check(lib().or_jvp(_ref(s), _p(U), _p(V), _p(Ut), _p(JV)))
    return Ut, JV


def rk_jvp(s: Setup, U, V, dt: float, nsteps: int):
    U, V = _f64(U).copy(), _f64(V).copy()
    _check(lib().or_rk_jvp(_ref(s), _p(U), _p(V), float(dt), int(nsteps)))
    return U, V


def integrals(s: Setup, X):
    X = _f64(X)
    out = np.zeros(5)
    _check(lib().or_integrals(_ref(s), _p(X), _p(out)))
    return out


def max_dt(s: Setup, U, cfl: float = 0.5) -> float:
    dt = lib().or_max_dt(_ref(s), _p(_f64(U)), float(cfl))
    if dt == -2.0:
        raise ValueError("state with a non-finite node or rho <= 0 or p <= 0: no time step")
    if dt < 0:
        raise ValueError("oracle rejected the setup")
    return dt


def rk_coefficients():
    A, B = np.zeros(5), np.zeros(5)
    lib().or_rk_coefficients(_p(A), _p(B))
    return A, B


def metrics(s: Setup):
    """Curved mesh: metric terms Ja (n_elems, 3 [i], 3 [m], n1, n1, n1) and J (n_elems, n1, n1, n1)."""
    n1 = s.N + 1
    Ja = np.zeros((s.n_elems, 3, 3, n1, n1, n1))
    J = np.zeros((s.n_elems, n1, n1, n1))
    _check(lib().or_metrics(_ref(s), _p(Ja), _p(J)))
    return Ja, J


def surface_flux_n(s: Setup, nv, L, R):
    """Surface flux along the unit normal nv."""
    f = np.zeros(5)
    lib().or_surface_flux_n(_ref(s), _p(_f64(nv)), _p(_f64(L)), _p(_f64(R)), _p(f))
    return f


def wall_friction_velocity(s: Setup, u: float, nu: float, h: float) -> float:
    """Friction velocity of the wall model (Spalding, van Driest per the setup)."""
    return lib().or_wall_friction_velocity(_ref(s), float(u), float(nu), float(h))


def spalding(up: float) -> float:
    """y+ of Spalding's law at u+."""
    return lib().or_spalding(float(up))
