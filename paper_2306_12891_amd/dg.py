"""ctypes binding of libdgmi.so (include/dg.h) with torch tensors.

Argument marshalling only: every step of the operator runs in the library's
HIP kernels.  PyTorch provides device memory and the stream: each call passes
``tensor.data_ptr()`` and ``torch.cuda.current_stream().cuda_stream``.

States are float64 CUDA(HIP) tensors of shape (nElems, 5, N+1, N+1, N+1),
contiguous, variables (rho, rho u, rho v, rho w, E), x index fastest.
"""
from __future__ import annotations

import ctypes
import math
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdgmi.so")

DG_OK, DG_EINVAL, DG_ENOMEM, DG_EHIP, DG_EUNSUPPORTED, DG_ENONFINITE, DG_ESTATE = 0, -1, -2, -3, -4, -5, -6
EULER, NS = 0, 1
KG, PI, CH, STD = 0, 1, 2, 3
LLF, ROE, CENTRAL = 0, 1, 2
HENNEMANN, PERSSON = 0, 1
FV_FIRST, FV_MINMOD = 0, 1
FP64, MIXED = 0, 1
LIFT_TWO_PASS, LIFT_SPLIT = 0, 1

EXPORTS = ["dg_default_options", "dg_init", "dg_set_options", "dg_get_options", "dg_set_stream",
           "dg_time_derivative", "rk_step", "dg_rk_steps", "dg_vjp", "rk_step_vjp", "dg_max_dt",
           "dg_integrals", "dg_alpha", "dg_check_finite", "dg_set_profiling", "dg_profile_read", "dg_node_weights",
           "dg_sizes", "dg_finalize", "dg_last_error", "dg_set_cs_field", "dg_set_geometry",
           "dg_set_connectivity", "dg_set_wall_model", "rk_step_record", "rk_step_vjp_recorded", "dg_vjp_noalloc"]


class DGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libdgmi error {code}: {msg}")
        self.code = code


class Mesh(ctypes.Structure):
    _fields_ = [("nelem", ctypes.c_int32 * 3), ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3)]


class Options(ctypes.Structure):
    _fields_ = [("equations", ctypes.c_int32), ("vol_flux", ctypes.c_int32), ("surf_flux", ctypes.c_int32),
                ("blending", ctypes.c_int32), ("indicator", ctypes.c_int32), ("fv_recon", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("lifting", ctypes.c_int32), ("Pr", ctypes.c_double),
                ("alpha_min", ctypes.c_double), ("alpha_max", ctypes.c_double), ("alpha_spread", ctypes.c_double),
                ("Cs", ctypes.c_double), ("Prt", ctypes.c_double)]


_lib = None


def lib() -> ctypes.CDLL:
    """Loads libdgmi.so; raises if it has not been built (no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "or python paper_2306_12891_amd/csrc/build.py")
        L = ctypes.CDLL(LIB_PATH)
        P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        sig = {
            "dg_default_options": ([P], None),
            "dg_init": ([P, I, D, D, P], I),
            "dg_set_options": ([P, P], I),
            "dg_get_options": ([P, P], I),
            "dg_set_stream": ([P, P], I),
            "dg_time_derivative": ([P, P, P], I),
            "rk_step": ([P, P, D], I),
            "dg_rk_steps": ([P, P, D, I], I),
            "dg_vjp": ([P, P, P, P], I),
            "dg_vjp_noalloc": ([P, P, P, P], I),
            "rk_step_vjp": ([P, P, D, P, P], I),
            "dg_max_dt": ([P, P, D, P], I),
            "dg_integrals": ([P, P, P], I),
            "dg_alpha": ([P, P, P], I),
            "dg_check_finite": ([P, P], I),
            "dg_set_profiling": ([P, I], I),
            "dg_profile_read": ([P, P, P], I),
            "dg_node_weights": ([P, P], I),
            "dg_sizes": ([P, P, P], I),
            "dg_finalize": ([P], I),
            "dg_last_error": ([P], ctypes.c_char_p),
            "dg_set_cs_field": ([P, P], I),
            "dg_set_geometry": ([P, P], I),
            "dg_set_connectivity": ([P, P], I),
            "dg_set_wall_model": ([P, I, ctypes.c_double, ctypes.c_double], I),
            "rk_step_record": ([P, P, ctypes.c_double, P], I),
            "rk_step_vjp_recorded": ([P, P, ctypes.c_double, P, P], I),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def default_options() -> Options:
    o = Options()
    lib().dg_default_options(ctypes.byref(o))
    return o


class DG:
    """One library context: a periodic Cartesian mesh, degree N, gamma, mu and options."""

    def __init__(self, nelem=(4, 4, 4), N: int = 3, gamma: float = 1.4, mu: float = 0.0,
                 lo=(0.0, 0.0, 0.0), hi=(2 * math.pi,) * 3, **options):
        self._ctx = ctypes.c_void_p()
        m = Mesh()
        for d in range(3):
            m.nelem[d] = int(nelem[d])
            m.lo[d] = float(lo[d])
            m.hi[d] = float(hi[d])
        rc = lib().dg_init(ctypes.byref(m), int(N), float(gamma), float(mu), ctypes.byref(self._ctx))
        if rc != DG_OK:
            raise DGError(rc, lib().dg_last_error(None).decode())
        self.N, self.nelem, self.gamma, self.mu = int(N), tuple(int(x) for x in nelem), float(gamma), float(mu)
        self.lo, self.hi = tuple(lo), tuple(hi)
        self.n_elems = int(nelem[0] * nelem[1] * nelem[2])
        n1 = self.N + 1
        self.shape = (self.n_elems, 5, n1, n1, n1)
        self.options = default_options()
        if options:
            self.set_options(**options)

    # -- plumbing ---------------------------------------------------------
    def _check(self, rc: int):
        if rc != DG_OK:
            raise DGError(rc, lib().dg_last_error(self._ctx).decode())

    def _stream(self):
        self._check(lib().dg_set_stream(self._ctx, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))

    def _state(self, x: torch.Tensor, name: str) -> int:
        if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype != torch.float64:
            raise TypeError(f"{name} must be a float64 GPU tensor")
        if tuple(x.shape) != self.shape or not x.is_contiguous():
            raise ValueError(f"{name} must be contiguous with shape {self.shape}, got {tuple(x.shape)}")
        return x.data_ptr()

    def set_options(self, **kw):
        o = Options()
        ctypes.memmove(ctypes.byref(o), ctypes.byref(self.options), ctypes.sizeof(o))
        for k, v in kw.items():
            if not hasattr(o, k):
                raise KeyError(k)
            setattr(o, k, v)
        self._check(lib().dg_set_options(self._ctx, ctypes.byref(o)))
        self.options = o

    def set_cs_field(self, cs: torch.Tensor | None):
        """Per-element Smagorinsky coefficients (float64 GPU tensor of n_elems
        values, copied), or None for the constant options.Cs."""
        if cs is None:
            self._check(lib().dg_set_cs_field(self._ctx, None))
            return
        if not isinstance(cs, torch.Tensor) or not cs.is_cuda or cs.dtype != torch.float64:
            raise TypeError("cs must be a float64 GPU tensor")
        if cs.numel() != self.n_elems or not cs.is_contiguous():
            raise ValueError(f"cs must be contiguous with {self.n_elems} values")
        self._stream()
        self._check(lib().dg_set_cs_field(self._ctx, ctypes.c_void_p(cs.data_ptr())))

    def set_geometry(self, X: torch.Tensor | None):
        """Curved mesh: node coordinates, float64 GPU tensor of shape
        (n_elems, 3, N+1, N+1, N+1) (x index fastest; read once, the library
        keeps the metric terms), or None for the Cartesian box."""
        if X is None:
            self._check(lib().dg_set_geometry(self._ctx, None))
            return
        n1 = self.N + 1
        if not isinstance(X, torch.Tensor) or not X.is_cuda or X.dtype != torch.float64:
            raise TypeError("X must be a float64 GPU tensor")
        if tuple(X.shape) != (self.n_elems, 3, n1, n1, n1) or not X.is_contiguous():
            raise ValueError(f"X must be contiguous of shape {(self.n_elems, 3, n1, n1, n1)}")
        self._stream()
        self._check(lib().dg_set_geometry(self._ctx, ctypes.c_void_p(X.data_ptr())))

    def set_connectivity(self, conn):
        """General connectivity of a curved mesh: int32 array (n_elems, 6, 3) of
        (neighbour, its local face, orientation) on the host (copied), or None
        for the structured periodic mesh."""
        import numpy as np
        if conn is None:
            self._check(lib().dg_set_connectivity(self._ctx, None))
            return
        c = np.ascontiguousarray(conn, dtype=np.int32)
        if c.shape != (self.n_elems, 6, 3):
            raise ValueError(f"conn must have shape {(self.n_elems, 6, 3)}")
        self._check(lib().dg_set_connectivity(self._ctx, ctypes.c_void_p(c.ctypes.data)))

    def set_wall_model(self, wall_dir: int, u_inf: float = 1.0, ma_inf: float = 0.0):
        """Wall-modelled boundaries on the two box faces normal to wall_dir
        (0, 1, 2; -1: periodic again): Spalding's law of the wall, van Driest
        transformed with freestream velocity u_inf and Mach number ma_inf > 0."""
        self._stream()
        self._check(lib().dg_set_wall_model(self._ctx, int(wall_dir), float(u_inf), float(ma_inf)))

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            lib().dg_finalize(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- operator ---------------------------------------------------------
    def time_derivative(self, U: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        pu = self._state(U, "U")
        if out is None:
            out = torch.empty_like(U)
        po = self._state(out, "Ut")
        self._stream()
        self._check(lib().dg_time_derivative(self._ctx, ctypes.c_void_p(pu), ctypes.c_void_p(po)))
        return out

    def rk_step(self, U: torch.Tensor, dt: float) -> torch.Tensor:
        pu = self._state(U, "U")
        self._stream()
        self._check(lib().rk_step(self._ctx, ctypes.c_void_p(pu), float(dt)))
        return U

    def rk_steps(self, U: torch.Tensor, dt: float, nsteps: int) -> torch.Tensor:
        pu = self._state(U, "U")
        self._stream()
        self._check(lib().dg_rk_steps(self._ctx, ctypes.c_void_p(pu), float(dt), int(nsteps)))
        return U

    def vjp(self, U: torch.Tensor, Ut_bar: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        pu, pb = self._state(U, "U"), self._state(Ut_bar, "Ut_bar")
        if out is None:
            out = torch.empty_like(U)
        po = self._state(out, "U_bar")
        self._stream()
        self._check(lib().dg_vjp(self._ctx, ctypes.c_void_p(pu), ctypes.c_void_p(pb), ctypes.c_void_p(po)))
        return out

    def vjp_noalloc(self, U: torch.Tensor, Ut_bar: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        """dg_vjp_noalloc: the reverse product into the caller's `out`, with
        the library's fixed device scratch (no allocation in the call)."""
        pu, pb, po = self._state(U, "U"), self._state(Ut_bar, "Ut_bar"), self._state(out, "U_bar")
        self._stream()
        self._check(lib().dg_vjp_noalloc(self._ctx, ctypes.c_void_p(pu), ctypes.c_void_p(pb), ctypes.c_void_p(po)))
        return out

    def rk_step_vjp(self, U_n: torch.Tensor, dt: float, U_bar_np1: torch.Tensor,
                    out: torch.Tensor | None = None) -> torch.Tensor:
        pu, pb = self._state(U_n, "U_n"), self._state(U_bar_np1, "U_bar_np1")
        if out is None:
            out = torch.empty_like(U_n)
        po = self._state(out, "U_bar_n")
        self._stream()
        self._check(lib().rk_step_vjp(self._ctx, ctypes.c_void_p(pu), float(dt), ctypes.c_void_p(pb),
                                      ctypes.c_void_p(po)))
        return out

    def _stages(self, Y: torch.Tensor) -> int:
        if not isinstance(Y, torch.Tensor) or not Y.is_cuda or Y.dtype != torch.float64:
            raise TypeError("Y must be a float64 GPU tensor")
        if tuple(Y.shape) != (5,) + self.shape or not Y.is_contiguous():
            raise ValueError(f"Y must be contiguous of shape {(5,) + self.shape}")
        return Y.data_ptr()

    def rk_step_record(self, U: torch.Tensor, dt: float, Y: torch.Tensor) -> torch.Tensor:
        """rk_step in place on U that also writes its five stage states into Y
        (shape (5,) + U.shape)."""
        pu, py = self._state(U, "U"), self._stages(Y)
        self._stream()
        self._check(lib().rk_step_record(self._ctx, ctypes.c_void_p(pu), float(dt), ctypes.c_void_p(py)))
        return U

    def rk_step_vjp_recorded(self, Y: torch.Tensor, dt: float, U_bar_np1: torch.Tensor,
                             out: torch.Tensor | None = None) -> torch.Tensor:
        """rk_step_vjp from the stage states recorded by rk_step_record."""
        py, pb = self._stages(Y), self._state(U_bar_np1, "U_bar_np1")
        if out is None:
            out = torch.empty_like(U_bar_np1)
        po = self._state(out, "U_bar_n")
        self._stream()
        self._check(lib().rk_step_vjp_recorded(self._ctx, ctypes.c_void_p(py), float(dt), ctypes.c_void_p(pb),
                                               ctypes.c_void_p(po)))
        return out

    # -- diagnostics ------------------------------------------------------
    def max_dt(self, U: torch.Tensor, cfl: float = 0.5) -> float:
        pu = self._state(U, "U")
        self._stream()
        dt = ctypes.c_double()
        self._check(lib().dg_max_dt(self._ctx, ctypes.c_void_p(pu), float(cfl), ctypes.byref(dt)))
        return dt.value

    def integrals(self, X: torch.Tensor):
        px = self._state(X, "X")
        self._stream()
        out = (ctypes.c_double * 5)()
        self._check(lib().dg_integrals(self._ctx, ctypes.c_void_p(px), out))
        return [out[v] for v in range(5)]

    def alpha(self, U: torch.Tensor) -> torch.Tensor:
        pu = self._state(U, "U")
        a = torch.empty(self.n_elems, dtype=torch.float64, device=U.device)
        self._stream()
        self._check(lib().dg_alpha(self._ctx, ctypes.c_void_p(pu), ctypes.c_void_p(a.data_ptr())))
        return a

    def check_finite(self, X: torch.Tensor) -> bool:
        px = self._state(X, "X")
        self._stream()
        rc = lib().dg_check_finite(self._ctx, ctypes.c_void_p(px))
        if rc == DG_ENONFINITE:
            return False
        self._check(rc)
        return True

    def set_profiling(self, on: bool):
        self._check(lib().dg_set_profiling(self._ctx, 1 if on else 0))

    def profile_read(self):
        """{kind: (total ms, launches)} for 'stage', 'lift', 'indicator', 'vjp', 'vjp_lift'."""
        ms = (ctypes.c_double * 5)()
        n = (ctypes.c_int64 * 5)()
        self._check(lib().dg_profile_read(self._ctx, ms, n))
        return {k: (ms[i], n[i]) for i, k in enumerate(("stage", "lift", "indicator", "vjp", "vjp_lift"))}

    def node_weights(self, device=None) -> torch.Tensor:
        """w_i w_j w_k J per node of an element, shape (N+1, N+1, N+1)."""
        n1 = self.N + 1
        w = (ctypes.c_double * (n1 ** 3))()
        self._check(lib().dg_node_weights(self._ctx, w))
        out = torch.tensor(list(w), dtype=torch.float64).reshape(n1, n1, n1)
        return out.to(device) if device is not None else out

    def last_error(self) -> str:
        return lib().dg_last_error(self._ctx).decode()

    def raw_call(self, name: str, *args) -> int:
        """Calls a C entry point with this context as first argument (error-path tests)."""
        return getattr(lib(), name)(self._ctx, *args)


# ---------------------------------------------------------------------------
# autograd: the operator and the Runge-Kutta step as differentiable functions
# whose backward passes call the library's reverse-mode kernels.
# ---------------------------------------------------------------------------
class DGOperator(torch.autograd.Function):
    """U_t = L(U); backward: U_bar = dg_vjp(U, U_t_bar)."""

    @staticmethod
    def forward(ctx, U, op):
        ctx.op = op
        ctx.save_for_backward(U)
        return op.time_derivative(U.detach().contiguous())

    @staticmethod
    def backward(ctx, g):
        (U,) = ctx.saved_tensors
        return ctx.op.vjp(U.detach().contiguous(), g.contiguous()), None


class RKStep(torch.autograd.Function):
    """One LSERK4 step (out of place); backward: rk_step_vjp."""

    @staticmethod
    def forward(ctx, U, op, dt):
        ctx.op, ctx.dt = op, float(dt)
        ctx.save_for_backward(U)
        V = U.detach().clone()
        op.rk_step(V, dt)
        return V

    @staticmethod
    def backward(ctx, g):
        (U,) = ctx.saved_tensors
        return ctx.op.rk_step_vjp(U.detach().contiguous(), ctx.dt, g.contiguous()), None, None


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, op, dt, nsteps, every):
        ctx.op, ctx.dt, ctx.nsteps, ctx.every = op, float(dt), int(nsteps), int(every)
        U = U0.detach().clone()
        ckpt = {0: U.clone()}
        s = 0
        while s < nsteps:  # one library call per segment (the same steps as rk_step, bitwise)
            k = min(every, nsteps - s)
            op.rk_steps(U, dt, k)
            s += k
            if s < nsteps:
                ckpt[s] = U.clone()
        ctx.ckpt = ckpt
        return U

    @staticmethod
    def backward(ctx, g):
        op, dt, every = ctx.op, ctx.dt, ctx.every
        Ub = g.contiguous().clone()
        Y = None
        for s0 in sorted(ctx.ckpt, reverse=True):
            s1 = min(s0 + every, ctx.nsteps)
            # recompute the segment once, keeping every step's stage states
            if Y is None or Y.shape[0] < s1 - s0:
                Y = torch.empty((s1 - s0, 5) + tuple(Ub.shape), dtype=Ub.dtype, device=Ub.device)
            U = ctx.ckpt[s0].clone()
            for k in range(s1 - s0):
                op.rk_step_record(U, dt, Y[k])
            for k in reversed(range(s1 - s0)):
                op.rk_step_vjp_recorded(Y[k], dt, Ub, out=Ub)
        ctx.ckpt = None
        return Ub, None, None, None, None


def rollout(op: DG, U0: torch.Tensor, dt: float, nsteps: int, checkpoint_every: int = 20) -> torch.Tensor:
    """nsteps LSERK4 steps from U0, differentiable with respect to U0: the
    forward keeps the state every checkpoint_every steps and the backward
    recomputes each segment from its checkpoint once, keeping the five stage
    states of every step, before running the reverse steps on them (memory:
    checkpoints + 5 x checkpoint_every states)."""
    return _Rollout.apply(U0, op, dt, nsteps, checkpoint_every)
