"""CPU checks of the C ABI: the library loads, and it exports every function
that include/dg.h declares (no compute call is made without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(", text, re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("dg_init", "dg_time_derivative", "rk_step", "dg_vjp", "rk_step_vjp", "dg_finalize"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2306_12891_amd import dg
    if not os.path.exists(dg.LIB_PATH):
        pytest.skip("libdgmi.so not built")
    L = ctypes.CDLL(dg.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name
    assert set(declared_functions()) == set(dg.EXPORTS)


def test_options_struct_layout():
    from paper_2306_12891_amd import dg
    assert ctypes.sizeof(dg.Options) == 8 * 4 + 6 * 8
    assert ctypes.sizeof(dg.Mesh) == 3 * 4 + 4 + 6 * 8  # 4 bytes of padding before lo


def test_default_options_and_init_rejects_bad_arguments():
    """dg_default_options and the argument checks of dg_init run on the host
    before any device call."""
    from paper_2306_12891_amd import dg
    if not os.path.exists(dg.LIB_PATH):
        pytest.skip("libdgmi.so not built")
    o = dg.default_options()
    assert (o.equations, o.vol_flux, o.surf_flux, o.blending) == (0, 0, 0, 0)
    assert (o.alpha_min, o.alpha_max, o.alpha_spread, o.Pr) == (0.01, 0.7, 0.5, 0.72)
    assert (o.Cs, o.Prt) == (0.0, 0.9)
    L = dg.lib()
    m = dg.Mesh()
    for d in range(3):
        m.nelem[d], m.lo[d], m.hi[d] = 2, 0.0, 1.0
    ctx = ctypes.c_void_p()
    assert L.dg_init(ctypes.byref(m), 0, 1.4, 0.0, ctypes.byref(ctx)) == dg.DG_EINVAL
    assert L.dg_init(ctypes.byref(m), 8, 1.4, 0.0, ctypes.byref(ctx)) == dg.DG_EINVAL
    assert L.dg_init(ctypes.byref(m), 3, 1.0, 0.0, ctypes.byref(ctx)) == dg.DG_EINVAL
    assert L.dg_init(ctypes.byref(m), 3, 1.4, -1.0, ctypes.byref(ctx)) == dg.DG_EINVAL
    m.nelem[1] = 0
    assert L.dg_init(ctypes.byref(m), 3, 1.4, 0.0, ctypes.byref(ctx)) == dg.DG_EINVAL
    assert b"nelem" in L.dg_last_error(None)
    assert not ctx.value
    assert L.dg_finalize(None) == dg.DG_OK
