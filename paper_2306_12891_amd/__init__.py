"""MI355X-native split-form DGSEM hot path (Euler / Navier-Stokes, periodic
Cartesian hexahedra) behind a C-ABI library.

The GPU binding lives in :mod:`paper_2306_12891_amd.dg`; importing this package
does not load the native library.
"""
__all__ = ["dg", "inputs"]
