"""CPU oracle for the staggered-grid stencil step (FP64).

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product path (the
GPU library and its Python binding) never imports, links or runs it.

The arithmetic lives in ``oracle.c`` (plain C loops, built with
``-O2 -ffp-contract=off``); this module builds it with gcc and wraps it with
ctypes over NumPy float64 buffers in the padded index layout
``p[off + i + j*jstride + k*kstride]``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

BC_ZWALL_ZEROGRAD, BC_ZWALL_NOPEN, BC_ZPERIODIC = 0, 1, 2

_lib = None


def build(src: str = SRC, out: str = LIB, openmp: bool = True) -> str:
    """Compile ``oracle.c`` into a shared library (gcc, FP contraction off)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-std=c99", src, "-o", out + ".tmp", "-lm"]
    if openmp:
        cmd.insert(1, "-fopenmp")
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def load(path: str | None = None):
    """Load (building first if absent) the oracle library; returns a ctypes CDLL."""
    global _lib
    if path is None:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        path = LIB
    lib = ctypes.CDLL(path)
    _declare(lib)
    if path == LIB:
        _lib = lib
    return lib


_P = ctypes.POINTER(ctypes.c_double)
_I, _L, _D = ctypes.c_int, ctypes.c_int64, ctypes.c_double


def _declare(lib):
    dims = [_I, _I, _I, _L, _L, _L]
    lib.ora_fill_ghosts.argtypes = dims + [_I, _P, _P, _P]
    lib.ora_advec_u.argtypes = dims + [_D, _D, _P, _P, _P, _P, _P]
    lib.ora_diff_uvw.argtypes = dims + [_D, _D, _P, _P, _D, _I, _P, _P, _P, _P, _P, _P]
    lib.ora_euler.argtypes = dims + [_I, _D, _P, _P, _P, _P, _P, _P]
    lib.ora_step.argtypes = dims + [_I, _D, _D, _P, _P, _D, _D, _L, _P, _P, _P, _P, _P, _P]
    lib.ora_conservation.argtypes = dims + [_I, _P, _P, _P, _P, _P, _P]
    lib.ora_checksums.argtypes = dims + [_P, _P]
    lib.ora_point.argtypes = dims + [_I, _D, _D, _P, _P, _D, _P, _P, _P, _I, _I, _I, _P]
    lib.ora_fill_ghosts_gc.argtypes = dims + [_I, _I, _P, _P, _P]
    lib.ora_fill_scalar.argtypes = dims + [_I, _I, _P]
    lib.ora_advec_u_2i5.argtypes = dims + [_D, _D, _P, _P, _P, _P, _P]
    lib.ora_diff_smag.argtypes = dims + [_D, _D, _P, _P, _I, _P, _P, _P, _P, _P, _P, _P]
    lib.ora_point_les.argtypes = dims + [_I, _D, _D, _P, _P, _P, _P, _P, _P, _I, _I, _I, _P]
    lib.ora_threads.argtypes = []
    lib.ora_threads.restype = ctypes.c_int
    lib.ora_set_threads.argtypes = [_I]
    lib.ora_set_threads.restype = None
    for f in ("ora_fill_ghosts", "ora_advec_u", "ora_diff_uvw", "ora_euler", "ora_step",
              "ora_conservation", "ora_checksums", "ora_point", "ora_fill_ghosts_gc",
              "ora_fill_scalar", "ora_advec_u_2i5", "ora_diff_smag", "ora_point_les"):
        getattr(lib, f).restype = None


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_P)


class Grid:
    """Interior sizes, padded layout and metrics of one grid (host, FP64);
    ``gc`` ghost cells per side in x and y (1, or 3 for advec_u_2i5)."""

    def __init__(self, itot, jtot, ktot, off, js, ks, alloc, dxi, dyi, dzi, dzhi,
                 bc=BC_ZWALL_ZEROGRAD, gc=1):
        self.itot, self.jtot, self.ktot = int(itot), int(jtot), int(ktot)
        self.off, self.js, self.ks, self.alloc = int(off), int(js), int(ks), int(alloc)
        self.dxi, self.dyi = float(dxi), float(dyi)
        self.dzi = np.ascontiguousarray(dzi, dtype=np.float64)
        self.dzhi = np.ascontiguousarray(dzhi, dtype=np.float64)
        self.bc = int(bc)
        self.gc = int(gc)

    @property
    def dims(self):
        return (self.itot, self.jtot, self.ktot, self.off, self.js, self.ks)


def fill_ghosts(g: Grid, u, v, w, lib=None):
    """Ghost cells of u, v, w (gc per side in x and y, one in z)."""
    if g.gc == 1:
        (lib or load()).ora_fill_ghosts(*g.dims, g.bc, _p(u), _p(v), _p(w))
    else:
        (lib or load()).ora_fill_ghosts_gc(*g.dims, g.gc, g.bc, _p(u), _p(v), _p(w))


def fill_scalar(g: Grid, f, lib=None):
    """Ghost cells of a cell-center scalar (the eddy viscosity)."""
    (lib or load()).ora_fill_scalar(*g.dims, g.gc, g.bc, _p(f))


def advec_u_2i5(g: Grid, ut, u, v, w, lib=None):
    """ut += advection of u with fifth-order interpolation (needs gc >= 3)."""
    assert g.gc >= 3, "advec_u_2i5 needs three ghost cells in x and y"
    (lib or load()).ora_advec_u_2i5(*g.dims, g.dxi, g.dyi, _p(g.dzi), _p(ut), _p(u), _p(v), _p(w))


def diff_smag(g: Grid, ut, vt, wt, u, v, w, evisc, lib=None):
    """(ut, vt, wt) += divergence of the viscous stress with eddy viscosity evisc."""
    (lib or load()).ora_diff_smag(*g.dims, g.dxi, g.dyi, _p(g.dzi), _p(g.dzhi), g.bc,
                                  _p(ut), _p(vt), _p(wt), _p(u), _p(v), _p(w), _p(evisc))


def point_les(g: Grid, u, v, w, evisc, i, j, k, lib=None) -> np.ndarray:
    """[advec_u_2i5, diff_smag u, v, w] at one interior point (needs gc >= 3)."""
    assert g.gc >= 3
    out = np.zeros(4)
    (lib or load()).ora_point_les(*g.dims, g.bc, g.dxi, g.dyi, _p(g.dzi), _p(g.dzhi),
                                  _p(u), _p(v), _p(w), _p(evisc), int(i), int(j), int(k), _p(out))
    return out


def advec_u(g: Grid, ut, u, v, w, lib=None):
    """ut += advec_u(u, v, w) on the interior."""
    (lib or load()).ora_advec_u(*g.dims, g.dxi, g.dyi, _p(g.dzi), _p(ut), _p(u), _p(v), _p(w))


def diff_uvw(g: Grid, ut, vt, wt, u, v, w, visc, lib=None):
    """(ut, vt, wt) += visc * Laplacian(u, v, w) on each field's computed range."""
    (lib or load()).ora_diff_uvw(*g.dims, g.dxi, g.dyi, _p(g.dzi), _p(g.dzhi), float(visc), g.bc,
                                 _p(ut), _p(vt), _p(wt), _p(u), _p(v), _p(w))


def euler(g: Grid, dt, u, v, w, ut, vt, wt, lib=None):
    (lib or load()).ora_euler(*g.dims, g.bc, float(dt), _p(u), _p(v), _p(w),
                              _p(ut), _p(vt), _p(wt))


def step(g: Grid, visc, dt, u, v, w, ut, vt, wt, lib=None):
    """One forward-Euler step of advec_u + diff_uvw, in place on u, v, w."""
    (lib or load()).ora_step(*g.dims, g.bc, g.dxi, g.dyi, _p(g.dzi), _p(g.dzhi), float(visc),
                             float(dt), g.alloc, _p(u), _p(v), _p(w), _p(ut), _p(vt), _p(wt))


def conservation(g: Grid, ut, vt, wt, lib=None) -> np.ndarray:
    out = np.zeros(3)
    (lib or load()).ora_conservation(*g.dims, g.bc, _p(g.dzi), _p(g.dzhi),
                                     _p(ut), _p(vt), _p(wt), _p(out))
    return out


def checksums(g: Grid, f, lib=None) -> np.ndarray:
    out = np.zeros(3)
    (lib or load()).ora_checksums(*g.dims, _p(f), _p(out))
    return out


def point(g: Grid, visc, u, v, w, i, j, k, lib=None) -> np.ndarray:
    """[advec_u, diff u, diff v, diff w] tendencies at one interior point."""
    out = np.zeros(4)
    (lib or load()).ora_point(*g.dims, g.bc, g.dxi, g.dyi, _p(g.dzi), _p(g.dzhi), float(visc),
                              _p(u), _p(v), _p(w), int(i), int(j), int(k), _p(out))
    return out
