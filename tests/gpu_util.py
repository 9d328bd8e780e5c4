"""Shared set-up of GPU parity tests: the same seeded inputs go to the HIP
path (through the C ABI) and to the CPU oracle.  No oracle input or expected
value comes from the GPU."""
from __future__ import annotations

import math

import numpy as np

import oracle
from paper_2303_12374_amd import inputs

VISC = 1e-5
TOL = {0: 1e-5, 1: 1e-12}  # normwise relative, by dtype (F32, F64)


def kl_mod():
    from paper_2303_12374_amd import kl
    return kl


class Case:
    """Device state + oracle state of one grid."""

    def __init__(self, itot, jtot, ktot, dtype, bc=0, seed=0, layout=None, recipe="random",
                 gamma=1.5, visc=VISC):
        kl = kl_mod()
        self.kl = kl
        self.g = kl.Grid(itot, jtot, ktot, dtype=dtype, bc=bc, gamma=gamma, layout=layout)
        g = self.g
        self.visc = visc
        if recipe == "random":
            fs = inputs.random_fields(seed, itot, jtot, ktot)
        else:
            fs = inputs.sinusoid_fields(seed, itot, jtot, ktot, g.zg)
        npd = kl.NP_DTYPE[dtype]
        self.fs = [np.ascontiguousarray(f.astype(npd)) for f in fs]  # what the GPU sees
        self.dev = [g.upload(f) for f in self.fs]
        kl.kl_fill_ghosts(g, *self.dev)
        # oracle: the same rounded values and metrics, in FP64
        self.og = oracle.Grid(itot, jtot, ktot, g.off, g.js, g.ks, g.alloc, g.dxi, g.dyi,
                              g.dzi_h.astype(np.float64), g.dzhi_h.astype(np.float64), bc)
        self.host = [inputs.embed(f.astype(np.float64), g.off, g.js, g.ks, g.alloc) for f in self.fs]
        oracle.fill_ghosts(self.og, *self.host)
        self.visc_eff = float(npd(visc))

    def oracle_tendencies(self):
        og = self.og
        outs = []
        for _ in range(4):
            b = np.full(og.alloc, np.nan)
            inputs.padded_view(b, og.itot, og.jtot, og.ktot, og.off, og.js, og.ks)[
                1:og.ktot + 1, 1:og.jtot + 1, 1:og.itot + 1] = 0.0
            outs.append(b)
        adv, ut, vt, wt = outs
        oracle.advec_u(og, adv, *self.host)
        oracle.diff_uvw(og, ut, vt, wt, *self.host, self.visc_eff)
        return [self.interior_np(b) for b in outs]

    def interior_np(self, buf):
        og = self.og
        return inputs.padded_view(buf, og.itot, og.jtot, og.ktot, og.off, og.js, og.ks)[
            1:og.ktot + 1, 1:og.jtot + 1, 1:og.itot + 1]

    def gpu_interior(self, t):
        return self.g.interior(t).cpu().numpy().astype(np.float64)


def rel_err(got, ref):
    """Normwise relative error max|got - ref| / max|ref| (0 if both are 0)."""
    num = float(np.max(np.abs(got - ref))) if got.size else 0.0
    den = float(np.max(np.abs(ref))) if ref.size else 0.0
    if den == 0.0:
        return num
    return num / den


def accumulate_bound(r, expect, dtype):
    """Bound on max|got - expect| for a kernel that adds its tendency t to a
    value x0 already in the output (got = fl(x0 + t), one rounding), where
    expect = x0 + r with r the oracle's tendency.  The tendency itself meets
    the kernel tolerance, |t - r| <= TOL * max|r|; the addition rounds once,
    at most half an ulp of |x0 + t| <= max|expect| + TOL * max|r|.  The bound
    takes a whole ulp (eps) for that rounding."""
    eps = float(np.finfo(np.float32 if dtype == 0 else np.float64).eps)
    rmax = float(np.max(np.abs(r))) if r.size else 0.0
    emax = float(np.max(np.abs(expect))) if expect.size else 0.0
    return TOL[dtype] * rmax + eps * (emax + TOL[dtype] * rmax)


def outside_interior_mask(g):
    """Boolean mask (flat, alloc) of cells outside the interior box."""
    m = np.ones(g.alloc, bool)
    k = np.arange(1, g.ktot + 1)[:, None, None]
    j = np.arange(1, g.jtot + 1)[None, :, None]
    i = np.arange(1, g.itot + 1)[None, None, :]
    m[(g.off + i + j * g.js + k * g.ks).ravel()] = False
    return m


def nan_equal(a, b):
    return np.array_equal(a, b, equal_nan=True)


def is_finite(x):
    return bool(np.all(np.isfinite(x)))


__all__ = ["Case", "rel_err", "accumulate_bound", "outside_interior_mask", "TOL", "VISC", "math"]
