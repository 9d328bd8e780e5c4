"""Pins of the CPU oracle to facts other than itself.

Each ``pin_*`` function raises AssertionError when the oracle library ``lib``
disagrees with a closed form, an invariant, a library routine or the
brute-force reference.  ``test_oracle_pins.py`` runs them on the real oracle;
``test_oracle_mutants.py`` runs them on copies of the oracle with planted
mistakes and requires that every mistake is caught by at least one pin.

The closed forms (second-order staggered finite differences):
* constant fields: every flux difference vanishes, tendencies are exactly 0;
* linear velocities: midpoint interpolation is exact and a centered
  difference of a quadratic flux is its exact derivative at the interval
  midpoint, so advec_u equals -[d(uu)/dx + d(uv)/dy](xh_i, y_j, z_k)
  - d(uw)/dz(xh_i, y_j, zm_k) with zm_k the midpoint of faces k and k+1;
* quadratics a x^2 + b y^2 + c z^2: the Laplacian 2(a+b+c) is exact for u and
  v on the stretched centers-primary grid, and for w on a uniform grid;
* smooth fields: errors fall as h^2 under refinement;
* fully periodic grid: the volume-weighted sum of a flux divergence is 0.
"""
from __future__ import annotations

import math

import numpy as np

import oracle
from paper_2303_12374_amd import inputs
import ref_tiny

U, V, W = 0, 1, 2


def odd_layout(itot, jtot, ktot):
    """A padded layout with off > 0 and row/plane padding, to exercise strides."""
    off = 3
    js = itot + 2 + 5
    ks = js * (jtot + 2) + 7
    alloc = off + ks * (ktot + 2) + 11
    return off, js, ks, alloc


def make_grid(itot, jtot, ktot, bc, gamma=1.5, layout=None):
    Lz = inputs.domain_height(itot, jtot, ktot)
    zg = inputs.zgrid(ktot, Lz, 0.0 if bc == oracle.BC_ZPERIODIC else gamma)
    off, js, ks, alloc = layout or odd_layout(itot, jtot, ktot)
    g = oracle.Grid(itot, jtot, ktot, off, js, ks, alloc, itot, jtot, zg["dzi"], zg["dzhi"], bc)
    return g, zg


def interior(g, buf):
    return inputs.padded_view(buf, g.itot, g.jtot, g.ktot, g.off, g.js, g.ks)[
        1:g.ktot + 1, 1:g.jtot + 1, 1:g.itot + 1]


def random_state(g, seed, fill_ghosts=True, lib=None):
    fs = inputs.random_fields(seed, g.itot, g.jtot, g.ktot)
    bufs = [inputs.embed(f, g.off, g.js, g.ks, g.alloc) for f in fs]
    if fill_ghosts:
        oracle.fill_ghosts(g, *bufs, lib=lib)
    return bufs


def zeros_like_bufs(g, n=3):
    out = []
    for _ in range(n):
        b = np.full(g.alloc, np.nan)
        interior(g, b)[...] = 0.0
        out.append(b)
    return out


def tendencies(g, u, v, w, visc, lib=None):
    ut, vt, wt = zeros_like_bufs(g)
    ua = np.full(g.alloc, np.nan)
    interior(g, ua)[...] = 0.0
    oracle.advec_u(g, ua, u, v, w, lib=lib)
    oracle.diff_uvw(g, ut, vt, wt, u, v, w, visc, lib=lib)
    return interior(g, ua), interior(g, ut), interior(g, vt), interior(g, wt)


def kw0(g):
    return 1 if g.bc == oracle.BC_ZPERIODIC else 2


# ---------------------------------------------------------------------------

def pin_constant_fields(lib):
    for bc in (0, 1, 2):
        g, _ = make_grid(9, 7, 8, bc)
        bufs = []
        for f, val in enumerate((1.25, -0.75, 0.5)):
            b = np.full(g.alloc, np.nan)
            inputs.padded_view(b, g.itot, g.jtot, g.ktot, g.off, g.js, g.ks)[...] = val
            bufs.append(b)
        if bc == 1:  # w = 0 at walls is the rule; a constant w needs that value
            inputs.padded_view(bufs[2], g.itot, g.jtot, g.ktot, g.off, g.js, g.ks)[...] = 0.0
        oracle.fill_ghosts(g, *bufs, lib=lib)
        adv, du, dv, dw = tendencies(g, *bufs, 1e-5, lib=lib)
        assert np.all(adv == 0.0), f"advec_u of constant fields not zero (bc={bc})"
        for d in (du, dv, dw):
            assert np.all(d == 0.0), f"diff_uvw of constant fields not zero (bc={bc})"


def _linear_fields(g, zg, rng):
    a = rng.uniform(-1, 1, 4)
    b = rng.uniform(-1, 1, 4)
    c = rng.uniform(-1, 1, 4)
    fns = [lambda X, Y, Z, p=p: p[0] + p[1] * X + p[2] * Y + p[3] * Z for p in (a, b, c)]
    bufs = [inputs.analytic_padded(fns[f], f, g.itot, g.jtot, g.ktot, zg, g.off, g.js, g.ks, g.alloc)
            for f in range(3)]
    return a, b, c, bufs


def pin_linear_advection(lib):
    rng = np.random.default_rng(11)
    g, zg = make_grid(6, 5, 7, 0, gamma=1.5)
    a, b, c, bufs = _linear_fields(g, zg, rng)
    adv, du, dv, dw = tendencies(g, *bufs, 1e-2, lib=lib)
    cc = inputs.coords(g.itot, g.jtot, zg)
    kt = g.ktot
    X = cc["xh"][1:g.itot + 1][None, None, :]
    Y = cc["y"][1:g.jtot + 1][None, :, None]
    Z = zg["z"][1:kt + 1][:, None, None]
    Zm = (0.5 * (zg["zh"][1:kt + 1] + zg["zh"][2:kt + 2]))[:, None, None]
    uf = lambda X, Y, Z: a[0] + a[1] * X + a[2] * Y + a[3] * Z
    vf = lambda X, Y, Z: b[0] + b[1] * X + b[2] * Y + b[3] * Z
    wf = lambda X, Y, Z: c[0] + c[1] * X + c[2] * Y + c[3] * Z
    exact = -(2 * uf(X, Y, Z) * a[1] + a[2] * vf(X, Y, Z) + uf(X, Y, Z) * b[2]) \
        - (a[3] * wf(X, Y, Zm) + uf(X, Y, Zm) * c[3])
    scale = np.max(np.abs(exact)) + 1.0
    err = np.max(np.abs(adv - exact))
    assert err <= 1e-12 * scale * max(g.itot, g.jtot, np.max(g.dzi)), f"linear advection err {err}"
    # diffusion of linear fields vanishes up to rounding of the differences
    dscale = 1e-2 * (g.dxi ** 2 + g.dyi ** 2 + np.max(g.dzi) * np.max(g.dzhi)) * 4.0
    for d, rng_k in ((du, slice(None)), (dv, slice(None)), (dw, slice(kw0(g) - 1, None))):
        assert np.max(np.abs(d[rng_k])) <= 1e-13 * dscale, "diffusion of a linear field not ~0"


def pin_quadratic_laplacian(lib):
    visc = 0.37
    a, b, c = 0.7, -1.3, 2.1
    q = lambda X, Y, Z: a * X * X + b * Y * Y + c * Z * Z
    exact = 2.0 * visc * (a + b + c)
    # u and v: exact on the stretched centers-primary grid
    g, zg = make_grid(6, 7, 9, 0, gamma=1.5)
    bufs = [inputs.analytic_padded(q, f, g.itot, g.jtot, g.ktot, zg, g.off, g.js, g.ks, g.alloc)
            for f in range(3)]
    _, du, dv, _ = tendencies(g, *bufs, visc, lib=lib)
    tol = 1e-12 * (g.dxi ** 2 + g.dyi ** 2 + np.max(g.dzi) * np.max(g.dzhi))
    assert np.max(np.abs(du - exact)) <= tol, f"u Laplacian err {np.max(np.abs(du - exact))}"
    assert np.max(np.abs(dv - exact)) <= tol, f"v Laplacian err {np.max(np.abs(dv - exact))}"
    # w on the stretched grid: exact in x and y (c = 0)
    q2 = lambda X, Y, Z: a * X * X + b * Y * Y + 0.0 * Z
    bw = [inputs.analytic_padded(q2, f, g.itot, g.jtot, g.ktot, zg, g.off, g.js, g.ks, g.alloc)
          for f in range(3)]
    _, _, _, dw = tendencies(g, *bw, visc, lib=lib)
    assert np.max(np.abs(dw[1:] - 2 * visc * (a + b))) <= tol, "w Laplacian (x, y) err"
    # w on a uniform grid: exact in all directions
    gu, zgu = make_grid(6, 7, 9, 0, gamma=0.0)
    bu = [inputs.analytic_padded(q, f, gu.itot, gu.jtot, gu.ktot, zgu, gu.off, gu.js, gu.ks, gu.alloc)
          for f in range(3)]
    _, du2, _, dw2 = tendencies(gu, *bu, visc, lib=lib)
    assert np.max(np.abs(dw2[1:] - exact)) <= tol, f"w Laplacian err {np.max(np.abs(dw2[1:] - exact))}"
    assert np.max(np.abs(du2 - exact)) <= tol


def _smooth(g, zg):
    kx = ky = 2 * math.pi
    kz = math.pi / zg["Lz"]
    A, B, C, U0, V0 = 0.8, 0.6, 0.5, 1.0, 0.5
    s, co = np.sin, np.cos
    uf = lambda X, Y, Z: U0 + A * s(kx * X) * co(ky * Y) * co(kz * Z)
    vf = lambda X, Y, Z: V0 + B * co(kx * X) * s(ky * Y) * co(kz * Z)
    wf = lambda X, Y, Z: C * co(kx * X) * co(ky * Y) * s(kz * Z)
    ux = lambda X, Y, Z: A * kx * co(kx * X) * co(ky * Y) * co(kz * Z)
    uy = lambda X, Y, Z: -A * ky * s(kx * X) * s(ky * Y) * co(kz * Z)
    uz = lambda X, Y, Z: -A * kz * s(kx * X) * co(ky * Y) * s(kz * Z)
    vy = lambda X, Y, Z: B * ky * co(kx * X) * co(ky * Y) * co(kz * Z)
    wz = lambda X, Y, Z: C * kz * co(kx * X) * co(ky * Y) * co(kz * Z)
    k2 = kx * kx + ky * ky + kz * kz
    return dict(fns=(uf, vf, wf), ux=ux, uy=uy, uz=uz, vy=vy, wz=wz, k2=k2, U0=U0, V0=V0)


def convergence_errors(lib, sizes=(16, 32, 64, 128), visc=0.05):
    errs = []
    for n in sizes:
        g, zg = make_grid(n, n, n, 0, gamma=1.5, layout=inputs.plain_layout(n, n, n))
        S = _smooth(g, zg)
        bufs = [inputs.analytic_padded(S["fns"][f], f, n, n, n, zg, g.off, g.js, g.ks, g.alloc)
                for f in range(3)]
        adv, du, dv, dw = tendencies(g, *bufs, visc, lib=lib)
        e = []
        for f, d in ((U, adv), (U, du), (V, dv), (W, dw)):
            Z, Y, X = inputs.staggered_positions(f, n, n, zg)
            Z, Y, X = Z[1:n + 1], Y[:, 1:n + 1], X[:, :, 1:n + 1]
            uf, vf, wf = S["fns"]
            if d is adv:
                ex = -(2 * uf(X, Y, Z) * S["ux"](X, Y, Z) + S["uy"](X, Y, Z) * vf(X, Y, Z)
                       + uf(X, Y, Z) * S["vy"](X, Y, Z) + S["uz"](X, Y, Z) * wf(X, Y, Z)
                       + uf(X, Y, Z) * S["wz"](X, Y, Z))
            else:
                base = (S["U0"], S["V0"], 0.0)[f]
                ex = -visc * S["k2"] * (S["fns"][f](X, Y, Z) - base)
            sl = slice(1, None) if f == W else slice(None)
            e.append(np.max(np.abs((d - ex)[sl])))
        errs.append(e)
    return np.array(errs)


def pin_second_order(lib):
    errs = convergence_errors(lib)
    order = np.log2(errs[:-1] / errs[1:])
    assert np.all(order[-1] >= 1.9), f"observed orders {order}"
    assert np.all(order >= 1.7), f"observed orders {order}"


def pin_conservation(lib):
    g, zg = make_grid(12, 10, 8, oracle.BC_ZPERIODIC)
    u, v, w = random_state(g, 5, lib=lib)
    visc = 0.01
    adv, du, dv, dw = tendencies(g, u, v, w, visc, lib=lib)
    dz = 1.0 / g.dzi[1:g.ktot + 1]
    vol = (1.0 / g.dxi) * (1.0 / g.dyi) * dz[:, None, None]
    umax = max(np.max(np.abs(interior(g, f))) for f in (u, v, w))
    n = g.itot * g.jtot * g.ktot
    A = 2 * n * np.max(vol) * umax * umax * (g.dxi + g.dyi + np.max(g.dzi))
    assert abs(np.sum(adv * vol)) <= 1e-14 * A, f"advec_u not conservative: {np.sum(adv * vol)} vs {A}"
    Ad = 4 * n * np.max(vol) * visc * umax * (g.dxi ** 2 + g.dyi ** 2 + np.max(g.dzi) ** 2)
    for d in (du, dv, dw):
        assert abs(np.sum(d * vol)) <= 1e-14 * Ad, f"diffusion not conservative: {np.sum(d * vol)}"
    # the FP64 conservation reduction equals the same weighted sums
    ut = np.zeros(g.alloc)
    interior(g, ut)[...] = adv
    vt = np.zeros(g.alloc)
    interior(g, vt)[...] = dv
    wt = np.zeros(g.alloc)
    interior(g, wt)[...] = dw
    c = oracle.conservation(g, ut, vt, wt, lib=lib)
    for got, d in zip(c, (adv, dv, dw)):
        assert abs(got - np.sum(d * dz[:, None, None])) <= 1e-12 * np.sum(np.abs(d) * dz[:, None, None])


def pin_translation_invariance(lib):
    for bc in (0, 2):
        g, zg = make_grid(11, 9, 6, bc)
        fs = inputs.random_fields(7, g.itot, g.jtot, g.ktot)
        sx, sy = 3, 5
        rolled = [np.roll(np.roll(f, sx, axis=2), sy, axis=1) for f in fs]
        outs = []
        for flds in (fs, rolled):
            bufs = [inputs.embed(f, g.off, g.js, g.ks, g.alloc) for f in flds]
            oracle.fill_ghosts(g, *bufs, lib=lib)
            outs.append(tendencies(g, *bufs, 0.02, lib=lib))
        for a, b in zip(outs[0], outs[1]):
            assert np.array_equal(np.roll(np.roll(a, sx, axis=2), sy, axis=1), b), "not shift-invariant"


def pin_brute_force(lib):
    for bc in (0, 1, 2):
        for (it, jt, kt) in ((5, 4, 6), (3, 2, 2), (1, 3, 4)):
            g, zg = make_grid(it, jt, kt, bc)
            u, v, w = random_state(g, 3 + bc, lib=lib)
            ours = tendencies(g, u, v, w, 0.3, lib=lib)
            fs = inputs.random_fields(3 + bc, it, jt, kt)
            ref = ref_tiny.tendencies(*fs, g.dxi, g.dyi, g.dzi, g.dzhi, 0.3, bc)
            for n, (a, b) in enumerate(zip(ours, ref)):
                scale = np.max(np.abs(b)) + 1e-300
                assert np.max(np.abs(a - b)) <= 1e-13 * scale, \
                    f"oracle vs brute force, output {n}, bc {bc}, {(it, jt, kt)}"
            # w is not advanced on the wall faces: its tendency stays untouched there
            if bc != oracle.BC_ZPERIODIC:
                assert np.all(ours[3][0] == 0.0), "wt written on the bottom wall face"


def pin_ghost_fill(lib):
    """Ghosts equal the field at the periodic image / wall rule of each cell."""
    it, jt, kt = 7, 5, 6
    for bc in (0, 1, 2):
        g, _ = make_grid(it, jt, kt, bc)
        rng = np.random.default_rng(bc)
        tables = [rng.integers(-1000, 1000, size=(kt, jt, it)).astype(np.float64) for _ in range(3)]
        bufs = [inputs.embed(t, g.off, g.js, g.ks, g.alloc) for t in tables]
        oracle.fill_ghosts(g, *bufs, lib=lib)
        F = ref_tiny.Fields(*tables, bc)
        for n in range(3):
            view = inputs.padded_view(bufs[n], it, jt, kt, g.off, g.js, g.ks)
            for k in range(kt + 2):
                for j in range(jt + 2):
                    for i in range(it + 2):
                        assert view[k, j, i] == F.get(n, i, j, k), f"ghost ({n},{i},{j},{k}) bc={bc}"
        # padding outside the (itot+2, jtot+2, ktot+2) box is never written
        mask = np.ones(g.alloc, bool)
        for n in range(3):
            pass
        idx = (g.off + np.arange(it + 2)[None, None, :] + g.js * np.arange(jt + 2)[None, :, None]
               + g.ks * np.arange(kt + 2)[:, None, None]).ravel()
        mask[idx] = False
        for n in range(3):
            assert np.all(np.isnan(bufs[n][mask])), "fill wrote outside the field"


def pin_reductions(lib):
    g, _ = make_grid(8, 6, 5, 0)
    u, v, w = random_state(g, 9, lib=lib)
    for f in (u, v, w):
        c = oracle.checksums(g, f, lib=lib)
        x = interior(g, f)
        assert abs(c[0] - np.sum(x)) <= 1e-12 * np.sum(np.abs(x))
        assert abs(c[1] - np.sum(x * x)) <= 1e-12 * np.sum(x * x)
        assert c[2] == np.max(np.abs(x))
    # conservation weights: dz for u, v and dzh for w on w's computed faces
    ut, vt, wt = [np.zeros(g.alloc) for _ in range(3)]
    interior(g, ut)[...] = 1.0
    interior(g, vt)[...] = 2.0
    interior(g, wt)[...] = 3.0
    c = oracle.conservation(g, ut, vt, wt, lib=lib)
    Lz = g.ktot / max(g.itot, g.jtot)
    zg = inputs.zgrid(g.ktot, Lz, 1.5)
    n2 = g.itot * g.jtot
    assert abs(c[0] - n2 * Lz) <= 1e-12 * n2 * Lz, "sum of dz over the column is Lz"
    assert abs(c[1] - 2 * n2 * Lz) <= 1e-12 * n2 * Lz
    span = zg["z"][g.ktot] - zg["z"][1]  # sum of dzh over faces 2..ktot
    assert abs(c[2] - 3 * n2 * span) <= 1e-12 * n2, "sum of dzh over inner faces"


def pin_step(lib):
    for bc in (0, 2):
        g, zg = make_grid(8, 7, 6, bc)
        u, v, w = random_state(g, 13, lib=lib)
        visc, dt = 0.01, 1e-3
        adv, du, dv, dw = tendencies(g, u, v, w, visc, lib=lib)
        u1, v1, w1 = (b.copy() for b in (u, v, w))
        tmp = [np.zeros(g.alloc) for _ in range(3)]
        oracle.step(g, visc, dt, u1, v1, w1, *tmp, lib=lib)
        scale = np.max(np.abs(adv)) * dt
        assert np.max(np.abs((interior(g, u1) - interior(g, u)) - dt * (adv + du))) <= 1e-13 * (1 + scale)
        assert np.max(np.abs((interior(g, v1) - interior(g, v)) - dt * dv)) <= 1e-13
        k0 = kw0(g) - 1
        assert np.max(np.abs((interior(g, w1) - interior(g, w))[k0:] - dt * dw[k0:])) <= 1e-13
        # ghosts are refilled after the update
        chk = [b.copy() for b in (u1, v1, w1)]
        oracle.fill_ghosts(g, *chk, lib=lib)
        for a, b in zip(chk, (u1, v1, w1)):
            assert np.array_equal(a, b, equal_nan=True), "step leaves ghosts stale"
        # periodic: the domain sums of u and v are conserved by a step
        if bc == 2:
            for new, old in ((u1, u), (v1, v)):
                assert abs(np.sum(interior(g, new)) - np.sum(interior(g, old))) <= 1e-11 * new.size


PINS = [pin_constant_fields, pin_linear_advection, pin_quadratic_laplacian, pin_second_order,
        pin_conservation, pin_translation_invariance, pin_brute_force, pin_ghost_fill,
        pin_reductions, pin_step]
