"""Pins of the oracle's fifth-order advection (advec_u_2i5), its
Smagorinsky-type diffusion (diff_smag) and its ghost fill with three ghost
cells, to facts other than the oracle itself.

Closed forms used:
* constant fields with dyadic values: every face value, flux and flux
  difference is exact, so the advection tendency is exactly 0; constant
  velocities give exactly 0 diffusion for any viscosity field;
* flux-form face values: the sixth-order centered part of the fifth-order
  face value is, for a polynomial p of degree <= 5, the value at the face of
  Phi = p - (h^2/24) p_xx + (7 h^4/5760) p_xxxx (the function whose centered
  difference quotient is exactly p_x), and its dissipation term is the fifth
  difference / 60, which vanishes for degree <= 4 and equals 2 c5 h^5 for
  c5 x^5; the fourth-order centered part of the third-order value is
  p - (h^2/24) p_xx at the face for degree <= 3, and its dissipation term
  adds sign(U) (third difference) / 12 = sign(U) c3 h^3 / 2 for c3 x^3;
* the textbook upwind-biased weights (2, -13, 47, 27, -3)/60 and
  (-1, 5, 2)/6 for positive velocity and their mirror images for negative;
* with a constant viscosity nu the stress divergence equals nu times the
  Laplacian plus nu times the gradient of the discrete divergence;
* a viscosity linear in one coordinate and velocities quadratic in one
  coordinate make every discrete derivative and edge mean exact;
* flux form on a fully periodic grid conserves the volume integral;
* the problem is symmetric under exchanging x and y (u and v).
"""
from __future__ import annotations

import numpy as np

import oracle
import ref_tiny
from paper_2303_12374_amd import inputs

U, V, W, E = 0, 1, 2, 3


def odd_layout_gc(itot, jtot, ktot, gc):
    """A padded layout with gc ghost cells in x and y, slack before the
    first ghost and row / plane padding, to exercise strides."""
    js = itot + 2 * gc + 5
    ks = js * (jtot + 2 * gc) + 7
    off = (gc - 1) * (js + 1) + 3
    alloc = off + ks * (ktot + 2) + 11
    return off, js, ks, alloc


def make_grid(itot, jtot, ktot, bc, gc=3, gamma=1.5, layout=None):
    Lz = inputs.domain_height(itot, jtot, ktot)
    zg = inputs.zgrid(ktot, Lz, 0.0 if bc == oracle.BC_ZPERIODIC else gamma)
    off, js, ks, alloc = layout or odd_layout_gc(itot, jtot, ktot, gc)
    g = oracle.Grid(itot, jtot, ktot, off, js, ks, alloc, itot, jtot, zg["dzi"], zg["dzhi"], bc, gc)
    return g, zg


def interior(g, buf):
    return inputs.interior_view(buf, g.itot, g.jtot, g.ktot, g.off, g.js, g.ks, g.gc)


def full(g, buf):
    return inputs.padded_view(buf, g.itot, g.jtot, g.ktot, g.off, g.js, g.ks, g.gc)


def embed(g, arr):
    return inputs.embed(arr, g.off, g.js, g.ks, g.alloc, gh=g.gc)


def analytic(g, zg, fn, field):
    return inputs.analytic_padded(fn, field, g.itot, g.jtot, g.ktot, zg, g.off, g.js, g.ks, g.alloc, g.gc)


def random_state(g, seed, lib=None, evisc_mean=1e-2):
    fs = inputs.random_fields(seed, g.itot, g.jtot, g.ktot)
    bufs = [embed(g, f) for f in fs]
    oracle.fill_ghosts(g, *bufs, lib=lib)
    e = embed(g, inputs.evisc_field(seed, g.itot, g.jtot, g.ktot, mean=evisc_mean))
    oracle.fill_scalar(g, e, lib=lib)
    return bufs, e


def zero_tendency(g):
    b = np.full(g.alloc, np.nan)
    interior(g, b)[...] = 0.0
    return b


def advec(g, u, v, w, lib=None):
    ut = zero_tendency(g)
    oracle.advec_u_2i5(g, ut, u, v, w, lib=lib)
    return interior(g, ut).copy()


def smag(g, u, v, w, e, lib=None):
    t = [zero_tendency(g) for _ in range(3)]
    oracle.diff_smag(g, *t, u, v, w, e, lib=lib)
    return [interior(g, x).copy() for x in t]


def kw0(g):
    return 1 if g.bc == oracle.BC_ZPERIODIC else 2


def const_buf(g, val):
    b = np.full(g.alloc, np.nan)
    full(g, b)[...] = val
    return b


# ---------------------------------------------------------------------------
# ghost fill with three ghost cells


def pin_ghost_fill_gc3(lib):
    """Every ghost equals the cell it is the periodic image / wall image of,
    for u, v, w and the cell-center scalar; padding is never written."""
    for (it, jt, kt) in ((7, 5, 6), (2, 1, 3)):
        for bc in (0, 1, 2):
            g, _ = make_grid(it, jt, kt, bc)
            rng = np.random.default_rng(10 * bc + it)
            tables = [rng.integers(-1000, 1000, size=(kt, jt, it)).astype(np.float64) for _ in range(4)]
            bufs = [embed(g, t) for t in tables]
            oracle.fill_ghosts(g, *bufs[:3], lib=lib)
            oracle.fill_scalar(g, bufs[3], lib=lib)
            F = ref_tiny.Fields(*tables[:3], bc, evisc=tables[3])
            for n in range(4):
                view = full(g, bufs[n])
                for k in range(kt + 2):
                    for jj in range(jt + 2 * g.gc):
                        for ii in range(it + 2 * g.gc):
                            i, j = ii + 1 - g.gc, jj + 1 - g.gc
                            assert view[k, jj, ii] == F.get(n, i, j, k), \
                                f"ghost of field {n} at ({i},{j},{k}) bc={bc} shape={(it, jt, kt)}"
                mask = np.ones(g.alloc, bool)
                start = g.off - (g.gc - 1) * (g.js + 1)
                idx = (start + np.arange(it + 2 * g.gc)[None, None, :]
                       + g.js * np.arange(jt + 2 * g.gc)[None, :, None]
                       + g.ks * np.arange(kt + 2)[:, None, None]).ravel()
                mask[idx] = False
                assert np.all(np.isnan(bufs[n][mask])), "fill wrote outside the field"


# ---------------------------------------------------------------------------
# advec_u_2i5


def pin_2i5_constant_fields(lib):
    for bc in (0, 1, 2):
        g, _ = make_grid(9, 7, 8, bc)
        vals = (1.25, -0.75, 0.0 if bc == 1 else 0.5)
        bufs = [const_buf(g, v) for v in vals]
        oracle.fill_ghosts(g, *bufs, lib=lib)
        assert np.all(advec(g, *bufs, lib=lib) == 0.0), f"2i5 advection of constant fields not 0 (bc={bc})"


def _phi(c, x, h):
    """Phi(x) = p - (h^2/24) p_xx + (7 h^4/5760) p_xxxx for p = sum c[n] x^n."""
    P = np.polynomial.Polynomial(c)
    return P(x) - h ** 2 / 24.0 * P.deriv(2)(x) + 7.0 * h ** 4 / 5760.0 * P.deriv(4)(x)


def _face5(c, xf, h, vel):
    """Fifth-order face value of the polynomial with coefficients c (degree <= 5)."""
    c5 = c[5] if len(c) > 5 else 0.0
    return _phi(c, xf, h) - np.sign(vel) * 2.0 * c5 * h ** 5


def _face3(c, xf, h, vel):
    """Third-order face value of the polynomial with coefficients c (degree <= 3)."""
    c3 = c[3] if len(c) > 3 else 0.0
    return _phi(c[:4], xf, h) + np.sign(vel) * 0.5 * c3 * h ** 3


def pin_2i5_polynomial_x(lib):
    """u = m + quintic in x only, v = w = 0: x fluxes in closed form."""
    for mean in (2.0, -2.0):
        g, zg = make_grid(10, 4, 5, 0)
        c = np.array([mean, 0.3, -0.7, 0.5, 0.9, 1.7])   # coefficients of x^0..x^5
        p = lambda X: sum(c[n] * X ** n for n in range(6))
        ub = analytic(g, zg, lambda X, Y, Z: p(X) + 0.0 * Y + 0.0 * Z, U)
        vb, wb = const_buf(g, 0.0), const_buf(g, 0.0)
        got = advec(g, ub, vb, wb, lib=lib)
        dx = 1.0 / g.itot
        xh = (np.arange(1, g.itot + 1) - 1.0) * dx            # u positions
        xe, xw = xh + 0.5 * dx, xh - 0.5 * dx                 # faces at cell centers
        Ue = 0.5 * (p(xh) + p(xh + dx))
        Uw = 0.5 * (p(xh - dx) + p(xh))
        fe = Ue * _face5(c, xe, dx, Ue)
        fw = Uw * _face5(c, xw, dx, Uw)
        exact = -(fe - fw) * g.dxi
        err = np.max(np.abs(got - exact[None, None, :]))
        assert err <= 1e-11 * np.max(np.abs(exact)), f"2i5 x closed form err {err} (mean {mean})"


def pin_2i5_polynomial_y(lib):
    """u = quintic in y, v = V0 + V1 y (one sign), w = 0: y fluxes in closed form."""
    for V0 in (3.0, -3.0):
        g, zg = make_grid(4, 12, 5, 0)
        c = np.array([0.2, -0.4, 0.6, 1.1, -0.8, 2.3])
        q = lambda Y: sum(c[n] * Y ** n for n in range(6))
        V1 = 0.5
        ub = analytic(g, zg, lambda X, Y, Z: q(Y) + 0.0 * X + 0.0 * Z, U)
        vb = analytic(g, zg, lambda X, Y, Z: V0 + V1 * Y + 0.0 * X + 0.0 * Z, V)
        wb = const_buf(g, 0.0)
        got = advec(g, ub, vb, wb, lib=lib)
        dy = 1.0 / g.jtot
        y = (np.arange(1, g.jtot + 1) - 0.5) * dy             # u positions in y
        yn, ys = y + 0.5 * dy, y - 0.5 * dy                   # v faces
        Vn, Vs = V0 + V1 * yn, V0 + V1 * ys
        exact = -(Vn * _face5(c, yn, dy, Vn) - Vs * _face5(c, ys, dy, Vs)) * g.dyi
        err = np.max(np.abs(got - exact[None, :, None]))
        assert err <= 1e-11 * np.max(np.abs(exact)), f"2i5 y closed form err {err} (V0 {V0})"


def pin_2i5_polynomial_z(lib):
    """Uniform z, u = cubic in z, w = W0 + W1 z: every face order in closed
    form (fifth and third order as in the module docstring; second order: the
    mean of the two levels); then a quintic on the levels whose two faces are
    both fifth order."""
    for W0 in (2.0, -2.0):
        g, zg = make_grid(3, 3, 10, 2, gamma=0.0)   # periodic mode: uniform z, same ladder
        kt = g.ktot
        h = zg["Lz"] / kt
        W1 = 0.3
        for deg, c in ((3, np.array([0.5, -1.0, 0.7, 1.9])), (5, np.array([0.1, 0.4, -0.3, 0.8, -1.2, 2.5]))):
            r = lambda Z, c=c: sum(c[n] * Z ** n for n in range(len(c)))
            ub = analytic(g, zg, lambda X, Y, Z: r(Z) + 0.0 * X + 0.0 * Y, U)
            vb = const_buf(g, 0.0)
            wb = analytic(g, zg, lambda X, Y, Z: W0 + W1 * Z + 0.0 * X + 0.0 * Y, W)
            got = advec(g, ub, vb, wb, lib=lib)[:, 0, 0]
            z, zh = zg["z"], zg["zh"]
            flux = {}
            for kf in range(1, kt + 2):
                Wf = W0 + W1 * zh[kf]
                order = ref_tiny.z_face_order(kf, kt)
                if order == 2:
                    fv = 0.5 * (r(z[kf - 1]) + r(z[kf]))
                elif order == 3:
                    fv = _face3(c, zh[kf], h, Wf) if deg == 3 else np.nan
                else:
                    fv = _face5(c, zh[kf], h, Wf)
                flux[kf] = Wf * fv
            exact = np.array([-(flux[k + 1] - flux[k]) * g.dzi[k] for k in range(1, kt + 1)])
            ks = np.arange(1, kt + 1)
            sel = np.ones(kt, bool) if deg == 3 else (ks >= 3) & (ks <= kt - 2)
            err = np.max(np.abs(got[sel] - exact[sel]))
            assert err <= 1e-11 * np.max(np.abs(exact[sel])), f"2i5 z closed form err {err} (deg {deg}, W0 {W0})"


def pin_2i5_textbook_weights(lib):
    """A unit impulse in u advected by a uniform v (or w) of either sign: the
    tendencies next to it follow the textbook upwind-biased weights."""
    w5 = {1: {-2: 2, -1: -13, 0: 47, 1: 27, 2: -3}, -1: {-1: -3, 0: 27, 1: 47, 2: -13, 3: 2}}
    w3 = {1: {-1: -1, 0: 5, 1: 2}, -1: {0: 2, 1: 5, 2: -1}}
    # y: impulse at (i0, j0, k0), v = s; check the column i0 for j != j0
    for s in (1.0, -1.0):
        g, zg = make_grid(5, 12, 4, 2, gamma=0.0)
        i0, j0, k0 = 3, 6, 2
        ua = np.zeros((g.ktot, g.jtot, g.itot))
        ua[k0 - 1, j0 - 1, i0 - 1] = 1.0
        ub = embed(g, ua)
        vb = const_buf(g, s)
        wb = const_buf(g, 0.0)
        oracle.fill_ghosts(g, ub, vb, wb, lib=lib)
        got = advec(g, ub, vb, wb, lib=lib)[k0 - 1, :, i0 - 1]
        wt = w5[int(s)]
        # face between u_j and u_j+1: value = sum_m wt[m] u_{j+m} / 60, m relative to a0 = u_j
        face = lambda j: wt.get(j0 - j, 0) / 60.0
        for j in range(1, g.jtot + 1):
            if j == j0:
                continue
            exact = -s * (face(j) - face(j - 1)) * g.dyi
            assert abs(got[j - 1] - exact) <= 1e-12 * g.dyi, f"y upwind weights, v={s}, j={j}"
    # z: impulse near each wall, w = s; third-order faces next to the walls
    for s in (1.0, -1.0):
        for k0 in (2, 7):
            g, zg = make_grid(3, 3, 8, 2, gamma=0.0)
            kt = g.ktot
            ua = np.zeros((kt, g.jtot, g.itot))
            ua[k0 - 1, 1, 1] = 1.0
            ub = embed(g, ua)
            vb = const_buf(g, 0.0)
            wb = const_buf(g, s)
            oracle.fill_ghosts(g, ub, vb, wb, lib=lib)
            got = advec(g, ub, vb, wb, lib=lib)[:, 1, 1]

            def face(kf):   # face between levels kf-1 (a0) and kf (a1)
                order = ref_tiny.z_face_order(kf, kt)
                m = k0 - (kf - 1)
                if order == 2:
                    return 0.5 if m in (0, 1) else 0.0
                if order == 3:
                    return w3[int(s)].get(m, 0) / 6.0
                return w5[int(s)].get(m, 0) / 60.0
            for k in range(1, kt + 1):
                if k == k0:
                    continue
                exact = -s * (face(k + 1) - face(k)) * g.dzi[k]
                assert abs(got[k - 1] - exact) <= 1e-12 * np.max(g.dzi), f"z weights, w={s}, k0={k0}, k={k}"


def pin_2i5_conservation(lib):
    g, zg = make_grid(12, 10, 8, oracle.BC_ZPERIODIC)
    (u, v, w), _ = random_state(g, 5, lib=lib)
    adv = advec(g, u, v, w, lib=lib)
    dz = 1.0 / g.dzi[1:g.ktot + 1]
    vol = (1.0 / g.dxi) * (1.0 / g.dyi) * dz[:, None, None]
    umax = max(np.max(np.abs(interior(g, f))) for f in (u, v, w))
    n = g.itot * g.jtot * g.ktot
    A = 4 * n * np.max(vol) * umax * umax * (g.dxi + g.dyi + np.max(g.dzi))
    assert abs(np.sum(adv * vol)) <= 1e-14 * A, f"2i5 advection not conservative: {np.sum(adv * vol)}"


def pin_2i5_translation(lib):
    for bc in (0, 2):
        g, zg = make_grid(11, 9, 6, bc)
        fs = inputs.random_fields(7, g.itot, g.jtot, g.ktot)
        sx, sy = 4, 5
        outs = []
        for flds in (fs, [np.roll(np.roll(f, sx, axis=2), sy, axis=1) for f in fs]):
            bufs = [embed(g, f) for f in flds]
            oracle.fill_ghosts(g, *bufs, lib=lib)
            outs.append(advec(g, *bufs, lib=lib))
        assert np.array_equal(np.roll(np.roll(outs[0], sx, axis=2), sy, axis=1), outs[1]), "2i5 not shift-invariant"


def pin_2i5_brute_force(lib):
    for bc in (0, 1, 2):
        for (it, jt, kt) in ((5, 4, 6), (3, 2, 2), (1, 3, 4), (7, 5, 9)):
            g, zg = make_grid(it, jt, kt, bc)
            (u, v, w), _ = random_state(g, 3 + bc, lib=lib)
            ours = advec(g, u, v, w, lib=lib)
            fs = inputs.random_fields(3 + bc, it, jt, kt)
            ref = ref_tiny.advec_u_2i5(*fs, g.dxi, g.dyi, g.dzi, bc)
            err = np.max(np.abs(ours - ref))
            assert err <= 1e-13 * np.max(np.abs(ref)), f"2i5 vs brute force bc {bc} {(it, jt, kt)}: {err}"


def pin_2i5_second_order(lib):
    """Smooth fields on a stretched grid: the error against the analytic
    -div(u u) falls as h^2."""
    import math
    errs = []
    for n in (16, 32, 64):
        g, zg = make_grid(n, n, n, 0, layout=inputs.plain_layout(n, n, n, 3))
        kx = ky = 2 * math.pi
        kz = math.pi / zg["Lz"]
        s, co = np.sin, np.cos
        uf = lambda X, Y, Z: 1.0 + 0.8 * s(kx * X) * co(ky * Y) * co(kz * Z)
        vf = lambda X, Y, Z: 0.5 + 0.6 * co(kx * X) * s(ky * Y) * co(kz * Z)
        wf = lambda X, Y, Z: 0.5 * co(kx * X) * co(ky * Y) * s(kz * Z)
        ux = lambda X, Y, Z: 0.8 * kx * co(kx * X) * co(ky * Y) * co(kz * Z)
        uy = lambda X, Y, Z: -0.8 * ky * s(kx * X) * s(ky * Y) * co(kz * Z)
        uz = lambda X, Y, Z: -0.8 * kz * s(kx * X) * co(ky * Y) * s(kz * Z)
        vy = lambda X, Y, Z: 0.6 * ky * co(kx * X) * co(ky * Y) * co(kz * Z)
        wz = lambda X, Y, Z: 0.5 * kz * co(kx * X) * co(ky * Y) * co(kz * Z)
        bufs = [analytic(g, zg, f, i) for i, f in enumerate((uf, vf, wf))]
        adv = advec(g, *bufs, lib=lib)
        Z, Y, X = inputs.staggered_positions(U, n, n, zg, 3)
        Z, Y, X = Z[1:n + 1], Y[:, 3:n + 3], X[:, :, 3:n + 3]
        ex = -(2 * uf(X, Y, Z) * ux(X, Y, Z) + uy(X, Y, Z) * vf(X, Y, Z) + uf(X, Y, Z) * vy(X, Y, Z)
               + uz(X, Y, Z) * wf(X, Y, Z) + uf(X, Y, Z) * wz(X, Y, Z))
        errs.append(np.max(np.abs(adv - ex)))
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(order >= 1.8), f"2i5 observed orders {order}"


# ---------------------------------------------------------------------------
# diff_smag


def pin_smag_constant_velocity(lib):
    for bc in (0, 1, 2):
        g, _ = make_grid(8, 7, 6, bc, gc=1)
        bufs = [const_buf(g, v) for v in (0.37, -1.1, 0.0 if bc == 1 else 0.3)]
        oracle.fill_ghosts(g, *bufs, lib=lib)
        _, e = random_state(g, 4, lib=lib)
        for d in smag(g, *bufs, e, lib=lib):
            assert np.all(d == 0.0), f"diffusion of constant velocity not 0 (bc={bc})"


def pin_smag_constant_viscosity_identity(lib):
    """nu constant: stress divergence = nu Laplacian (the oracle's pinned
    diff_uvw) + nu times the discrete gradient of the divergence
    D = du/dx + dv/dy + dw/dz at cell centers."""
    nu = 0.013
    for bc in (0, 1, 2):
        g, zg = make_grid(9, 8, 7, bc, gc=1)
        (u, v, w), _ = random_state(g, 21 + bc, lib=lib)
        e = const_buf(g, nu)
        got = smag(g, u, v, w, e, lib=lib)
        lap = [zero_tendency(g) for _ in range(3)]
        oracle.diff_uvw(g, *lap, u, v, w, nu, lib=lib)
        lap = [interior(g, x) for x in lap]
        F = [full(g, f) for f in (u, v, w)]       # [k, j, i] with index 0 the first ghost
        it, jt, kt = g.itot, g.jtot, g.ktot
        dzi = g.dzi[:, None, None]
        # D at centers k = 0..kt, j = 0..jt, i = 0..it (padded index = logical index for gc = 1)
        D = ((F[0][0:kt + 1, 0:jt + 1, 1:it + 2] - F[0][0:kt + 1, 0:jt + 1, 0:it + 1]) * g.dxi
             + (F[1][0:kt + 1, 1:jt + 2, 0:it + 1] - F[1][0:kt + 1, 0:jt + 1, 0:it + 1]) * g.dyi
             + (F[2][1:kt + 2, 0:jt + 1, 0:it + 1] - F[2][0:kt + 1, 0:jt + 1, 0:it + 1]) * dzi[0:kt + 1])
        exp_u = lap[0] + nu * (D[1:, 1:, 1:] - D[1:, 1:, :-1]) * g.dxi
        exp_v = lap[1] + nu * (D[1:, 1:, 1:] - D[1:, :-1, 1:]) * g.dyi
        exp_w = lap[2] + nu * (D[1:, 1:, 1:] - D[:-1, 1:, 1:]) * g.dzhi[1:kt + 1, None, None]
        k0 = kw0(g) - 1
        for name, a, b in (("u", got[0], exp_u), ("v", got[1], exp_v), ("w", got[2][k0:], exp_w[k0:])):
            err = np.max(np.abs(a - b))
            assert err <= 1e-11 * np.max(np.abs(b)), f"constant-viscosity identity ({name}, bc {bc}): {err}"
        if k0:
            assert np.all(got[2][0] == 0.0), "wt written on the bottom wall face"


def pin_smag_polynomials(lib):
    """Viscosity linear in one coordinate, one velocity component quadratic:
    closed forms for every tendency (stretched z)."""
    a, b, c = 0.7, 0.4, 1.3
    g, zg = make_grid(6, 7, 8, 0, gc=1)
    cc = inputs.coords(g.itot, g.jtot, zg)
    xh, x = cc["xh"][1:g.itot + 1], cc["x"][1:g.itot + 1]
    yh, y = cc["yh"][1:g.jtot + 1], cc["y"][1:g.jtot + 1]
    zh, z = zg["zh"][1:g.ktot + 1], zg["z"][1:g.ktot + 1]
    zm = 0.5 * (zg["zh"][1:g.ktot + 1] + zg["zh"][2:g.ktot + 2])
    Xh, X = xh[None, None, :], x[None, None, :]
    Yh, Y = yh[None, :, None], y[None, :, None]
    Zh, Z, Zm = zh[:, None, None], z[:, None, None], zm[:, None, None]
    zero = lambda X_, Y_, Z_: 0.0 * X_ + 0.0 * Y_ + 0.0 * Z_
    cases = [
        # (velocity field, its profile, viscosity profile, expected (ut, vt, wt))
        ("u=cx^2, nu(x)", U, lambda X_, Y_, Z_: c * X_ ** 2, lambda X_, Y_, Z_: a + b * X_,
         (4 * c * (a + 2 * b * Xh), 0.0, 0.0)),
        ("u=cy^2, nu(y)", U, lambda X_, Y_, Z_: c * Y_ ** 2, lambda X_, Y_, Z_: a + b * Y_,
         (2 * c * (a + 2 * b * Y), 0.0, 0.0)),
        ("u=cz^2, nu(z)", U, lambda X_, Y_, Z_: c * Z_ ** 2, lambda X_, Y_, Z_: a + b * Z_,
         (2 * c * (a + 2 * b * Zm), 0.0, 0.0)),
        ("v=cx^2, nu(y)", V, lambda X_, Y_, Z_: c * X_ ** 2, lambda X_, Y_, Z_: a + b * Y_,
         (2 * b * c * Xh, 2 * c * (a + b * Yh), 0.0)),
        ("w=cx^2, nu(z)", W, lambda X_, Y_, Z_: c * X_ ** 2, lambda X_, Y_, Z_: a + b * Z_,
         (2 * b * c * Xh, 0.0, 2 * c * (a + b * Zh))),
        ("w=cy^2, nu(z)", W, lambda X_, Y_, Z_: c * Y_ ** 2, lambda X_, Y_, Z_: a + b * Z_,
         (0.0, 2 * b * c * Yh, 2 * c * (a + b * Zh))),
        ("v=cy^2, nu(y)", V, lambda X_, Y_, Z_: c * Y_ ** 2, lambda X_, Y_, Z_: a + b * Y_,
         (0.0, 4 * c * (a + 2 * b * Yh), 0.0)),
    ]
    for name, fld, prof, nuf, expect in cases:
        bufs = [analytic(g, zg, prof if n == fld else zero, n) for n in range(3)]
        e = analytic(g, zg, nuf, E)
        got = smag(g, *bufs, e, lib=lib)
        for n in range(3):
            ex = np.broadcast_to(np.asarray(expect[n], dtype=float), got[n].shape)
            sl = slice(kw0(g) - 1, None) if n == 2 else slice(None)
            err = np.max(np.abs(got[n][sl] - ex[sl]))
            scale = np.max(np.abs(ex)) + 1.0
            assert err <= 1e-14 * scale * (g.dxi ** 2 + g.dyi ** 2 + np.max(g.dzi) ** 2), \
                f"{name}: tendency {n} err {err}"


def pin_smag_conservation(lib):
    g, zg = make_grid(12, 10, 8, oracle.BC_ZPERIODIC, gc=1)
    (u, v, w), e = random_state(g, 6, lib=lib, evisc_mean=0.05)
    dz = 1.0 / g.dzi[1:g.ktot + 1]
    vol = (1.0 / g.dxi) * (1.0 / g.dyi) * dz[:, None, None]
    n = g.itot * g.jtot * g.ktot
    Ad = 8 * n * np.max(vol) * 0.075 * 2.0 * (g.dxi ** 2 + g.dyi ** 2 + np.max(g.dzi) ** 2)
    for d in smag(g, u, v, w, e, lib=lib):
        assert abs(np.sum(d * vol)) <= 1e-14 * Ad, f"stress divergence not conservative: {np.sum(d * vol)}"


def pin_smag_xy_symmetry(lib):
    """Exchanging x and y (u <-> v) on a square grid exchanges ut and vt."""
    for bc in (0, 2):
        g, zg = make_grid(8, 8, 6, bc, gc=1)
        fs = inputs.random_fields(31, 8, 8, 6)
        ev = inputs.evisc_field(31, 8, 8, 6, mean=0.02)
        tr = lambda a: np.ascontiguousarray(np.swapaxes(a, 1, 2))
        outs = []
        for (uu, vv, ww, ee) in ((fs[0], fs[1], fs[2], ev), (tr(fs[1]), tr(fs[0]), tr(fs[2]), tr(ev))):
            bufs = [embed(g, f) for f in (uu, vv, ww)]
            oracle.fill_ghosts(g, *bufs, lib=lib)
            e = embed(g, ee)
            oracle.fill_scalar(g, e, lib=lib)
            outs.append(smag(g, *bufs, e, lib=lib))
        a, bt = outs
        scale = max(np.max(np.abs(x)) for x in a)
        for got, ref in ((bt[0], tr(a[1])), (bt[1], tr(a[0])), (bt[2], tr(a[2]))):
            assert np.max(np.abs(got - ref)) <= 1e-13 * scale, f"x-y symmetry broken (bc {bc})"


def pin_smag_brute_force(lib):
    for bc in (0, 1, 2):
        for (it, jt, kt) in ((5, 4, 6), (3, 2, 2), (1, 3, 4)):
            g, zg = make_grid(it, jt, kt, bc, gc=1)
            (u, v, w), e = random_state(g, 8 + bc, lib=lib)
            ours = smag(g, u, v, w, e, lib=lib)
            fs = inputs.random_fields(8 + bc, it, jt, kt)
            ev = inputs.evisc_field(8 + bc, it, jt, kt, mean=1e-2)
            ref = ref_tiny.diff_smag(*fs, ev, g.dxi, g.dyi, g.dzi, g.dzhi, bc)
            for n, (a_, b_) in enumerate(zip(ours, ref)):
                err = np.max(np.abs(a_ - b_))
                assert err <= 1e-13 * (np.max(np.abs(b_)) + 1e-300), \
                    f"diff_smag vs brute force, output {n}, bc {bc}, {(it, jt, kt)}: {err}"


def pin_point_les(lib):
    """Single-point evaluation equals the sweeps."""
    g, zg = make_grid(9, 8, 7, 0)
    (u, v, w), e = random_state(g, 17, lib=lib)
    adv = advec(g, u, v, w, lib=lib)
    d = smag(g, u, v, w, e, lib=lib)
    for (i, j, k) in ((1, 1, 1), (9, 8, 7), (4, 3, 2), (5, 8, 6)):
        p = oracle.point_les(g, u, v, w, e, i, j, k, lib=lib)
        assert p[0] == adv[k - 1, j - 1, i - 1]
        for n in range(3):
            assert p[1 + n] == d[n][k - 1, j - 1, i - 1]


PINS = [pin_ghost_fill_gc3, pin_2i5_constant_fields, pin_2i5_polynomial_x, pin_2i5_polynomial_y,
        pin_2i5_polynomial_z, pin_2i5_textbook_weights, pin_2i5_conservation, pin_2i5_translation,
        pin_2i5_brute_force, pin_2i5_second_order, pin_smag_constant_velocity,
        pin_smag_constant_viscosity_identity, pin_smag_polynomials, pin_smag_conservation,
        pin_smag_xy_symmetry, pin_smag_brute_force, pin_point_les]
