"""Brute-force finite-volume reference for tiny grids (pure Python loops).

Independent of the oracle's strided arrays: it reads the interior fields by
(i, j, k) coordinates, applies the boundary rules by index mapping instead of
ghost arrays, builds explicit face-flux / face-gradient tables and takes
their divergence.  Used to cross-check the oracle's indexing on grids of a
few cells.
"""
from __future__ import annotations

import numpy as np

U, V, W, E = 0, 1, 2, 3


class Fields:
    def __init__(self, u, v, w, bc, evisc=None):
        self.f = (u, v, w, evisc)  # interior arrays [k-1][j-1][i-1]
        self.ktot, self.jtot, self.itot = u.shape
        self.bc = bc

    def get(self, n, i, j, k):
        """Field n at 1-based index (i, j, k), ghosts resolved by the rules."""
        it, jt, kt = self.itot, self.jtot, self.ktot
        i = (i - 1) % it + 1
        j = (j - 1) % jt + 1
        sign = 1.0
        if self.bc == 2:
            k = (k - 1) % kt + 1
        elif n in (U, V, E):
            k = 1 if k == 0 else (kt if k == kt + 1 else k)
        else:
            if self.bc == 0:  # zero gradient: w1 = w2, w_{kt+1} = w_kt, w0 = w2
                k = 2 if k in (0, 1) else (kt if k == kt + 1 else k)
            else:  # no penetration: w1 = w_{kt+1} = 0, w0 = -w2
                if k in (1, kt + 1):
                    return 0.0
                if k == 0:
                    k, sign = 2, -1.0
        return sign * float(self.f[n][k - 1, j - 1, i - 1])


def tendencies(u, v, w, dxi, dyi, dzi, dzhi, visc, bc):
    """Return (ut_adv, ut_diff, vt_diff, wt_diff) as interior arrays."""
    F = Fields(u, v, w, bc)
    kt, jt, it = u.shape
    h = 0.5
    out = [np.zeros((kt, jt, it)) for _ in range(4)]
    kw0 = 1 if bc == 2 else 2
    for j in range(1, jt + 1):
        for k in range(1, kt + 1):
            # x fluxes of u-momentum at cell centers c = 0..itot (between faces c, c+1)
            Fx = {c: (h * (F.get(U, c, j, k) + F.get(U, c + 1, j, k))) ** 2 for c in range(0, it + 1)}
            for i in range(1, it + 1):
                out[0][k - 1, j - 1, i - 1] -= (Fx[i] - Fx[i - 1]) * dxi
    for i in range(1, it + 1):
        for k in range(1, kt + 1):
            Fy = {jf: h * (F.get(V, i - 1, jf, k) + F.get(V, i, jf, k))
                  * h * (F.get(U, i, jf - 1, k) + F.get(U, i, jf, k)) for jf in range(1, jt + 2)}
            for j in range(1, jt + 1):
                out[0][k - 1, j - 1, i - 1] -= (Fy[j + 1] - Fy[j]) * dyi
        for j in range(1, jt + 1):
            Fz = {kf: h * (F.get(W, i - 1, j, kf) + F.get(W, i, j, kf))
                  * h * (F.get(U, i, j, kf - 1) + F.get(U, i, j, kf)) for kf in range(1, kt + 2)}
            for k in range(1, kt + 1):
                out[0][k - 1, j - 1, i - 1] -= (Fz[k + 1] - Fz[k]) * dzi[k]
    # diffusion: divergence of face gradients
    for n, slot in ((U, 1), (V, 2), (W, 3)):
        for k in range(1, kt + 1):
            if n == W and k < kw0:
                continue
            for j in range(1, jt + 1):
                for i in range(1, it + 1):
                    g = lambda a, b, c: F.get(n, a, b, c)
                    gx = ((g(i + 1, j, k) - g(i, j, k)) * dxi - (g(i, j, k) - g(i - 1, j, k)) * dxi) * dxi
                    gy = ((g(i, j + 1, k) - g(i, j, k)) * dyi - (g(i, j, k) - g(i, j - 1, k)) * dyi) * dyi
                    if n == W:  # gradients at centers k, k-1; divide by dzh_k
                        gz = ((g(i, j, k + 1) - g(i, j, k)) * dzi[k]
                              - (g(i, j, k) - g(i, j, k - 1)) * dzi[k - 1]) * dzhi[k]
                    else:  # gradients at faces k+1, k; divide by dz_k
                        gz = ((g(i, j, k + 1) - g(i, j, k)) * dzhi[k + 1]
                              - (g(i, j, k) - g(i, j, k - 1)) * dzhi[k]) * dzi[k]
                    out[slot][k - 1, j - 1, i - 1] = visc * (gx + gy + gz)
    return out


# ---------------------------------------------------------------------------
# Fifth-order advection and Smagorinsky-type diffusion, written independently
# of the oracle: face values from the textbook upwind-biased weight tables
# (chosen by the sign of the advecting velocity), fluxes tabulated per face,
# stresses tabulated per cell center / edge.

# weights on (a_-2, a_-1, a0, a1, a2, a3) for the face between a0 and a1
W5_POS = (2, -13, 47, 27, -3, 0)
W5_NEG = (0, -3, 27, 47, -13, 2)
W6_CEN = (1, -8, 37, 37, -8, 1)
# weights on (a_-1, a0, a1, a2)
W3_POS = (-2, 10, 4, 0)
W3_NEG = (0, 4, 10, -2)
W4_CEN = (-1, 7, 7, -1)


def face_value(vel, vals, order):
    """Upwind-biased face value between the middle two of ``vals``."""
    if order == 2:
        return 0.5 * (vals[0] + vals[1])
    if order == 3:
        wt = W3_POS if vel > 0 else (W3_NEG if vel < 0 else W4_CEN)
        den = 12.0
    else:
        wt = W5_POS if vel > 0 else (W5_NEG if vel < 0 else W6_CEN)
        den = 60.0
    return sum(c * a for c, a in zip(wt, vals)) / den


def z_face_order(kf, kt):
    if kf in (1, kt + 1):
        return 2
    if kf in (2, kt):
        return 3
    return 5


def advec_u_2i5(u, v, w, dxi, dyi, dzi, bc):
    """Tendency of u from fifth-order-interpolated advection (interior array)."""
    F = Fields(u, v, w, bc)
    kt, jt, it = u.shape
    out = np.zeros((kt, jt, it))
    g = F.get
    for k in range(1, kt + 1):
        for j in range(1, jt + 1):
            # x faces c = 0..it sit between u_c and u_c+1
            Fx = {}
            for c in range(0, it + 1):
                vel = 0.5 * (g(U, c, j, k) + g(U, c + 1, j, k))
                Fx[c] = vel * face_value(vel, [g(U, c + d, j, k) for d in range(-2, 4)], 5)
            for i in range(1, it + 1):
                out[k - 1, j - 1, i - 1] -= (Fx[i] - Fx[i - 1]) * dxi
    for k in range(1, kt + 1):
        for i in range(1, it + 1):
            # y faces jf = 1..jt+1 sit between u_jf-1 and u_jf
            Fy = {}
            for jf in range(1, jt + 2):
                vel = 0.5 * (g(V, i - 1, jf, k) + g(V, i, jf, k))
                Fy[jf] = vel * face_value(vel, [g(U, i, jf - 1 + d, k) for d in range(-2, 4)], 5)
            for j in range(1, jt + 1):
                out[k - 1, j - 1, i - 1] -= (Fy[j + 1] - Fy[j]) * dyi
    for j in range(1, jt + 1):
        for i in range(1, it + 1):
            Fz = {}
            for kf in range(1, kt + 2):
                vel = 0.5 * (g(W, i - 1, j, kf) + g(W, i, j, kf))
                order = z_face_order(kf, kt)
                lo = {2: 0, 3: -1, 5: -2}[order]
                hi = {2: 1, 3: 2, 5: 3}[order]
                vals = [g(U, i, j, kf - 1 + d) for d in range(lo, hi + 1)]
                Fz[kf] = vel * face_value(vel, vals, order)
            for k in range(1, kt + 1):
                out[k - 1, j - 1, i - 1] -= (Fz[k + 1] - Fz[k]) * dzi[k]
    return out


def diff_smag(u, v, w, evisc, dxi, dyi, dzi, dzhi, bc):
    """Divergence of nu (grad u + grad u^T) with nu at cell centers.

    Stresses are tabulated where they live: normal stresses at cell centers,
    shear stresses at cell edges (nu = mean of the four surrounding centers).
    Returns (ut, vt, wt) interior arrays (wt zero on wall faces).
    """
    F = Fields(u, v, w, bc, evisc)
    kt, jt, it = u.shape
    g = F.get
    # position-aware derivatives; spacing in z from the metric arrays
    du_dx = lambda i, j, k: (g(U, i + 1, j, k) - g(U, i, j, k)) * dxi      # at center (i, j, k)
    dv_dy = lambda i, j, k: (g(V, i, j + 1, k) - g(V, i, j, k)) * dyi      # at center
    dw_dz = lambda i, j, k: (g(W, i, j, k + 1) - g(W, i, j, k)) * dzi[k]   # at center
    nu_c = lambda i, j, k: g(E, i, j, k)

    def nu_xy(i, j, k):  # edge (xh_i, yh_j, z_k)
        return 0.25 * (g(E, i - 1, j - 1, k) + g(E, i, j - 1, k) + g(E, i - 1, j, k) + g(E, i, j, k))

    def nu_xz(i, j, k):  # edge (xh_i, y_j, zh_k)
        return 0.25 * (g(E, i - 1, j, k - 1) + g(E, i, j, k - 1) + g(E, i - 1, j, k) + g(E, i, j, k))

    def nu_yz(i, j, k):  # edge (x_i, yh_j, zh_k)
        return 0.25 * (g(E, i, j - 1, k - 1) + g(E, i, j, k - 1) + g(E, i, j - 1, k) + g(E, i, j, k))

    def t_xy(i, j, k):
        return nu_xy(i, j, k) * ((g(U, i, j, k) - g(U, i, j - 1, k)) * dyi
                                 + (g(V, i, j, k) - g(V, i - 1, j, k)) * dxi)

    def t_xz(i, j, k):
        return nu_xz(i, j, k) * ((g(U, i, j, k) - g(U, i, j, k - 1)) * dzhi[k]
                                 + (g(W, i, j, k) - g(W, i - 1, j, k)) * dxi)

    def t_yz(i, j, k):
        return nu_yz(i, j, k) * ((g(V, i, j, k) - g(V, i, j, k - 1)) * dzhi[k]
                                 + (g(W, i, j, k) - g(W, i, j - 1, k)) * dyi)

    out = [np.zeros((kt, jt, it)) for _ in range(3)]
    kw0 = 1 if bc == 2 else 2
    for k in range(1, kt + 1):
        for j in range(1, jt + 1):
            for i in range(1, it + 1):
                t_xx = lambda a: 2.0 * nu_c(a, j, k) * du_dx(a, j, k)
                out[0][k - 1, j - 1, i - 1] = ((t_xx(i) - t_xx(i - 1)) * dxi
                                               + (t_xy(i, j + 1, k) - t_xy(i, j, k)) * dyi
                                               + (t_xz(i, j, k + 1) - t_xz(i, j, k)) * dzi[k])
                t_yy = lambda b: 2.0 * nu_c(i, b, k) * dv_dy(i, b, k)
                out[1][k - 1, j - 1, i - 1] = ((t_xy(i + 1, j, k) - t_xy(i, j, k)) * dxi
                                               + (t_yy(j) - t_yy(j - 1)) * dyi
                                               + (t_yz(i, j, k + 1) - t_yz(i, j, k)) * dzi[k])
                if k >= kw0:
                    t_zz = lambda c: 2.0 * nu_c(i, j, c) * dw_dz(i, j, c)
                    out[2][k - 1, j - 1, i - 1] = ((t_xz(i + 1, j, k) - t_xz(i, j, k)) * dxi
                                                   + (t_yz(i, j + 1, k) - t_yz(i, j, k)) * dyi
                                                   + (t_zz(k) - t_zz(k - 1)) * dzhi[k])
    return out
