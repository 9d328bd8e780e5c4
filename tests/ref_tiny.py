"""Brute-force finite-volume reference for tiny grids (pure Python loops).

Independent of the oracle's strided arrays: it reads the interior fields by
(i, j, k) coordinates, applies the boundary rules by index mapping instead of
ghost arrays, builds explicit face-flux / face-gradient tables and takes
their divergence.  Used to cross-check the oracle's indexing on grids of a
few cells.
"""
from __future__ import annotations

import numpy as np

U, V, W = 0, 1, 2


class Fields:
    def __init__(self, u, v, w, bc):
        self.f = (u, v, w)  # interior arrays [k-1][j-1][i-1]
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
        elif n in (U, V):
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
