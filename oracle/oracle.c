/*
 * Oracle: a plain, slow, FP64 CPU definition of the staggered-grid stencil
 * step.  TEST INFRASTRUCTURE ONLY: it is called by the test suite, by the
 * smoke check and by the benchmark's CPU-baseline leg, never by the product
 * path.  It shares no code with the GPU library.
 *
 * What it computes.  The paper evaluates its tuner on two kernels of a CFD
 * code: "advec_u", the advection of the x-velocity u, and "diff_uvw", the
 * diffusion of u, v and w, on a 3-D grid in float or double (Section
 * "Application", Section "Tunable Parameters").  The paper gives no formulas;
 * this library fixes the schemes as a second-order flux-form advection of u
 * and a second-order constant-viscosity Laplacian on a staggered (Arakawa C)
 * grid with one ghost cell per side, and adds the paper's named schemes:
 * advection with fifth-order interpolation (three ghost cells in x and y)
 * and Smagorinsky-type diffusion with a given eddy viscosity.  Each function
 * below writes its definition out point by point, in the order of the
 * formula, with no blocking or fusion.
 *
 * Layout: element (i, j, k) of every field is p[off + i + j*js + k*ks],
 * i in [1-gc, itot+gc] (interior [1, itot]), likewise j, and k in
 * [0, ktot+1]; gc is 1, or 3 for the fifth-order advection.
 * Staggering: u at (xh_i, y_j, z_k), v at (x_i, yh_j, z_k), w at (x_i, y_j, zh_k).
 * Metrics: dxi = 1/dx, dyi = 1/dy, dzi[k] = 1/(zh[k+1]-zh[k]),
 *          dzhi[k] = 1/(z[k]-z[k-1]).
 *
 * Boundary modes (bc): 0 = z walls, zero gradient; 1 = z walls, w = 0 at the
 * walls; 2 = periodic in z.  x and y are always periodic.
 *
 * Built with -O2 -ffp-contract=off so that every multiply and add rounds on
 * its own, as written.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define BC_ZWALL_ZEROGRAD 0
#define BC_ZWALL_NOPEN 1
#define BC_ZPERIODIC 2

typedef struct {
    int itot, jtot, ktot;
    int64_t off, js, ks;
    int gc; /* ghost cells per side in x and y; z always has one */
} grid;

static inline int64_t at(const grid *g, int i, int j, int k)
{
    return g->off + (int64_t)i + (int64_t)j * g->js + (int64_t)k * g->ks;
}

static inline double interp(double a, double b) { return 0.5 * (a + b); }

/* Interior index that periodic index p (any integer) is the image of. */
static inline int wrap(int p, int n) { return 1 + (((p - 1) % n) + n) % n; }

/* ---------------------------------------------------------------------------
 * Ghost cells.  Periodic in x, then periodic in y over whole rows (so the
 * x-ghost columns are carried into the y-ghost rows), then the z rule over
 * whole planes (so edges and corners are carried too).  x and y have gc
 * ghost cells per side, z has one.
 * ------------------------------------------------------------------------- */
static void fill_xy(const grid *g, double *f)
{
    const int gc = g->gc;
    for (int k = 1; k <= g->ktot; ++k)
        for (int j = 1; j <= g->jtot; ++j)
            for (int m = 1; m <= gc; ++m) {
                f[at(g, 1 - m, j, k)] = f[at(g, wrap(1 - m, g->itot), j, k)];
                f[at(g, g->itot + m, j, k)] = f[at(g, wrap(g->itot + m, g->itot), j, k)];
            }
    for (int k = 1; k <= g->ktot; ++k)
        for (int m = 1; m <= gc; ++m)
            for (int i = 1 - gc; i <= g->itot + gc; ++i) {
                f[at(g, i, 1 - m, k)] = f[at(g, i, wrap(1 - m, g->jtot), k)];
                f[at(g, i, g->jtot + m, k)] = f[at(g, i, wrap(g->jtot + m, g->jtot), k)];
            }
}

static void copy_plane(const grid *g, double *f, int kdst, int ksrc, double sign)
{
    for (int j = 1 - g->gc; j <= g->jtot + g->gc; ++j)
        for (int i = 1 - g->gc; i <= g->itot + g->gc; ++i)
            f[at(g, i, j, kdst)] = sign * f[at(g, i, j, ksrc)];
}

static void set_plane(const grid *g, double *f, int kdst, double value)
{
    for (int j = 1 - g->gc; j <= g->jtot + g->gc; ++j)
        for (int i = 1 - g->gc; i <= g->itot + g->gc; ++i)
            f[at(g, i, j, kdst)] = value;
}

static void fill_all(const grid *g, int bc, double *u, double *v, double *w)
{
    double *f3[3] = {u, v, w};
    for (int n = 0; n < 3; ++n) fill_xy(g, f3[n]);
    const int kt = g->ktot;
    if (bc == BC_ZPERIODIC) {
        for (int n = 0; n < 3; ++n) {
            copy_plane(g, f3[n], 0, kt, 1.0);
            copy_plane(g, f3[n], kt + 1, 1, 1.0);
        }
        return;
    }
    /* u and v: zero gradient across both walls (free slip). */
    for (int n = 0; n < 2; ++n) {
        copy_plane(g, f3[n], 0, 1, 1.0);
        copy_plane(g, f3[n], kt + 1, kt, 1.0);
    }
    /* w lives on the faces; face 1 is the bottom wall, face kt+1 the top. */
    if (bc == BC_ZWALL_ZEROGRAD) {
        copy_plane(g, w, 1, 2, 1.0);
        copy_plane(g, w, kt + 1, kt, 1.0);
        copy_plane(g, w, 0, 2, 1.0);
    } else {
        set_plane(g, w, 1, 0.0);
        set_plane(g, w, kt + 1, 0.0);
        copy_plane(g, w, 0, 2, -1.0);
    }
}

void ora_fill_ghosts(int itot, int jtot, int ktot, int64_t off, int64_t js, int64_t ks,
                     int bc, double *u, double *v, double *w)
{
    grid g = {itot, jtot, ktot, off, js, ks, 1};
    fill_all(&g, bc, u, v, w);
}

void ora_fill_ghosts_gc(int itot, int jtot, int ktot, int64_t off, int64_t js, int64_t ks,
                        int gc, int bc, double *u, double *v, double *w)
{
    grid g = {itot, jtot, ktot, off, js, ks, gc};
    fill_all(&g, bc, u, v, w);
}

/* A cell-center scalar (the eddy viscosity): periodic in x and y, and in z
 * periodic or zero gradient across the walls, as u and v. */
void ora_fill_scalar(int itot, int jtot, int ktot, int64_t off, int64_t js, int64_t ks,
                     int gc, int bc, double *f)
{
    grid g = {itot, jtot, ktot, off, js, ks, gc};
    fill_xy(&g, f);
    if (bc == BC_ZPERIODIC) {
        copy_plane(&g, f, 0, ktot, 1.0);
        copy_plane(&g, f, ktot + 1, 1, 1.0);
    } else {
        copy_plane(&g, f, 0, 1, 1.0);
        copy_plane(&g, f, ktot + 1, ktot, 1.0);
    }
}

/* ---------------------------------------------------------------------------
 * advec_u: tendency of u from the divergence of the momentum flux u*(u,v,w),
 * second order, flux form.  Each flux is a product of midpoint
 * interpolations onto the face of the u control volume:
 *   x faces at cell centers x_{i-1}, x_i:   (I(u))^2
 *   y faces at (xh_i, yh_j), (xh_i, yh_{j+1}):  I_x(v) * I_y(u)
 *   z faces at (xh_i, zh_k), (xh_i, zh_{k+1}):  I_x(w) * I_z(u)
 * and ut += -(dF_x/dx + dF_y/dy + dF_z/dz).
 * ------------------------------------------------------------------------- */
static double advec_u_at(const grid *g, double dxi, double dyi, const double *dzi,
                         const double *u, const double *v, const double *w,
                         int i, int j, int k)
{
    const double uc = u[at(g, i, j, k)];
    const double fx_hi = interp(uc, u[at(g, i + 1, j, k)]);
    const double fx_lo = interp(u[at(g, i - 1, j, k)], uc);
    const double adv_x = (fx_hi * fx_hi - fx_lo * fx_lo) * dxi;

    const double vn = interp(v[at(g, i - 1, j + 1, k)], v[at(g, i, j + 1, k)]);
    const double vs = interp(v[at(g, i - 1, j, k)], v[at(g, i, j, k)]);
    const double un = interp(uc, u[at(g, i, j + 1, k)]);
    const double us = interp(u[at(g, i, j - 1, k)], uc);
    const double adv_y = (vn * un - vs * us) * dyi;

    const double wt = interp(w[at(g, i - 1, j, k + 1)], w[at(g, i, j, k + 1)]);
    const double wb = interp(w[at(g, i - 1, j, k)], w[at(g, i, j, k)]);
    const double ut = interp(uc, u[at(g, i, j, k + 1)]);
    const double ub = interp(u[at(g, i, j, k - 1)], uc);
    const double adv_z = (wt * ut - wb * ub) * dzi[k];

    return -(adv_x + adv_y + adv_z);
}

void ora_advec_u(int itot, int jtot, int ktot, int64_t off, int64_t js, int64_t ks,
                 double dxi, double dyi, const double *dzi,
                 double *ut, const double *u, const double *v, const double *w)
{
    grid g = {itot, jtot, ktot, off, js, ks, 1};
#pragma omp parallel for schedule(static)
    for (int k = 1; k <= ktot; ++k)
        for (int j = 1; j <= jtot; ++j)
            for (int i = 1; i <= itot; ++i)
                ut[at(&g, i, j, k)] += advec_u_at(&g, dxi, dyi, dzi, u, v, w, i, j, k);
}

/* ---------------------------------------------------------------------------
 * diff_uvw: constant-viscosity Laplacian of u, v (cell-center levels) and w
 * (face levels).  For u and v the vertical second derivative takes the
 * gradient at faces zh_k, zh_{k+1} (spacing dzh) and divides by dz_k; for w
 * it takes the gradient at centers z_{k-1}, z_k (spacing dz) and divides by
 * dzh_k.  w is advanced only on faces between the walls (k in [2, ktot]) in
 * wall modes and on all faces k in [1, ktot] when z is periodic.
 * ------------------------------------------------------------------------- */
static double lap_xy(const grid *g, const double *f, int i, int j, int k,
                     double dxi2, double dyi2)
{
    const double c = f[at(g, i, j, k)];
    return (f[at(g, i + 1, j, k)] - 2.0 * c + f[at(g, i - 1, j, k)]) * dxi2
         + (f[at(g, i, j + 1, k)] - 2.0 * c + f[at(g, i, j - 1, k)]) * dyi2;
}

/* Laplacian of u or v at a cell-center level k. */
static double diff_c_at(const grid *g, const double *f, double dxi2, double dyi2,
                        const double *dzi, const double *dzhi, double visc, int i, int j, int k)
{
    const double c = f[at(g, i, j, k)];
    const double fz = ((f[at(g, i, j, k + 1)] - c) * dzhi[k + 1]
                     - (c - f[at(g, i, j, k - 1)]) * dzhi[k]) * dzi[k];
    return visc * (lap_xy(g, f, i, j, k, dxi2, dyi2) + fz);
}

/* Laplacian of w at face level k. */
static double diff_w_at(const grid *g, const double *w, double dxi2, double dyi2,
                        const double *dzi, const double *dzhi, double visc, int i, int j, int k)
{
    const double c = w[at(g, i, j, k)];
    const double fz = ((w[at(g, i, j, k + 1)] - c) * dzi[k]
                     - (c - w[at(g, i, j, k - 1)]) * dzi[k - 1]) * dzhi[k];
    return visc * (lap_xy(g, w, i, j, k, dxi2, dyi2) + fz);
}

void ora_diff_uvw(int itot, int jtot, int ktot, int64_t off, int64_t js, int64_t ks,
                  double dxi, double dyi, const double *dzi, const double *dzhi, double visc,
                  int bc, double *ut, double *vt, double *wt,
                  const double *u, const double *v, const double *w)
{
    grid g = {itot, jtot, ktot, off, js, ks, 1};
    const double dxi2 = dxi * dxi, dyi2 = dyi * dyi;
    const int kw0 = (bc == BC_ZPERIODIC) ? 1 : 2;
#pragma omp parallel for schedule(static)
    for (int k = 1; k <= ktot; ++k)
        for (int j = 1; j <= jtot; ++j)
            for (int i = 1; i <= itot; ++i) {
                const int64_t c = at(&g, i, j, k);
                ut[c] += diff_c_at(&g, u, dxi2, dyi2, dzi, dzhi, visc, i, j, k);
                vt[c] += diff_c_at(&g, v, dxi2, dyi2, dzi, dzhi, visc, i, j, k);
                if (k >= kw0)
                    wt[c] += diff_w_at(&g, w, dxi2, dyi2, dzi, dzhi, visc, i, j, k);
            }
}

/* ---------------------------------------------------------------------------
 * advec_u_2i5: the paper's advection of u is "second order with fifth order
 * interpolation" (Section "Tunable Parameters").  The flux divergence and
 * the interpolation of the advecting velocity to a face are second order
 * (midpoints, as in advec_u above); the advected u is interpolated to the
 * face with the fifth-order upwind-biased formula of Wicker and Skamarock
 * (Mon. Wea. Rev. 130, 2002), written as a sixth-order centered value minus a
 * dissipation term that takes the sign of the advecting velocity U:
 *   face(U; a_-2 .. a_3) = U c6 - |U| d5,
 *   c6 = (37 (a0 + a1) - 8 (a_-1 + a2) + (a_-2 + a3)) / 60,
 *   d5 = (10 (a1 - a0) - 5 (a2 - a_-1) + (a3 - a_-2)) / 60,
 * where the face lies between a0 and a1.  Three ghost cells are needed in x
 * and y.  z has one ghost level, so the order drops near the z boundaries:
 * a face k (between levels k-1 and k) uses fifth order where a_-2 .. a3 lie
 * in [0, ktot+1], else the third-order upwind-biased formula
 *   U c4 - |U| d3,  c4 = (7 (a0 + a1) - (a_-1 + a2)) / 12,
 *                   d3 = (3 (a1 - a0) - (a2 - a_-1)) / 12,
 * where a_-1 .. a2 fit, else the midpoint U (a0 + a1) / 2: faces 1 and
 * ktot+1 are second order, faces 2 and ktot third order, the rest fifth
 * order, in every boundary mode.
 * ------------------------------------------------------------------------- */
static double flux5(double U, double am2, double am1, double a0, double a1, double a2, double a3)
{
    const double c6 = (37.0 * (a0 + a1) - 8.0 * (am1 + a2) + (am2 + a3)) / 60.0;
    const double d5 = (10.0 * (a1 - a0) - 5.0 * (a2 - am1) + (a3 - am2)) / 60.0;
    return U * c6 - fabs(U) * d5;
}

static double flux3(double U, double am1, double a0, double a1, double a2)
{
    const double c4 = (7.0 * (a0 + a1) - (am1 + a2)) / 12.0;
    const double d3 = (3.0 * (a1 - a0) - (a2 - am1)) / 12.0;
    return U * c4 - fabs(U) * d3;
}

/* z flux of u-momentum through face kf of the u control volume at (i, j). */
static double flux_z_2i5(const grid *g, const double *u, const double *w, int i, int j, int kf)
{
    const double W = interp(w[at(g, i - 1, j, kf)], w[at(g, i, j, kf)]);
    if (kf == 1 || kf == g->ktot + 1)
        return W * interp(u[at(g, i, j, kf - 1)], u[at(g, i, j, kf)]);
    if (kf == 2 || kf == g->ktot)
        return flux3(W, u[at(g, i, j, kf - 2)], u[at(g, i, j, kf - 1)], u[at(g, i, j, kf)],
                     u[at(g, i, j, kf + 1)]);
    return flux5(W, u[at(g, i, j, kf - 3)], u[at(g, i, j, kf - 2)], u[at(g, i, j, kf - 1)],
                 u[at(g, i, j, kf)], u[at(g, i, j, kf + 1)], u[at(g, i, j, kf + 2)]);
}

static double advec_u_2i5_at(const grid *g, double dxi, double dyi, const double *dzi,
                             const double *u, const double *v, const double *w,
                             int i, int j, int k)
{
    /* x faces at the cell centers x_i (between u_i and u_i+1) and x_i-1 */
    const double Ue = interp(u[at(g, i, j, k)], u[at(g, i + 1, j, k)]);
    const double Uw = interp(u[at(g, i - 1, j, k)], u[at(g, i, j, k)]);
    const double fe = flux5(Ue, u[at(g, i - 2, j, k)], u[at(g, i - 1, j, k)], u[at(g, i, j, k)],
                            u[at(g, i + 1, j, k)], u[at(g, i + 2, j, k)], u[at(g, i + 3, j, k)]);
    const double fw = flux5(Uw, u[at(g, i - 3, j, k)], u[at(g, i - 2, j, k)], u[at(g, i - 1, j, k)],
                            u[at(g, i, j, k)], u[at(g, i + 1, j, k)], u[at(g, i + 2, j, k)]);
    const double adv_x = (fe - fw) * dxi;

    /* y faces at yh_j+1 (between u_j and u_j+1) and yh_j */
    const double Vn = interp(v[at(g, i - 1, j + 1, k)], v[at(g, i, j + 1, k)]);
    const double Vs = interp(v[at(g, i - 1, j, k)], v[at(g, i, j, k)]);
    const double fn = flux5(Vn, u[at(g, i, j - 2, k)], u[at(g, i, j - 1, k)], u[at(g, i, j, k)],
                            u[at(g, i, j + 1, k)], u[at(g, i, j + 2, k)], u[at(g, i, j + 3, k)]);
    const double fs = flux5(Vs, u[at(g, i, j - 3, k)], u[at(g, i, j - 2, k)], u[at(g, i, j - 1, k)],
                            u[at(g, i, j, k)], u[at(g, i, j + 1, k)], u[at(g, i, j + 2, k)]);
    const double adv_y = (fn - fs) * dyi;

    const double adv_z = (flux_z_2i5(g, u, w, i, j, k + 1) - flux_z_2i5(g, u, w, i, j, k)) * dzi[k];

    return -(adv_x + adv_y + adv_z);
}

void ora_advec_u_2i5(int itot, int jtot, int ktot, int64_t off, int64_t js, int64_t ks,
                     double dxi, double dyi, const double *dzi,
                     double *ut, const double *u, const double *v, const double *w)
{
    grid g = {itot, jtot, ktot, off, js, ks, 3};
#pragma omp parallel for schedule(static)
    for (int k = 1; k <= ktot; ++k)
        for (int j = 1; j <= jtot; ++j)
            for (int i = 1; i <= itot; ++i)
                ut[at(&g, i, j, k)] += advec_u_2i5_at(&g, dxi, dyi, dzi, u, v, w, i, j, k);
}

/* ---------------------------------------------------------------------------
 * diff_smag: the paper's diffusion kernel belongs to "second order
 * Smagorinsky diffusion" (Section "Tunable Parameters"): the divergence of
 * the viscous stress tau_ij = nu (d_j u_i + d_i u_j) with a spatially varying
 * eddy viscosity nu given at cell centers (evisc, one ghost cell).  Second
 * order on the staggered grid:
 *   normal stresses  2 nu d_i u_i  at cell centers, where nu lives;
 *   shear stresses   nu (d_j u_i + d_i u_j) on cell edges, with nu the mean
 *                    of the four cell centers around the edge;
 *   tendency of u_i  = sum_j (tau_ij(upper face) - tau_ij(lower face)) / width.
 * z widths: dz_k for u and v (their faces are w levels, gradients there use
 * dzh), dzh_k for w (its faces are cell centers, gradients use dz).  w is
 * advanced on the same faces as in diff_uvw.
 * ------------------------------------------------------------------------- */
static inline double mean4(double a, double b, double c, double d) { return 0.25 * (a + b + c + d); }

static double smag_u_at(const grid *g, double dxi, double dyi, const double *dzi, const double *dzhi,
                        const double *u, const double *v, const double *w, const double *e,
                        int i, int j, int k)
{
    const double uc = u[at(g, i, j, k)];
    const double tx = (e[at(g, i, j, k)] * (u[at(g, i + 1, j, k)] - uc)
                     - e[at(g, i - 1, j, k)] * (uc - u[at(g, i - 1, j, k)])) * (2.0 * dxi * dxi);
    const double en = mean4(e[at(g, i - 1, j, k)], e[at(g, i, j, k)],
                            e[at(g, i - 1, j + 1, k)], e[at(g, i, j + 1, k)]);
    const double es = mean4(e[at(g, i - 1, j - 1, k)], e[at(g, i, j - 1, k)],
                            e[at(g, i - 1, j, k)], e[at(g, i, j, k)]);
    const double ty = (en * ((u[at(g, i, j + 1, k)] - uc) * dyi
                             + (v[at(g, i, j + 1, k)] - v[at(g, i - 1, j + 1, k)]) * dxi)
                     - es * ((uc - u[at(g, i, j - 1, k)]) * dyi
                             + (v[at(g, i, j, k)] - v[at(g, i - 1, j, k)]) * dxi)) * dyi;
    const double et = mean4(e[at(g, i - 1, j, k)], e[at(g, i, j, k)],
                            e[at(g, i - 1, j, k + 1)], e[at(g, i, j, k + 1)]);
    const double eb = mean4(e[at(g, i - 1, j, k - 1)], e[at(g, i, j, k - 1)],
                            e[at(g, i - 1, j, k)], e[at(g, i, j, k)]);
    const double tz = (et * ((u[at(g, i, j, k + 1)] - uc) * dzhi[k + 1]
                             + (w[at(g, i, j, k + 1)] - w[at(g, i - 1, j, k + 1)]) * dxi)
                     - eb * ((uc - u[at(g, i, j, k - 1)]) * dzhi[k]
                             + (w[at(g, i, j, k)] - w[at(g, i - 1, j, k)]) * dxi)) * dzi[k];
    return tx + ty + tz;
}

static double smag_v_at(const grid *g, double dxi, double dyi, const double *dzi, const double *dzhi,
                        const double *u, const double *v, const double *w, const double *e,
                        int i, int j, int k)
{
    const double vc = v[at(g, i, j, k)];
    const double ee = mean4(e[at(g, i, j - 1, k)], e[at(g, i + 1, j - 1, k)],
                            e[at(g, i, j, k)], e[at(g, i + 1, j, k)]);
    const double ew = mean4(e[at(g, i - 1, j - 1, k)], e[at(g, i, j - 1, k)],
                            e[at(g, i - 1, j, k)], e[at(g, i, j, k)]);
    const double tx = (ee * ((v[at(g, i + 1, j, k)] - vc) * dxi
                             + (u[at(g, i + 1, j, k)] - u[at(g, i + 1, j - 1, k)]) * dyi)
                     - ew * ((vc - v[at(g, i - 1, j, k)]) * dxi
                             + (u[at(g, i, j, k)] - u[at(g, i, j - 1, k)]) * dyi)) * dxi;
    const double ty = (e[at(g, i, j, k)] * (v[at(g, i, j + 1, k)] - vc)
                     - e[at(g, i, j - 1, k)] * (vc - v[at(g, i, j - 1, k)])) * (2.0 * dyi * dyi);
    const double et = mean4(e[at(g, i, j - 1, k)], e[at(g, i, j, k)],
                            e[at(g, i, j - 1, k + 1)], e[at(g, i, j, k + 1)]);
    const double eb = mean4(e[at(g, i, j - 1, k - 1)], e[at(g, i, j, k - 1)],
                            e[at(g, i, j - 1, k)], e[at(g, i, j, k)]);
    const double tz = (et * ((v[at(g, i, j, k + 1)] - vc) * dzhi[k + 1]
                             + (w[at(g, i, j, k + 1)] - w[at(g, i, j - 1, k + 1)]) * dyi)
                     - eb * ((vc - v[at(g, i, j, k - 1)]) * dzhi[k]
                             + (w[at(g, i, j, k)] - w[at(g, i, j - 1, k)]) * dyi)) * dzi[k];
    return tx + ty + tz;
}

static double smag_w_at(const grid *g, double dxi, double dyi, const double *dzi, const double *dzhi,
                        const double *u, const double *v, const double *w, const double *e,
                        int i, int j, int k)
{
    const double wc = w[at(g, i, j, k)];
    const double ee = mean4(e[at(g, i, j, k - 1)], e[at(g, i + 1, j, k - 1)],
                            e[at(g, i, j, k)], e[at(g, i + 1, j, k)]);
    const double ew = mean4(e[at(g, i - 1, j, k - 1)], e[at(g, i, j, k - 1)],
                            e[at(g, i - 1, j, k)], e[at(g, i, j, k)]);
    const double tx = (ee * ((w[at(g, i + 1, j, k)] - wc) * dxi
                             + (u[at(g, i + 1, j, k)] - u[at(g, i + 1, j, k - 1)]) * dzhi[k])
                     - ew * ((wc - w[at(g, i - 1, j, k)]) * dxi
                             + (u[at(g, i, j, k)] - u[at(g, i, j, k - 1)]) * dzhi[k])) * dxi;
    const double en = mean4(e[at(g, i, j, k - 1)], e[at(g, i, j + 1, k - 1)],
                            e[at(g, i, j, k)], e[at(g, i, j + 1, k)]);
    const double es = mean4(e[at(g, i, j - 1, k - 1)], e[at(g, i, j, k - 1)],
                            e[at(g, i, j - 1, k)], e[at(g, i, j, k)]);
    const double ty = (en * ((w[at(g, i, j + 1, k)] - wc) * dyi
                             + (v[at(g, i, j + 1, k)] - v[at(g, i, j + 1, k - 1)]) * dzhi[k])
                     - es * ((wc - w[at(g, i, j - 1, k)]) * dyi
                             + (v[at(g, i, j, k)] - v[at(g, i, j, k - 1)]) * dzhi[k])) * dyi;
    const double tz = (e[at(g, i, j, k)] * (w[at(g, i, j, k + 1)] - wc) * dzi[k]
                     - e[at(g, i, j, k - 1)] * (wc - w[at(g, i, j, k - 1)]) * dzi[k - 1]) * (2.0 * dzhi[k]);
    return tx + ty + tz;
}

void ora_diff_smag(int itot, int jtot, int ktot, int64_t off, int64_t js, int64_t ks,
                   double dxi, double dyi, const double *dzi, const double *dzhi,
                   int bc, double *ut, double *vt, double *wt,
                   const double *u, const double *v, const double *w, const double *evisc)
{
    grid g = {itot, jtot, ktot, off, js, ks, 1};
    const int kw0 = (bc == BC_ZPERIODIC) ? 1 : 2;
#pragma omp parallel for schedule(static)
    for (int k = 1; k <= ktot; ++k)
        for (int j = 1; j <= jtot; ++j)
            for (int i = 1; i <= itot; ++i) {
                const int64_t c = at(&g, i, j, k);
                ut[c] += smag_u_at(&g, dxi, dyi, dzi, dzhi, u, v, w, evisc, i, j, k);
                vt[c] += smag_v_at(&g, dxi, dyi, dzi, dzhi, u, v, w, evisc, i, j, k);
                if (k >= kw0)
                    wt[c] += smag_w_at(&g, dxi, dyi, dzi, dzhi, u, v, w, evisc, i, j, k);
            }
}

/* Single-point values of the two schemes above: out[0] = advec_u_2i5 (needs
 * three ghost cells in x and y), out[1..3] = diff_smag of u, v, w (w's entry
 * is 0 where w is not advanced). */
void ora_point_les(int itot, int jtot, int ktot, int64_t off, int64_t js, int64_t ks, int bc,
                   double dxi, double dyi, const double *dzi, const double *dzhi,
                   const double *u, const double *v, const double *w, const double *evisc,
                   int i, int j, int k, double *out)
{
    grid g = {itot, jtot, ktot, off, js, ks, 3};
    const int kw0 = (bc == BC_ZPERIODIC) ? 1 : 2;
    out[0] = advec_u_2i5_at(&g, dxi, dyi, dzi, u, v, w, i, j, k);
    out[1] = smag_u_at(&g, dxi, dyi, dzi, dzhi, u, v, w, evisc, i, j, k);
    out[2] = smag_v_at(&g, dxi, dyi, dzi, dzhi, u, v, w, evisc, i, j, k);
    out[3] = (k >= kw0) ? smag_w_at(&g, dxi, dyi, dzi, dzhi, u, v, w, evisc, i, j, k) : 0.0;
}

/* ---------------------------------------------------------------------------
 * One forward-Euler time step of the two processes (the paper names no time
 * integrator; this library uses forward Euler):
 *   tendencies = 0; ghosts; ut += advec_u; (ut, vt, wt) += diff_uvw;
 *   f += dt * ft on each field's computed range; ghosts.
 * ------------------------------------------------------------------------- */
void ora_euler(int itot, int jtot, int ktot, int64_t off, int64_t js, int64_t ks, int bc,
               double dt, double *u, double *v, double *w,
               const double *ut, const double *vt, const double *wt)
{
    grid g = {itot, jtot, ktot, off, js, ks, 1};
    const int kw0 = (bc == BC_ZPERIODIC) ? 1 : 2;
    for (int k = 1; k <= ktot; ++k)
        for (int j = 1; j <= jtot; ++j)
            for (int i = 1; i <= itot; ++i) {
                const int64_t c = at(&g, i, j, k);
                u[c] += dt * ut[c];
                v[c] += dt * vt[c];
                if (k >= kw0) w[c] += dt * wt[c];
            }
    ora_fill_ghosts(itot, jtot, ktot, off, js, ks, bc, u, v, w);
}

void ora_step(int itot, int jtot, int ktot, int64_t off, int64_t js, int64_t ks, int bc,
              double dxi, double dyi, const double *dzi, const double *dzhi, double visc,
              double dt, int64_t alloc, double *u, double *v, double *w,
              double *ut, double *vt, double *wt)
{
    memset(ut, 0, sizeof(double) * (size_t)alloc);
    memset(vt, 0, sizeof(double) * (size_t)alloc);
    memset(wt, 0, sizeof(double) * (size_t)alloc);
    ora_fill_ghosts(itot, jtot, ktot, off, js, ks, bc, u, v, w);
    ora_advec_u(itot, jtot, ktot, off, js, ks, dxi, dyi, dzi, ut, u, v, w);
    ora_diff_uvw(itot, jtot, ktot, off, js, ks, dxi, dyi, dzi, dzhi, visc, bc,
                 ut, vt, wt, u, v, w);
    ora_euler(itot, jtot, ktot, off, js, ks, bc, dt, u, v, w, ut, vt, wt);
}

/* ---------------------------------------------------------------------------
 * FP64 reductions.
 * Conservation: out[0] = sum ut*dz_k, out[1] = sum vt*dz_k over the interior,
 * out[2] = sum wt*dzh_k over w's computed faces; dz_k = 1/dzi[k] and
 * dzh_k = 1/dzhi[k] (dx*dy is a common factor and left out).
 * Checksums of one field: sum f, sum f^2, max |f| over the interior.
 * Sequential sums in k, j, i order.
 * ------------------------------------------------------------------------- */
void ora_conservation(int itot, int jtot, int ktot, int64_t off, int64_t js, int64_t ks,
                      int bc, const double *dzi, const double *dzhi,
                      const double *ut, const double *vt, const double *wt, double *out)
{
    grid g = {itot, jtot, ktot, off, js, ks, 1};
    const int kw0 = (bc == BC_ZPERIODIC) ? 1 : 2;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int k = 1; k <= ktot; ++k)
        for (int j = 1; j <= jtot; ++j)
            for (int i = 1; i <= itot; ++i) {
                const int64_t c = at(&g, i, j, k);
                s0 += ut[c] * (1.0 / dzi[k]);
                s1 += vt[c] * (1.0 / dzi[k]);
                if (k >= kw0) s2 += wt[c] * (1.0 / dzhi[k]);
            }
    out[0] = s0;
    out[1] = s1;
    out[2] = s2;
}

void ora_checksums(int itot, int jtot, int ktot, int64_t off, int64_t js, int64_t ks,
                   const double *f, double *out)
{
    grid g = {itot, jtot, ktot, off, js, ks, 1};
    double s = 0.0, s2 = 0.0, m = 0.0;
    for (int k = 1; k <= ktot; ++k)
        for (int j = 1; j <= jtot; ++j)
            for (int i = 1; i <= itot; ++i) {
                const double x = f[at(&g, i, j, k)];
                s += x;
                s2 += x * x;
                if (fabs(x) > m) m = fabs(x);
            }
    out[0] = s;
    out[1] = s2;
    out[2] = m;
}

/* Single-point tendencies (for sampled checks of grids too large to sweep on
 * the host): the same definitions as above evaluated at one (i, j, k).
 * out[0..2] = advec_u of u, and diff_uvw of u, v, w (w's entry is 0 where w
 * is not advanced). */
void ora_point(int itot, int jtot, int ktot, int64_t off, int64_t js, int64_t ks, int bc,
               double dxi, double dyi, const double *dzi, const double *dzhi, double visc,
               const double *u, const double *v, const double *w, int i, int j, int k,
               double *out)
{
    grid g = {itot, jtot, ktot, off, js, ks, 1};
    const double dxi2 = dxi * dxi, dyi2 = dyi * dyi;
    const int kw0 = (bc == BC_ZPERIODIC) ? 1 : 2;
    out[0] = advec_u_at(&g, dxi, dyi, dzi, u, v, w, i, j, k);
    out[1] = diff_c_at(&g, u, dxi2, dyi2, dzi, dzhi, visc, i, j, k);
    out[2] = diff_c_at(&g, v, dxi2, dyi2, dzi, dzhi, visc, i, j, k);
    out[3] = (k >= kw0) ? diff_w_at(&g, w, dxi2, dyi2, dzi, dzhi, visc, i, j, k) : 0.0;
}

/* Number of OpenMP threads the parallel loops above use. */
/* ora_set_threads(n) sets it (n >= 1); the arithmetic of every loop is the
 * same for any thread count (each output cell is written by one iteration). */
#ifdef _OPENMP
#include <omp.h>
int ora_threads(void) { return omp_get_max_threads(); }
void ora_set_threads(int n) { if (n >= 1) omp_set_num_threads(n); }
#else
int ora_threads(void) { return 1; }
void ora_set_threads(int n) { (void)n; }
#endif
