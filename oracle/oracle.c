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
 * grid with one ghost cell per side.  Each function below writes that
 * definition out point by point, in the order of the formula, with no
 * blocking or fusion.
 *
 * Layout: element (i, j, k) of every field is p[off + i + j*js + k*ks],
 * i in [0, itot+1] (interior [1, itot]), likewise j and k.
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
} grid;

static inline int64_t at(const grid *g, int i, int j, int k)
{
    return g->off + (int64_t)i + (int64_t)j * g->js + (int64_t)k * g->ks;
}

static inline double interp(double a, double b) { return 0.5 * (a + b); }

/* ---------------------------------------------------------------------------
 * Ghost cells.  Periodic in x, then periodic in y over whole rows (so the
 * x-ghost columns are carried into the y-ghost rows), then the z rule over
 * whole planes (so edges and corners are carried too).
 * ------------------------------------------------------------------------- */
static void fill_xy(const grid *g, double *f)
{
    for (int k = 1; k <= g->ktot; ++k)
        for (int j = 1; j <= g->jtot; ++j) {
            f[at(g, 0, j, k)] = f[at(g, g->itot, j, k)];
            f[at(g, g->itot + 1, j, k)] = f[at(g, 1, j, k)];
        }
    for (int k = 1; k <= g->ktot; ++k)
        for (int i = 0; i <= g->itot + 1; ++i) {
            f[at(g, i, 0, k)] = f[at(g, i, g->jtot, k)];
            f[at(g, i, g->jtot + 1, k)] = f[at(g, i, 1, k)];
        }
}

static void copy_plane(const grid *g, double *f, int kdst, int ksrc, double sign)
{
    for (int j = 0; j <= g->jtot + 1; ++j)
        for (int i = 0; i <= g->itot + 1; ++i)
            f[at(g, i, j, kdst)] = sign * f[at(g, i, j, ksrc)];
}

static void set_plane(const grid *g, double *f, int kdst, double value)
{
    for (int j = 0; j <= g->jtot + 1; ++j)
        for (int i = 0; i <= g->itot + 1; ++i)
            f[at(g, i, j, kdst)] = value;
}

void ora_fill_ghosts(int itot, int jtot, int ktot, int64_t off, int64_t js, int64_t ks,
                     int bc, double *u, double *v, double *w)
{
    grid g = {itot, jtot, ktot, off, js, ks};
    double *f3[3] = {u, v, w};
    for (int n = 0; n < 3; ++n) fill_xy(&g, f3[n]);
    const int kt = ktot;
    if (bc == BC_ZPERIODIC) {
        for (int n = 0; n < 3; ++n) {
            copy_plane(&g, f3[n], 0, kt, 1.0);
            copy_plane(&g, f3[n], kt + 1, 1, 1.0);
        }
        return;
    }
    /* u and v: zero gradient across both walls (free slip). */
    for (int n = 0; n < 2; ++n) {
        copy_plane(&g, f3[n], 0, 1, 1.0);
        copy_plane(&g, f3[n], kt + 1, kt, 1.0);
    }
    /* w lives on the faces; face 1 is the bottom wall, face kt+1 the top. */
    if (bc == BC_ZWALL_ZEROGRAD) {
        copy_plane(&g, w, 1, 2, 1.0);
        copy_plane(&g, w, kt + 1, kt, 1.0);
        copy_plane(&g, w, 0, 2, 1.0);
    } else {
        set_plane(&g, w, 1, 0.0);
        set_plane(&g, w, kt + 1, 0.0);
        copy_plane(&g, w, 0, 2, -1.0);
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
    grid g = {itot, jtot, ktot, off, js, ks};
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
    grid g = {itot, jtot, ktot, off, js, ks};
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
 * One forward-Euler time step of the two processes (the paper names no time
 * integrator; this library uses forward Euler):
 *   tendencies = 0; ghosts; ut += advec_u; (ut, vt, wt) += diff_uvw;
 *   f += dt * ft on each field's computed range; ghosts.
 * ------------------------------------------------------------------------- */
void ora_euler(int itot, int jtot, int ktot, int64_t off, int64_t js, int64_t ks, int bc,
               double dt, double *u, double *v, double *w,
               const double *ut, const double *vt, const double *wt)
{
    grid g = {itot, jtot, ktot, off, js, ks};
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
    grid g = {itot, jtot, ktot, off, js, ks};
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
    grid g = {itot, jtot, ktot, off, js, ks};
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
    grid g = {itot, jtot, ktot, off, js, ks};
    const double dxi2 = dxi * dxi, dyi2 = dyi * dyi;
    const int kw0 = (bc == BC_ZPERIODIC) ? 1 : 2;
    out[0] = advec_u_at(&g, dxi, dyi, dzi, u, v, w, i, j, k);
    out[1] = diff_c_at(&g, u, dxi2, dyi2, dzi, dzhi, visc, i, j, k);
    out[2] = diff_c_at(&g, v, dxi2, dyi2, dzi, dzhi, visc, i, j, k);
    out[3] = (k >= kw0) ? diff_w_at(&g, w, dxi2, dyi2, dzi, dzhi, visc, i, j, k) : 0.0;
}

/* Number of OpenMP threads the parallel loops above use. */
#ifdef _OPENMP
#include <omp.h>
int ora_threads(void) { return omp_get_max_threads(); }
#else
int ora_threads(void) { return 1; }
#endif
