// Fused time step: one kernel reads u, v, w (ghost-filled) once and writes
// the next state into a second set of fields, ghost cells included:
//   u' = u + dt * ((0 + advec_u) + diff_u),  v' = v + dt * (0 + diff_v),
//   w' = w + dt * (0 + diff_w) on w's computed range,
// then every updated value is also written to the ghost cells it is the
// source of.  The operations and their order are those of the separate
// path (tendencies zeroed, advec_u accumulated, diff_uvw accumulated,
// forward Euler, ghost refill), so the result is bitwise identical to it
// while HBM traffic drops from 26 to 6 values per point.
//
// Tile and data flow as the LDS-staged z-march (stencil_zl.hpp): a wave per
// row, VX points per lane, a 4- or 6-slot register ring per field in z, LDS
// rows for the y neighbours, shuffles for the x neighbours.  The x edge
// values are prefetched as far ahead as the field ring because the w stencil
// of advec_u needs them at level k+1.  The halo rows are prefetched one level
// ahead, or (FUSE_HALO3) as far ahead as the ring: a halo row is a
// neighbouring tile's own row, and requesting it at about the time that
// tile does lets L2 serve one of the two requests.
#pragma once

#include "stencil_zl.hpp"

namespace kl {

// Store a VX-vector of new values at (i0.., j, k) and at its x images (the
// ghost columns 0 and itot+1 of the same row, periodic x).
template <typename T, int VX, int NT>
__device__ __forceinline__ void put_with_x_images(T *f, const StencilArgs<T> &a, int i0, int j, int k,
                                                  const T (&val)[VX])
{
    const int64_t base = a.off + (int64_t)j * a.js + (int64_t)k * a.ks;
    tstore<NT, T, VX>(f + base + i0, val);
    if (i0 == 1) f[base + a.itot + 1] = val[0];
    if (i0 + VX - 1 == a.itot) f[base] = val[VX - 1];
}

// Store a VX-vector of new values at (i0.., j, k) of field `fld` and at all
// ghost cells whose source it is (periodic x and y; z by the boundary rule).
// The point itself and its x images are stored on every row; the y and z
// images exist only on the first and last rows and levels, so the wave takes
// a uniform branch around them everywhere else and spends no instructions on
// their addresses and values.
template <typename T, int VX, int NT>
__device__ __forceinline__ void put_with_images(T *f, const StencilArgs<T> &a, int fld, int i0, int j, int k,
                                                const T (&val)[VX])
{
    const int kt = a.ktot;
    const bool x_lo = i0 == 1, x_hi = i0 + VX - 1 == a.itot;
    {
        const int64_t base = a.off + (int64_t)j * a.js + (int64_t)k * a.ks;
        tstore<NT, T, VX>(f + base + i0, val);
        if (x_lo) f[base + a.itot + 1] = val[0];
        if (x_hi) f[base] = val[VX - 1];
    }
    if (!(j == 1 || j == a.jtot || k <= 2 || k == kt)) return;
    int zk[4], zs[4], nz = 1;
    zk[0] = k;
    zs[0] = 1;
    if (a.bc == KL_BC_ZPERIODIC) {
        if (k == kt) { zk[nz] = 0; zs[nz++] = 1; }
        if (k == 1) { zk[nz] = kt + 1; zs[nz++] = 1; }
    } else if (fld < 2) {
        if (k == 1) { zk[nz] = 0; zs[nz++] = 1; }
        if (k == kt) { zk[nz] = kt + 1; zs[nz++] = 1; }
    } else if (a.bc == KL_BC_ZWALL_ZEROGRAD) {
        if (k == 2) { zk[nz] = 0; zs[nz++] = 1; zk[nz] = 1; zs[nz++] = 1; }
        if (k == kt) { zk[nz] = kt + 1; zs[nz++] = 1; }
    } else {
        if (k == 2) { zk[nz] = 0; zs[nz++] = -1; zk[nz] = 1; zs[nz++] = 0; }
        if (k == kt) { zk[nz] = kt + 1; zs[nz++] = 0; }
    }
    int yj[3], ny = 1;
    yj[0] = j;
    if (j == a.jtot) yj[ny++] = 0;
    if (j == 1) yj[ny++] = a.jtot + 1;
    // fixed trip counts (at most 4 z images and 3 y images), unrolled: the
    // number of stores a wave issues is then known on every path, which
    // keeps the compiler's waits for earlier loads exact
#pragma unroll
    for (int z = 0; z < 4; ++z) {
        if (z < nz) {
            T v[VX];
#pragma unroll
            for (int n = 0; n < VX; ++n) v[n] = zs[z] == 0 ? T(0) : (zs[z] < 0 ? -val[n] : val[n]);
#pragma unroll
            for (int y = 0; y < 3; ++y) {
                if (y < ny && (z > 0 || y > 0)) {
                    const int64_t base = a.off + (int64_t)yj[y] * a.js + (int64_t)zk[z] * a.ks;
                    vstore<T, VX>(f + base + i0, v);
                    if (x_lo) f[base + a.itot + 1] = v[0];
                    if (x_hi) f[base] = v[VX - 1];
                }
            }
        }
    }
}

// MODE: FUSE_STEP or FUSE_PAIR, plus FUSE_HALO3 to load the halo rows as far
// ahead as the field ring (three levels for the 4-slot ring, two for the
// 6-slot one) instead of one, plus FUSE_RING6 for a 6-slot field ring (own
// rows loaded five levels ahead instead of three), plus FUSE_NOYZ (step
// only): the kernel stores the new values and their x images only, and the
// launcher refills the y and z ghost cells afterwards with the ghost fill's
// copies (the same values: every image is a copy, a negation or a zero of a
// new value), which keeps the slow path of the first and last rows and
// levels out of the level loop.
enum { FUSE_STEP = 0, FUSE_PAIR = 1, FUSE_HALO3 = 2, FUSE_RING6 = 4, FUSE_NOYZ = 8 };

template <typename T, int VX, int BY, int KB, int NT, int MODE = FUSE_STEP>
__device__ __forceinline__ void step_zl_tile(const StencilArgs<T> &a, int tx, int ty, int tz)
{
    static_assert(BY >= 2, "two halo rows need two waves");
    constexpr int TX = 64 * VX;
    typedef T RowT[TX];
    // LDS rows 0..BY+1 hold the tile's rows and its two halo rows; row BY+2
    // and the 64 trailing v-edge slots take the writes of waves and lanes
    // that have nothing to contribute, so every prefetched register is
    // consumed on every path (see the level loop)
    __shared__ __align__(16) RowT sh[2][3][BY + 3];
    __shared__ T shvl[2][BY + 2 + 64];  // v left of the segment, per LDS row
    __syncthreads();

    const ZlTile<VX, BY, KB> t(a.itot, a.jtot, a.ktot, tx, ty, tz);
    const int64_t js = a.js, ks = a.ks;
    // every load of the level loop is unconditional and inside the field
    // (clamped lane and row, a re-read of the own row for waves without a
    // halo row, level k1 for the last levels' prefetch, one scalar load per
    // field for both x edges), as in the diff_uvw tile
    const int lane_c = min(t.lane, t.nlanes - 1);
    const int64_t row_c = a.off + t.i0w + (int64_t)min(t.j0 + t.r, a.jtot) * js;
    const int64_t c_own = row_c + lane_c * VX;
    const bool x_is_top = t.xrow_g >= 0 && t.xrow_l > 0;
    const int64_t xrow0 = a.off + t.i0w + (int64_t)max(t.xrow_g, 0) * js;
    const int64_t c_x = t.xrow_g >= 0 ? xrow0 + lane_c * VX : c_own;
    const int le = max(t.nlanes - 1, 1);
    const int64_t c_e = t.lane == 0 ? row_c + t.xl : (t.lane == le ? row_c + t.xr : c_own);
    const int64_t c_xv = x_is_top && t.lane == 0 ? xrow0 + t.xl : c_own;  // v left of the top halo row
    const bool ld_own = t.own && t.lane_on;
    const T *F[3] = {a.u, a.v, a.w};
    T *O[3] = {a.ut, a.vt, a.wt};  // output fields (FUSE_STEP) or tendencies (FUSE_PAIR)
    const T dxi = a.dxi, dyi = a.dyi, dxi2 = a.dxi * a.dxi, dyi2 = a.dyi * a.dyi, visc = a.visc, dt = a.dt;
    const int kw0 = a.kw0;
    const int j = t.j0 + t.r;

    constexpr bool PAIR = (MODE & FUSE_PAIR) != 0;
    constexpr int RS = (MODE & FUSE_RING6) ? 6 : 4;                 // field ring slots
    constexpr int HL = (MODE & FUSE_HALO3) ? (RS == 4 ? 3 : 2) : 1;  // halo rows are loaded HL levels ahead
    constexpr int HS = HL + 1;
    static_assert(RS % HS == 0 && RS % 2 == 0, "ring slots are indexed by the unrolled level");
    T R[RS][3][VX];       // field ring: slot s % RS holds level kk+s
    T E[RS][3];           // x edge values (left in lane 0, right in lane le), same ring
    T X[HS][3][VX];       // halo row (or a re-read of the own row), slot (level - k0) % HS
    T XVL[HS];            // v left edge of the top halo row (lane 0)
    T Q[PAIR ? 2 : 1][3][VX];  // tendencies of levels k, k+1 by parity (FUSE_PAIR)

    const int k0 = t.k0, k1 = t.k1;
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        vload<T, VX>(R[RS - 1][f], F[f] + c_own + (int64_t)(k0 - 1) * ks);
#pragma unroll
        for (int h = 0; h < RS - 1; ++h) vload<T, VX>(R[h][f], F[f] + c_own + (int64_t)min(k0 + h, k1) * ks);
#pragma unroll
        for (int h = 0; h < HL; ++h) vload<T, VX>(X[h][f], F[f] + c_x + (int64_t)min(k0 + h, k1) * ks);
#pragma unroll
        for (int q = 0; q < RS - 1; ++q) E[q][f] = F[f][c_e + (int64_t)min(k0 + q, k1) * ks];
        if constexpr (PAIR) tload<NT, T, VX>(Q[0][f], O[f] + c_own + (int64_t)k0 * ks);
    }
#pragma unroll
    for (int h = 0; h < HL; ++h) XVL[h] = a.v[c_xv + (int64_t)min(k0 + h, k1) * ks];

    vm_drain();
    for (int kk = k0;; kk += RS) {
#pragma unroll
        for (int s = 0; s < RS; ++s) {
            const int k = kk + s;
            if (k >= k1) return;
            const int p = s & 1, q = p ^ 1;
            T(&b)[3][VX] = R[(s + RS - 1) % RS];  // level k-1; refilled with k+RS-1 after use
            T(&c)[3][VX] = R[s % RS];
            T(&tp)[3][VX] = R[(s + 1) % RS];
            // halo row of level k+HL (clamped to k1 <= ktot+1) into the slot
            // of level k-1
            const int xs = s % HS, xn = (s + HL) % HS;
            const int64_t lh = (int64_t)min(k + HL, k1) * ks;
#pragma unroll
            for (int f = 0; f < 3; ++f) vload<T, VX>(X[xn][f], F[f] + c_x + lh);
            XVL[xn] = a.v[c_xv + lh];
            if constexpr (PAIR) {
#pragma unroll
                for (int f = 0; f < 3; ++f) tload<NT, T, VX>(Q[q][f], O[f] + c_own + (int64_t)(k + 1) * ks);
            }
            // level-k rows into LDS.  Every value loaded ahead (ring, halo row,
            // edges, tendencies) is consumed on every path through the level:
            // the halo row of a wave without one goes to the spare LDS row,
            // and all lanes compute (clamped loads keep the inputs of idle
            // lanes and rows valid) while only the stores are predicated.  A
            // load whose register is left unconsumed on some path makes the
            // compiler wait for all outstanding memory operations at the next
            // reuse of that register, which would undo the prefetch.
            const int xrow = t.xrow_l >= 0 ? t.xrow_l : BY + 2;
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                if (t.own) vstore<T, VX>(&sh[p][f][t.r + 1][t.lane * VX], c[f]);
                vstore<T, VX>(&sh[p][f][xrow][t.lane * VX], X[xs][f]);
            }
            if (t.own && t.lane == 0) shvl[p][t.r + 1] = E[s % RS][1];
            shvl[p][x_is_top && t.lane == 0 ? t.xrow_l : BY + 2 + t.lane] = XVL[xs];
            __syncthreads();
            T nn[3][VX], ss[3][VX], left[3], right[3];
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                vload<T, VX>(nn[f], &sh[p][f][t.r + 2][t.lane * VX]);
                vload<T, VX>(ss[f], &sh[p][f][t.r][t.lane * VX]);
                left[f] = shfl_up1<T>(c[f][VX - 1]);
                right[f] = shfl_down1<T>(c[f][0]);
                T er = E[s % RS][f];
                if (t.nlanes == 1) er = __shfl(er, 1, 64);
                if (t.lane == 0) left[f] = E[s % RS][f];
                if (t.lane == t.nlanes - 1) right[f] = er;
            }
            T vnleft = shfl_up1<T>(nn[1][VX - 1]);
            T wtleft = shfl_up1<T>(tp[2][VX - 1]);
            if (t.lane == 0) {
                vnleft = shvl[p][t.r + 2];
                wtleft = E[(s + 1) % RS][2];
            }
            {
                const T dzik = kload(a.dzi, k), dzikm1 = kload(a.dzi, k - 1), dzhik = kload(a.dzhi, k),
                        dzhik1 = kload(a.dzhi, k + 1);
                T nu[VX], nv[VX], nw[VX];
#pragma unroll
                for (int n = 0; n < VX; ++n) {
                    const T uw = n == 0 ? left[0] : c[0][n - 1];
                    const T ue = n == VX - 1 ? right[0] : c[0][n + 1];
                    const T vw = n == 0 ? left[1] : c[1][n - 1];
                    const T ve = n == VX - 1 ? right[1] : c[1][n + 1];
                    const T ww = n == 0 ? left[2] : c[2][n - 1];
                    const T we = n == VX - 1 ? right[2] : c[2][n + 1];
                    const T v_nw = n == 0 ? vnleft : nn[1][n - 1];
                    const T w_tw = n == 0 ? wtleft : tp[2][n - 1];
                    const T adv = advec_u_point<T>(c[0][n], ue, uw, nn[0][n], ss[0][n], tp[0][n], b[0][n], vw,
                                                   c[1][n], v_nw, nn[1][n], ww, c[2][n], w_tw, tp[2][n], dxi,
                                                   dyi, dzik);
                    const T du = diff_c_point<T>(c[0][n], ue, uw, nn[0][n], ss[0][n], tp[0][n], b[0][n], dxi2,
                                                 dyi2, dzik, dzhik1, dzhik, visc);
                    const T dv = diff_c_point<T>(c[1][n], ve, vw, nn[1][n], ss[1][n], tp[1][n], b[1][n], dxi2,
                                                 dyi2, dzik, dzhik1, dzhik, visc);
                    if constexpr (PAIR) {
                        nu[n] = (Q[p][0][n] + adv) + du;
                        nv[n] = Q[p][1][n] + dv;
                    } else {
                        const T tu = (T(0) + adv) + du;
                        const T tv = T(0) + dv;
                        nu[n] = euler_value<T>(c[0][n], dt, tu);
                        nv[n] = euler_value<T>(c[1][n], dt, tv);
                    }
                    // w's value below its first computed level (k < kw0) is
                    // formed but not stored
                    const T dw = diff_w_point<T>(c[2][n], we, ww, nn[2][n], ss[2][n], tp[2][n], b[2][n], dxi2,
                                                 dyi2, dzik, dzikm1, dzhik, visc);
                    if constexpr (PAIR)
                        nw[n] = Q[p][2][n] + dw;
                    else
                        nw[n] = euler_value<T>(c[2][n], dt, T(0) + dw);
                }
                if constexpr (PAIR) {
#pragma unroll
                    for (int f = 0; f < 3; ++f) settle(Q[p][f]);
                }
                if (ld_own) {
                    if constexpr (PAIR) {
                        const int64_t o = c_own + (int64_t)k * ks;
                        tstore<NT, T, VX>(O[0] + o, nu);
                        tstore<NT, T, VX>(O[1] + o, nv);
                        if (k >= kw0) tstore<NT, T, VX>(O[2] + o, nw);
                    } else {
                        if constexpr ((MODE & FUSE_NOYZ) != 0) {
                            put_with_x_images<T, VX, NT>(O[0], a, t.i0, j, k, nu);
                            put_with_x_images<T, VX, NT>(O[1], a, t.i0, j, k, nv);
                            if (k >= kw0) put_with_x_images<T, VX, NT>(O[2], a, t.i0, j, k, nw);
                        } else {
                            put_with_images<T, VX, NT>(O[0], a, 0, t.i0, j, k, nu);
                            put_with_images<T, VX, NT>(O[1], a, 1, t.i0, j, k, nv);
                            if (k >= kw0) put_with_images<T, VX, NT>(O[2], a, 2, t.i0, j, k, nw);
                        }
                    }
                }
            }
            // level k-1 is no longer needed: its slot takes level k+RS-1 (clamped
            // to k1 near the end of the tile, where it is not used)
            const int64_t l3 = (int64_t)min(k + RS - 1, k1) * ks;
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                fload<NT, T, VX>(b[f], F[f] + c_own + l3);
                E[(s + RS - 1) % RS][f] = F[f][c_e + l3];
            }
        }
    }
}

template <typename T, int VX, int BY, int KB, int XCD, int NT = 0, int WPE = 1, int MODE = FUSE_STEP>
__global__ __launch_bounds__(64 * BY, WPE) void step_zl(StencilArgs<T> a)
{
    int tx, ty, tz;
    tile_of<64, BY, XCD>(a.nbx, a.nby, a.nbz, tx, ty, tz);
    step_zl_tile<T, VX, BY, KB, NT, MODE>(a, tx, ty, tz);
}

template <typename T, int VX, int BY, int KB, int NT = 0, int WPE = 1, int MODE = FUSE_STEP>
__global__ __launch_bounds__(64 * BY, WPE) void step_zl_batch(const StencilArgs<T> *__restrict__ grids,
                                                             const int4 *__restrict__ tiles, int ntiles,
                                                             int *queue)
{
    for (int n = next_tile(queue, -1); n < ntiles; n = next_tile(queue, n)) {
        const int4 tl = tiles[n];
        const StencilArgs<T> a = global_args(grids[tl.x]);
        step_zl_tile<T, VX, BY, KB, NT, MODE>(a, tl.y, tl.z, tl.w);
    }
    walk_done(queue);
}

// Default configuration of the fused advec_u + diff_uvw pass: one thread per
// point, 256 threads along x (the two default kernels' arithmetic, in their
// order, at one point).
template <typename T>
__global__ __launch_bounds__(256) void advec_diff_plain(StencilArgs<T> a)
{
    unsigned b = blockIdx.x;
    const int bx = b % a.nbx;
    b /= a.nbx;
    const int j = 1 + (int)(b % a.jtot);
    const int k = 1 + (int)(b / a.jtot);
    const int i = 1 + bx * 256 + (int)threadIdx.x;
    if (i > a.itot) return;
    const int64_t c = a.off + i + j * a.js + (int64_t)k * a.ks;
    const int64_t js = a.js, ks = a.ks;
    const T dxi2 = a.dxi * a.dxi, dyi2 = a.dyi * a.dyi;
    const T dzik = a.dzi[k], dzhik = a.dzhi[k], dzhik1 = a.dzhi[k + 1];
    const T *u = a.u, *v = a.v, *w = a.w;
    const T adv = advec_u_point<T>(u[c], u[c + 1], u[c - 1], u[c + js], u[c - js], u[c + ks], u[c - ks],
                                   v[c - 1], v[c], v[c - 1 + js], v[c + js],
                                   w[c - 1], w[c], w[c - 1 + ks], w[c + ks],
                                   a.dxi, a.dyi, dzik);
    const T du = diff_c_point<T>(u[c], u[c + 1], u[c - 1], u[c + js], u[c - js], u[c + ks], u[c - ks], dxi2,
                                 dyi2, dzik, dzhik1, dzhik, a.visc);
    a.ut[c] = (a.ut[c] + adv) + du;
    a.vt[c] = a.vt[c] + diff_c_point<T>(v[c], v[c + 1], v[c - 1], v[c + js], v[c - js], v[c + ks],
                                        v[c - ks], dxi2, dyi2, dzik, dzhik1, dzhik, a.visc);
    if (k >= a.kw0)
        a.wt[c] = a.wt[c] + diff_w_point<T>(w[c], w[c + 1], w[c - 1], w[c + js], w[c - js], w[c + ks],
                                            w[c - ks], dxi2, dyi2, dzik, a.dzi[k - 1], dzhik, a.visc);
}

}  // namespace kl
