// LDS-staged z-marching configuration of advec_u_2i5.
//
// Workgroup = 64 x BY threads: wave r owns row j0 + r of a tile 64*VX wide
// in x and BY rows in y, each lane VX consecutive points; the tile walks the
// levels [k0, k0 + KB).  Per level k:
//   * every wave writes its row of u (level k, from its register window) and
//     of v into double-buffered LDS planes: u with three halo rows and
//     columns on each side ((BY+6) x (TX+6)), v with one halo row above and
//     one column to the left ((BY+1) x (TX+1)); the six u halo rows and the
//     v halo row are loaded by the waves in turn, the halo columns by the
//     edge lanes; one barrier per level;
//   * x faces: each lane reads VX+6 values of its LDS row and evaluates the
//     VX+1 faces around its points once (a face is shared by two points);
//   * y faces: two per point, from the seven LDS rows of its column;
//   * z faces: the u column lives in a six-level register window (levels
//     k-2 .. k+3, level k+4 loaded during level k); the lower face's flux is
//     the upper face's flux of the level below, carried over; the advecting
//     w of the left neighbour comes from the neighbouring lane by a shuffle.
// Every global load is issued one level ahead, except ut, which is loaded at
// the start of its own level and used at its end.  The x halo columns beyond
// the ends of a row are read from their periodic images in the row's
// interior (x is periodic in every mode), so no line of x ghost cells is
// fetched.  The per-face and per-point
// arithmetic is the shared one of stencil_les.hpp with the same operands, so
// results equal the default configuration's bitwise.
#pragma once

#include <type_traits>

#include "stencil_les.hpp"
#include "stencil_zl.hpp"

namespace kl {

// Level l of a column at address p + l*ks into d (VX values), or zeros
// outside [0, ktot+1].
template <typename T, int VX>
__device__ __forceinline__ void col_load(T (&d)[VX], const T *p, int64_t ks, int l, int ktot, bool on)
{
    if (on && l >= 0 && l <= ktot + 1) {
        vload<T, VX>(d, p + (int64_t)l * ks);
    } else {
#pragma unroll
        for (int n = 0; n < VX; ++n) d[n] = T(0);
    }
}

// LDS row of W columns stored as VX planes: column c at (c % VX) * P + c / VX
// with P = ceil(W / VX).  Lane l's points c = VX*l + m then sit at unit stride
// across the lanes for every fixed m, so a wave's row access is free of bank
// conflicts (with VX consecutive 4-byte columns per lane a plain row is read
// at stride VX).  VX = 1 is the plain row.  Used for 4-byte elements only:
// 8-byte elements at a 16-byte lane stride measured faster in plain rows.
template <typename T, int VX>
constexpr int planar_vx()
{
    return sizeof(T) == 4 ? VX : 1;
}

template <int VX, int W>
struct PlanarRow {
    static constexpr int P = (W + VX - 1) / VX;
    static constexpr int SIZE = VX * P;
    __device__ static __forceinline__ int at(int c) { return (c % VX) * P + c / VX; }
};

// YS = 1 evaluates every y face once: each wave its row's north face, wave 0
// also the tile's south face, exchanged through an LDS row (a second barrier
// per level).  A face's operands are the same for the two rows it separates,
// so the values are bitwise those of YS = 0.
template <typename T, int VX, int BY, int KB, int XCD, int NT, int WPE, int YS = 0>
__global__ __launch_bounds__(64 * BY, WPE) void advec_u_2i5_zl(StencilArgs<T> a)
{
    constexpr int TX = 64 * VX;
    constexpr int SW = TX + 6;               // u row in LDS: columns i0w-3 .. i0w+TX+2
    constexpr int VW = TX + 1;               // v row in LDS: columns i0w-1 .. i0w+TX-1
    constexpr int NH = (6 + BY - 1) / BY;    // u halo rows per wave (upper bound)
    typedef PlanarRow<planar_vx<T, VX>(), SW> UR;  // u rows, planar by VX (4-byte T)
    typedef PlanarRow<planar_vx<T, VX>(), VW> VR;  // v rows, likewise
    __shared__ __align__(16) T su[2][BY + 6][UR::SIZE];
    __shared__ __align__(16) T sv[2][BY + 1][VR::SIZE];
    __shared__ __align__(16) T sfy[YS ? BY + 1 : 1][YS ? TX : 1];  // y-face fluxes of one level

    int tx, ty, tz;
    tile_of<64, BY, XCD>(a.nbx, a.nby, a.nbz, tx, ty, tz);
    const int lane = (int)threadIdx.x, r = wave_row();
    const int i0w = 1 + tx * TX;
    const int nlanes = min(64, (a.itot - i0w + 1) / VX);
    const bool lane_on = lane < nlanes;
    const int xo = lane * VX;
    const bool edge_l = lane == 0;
    const int j0 = 1 + ty * BY;
    const int nv = min(BY, a.jtot - j0 + 1);
    const bool own = r < nv;
    const int k0 = 1 + tz * KB, k1 = min(k0 + KB, a.ktot + 1);
    const int kt = a.ktot;
    const int64_t js = a.js, ks = a.ks;
    const T *u = a.u, *v = a.v, *w = a.w;
    T *ut = a.ut;
    const T dxi = a.dxi, dyi = a.dyi;

    // Level-0 addresses.  Every load of the level loop is unconditional and
    // inside the field: lanes beyond the grid read the last active lane's
    // points, waves beyond the last row read the last row, waves without a
    // halo row read their own row.  One scalar load per row carries its x halo:
    // lanes 0..2 the three columns left of the tile, lanes 3..5 the three
    // right of it (u rows); lane 0 the column left of the own v row, lane 1 the
    // one left of the v halo row.
    const int lane_c = min(lane, nlanes - 1);
    const int64_t rowo = a.off + i0w + (int64_t)min(j0 + r, a.jtot) * js;   // (i0w, own row, 0)
    const int64_t c_own = rowo + lane_c * VX;
    const int ecol = lane < 3 ? wrap_x(i0w - 3 + lane, a.itot) - i0w
                              : (lane < 6 ? wrap_x(i0w + nlanes * VX + lane - 3, a.itot) - i0w : lane_c * VX);
    const int64_t e_own = rowo + ecol;
    const int xl1 = wrap_x(i0w - 1, a.itot) - i0w;                        // column left of the tile
    int hrho[NH];   // LDS rows of this wave's u halo rows, -1 if none
    int64_t hc[NH], he[NH];
#pragma unroll
    for (int m = 0; m < NH; ++m) {
        const int h = r + m * BY;
        hrho[m] = h < 6 ? (h < 3 ? h : nv + h) : -1;
        const int64_t hrow0 = a.off + i0w + (int64_t)(j0 - 3 + (hrho[m] < 0 ? 3 : hrho[m])) * js;
        hc[m] = hrho[m] < 0 ? c_own : hrow0 + lane_c * VX;
        he[m] = hrho[m] < 0 ? c_own : hrow0 + ecol;
    }
    const bool vhalo = r == BY - 1;                                       // loads v row j0 + nv
    const int64_t vrow = a.off + i0w + (int64_t)(j0 + nv) * js;           // (i0w, j0 + nv, 0)
    const int64_t c_vh = vhalo ? vrow + lane_c * VX : c_own;
    const int64_t e_v = lane == 0 ? rowo + xl1 : (lane == 1 && vhalo ? vrow + xl1 : c_own);
    const int64_t e_w = lane == 0 ? rowo + xl1 : c_own;
    const int lx_u = lane < 3 ? lane : nlanes * VX + lane;                // LDS column of a lane's u halo value

    // registers: current (level k) and next (level k+1) copies of what the
    // LDS planes receive, the w row at k+1 (next: k+2), ut at k (loaded at
    // the start of level k, used at its end)
    T S[6][VX];                              // u(k-2) .. u(k+3) of the own column
    T HU[2][NH][VX], HE[2][NH];              // u halo rows and their x-halo values
    T OE[2];                                 // x-halo value of the own u row
    T VO[2][VX], VH[2][VX], VE[2];           // own v row, v halo row, their left halo values
    T WR[2][VX], WL[2];                      // w at k+1 (and k+2), left neighbour cell (lane 0)
    T UT[VX];

    auto load_level = [&](int q, int k) {    // everything level k needs, into slot q (k <= ktot)
        const int64_t lk = (int64_t)k * ks;
#pragma unroll
        for (int m = 0; m < NH; ++m) {
            vload<T, VX>(HU[q][m], u + hc[m] + lk);
            HE[q][m] = u[he[m] + lk];
        }
        OE[q] = u[e_own + lk];
        vload<T, VX>(VO[q], v + c_own + lk);
        vload<T, VX>(VH[q], v + c_vh + lk);
        VE[q] = v[e_v + lk];
        vload<T, VX>(WR[q], w + c_own + lk + ks);
        WL[q] = w[e_w + lk + ks];
    };

    // prologue: the u window, the flux through face k0, level k0's data
#pragma unroll
    for (int m = 0; m < 6; ++m) col_load<T, VX>(S[m], u + c_own, ks, k0 - 2 + m, kt, true);
    T FB[VX];
    {
        T ub3[VX], w0[VX];
        col_load<T, VX>(ub3, u + c_own, ks, k0 - 3, kt, true);
        col_load<T, VX>(w0, w + c_own, ks, k0, kt, true);
        T wl0 = w[e_w + (int64_t)k0 * ks];
        const T sh = shfl_up1(w0[VX - 1]);
        if (!edge_l) wl0 = sh;
#pragma unroll
        for (int n = 0; n < VX; ++n) {
            const T wm = n == 0 ? wl0 : w0[n - 1];
            FB[n] = flux_z_2i5(mid(wm, w0[n]), ub3[n], S[0][n], S[1][n], S[2][n], S[3][n], S[4][n], k0, kt);
        }
    }
    load_level(0, k0);

    vm_drain();
    for (int k = k0; k < k1; ++k) {
        const int p = k & 1;
        // 1. level k into LDS plane p
        if (own && lane_on) {
#pragma unroll
            for (int n = 0; n < VX; ++n) {
                su[p][r + 3][UR::at(3 + xo + n)] = S[2][n];
                sv[p][r][VR::at(1 + xo + n)] = VO[0][n];
            }
        }
        if (own && lane < 6) su[p][r + 3][UR::at(lx_u)] = OE[0];
        if (own && lane == 0) sv[p][r][VR::at(0)] = VE[0];
#pragma unroll
        for (int m = 0; m < NH; ++m) {
            const int rho = hrho[m];
            if (rho >= 0) {
                if (lane_on) {
#pragma unroll
                    for (int n = 0; n < VX; ++n) su[p][rho][UR::at(3 + xo + n)] = HU[0][m][n];
                }
                if (lane < 6) su[p][rho][UR::at(lx_u)] = HE[0][m];
            }
        }
        if (vhalo) {
            if (lane_on) {
#pragma unroll
                for (int n = 0; n < VX; ++n) sv[p][nv][VR::at(1 + xo + n)] = VH[0][n];
            }
            if (lane == 1) sv[p][nv][VR::at(0)] = VE[0];
        }
        // 2. ut of level k (waited for at the end of the level's arithmetic),
        //    then the prefetch of level k+1 and of the u window's next level
        tload<NT, T, VX>(UT, ut + c_own + (int64_t)k * ks);
        load_level(1, min(k + 1, k1 - 1));   // clamped at the last level, where it is unused
        T unext[VX];
        col_load<T, VX>(unext, u + c_own, ks, k + 4, kt, k + 1 < k1);
        __syncthreads();

        // 3. compute level k
        const T sh = shfl_up1(WR[0][VX - 1]);
        const T wl = edge_l ? WL[0] : sh;
        T FN[VX], FS[VX];
        if constexpr (YS) {
            if (own && lane_on) {
#pragma unroll
                for (int n = 0; n < VX; ++n) {
                    const int xu = UR::at(3 + xo + n);
                    T col[7];
#pragma unroll
                    for (int m = 1; m < 7; ++m) col[m] = su[p][r + m][xu];
                    const T vn = mid(sv[p][r + 1][VR::at(xo + n)], sv[p][r + 1][VR::at(xo + n + 1)]);
                    FN[n] = flux5(vn, col[1], col[2], col[3], col[4], col[5], col[6]);
                    if (r == 0) {
                        col[0] = su[p][0][xu];
                        const T vs = mid(sv[p][0][VR::at(xo + n)], sv[p][0][VR::at(xo + n + 1)]);
                        FS[n] = flux5(vs, col[0], col[1], col[2], col[3], col[4], col[5]);
                    }
                }
                vstore<T, VX>(&sfy[r + 1][xo], FN);
                if (r == 0) vstore<T, VX>(&sfy[0][xo], FS);
            }
            __syncthreads();
            if (own && lane_on && r > 0) vload<T, VX>(FS, &sfy[r][xo]);
        }
        if (own && lane_on) {
            T uxr[VX + 6];
#pragma unroll
            for (int m = 0; m < VX + 6; ++m) uxr[m] = su[p][r + 3][UR::at(xo + m)];
            T FX[VX + 1];
#pragma unroll
            for (int f = 0; f <= VX; ++f)
                FX[f] = flux5(mid(uxr[f + 2], uxr[f + 3]), uxr[f], uxr[f + 1], uxr[f + 2], uxr[f + 3],
                              uxr[f + 4], uxr[f + 5]);
            const T dzik = kload(a.dzi, k);
            T res[VX];
#pragma unroll
            for (int n = 0; n < VX; ++n) {
                T fn, fs;
                if constexpr (YS) {
                    fn = FN[n];
                    fs = FS[n];
                } else {
                    const int xu = UR::at(3 + xo + n);
                    T col[7];
#pragma unroll
                    for (int m = 0; m < 7; ++m) col[m] = su[p][r + m][xu];
                    const T vn = mid(sv[p][r + 1][VR::at(xo + n)], sv[p][r + 1][VR::at(xo + n + 1)]);
                    const T vs = mid(sv[p][r][VR::at(xo + n)], sv[p][r][VR::at(xo + n + 1)]);
                    fn = flux5(vn, col[1], col[2], col[3], col[4], col[5], col[6]);
                    fs = flux5(vs, col[0], col[1], col[2], col[3], col[4], col[5]);
                }
                const T wm = n == 0 ? wl : WR[0][n - 1];
                const T ft = flux_z_2i5(mid(wm, WR[0][n]), S[0][n], S[1][n], S[2][n], S[3][n], S[4][n], S[5][n],
                                        k + 1, kt);
                res[n] = UT[n] + advec_2i5_combine(FX[n + 1], FX[n], fn, fs, ft, FB[n], dxi, dyi, dzik);
                FB[n] = ft;
            }
            tstore<NT, T, VX>(ut + c_own + (int64_t)k * ks, res);
        }

        // 4. advance the window and the register slots
#pragma unroll
        for (int m = 0; m < 5; ++m)
#pragma unroll
            for (int n = 0; n < VX; ++n) S[m][n] = S[m + 1][n];
#pragma unroll
        for (int n = 0; n < VX; ++n) {
            S[5][n] = unext[n];
            VO[0][n] = VO[1][n];
            VH[0][n] = VH[1][n];
            WR[0][n] = WR[1][n];
        }
        VE[0] = VE[1];
        WL[0] = WL[1];
        OE[0] = OE[1];
#pragma unroll
        for (int m = 0; m < NH; ++m) {
#pragma unroll
            for (int n = 0; n < VX; ++n) HU[0][m][n] = HU[1][m][n];
            HE[0][m] = HE[1][m];
        }
    }
}

// The same tile with the z-march unrolled by pairs of levels: the two
// register slots and the two LDS planes alternate with compile-time indices
// and the u window moves two levels at a time, so no per-level register
// copies remain (more live registers, fewer instructions).
template <typename T, int VX, int BY, int KB, int XCD, int NT, int WPE>
__global__ __launch_bounds__(64 * BY, WPE) void advec_u_2i5_zlp(StencilArgs<T> a)
{
    constexpr int TX = 64 * VX;
    constexpr int SW = TX + 6;               // u row in LDS: columns i0w-3 .. i0w+TX+2
    constexpr int VW = TX + 1;               // v row in LDS: columns i0w-1 .. i0w+TX-1
    constexpr int NH = (6 + BY - 1) / BY;    // u halo rows per wave (upper bound)
    typedef PlanarRow<planar_vx<T, VX>(), SW> UR;  // u rows, planar by VX (4-byte T)
    typedef PlanarRow<planar_vx<T, VX>(), VW> VR;  // v rows, likewise
    __shared__ __align__(16) T su[2][BY + 6][UR::SIZE];
    __shared__ __align__(16) T sv[2][BY + 1][VR::SIZE];

    int tx, ty, tz;
    tile_of<64, BY, XCD>(a.nbx, a.nby, a.nbz, tx, ty, tz);
    const int lane = (int)threadIdx.x, r = wave_row();
    const int i0w = 1 + tx * TX;
    const int nlanes = min(64, (a.itot - i0w + 1) / VX);
    const bool lane_on = lane < nlanes;
    const int xo = lane * VX;
    const bool edge_l = lane == 0, edge_r = lane == nlanes - 1;
    const int j0 = 1 + ty * BY;
    const int nv = min(BY, a.jtot - j0 + 1);
    const bool own = r < nv;
    const int k0 = 1 + tz * KB, k1 = min(k0 + KB, a.ktot + 1);
    const int kt = a.ktot;
    const int64_t js = a.js, ks = a.ks;
    const T *u = a.u, *v = a.v, *w = a.w;
    T *ut = a.ut;
    const T dxi = a.dxi, dyi = a.dyi;

    // level-0 addresses of this lane's points in the own row and the halo rows
    const int64_t row0 = a.off + i0w + xo;
    const int64_t c_own = row0 + (int64_t)(j0 + r) * js;
    const int64_t e_own = a.off + i0w + (int64_t)(j0 + r) * js;           // (i0w, j0 + r, 0)
    const int iend = i0w + nlanes * VX - 1;                               // last point of the tile
    // offsets from i0w of the periodic images of the x halo columns
    int xlo[3], xhi[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        xlo[e] = wrap_x(i0w - 3 + e, a.itot) - i0w;
        xhi[e] = wrap_x(iend + 1 + e, a.itot) - i0w;
    }
    const int xl1 = xlo[2];
    int hrho[NH];   // LDS rows of this wave's u halo rows, -1 if none
    int64_t hc[NH], he[NH];
#pragma unroll
    for (int m = 0; m < NH; ++m) {
        const int h = r + m * BY;
        hrho[m] = h < 6 ? (h < 3 ? h : nv + h) : -1;
        const int jg = j0 - 3 + (hrho[m] < 0 ? 3 : hrho[m]);
        hc[m] = row0 + (int64_t)jg * js;
        he[m] = a.off + i0w + (int64_t)jg * js;
    }
    const bool vhalo = r == BY - 1;                                       // loads v row j0 + nv
    const int64_t c_vh = row0 + (int64_t)(j0 + nv) * js;
    const int64_t e_vh = a.off + i0w + (int64_t)(j0 + nv) * js;

    // registers, in two slots used in turn by the two levels of a pair: what
    // the LDS planes receive, the w row at k+1, ut at k
    T S[9][VX];                              // u(k-2) .. u(k+6) of the own column, k = even level of a pair
    T HU[2][NH][VX], HUL[2][NH][3], HUR[2][NH][3];
    T OUL[2][3], OUR[2][3];                  // x halo of the own u row
    T VO[2][VX], VOL[2];                     // own v row and its left halo cell
    T VH[2][VX], VHL[2];                     // v halo row and its left halo cell
    T WR[2][VX], WL[2];                      // w at k+1, left neighbour cell (lane 0)
    T UT[2][VX];

    auto load_level = [&](auto qc, int k) {  // everything level k needs, into slot q
        constexpr int q = decltype(qc)::value;
#pragma unroll
        for (int m = 0; m < NH; ++m) {
            const bool on = hrho[m] >= 0;
            if (on && lane_on) vload<T, VX>(HU[q][m], u + hc[m] + (int64_t)k * ks);
            if (on && edge_l) {
#pragma unroll
                for (int e = 0; e < 3; ++e) HUL[q][m][e] = u[he[m] + (int64_t)k * ks + xlo[e]];
            }
            if (on && edge_r) {
#pragma unroll
                for (int e = 0; e < 3; ++e) HUR[q][m][e] = u[he[m] + (int64_t)k * ks + xhi[e]];
            }
        }
        if (own) {
            if (edge_l) {
#pragma unroll
                for (int e = 0; e < 3; ++e) OUL[q][e] = u[e_own + (int64_t)k * ks + xlo[e]];
                VOL[q] = v[e_own + (int64_t)k * ks + xl1];
            }
            if (edge_r) {
#pragma unroll
                for (int e = 0; e < 3; ++e) OUR[q][e] = u[e_own + (int64_t)k * ks + xhi[e]];
            }
            if (lane_on) {
                vload<T, VX>(VO[q], v + c_own + (int64_t)k * ks);
                vload<T, VX>(WR[q], w + c_own + (int64_t)(k + 1) * ks);
                tload<NT, T, VX>(UT[q], ut + c_own + (int64_t)k * ks);
            }
            if (edge_l) WL[q] = w[e_own + (int64_t)(k + 1) * ks + xl1];
        }
        if (vhalo) {
            if (lane_on) vload<T, VX>(VH[q], v + c_vh + (int64_t)k * ks);
            if (edge_l) VHL[q] = v[e_vh + (int64_t)k * ks + xl1];
        }
    };

    // prologue: the u window, the flux through face k0, level k0's data
#pragma unroll
    for (int m = 0; m < 7; ++m) col_load<T, VX>(S[m], u + c_own, ks, k0 - 2 + m, kt, own && lane_on);
#pragma unroll
    for (int n = 0; n < VX; ++n) S[7][n] = S[8][n] = T(0);
    T FB[VX];
    {
        T ub3[VX], w0[VX];
        col_load<T, VX>(ub3, u + c_own, ks, k0 - 3, kt, own && lane_on);
        col_load<T, VX>(w0, w + c_own, ks, k0, kt, own && lane_on);
        T wl0 = (own && edge_l) ? w[e_own + (int64_t)k0 * ks + xl1] : T(0);
        const T sh = shfl_up1(w0[VX - 1]);
        if (!edge_l) wl0 = sh;
#pragma unroll
        for (int n = 0; n < VX; ++n) {
            const T wm = n == 0 ? wl0 : w0[n - 1];
            FB[n] = flux_z_2i5(mid(wm, w0[n]), ub3[n], S[0][n], S[1][n], S[2][n], S[3][n], S[4][n], k0, kt);
        }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
#pragma unroll
        for (int n = 0; n < VX; ++n) VO[q][n] = VH[q][n] = WR[q][n] = UT[q][n] = T(0);
#pragma unroll
        for (int m = 0; m < NH; ++m) {
#pragma unroll
            for (int n = 0; n < VX; ++n) HU[q][m][n] = T(0);
#pragma unroll
            for (int e = 0; e < 3; ++e) HUL[q][m][e] = HUR[q][m][e] = T(0);
        }
#pragma unroll
        for (int e = 0; e < 3; ++e) OUL[q][e] = OUR[q][e] = T(0);
        VOL[q] = VHL[q] = WL[q] = T(0);
    }
    load_level(std::integral_constant<int, 0>(), k0);

    // One level; P is its position in the pair (LDS plane P, register slot
    // P, u window offset P).
    auto level = [&](auto pc, int k) {
        constexpr int P = decltype(pc)::value;
        constexpr int Q = P ^ 1;
        // 1. level k into LDS plane P
        if (own && lane_on) {
#pragma unroll
            for (int n = 0; n < VX; ++n) {
                su[P][r + 3][UR::at(3 + xo + n)] = S[2 + P][n];
                sv[P][r][VR::at(1 + xo + n)] = VO[P][n];
            }
        }
        if (own && edge_l) {
#pragma unroll
            for (int e = 0; e < 3; ++e) su[P][r + 3][UR::at(e)] = OUL[P][e];
            sv[P][r][VR::at(0)] = VOL[P];
        }
        if (own && edge_r) {
#pragma unroll
            for (int e = 0; e < 3; ++e) su[P][r + 3][UR::at(3 + nlanes * VX + e)] = OUR[P][e];
        }
#pragma unroll
        for (int m = 0; m < NH; ++m) {
            const int rho = hrho[m];
            if (rho >= 0) {
                if (lane_on) {
#pragma unroll
                    for (int n = 0; n < VX; ++n) su[P][rho][UR::at(3 + xo + n)] = HU[P][m][n];
                }
                if (edge_l) {
#pragma unroll
                    for (int e = 0; e < 3; ++e) su[P][rho][UR::at(e)] = HUL[P][m][e];
                }
                if (edge_r) {
#pragma unroll
                    for (int e = 0; e < 3; ++e) su[P][rho][UR::at(3 + nlanes * VX + e)] = HUR[P][m][e];
                }
            }
        }
        if (vhalo) {
            if (lane_on) {
#pragma unroll
                for (int n = 0; n < VX; ++n) sv[P][nv][VR::at(1 + xo + n)] = VH[P][n];
            }
            if (edge_l) sv[P][nv][VR::at(0)] = VHL[P];
        }
        // 2. prefetch level k+1 into the other slot and the u window's k+5
        if (k + 1 < k1) load_level(std::integral_constant<int, Q>(), k + 1);
        col_load<T, VX>(S[7 + P], u + c_own, ks, k + 5, kt, own && lane_on && k + 1 < k1);
        __syncthreads();

        // 3. compute level k from plane P and the window S[P .. P+5]
        const T sh = shfl_up1(WR[P][VX - 1]);
        const T wl = edge_l ? WL[P] : sh;
        if (own && lane_on) {
            T uxr[VX + 6];
#pragma unroll
            for (int m = 0; m < VX + 6; ++m) uxr[m] = su[P][r + 3][UR::at(xo + m)];
            T FX[VX + 1];
#pragma unroll
            for (int f = 0; f <= VX; ++f)
                FX[f] = flux5(mid(uxr[f + 2], uxr[f + 3]), uxr[f], uxr[f + 1], uxr[f + 2], uxr[f + 3],
                              uxr[f + 4], uxr[f + 5]);
            const T dzik = kload(a.dzi, k);
            T res[VX];
#pragma unroll
            for (int n = 0; n < VX; ++n) {
                const int xu = UR::at(3 + xo + n);
                T col[7];
#pragma unroll
                for (int m = 0; m < 7; ++m) col[m] = su[P][r + m][xu];
                const T vn = mid(sv[P][r + 1][VR::at(xo + n)], sv[P][r + 1][VR::at(xo + n + 1)]);
                const T vs = mid(sv[P][r][VR::at(xo + n)], sv[P][r][VR::at(xo + n + 1)]);
                const T fn = flux5(vn, col[1], col[2], col[3], col[4], col[5], col[6]);
                const T fs = flux5(vs, col[0], col[1], col[2], col[3], col[4], col[5]);
                const T wm = n == 0 ? wl : WR[P][n - 1];
                const T ft = flux_z_2i5(mid(wm, WR[P][n]), S[P][n], S[P + 1][n], S[P + 2][n], S[P + 3][n],
                                        S[P + 4][n], S[P + 5][n], k + 1, kt);
                res[n] = UT[P][n] + advec_2i5_combine(FX[n + 1], FX[n], fn, fs, ft, FB[n], dxi, dyi, dzik);
                FB[n] = ft;
            }
            tstore<NT, T, VX>(ut + c_own + (int64_t)k * ks, res);
        }
    };

    vm_drain();
    for (int k = k0; k < k1; k += 2) {
        level(std::integral_constant<int, 0>(), k);
        if (k + 1 < k1) level(std::integral_constant<int, 1>(), k + 1);
        // the window moves two levels
#pragma unroll
        for (int m = 0; m < 7; ++m)
#pragma unroll
            for (int n = 0; n < VX; ++n) S[m][n] = S[m + 2][n];
    }
}

}  // namespace kl

namespace kl {

// The tile of advec_u_2i5_zl with its level loop unrolled by two (by the
// halo ring's period when HL > 1, below) and every value loaded ahead held
// in a slot chosen by the level's parity at compile time, so no register is
// copied at the end of a level:
//   * level k+1's rows, the edge values, w at k+2 and ut at k+1 are loaded
//     during level k into the other parity's slots; the u window's next top
//     level (k+5) is loaded two levels before it enters the window;
//   * every wave and lane runs every LDS write and the whole arithmetic
//     (clamped loads keep idle rows and lanes on valid data; their LDS writes
//     go to a spare row); only the store of ut is predicated.
// A register filled by a load and copied or left unused on some path in the
// same level makes the compiler wait for every load in flight at that point,
// which reduces the prefetch to nothing; here each load is waited for only
// when the level it belongs to begins.  The field accesses take a uniform
// base (the tile's corner row j0-3 at i = 1, on the level) and a 32-bit
// per-lane offset from it.  Same operands, same order, so results equal the
// other configurations bitwise.
//
// HL > 1 loads the u halo rows HL levels ahead, into a ring of HL + 1
// slots: the neighbouring tile loads the same row as its own (the window's
// top) five levels ahead, so with HL = 5 both requests meet in L2 and the
// row is fetched from HBM once.
template <typename T, int VX, int BY, int KB, int XCD, int NT, int WPE, int HL = 1>
__global__ __launch_bounds__(64 * BY, WPE) void advec_u_2i5_zr(StencilArgs<T> a)
{
    constexpr int TX = 64 * VX;
    constexpr int SW = TX + 6;               // u row in LDS: columns i0w-3 .. i0w+TX+2
    constexpr int VW = TX + 1;               // v row in LDS: columns i0w-1 .. i0w+TX-1
    constexpr int NH = (6 + BY - 1) / BY;    // u halo rows per wave (upper bound)
    constexpr int SU = BY + 6, SV = BY + 1;  // spare LDS rows (never read)
    typedef PlanarRow<planar_vx<T, VX>(), SW> UR;
    typedef PlanarRow<planar_vx<T, VX>(), VW> VR;
    static_assert(SW >= 64 && VW >= 64, "a spare row holds one column per lane");
    __shared__ __align__(16) T su[2][BY + 7][UR::SIZE];
    __shared__ __align__(16) T sv[2][BY + 2][VR::SIZE];

    int tx, ty, tz;
    tile_of<64, BY, XCD>(a.nbx, a.nby, a.nbz, tx, ty, tz);
    const int lane = (int)threadIdx.x, r = wave_row();
    const int i0w = 1 + tx * TX;
    const int nlanes = min(64, (a.itot - i0w + 1) / VX);
    const int xo = lane * VX;
    const int j0 = 1 + ty * BY;
    const int nv = min(BY, a.jtot - j0 + 1);
    const bool own = r < nv;
    const bool st_on = own && lane < nlanes;
    const int k0 = 1 + tz * KB, k1 = min(k0 + KB, a.ktot + 1);
    const int kt = a.ktot;
    const int64_t ks = a.ks;
    const int js = (int)a.js;
    const T dxi = a.dxi, dyi = a.dyi;

    // Offsets (elements) from the uniform base (i = 1, j = j0 - 3) of the
    // level; the grid's rows j0-3 .. j0+BY+2 and columns 1 .. itot keep them
    // non-negative.  Lanes beyond the grid read the last active lane's
    // points, waves beyond the last row read the last row, waves without a
    // halo row read their own row.
    const int lane_c = min(lane, nlanes - 1);
    const int rown = 3 + min(r, a.jtot - j0);                     // own row (relative)
    const int cx = i0w - 1 + lane_c * VX;                         // a lane's first column (relative)
    const int o_own = rown * js + cx;
    const int ecol = lane < 3 ? wrap_x(i0w - 3 + lane, a.itot) - 1
                              : (lane < 6 ? wrap_x(i0w + nlanes * VX + lane - 3, a.itot) - 1 : cx);
    const int o_eown = rown * js + ecol;
    const int xl1 = wrap_x(i0w - 1, a.itot) - 1;                  // column left of the tile
    int hrow[NH], o_hc[NH], o_he[NH];                             // LDS row (SU: none), offsets
#pragma unroll
    for (int m = 0; m < NH; ++m) {
        const int h = r + m * BY;
        const int rho = h < 6 ? (h < 3 ? h : nv + h) : -1;
        hrow[m] = rho >= 0 ? rho : SU;
        o_hc[m] = rho >= 0 ? rho * js + cx : o_own;
        o_he[m] = rho >= 0 ? rho * js + ecol : o_own;
    }
    const bool vhalo = r == BY - 1;                               // loads v row j0 + nv
    const int vrel = 3 + nv;
    const int o_vh = vhalo ? vrel * js + cx : o_own;
    const int o_ev = lane == 0 ? rown * js + xl1 : (lane == 1 && vhalo ? vrel * js + xl1 : o_own);
    const int o_ew = lane == 0 ? rown * js + xl1 : o_own;
    // LDS destinations: rows of this wave (spare when it has none), and the
    // x-halo values of lanes 0..5 (u) and 0..1 (v); other lanes write a
    // column of the spare row
    const int ou = own ? r + 3 : SU, ov = own ? r : SV, vhr = vhalo ? nv : SV;
    const int lx_u = lane < 3 ? lane : nlanes * VX + lane;
    const int eu_col = lane < 6 ? UR::at(lx_u) : UR::at(lane);
    const int eu_row = lane < 6 ? ou : SU;
    const int ev_row = lane == 0 ? ov : (lane == 1 ? vhr : SV);
    const int ev_col = VR::at(lane < 2 ? 0 : lane);

    const int64_t tb = a.off + 1 + (int64_t)(j0 - 3) * a.js;
    const T *u = a.u + tb, *v = a.v + tb, *w = a.w + tb;
    T *ut = a.ut + tb;
    auto at = [&](auto *f, int l, int o) { return boff(f + (int64_t)l * ks, (uint32_t)o * (uint32_t)sizeof(T)); };

    T S[6][VX];                              // u(k-2) .. u(k+3) of the own column
    T UN[2][VX];                             // window tops in flight
    constexpr int HS = HL + 1;               // halo ring slots
    constexpr int RS = HS % 2 ? 2 * HS : HS; // levels per unrolled pass (slot indices fixed)
    T HU[HS][NH][VX], HE[HS][NH];            // u halo rows and their x-halo values (ring)
    T OE[2];                                 // x-halo values of the own u row (by parity)
    T VO[2][VX], VH[2][VX], VE[2];           // own v row, v halo row, left halo values
    T WR[2][VX], WL[2];                      // w one level up, left neighbour cell (lane 0)
    T UT[2][VX];                             // ut of the level

    auto load_halo = [&](int h, int k) {     // u halo rows of level k into ring slot h
#pragma unroll
        for (int m = 0; m < NH; ++m) {
            vload<T, VX>(HU[h][m], at(u, k, o_hc[m]));
            HE[h][m] = *at(u, k, o_he[m]);
        }
    };
    auto load_level = [&](int q, int k) {    // level k's other operands into slot q (k <= ktot)
        OE[q] = *at(u, k, o_eown);
        vload<T, VX>(VO[q], at(v, k, o_own));
        vload<T, VX>(VH[q], at(v, k, o_vh));
        VE[q] = *at(v, k, o_ev);
        vload<T, VX>(WR[q], at(w, k + 1, o_own));
        WL[q] = *at(w, k + 1, o_ew);
        tload<NT, T, VX>(UT[q], at(ut, k, o_own));
    };

    // prologue: the u window (levels outside [0, ktot+1] clamped: the z
    // fluxes never use them), the flux through face k0, level k0's operands
    // and the window top of level k0+1
#pragma unroll
    for (int m = 0; m < 6; ++m) vload<T, VX>(S[m], at(u, min(max(k0 - 2 + m, 0), kt + 1), o_own));
    T FB[VX];
    {
        T ub3[VX], w0[VX];
        vload<T, VX>(ub3, at(u, max(k0 - 3, 0), o_own));
        vload<T, VX>(w0, at(w, k0, o_own));
        const T wl0 = *at(w, k0, o_ew);
        const T sh = shfl_up1(w0[VX - 1]);
        const T wl = lane == 0 ? wl0 : sh;
#pragma unroll
        for (int n = 0; n < VX; ++n) {
            const T wm = n == 0 ? wl : w0[n - 1];
            FB[n] = flux_z_2i5(mid(wm, w0[n]), ub3[n], S[0][n], S[1][n], S[2][n], S[3][n], S[4][n], k0, kt);
        }
    }
#pragma unroll
    for (int h = 0; h < HL; ++h) load_halo(h, min(k0 + h, k1 - 1));
    load_level(0, k0);
    vload<T, VX>(UN[1], at(u, min(k0 + 4, kt + 1), o_own));

    vm_drain();
    for (int kk = k0;; kk += RS) {
#pragma unroll
        for (int s = 0; s < RS; ++s) {
            const int k = kk + s;
            if (k >= k1) return;
            const int p = s & 1, q = p ^ 1, hs = s % HS;
            // 1. operands of level k+1 and halo rows of level k+HL (clamped at
            //    the tile's last level, where they are unused), the window top
            //    of level k+2
            load_halo((s + HL) % HS, min(k + HL, k1 - 1));
            load_level(q, min(k + 1, k1 - 1));
            vload<T, VX>(UN[p], at(u, min(k + 5, kt + 1), o_own));
            // 2. level k into LDS plane p
#pragma unroll
            for (int n = 0; n < VX; ++n) {
                su[p][ou][UR::at(3 + xo + n)] = S[2][n];
                sv[p][ov][VR::at(1 + xo + n)] = VO[p][n];
                sv[p][vhr][VR::at(1 + xo + n)] = VH[p][n];
            }
#pragma unroll
            for (int m = 0; m < NH; ++m)
#pragma unroll
                for (int n = 0; n < VX; ++n) su[p][hrow[m]][UR::at(3 + xo + n)] = HU[hs][m][n];
            // the x-halo values after the rows: a lane beyond the grid writes
            // its row values into the right halo columns, which these replace
            su[p][eu_row][eu_col] = OE[p];
#pragma unroll
            for (int m = 0; m < NH; ++m) su[p][lane < 6 ? hrow[m] : SU][eu_col] = HE[hs][m];
            sv[p][ev_row][ev_col] = VE[p];
            __syncthreads();

            // 3. level k
            const T sh = shfl_up1(WR[p][VX - 1]);
            const T wl = lane == 0 ? WL[p] : sh;
            T uxr[VX + 6];
#pragma unroll
            for (int m = 0; m < VX + 6; ++m) uxr[m] = su[p][r + 3][UR::at(xo + m)];
            T FX[VX + 1];
#pragma unroll
            for (int f = 0; f <= VX; ++f)
                FX[f] = flux5(mid(uxr[f + 2], uxr[f + 3]), uxr[f], uxr[f + 1], uxr[f + 2], uxr[f + 3], uxr[f + 4],
                              uxr[f + 5]);
            const T dzik = kload(a.dzi, k);
            T res[VX];
#pragma unroll
            for (int n = 0; n < VX; ++n) {
                const int xu = UR::at(3 + xo + n);
                T col[7];
#pragma unroll
                for (int m = 0; m < 7; ++m) col[m] = su[p][r + m][xu];
                const T vn = mid(sv[p][r + 1][VR::at(xo + n)], sv[p][r + 1][VR::at(xo + n + 1)]);
                const T vs = mid(sv[p][r][VR::at(xo + n)], sv[p][r][VR::at(xo + n + 1)]);
                const T fn = flux5(vn, col[1], col[2], col[3], col[4], col[5], col[6]);
                const T fs = flux5(vs, col[0], col[1], col[2], col[3], col[4], col[5]);
                const T wm = n == 0 ? wl : WR[p][n - 1];
                const T ft = flux_z_2i5(mid(wm, WR[p][n]), S[0][n], S[1][n], S[2][n], S[3][n], S[4][n], S[5][n],
                                        k + 1, kt);
                res[n] = UT[p][n] + advec_2i5_combine(FX[n + 1], FX[n], fn, fs, ft, FB[n], dxi, dyi, dzik);
                FB[n] = ft;
            }
            if (st_on) tstore<NT, T, VX>(at(ut, k, o_own), res);

            // 4. the window moves up one level; its new top was loaded a level ago
#pragma unroll
            for (int m = 0; m < 5; ++m)
#pragma unroll
                for (int n = 0; n < VX; ++n) S[m][n] = S[m + 1][n];
#pragma unroll
            for (int n = 0; n < VX; ++n) S[5][n] = UN[q][n];
        }
    }
}

// ---------------------------------------------------------------------------
// LDS-staged z-marching configuration of diff_smag.
//
// Workgroup = 64 x BY threads (wave r owns row j0 + r, each lane VX points),
// tile 64*VX x BY, levels [k0, k0 + KB).  The stencil of a point reaches one
// cell in every direction, in all four inputs (u, v, w, evisc), on levels
// k-1, k and k+1.  The operands on level k-1 are exactly the ones the same
// lane read on level k one step earlier, so they are carried in registers
// (struct Below) together with the bottom faces, and LDS holds only levels k
// and k+1 of each input, plus the plane being refilled: a ring of three
// planes of (BY+2) x (TX+2) cells (one halo cell on each side).  At level k
// the waves read levels k and k+1 and then write level k+2 into the plane of
// level k-1, whose last readers finished before this level's barrier, so
// one barrier per level suffices.  The global loads of level k+2 are issued
// before the arithmetic of level k, after those of the tendencies of level
// k.  Every point calls the shared per-component functions with the default
// configuration's operands, so results are bitwise identical.
// ---------------------------------------------------------------------------

template <typename T>
struct SmagBelow {                          // operands of level k-1 at one point
    T u, ue, v, vn, e, ew, ee, es, en;
};

template <typename T, int VX, int BY, int KB, int XCD, int NT, int WPE>
__global__ __launch_bounds__(64 * BY, WPE) void diff_smag_zl(StencilArgs<T> a)
{
    constexpr int TX = 64 * VX;
    constexpr int PW = TX + 2;              // plane row: columns i0w-1 .. i0w+TX
    constexpr int PH = BY + 2;              // plane rows: j0-1 .. j0+BY
    constexpr int NH = (8 + BY - 1) / BY;   // halo rows per wave (8 = 2 rows x 4 fields)
    typedef PlanarRow<planar_vx<T, VX>(), PW> SR;  // plane rows, planar by VX (4-byte T)
    __shared__ __align__(16) T pl[4][3][PH][SR::SIZE];  // [field][ring plane][row][column]

    int tx, ty, tz;
    tile_of<64, BY, XCD>(a.nbx, a.nby, a.nbz, tx, ty, tz);
    const int lane = (int)threadIdx.x, r = wave_row();
    const int i0w = 1 + tx * TX;
    const int nlanes = min(64, (a.itot - i0w + 1) / VX);
    const bool lane_on = lane < nlanes;
    const int xo = lane * VX;
    const int j0 = 1 + ty * BY;
    const int nv = min(BY, a.jtot - j0 + 1);
    const bool own = r < nv;
    const int k0 = 1 + tz * KB, k1 = min(k0 + KB, a.ktot + 1);
    const int64_t js = a.js, ks = a.ks;
    const T *F[4] = {a.u, a.v, a.w, a.evisc};
    const int xr = 1 + nlanes * VX;         // LDS column of the right halo cell

    // Every global load below is unconditional, from an address inside the
    // field: lanes beyond the grid re-read the last active lane's points,
    // waves beyond the last row re-read the last row, waves without a halo
    // row re-read their own row, and one scalar load per row carries both
    // halo columns (the left one in lane 0, the right one in lane le).  No
    // load sits behind a branch, so the compiler counts the loads in flight
    // exactly and does not drain the prefetch of level k+2 before it is due.
    const int lane_c = min(lane, nlanes - 1);
    const int le = max(nlanes - 1, 1);      // lane loading the right halo cell
    // Addresses: a wave-uniform row start (column 0) plus a per-lane byte
    // offset, own point (i0w + lane_c*VX) or halo column (in lane 0 the
    // periodic image of column i0w-1, in lane le that of i0w + nlanes*VX:
    // x is periodic, so the halo columns come from the row's interior and no
    // x ghost line is fetched); the level offset goes into the uniform part.
    const int64_t row_c = a.off + (int64_t)min(j0 + r, a.jtot) * js;
    const uint32_t o_pt = (uint32_t)(i0w + lane_c * VX) * sizeof(T);
    const uint32_t o_e = lane == 0 ? (uint32_t)wrap_x(i0w - 1, a.itot) * sizeof(T)
                                   : (lane == le ? (uint32_t)wrap_x(i0w + nlanes * VX, a.itot) * sizeof(T) : o_pt);

    // rows this wave stages: its own (LDS row r+1) and halo rows h = r, r+BY,
    // ... of the 8 (field h/2; LDS row 0 for even h, nv+1 for odd h)
    int hf[NH], hrow[NH];
    int64_t hr0[NH];
#pragma unroll
    for (int m = 0; m < NH; ++m) {
        const int h = r + m * BY;
        hf[m] = h < 8 ? h >> 1 : -1;
        hrow[m] = (h & 1) ? nv + 1 : 0;
        hr0[m] = hf[m] < 0 ? row_c : a.off + (int64_t)(j0 - 1 + hrow[m]) * js;
    }

    T O[4][VX], OE[4];                      // own row of the 4 inputs at one level, halo columns
    T H[NH][VX], HE[NH];                    // halo rows
    T TT[3][VX];                            // ut, vt, wt at level k

    auto load_plane = [&](int l) {           // level l of everything this wave stages
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            const T *row = F[f] + row_c + (int64_t)l * ks;
            vload<T, VX>(O[f], boff(row, o_pt));
            OE[f] = *boff(row, o_e);
        }
#pragma unroll
        for (int m = 0; m < NH; ++m) {
            // a select, not an indexed pointer array, keeps these global loads
            const T *p = hf[m] == 1 ? a.v : (hf[m] == 2 ? a.w : (hf[m] == 3 ? a.evisc : a.u));
            const T *row = p + hr0[m] + (int64_t)l * ks;
            vload<T, VX>(H[m], boff(row, o_pt));
            HE[m] = *boff(row, o_e);
        }
    };
    auto store_plane = [&](int b) {          // the staged level into ring plane b
        if (own) {
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                if (lane_on) {
#pragma unroll
                    for (int n = 0; n < VX; ++n) pl[f][b][r + 1][SR::at(1 + xo + n)] = O[f][n];
                }
                if (lane == 0) pl[f][b][r + 1][SR::at(0)] = OE[f];
                if (lane == le) pl[f][b][r + 1][SR::at(xr)] = OE[f];
            }
        }
#pragma unroll
        for (int m = 0; m < NH; ++m) {
            if (hf[m] < 0) continue;
            if (lane_on) {
#pragma unroll
                for (int n = 0; n < VX; ++n) pl[hf[m]][b][hrow[m]][SR::at(1 + xo + n)] = H[m][n];
            }
            if (lane == 0) pl[hf[m]][b][hrow[m]][SR::at(0)] = HE[m];
            if (lane == le) pl[hf[m]][b][hrow[m]][SR::at(xr)] = HE[m];
        }
    };

    // prologue: levels k0-1, k0 and k0+1 into ring planes 0, 1 and 2; the
    // operands and vertical faces of level k0-1 into registers
    load_plane(k0 - 1);
    store_plane(0);
    load_plane(k0);
    store_plane(1);
    load_plane(k0 + 1);
    const T dxi = a.dxi, dyi = a.dyi;
    SmagFace<T> BU[VX], BV[VX];
    T BW[VX];
    SmagBelow<T> L[VX];
    __syncthreads();
    if (own && lane_on) {
        const int rr = r + 1;
        const T dzhik = kload(a.dzhi, k0);
#pragma unroll
        for (int n = 0; n < VX; ++n) {
            const int x = 1 + xo + n;
#define P(f, b, dj, di) pl[f][b][rr + (dj)][SR::at(x + (di))]
            const T uc = P(0, 1, 0, 0), ub = P(0, 0, 0, 0), vc = P(1, 1, 0, 0), vb = P(1, 0, 0, 0);
            const T wc = P(2, 1, 0, 0), ww = P(2, 1, 0, -1), ws = P(2, 1, -1, 0), wb = P(2, 0, 0, 0);
            const T ec = P(3, 1, 0, 0), ew = P(3, 1, 0, -1), es = P(3, 1, -1, 0), eb = P(3, 0, 0, 0),
                    ebw = P(3, 0, 0, -1), ebs = P(3, 0, -1, 0);
            L[n] = {ub, P(0, 0, 0, 1), vb, P(1, 0, 1, 0), eb, ebw, P(3, 0, 0, 1), ebs, P(3, 0, 1, 0)};
#undef P
            BU[n] = smag_u_zface<T>(ebw, eb, ew, ec, uc, ub, wc, ww, dxi, dzhik);
            BV[n] = smag_v_zface<T>(ebs, eb, es, ec, vc, vb, wc, ws, dyi, dzhik);
            BW[n] = smag_w_zcenter<T>(eb, wc, wb);
        }
    }
    store_plane(2);
    vm_drain();

    // ring planes of levels k-1, k and k+1, rotated every level
    int bm = 0, bc = 1, bp = 2;
    for (int k = k0; k < k1; ++k) {
        __syncthreads();                     // level k+1 visible, level k-1 no longer read
        // the tendencies of level k, then level k+2 (clamped at the end of
        // the tile, where it is unused): the arithmetic waits for the former only
#pragma unroll
        for (int f = 0; f < 3; ++f)
            tload<NT, T, VX>(TT[f], boff((f == 0 ? a.ut : (f == 1 ? a.vt : a.wt)) + row_c + (int64_t)k * ks, o_pt));
        load_plane(min(k + 2, k1));

        if (own && lane_on) {
            const T dzik = kload(a.dzi, k), dzikm1 = kload(a.dzi, k - 1), dzhik = kload(a.dzhi, k), dzhik1 = kload(a.dzhi, k + 1);
            const int rr = r + 1;
            T o0[VX], o1[VX], o2[VX];
#pragma unroll
            for (int n = 0; n < VX; ++n) {
                const int x = 1 + xo + n;
                // operand names: <field><offset>; offsets e/w (x), n/s (y), t/b (z)
#define P(f, b, dj, di) pl[f][b][rr + (dj)][SR::at(x + (di))]
                const T uc = P(0, bc, 0, 0), ue = P(0, bc, 0, 1), uw = P(0, bc, 0, -1), un = P(0, bc, 1, 0),
                        us = P(0, bc, -1, 0), ut_ = P(0, bp, 0, 0), use = P(0, bc, -1, 1);
                const T vc = P(1, bc, 0, 0), ve = P(1, bc, 0, 1), vw = P(1, bc, 0, -1), vn = P(1, bc, 1, 0),
                        vs = P(1, bc, -1, 0), vt_ = P(1, bp, 0, 0), vnw = P(1, bc, 1, -1);
                const T wc = P(2, bc, 0, 0), we = P(2, bc, 0, 1), ww = P(2, bc, 0, -1), wn = P(2, bc, 1, 0),
                        ws = P(2, bc, -1, 0), wt_ = P(2, bp, 0, 0), wtw = P(2, bp, 0, -1),
                        wts = P(2, bp, -1, 0);
                const T ec = P(3, bc, 0, 0), ee = P(3, bc, 0, 1), ew = P(3, bc, 0, -1), en = P(3, bc, 1, 0),
                        es = P(3, bc, -1, 0), et = P(3, bp, 0, 0), enw = P(3, bc, 1, -1),
                        esw = P(3, bc, -1, -1), ese = P(3, bc, -1, 1), etw = P(3, bp, 0, -1), ets = P(3, bp, -1, 0);
#undef P
                const SmagBelow<T> b = L[n];
                // the same operations as smag_u/v/w, with the bottom faces carried
                const SmagFace<T> tu = smag_u_zface<T>(ew, ec, etw, et, ut_, uc, wt_, wtw, dxi, dzhik1);
                const SmagFace<T> tv = smag_v_zface<T>(es, ec, ets, et, vt_, vc, wt_, wts, dyi, dzhik1);
                const T tw = smag_w_zcenter<T>(ec, wt_, wc);
                o0[n] = TT[0][n] + smag_uv_total<T>(smag_u_xy<T>(uc, ue, uw, un, us, vn, vnw, vc, vw, ec, ew, en,
                                                                 enw, es, esw, dxi, dyi),
                                                    tu, BU[n], dzik);
                o1[n] = TT[1][n] + smag_uv_total<T>(smag_v_xy<T>(vc, ve, vw, vn, vs, ue, use, uc, us, ec, es, ee,
                                                                 ese, ew, esw, dxi, dyi),
                                                    tv, BV[n], dzik);
                o2[n] = TT[2][n] + smag_w_total<T>(smag_w_xy<T>(wc, we, ww, wn, ws, ue, b.ue, uc, b.u, vn, b.vn, vc,
                                                                b.v, ec, b.e, ee, b.ee, ew, b.ew, en, b.en, es, b.es,
                                                                dxi, dyi, dzhik),
                                                   tw, BW[n], dzik, dzikm1, dzhik);
                BU[n] = tu;
                BV[n] = tv;
                BW[n] = tw;
                L[n] = {uc, ue, vc, vn, ec, ew, ee, es, en};
            }
            tstore<NT, T, VX>(boff(a.ut + row_c + (int64_t)k * ks, o_pt), o0);
            tstore<NT, T, VX>(boff(a.vt + row_c + (int64_t)k * ks, o_pt), o1);
            if (k >= a.kw0) tstore<NT, T, VX>(boff(a.wt + row_c + (int64_t)k * ks, o_pt), o2);
        }

        store_plane(bm);                     // level k+2 over level k-1
        const int t = bm;
        bm = bc;
        bc = bp;
        bp = t;
    }
}

// diff_smag_zl with the staged rows loaded one level further ahead into two
// register slots chosen by the level's parity at compile time (level loop
// unrolled by two), every wave and lane writing LDS and computing, and only
// the stores predicated, as in advec_u_2i5_zr: a level then waits only for
// loads issued a level earlier.  Same operands, same order: bitwise the
// other configurations.
template <typename T, int VX, int BY, int KB, int XCD, int NT, int WPE>
__global__ __launch_bounds__(64 * BY, WPE) void diff_smag_zr(StencilArgs<T> a)
{
    constexpr int TX = 64 * VX;
    constexpr int PW = TX + 2;              // plane row: columns i0w-1 .. i0w+TX
    constexpr int PH = BY + 2;              // plane rows: j0-1 .. j0+BY
    constexpr int NH = (8 + BY - 1) / BY;   // halo rows per wave (8 = 2 rows x 4 fields)
    typedef PlanarRow<planar_vx<T, VX>(), PW> SR;  // plane rows, planar by VX (4-byte T)
    __shared__ __align__(16) T pl[4][3][PH + 1][SR::SIZE];  // [field][ring plane][row][column]; row PH is a spare

    int tx, ty, tz;
    tile_of<64, BY, XCD>(a.nbx, a.nby, a.nbz, tx, ty, tz);
    const int lane = (int)threadIdx.x, r = wave_row();
    const int i0w = 1 + tx * TX;
    const int nlanes = min(64, (a.itot - i0w + 1) / VX);
    const bool lane_on = lane < nlanes;
    const int xo = lane * VX;
    const int j0 = 1 + ty * BY;
    const int nv = min(BY, a.jtot - j0 + 1);
    const bool own = r < nv;
    const int k0 = 1 + tz * KB, k1 = min(k0 + KB, a.ktot + 1);
    const int64_t js = a.js, ks = a.ks;
    const T *F[4] = {a.u, a.v, a.w, a.evisc};
    const int xr = 1 + nlanes * VX;         // LDS column of the right halo cell

    // Every global load below is unconditional, from an address inside the
    // field: lanes beyond the grid re-read the last active lane's points,
    // waves beyond the last row re-read the last row, waves without a halo
    // row re-read their own row, and one scalar load per row carries both
    // halo columns (the left one in lane 0, the right one in lane le).  No
    // load sits behind a branch, so the compiler counts the loads in flight
    // exactly and does not drain the prefetch of level k+2 before it is due.
    const int lane_c = min(lane, nlanes - 1);
    const int le = max(nlanes - 1, 1);      // lane loading the right halo cell
    // Addresses: a wave-uniform row start (column 0) plus a per-lane byte
    // offset, own point (i0w + lane_c*VX) or halo column (in lane 0 the
    // periodic image of column i0w-1, in lane le that of i0w + nlanes*VX:
    // x is periodic, so the halo columns come from the row's interior and no
    // x ghost line is fetched); the level offset goes into the uniform part.
    const int64_t row_c = a.off + (int64_t)min(j0 + r, a.jtot) * js;
    const uint32_t o_pt = (uint32_t)(i0w + lane_c * VX) * sizeof(T);
    const uint32_t o_e = lane == 0 ? (uint32_t)wrap_x(i0w - 1, a.itot) * sizeof(T)
                                   : (lane == le ? (uint32_t)wrap_x(i0w + nlanes * VX, a.itot) * sizeof(T) : o_pt);

    // rows this wave stages: its own (LDS row r+1) and halo rows h = r, r+BY,
    // ... of the 8 (field h/2; LDS row 0 for even h, nv+1 for odd h)
    int hf[NH], hrow[NH];
    int64_t hr0[NH];
#pragma unroll
    for (int m = 0; m < NH; ++m) {
        const int h = r + m * BY;
        hf[m] = h < 8 ? h >> 1 : -1;
        hrow[m] = (h & 1) ? nv + 1 : 0;
        hr0[m] = hf[m] < 0 ? row_c : a.off + (int64_t)(j0 - 1 + hrow[m]) * js;
    }

    // Staged rows in two slots by level parity: level l's rows are loaded
    // two levels before they are written to LDS (at the end of level l-2,
    // into the plane of level l-3), so no level waits for the rows it
    // loads.  The tendencies of level k are loaded first in level k and
    // waited for by its arithmetic only.
    T O[2][4][VX], OE[2][4];                // own row of the 4 inputs, halo columns
    T H[2][NH][VX], HE[2][NH];              // halo rows
    T TT[3][VX];                            // ut, vt, wt of the level
    // LDS destinations: every wave writes every row it could stage (the
    // spare row PH when it has none) and every lane writes an edge value
    // (lanes other than 0 and le into a column of the spare row)
    const int orow = own ? r + 1 : PH;
    const int ecol = lane == 0 ? SR::at(0) : (lane == le ? SR::at(xr) : SR::at(lane));
    const int erow = lane == 0 || lane == le ? orow : PH;
    int hfs[NH], hrs[NH], hre[NH];
#pragma unroll
    for (int m = 0; m < NH; ++m) {
        hfs[m] = hf[m] < 0 ? 0 : hf[m];
        hrs[m] = hf[m] < 0 ? PH : hrow[m];
        hre[m] = lane == 0 || lane == le ? hrs[m] : PH;
    }

    auto load_plane = [&](int q, int l) {    // level l of everything this wave stages, into slot q
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            const T *row = F[f] + row_c + (int64_t)l * ks;
            vload<T, VX>(O[q][f], boff(row, o_pt));
            OE[q][f] = *boff(row, o_e);
        }
#pragma unroll
        for (int m = 0; m < NH; ++m) {
            // a select, not an indexed pointer array, keeps these global loads
            const T *p = hf[m] == 1 ? a.v : (hf[m] == 2 ? a.w : (hf[m] == 3 ? a.evisc : a.u));
            const T *row = p + hr0[m] + (int64_t)l * ks;
            vload<T, VX>(H[q][m], boff(row, o_pt));
            HE[q][m] = *boff(row, o_e);
        }
    };
    auto load_tend = [&](int l) {
#pragma unroll
        for (int f = 0; f < 3; ++f)
            tload<NT, T, VX>(TT[f], boff((f == 0 ? a.ut : (f == 1 ? a.vt : a.wt)) + row_c + (int64_t)l * ks, o_pt));
    };
    auto store_plane = [&](int q, int b) {   // slot q into ring plane b; the edge values after the rows
#pragma unroll
        for (int f = 0; f < 4; ++f) {
#pragma unroll
            for (int n = 0; n < VX; ++n) pl[f][b][orow][SR::at(1 + xo + n)] = O[q][f][n];
        }
#pragma unroll
        for (int m = 0; m < NH; ++m) {
#pragma unroll
            for (int n = 0; n < VX; ++n) pl[hfs[m]][b][hrs[m]][SR::at(1 + xo + n)] = H[q][m][n];
        }
#pragma unroll
        for (int f = 0; f < 4; ++f) pl[f][b][erow][ecol] = OE[q][f];
#pragma unroll
        for (int m = 0; m < NH; ++m) pl[hfs[m]][b][hre[m]][ecol] = HE[q][m];
    };

    // prologue: levels k0-1, k0 and k0+1 into ring planes 0, 1 and 2; the
    // operands and vertical faces of level k0-1 into registers
    load_plane(0, k0 - 1);
    store_plane(0, 0);
    load_plane(0, k0);
    store_plane(0, 1);
    load_plane(1, k0 + 1);
    load_plane(0, min(k0 + 2, k1));
    const T dxi = a.dxi, dyi = a.dyi;
    SmagFace<T> BU[VX], BV[VX];
    T BW[VX];
    SmagBelow<T> L[VX];
    __syncthreads();
    {
        const int rr = r + 1;
        const T dzhik = kload(a.dzhi, k0);
#pragma unroll
        for (int n = 0; n < VX; ++n) {
            const int x = 1 + xo + n;
#define P(f, b, dj, di) pl[f][b][rr + (dj)][SR::at(x + (di))]
            const T uc = P(0, 1, 0, 0), ub = P(0, 0, 0, 0), vc = P(1, 1, 0, 0), vb = P(1, 0, 0, 0);
            const T wc = P(2, 1, 0, 0), ww = P(2, 1, 0, -1), ws = P(2, 1, -1, 0), wb = P(2, 0, 0, 0);
            const T ec = P(3, 1, 0, 0), ew = P(3, 1, 0, -1), es = P(3, 1, -1, 0), eb = P(3, 0, 0, 0),
                    ebw = P(3, 0, 0, -1), ebs = P(3, 0, -1, 0);
            L[n] = {ub, P(0, 0, 0, 1), vb, P(1, 0, 1, 0), eb, ebw, P(3, 0, 0, 1), ebs, P(3, 0, 1, 0)};
#undef P
            BU[n] = smag_u_zface<T>(ebw, eb, ew, ec, uc, ub, wc, ww, dxi, dzhik);
            BV[n] = smag_v_zface<T>(ebs, eb, es, ec, vc, vb, wc, ws, dyi, dzhik);
            BW[n] = smag_w_zcenter<T>(eb, wc, wb);
        }
    }
    store_plane(1, 2);
    vm_drain();

    // ring planes of levels k-1, k and k+1, rotated every level
    int bm = 0, bc = 1, bp = 2;
    for (int kk = k0;; kk += 2) {
#pragma unroll
        for (int p = 0; p < 2; ++p) {
        const int k = kk + p;
        if (k >= k1) return;
        const int q = p ^ 1;
        __syncthreads();                     // level k+1 visible, level k-1 no longer read
        // level k's tendencies, then level k+3's rows (clamped at the end of
        // the tile, where they are unused) into the other slot
        load_tend(k);
        load_plane(q, min(k + 3, k1));

        {
            const T dzik = kload(a.dzi, k), dzikm1 = kload(a.dzi, k - 1), dzhik = kload(a.dzhi, k), dzhik1 = kload(a.dzhi, k + 1);
            const int rr = r + 1;
            T o0[VX], o1[VX], o2[VX];
#pragma unroll
            for (int n = 0; n < VX; ++n) {
                const int x = 1 + xo + n;
                // operand names: <field><offset>; offsets e/w (x), n/s (y), t/b (z)
#define P(f, b, dj, di) pl[f][b][rr + (dj)][SR::at(x + (di))]
                const T uc = P(0, bc, 0, 0), ue = P(0, bc, 0, 1), uw = P(0, bc, 0, -1), un = P(0, bc, 1, 0),
                        us = P(0, bc, -1, 0), ut_ = P(0, bp, 0, 0), use = P(0, bc, -1, 1);
                const T vc = P(1, bc, 0, 0), ve = P(1, bc, 0, 1), vw = P(1, bc, 0, -1), vn = P(1, bc, 1, 0),
                        vs = P(1, bc, -1, 0), vt_ = P(1, bp, 0, 0), vnw = P(1, bc, 1, -1);
                const T wc = P(2, bc, 0, 0), we = P(2, bc, 0, 1), ww = P(2, bc, 0, -1), wn = P(2, bc, 1, 0),
                        ws = P(2, bc, -1, 0), wt_ = P(2, bp, 0, 0), wtw = P(2, bp, 0, -1),
                        wts = P(2, bp, -1, 0);
                const T ec = P(3, bc, 0, 0), ee = P(3, bc, 0, 1), ew = P(3, bc, 0, -1), en = P(3, bc, 1, 0),
                        es = P(3, bc, -1, 0), et = P(3, bp, 0, 0), enw = P(3, bc, 1, -1),
                        esw = P(3, bc, -1, -1), ese = P(3, bc, -1, 1), etw = P(3, bp, 0, -1), ets = P(3, bp, -1, 0);
#undef P
                const SmagBelow<T> b = L[n];
                // the same operations as smag_u/v/w, with the bottom faces carried
                const SmagFace<T> tu = smag_u_zface<T>(ew, ec, etw, et, ut_, uc, wt_, wtw, dxi, dzhik1);
                const SmagFace<T> tv = smag_v_zface<T>(es, ec, ets, et, vt_, vc, wt_, wts, dyi, dzhik1);
                const T tw = smag_w_zcenter<T>(ec, wt_, wc);
                o0[n] = TT[0][n] + smag_uv_total<T>(smag_u_xy<T>(uc, ue, uw, un, us, vn, vnw, vc, vw, ec, ew, en,
                                                                 enw, es, esw, dxi, dyi),
                                                    tu, BU[n], dzik);
                o1[n] = TT[1][n] + smag_uv_total<T>(smag_v_xy<T>(vc, ve, vw, vn, vs, ue, use, uc, us, ec, es, ee,
                                                                 ese, ew, esw, dxi, dyi),
                                                    tv, BV[n], dzik);
                o2[n] = TT[2][n] + smag_w_total<T>(smag_w_xy<T>(wc, we, ww, wn, ws, ue, b.ue, uc, b.u, vn, b.vn, vc,
                                                                b.v, ec, b.e, ee, b.ee, ew, b.ew, en, b.en, es, b.es,
                                                                dxi, dyi, dzhik),
                                                   tw, BW[n], dzik, dzikm1, dzhik);
                BU[n] = tu;
                BV[n] = tv;
                BW[n] = tw;
                L[n] = {uc, ue, vc, vn, ec, ew, ee, es, en};
            }
            // the arithmetic only feeds the predicated stores: its loaded
            // operands are marked as read on every path
#pragma unroll
            for (int f = 0; f < 3; ++f) settle(TT[f]);
            if (own && lane_on) {
                tstore<NT, T, VX>(boff(a.ut + row_c + (int64_t)k * ks, o_pt), o0);
                tstore<NT, T, VX>(boff(a.vt + row_c + (int64_t)k * ks, o_pt), o1);
                if (k >= a.kw0) tstore<NT, T, VX>(boff(a.wt + row_c + (int64_t)k * ks, o_pt), o2);
            }
        }

        store_plane(p, bm);                  // level k+2 (loaded a level ago) over level k-1
        const int t = bm;
        bm = bc;
        bc = bp;
        bp = t;
        }
    }
}


}  // namespace kl
