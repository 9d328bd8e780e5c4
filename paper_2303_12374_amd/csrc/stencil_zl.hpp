// LDS-staged z-marching configurations of the tendency kernels.
//
// Workgroup = 64 x BY threads: wave r owns row j0 + r of a tile 64*VX wide
// in x and BY rows in y, each lane VX consecutive x points, and the tile
// walks levels [k0, k0 + KB).  Per level each row is read from global memory
// once:
//   * z neighbours: a 4-slot register ring per field (levels k-1, k, k+1 and
//     the prefetch of k+2), unrolled so the slots never move;
//   * y neighbours: every wave writes its level-k row to a double-buffered
//     LDS plane, the two halo rows (j0-1 and the row after the last valid
//     one) are written by wave 0 and by the "top" wave; one barrier a level;
//   * x neighbours: lane shuffles, with the two values beyond the wave's
//     segment loaded by the edge lanes.  x is periodic in every boundary
//     mode, so at the ends of a row those two values are read from the
//     row's interior (the periodic images that the ghost cells hold after
//     the ghost fill): no line of x ghost cells is fetched.
// The per-point arithmetic is the shared one of stencil.hpp, so results are
// bitwise equal to every other configuration.
#pragma once

#include "stencil.hpp"

namespace kl {

template <typename T>
__device__ __forceinline__ T shfl_up1(T x)
{
    return __shfl_up(x, 1u, 64);
}

template <typename T>
__device__ __forceinline__ T shfl_down1(T x)
{
    return __shfl_down(x, 1u, 64);
}

// Interior x index of the periodic image of column c (any integer): x is
// periodic in every boundary mode, and after the ghost fill a ghost column
// holds the value of this interior column.
__device__ __forceinline__ int wrap_x(int c, int itot)
{
    int q = (c - 1) % itot;
    if (q < 0) q += itot;
    return q + 1;
}

// Geometry of one zl tile as seen by one thread.
template <int VX, int BY, int KB>
struct ZlTile {
    int lane, r, i0w, i0, j0, nv, k0, k1, nlanes, top;
    int xl, xr;  // offsets from i0w of the left and right x neighbours of the segment (periodic)
    bool lane_on, own;
    int xrow_g, xrow_l;  // extra (halo) row of this wave: global row and LDS row, -1 if none

    __device__ __forceinline__ ZlTile(int itot, int jtot, int ktot, int tx, int ty, int tz)
    {
        constexpr int TX = 64 * VX;
        lane = (int)threadIdx.x;
        r = wave_row();
        i0w = 1 + tx * TX;
        i0 = i0w + lane * VX;
        j0 = 1 + ty * BY;
        nv = min(BY, jtot - j0 + 1);
        k0 = 1 + tz * KB;
        k1 = min(k0 + KB, ktot + 1);
        nlanes = min(64, (itot - i0w + 1) / VX);
        lane_on = lane < nlanes;
        own = r < nv;
        xl = i0w == 1 ? itot - 1 : -1;
        xr = i0w + nlanes * VX > itot ? 1 - i0w : nlanes * VX;
        top = nv < BY ? nv : BY - 1;
        xrow_g = xrow_l = -1;
        if (r == 0) {
            xrow_g = j0 - 1;
            xrow_l = 0;
        } else if (r == top) {
            xrow_g = j0 + nv;
            xrow_l = nv + 1;
        }
    }
};

// ---------------------------------------------------------------------------
// diff_uvw
// ---------------------------------------------------------------------------
// Field mask FM (bit f: field f of u, v, w is computed) and the LDS slot of a
// computed field; FM = 7 is the whole kernel, single bits are the
// per-component passes of the split configurations.
__host__ __device__ constexpr int fslot(int fm, int f)
{
    return (f > 0 ? (fm & 1) : 0) + (f > 1 ? ((fm >> 1) & 1) : 0);
}

// One tile (tx, ty, tz) of diff_uvw; called by the single-grid kernel and by
// the persistent batched kernel.  Starts with a barrier so that a block can
// run tiles back to back on the same LDS.
//
// Every global load of the level loop is unconditional, from an address
// inside the field: lanes beyond the grid and waves beyond the last row
// re-read a point of their clamped own row, waves without a halo row re-read
// their own row, and one scalar load per field carries both x-edge values
// (the left one in lane 0, the right one in the last active lane, or in lane 1
// when only lane 0 is active).  No load then sits behind a branch, so the
// compiler counts the loads in flight exactly and a level waits only for the
// data it uses, not for the prefetch of the levels after it.
template <typename T, int VX, int BY, int KB, int NT, int FM = 7>
__device__ __forceinline__ void diff_uvw_zl_tile(const StencilArgs<T> &a, int tx, int ty, int tz)
{
    static_assert(BY >= 2, "two halo rows need two waves");
    constexpr int TX = 64 * VX;
    typedef T RowT[TX];
    constexpr int NFL = (FM & 1) + ((FM >> 1) & 1) + ((FM >> 2) & 1);  // fields computed
    __shared__ __align__(16) RowT sh[2][NFL][BY + 2];
    __syncthreads();

    const ZlTile<VX, BY, KB> t(a.itot, a.jtot, a.ktot, tx, ty, tz);
    const int64_t js = a.js, ks = a.ks;
    const int lane_c = min(t.lane, t.nlanes - 1);                      // clamped lane
    const int64_t row_c = a.off + t.i0w + (int64_t)min(t.j0 + t.r, a.jtot) * js;  // (i0w, clamped row, 0)
    const int64_t c_own = row_c + lane_c * VX;                         // own point (clamped)
    const int64_t c_x = t.xrow_g >= 0 ? a.off + t.i0w + lane_c * VX + (int64_t)t.xrow_g * js : c_own;
    const int le = max(t.nlanes - 1, 1);                               // lane loading the right edge
    const int64_t c_e = t.lane == 0 ? row_c + t.xl : (t.lane == le ? row_c + t.xr : c_own);
    const bool ld_own = t.own && t.lane_on;
    const T *F[3] = {a.u, a.v, a.w};
    T *Tt[3] = {a.ut, a.vt, a.wt};
    const T dxi2 = a.dxi * a.dxi, dyi2 = a.dyi * a.dyi, visc = a.visc;
    const int kw0 = a.kw0;

    T R[4][3][VX];        // field ring: slot s%4 holds level kk+s
    T X[2][3][VX];        // halo row (or a re-read of the own row), by level parity
    T Q[2][3][VX];        // tendencies, by level parity
    T E[2][3];            // x edge values, by level parity

    const int k0 = t.k0, k1 = t.k1;
    // prologue: levels k0-1, k0, k0+1 and k0+2 of the own row (k0+2 <= ktot+1)
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        if (!((FM >> f) & 1)) continue;
        vload<T, VX>(R[3][f], F[f] + c_own + (int64_t)(k0 - 1) * ks);
        vload<T, VX>(R[0][f], F[f] + c_own + (int64_t)k0 * ks);
        vload<T, VX>(R[1][f], F[f] + c_own + (int64_t)(k0 + 1) * ks);
        vload<T, VX>(R[2][f], F[f] + c_own + (int64_t)min(k0 + 2, k1) * ks);
        tload<NT, T, VX>(Q[0][f], Tt[f] + c_own + (int64_t)k0 * ks);
        vload<T, VX>(X[0][f], F[f] + c_x + (int64_t)k0 * ks);
        E[0][f] = F[f][c_e + (int64_t)k0 * ks];
    }

    vm_drain();
    for (int kk = k0;; kk += 4) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int k = kk + s;
            if (k >= k1) return;
            const int p = s & 1, q = p ^ 1;
            T(&b)[3][VX] = R[(s + 3) & 3];  // level k-1; refilled with k+3 after use
            T(&c)[3][VX] = R[s & 3];
            T(&tp)[3][VX] = R[(s + 1) & 3];  // R[(s+2)&3] already holds level k+2
            // prefetch level k+1 (<= k1 <= ktot+1) of tendencies, halo row and edges
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                if (!((FM >> f) & 1)) continue;
                tload<NT, T, VX>(Q[q][f], Tt[f] + c_own + (int64_t)(k + 1) * ks);
                vload<T, VX>(X[q][f], F[f] + c_x + (int64_t)(k + 1) * ks);
                E[q][f] = F[f][c_e + (int64_t)(k + 1) * ks];
            }
            // level k rows into LDS
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                if (!((FM >> f) & 1)) continue;
                if (t.own) vstore<T, VX>(&sh[p][fslot(FM, f)][t.r + 1][t.lane * VX], c[f]);
                if (t.xrow_l >= 0) vstore<T, VX>(&sh[p][fslot(FM, f)][t.xrow_l][t.lane * VX], X[p][f]);
            }
            __syncthreads();
            const T dzik = kload(a.dzi, k), dzikm1 = kload(a.dzi, k - 1), dzhik = kload(a.dzhi, k),
                    dzhik1 = kload(a.dzhi, k + 1);
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                if (!((FM >> f) & 1)) continue;
                T nn[VX], ss[VX];
                vload<T, VX>(nn, &sh[p][fslot(FM, f)][t.r + 2][t.lane * VX]);
                vload<T, VX>(ss, &sh[p][fslot(FM, f)][t.r][t.lane * VX]);
                T left = shfl_up1<T>(c[f][VX - 1]);
                T right = shfl_down1<T>(c[f][0]);
                T er = E[p][f];
                if (t.nlanes == 1) er = __shfl(er, 1, 64);
                if (t.lane == 0) left = E[p][f];
                if (t.lane == t.nlanes - 1) right = er;
                if (ld_own && (f < 2 || k >= kw0)) {
#pragma unroll
                    for (int n = 0; n < VX; ++n) {
                        const T w_ = n == 0 ? left : c[f][n - 1];
                        const T e_ = n == VX - 1 ? right : c[f][n + 1];
                        const T d = f < 2 ? diff_c_point<T>(c[f][n], e_, w_, nn[n], ss[n], tp[f][n], b[f][n],
                                                            dxi2, dyi2, dzik, dzhik1, dzhik, visc)
                                          : diff_w_point<T>(c[f][n], e_, w_, nn[n], ss[n], tp[f][n], b[f][n],
                                                            dxi2, dyi2, dzik, dzikm1, dzhik, visc);
                        Q[p][f][n] = Q[p][f][n] + d;
                    }
                    tstore<NT, T, VX>(Tt[f] + c_own + (int64_t)k * ks, Q[p][f]);
                }
            }
            // level k-1 is no longer needed: its slot takes the k+3 prefetch
            // (clamped to k1 near the end of the tile, where it is not used)
#pragma unroll
            for (int f = 0; f < 3; ++f)
                if ((FM >> f) & 1) fload<NT, T, VX>(b[f], F[f] + c_own + (int64_t)min(k + 3, k1) * ks);
        }
    }
}

// ---------------------------------------------------------------------------
// advec_u
// ---------------------------------------------------------------------------
// The loads of the level loop are unconditional, as in diff_uvw_zl_tile:
// per field one scalar load carries the x-edge values (u: left in lane 0,
// right in the last active lane or lane 1; v: the own row's left value in
// lane 0, the top halo row's in lane 1; w: left in lane 0).
template <typename T, int VX, int BY, int KB, int NT, int WPE = 1>
__device__ __forceinline__ void advec_u_zl_tile(const StencilArgs<T> &a, int tx, int ty, int tz)
{
    static_assert(BY >= 2, "two halo rows need two waves");
    // Every wave and lane writes LDS and computes (ALL) only where the
    // launch's register cap (512 / the waves per SIMD it needs) is above 128
    // per lane: at 128 the longer live ranges spill, and the predicated form
    // is kept there.
    constexpr int NW = BY / 4 > WPE ? BY / 4 : WPE;
    constexpr bool ALL = 512 / NW > 128;
    constexpr int TX = 64 * VX;
    typedef T RowT[TX];
    __shared__ __align__(16) RowT shu[2][BY + 3];  // u rows j0-1 .. j0+nv; row BY+2 is a spare
    __shared__ __align__(16) RowT shv[2][BY + 3];  // v rows j0 .. j0+nv (LDS row r+1 = tile row r); spare
    __shared__ T shvl[2][BY + 2 + 64];              // v left of the segment, same rows; one spare per lane
    __syncthreads();

    const ZlTile<VX, BY, KB> t(a.itot, a.jtot, a.ktot, tx, ty, tz);
    const int64_t js = a.js, ks = a.ks;
    const int lane_c = min(t.lane, t.nlanes - 1);                      // clamped lane
    const int64_t row_c = a.off + t.i0w + (int64_t)min(t.j0 + t.r, a.jtot) * js;  // (i0w, clamped row, 0)
    const int64_t c_own = row_c + lane_c * VX;                         // own point (clamped)
    const bool x_is_top = t.xrow_g >= 0 && t.xrow_l > 0;              // the top halo row also needs v
    const int64_t xrow0 = a.off + t.i0w + (int64_t)max(t.xrow_g, 0) * js;   // (i0w, halo row, 0)
    const int64_t c_x = t.xrow_g >= 0 ? xrow0 + lane_c * VX : c_own;
    const int le = max(t.nlanes - 1, 1);                               // lane loading the right u edge
    const int64_t c_eu = t.lane == 0 ? row_c + t.xl : (t.lane == le ? row_c + t.xr : c_own);
    const int64_t c_ev = t.lane == 0 ? row_c + t.xl : (t.lane == 1 && x_is_top ? xrow0 + t.xl : c_own);
    const int64_t c_ew = t.lane == 0 ? row_c + t.xl : c_own;
    const bool ld_own = t.own && t.lane_on;
    const T dxi = a.dxi, dyi = a.dyi;
    const T *U = a.u, *V = a.v, *W = a.w;
    constexpr int SPARE = BY + 2;
    const int orow = t.own ? t.r + 1 : SPARE;
    const int xrow = t.xrow_l >= 0 ? t.xrow_l : SPARE;
    const int xvrow = x_is_top ? t.xrow_l : SPARE;
    const int evslot = t.own && t.lane == 0 ? t.r + 1 : (x_is_top && t.lane == 1 ? t.xrow_l : BY + 2 + t.lane);

    T RU[4][VX], RW[4][VX];   // u and w rings (u: k-1..k+2, w: k..k+2)
    T RV[2][VX];              // v at level k, k+1
    T XU[2][VX], XV[2][VX];   // extra row u and v (a re-read of the own row where there is none)
    T Q[2][VX];               // ut
    T EU[2], EV[2];           // u and v edge values by level parity
    T EW[4];                  // w left edge, ring like RW

    const int k0 = t.k0, k1 = t.k1;
    const int k2 = min(k0 + 2, k1);
    vload<T, VX>(RU[3], U + c_own + (int64_t)(k0 - 1) * ks);
    vload<T, VX>(RU[0], U + c_own + (int64_t)k0 * ks);
    vload<T, VX>(RU[1], U + c_own + (int64_t)(k0 + 1) * ks);
    vload<T, VX>(RU[2], U + c_own + (int64_t)k2 * ks);
    vload<T, VX>(RW[0], W + c_own + (int64_t)k0 * ks);
    vload<T, VX>(RW[1], W + c_own + (int64_t)(k0 + 1) * ks);
    vload<T, VX>(RW[2], W + c_own + (int64_t)k2 * ks);
    vload<T, VX>(RV[0], V + c_own + (int64_t)k0 * ks);
    tload<NT, T, VX>(Q[0], a.ut + c_own + (int64_t)k0 * ks);
    vload<T, VX>(XU[0], U + c_x + (int64_t)k0 * ks);
    vload<T, VX>(XV[0], V + c_x + (int64_t)k0 * ks);
    EU[0] = U[c_eu + (int64_t)k0 * ks];
    EV[0] = V[c_ev + (int64_t)k0 * ks];
    EW[0] = W[c_ew + (int64_t)k0 * ks];
    EW[1] = W[c_ew + (int64_t)(k0 + 1) * ks];
    EW[2] = W[c_ew + (int64_t)k2 * ks];

    vm_drain();
    for (int kk = k0;; kk += 4) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int k = kk + s;
            if (k >= k1) return;
            const int p = s & 1, q = p ^ 1;
            T(&ub)[VX] = RU[(s + 3) & 3];  // level k-1; refilled with k+3 after use
            T(&uc)[VX] = RU[s & 3];
            T(&ut_)[VX] = RU[(s + 1) & 3];
            T(&wc)[VX] = RW[s & 3];
            T(&wt)[VX] = RW[(s + 1) & 3];
            T(&wnx)[VX] = RW[(s + 3) & 3];  // w of level k-1 is not needed: prefetch k+3
            // prefetches, clamped to level k1 (<= ktot+1) near the end of the tile where unused
            const int64_t l3 = (int64_t)min(k + 3, k1) * ks, l1 = (int64_t)(k + 1) * ks;
            fload<NT, T, VX>(wnx, W + c_own + l3);
            EW[(s + 3) & 3] = W[c_ew + l3];
            fload<NT, T, VX>(RV[q], V + c_own + l1);
            tload<NT, T, VX>(Q[q], a.ut + c_own + l1);
            vload<T, VX>(XU[q], U + c_x + l1);
            vload<T, VX>(XV[q], V + c_x + l1);
            EU[q] = U[c_eu + l1];
            EV[q] = V[c_ev + l1];
            // level-k rows into LDS: u (own + halo rows), v (own + top halo) and
            // v's left edge.  Every wave and lane writes (a wave without such
            // a row into the spare row, lanes without an edge value into
            // their spare slot) and every lane computes, only the store being
            // predicated: a loaded value consumed on one path only makes the
            // compiler wait for all loads in flight where its register is
            // next written, which undoes the prefetch.
            if constexpr (ALL) {
                vstore<T, VX>(&shu[p][orow][t.lane * VX], uc);
                vstore<T, VX>(&shv[p][orow][t.lane * VX], RV[p]);
                vstore<T, VX>(&shu[p][xrow][t.lane * VX], XU[p]);
                vstore<T, VX>(&shv[p][xvrow][t.lane * VX], XV[p]);
                shvl[p][evslot] = EV[p];
            } else {
                if (t.own) {
                    vstore<T, VX>(&shu[p][t.r + 1][t.lane * VX], uc);
                    vstore<T, VX>(&shv[p][t.r + 1][t.lane * VX], RV[p]);
                    if (t.lane == 0) shvl[p][t.r + 1] = EV[p];
                }
                if (t.xrow_l >= 0) vstore<T, VX>(&shu[p][t.xrow_l][t.lane * VX], XU[p]);
                if (x_is_top) {
                    vstore<T, VX>(&shv[p][t.xrow_l][t.lane * VX], XV[p]);
                    if (t.lane == 1) shvl[p][t.xrow_l] = EV[p];
                }
            }
            __syncthreads();
            T un[VX], us[VX], vn[VX];
            vload<T, VX>(un, &shu[p][t.r + 2][t.lane * VX]);
            vload<T, VX>(us, &shu[p][t.r][t.lane * VX]);
            vload<T, VX>(vn, &shv[p][t.r + 2][t.lane * VX]);
            const T vnl_edge = shvl[p][t.r + 2];
            T uleft = shfl_up1<T>(uc[VX - 1]);
            T uright = shfl_down1<T>(uc[0]);
            T vleft = shfl_up1<T>(RV[p][VX - 1]);
            T vnleft = shfl_up1<T>(vn[VX - 1]);
            T wleft = shfl_up1<T>(wc[VX - 1]);
            T wtleft = shfl_up1<T>(wt[VX - 1]);
            T ur = EU[p];
            if (t.nlanes == 1) ur = __shfl(ur, 1, 64);
            if (t.lane == 0) {
                uleft = EU[p];
                vleft = EV[p];
                vnleft = vnl_edge;
                wleft = EW[s & 3];
                wtleft = EW[(s + 1) & 3];
            }
            if (t.lane == t.nlanes - 1) uright = ur;
            if (ALL || ld_own) {
                const T dzik = kload(a.dzi, k);
#pragma unroll
                for (int n = 0; n < VX; ++n) {
                    const T uw = n == 0 ? uleft : uc[n - 1];
                    const T ue = n == VX - 1 ? uright : uc[n + 1];
                    const T v_w = n == 0 ? vleft : RV[p][n - 1];
                    const T v_nw = n == 0 ? vnleft : vn[n - 1];
                    const T w_w = n == 0 ? wleft : wc[n - 1];
                    const T w_tw = n == 0 ? wtleft : wt[n - 1];
                    Q[p][n] = Q[p][n] + advec_u_point<T>(uc[n], ue, uw, un[n], us[n], ut_[n], ub[n], v_w,
                                                         RV[p][n], v_nw, vn[n], w_w, wc[n], w_tw, wt[n], dxi,
                                                         dyi, dzik);
                }
                if constexpr (ALL) {
                    // the compiler sinks this arithmetic into the predicated
                    // store: its loaded operands are marked as read on every path
                    settle(Q[p]);
                    settle(ub);
                    settle(ut_);
                    settle(wc);
                    settle(wt);
                    const T ew2[3] = {EU[p], EW[s & 3], EW[(s + 1) & 3]};
                    settle(ew2);
                }
                if (ld_own) tstore<NT, T, VX>(a.ut + c_own + (int64_t)k * ks, Q[p]);
            }
            fload<NT, T, VX>(ub, U + c_own + l3);
        }
    }
}

// Single-grid kernels: one block per tile.  NT streams the tendency arrays;
// WPE asks the compiler for at least that many waves per SIMD.
template <typename T, int VX, int BY, int KB, int XCD, int NT = 0, int WPE = 1, int FM = 7>
__global__ __launch_bounds__(64 * BY, WPE) void diff_uvw_zl(StencilArgs<T> a)
{
    int tx, ty, tz;
    tile_of<64, BY, XCD>(a.nbx, a.nby, a.nbz, tx, ty, tz);
    diff_uvw_zl_tile<T, VX, BY, KB, NT, FM>(a, tx, ty, tz);
}

template <typename T, int VX, int BY, int KB, int XCD, int NT = 0, int WPE = 1>
__global__ __launch_bounds__(64 * BY, WPE) void advec_u_zl(StencilArgs<T> a)
{
    int tx, ty, tz;
    tile_of<64, BY, XCD>(a.nbx, a.nby, a.nbz, tx, ty, tz);
    advec_u_zl_tile<T, VX, BY, KB, NT, WPE>(a, tx, ty, tz);
}

// Next tile of a block in a persistent walk over a tile list (prev = -1 for
// the first).  Without a queue the assignment is static: block b takes tiles
// b, b + gridDim.x, ...  With a queue (two device ints, both 0 at launch)
// one lane draws the next ticket from queue[0], so blocks that finish their
// tiles early take more and the walk ends with the blocks about level.
// Every tile is computed once, by one block, with the same arithmetic, so
// the results do not depend on which block takes which tile.
__device__ __forceinline__ int next_tile(int *queue, int prev)
{
    if (!queue) return prev < 0 ? (int)blockIdx.x : prev + (int)gridDim.x;
    __shared__ int ticket;
    __syncthreads();  // every wave has read the previous ticket
    if (threadIdx.x == 0 && threadIdx.y == 0) ticket = atomicAdd(queue, 1);
    __syncthreads();
    return ticket;
}

// End of a block's walk: the last block to finish returns the queue to 0 for
// the next launch (each block counts itself in queue[1] after its last draw).
__device__ __forceinline__ void walk_done(int *queue)
{
    if (!queue || threadIdx.x != 0 || threadIdx.y != 0) return;
    __threadfence();
    if (atomicAdd(queue + 1, 1) == (int)gridDim.x - 1) {
        __threadfence();
        atomicExch(queue, 0);
        atomicExch(queue + 1, 0);
    }
}

// Persistent batched kernels: each block walks tiles of a tile list
// (next_tile); tile = (grid, tx, ty, tz) into a table of per-grid arguments.
template <typename T, int VX, int BY, int KB, int NT = 0, int WPE = 1>
__global__ __launch_bounds__(64 * BY, WPE) void diff_uvw_zl_batch(const StencilArgs<T> *__restrict__ grids,
                                                                 const int4 *__restrict__ tiles, int ntiles,
                                                                 int *queue)
{
    for (int n = next_tile(queue, -1); n < ntiles; n = next_tile(queue, n)) {
        const int4 tl = tiles[n];
        const StencilArgs<T> a = global_args(grids[tl.x]);
        diff_uvw_zl_tile<T, VX, BY, KB, NT>(a, tl.y, tl.z, tl.w);
    }
    walk_done(queue);
}

template <typename T, int VX, int BY, int KB, int NT = 0, int WPE = 1>
__global__ __launch_bounds__(64 * BY, WPE) void advec_u_zl_batch(const StencilArgs<T> *__restrict__ grids,
                                                                const int4 *__restrict__ tiles, int ntiles,
                                                                int *queue)
{
    for (int n = next_tile(queue, -1); n < ntiles; n = next_tile(queue, n)) {
        const int4 tl = tiles[n];
        const StencilArgs<T> a = global_args(grids[tl.x]);
        advec_u_zl_tile<T, VX, BY, KB, NT, WPE>(a, tl.y, tl.z, tl.w);
    }
    walk_done(queue);
}

// Batched zeroing of the tendencies: tile = (grid, first row, end row) over
// the rows (j, k) of the interior, rows numbered j-1 + jtot*(k-1).
template <typename T>
__global__ __launch_bounds__(256) void zero_tendencies_batch(const StencilArgs<T> *__restrict__ grids,
                                                            const int4 *__restrict__ tiles, int ntiles)
{
    for (int n = blockIdx.x; n < ntiles; n += gridDim.x) {
        const int4 tl = tiles[n];
        const StencilArgs<T> a = global_args(grids[tl.x]);
        for (int r = tl.y; r < tl.z; ++r) {
            const int j = 1 + r % a.jtot, k = 1 + r / a.jtot;
            const int64_t base = a.off + (int64_t)j * a.js + (int64_t)k * a.ks;
            for (int i = 1 + (int)threadIdx.x; i <= a.itot; i += 256) {
                a.ut[base + i] = T(0);
                a.vt[base + i] = T(0);
                a.wt[base + i] = T(0);
            }
        }
    }
}

}  // namespace kl
