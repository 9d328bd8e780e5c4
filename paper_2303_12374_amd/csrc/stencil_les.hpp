// Device code of the paper's own schemes (Section "Tunable Parameters"):
//   advec_u_2i5 - advection of u, second-order flux form with the
//                 fifth-order upwind-biased face interpolation of Wicker and
//                 Skamarock (2002); three ghost cells in x and y;
//   diff_smag   - divergence of the viscous stress nu (grad u + grad u^T)
//                 with a cell-center eddy viscosity nu (Smagorinsky-type
//                 diffusion), second order on the staggered grid.
//
// The per-point arithmetic is written once, as functions of values (with
// explicit fused multiply-adds), and every configuration calls it with the
// same operands in the same order (-ffp-contract=off elsewhere), so all
// configurations agree bitwise.
#pragma once

#include "stencil.hpp"

namespace kl {

// ---------------------------------------------------------------------------
// fifth-order advection: face fluxes
// ---------------------------------------------------------------------------

// The face and stress functions below are written with explicit fused
// operations (tfma, stencil.hpp): fewer instructions on a path that is close
// to the ALU limit; every configuration calls the same functions, so
// configurations still agree bitwise.

// Face between a0 and a1, advecting velocity U: U * c6 - |U| * d5 with the
// sixth-order centered value c6 and the fifth-difference dissipation d5,
// c6 = (37 (a0+a1) - 8 (a-1+a2) + (a-2+a3)) / 60,
// d5 = (10 (a1-a0) - 5 (a2-a-1) + (a3-a-2)) / 60.
// For U >= 0, c6 - d5 is the upwind-biased value (2 a-2 - 13 a-1 + 47 a0 +
// 27 a1 - 3 a2) / 60, and for U < 0, c6 + d5 is its mirror image (the same
// weights on a3, a2, a1, a0, a-1).  In FP32 the operands are selected by the
// sign of U and the value is one chain of fused operations (fewer
// instructions); in FP64, where a select of two 8-byte values costs two
// instructions, c6 and d5 are formed as written.
template <typename T>
__device__ __forceinline__ T flux5(T U, T am2, T am1, T a0, T a1, T a2, T a3)
{
    if constexpr (sizeof(T) == 4) {
        const bool up = U >= T(0);
        const T b0 = up ? am2 : a3, b1 = up ? am1 : a2, b2 = up ? a0 : a1, b3 = up ? a1 : a0, b4 = up ? a2 : am1;
        T f = T(2.0 / 60.0) * b0;
        f = tfma(T(-13.0 / 60.0), b1, f);
        f = tfma(T(47.0 / 60.0), b2, f);
        f = tfma(T(27.0 / 60.0), b3, f);
        f = tfma(T(-3.0 / 60.0), b4, f);
        return U * f;
    } else {
        const T c37 = T(37.0 / 60.0), c8 = T(-8.0 / 60.0), c1 = T(1.0 / 60.0);
        const T c10 = T(10.0 / 60.0), c5 = T(-5.0 / 60.0);
        const T c6 = tfma(c37, a0 + a1, tfma(c8, am1 + a2, c1 * (am2 + a3)));
        const T d5 = tfma(c10, a1 - a0, tfma(c5, a2 - am1, c1 * (a3 - am2)));
        return tfma(U, c6, -(tabs(U) * d5));
    }
}

// Third-order upwind-biased face value times U:
// c4 = (7 (a0+a1) - (a-1+a2)) / 12, d3 = (3 (a1-a0) - (a2-a-1)) / 12, so the
// value is (-a-1 + 5 a0 + 2 a1) / 6 for U >= 0 and its mirror image
// otherwise (FP32 as a select and a chain, FP64 as written).
template <typename T>
__device__ __forceinline__ T flux3(T U, T am1, T a0, T a1, T a2)
{
    if constexpr (sizeof(T) == 4) {
        const bool up = U >= T(0);
        const T b0 = up ? am1 : a2, b1 = up ? a0 : a1, b2 = up ? a1 : a0;
        T f = T(-1.0 / 6.0) * b0;
        f = tfma(T(5.0 / 6.0), b1, f);
        f = tfma(T(2.0 / 6.0), b2, f);
        return U * f;
    } else {
        const T c7 = T(7.0 / 12.0), cm1 = T(-1.0 / 12.0), c3 = T(3.0 / 12.0);
        const T c4 = tfma(c7, a0 + a1, cm1 * (am1 + a2));
        const T d3 = tfma(c3, a1 - a0, cm1 * (a2 - am1));
        return tfma(U, c4, -(tabs(U) * d3));
    }
}

// Midpoint interpolation (also the advecting velocity at a face).
template <typename T>
__device__ __forceinline__ T mid(T a, T b)
{
    return T(0.5) * (a + b);
}

// z flux through face kf (between levels kf-1 and kf) of the u column:
// a[0..5] = u at levels kf-3 .. kf+2 (entries outside [0, ktot+1] unused).
// Second order at faces 1 and ktot+1, third order at faces 2 and ktot,
// fifth order elsewhere.
template <typename T>
__device__ __forceinline__ T flux_z_2i5(T W, T a0, T a1, T a2, T a3, T a4, T a5, int kf, int ktot)
{
    if (kf == 1 || kf == ktot + 1) return W * mid(a2, a3);
    if (kf == 2 || kf == ktot) return flux3(W, a1, a2, a3, a4);
    return flux5(W, a0, a1, a2, a3, a4, a5);
}

// The tendency from the six face fluxes of the u control volume.
template <typename T>
__device__ __forceinline__ T advec_2i5_combine(T fe, T fw, T fn, T fs, T ft, T fb, T dxi, T dyi, T dzik)
{
    const T adv_xy = tfma(fe - fw, dxi, (fn - fs) * dyi);
    return -tfma(ft - fb, dzik, adv_xy);
}

// ---------------------------------------------------------------------------
// stress divergence: one function per component, operands named by their
// offset from the point (e = east i+1, w = west i-1, n = j+1, s = j-1,
// t = k+1, b = k-1; combinations such as nw = (i-1, j+1)).
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ T mean4(T a, T b, T c, T d)
{
    return T(0.25) * ((a + b) + (c + d));
}

// The vertical stress terms of u and v are differences of two horizontal
// face values, each a product of a face viscosity (mean of four centers) and
// a face gradient; w's vertical term is a difference of two center values.
// A face's value is the same function of its own operands whichever point
// uses it, so a z-march computes the top face of level k once and reuses it,
// bit for bit, as the bottom face of level k+1.
template <typename T>
struct SmagFace {
    T e, g;  // face viscosity and face gradient (the stress is e * g)
};

// u's face at z_{k+1/2} between u(k) = uc and u(k+1) = ut, with the centers
// e_w, e_c of level k and e_tw, e_t of level k+1 around it and w_t, w_tw at
// the face; dzh = dzhi[k+1].
template <typename T>
__device__ __forceinline__ SmagFace<T> smag_u_zface(T e_w, T e_c, T e_tw, T e_t, T ut, T uc, T w_t, T w_tw,
                                                    T dxi, T dzh)
{
    return {mean4(e_w, e_c, e_tw, e_t), tfma(ut - uc, dzh, (w_t - w_tw) * dxi)};
}

// v's face at z_{k+1/2}: e_s, e_c (level k), e_ts, e_t (level k+1), v(k+1) =
// vt, v(k) = vc, w_t, w_ts at the face; dzh = dzhi[k+1].
template <typename T>
__device__ __forceinline__ SmagFace<T> smag_v_zface(T e_s, T e_c, T e_ts, T e_t, T vt, T vc, T w_t, T w_ts,
                                                    T dyi, T dzh)
{
    return {mean4(e_s, e_c, e_ts, e_t), tfma(vt - vc, dzh, (w_t - w_ts) * dyi)};
}

// w's center value between w(k) = wc and w(k+1) = wt: e_c * (wt - wc).
template <typename T>
__device__ __forceinline__ T smag_w_zcenter(T e_c, T wt, T wc)
{
    return e_c * (wt - wc);
}

// The horizontal (x and y) stress terms of u, v and w at one point, summed
// as tx + ty.
template <typename T>
__device__ __forceinline__ T smag_u_xy(T uc, T ue, T uw, T un, T us, T v_n, T v_nw, T v_c, T v_w,
                                       T e_c, T e_w, T e_n, T e_nw, T e_s, T e_sw, T dxi, T dyi)
{
    const T tx = tfma(e_c, ue - uc, -(e_w * (uc - uw))) * (T(2) * dxi * dxi);
    const T en = mean4(e_w, e_c, e_nw, e_n);
    const T es = mean4(e_sw, e_s, e_w, e_c);
    const T gn = tfma(un - uc, dyi, (v_n - v_nw) * dxi), gs = tfma(uc - us, dyi, (v_c - v_w) * dxi);
    const T ty = tfma(en, gn, -(es * gs)) * dyi;
    return tx + ty;
}

template <typename T>
__device__ __forceinline__ T smag_v_xy(T vc, T ve, T vw, T vn, T vs, T u_e, T u_se, T u_c, T u_s,
                                       T e_c, T e_s, T e_e, T e_se, T e_w, T e_sw, T dxi, T dyi)
{
    const T ee = mean4(e_s, e_se, e_c, e_e);
    const T ew = mean4(e_sw, e_s, e_w, e_c);
    const T ge = tfma(ve - vc, dxi, (u_e - u_se) * dyi), gw = tfma(vc - vw, dxi, (u_c - u_s) * dyi);
    const T tx = tfma(ee, ge, -(ew * gw)) * dxi;
    const T ty = tfma(e_c, vn - vc, -(e_s * (vc - vs))) * (T(2) * dyi * dyi);
    return tx + ty;
}

template <typename T>
__device__ __forceinline__ T smag_w_xy(T wc, T we, T ww, T wn, T ws, T u_e, T u_be, T u_c, T u_b,
                                       T v_n, T v_bn, T v_c, T v_b,
                                       T e_c, T e_b, T e_e, T e_be, T e_w, T e_bw, T e_n, T e_bn, T e_s, T e_bs,
                                       T dxi, T dyi, T dzhik)
{
    const T ee = mean4(e_b, e_be, e_c, e_e);
    const T ew = mean4(e_bw, e_b, e_w, e_c);
    const T ge = tfma(we - wc, dxi, (u_e - u_be) * dzhik), gw = tfma(wc - ww, dxi, (u_c - u_b) * dzhik);
    const T tx = tfma(ee, ge, -(ew * gw)) * dxi;
    const T en = mean4(e_b, e_bn, e_c, e_n);
    const T es = mean4(e_bs, e_b, e_s, e_c);
    const T gn = tfma(wn - wc, dyi, (v_n - v_bn) * dzhik), gs = tfma(wc - ws, dyi, (v_c - v_b) * dzhik);
    const T ty = tfma(en, gn, -(es * gs)) * dyi;
    return tx + ty;
}

// Whole tendencies from the horizontal sum and the two vertical face values.
template <typename T>
__device__ __forceinline__ T smag_uv_total(T txy, SmagFace<T> top, SmagFace<T> bot, T dzik)
{
    const T tz = tfma(top.e, top.g, -(bot.e * bot.g)) * dzik;
    return txy + tz;
}

template <typename T>
__device__ __forceinline__ T smag_w_total(T txy, T top, T bot, T dzik, T dzikm1, T dzhik)
{
    const T tz = tfma(top, dzik, -(bot * dzikm1)) * (T(2) * dzhik);
    return txy + tz;
}

// u at (xh_i, y_j, z_k).  v_n/v_nw: v(i, j+1), v(i-1, j+1); v_c/v_w: v(i, j),
// v(i-1, j); w_t/w_tw: w(i, k+1), w(i-1, k+1); w_c/w_w: w(i, k), w(i-1, k).
template <typename T>
__device__ __forceinline__ T smag_u(T uc, T ue, T uw, T un, T us, T ut, T ub,
                                    T v_n, T v_nw, T v_c, T v_w,
                                    T w_t, T w_tw, T w_c, T w_w,
                                    T e_c, T e_w, T e_n, T e_nw, T e_s, T e_sw, T e_t, T e_tw, T e_b, T e_bw,
                                    T dxi, T dyi, T dzik, T dzhik, T dzhik1)
{
    const T txy = smag_u_xy(uc, ue, uw, un, us, v_n, v_nw, v_c, v_w, e_c, e_w, e_n, e_nw, e_s, e_sw, dxi, dyi);
    return smag_uv_total(txy, smag_u_zface(e_w, e_c, e_tw, e_t, ut, uc, w_t, w_tw, dxi, dzhik1),
                         smag_u_zface(e_bw, e_b, e_w, e_c, uc, ub, w_c, w_w, dxi, dzhik), dzik);
}

// v at (x_i, yh_j, z_k).  u_e/u_se: u(i+1, j), u(i+1, j-1); u_c/u_s: u(i, j),
// u(i, j-1); w_t/w_ts: w(j, k+1), w(j-1, k+1); w_c/w_s: w(j, k), w(j-1, k).
template <typename T>
__device__ __forceinline__ T smag_v(T vc, T ve, T vw, T vn, T vs, T vt, T vb,
                                    T u_e, T u_se, T u_c, T u_s,
                                    T w_t, T w_ts, T w_c, T w_s,
                                    T e_c, T e_s, T e_e, T e_se, T e_w, T e_sw, T e_t, T e_ts, T e_b, T e_bs,
                                    T dxi, T dyi, T dzik, T dzhik, T dzhik1)
{
    const T txy = smag_v_xy(vc, ve, vw, vn, vs, u_e, u_se, u_c, u_s, e_c, e_s, e_e, e_se, e_w, e_sw, dxi, dyi);
    return smag_uv_total(txy, smag_v_zface(e_s, e_c, e_ts, e_t, vt, vc, w_t, w_ts, dyi, dzhik1),
                         smag_v_zface(e_bs, e_b, e_s, e_c, vc, vb, w_c, w_s, dyi, dzhik), dzik);
}

// w at (x_i, y_j, zh_k).  u_e/u_be: u(i+1, k), u(i+1, k-1); u_c/u_b: u(i, k),
// u(i, k-1); v_n/v_bn: v(j+1, k), v(j+1, k-1); v_c/v_b: v(j, k), v(j, k-1).
template <typename T>
__device__ __forceinline__ T smag_w(T wc, T we, T ww, T wn, T ws, T wt, T wb,
                                    T u_e, T u_be, T u_c, T u_b,
                                    T v_n, T v_bn, T v_c, T v_b,
                                    T e_c, T e_b, T e_e, T e_be, T e_w, T e_bw, T e_n, T e_bn, T e_s, T e_bs,
                                    T dxi, T dyi, T dzik, T dzikm1, T dzhik)
{
    const T txy = smag_w_xy(wc, we, ww, wn, ws, u_e, u_be, u_c, u_b, v_n, v_bn, v_c, v_b, e_c, e_b, e_e, e_be, e_w,
                            e_bw, e_n, e_bn, e_s, e_bs, dxi, dyi, dzhik);
    return smag_w_total(txy, smag_w_zcenter(e_c, wt, wc), smag_w_zcenter(e_b, wc, wb), dzik, dzikm1, dzhik);
}

// ---------------------------------------------------------------------------
// default configuration: one thread per point, 256 threads along x, blocks
// unravelled x, then y, then z (the paper's default launch).
// ---------------------------------------------------------------------------

// Load level l of a column at c0 + l*ks, or 0 outside [0, ktot+1].
template <typename T>
__device__ __forceinline__ T col_at(const T *p, int64_t c0, int64_t ks, int l, int ktot)
{
    return (l >= 0 && l <= ktot + 1) ? p[c0 + (int64_t)l * ks] : T(0);
}

template <typename T>
__device__ __forceinline__ T advec_u_2i5_at(const StencilArgs<T> &a, int i, int j, int k)
{
    const int64_t js = a.js, ks = a.ks;
    const int64_t c = a.off + i + j * js + (int64_t)k * ks;
    const T *u = a.u, *v = a.v, *w = a.w;
    // x faces between u_i, u_i+1 and between u_i-1, u_i
    const T fe = flux5(mid(u[c], u[c + 1]), u[c - 2], u[c - 1], u[c], u[c + 1], u[c + 2], u[c + 3]);
    const T fw = flux5(mid(u[c - 1], u[c]), u[c - 3], u[c - 2], u[c - 1], u[c], u[c + 1], u[c + 2]);
    // y faces between u_j, u_j+1 and between u_j-1, u_j
    const T fn = flux5(mid(v[c - 1 + js], v[c + js]), u[c - 2 * js], u[c - js], u[c], u[c + js], u[c + 2 * js],
                       u[c + 3 * js]);
    const T fs = flux5(mid(v[c - 1], v[c]), u[c - 3 * js], u[c - 2 * js], u[c - js], u[c], u[c + js], u[c + 2 * js]);
    // z faces k+1 and k
    const int64_t c0 = c - (int64_t)k * ks;
    const int kt = a.ktot;
    const T ft = flux_z_2i5(mid(w[c - 1 + ks], w[c + ks]), col_at(u, c0, ks, k - 2, kt), col_at(u, c0, ks, k - 1, kt),
                            col_at(u, c0, ks, k, kt), col_at(u, c0, ks, k + 1, kt), col_at(u, c0, ks, k + 2, kt),
                            col_at(u, c0, ks, k + 3, kt), k + 1, kt);
    const T fb = flux_z_2i5(mid(w[c - 1], w[c]), col_at(u, c0, ks, k - 3, kt), col_at(u, c0, ks, k - 2, kt),
                            col_at(u, c0, ks, k - 1, kt), col_at(u, c0, ks, k, kt), col_at(u, c0, ks, k + 1, kt),
                            col_at(u, c0, ks, k + 2, kt), k, kt);
    return advec_2i5_combine(fe, fw, fn, fs, ft, fb, a.dxi, a.dyi, a.dzi[k]);
}

template <typename T>
__global__ __launch_bounds__(256) void advec_u_2i5_plain(StencilArgs<T> a)
{
    unsigned b = blockIdx.x;
    const int bx = b % a.nbx;
    b /= a.nbx;
    const int j = 1 + (int)(b % a.jtot);
    const int k = 1 + (int)(b / a.jtot);
    const int i = 1 + bx * 256 + (int)threadIdx.x;
    if (i > a.itot) return;
    const int64_t c = a.off + i + j * a.js + (int64_t)k * a.ks;
    a.ut[c] = a.ut[c] + advec_u_2i5_at(a, i, j, k);
}

template <typename T>
__global__ __launch_bounds__(256) void diff_smag_plain(StencilArgs<T> a)
{
    unsigned b = blockIdx.x;
    const int bx = b % a.nbx;
    b /= a.nbx;
    const int j = 1 + (int)(b % a.jtot);
    const int k = 1 + (int)(b / a.jtot);
    const int i = 1 + bx * 256 + (int)threadIdx.x;
    if (i > a.itot) return;
    const int64_t js = a.js, ks = a.ks;
    const int64_t c = a.off + i + j * js + (int64_t)k * ks;
    const T *u = a.u, *v = a.v, *w = a.w, *e = a.evisc;
    const T dxi = a.dxi, dyi = a.dyi, dzik = a.dzi[k], dzhik = a.dzhi[k], dzhik1 = a.dzhi[k + 1];
    a.ut[c] = a.ut[c] + smag_u<T>(u[c], u[c + 1], u[c - 1], u[c + js], u[c - js], u[c + ks], u[c - ks],
                                  v[c + js], v[c - 1 + js], v[c], v[c - 1],
                                  w[c + ks], w[c - 1 + ks], w[c], w[c - 1],
                                  e[c], e[c - 1], e[c + js], e[c - 1 + js], e[c - js], e[c - 1 - js],
                                  e[c + ks], e[c - 1 + ks], e[c - ks], e[c - 1 - ks], dxi, dyi, dzik, dzhik, dzhik1);
    a.vt[c] = a.vt[c] + smag_v<T>(v[c], v[c + 1], v[c - 1], v[c + js], v[c - js], v[c + ks], v[c - ks],
                                  u[c + 1], u[c + 1 - js], u[c], u[c - js],
                                  w[c + ks], w[c - js + ks], w[c], w[c - js],
                                  e[c], e[c - js], e[c + 1], e[c + 1 - js], e[c - 1], e[c - 1 - js],
                                  e[c + ks], e[c - js + ks], e[c - ks], e[c - js - ks], dxi, dyi, dzik, dzhik, dzhik1);
    if (k >= a.kw0)
        a.wt[c] = a.wt[c] + smag_w<T>(w[c], w[c + 1], w[c - 1], w[c + js], w[c - js], w[c + ks], w[c - ks],
                                      u[c + 1], u[c + 1 - ks], u[c], u[c - ks],
                                      v[c + js], v[c + js - ks], v[c], v[c - ks],
                                      e[c], e[c - ks], e[c + 1], e[c + 1 - ks], e[c - 1], e[c - 1 - ks],
                                      e[c + js], e[c + js - ks], e[c - js], e[c - js - ks], dxi, dyi, dzik,
                                      a.dzi[k - 1], dzhik);
}

}  // namespace kl
