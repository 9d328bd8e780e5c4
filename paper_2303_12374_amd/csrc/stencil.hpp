// Device code of the two tendency kernels (advec_u, diff_uvw) for gfx950.
//
// All configurations share the per-point arithmetic below, compiled with
// -ffp-contract=off, so every configuration (default, z-marching, batched,
// served) produces bitwise-identical tendencies.
//
// Index layout: element (i, j, k) at off + i + j*js + k*ks, interior
// [1, itot] x [1, jtot] x [1, ktot], at least one ghost cell per side.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace kl {

// Arguments of every tendency kernel (passed by value).
template <typename T>
struct StencilArgs {
    int itot, jtot, ktot;
    int kw0;                 // first w level advanced: 2 with z walls, 1 periodic
    int bc;                  // KL_BC_* (used by the batched Euler update)
    int64_t off, js, ks;
    T dxi, dyi, visc;
    T dt;                    // time step of the fused step kernels
    const T *__restrict__ dzi;
    const T *__restrict__ dzhi;
    T *ut, *vt, *wt;
    const T *u, *v, *w;
    int nbx, nby, nbz;       // tiles per axis (1-D grid unravelled x fastest)
    const T *evisc;          // eddy viscosity at cell centers (diff_smag only)
};

// The batched kernels read their descriptors from memory, so the compiler
// cannot see that the pointers in them address global memory and would use
// flat instructions (counted as both vector-memory and LDS operations, and
// waited for conservatively).  Passing each pointer through the global
// address space states the fact; the compiler's address-space inference then
// selects global loads and stores for every access derived from it.
template <typename T>
__device__ __forceinline__ T *as_global(T *p)
{
    typedef __attribute__((address_space(1))) T GT;
    return (T *)(GT *)(uintptr_t)p;
}

template <typename T>
__device__ __forceinline__ StencilArgs<T> global_args(const StencilArgs<T> &in)
{
    StencilArgs<T> a = in;
    a.u = as_global(a.u);
    a.v = as_global(a.v);
    a.w = as_global(a.w);
    a.ut = as_global(a.ut);
    a.vt = as_global(a.vt);
    a.wt = as_global(a.wt);
    a.evisc = as_global(a.evisc);
    return a;
}

// ---------------------------------------------------------------------------
// per-point arithmetic
// ---------------------------------------------------------------------------

// Fused multiply-add and absolute value of the field type.  The per-point
// functions use explicit fused operations where they save instructions (the
// tiles are partly bound by their arithmetic); every configuration calls the
// same functions with the same operands, and the rest of the code is built
// with -ffp-contract=off, so all configurations still agree bitwise.
__device__ __forceinline__ float tfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double tfma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float tabs(float a) { return __builtin_fabsf(a); }
__device__ __forceinline__ double tabs(double a) { return __builtin_fabs(a); }

// advec_u tendency at one u point.  Arguments are named by their offset from
// the point: u at (i,j,k) and its six neighbours, v at (i-1..i, j..j+1, k),
// w at (i-1..i, j, k..k+1).  Every face value is a midpoint (a+b)/2; each
// flux is a product of two of them, so the two factors 1/2 are applied once,
// exactly, as 1/4 of the grid factor (a power-of-two scaling rounds
// nothing).  The x flux's sums and squares are functions of the face only,
// so a lane's neighbouring points share them.
template <typename T>
__device__ __forceinline__ T advec_u_point(T uc, T ue, T uw, T un_, T us_, T ut_, T ub_,
                                           T v_w, T v_c, T v_nw, T v_n,
                                           T w_w, T w_c, T w_tw, T w_t,
                                           T dxi, T dyi, T dzik)
{
    const T sx_hi = uc + ue;
    const T sx_lo = uw + uc;
    const T adv_x = (sx_hi * sx_hi - sx_lo * sx_lo) * (T(0.25) * dxi);
    const T adv_y = tfma(v_nw + v_n, uc + un_, -((v_w + v_c) * (us_ + uc))) * (T(0.25) * dyi);
    const T adv_z = tfma(w_tw + w_t, uc + ut_, -((w_w + w_c) * (ub_ + uc)));
    return -tfma(adv_z, T(0.25) * dzik, adv_x + adv_y);
}

// Horizontal part of the Laplacian (phi_e - 2 phi + phi_w) dxi^2 + (phi_n -
// 2 phi + phi_s) dyi^2; phi_e - 2 phi is one fused operation (exact 2 phi).
template <typename T>
__device__ __forceinline__ T lap_xy(T c, T e, T w, T n, T s, T dxi2, T dyi2)
{
    return tfma(tfma(T(-2), c, e) + w, dxi2, (tfma(T(-2), c, n) + s) * dyi2);
}

// diff tendency of u or v at a cell-center level k: the vertical term takes
// face gradients with dzhi[k+1], dzhi[k] and divides by dz_k.
template <typename T>
__device__ __forceinline__ T diff_c_point(T c, T e, T w, T n, T s, T t, T b,
                                          T dxi2, T dyi2, T dzi_k, T dzhi_k1, T dzhi_k, T visc)
{
    const T fz = tfma(t - c, dzhi_k1, -((c - b) * dzhi_k)) * dzi_k;
    return visc * (lap_xy(c, e, w, n, s, dxi2, dyi2) + fz);
}

// diff tendency of w at face level k: center gradients with dzi[k], dzi[k-1],
// divided by dzh_k.
template <typename T>
__device__ __forceinline__ T diff_w_point(T c, T e, T w, T n, T s, T t, T b,
                                          T dxi2, T dyi2, T dzi_k, T dzi_km1, T dzhi_k, T visc)
{
    const T fz = tfma(t - c, dzi_k, -((c - b) * dzi_km1)) * dzhi_k;
    return visc * (lap_xy(c, e, w, n, s, dxi2, dyi2) + fz);
}

// Forward-Euler update of one value: f + dt * ft, one fused operation.
template <typename T>
__device__ __forceinline__ T euler_value(T f, T dt, T ft)
{
    return tfma(dt, ft, f);
}

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

template <typename T, int N> struct VecOf;
template <> struct VecOf<float, 2> { typedef float type __attribute__((ext_vector_type(2))); };
template <> struct VecOf<float, 4> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct VecOf<double, 2> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct VecOf<double, 4> { typedef double type __attribute__((ext_vector_type(4))); };

// Load N consecutive elements starting at an N*sizeof(T)-aligned address.
template <typename T, int N>
__device__ __forceinline__ void vload(T (&d)[N], const T *p)
{
    if constexpr (N == 1) {
        d[0] = *p;
    } else {
        typedef typename VecOf<T, N>::type V;
        const V x = *reinterpret_cast<const V *>(p);
#pragma unroll
        for (int n = 0; n < N; ++n) d[n] = x[n];
    }
}

template <typename T, int N>
__device__ __forceinline__ void vstore(T *p, const T (&s)[N])
{
    if constexpr (N == 1) {
        *p = s[0];
    } else {
        typedef typename VecOf<T, N>::type V;
        V x;
#pragma unroll
        for (int n = 0; n < N; ++n) x[n] = s[n];
        *reinterpret_cast<V *>(p) = x;
    }
}

// Streaming (non-temporal) variants for data touched exactly once.
template <typename T, int N>
__device__ __forceinline__ void vload_nt(T (&d)[N], const T *p)
{
    if constexpr (N == 1) {
        d[0] = __builtin_nontemporal_load(p);
    } else {
        typedef typename VecOf<T, N>::type V;
        const V x = __builtin_nontemporal_load(reinterpret_cast<const V *>(p));
#pragma unroll
        for (int n = 0; n < N; ++n) d[n] = x[n];
    }
}

template <typename T, int N>
__device__ __forceinline__ void vstore_nt(T *p, const T (&s)[N])
{
    if constexpr (N == 1) {
        __builtin_nontemporal_store(s[0], p);
    } else {
        typedef typename VecOf<T, N>::type V;
        V x;
#pragma unroll
        for (int n = 0; n < N; ++n) x[n] = s[n];
        __builtin_nontemporal_store(x, reinterpret_cast<V *>(p));
    }
}

// Tendency load/store: cached, or streaming when NT is set.
template <int NT, typename T, int N>
__device__ __forceinline__ void tload(T (&d)[N], const T *p)
{
    if constexpr (NT) vload_nt<T, N>(d, p); else vload<T, N>(d, p);
}

template <int NT, typename T, int N>
__device__ __forceinline__ void tstore(T *p, const T (&s)[N])
{
    if constexpr (NT) vstore_nt<T, N>(p, s); else vstore<T, N>(p, s);
}

// A read of a vertical metric (dzi, dzhi) at a wave-uniform level k.  The
// metrics are never written while a kernel runs, so they are read through the
// constant address space: the load is a scalar-memory read, counted apart
// from the vector loads of the fields, and waiting for it does not also wait
// for the prefetched levels in flight.
template <typename T>
__device__ __forceinline__ T kload(const T *p, int k)
{
    typedef __attribute__((address_space(4))) const T CT;
    return reinterpret_cast<CT *>(reinterpret_cast<uintptr_t>(p))[k];
}

// Wait for every outstanding vector-memory load of this wave (s_waitcnt with
// vmcnt = 0 and the export and LDS counters left at their maxima; GFX9
// encoding: vmcnt in bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8).  Called
// once at the end of a z-march prologue: the loop is then entered with no
// load in flight, so the compiler's wait placement inside the loop need not
// allow for the prologue's loads still being outstanding on the first pass.
__device__ __forceinline__ void vm_drain()
{
    __builtin_amdgcn_s_waitcnt(0x0F70);
}

// Mark the values as read here (an empty asm statement with the registers as
// inputs).  The compiler then waits for the loads that filled them at this
// point on every path, even where their arithmetic was moved into a branch
// (a value used only by a predicated store).  A prefetched register that is
// left pending on one path makes the compiler's wait placement merge the
// paths conservatively and wait for every outstanding memory operation
// before the register is next reused, which defeats the prefetch.
template <typename T, int N>
__device__ __forceinline__ void settle(const T (&v)[N])
{
#pragma unroll
    for (int n = 0; n < N; ++n) asm volatile("" ::"v"(v[n]));
}

// p advanced by a byte offset.  Written as a uniform base plus a 32-bit
// per-lane offset, a global access takes its base from scalar registers
// (global_load ... v_off, s[base]) and needs no 64-bit vector address math.
template <typename T>
__device__ __forceinline__ T *boff(T *p, uint32_t bytes)
{
    typedef typename std::conditional<std::is_const<T>::value, const char, char>::type C;
    return reinterpret_cast<T *>(reinterpret_cast<C *>(p) + bytes);
}

// The row of the block a wave works on: threadIdx.y is the same in all lanes
// of a wave (the blocks are 64 lanes wide), and saying so lets the compiler
// keep everything derived from it in scalar registers.
__device__ __forceinline__ int wave_row()
{
    return __builtin_amdgcn_readfirstlane((int)threadIdx.y);
}

// Field load: cached, or streaming when NT >= 2.
template <int NT, typename T, int N>
__device__ __forceinline__ void fload(T (&d)[N], const T *p)
{
    if constexpr (NT >= 2) vload_nt<T, N>(d, p); else vload<T, N>(d, p);
}

// Map a hardware workgroup id to a logical tile id so that the tiles each of
// the 8 XCDs receives (the dispatcher deals workgroups to XCDs round robin)
// are contiguous in the logical x-fastest order: neighbouring tiles, which
// share halo rows, then run under the same L2.
__device__ __forceinline__ unsigned xcd_remap(unsigned b, unsigned nb)
{
    const unsigned q = nb >> 3, r = nb & 7u;
    const unsigned x = b & 7u, local = b >> 3;
    return x * q + (x < r ? x : r) + local;
}

// ---------------------------------------------------------------------------
// default configuration: one thread per point, 256 threads along x,
// 1-D list of blocks unravelled x, then y, then z (the paper's default).
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void advec_u_plain(StencilArgs<T> a)
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
    const T *u = a.u, *v = a.v, *w = a.w;
    const T t = advec_u_point<T>(u[c], u[c + 1], u[c - 1], u[c + js], u[c - js], u[c + ks], u[c - ks],
                                 v[c - 1], v[c], v[c - 1 + js], v[c + js],
                                 w[c - 1], w[c], w[c - 1 + ks], w[c + ks],
                                 a.dxi, a.dyi, a.dzi[k]);
    a.ut[c] = a.ut[c] + t;
}

template <typename T>
__global__ __launch_bounds__(256) void diff_uvw_plain(StencilArgs<T> a)
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
    a.ut[c] = a.ut[c] + diff_c_point<T>(u[c], u[c + 1], u[c - 1], u[c + js], u[c - js], u[c + ks],
                                        u[c - ks], dxi2, dyi2, dzik, dzhik1, dzhik, a.visc);
    a.vt[c] = a.vt[c] + diff_c_point<T>(v[c], v[c + 1], v[c - 1], v[c + js], v[c - js], v[c + ks],
                                        v[c - ks], dxi2, dyi2, dzik, dzhik1, dzhik, a.visc);
    if (k >= a.kw0)
        a.wt[c] = a.wt[c] + diff_w_point<T>(w[c], w[c + 1], w[c - 1], w[c + js], w[c - js], w[c + ks],
                                            w[c - ks], dxi2, dyi2, dzik, a.dzi[k - 1], dzhik, a.visc);
}

// ---------------------------------------------------------------------------
// z-marching configuration: each thread owns VX consecutive x points of one
// row and walks KB levels upward.  The z neighbours of the center column
// stay in registers from level to level; x neighbours at the vector edges
// and y neighbours come from global memory (L1/L2 hits: they are the center
// data of the neighbouring lanes and rows of the same workgroup).  Block =
// BX x BY threads, tile = BX*VX x BY x KB points.  XCD selects the
// XCD-contiguous tile order.
// ---------------------------------------------------------------------------

// Tile order.  XCD = 0: hardware order (x fastest, then y, then z);
// XCD = 1: each XCD gets one contiguous range of the whole tile list;
// XCD = 2: each XCD gets one contiguous range of every z slab of tiles (when
// the slab holds a multiple of 8 tiles), so all XCDs sweep the same levels
// together while neighbouring rows stay under one L2; XCD = 3: as 2 with the
// slabs taken from the top down, so a kernel that follows one sweeping
// upward starts on the levels still held in the memory-side cache.
template <int BX, int BY, int XCD>
__device__ __forceinline__ void tile_of(int nbx, int nby, int nbz, int &tx, int &ty, int &tz)
{
    unsigned b = blockIdx.x;
    if (XCD == 1) b = xcd_remap(b, (unsigned)(nbx * nby * nbz));
    if (XCD >= 2) {
        const unsigned S = (unsigned)(nbx * nby);
        if ((S & 7u) == 0) b = (b / S) * S + xcd_remap(b % S, S);
    }
    tx = (int)(b % (unsigned)nbx);
    b /= (unsigned)nbx;
    ty = (int)(b % (unsigned)nby);
    tz = (int)(b / (unsigned)nby);
    if (XCD == 3) tz = nbz - 1 - tz;  // top slab first
}

template <typename T, int VX, int BX, int BY, int KB, int XCD, int NT = 0, int WPE = 1>
__global__ __launch_bounds__(BX *BY, WPE) void advec_u_zc(StencilArgs<T> a)
{
    int tx, ty, tz;
    tile_of<BX, BY, XCD>(a.nbx, a.nby, a.nbz, tx, ty, tz);
    const int i0 = 1 + (tx * BX + (int)threadIdx.x) * VX;
    const int j = 1 + ty * BY + (int)threadIdx.y;
    if (i0 > a.itot || j > a.jtot) return;
    const int k0 = 1 + tz * KB;
    const int k1 = min(k0 + KB, a.ktot + 1);
    const int64_t js = a.js, ks = a.ks;
    const T dxi = a.dxi, dyi = a.dyi;

    const int64_t c0 = a.off + i0 + j * js + (int64_t)k0 * ks;
    const T *pu = a.u + c0, *pv = a.v + c0, *pw = a.w + c0;
    T *put = a.ut + c0;

    // registers of the center column
    T ub[VX], uc[VX], ucw, uce, wc[VX], wcw;
    vload<T, VX>(ub, pu - ks);
    vload<T, VX>(uc, pu);
    ucw = pu[-1];
    uce = pu[VX];
    vload<T, VX>(wc, pw);
    wcw = pw[-1];

    for (int k = k0; k < k1; ++k) {
        T utp[VX], utw, ute, un[VX], us[VX], vc[VX], vcw, vn[VX], vnw, wt[VX], wtw, tt[VX];
        fload<NT, T, VX>(utp, pu + ks);
        utw = pu[ks - 1];
        ute = pu[ks + VX];
        vload<T, VX>(un, pu + js);
        vload<T, VX>(us, pu - js);
        fload<NT, T, VX>(vc, pv);
        vcw = pv[-1];
        vload<T, VX>(vn, pv + js);
        vnw = pv[js - 1];
        fload<NT, T, VX>(wt, pw + ks);
        wtw = pw[ks - 1];
        tload<NT, T, VX>(tt, put);
        const T dzik = a.dzi[k];
#pragma unroll
        for (int n = 0; n < VX; ++n) {
            const T uw = n == 0 ? ucw : uc[n - 1];
            const T ue = n == VX - 1 ? uce : uc[n + 1];
            const T v_w = n == 0 ? vcw : vc[n - 1];
            const T v_nw = n == 0 ? vnw : vn[n - 1];
            const T w_w = n == 0 ? wcw : wc[n - 1];
            const T w_tw = n == 0 ? wtw : wt[n - 1];
            tt[n] = tt[n] + advec_u_point<T>(uc[n], ue, uw, un[n], us[n], utp[n], ub[n],
                                             v_w, vc[n], v_nw, vn[n], w_w, wc[n], w_tw, wt[n],
                                             dxi, dyi, dzik);
        }
        tstore<NT, T, VX>(put, tt);
#pragma unroll
        for (int n = 0; n < VX; ++n) {
            ub[n] = uc[n];
            uc[n] = utp[n];
            wc[n] = wt[n];
        }
        ucw = utw;
        uce = ute;
        wcw = wtw;
        pu += ks;
        pv += ks;
        pw += ks;
        put += ks;
    }
}

template <typename T, int VX, int BX, int BY, int KB, int XCD, int NT = 0, int WPE = 1>
__global__ __launch_bounds__(BX *BY, WPE) void diff_uvw_zc(StencilArgs<T> a)
{
    int tx, ty, tz;
    tile_of<BX, BY, XCD>(a.nbx, a.nby, a.nbz, tx, ty, tz);
    const int i0 = 1 + (tx * BX + (int)threadIdx.x) * VX;
    const int j = 1 + ty * BY + (int)threadIdx.y;
    if (i0 > a.itot || j > a.jtot) return;
    const int k0 = 1 + tz * KB;
    const int k1 = min(k0 + KB, a.ktot + 1);
    const int64_t js = a.js, ks = a.ks;
    const T dxi2 = a.dxi * a.dxi, dyi2 = a.dyi * a.dyi, visc = a.visc;
    const int kw0 = a.kw0;

    const int64_t c0 = a.off + i0 + j * js + (int64_t)k0 * ks;
    const T *pf[3] = {a.u + c0, a.v + c0, a.w + c0};
    T *pt[3] = {a.ut + c0, a.vt + c0, a.wt + c0};

    T fb[3][VX], fc[3][VX], fw[3], fe[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        vload<T, VX>(fb[f], pf[f] - ks);
        vload<T, VX>(fc[f], pf[f]);
        fw[f] = pf[f][-1];
        fe[f] = pf[f][VX];
    }

    for (int k = k0; k < k1; ++k) {
        const T dzik = a.dzi[k], dzikm1 = a.dzi[k - 1], dzhik = a.dzhi[k], dzhik1 = a.dzhi[k + 1];
        T ft[3][VX], ftw[3], fte[3];
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            const T *p = pf[f];
            fload<NT, T, VX>(ft[f], p + ks);
            ftw[f] = p[ks - 1];
            fte[f] = p[ks + VX];
            T fn[VX], fs[VX], tt[VX];
            vload<T, VX>(fn, p + js);
            vload<T, VX>(fs, p - js);
            const bool active = f < 2 || k >= kw0;
            if (active) {
                tload<NT, T, VX>(tt, pt[f]);
#pragma unroll
                for (int n = 0; n < VX; ++n) {
                    const T w_ = n == 0 ? fw[f] : fc[f][n - 1];
                    const T e_ = n == VX - 1 ? fe[f] : fc[f][n + 1];
                    const T d = f < 2 ? diff_c_point<T>(fc[f][n], e_, w_, fn[n], fs[n], ft[f][n], fb[f][n],
                                                        dxi2, dyi2, dzik, dzhik1, dzhik, visc)
                                      : diff_w_point<T>(fc[f][n], e_, w_, fn[n], fs[n], ft[f][n], fb[f][n],
                                                        dxi2, dyi2, dzik, dzikm1, dzhik, visc);
                    tt[n] = tt[n] + d;
                }
                tstore<NT, T, VX>(pt[f], tt);
            }
        }
#pragma unroll
        for (int f = 0; f < 3; ++f) {
#pragma unroll
            for (int n = 0; n < VX; ++n) {
                fb[f][n] = fc[f][n];
                fc[f][n] = ft[f][n];
            }
            fw[f] = ftw[f];
            fe[f] = fte[f];
            pf[f] += ks;
            pt[f] += ks;
        }
    }
}

}  // namespace kl
