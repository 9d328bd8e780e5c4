// Launchers of the tendency-kernel configurations and the macro that
// builds a registry list.  Included by one translation unit per field type.
#pragma once

#include "kl_internal.hpp"
#include "stencil.hpp"
#include "stencil_zl.hpp"
#include "stencil_step.hpp"
#include "stencil_les.hpp"
#include "stencil_les_zl.hpp"

namespace kl {

inline unsigned cdivu(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

template <typename T>
StencilArgs<T> device_args(const HostArgs &h)
{
    StencilArgs<T> a;
    a.itot = h.itot;
    a.jtot = h.jtot;
    a.ktot = h.ktot;
    a.kw0 = h.kw0;
    a.bc = h.bc;
    a.off = h.off;
    a.js = h.js;
    a.ks = h.ks;
    a.dxi = (T)h.dxi;
    a.dyi = (T)h.dyi;
    a.visc = (T)h.visc;
    a.dt = (T)h.dt;
    a.dzi = (const T *)h.dzi;
    a.dzhi = (const T *)h.dzhi;
    a.ut = (T *)h.ut;
    a.vt = (T *)h.vt;
    a.wt = (T *)h.wt;
    a.u = (const T *)h.u;
    a.v = (const T *)h.v;
    a.w = (const T *)h.w;
    a.nbx = a.nby = a.nbz = 1;
    a.evisc = (const T *)h.evisc;
    return a;
}

// 1-D grids only: total threads must fit the 32-bit grid size.
inline bool grid_fits(uint64_t blocks, uint64_t threads) { return blocks * threads < (1ull << 32); }

template <typename T, int KERNEL>
hipError_t launch_plain(const HostArgs &h, hipStream_t s)
{
    StencilArgs<T> a = device_args<T>(h);
    a.nbx = (int)cdivu(h.itot, 256);
    a.nby = h.jtot;
    a.nbz = h.ktot;
    const uint64_t nb = (uint64_t)a.nbx * a.nby * a.nbz;
    if (!grid_fits(nb, 256)) return hipErrorInvalidConfiguration;
    if (KERNEL == KL_KERNEL_ADVEC_U)
        hipLaunchKernelGGL(advec_u_plain<T>, dim3((unsigned)nb), dim3(256), 0, s, a);
    else if (KERNEL == KL_KERNEL_DIFF_UVW)
        hipLaunchKernelGGL(diff_uvw_plain<T>, dim3((unsigned)nb), dim3(256), 0, s, a);
    else if (KERNEL == KL_KERNEL_ADVEC_U_2I5)
        hipLaunchKernelGGL(advec_u_2i5_plain<T>, dim3((unsigned)nb), dim3(256), 0, s, a);
    else if (KERNEL == KL_KERNEL_ADVEC_DIFF)
        hipLaunchKernelGGL(advec_diff_plain<T>, dim3((unsigned)nb), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(diff_smag_plain<T>, dim3((unsigned)nb), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename T, int KERNEL, int VX, int BX, int BY, int KB, int XCD, int NT = 0, int WPE = 1>
hipError_t launch_zc(const HostArgs &h, hipStream_t s)
{
    StencilArgs<T> a = device_args<T>(h);
    a.nbx = (int)cdivu(h.itot, (int64_t)BX * VX);
    a.nby = (int)cdivu(h.jtot, BY);
    a.nbz = (int)cdivu(h.ktot, KB);
    const uint64_t nb = (uint64_t)a.nbx * a.nby * a.nbz;
    if (!grid_fits(nb, BX * BY)) return hipErrorInvalidConfiguration;
    if (KERNEL == KL_KERNEL_ADVEC_U)
        hipLaunchKernelGGL((advec_u_zc<T, VX, BX, BY, KB, XCD, NT, WPE>), dim3((unsigned)nb), dim3(BX, BY), 0, s, a);
    else
        hipLaunchKernelGGL((diff_uvw_zc<T, VX, BX, BY, KB, XCD, NT, WPE>), dim3((unsigned)nb), dim3(BX, BY), 0, s, a);
    return hipGetLastError();
}

template <typename T, int KERNEL, int VX, int BY, int KB, int XCD, int NT = 0, int WPE = 1>
hipError_t launch_zl(const HostArgs &h, hipStream_t s)
{
    StencilArgs<T> a = device_args<T>(h);
    a.nbx = (int)cdivu(h.itot, (int64_t)64 * VX);
    a.nby = (int)cdivu(h.jtot, BY);
    a.nbz = (int)cdivu(h.ktot, KB);
    const uint64_t nb = (uint64_t)a.nbx * a.nby * a.nbz;
    if (!grid_fits(nb, 64 * BY)) return hipErrorInvalidConfiguration;
    if (KERNEL == KL_KERNEL_ADVEC_U)
        hipLaunchKernelGGL((advec_u_zl<T, VX, BY, KB, XCD, NT, WPE>), dim3((unsigned)nb), dim3(64, BY), 0, s, a);
    else
        hipLaunchKernelGGL((diff_uvw_zl<T, VX, BY, KB, XCD, NT, WPE>), dim3((unsigned)nb), dim3(64, BY), 0, s, a);
    return hipGetLastError();
}

template <typename T, int KERNEL, int VX, int BY, int KB, int NT = 0, int WPE = 1>
hipError_t launch_zl_batch(const void *descs, const void *tiles, int ntiles, int nblocks, int *queue, hipStream_t s)
{
    if (KERNEL == KL_KERNEL_ADVEC_U)
        hipLaunchKernelGGL((advec_u_zl_batch<T, VX, BY, KB, NT, WPE>), dim3(nblocks), dim3(64, BY), 0, s,
                           (const StencilArgs<T> *)descs, (const int4 *)tiles, ntiles, queue);
    else
        hipLaunchKernelGGL((diff_uvw_zl_batch<T, VX, BY, KB, NT, WPE>), dim3(nblocks), dim3(64, BY), 0, s,
                           (const StencilArgs<T> *)descs, (const int4 *)tiles, ntiles, queue);
    return hipGetLastError();
}

template <typename T, int KERNEL, int VX, int BY, int KB, int NT = 0, int WPE = 1>
int zl_batch_occupancy()
{
    int n = 0;
    hipError_t e;
    if (KERNEL == KL_KERNEL_ADVEC_U)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, advec_u_zl_batch<T, VX, BY, KB, NT, WPE>, 64 * BY, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, diff_uvw_zl_batch<T, VX, BY, KB, NT, WPE>, 64 * BY, 0);
    return e == hipSuccess && n > 0 ? n : 1;
}

template <typename T, int VX, int BY, int KB, int XCD, int NT = 0, int WPE = 1, int MODE = FUSE_STEP>
hipError_t launch_step(const HostArgs &h, hipStream_t s)
{
    StencilArgs<T> a = device_args<T>(h);
    a.nbx = (int)cdivu(h.itot, (int64_t)64 * VX);
    a.nby = (int)cdivu(h.jtot, BY);
    a.nbz = (int)cdivu(h.ktot, KB);
    const uint64_t nb = (uint64_t)a.nbx * a.nby * a.nbz;
    if (!grid_fits(nb, 64 * BY)) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((step_zl<T, VX, BY, KB, XCD, NT, WPE, MODE>), dim3((unsigned)nb), dim3(64, BY), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && (MODE & FUSE_NOYZ)) e = launch_fill_yz_images(h, h.ut, h.vt, h.wt, s);
    return e;
}

template <typename T, int VX, int BY, int KB, int NT = 0, int WPE = 1, int MODE = FUSE_STEP>
hipError_t launch_step_batch(const void *descs, const void *tiles, int ntiles, int nblocks, int *queue,
                             hipStream_t s)
{
    hipLaunchKernelGGL((step_zl_batch<T, VX, BY, KB, NT, WPE, MODE>), dim3(nblocks), dim3(64, BY), 0, s,
                       (const StencilArgs<T> *)descs, (const int4 *)tiles, ntiles, queue);
    return hipGetLastError();
}

template <typename T, int VX, int BY, int KB, int NT = 0, int WPE = 1, int MODE = FUSE_STEP>
int step_batch_occupancy()
{
    int n = 0;
    const hipError_t e =
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_zl_batch<T, VX, BY, KB, NT, WPE, MODE>, 64 * BY, 0);
    return e == hipSuccess && n > 0 ? n : 1;
}

// diff_uvw as three single-component passes (u, then v, then w) of the LDS
// z-march: the same values and arithmetic, three read/write streams in
// flight at a time instead of nine.
template <typename T, int VX, int BY, int KB, int XCD, int NT = 0>
hipError_t launch_zl_split(const HostArgs &h, hipStream_t s)
{
    StencilArgs<T> a = device_args<T>(h);
    a.nbx = (int)cdivu(h.itot, (int64_t)64 * VX);
    a.nby = (int)cdivu(h.jtot, BY);
    a.nbz = (int)cdivu(h.ktot, KB);
    const uint64_t nb = (uint64_t)a.nbx * a.nby * a.nbz;
    if (!grid_fits(nb, 64 * BY)) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((diff_uvw_zl<T, VX, BY, KB, XCD, NT, 1, 1>), dim3((unsigned)nb), dim3(64, BY), 0, s, a);
    hipLaunchKernelGGL((diff_uvw_zl<T, VX, BY, KB, XCD, NT, 1, 2>), dim3((unsigned)nb), dim3(64, BY), 0, s, a);
    hipLaunchKernelGGL((diff_uvw_zl<T, VX, BY, KB, XCD, NT, 1, 4>), dim3((unsigned)nb), dim3(64, BY), 0, s, a);
    return hipGetLastError();
}

template <typename T, int VX, int BY, int KB, int XCD, int NT = 0, int WPE = 1, int PAIR = 0, int YS = 0>
hipError_t launch_advec5_zl(const HostArgs &h, hipStream_t s)
{
    StencilArgs<T> a = device_args<T>(h);
    a.nbx = (int)cdivu(h.itot, (int64_t)64 * VX);
    a.nby = (int)cdivu(h.jtot, BY);
    a.nbz = (int)cdivu(h.ktot, KB);
    const uint64_t nb = (uint64_t)a.nbx * a.nby * a.nbz;
    if (!grid_fits(nb, 64 * BY)) return hipErrorInvalidConfiguration;
    if (PAIR)
        hipLaunchKernelGGL((advec_u_2i5_zlp<T, VX, BY, KB, XCD, NT, WPE>), dim3((unsigned)nb), dim3(64, BY), 0, s, a);
    else
        hipLaunchKernelGGL((advec_u_2i5_zl<T, VX, BY, KB, XCD, NT, WPE, YS>), dim3((unsigned)nb), dim3(64, BY), 0, s,
                           a);
    return hipGetLastError();
}

template <typename T, int VX, int BY, int KB, int XCD, int NT = 0, int HL = 1>
hipError_t launch_advec5_zr(const HostArgs &h, hipStream_t s)
{
    StencilArgs<T> a = device_args<T>(h);
    a.nbx = (int)cdivu(h.itot, (int64_t)64 * VX);
    a.nby = (int)cdivu(h.jtot, BY);
    a.nbz = (int)cdivu(h.ktot, KB);
    const uint64_t nb = (uint64_t)a.nbx * a.nby * a.nbz;
    if (!grid_fits(nb, 64 * BY)) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((advec_u_2i5_zr<T, VX, BY, KB, XCD, NT, 1, HL>), dim3((unsigned)nb), dim3(64, BY), 0, s, a);
    return hipGetLastError();
}

template <typename T, int VX, int BY, int KB, int XCD, int NT = 0, int WPE = 1, int RING = 0>
hipError_t launch_smag_zl(const HostArgs &h, hipStream_t s)
{
    StencilArgs<T> a = device_args<T>(h);
    a.nbx = (int)cdivu(h.itot, (int64_t)64 * VX);
    a.nby = (int)cdivu(h.jtot, BY);
    a.nbz = (int)cdivu(h.ktot, KB);
    const uint64_t nb = (uint64_t)a.nbx * a.nby * a.nbz;
    if (!grid_fits(nb, 64 * BY)) return hipErrorInvalidConfiguration;
    if constexpr (RING)
        hipLaunchKernelGGL((diff_smag_zr<T, VX, BY, KB, XCD, NT, WPE>), dim3((unsigned)nb), dim3(64, BY), 0, s, a);
    else
        hipLaunchKernelGGL((diff_smag_zl<T, VX, BY, KB, XCD, NT, WPE>), dim3((unsigned)nb), dim3(64, BY), 0, s, a);
    return hipGetLastError();
}

}  // namespace kl

#define KL_STR2(x) #x
#define KL_STR(x) KL_STR2(x)

// One z-marching configuration entry.
#define KL_ZC(T, DT, KERN, VX, BX, BY, KB, XCD)                                                   \
    Variant{"zc_v" KL_STR(VX) "_b" KL_STR(BX) "x" KL_STR(BY) "_k" KL_STR(KB) "_x" KL_STR(XCD), \
            KERN, DT, FAMILY_ZC, VX, BX, BY, KB, XCD, &launch_zc<T, KERN, VX, BX, BY, KB, XCD>, nullptr, \
            nullptr}

#define KL_ZC_XCD(T, DT, KERN, VX, BX, BY, KB) \
    KL_ZC(T, DT, KERN, VX, BX, BY, KB, 0), KL_ZC(T, DT, KERN, VX, BX, BY, KB, 1)

#define KL_ZC_KB(T, DT, KERN, VX, BX, BY) \
    KL_ZC_XCD(T, DT, KERN, VX, BX, BY, 16), KL_ZC_XCD(T, DT, KERN, VX, BX, BY, 64)

#define KL_ZC_BLOCKS(T, DT, KERN, VX)                                           \
    KL_ZC_KB(T, DT, KERN, VX, 64, 1), KL_ZC_KB(T, DT, KERN, VX, 64, 4),          \
        KL_ZC_KB(T, DT, KERN, VX, 128, 2), KL_ZC_KB(T, DT, KERN, VX, 256, 1)

// One LDS-staged z-marching configuration entry (block 64 x BY).
#define KL_ZL(T, DT, KERN, VX, BY, KB, XCD)                                                   \
    Variant{"zl_v" KL_STR(VX) "_b64x" KL_STR(BY) "_k" KL_STR(KB) "_x" KL_STR(XCD), KERN, DT, \
            FAMILY_ZL, VX, 64, BY, KB, XCD, &launch_zl<T, KERN, VX, BY, KB, XCD>,             \
            &launch_zl_batch<T, KERN, VX, BY, KB>, &zl_batch_occupancy<T, KERN, VX, BY, KB>}

#define KL_ZL_XCD(T, DT, KERN, VX, BY, KB) KL_ZL(T, DT, KERN, VX, BY, KB, 0), KL_ZL(T, DT, KERN, VX, BY, KB, 1)

#define KL_ZL_KB(T, DT, KERN, VX, BY)                                                \
    KL_ZL_XCD(T, DT, KERN, VX, BY, 32), KL_ZL_XCD(T, DT, KERN, VX, BY, 64), \
        KL_ZL_XCD(T, DT, KERN, VX, BY, 128)

#define KL_ZL_BLOCKS(T, DT, KERN, VX) \
    KL_ZL_KB(T, DT, KERN, VX, 4), KL_ZL_KB(T, DT, KERN, VX, 8), KL_ZL_KB(T, DT, KERN, VX, 16)

// Extra configurations: streaming tendencies (NT), slab-local XCD order and
// a waves-per-SIMD floor (WPE), named ..._x<XCD>_nt<NT>_w<WPE>.
#define KL_ZLX(T, DT, KERN, VX, BY, KB, XCD, NT, WPE)                                                 \
    Variant{"zl_v" KL_STR(VX) "_b64x" KL_STR(BY) "_k" KL_STR(KB) "_x" KL_STR(XCD) "_nt" KL_STR(NT)     \
            "_w" KL_STR(WPE),                                                                         \
            KERN, DT, FAMILY_ZL, VX, 64, BY, KB, XCD, &launch_zl<T, KERN, VX, BY, KB, XCD, NT, WPE>,   \
            &launch_zl_batch<T, KERN, VX, BY, KB, NT, WPE>, &zl_batch_occupancy<T, KERN, VX, BY, KB, NT, WPE>}

#define KL_ZCX(T, DT, KERN, VX, BX, BY, KB, XCD, NT, WPE)                                              \
    Variant{"zc_v" KL_STR(VX) "_b" KL_STR(BX) "x" KL_STR(BY) "_k" KL_STR(KB) "_x" KL_STR(XCD) "_nt"    \
            KL_STR(NT) "_w" KL_STR(WPE),                                                              \
            KERN, DT, FAMILY_ZC, VX, BX, BY, KB, XCD, &launch_zc<T, KERN, VX, BX, BY, KB, XCD, NT, WPE>, \
            nullptr, nullptr}

#define KL_ZLX_SET(T, DT, KERN, VX)                                                                     \
    KL_ZLX(T, DT, KERN, VX, 8, 32, 2, 0, 1), KL_ZLX(T, DT, KERN, VX, 8, 32, 2, 1, 1),                  \
        KL_ZLX(T, DT, KERN, VX, 8, 32, 0, 1, 1), KL_ZLX(T, DT, KERN, VX, 8, 128, 2, 0, 1),             \
        KL_ZLX(T, DT, KERN, VX, 8, 128, 2, 1, 1), KL_ZLX(T, DT, KERN, VX, 8, 128, 0, 1, 1),            \
        KL_ZLX(T, DT, KERN, VX, 8, 32, 0, 0, 4), KL_ZLX(T, DT, KERN, VX, 8, 32, 2, 1, 4),              \
        KL_ZLX(T, DT, KERN, VX, 4, 64, 2, 1, 1), KL_ZLX(T, DT, KERN, VX, 16, 64, 2, 1, 1)

#define KL_NT2_SET(T, DT, KERN, VX)                                                                     \
    KL_ZLX(T, DT, KERN, VX, 4, 64, 2, 2, 1), KL_ZLX(T, DT, KERN, VX, 4, 128, 2, 1, 1),                 \
        KL_ZLX(T, DT, KERN, VX, 4, 128, 2, 2, 1), KL_ZLX(T, DT, KERN, VX, 4, 256, 2, 1, 1),            \
        KL_ZLX(T, DT, KERN, VX, 8, 64, 2, 1, 1), KL_ZLX(T, DT, KERN, VX, 8, 64, 2, 2, 1),              \
        KL_ZLX(T, DT, KERN, VX, 4, 64, 0, 1, 1), KL_ZCX(T, DT, KERN, VX, 64, 4, 16, 2, 2, 1),          \
        KL_ZCX(T, DT, KERN, VX, 64, 2, 16, 2, 1, 1), KL_ZCX(T, DT, KERN, VX, 64, 8, 16, 2, 1, 1)

#define KL_ZCX_SET(T, DT, KERN, VX)                                                                     \
    KL_ZCX(T, DT, KERN, VX, 64, 4, 16, 2, 0, 1), KL_ZCX(T, DT, KERN, VX, 64, 4, 16, 2, 1, 1),          \
        KL_ZCX(T, DT, KERN, VX, 64, 4, 16, 0, 1, 1), KL_ZCX(T, DT, KERN, VX, 64, 4, 32, 0, 1, 1)

// Fused-step configurations (kernel KL_KERNEL_STEP).
#define KL_ST(T, DT, VX, BY, KB, XCD, NT)                                                                  \
    Variant{"step_v" KL_STR(VX) "_b64x" KL_STR(BY) "_k" KL_STR(KB) "_x" KL_STR(XCD) "_nt" KL_STR(NT),    \
            KL_KERNEL_STEP, DT, FAMILY_ZL, VX, 64, BY, KB, XCD, &launch_step<T, VX, BY, KB, XCD, NT>,     \
            &launch_step_batch<T, VX, BY, KB, NT>, &step_batch_occupancy<T, VX, BY, KB, NT>}

// The same with a register cap of 512 / WPE per lane (WPE waves per SIMD)
// and the ring options of MODE (FUSE_HALO3, FUSE_RING6), named by TAG.
#define KL_STW(T, DT, VX, BY, KB, XCD, NT, WPE, MODE, TAG)                                               \
    Variant{"step_v" KL_STR(VX) "_b64x" KL_STR(BY) "_k" KL_STR(KB) "_x" KL_STR(XCD) "_nt" KL_STR(NT)     \
            "_w" KL_STR(WPE) TAG,                                                                        \
            KL_KERNEL_STEP, DT, FAMILY_ZL, VX, 64, BY, KB, XCD, &launch_step<T, VX, BY, KB, XCD, NT, WPE, MODE>, \
            &launch_step_batch<T, VX, BY, KB, NT, WPE, MODE>, &step_batch_occupancy<T, VX, BY, KB, NT, WPE, MODE>}

// A fused step whose y and z ghost cells are refilled by a second kernel
// (FUSE_NOYZ).  Its persistent form (served ticks) is the same tile writing
// those ghost cells itself, which gives the same bits without a refill
// launch per tick.
#define KL_STY(T, DT, VX, BY, KB, XCD, NT, MODE, TAG)                                                    \
    Variant{"step_v" KL_STR(VX) "_b64x" KL_STR(BY) "_k" KL_STR(KB) "_x" KL_STR(XCD) "_nt" KL_STR(NT)     \
            "_w1" TAG,                                                                                   \
            KL_KERNEL_STEP, DT, FAMILY_ZL, VX, 64, BY, KB, XCD, &launch_step<T, VX, BY, KB, XCD, NT, 1, (MODE) | FUSE_NOYZ>, \
            &launch_step_batch<T, VX, BY, KB, NT, 1, MODE>, &step_batch_occupancy<T, VX, BY, KB, NT, 1, MODE>}

#define KL_ST_SET(T, DT, VX)                                                                             \
    KL_ST(T, DT, VX, 8, 32, 0, 0), KL_ST(T, DT, VX, 4, 64, 2, 1), KL_ST(T, DT, VX, 8, 32, 2, 1),         \
        KL_ST(T, DT, VX, 4, 128, 2, 1), KL_ST(T, DT, VX, 8, 64, 0, 1), KL_ST(T, DT, VX, 4, 32, 0, 0),    \
        KL_ST(T, DT, VX, 4, 8, 0, 0), KL_ST(T, DT, VX, 4, 16, 0, 0), KL_ST(T, DT, VX, 8, 8, 0, 0),       \
        KL_ST(T, DT, VX, 2, 16, 0, 0)

// Fused advec_u + diff_uvw configurations (kernel KL_KERNEL_ADVEC_DIFF): the
// fused-step tile accumulating into the tendencies.
#define KL_AD(T, DT, VX, BY, KB, XCD, NT)                                                                 \
    Variant{"ad_v" KL_STR(VX) "_b64x" KL_STR(BY) "_k" KL_STR(KB) "_x" KL_STR(XCD) "_nt" KL_STR(NT),      \
            KL_KERNEL_ADVEC_DIFF, DT, FAMILY_ZL, VX, 64, BY, KB, XCD,                                    \
            &launch_step<T, VX, BY, KB, XCD, NT, 1, FUSE_PAIR>, &launch_step_batch<T, VX, BY, KB, NT, 1, FUSE_PAIR>, \
            &step_batch_occupancy<T, VX, BY, KB, NT, 1, FUSE_PAIR>}

#define KL_ADW(T, DT, VX, BY, KB, XCD, NT, WPE, MODE, TAG)                                               \
    Variant{"ad_v" KL_STR(VX) "_b64x" KL_STR(BY) "_k" KL_STR(KB) "_x" KL_STR(XCD) "_nt" KL_STR(NT)       \
            "_w" KL_STR(WPE) TAG,                                                                        \
            KL_KERNEL_ADVEC_DIFF, DT, FAMILY_ZL, VX, 64, BY, KB, XCD,                                    \
            &launch_step<T, VX, BY, KB, XCD, NT, WPE, FUSE_PAIR | (MODE)>,                                \
            &launch_step_batch<T, VX, BY, KB, NT, WPE, FUSE_PAIR | (MODE)>,                               \
            &step_batch_occupancy<T, VX, BY, KB, NT, WPE, FUSE_PAIR | (MODE)>}

#define KL_AD_SET(T, DT, VX)                                                                             \
    KL_AD(T, DT, VX, 4, 8, 0, 0), KL_AD(T, DT, VX, 8, 8, 0, 0), KL_AD(T, DT, VX, 4, 32, 0, 0),           \
        KL_AD(T, DT, VX, 8, 32, 0, 0), KL_AD(T, DT, VX, 8, 32, 2, 1), KL_AD(T, DT, VX, 4, 64, 2, 1),     \
        KL_AD(T, DT, VX, 8, 64, 2, 1), KL_AD(T, DT, VX, 4, 128, 2, 1), KL_AD(T, DT, VX, 8, 128, 2, 1),   \
        KL_AD(T, DT, VX, 8, 256, 2, 1), KL_AD(T, DT, VX, 4, 256, 2, 1)

// Top-down slab order (XCD = 3) for a kernel that follows another sweep.
#define KL_REV_SET(T, DT, KERN, VX)                                                                     \
    KL_ZLX(T, DT, KERN, VX, 4, 64, 3, 1, 1), KL_ZLX(T, DT, KERN, VX, 4, 128, 3, 1, 1),                 \
        KL_ZLX(T, DT, KERN, VX, 4, 256, 3, 1, 1), KL_ZLX(T, DT, KERN, VX, 8, 32, 3, 1, 1),             \
        KL_ZLX(T, DT, KERN, VX, 8, 128, 3, 1, 1), KL_ZLX(T, DT, KERN, VX, 4, 128, 3, 0, 1)

// Waves-per-SIMD floors of 3 and 4 on the top-down slab configurations
// (fewer registers, more waves in flight).
#define KL_OCC_SET(T, DT, KERN, VX)                                                                     \
    KL_ZLX(T, DT, KERN, VX, 4, 256, 3, 1, 3), KL_ZLX(T, DT, KERN, VX, 4, 256, 3, 1, 4),                \
        KL_ZLX(T, DT, KERN, VX, 4, 128, 3, 1, 3), KL_ZLX(T, DT, KERN, VX, 4, 64, 3, 1, 4)

// Short z-marches for small grids (more tiles, shorter chains).
#define KL_SMALL_SET(T, DT, KERN, VX)                                                                   \
    KL_ZLX(T, DT, KERN, VX, 4, 8, 0, 0, 1), KL_ZLX(T, DT, KERN, VX, 4, 16, 0, 0, 1),                   \
        KL_ZLX(T, DT, KERN, VX, 8, 8, 0, 0, 1), KL_ZLX(T, DT, KERN, VX, 8, 16, 0, 1, 1)

// advec_u_2i5 LDS z-march configurations, named a5_v<VX>_b64x<BY>_k<KB>_x<XCD>_nt<NT>.
// The pair-unrolled march, named a5p_...
#define KL_A5P(T, DT, VX, BY, KB, XCD, NT)                                                                  \
    Variant{"a5p_v" KL_STR(VX) "_b64x" KL_STR(BY) "_k" KL_STR(KB) "_x" KL_STR(XCD) "_nt" KL_STR(NT),       \
            KL_KERNEL_ADVEC_U_2I5, DT, FAMILY_ZL, VX, 64, BY, KB, XCD,                                     \
            &launch_advec5_zl<T, VX, BY, KB, XCD, NT, 1, 1>, nullptr, nullptr}

// advec_u_2i5 with each y face evaluated once (shared through LDS), named
// a5s_v<VX>_b64x<BY>_k<KB>_x<XCD>_nt<NT>.
#define KL_A5S(T, DT, VX, BY, KB, XCD, NT)                                                                  \
    Variant{"a5s_v" KL_STR(VX) "_b64x" KL_STR(BY) "_k" KL_STR(KB) "_x" KL_STR(XCD) "_nt" KL_STR(NT),       \
            KL_KERNEL_ADVEC_U_2I5, DT, FAMILY_ZL, VX, 64, BY, KB, XCD,                                     \
            &launch_advec5_zl<T, VX, BY, KB, XCD, NT, 1, 0, 1>, nullptr, nullptr}

// The parity-slot march (no register copies at the end of a level), named a5r_...
#define KL_A5R(T, DT, VX, BY, KB, XCD, NT)                                                                  \
    Variant{"a5r_v" KL_STR(VX) "_b64x" KL_STR(BY) "_k" KL_STR(KB) "_x" KL_STR(XCD) "_nt" KL_STR(NT),       \
            KL_KERNEL_ADVEC_U_2I5, DT, FAMILY_ZL, VX, 64, BY, KB, XCD,                                     \
            &launch_advec5_zr<T, VX, BY, KB, XCD, NT>, nullptr, nullptr}

// The same with the u halo rows loaded HL levels ahead, named a5r_..._h<HL>.
#define KL_A5RH(T, DT, VX, BY, KB, XCD, NT, HL)                                                             \
    Variant{"a5r_v" KL_STR(VX) "_b64x" KL_STR(BY) "_k" KL_STR(KB) "_x" KL_STR(XCD) "_nt" KL_STR(NT)        \
            "_h" KL_STR(HL),                                                                                \
            KL_KERNEL_ADVEC_U_2I5, DT, FAMILY_ZL, VX, 64, BY, KB, XCD,                                     \
            &launch_advec5_zr<T, VX, BY, KB, XCD, NT, HL>, nullptr, nullptr}

#define KL_A5(T, DT, VX, BY, KB, XCD, NT)                                                                   \
    Variant{"a5_v" KL_STR(VX) "_b64x" KL_STR(BY) "_k" KL_STR(KB) "_x" KL_STR(XCD) "_nt" KL_STR(NT),        \
            KL_KERNEL_ADVEC_U_2I5, DT, FAMILY_ZL, VX, 64, BY, KB, XCD,                                     \
            &launch_advec5_zl<T, VX, BY, KB, XCD, NT>, nullptr, nullptr}

// diff_smag LDS z-march configurations, named s2_v<VX>_b64x<BY>_k<KB>_x<XCD>_nt<NT>.
#define KL_S2(T, DT, VX, BY, KB, XCD, NT)                                                                   \
    Variant{"s2_v" KL_STR(VX) "_b64x" KL_STR(BY) "_k" KL_STR(KB) "_x" KL_STR(XCD) "_nt" KL_STR(NT),        \
            KL_KERNEL_DIFF_SMAG, DT, FAMILY_ZL, VX, 64, BY, KB, XCD,                                       \
            &launch_smag_zl<T, VX, BY, KB, XCD, NT>, nullptr, nullptr}

// diff_smag with the parity-slot march, named s2r_v<VX>_b64x<BY>_k<KB>_x<XCD>_nt<NT>.
#define KL_S2R(T, DT, VX, BY, KB, XCD, NT)                                                                  \
    Variant{"s2r_v" KL_STR(VX) "_b64x" KL_STR(BY) "_k" KL_STR(KB) "_x" KL_STR(XCD) "_nt" KL_STR(NT),       \
            KL_KERNEL_DIFF_SMAG, DT, FAMILY_ZL, VX, 64, BY, KB, XCD,                                       \
            &launch_smag_zl<T, VX, BY, KB, XCD, NT, 1, 1>, nullptr, nullptr}

// diff_uvw split into per-component passes, named zl3_v<VX>_b64x<BY>_k<KB>_x<XCD>_nt<NT>.
#define KL_ZL3(T, DT, VX, BY, KB, XCD, NT)                                                                  \
    Variant{"zl3_v" KL_STR(VX) "_b64x" KL_STR(BY) "_k" KL_STR(KB) "_x" KL_STR(XCD) "_nt" KL_STR(NT),       \
            KL_KERNEL_DIFF_UVW, DT, FAMILY_ZL, VX, 64, BY, KB, XCD, &launch_zl_split<T, VX, BY, KB, XCD, NT>, \
            nullptr, nullptr}
