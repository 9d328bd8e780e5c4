// Streaming probe: the HBM ceiling the stencil kernels are measured against.
//
// kl_stream_probe moves `bytes` from each of nread source arrays and to each
// of nwrite destination arrays in one kernel, 16 bytes per lane per access,
// with no reuse: the access mix of a tendency kernel (advec_u reads 4 arrays
// and writes 1, diff_uvw reads 6 and writes 3, ...) without its stencil.
// Each destination chunk is the XOR of the source chunks, so every load is
// used and nothing is left for the compiler to remove.  Loads of a thread's
// UNROLL chunks are all issued before the first store.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "kl_internal.hpp"

namespace kl {
namespace {

constexpr int PT = 256;     // threads per block
constexpr int UNROLL = 4;   // 16-byte chunks per thread per pass
constexpr int64_t BLOCK_CHUNKS = (int64_t)PT * UNROLL;

typedef unsigned int U4 __attribute__((ext_vector_type(4)));

struct ProbePtrs {
    const U4 *src[8];
    U4 *dst[4];
};

// nchunks is a multiple of BLOCK_CHUNKS, so every chunk of a pass a block
// starts is in range and no access is conditional.
template <int NR, int NW, bool NT>
__global__ __launch_bounds__(PT) void stream_probe_kernel(ProbePtrs p, int64_t nchunks)
{
    const int64_t stride = (int64_t)gridDim.x * BLOCK_CHUNKS;
    for (int64_t bs = (int64_t)blockIdx.x * BLOCK_CHUNKS; bs < nchunks; bs += stride) {
        const int64_t c0 = bs + threadIdx.x;
        U4 acc[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) acc[u] = U4{0u, 0u, 0u, 0u};
#pragma unroll
        for (int r = 0; r < NR; ++r) {
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                const U4 *q = p.src[r] + c0 + (int64_t)u * PT;
                acc[u] ^= NT ? __builtin_nontemporal_load(q) : *q;
            }
        }
#pragma unroll
        for (int w = 0; w < NW; ++w) {
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                U4 *q = p.dst[w] + c0 + (int64_t)u * PT;
                if (NT)
                    __builtin_nontemporal_store(acc[u], q);
                else
                    *q = acc[u];
            }
        }
    }
}

template <int NR, int NW>
hipError_t launch_mix(const ProbePtrs &p, int64_t nchunks, bool nt, int nblocks, hipStream_t s)
{
    if (nt)
        hipLaunchKernelGGL((stream_probe_kernel<NR, NW, true>), dim3(nblocks), dim3(PT), 0, s, p, nchunks);
    else
        hipLaunchKernelGGL((stream_probe_kernel<NR, NW, false>), dim3(nblocks), dim3(PT), 0, s, p, nchunks);
    return hipGetLastError();
}

}  // namespace
}  // namespace kl

using namespace kl;

extern "C" int kl_stream_probe(int32_t nread, int32_t nwrite, const void *const *src, void *const *dst,
                               int64_t bytes, int32_t nontemporal, void *stream)
{
    clear_error();
    if (!src || !dst) return fail(KL_ERR_INVALID, "NULL pointer array");
    if (bytes <= 0 || bytes % (16 * BLOCK_CHUNKS))
        return fail(KL_ERR_INVALID, "bytes %lld must be a positive multiple of %lld", (long long)bytes,
                    (long long)(16 * BLOCK_CHUNKS));
    if (nread < 1 || nread > 8 || nwrite < 1 || nwrite > 4)
        return fail(KL_ERR_INVALID, "nread %d / nwrite %d out of range", nread, nwrite);
    ProbePtrs p = {};
    for (int r = 0; r < nread; ++r) {
        if (!src[r] || (uintptr_t)src[r] % 16) return fail(KL_ERR_INVALID, "source %d is NULL or not 16-byte aligned", r);
        p.src[r] = (const U4 *)src[r];
    }
    for (int w = 0; w < nwrite; ++w) {
        if (!dst[w] || (uintptr_t)dst[w] % 16)
            return fail(KL_ERR_INVALID, "destination %d is NULL or not 16-byte aligned", w);
        p.dst[w] = (U4 *)dst[w];
    }
    const int64_t nchunks = bytes / 16;
    // enough blocks to fill the chip many times over, each with a few passes
    const int nblocks = (int)std::min<int64_t>(nchunks / BLOCK_CHUNKS, 256 * 32);
    const bool nt = nontemporal != 0;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    switch (nread * 10 + nwrite) {
    case 11: e = launch_mix<1, 1>(p, nchunks, nt, nblocks, s); break;
    case 21: e = launch_mix<2, 1>(p, nchunks, nt, nblocks, s); break;
    case 33: e = launch_mix<3, 3>(p, nchunks, nt, nblocks, s); break;
    case 41: e = launch_mix<4, 1>(p, nchunks, nt, nblocks, s); break;
    case 63: e = launch_mix<6, 3>(p, nchunks, nt, nblocks, s); break;
    case 73: e = launch_mix<7, 3>(p, nchunks, nt, nblocks, s); break;
    default:
        return fail(KL_ERR_INVALID, "stream mix r%dw%d not built (r1w1, r2w1, r3w3, r4w1, r6w3, r7w3)", nread,
                    nwrite);
    }
    return e == hipSuccess ? KL_OK : hip_fail(e, "stream_probe");
}
