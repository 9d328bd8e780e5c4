// Auxiliary kernels: ghost fill, fused Euler update + ghost refill, interior
// zeroing, FP64 reductions, bit hash and the device-side field generator.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "kl_internal.hpp"
#include "stencil.hpp"

namespace kl {
namespace {

struct Dims {
    int itot, jtot, ktot, bc;
    int64_t off, js, ks;
    int gc;  // ghost cells per side in x and y
};

inline Dims dims_of(const HostArgs &a) { return Dims{a.itot, a.jtot, a.ktot, a.bc, a.off, a.js, a.ks, a.gc}; }

__device__ __forceinline__ int64_t at(const Dims &d, int i, int j, int k)
{
    return d.off + i + (int64_t)j * d.js + (int64_t)k * d.ks;
}

// Interior index of which periodic index p (p >= 1 - gc) is the image.
__device__ __forceinline__ int wrap_n(int p, int n)
{
    int q = (p - 1) % n;
    if (q < 0) q += n;
    return q + 1;
}
__device__ __forceinline__ int wrap_i(const Dims &d, int i) { return wrap_n(i, d.itot); }
__device__ __forceinline__ int wrap_j(const Dims &d, int j) { return wrap_n(j, d.jtot); }

// Source level and factor of level k of field f (0 u, 1 v, 2 w) under the
// boundary rule; factor 0 means the cell is set to zero.
__device__ __forceinline__ int src_k(const Dims &d, int f, int k, int &sign)
{
    sign = 1;
    const int kt = d.ktot;
    if (d.bc == KL_BC_ZPERIODIC) return k == 0 ? kt : (k == kt + 1 ? 1 : k);
    if (f < 2) return k == 0 ? 1 : (k == kt + 1 ? kt : k);
    if (d.bc == KL_BC_ZWALL_ZEROGRAD) return (k == 0 || k == 1) ? 2 : (k == kt + 1 ? kt : k);
    // no penetration
    if (k == 1 || k == kt + 1) {
        sign = 0;
        return 2;
    }
    if (k == 0) {
        sign = -1;
        return 2;
    }
    return k;
}

// One thread per ghost cell (region R0: the whole planes k = 0 and ktot+1;
// R1: the 2 gc ghost rows of levels 1..ktot; R2: the 2 gc ghost columns of
// the interior rows of levels 1..ktot; R3: the interior of plane k = 1, for
// w in wall modes).  Every source cell is an interior cell that no thread
// writes, so the cells can be filled in any order.  kind[f] is the z rule
// of field f (0 and 1: the u/v rule, 2: the w rule); a NULL field is skipped.
// The cell index math is 32-bit: the launchers refuse grids with 2^32 or
// more ghost cells (64-bit divisions cost tens of instructions each).
// r3_wide: region R3 spans the x ghost columns of plane k = 1 too (for a
// refill that skips R2, whose columns at k = 1 belong to w's wall plane).
template <typename T>
__device__ __forceinline__ void fill_cell(const Dims &d, T *u, T *v, T *w, int k0, int k1, int k2, int64_t n0_,
                                          int64_t n1_, int64_t n2_, int64_t n3_, int64_t t_, bool r3_wide = false)
{
    const uint32_t n0 = (uint32_t)n0_, n01 = (uint32_t)(n0_ + n1_), n012 = (uint32_t)(n0_ + n1_ + n2_),
                   nall = (uint32_t)(n0_ + n1_ + n2_ + n3_);
    if (t_ >= (int64_t)nall) return;
    const uint32_t t = (uint32_t)t_;
    const int gc = d.gc;
    const uint32_t ic = (uint32_t)(d.itot + 2 * gc), plane = ic * (uint32_t)(d.jtot + 2 * gc);
    const uint32_t g2 = 2u * (uint32_t)gc;
    int i, j, k;
    bool w_only = false;
    if (t < n0) {
        const uint32_t p = t < plane ? t : t - plane;
        k = t < plane ? 0 : d.ktot + 1;
        j = (int)(p / ic) + 1 - gc;
        i = (int)(p % ic) + 1 - gc;
    } else if (t < n01) {
        const uint32_t q = t - n0;
        const uint32_t r = q / ic;  // ghost row index over (level, row)
        i = (int)(q % ic) + 1 - gc;
        k = 1 + (int)(r / g2);
        const int jr = (int)(r % g2);
        j = jr < gc ? 1 - gc + jr : d.jtot + 1 + (jr - gc);
    } else if (t < n012) {
        const uint32_t q = t - n01;
        const int c = (int)(q % g2);
        const uint32_t rest = q / g2;
        j = 1 + (int)(rest % (uint32_t)d.jtot);
        k = 1 + (int)(rest / (uint32_t)d.jtot);
        i = c < gc ? 1 - gc + c : d.itot + 1 + (c - gc);
    } else {
        const uint32_t q = t - n012;
        const uint32_t rw = r3_wide ? ic : (uint32_t)d.itot;
        k = 1;
        j = 1 + (int)(q / rw);
        i = 1 + (int)(q % rw) - (r3_wide ? gc : 0);
        w_only = true;
    }
    const int si = wrap_i(d, i), sj = wrap_j(d, j);
    const int64_t dst = at(d, i, j, k);
    T *f3[3] = {u, v, w};
    const int kind[3] = {k0, k1, k2};
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        T *p = f3[f];
        if (!p || (w_only && kind[f] != 2)) continue;
        int sign;
        const int sk = src_k(d, kind[f], k, sign);
        p[dst] = sign == 0 ? T(0) : (sign < 0 ? -p[at(d, si, sj, sk)] : p[at(d, si, sj, sk)]);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void fill_ghosts_kernel(Dims d, T *u, T *v, T *w, int k0, int k1, int k2,
                                                         int64_t n0, int64_t n1, int64_t n2, int64_t n3,
                                                         bool r3_wide)
{
    fill_cell<T>(d, u, v, w, k0, k1, k2, n0, n1, n2, n3, (int64_t)blockIdx.x * 256 + threadIdx.x, r3_wide);
}

// Ghost fill of the velocity fields of many grids in one launch: block b
// fills cells [256 lb, 256 lb + 256) of grid job g, (g, lb) = blocks[b];
// the same cell map and copies as the single-grid fill.
struct FillJob {
    Dims d;
    void *u, *v, *w;
    int64_t n0, n1, n2, n3;
};

template <typename T>
__global__ __launch_bounds__(256) void fill_ghosts_batch_kernel(const FillJob *__restrict__ jobs,
                                                               const int2 *__restrict__ blocks)
{
    const int2 b = blocks[blockIdx.x];
    const FillJob j = jobs[b.x];
    fill_cell<T>(j.d, as_global((T *)j.u), as_global((T *)j.v), as_global((T *)j.w), 0, 1, 2, j.n0, j.n1, j.n2,
                 j.n3, (int64_t)b.y * 256 + threadIdx.x);
}

// Forward Euler at one interior point: the thread writes the updated cell
// and every ghost cell whose source it is (the inverse of the fill map).
template <typename T>
__device__ __forceinline__ void euler_point(const Dims &d, T dt, int kw0, T *u, T *v, T *w, const T *ut,
                                            const T *vt, const T *wt, int i, int j, int k)
{
    const int64_t c = at(d, i, j, k);
    // x and y images of (i, j)
    int xi[3], yj[3], nx = 1, ny = 1;
    xi[0] = i;
    yj[0] = j;
    if (i == d.itot) xi[nx++] = 0;
    if (i == 1) xi[nx++] = d.itot + 1;
    if (j == d.jtot) yj[ny++] = 0;
    if (j == 1) yj[ny++] = d.jtot + 1;
    T *f3[3] = {u, v, w};
    const T *t3[3] = {ut, vt, wt};
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        if (f == 2 && k < kw0) continue;
        T *p = f3[f];
        const T val = euler_value<T>(p[c], dt, t3[f][c]);
        // z images with their factors
        int zk[4], zs[4], nz = 1;
        zk[0] = k;
        zs[0] = 1;
        const int kt = d.ktot;
        if (d.bc == KL_BC_ZPERIODIC) {
            if (k == kt) { zk[nz] = 0; zs[nz++] = 1; }
            if (k == 1) { zk[nz] = kt + 1; zs[nz++] = 1; }
        } else if (f < 2) {
            if (k == 1) { zk[nz] = 0; zs[nz++] = 1; }
            if (k == kt) { zk[nz] = kt + 1; zs[nz++] = 1; }
        } else if (d.bc == KL_BC_ZWALL_ZEROGRAD) {
            if (k == 2) { zk[nz] = 0; zs[nz++] = 1; zk[nz] = 1; zs[nz++] = 1; }
            if (k == kt) { zk[nz] = kt + 1; zs[nz++] = 1; }
        } else {
            if (k == 2) { zk[nz] = 0; zs[nz++] = -1; zk[nz] = 1; zs[nz++] = 0; }
            if (k == kt) { zk[nz] = kt + 1; zs[nz++] = 0; }
        }
        for (int a = 0; a < nz; ++a) {
            const T zv = zs[a] == 0 ? T(0) : (zs[a] < 0 ? -val : val);
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) p[at(d, xi[x], yj[y], zk[a])] = zv;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void euler_kernel(Dims d, T dt, int kw0, T *u, T *v, T *w,
                                                   const T *ut, const T *vt, const T *wt, int nbx)
{
    unsigned b = blockIdx.x;
    const int bx = b % nbx;
    b /= nbx;
    const int j = 1 + (int)(b % d.jtot);
    const int k = 1 + (int)(b / d.jtot);
    const int i = 1 + bx * 256 + (int)threadIdx.x;
    if (i > d.itot) return;
    euler_point<T>(d, dt, kw0, u, v, w, ut, vt, wt, i, j, k);
}

template <typename T>
__global__ __launch_bounds__(256) void zero_interior_kernel(Dims d, T *f, int nbx)
{
    unsigned b = blockIdx.x;
    const int bx = b % nbx;
    b /= nbx;
    const int j = 1 + (int)(b % d.jtot);
    const int k = 1 + (int)(b / d.jtot);
    const int i = 1 + bx * 256 + (int)threadIdx.x;
    if (i > d.itot) return;
    f[at(d, i, j, k)] = T(0);
}

// ---------------------------------------------------------------------------
// FP64 reductions: pass 1 gives each of RB blocks a fixed set of rows
// (row r = (j, k) pairs, rows b, b + RB, ...), each thread a fixed set of
// row slots and columns; block partials are combined by a fixed LDS tree.  Pass 2 reduces
// the RB partials in one block the same way.  No atomics, so the result is
// bitwise reproducible.
// ---------------------------------------------------------------------------
constexpr int RB = 4096;   // pass-1 blocks
constexpr int RT = 256;    // threads per block
constexpr int RQ = 9;      // values per partial

__device__ __forceinline__ double comb(int q_is_max, double a, double b)
{
    return q_is_max ? fmax(a, b) : a + b;
}

template <int NQ>
__device__ void block_tree(double (&acc)[NQ], const int (&is_max)[NQ], double *out)
{
    __shared__ double sh[RT][NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) sh[threadIdx.x][q] = acc[q];
    __syncthreads();
    for (int s = RT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int q = 0; q < NQ; ++q)
                sh[threadIdx.x][q] = comb(is_max[q], sh[threadIdx.x][q], sh[threadIdx.x + s][q]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) out[q] = sh[0][q];
    }
}

// Pass 1.  Each thread reads V consecutive points of a row with one vector
// load (V > 1 when the rows are aligned to it).  A row has cpr = itot / V
// chunks; when a row has fewer chunks than the block has threads, a pass
// covers rpp = RT / cpr rows at once (thread t: row slot t / cpr, chunk
// t % cpr).  Block b owns rows b, b + RB, b + 2 RB, ...; slot s takes the
// n-th of them for n = s, s + rpp, ...; two rows are loaded before either
// is accumulated.  The mapping depends only on the grid, so the result is
// the same on every run.
template <typename T, int V>
__device__ __forceinline__ void red_load(T (&x)[V], const T *p)
{
    if constexpr (V == 1) {
        x[0] = *p;
    } else {
        typedef T VT __attribute__((ext_vector_type(V)));
        const VT y = *reinterpret_cast<const VT *>(p);
#pragma unroll
        for (int n = 0; n < V; ++n) x[n] = y[n];
    }
}

// Pass-1 block b of a reduction (partial + b * RQ receives its partial).
template <typename T, int V>
__device__ __forceinline__ void reduce_block(const Dims &d, int what, int kw0, const T *f0, const T *f1,
                                             const T *f2, const T *dzi, const T *dzhi, int b, double *partial)
{
    double acc[RQ];
    int is_max[RQ];
#pragma unroll
    for (int q = 0; q < RQ; ++q) {
        acc[q] = 0.0;
        is_max[q] = (what == 1 && q % 3 == 2);
    }
    const int64_t nrows = (int64_t)d.jtot * d.ktot;
    const int cpr = d.itot / V;
    const bool wide = cpr >= RT;
    const int rpp = wide ? 1 : RT / cpr;
    const int slot = wide ? 0 : (int)threadIdx.x / cpr;
    const int c0 = wide ? (int)threadIdx.x : (int)threadIdx.x % cpr;
    const int cstep = wide ? RT : cpr;
    const int64_t rstep = (int64_t)rpp * RB;
    const T *f3[3] = {f0, f1, f2};

    // one row's contribution of chunk c, values already loaded
    auto add = [&](const T (&x)[3][V], int k) {
        if (what == 0) {
            const double wz = 1.0 / (double)dzi[k], wzh = 1.0 / (double)dzhi[k];
#pragma unroll
            for (int n = 0; n < V; ++n) {
                acc[0] += (double)x[0][n] * wz;
                acc[1] += (double)x[1][n] * wz;
                if (k >= kw0) acc[2] += (double)x[2][n] * wzh;
            }
        } else {
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                if (f3[f] == nullptr) continue;
#pragma unroll
                for (int n = 0; n < V; ++n) {
                    const double y = (double)x[f][n];
                    acc[3 * f] += y;
                    acc[3 * f + 1] += y * y;
                    acc[3 * f + 2] = fmax(acc[3 * f + 2], fabs(y));
                }
            }
        }
    };
    auto load = [&](T (&x)[3][V], int64_t base) {
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            if (f3[f] != nullptr)
                red_load<T, V>(x[f], f3[f] + base);
            else
#pragma unroll
                for (int n = 0; n < V; ++n) x[f][n] = T(0);
        }
    };

    if (slot < rpp) {
        int64_t r = (int64_t)b + (int64_t)slot * RB;
        for (; r + rstep < nrows; r += 2 * rstep) {
            // 32-bit row arithmetic (the launchers refuse 2^31 or more rows)
            const uint32_t ra = (uint32_t)r, rb = (uint32_t)(r + rstep), jt = (uint32_t)d.jtot;
            const int ja = 1 + (int)(ra % jt), ka = 1 + (int)(ra / jt);
            const int jb = 1 + (int)(rb % jt), kb = 1 + (int)(rb / jt);
            for (int c = c0; c < cpr; c += cstep) {
                T xa[3][V], xb[3][V];
                load(xa, at(d, 1 + c * V, ja, ka));
                load(xb, at(d, 1 + c * V, jb, kb));
                add(xa, ka);
                add(xb, kb);
            }
        }
        if (r < nrows) {
            const uint32_t ru = (uint32_t)r, jt = (uint32_t)d.jtot;
            const int j = 1 + (int)(ru % jt), k = 1 + (int)(ru / jt);
            for (int c = c0; c < cpr; c += cstep) {
                T x[3][V];
                load(x, at(d, 1 + c * V, j, k));
                add(x, k);
            }
        }
    }
    block_tree<RQ>(acc, is_max, partial + (int64_t)b * RQ);
}

template <typename T, int V>
__global__ __launch_bounds__(RT) void reduce_pass1(Dims d, int what, int kw0, const T *f0, const T *f1,
                                                  const T *f2, const T *dzi, const T *dzhi,
                                                  double *partial)
{
    reduce_block<T, V>(d, what, kw0, f0, f1, f2, dzi, dzhi, (int)blockIdx.x, partial);
}

// Pass 2 over the RB partials at `partial` into out[0 .. nout-1].
__device__ __forceinline__ void reduce_final(int what, const double *partial, double *out)
{
    double acc[RQ];
    int is_max[RQ];
#pragma unroll
    for (int q = 0; q < RQ; ++q) {
        acc[q] = 0.0;
        is_max[q] = (what == 1 && q % 3 == 2);
    }
    for (int b = threadIdx.x; b < RB; b += RT)
#pragma unroll
        for (int q = 0; q < RQ; ++q) acc[q] = comb(is_max[q], acc[q], partial[(int64_t)b * RQ + q]);
    __shared__ double res[RQ];
    block_tree<RQ>(acc, is_max, res);
    __syncthreads();
    const int nout = what == 0 ? 3 : 9;
    if ((int)threadIdx.x < nout) out[threadIdx.x] = res[threadIdx.x];
}

__global__ __launch_bounds__(RT) void reduce_pass2(int what, const double *partial, double *out)
{
    reduce_final(what, partial, out);
}

// Conservation sums (what = 0) of many grids in two launches: pass-1 block
// blockIdx.x is block b of job g, (g, b) = blocks[blockIdx.x], into that
// job's own RB partials; pass 2 reduces each slot's partials in one block.
// Per grid the blocks, their rows and the trees are those of the single-grid
// reduction, so each grid's sums are bitwise those of kl_reduce_fp64.  Only
// blocks that own rows (b < jtot*ktot) are launched: a block without rows
// gives the partial +0.0, which the partials hold from their allocation, and
// adding +0.0 changes no sum that pass 2 forms (its sums start at +0.0).
struct SumJob {
    Dims d;
    int kw0, slot;
    const void *f0, *f1, *f2, *dzi, *dzhi;
};

template <typename T, int V>
__global__ __launch_bounds__(RT) void sums_batch_pass1(const SumJob *__restrict__ jobs,
                                                      const int2 *__restrict__ blocks, double *partials)
{
    const int2 gb = blocks[blockIdx.x];
    const SumJob j = jobs[gb.x];
    reduce_block<T, V>(j.d, 0, j.kw0, as_global((const T *)j.f0), as_global((const T *)j.f1),
                       as_global((const T *)j.f2), as_global((const T *)j.dzi), as_global((const T *)j.dzhi),
                       gb.y, partials + (int64_t)j.slot * RB * RQ);
}

__global__ __launch_bounds__(RT) void sums_batch_pass2(const double *partials, double *out)
{
    reduce_final(0, partials + (int64_t)blockIdx.x * RB * RQ, out + 3 * (int64_t)blockIdx.x);
}

// Bit hash: sum over interior cells (mod 2^64) of SplitMix64(bits ^ cell key).
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <typename T>
__device__ __forceinline__ uint64_t bits_of(T x)
{
    if constexpr (sizeof(T) == 8) {
        return (uint64_t)__double_as_longlong(x);
    } else {
        return (uint64_t)(uint32_t)__float_as_uint(x);
    }
}

template <typename T>
__global__ __launch_bounds__(RT) void hash_pass1(Dims d, const T *f, uint64_t *partial)
{
    uint64_t acc = 0;
    const int64_t nrows = (int64_t)d.jtot * d.ktot;
    for (int64_t r = blockIdx.x; r < nrows; r += RB) {
        const int j = 1 + (int)(r % d.jtot);
        const int k = 1 + (int)(r / d.jtot);
        const int64_t base = at(d, 0, j, k);
        for (int i = 1 + (int)threadIdx.x; i <= d.itot; i += RT) {
            const uint64_t key = (uint64_t)i + ((uint64_t)j << 21) + ((uint64_t)k << 42);
            acc += mix64(bits_of<T>(f[base + i]) ^ mix64(key));
        }
    }
    __shared__ uint64_t sh[RT];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = RT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(RT) void hash_pass2(const uint64_t *partial, uint64_t *out)
{
    uint64_t acc = 0;
    for (int b = threadIdx.x; b < RB; b += RT) acc += partial[b];
    __shared__ uint64_t sh[RT];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = RT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

// Device generator of the served initial state: U[-1,1) noise from the
// counter-based SplitMix64 recipe plus the mean flow (1, 0.5, 0), rounded to
// the field type.  Counter of interior point (i-1, j-1, k-1) of field f:
// ((seed*8 + f) << 40) + (i-1) + itot*((j-1) + jtot*(k-1)).
template <typename T>
__global__ __launch_bounds__(256) void gen_uniform_kernel(Dims d, uint64_t seed, T *u, T *v, T *w, int nbx)
{
    unsigned b = blockIdx.x;
    const int bx = b % nbx;
    b /= nbx;
    const int j = 1 + (int)(b % d.jtot);
    const int k = 1 + (int)(b / d.jtot);
    const int i = 1 + bx * 256 + (int)threadIdx.x;
    if (i > d.itot) return;
    const int64_t c = at(d, i, j, k);
    const uint64_t cnt = (uint64_t)(i - 1) + (uint64_t)d.itot * ((uint64_t)(j - 1) + (uint64_t)d.jtot * (uint64_t)(k - 1));
    const double mean[3] = {1.0, 0.5, 0.0};
    T *f3[3] = {u, v, w};
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        const uint64_t key = ((seed * 8u + (uint64_t)f) << 40) + cnt;
        const double r = (double)(mix64(key) >> 11) * 0x1.0p-53;
        f3[f][c] = (T)((2.0 * r - 1.0) + mean[f]);
    }
}

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

size_t reduce_scratch_bytes() { return (size_t)RB * RQ * sizeof(double); }

namespace {
hipError_t fill_launch(const HostArgs &a, void *u, void *v, void *w, int k0, int k1, int k2, bool w_faces,
                       hipStream_t s, bool x_columns = true)
{
    const Dims d = dims_of(a);
    const int64_t gc = a.gc;
    const int64_t ic = a.itot + 2 * gc, jc = a.jtot + 2 * gc;
    const int64_t n0 = 2 * ic * jc, n1 = 2 * gc * ic * a.ktot;
    const int64_t n2 = x_columns ? 2 * gc * (int64_t)a.jtot * a.ktot : 0;  // region R2 (x ghost columns)
    // R3 (w's plane k = 1 in wall modes) with its x ghost columns when R2 is skipped
    const int64_t n3 = (w_faces && a.bc != KL_BC_ZPERIODIC) ? (x_columns ? a.itot : ic) * (int64_t)a.jtot : 0;
    if (n0 + n1 + n2 + n3 >= ((int64_t)1 << 32)) return hipErrorInvalidValue;  // 32-bit cell index
    const unsigned nb = cdiv(n0 + n1 + n2 + n3, 256);
    if (a.dtype == KL_F32)
        hipLaunchKernelGGL(fill_ghosts_kernel<float>, dim3(nb), dim3(256), 0, s, d, (float *)u, (float *)v,
                           (float *)w, k0, k1, k2, n0, n1, n2, n3, !x_columns);
    else
        hipLaunchKernelGGL(fill_ghosts_kernel<double>, dim3(nb), dim3(256), 0, s, d, (double *)u,
                           (double *)v, (double *)w, k0, k1, k2, n0, n1, n2, n3, !x_columns);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_fill_ghosts(const HostArgs &a, void *u, void *v, void *w, hipStream_t s)
{
    return fill_launch(a, u, v, w, 0, 1, 2, true, s);
}

hipError_t launch_fill_yz_images(const HostArgs &a, void *u, void *v, void *w, hipStream_t s)
{
    return fill_launch(a, u, v, w, 0, 1, 2, true, s, false);
}

hipError_t launch_fill_scalar(const HostArgs &a, void *f, hipStream_t s)
{
    return fill_launch(a, f, nullptr, nullptr, 0, 0, 0, false, s);
}

hipError_t launch_euler(const HostArgs &a, double dt, void *u, void *v, void *w, hipStream_t s)
{
    const Dims d = dims_of(a);
    const int nbx = (int)cdiv(a.itot, 256);
    const unsigned nb = (unsigned)nbx * a.jtot * a.ktot;
    if (a.dtype == KL_F32)
        hipLaunchKernelGGL(euler_kernel<float>, dim3(nb), dim3(256), 0, s, d, (float)dt, a.kw0, (float *)u,
                           (float *)v, (float *)w, (const float *)a.ut, (const float *)a.vt,
                           (const float *)a.wt, nbx);
    else
        hipLaunchKernelGGL(euler_kernel<double>, dim3(nb), dim3(256), 0, s, d, dt, a.kw0, (double *)u,
                           (double *)v, (double *)w, (const double *)a.ut, (const double *)a.vt,
                           (const double *)a.wt, nbx);
    return hipGetLastError();
}

hipError_t launch_zero_interior(const HostArgs &a, void *f, hipStream_t s)
{
    const Dims d = dims_of(a);
    const int nbx = (int)cdiv(a.itot, 256);
    const unsigned nb = (unsigned)nbx * a.jtot * a.ktot;
    if (a.dtype == KL_F32)
        hipLaunchKernelGGL(zero_interior_kernel<float>, dim3(nb), dim3(256), 0, s, d, (float *)f, nbx);
    else
        hipLaunchKernelGGL(zero_interior_kernel<double>, dim3(nb), dim3(256), 0, s, d, (double *)f, nbx);
    return hipGetLastError();
}

// Vector width of the reductions' loads: 4 floats or 2 doubles (16 bytes)
// when every row start of the interior and every field pointer is aligned to
// it (true), else 1 (false).
bool reduce_vectorized(const HostArgs &a, const void *f0, const void *f1, const void *f2)
{
    const int vw = a.dtype == KL_F32 ? 4 : 2;
    const size_t vb = (size_t)vw * (a.dtype == KL_F32 ? 4 : 8);
    bool vec = a.itot % vw == 0 && (a.off + 1) % vw == 0 && a.js % vw == 0 && a.ks % vw == 0;
    for (const void *p : {f0, f1, f2})
        if (p && (uintptr_t)p % vb) vec = false;
    return vec;
}

hipError_t launch_reduce(const HostArgs &a, int what, const void *f0, const void *f1, const void *f2,
                         double *out, void *scratch, hipStream_t s)
{
    const Dims d = dims_of(a);
    double *partial = (double *)scratch;
    if ((int64_t)a.jtot * a.ktot >= ((int64_t)1 << 31)) return hipErrorInvalidValue;  // 32-bit row index
    const bool vec = reduce_vectorized(a, f0, f1, f2);
    if (a.dtype == KL_F32) {
        if (vec)
            hipLaunchKernelGGL((reduce_pass1<float, 4>), dim3(RB), dim3(RT), 0, s, d, what, a.kw0,
                               (const float *)f0, (const float *)f1, (const float *)f2, (const float *)a.dzi,
                               (const float *)a.dzhi, partial);
        else
            hipLaunchKernelGGL((reduce_pass1<float, 1>), dim3(RB), dim3(RT), 0, s, d, what, a.kw0,
                               (const float *)f0, (const float *)f1, (const float *)f2, (const float *)a.dzi,
                               (const float *)a.dzhi, partial);
    } else {
        if (vec)
            hipLaunchKernelGGL((reduce_pass1<double, 2>), dim3(RB), dim3(RT), 0, s, d, what, a.kw0,
                               (const double *)f0, (const double *)f1, (const double *)f2, (const double *)a.dzi,
                               (const double *)a.dzhi, partial);
        else
            hipLaunchKernelGGL((reduce_pass1<double, 1>), dim3(RB), dim3(RT), 0, s, d, what, a.kw0,
                               (const double *)f0, (const double *)f1, (const double *)f2, (const double *)a.dzi,
                               (const double *)a.dzhi, partial);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_pass2, dim3(1), dim3(RT), 0, s, what, (const double *)partial, out);
    return hipGetLastError();
}

// ---- batched ghost fill and conservation sums (used by the batched form) ----

size_t fill_job_bytes() { return sizeof(FillJob); }

int64_t fill_cell_count(const HostArgs &a)
{
    const int64_t gc = a.gc;
    const int64_t ic = a.itot + 2 * gc, jc = a.jtot + 2 * gc;
    return 2 * ic * jc + 2 * gc * ic * a.ktot + 2 * gc * (int64_t)a.jtot * a.ktot +
           (a.bc != KL_BC_ZPERIODIC ? (int64_t)a.itot * a.jtot : 0);
}

void append_fill_job(const HostArgs &a, void *u, void *v, void *w, std::vector<char> &jobs,
                     std::vector<int2> &blocks)
{
    const int64_t gc = a.gc;
    const int64_t ic = a.itot + 2 * gc, jc = a.jtot + 2 * gc;
    FillJob j;
    j.d = dims_of(a);
    j.u = u;
    j.v = v;
    j.w = w;
    j.n0 = 2 * ic * jc;
    j.n1 = 2 * gc * ic * a.ktot;
    j.n2 = 2 * gc * (int64_t)a.jtot * a.ktot;
    j.n3 = a.bc != KL_BC_ZPERIODIC ? (int64_t)a.itot * a.jtot : 0;  // the velocity fill: w's wall faces
    const int job = (int)(jobs.size() / sizeof(FillJob));
    const char *p = (const char *)&j;
    jobs.insert(jobs.end(), p, p + sizeof j);
    const unsigned nb = cdiv(j.n0 + j.n1 + j.n2 + j.n3, 256);
    for (unsigned b = 0; b < nb; ++b) blocks.push_back(make_int2(job, (int)b));
}

hipError_t launch_fill_batch(int dtype, const void *jobs, const void *blocks, int nblocks, hipStream_t s)
{
    if (nblocks <= 0) return hipSuccess;
    if (dtype == KL_F32)
        hipLaunchKernelGGL(fill_ghosts_batch_kernel<float>, dim3(nblocks), dim3(256), 0, s, (const FillJob *)jobs,
                           (const int2 *)blocks);
    else
        hipLaunchKernelGGL(fill_ghosts_batch_kernel<double>, dim3(nblocks), dim3(256), 0, s, (const FillJob *)jobs,
                           (const int2 *)blocks);
    return hipGetLastError();
}

size_t sum_job_bytes() { return sizeof(SumJob); }

size_t sums_partial_bytes(int nslots) { return (size_t)nslots * RB * RQ * sizeof(double); }

void append_sum_job(const HostArgs &a, const void *ut, const void *vt, const void *wt, int slot, std::vector<char> &jobs,
                    std::vector<int2> &blocks)
{
    const int job = (int)(jobs.size() / sizeof(SumJob));
    const int64_t nb = std::min<int64_t>(RB, (int64_t)a.jtot * a.ktot);
    for (int b = 0; b < (int)nb; ++b) blocks.push_back(make_int2(job, b));
    SumJob j;
    j.d = dims_of(a);
    j.kw0 = a.kw0;
    j.slot = slot;
    j.f0 = ut;
    j.f1 = vt;
    j.f2 = wt;
    j.dzi = a.dzi;
    j.dzhi = a.dzhi;
    const char *p = (const char *)&j;
    jobs.insert(jobs.end(), p, p + sizeof j);
}

hipError_t launch_sums_batch(int dtype, bool vec, const void *jobs, const void *blocks, int nblocks, double *partials,
                             hipStream_t s)
{
    if (nblocks <= 0) return hipSuccess;
    const dim3 grid((unsigned)nblocks);
    const SumJob *j = (const SumJob *)jobs;
    const int2 *bl = (const int2 *)blocks;
    if (dtype == KL_F32) {
        if (vec)
            hipLaunchKernelGGL((sums_batch_pass1<float, 4>), grid, dim3(RT), 0, s, j, bl, partials);
        else
            hipLaunchKernelGGL((sums_batch_pass1<float, 1>), grid, dim3(RT), 0, s, j, bl, partials);
    } else {
        if (vec)
            hipLaunchKernelGGL((sums_batch_pass1<double, 2>), grid, dim3(RT), 0, s, j, bl, partials);
        else
            hipLaunchKernelGGL((sums_batch_pass1<double, 1>), grid, dim3(RT), 0, s, j, bl, partials);
    }
    return hipGetLastError();
}

hipError_t launch_sums_finish(const double *partials, int nslots, double *out, hipStream_t s)
{
    if (nslots <= 0) return hipSuccess;
    hipLaunchKernelGGL(sums_batch_pass2, dim3((unsigned)nslots), dim3(RT), 0, s, partials, out);
    return hipGetLastError();
}

hipError_t launch_hash(const HostArgs &a, const void *f, uint64_t *out, void *scratch, hipStream_t s)
{
    const Dims d = dims_of(a);
    uint64_t *partial = (uint64_t *)scratch;
    if (a.dtype == KL_F32)
        hipLaunchKernelGGL(hash_pass1<float>, dim3(RB), dim3(RT), 0, s, d, (const float *)f, partial);
    else
        hipLaunchKernelGGL(hash_pass1<double>, dim3(RB), dim3(RT), 0, s, d, (const double *)f, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(hash_pass2, dim3(1), dim3(RT), 0, s, (const uint64_t *)partial, out);
    return hipGetLastError();
}

hipError_t launch_gen_uniform(const HostArgs &a, uint64_t seed, void *u, void *v, void *w, hipStream_t s)
{
    const Dims d = dims_of(a);
    const int nbx = (int)cdiv(a.itot, 256);
    const unsigned nb = (unsigned)nbx * a.jtot * a.ktot;
    if (a.dtype == KL_F32)
        hipLaunchKernelGGL(gen_uniform_kernel<float>, dim3(nb), dim3(256), 0, s, d, seed, (float *)u,
                           (float *)v, (float *)w, nbx);
    else
        hipLaunchKernelGGL(gen_uniform_kernel<double>, dim3(nb), dim3(256), 0, s, d, seed, (double *)u,
                           (double *)v, (double *)w, nbx);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Reductions without allocation.  The pass-1 partials go to a fixed array in
// device memory that the code object brings with it, so the call needs no
// hipMalloc.  Each device holds its own copy until the process ends; its
// address is looked up once per device, with that device current.  In host
// code `scratch` names a host-side stand-in, so only the looked-up address is
// ever handed to a kernel.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[RB * RQ];
constexpr size_t NOALLOC_SCRATCH_BYTES = sizeof(double) * RB * RQ;  // 288 KiB
constexpr int NOALLOC_MAX_DEVICES = 64;

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[NOALLOC_MAX_DEVICES];
}  // namespace

}  // namespace kl

extern "C" int kl_reduce_fp64_noalloc(const kl_grid_t *g, int32_t what, const void *f0, const void *f1,
                                      const void *f2, double *out, void *stream)
{
    using namespace kl;
    clear_error();
    int rc = check_grid(g);
    if (rc) return rc;
    if (what != 0 && what != 1) return fail(KL_ERR_INVALID, "what=%d", what);
    if (!out) return fail(KL_ERR_INVALID, "out is NULL");
    if (what == 0 && (!f0 || !f1 || !f2)) return fail(KL_ERR_INVALID, "conservation sums need ut, vt, wt");
    // the partial count is fixed (one row of RQ values per pass-1 block), not
    // a function of the grid; refuse if it ever outgrew the array
    if (reduce_scratch_bytes() > NOALLOC_SCRATCH_BYTES)
        return fail(KL_ERR_INVALID, "reduction needs %zu B of scratch, the fixed array holds %zu B",
                    reduce_scratch_bytes(), NOALLOC_SCRATCH_BYTES);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return fail(KL_ERR_INVALID, "device %d beyond the %d the fixed scratch table covers", dev,
                    NOALLOC_MAX_DEVICES);
    void *ptr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            e = hipGetSymbolAddress(&g_scratch_ptr[dev], HIP_SYMBOL(scratch));
            if (e != hipSuccess) {
                g_scratch_ptr[dev] = nullptr;
                return hip_fail(e, "hipGetSymbolAddress(scratch)");
            }
        }
        ptr = g_scratch_ptr[dev];
    }
    e = launch_reduce(make_args(g), what, f0, f1, f2, out, ptr, (hipStream_t)stream);
    return e == hipSuccess ? KL_OK : hip_fail(e, "reduce_noalloc");
}
