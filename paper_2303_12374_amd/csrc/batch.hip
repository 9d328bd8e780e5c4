// Batched form: many independent grids advanced by persistent tile-walking
// kernels captured once in a HIP graph.
//
// Each grid gets its configurations from the wisdom files like a single-grid
// launch (nearest problem size on this GPU, Section "Kernel Selection and
// Compilation"); grids whose selected configuration has no persistent form
// use an LDS z-march configuration sized to the grid.  The configuration
// selected for the most grid points then takes every grid it can serve, the
// next one the rest it can serve, and so on (all configurations give the same
// bits).  Grids are grouped by (kernel, dtype, configuration); every group
// becomes one persistent kernel walking a static tile list, so the graph
// holds: [zero tendencies] -> advec_u groups -> diff_uvw groups.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <tuple>
#include <vector>

#include "kl_internal.hpp"
#include "variants.hpp"

namespace kl {
namespace {

struct Group {
    int kernel, dtype, variant;
    std::vector<int4> tiles;
    void *d_tiles = nullptr;
    int nblocks = 0;
};

struct Batch {
    std::vector<kl_grid_t> grids;
    double visc = 0;
    bool zero = false;
    void *d_desc[2] = {nullptr, nullptr};  // StencilArgs<float>[] and StencilArgs<double>[], indexed by grid
    std::vector<int4> ztiles[2];
    void *d_ztiles[2] = {nullptr, nullptr};
    int zblocks[2] = {0, 0};
    std::vector<Group> groups;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t ntiles = 0;
    int nkernels = 0;

    ~Batch()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (int d = 0; d < 2; ++d) {
            if (d_desc[d]) (void)hipFree(d_desc[d]);
            if (d_ztiles[d]) (void)hipFree(d_ztiles[d]);
        }
        for (auto &g : groups)
            if (g.d_tiles) (void)hipFree(g.d_tiles);
    }
};

}  // namespace

// Configuration of grid g for `kernel` in batched form.
int batch_variant(const kl_grid_t *g, int kernel, void *const f[6])
{
    const auto &vs = variants(kernel, g->dtype);
    const void *ptrs[6] = {f[0], f[1], f[2], f[3], f[4], f[5]};
    const int nptr = kernel == KL_KERNEL_ADVEC_U ? 4 : 6;
    const int sel = select_variant(g, kernel);
    // a selected configuration whose wave segment (64 * vx points) is wider
    // than the grid's rows would leave most lanes idle: size one to the grid
    if (vs[sel].batch && variant_eligible(vs[sel], g, ptrs, nptr) && 64 * vs[sel].vx <= std::max(64, g->itot))
        return sel;
    // fallback: widest vector that divides itot and does not exceed the row
    const int vmax = g->dtype == KL_F32 ? 4 : 2;
    for (int vx = vmax; vx >= 1; vx /= 2) {
        if (g->itot % vx || 64 * vx > std::max(64, g->itot)) continue;
        for (size_t n = 0; n < vs.size(); ++n) {
            const Variant &v = vs[n];
            if (v.family == FAMILY_ZL && v.vx == vx && v.by == 8 && v.kb == 32 && v.xcd == 0 &&
                variant_eligible(v, g, ptrs, nptr))
                return (int)n;
        }
    }
    return -1;
}

// Regroup the grids of one kernel: the configurations in decreasing order of
// the grid points they were selected for, each taking every remaining grid
// it can serve (a persistent form, eligible, a wave segment no wider than
// the grid's rows).  Fewer groups mean fewer serial persistent kernels and
// fewer partly idle ends of their tile lists.
void merge_batch_groups(int kernel, const std::vector<kl_grid_t> &grids, void *const *fields, std::vector<int> &sel)
{
    const int nptr = kernel == KL_KERNEL_ADVEC_U ? 4 : 6;
    std::map<std::pair<int, int>, int64_t> weight;  // (dtype, configuration) -> grid points
    for (size_t n = 0; n < grids.size(); ++n)
        weight[{grids[n].dtype, sel[n]}] += (int64_t)grids[n].itot * grids[n].jtot * grids[n].ktot;
    std::vector<std::pair<int64_t, std::pair<int, int>>> order;
    for (const auto &w : weight) order.push_back({w.second, w.first});
    std::stable_sort(order.begin(), order.end(), [](const auto &x, const auto &y) { return x.first > y.first; });
    std::vector<char> placed(grids.size(), 0);
    for (const auto &o : order) {
        const int dtype = o.second.first, vi = o.second.second;
        const Variant &v = variants(kernel, dtype)[vi];
        for (size_t n = 0; n < grids.size(); ++n) {
            const kl_grid_t *g = &grids[n];
            if (placed[n] || g->dtype != dtype) continue;
            void *const *f = fields + 6 * n;
            const void *ptrs[6] = {f[0], f[1], f[2], f[3], f[4], f[5]};
            if (sel[n] == vi ||
                (v.batch && 64 * v.vx <= std::max(64, g->itot) && variant_eligible(v, g, ptrs, nptr))) {
                sel[n] = vi;
                placed[n] = 1;
            }
        }
    }
}

hipError_t launch_zero_batch(int dtype, const void *descs, const void *tiles, int ntiles, int nblocks, hipStream_t s)
{
    if (dtype == KL_F32)
        hipLaunchKernelGGL(zero_tendencies_batch<float>, dim3(nblocks), dim3(256), 0, s,
                           (const StencilArgs<float> *)descs, (const int4 *)tiles, ntiles);
    else
        hipLaunchKernelGGL(zero_tendencies_batch<double>, dim3(nblocks), dim3(256), 0, s,
                           (const StencilArgs<double> *)descs, (const int4 *)tiles, ntiles);
    return hipGetLastError();
}

namespace {

template <typename T>
std::vector<StencilArgs<T>> descriptors(const std::vector<kl_grid_t> &grids, void *const *fields, double visc)
{
    std::vector<StencilArgs<T>> out(grids.size());
    for (size_t n = 0; n < grids.size(); ++n) {
        HostArgs a = make_args(&grids[n]);
        void *const *f = fields + 6 * n;
        a.u = f[0];
        a.v = f[1];
        a.w = f[2];
        a.ut = f[3];
        a.vt = f[4];
        a.wt = f[5];
        a.visc = visc;
        out[n] = device_args<T>(a);
    }
    return out;
}

hipError_t upload(void **dst, const void *src, size_t bytes)
{
    if (bytes == 0) return hipSuccess;
    hipError_t e = hipMalloc(dst, bytes);
    if (e != hipSuccess) return e;
    return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
}

int build(Batch &b, void *const *fields)
{
    int dev = 0;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(e, "device properties");
    const int ncu = prop.multiProcessorCount;

    // descriptor tables per dtype (entries of the other dtype are never referenced)
    {
        auto df = descriptors<float>(b.grids, fields, b.visc);
        auto dd = descriptors<double>(b.grids, fields, b.visc);
        if ((e = upload(&b.d_desc[0], df.data(), df.size() * sizeof(df[0]))) != hipSuccess) return hip_fail(e, "desc");
        if ((e = upload(&b.d_desc[1], dd.data(), dd.size() * sizeof(dd[0]))) != hipSuccess) return hip_fail(e, "desc");
    }
    // groups
    std::map<std::tuple<int, int, int>, size_t> gidx;
    for (int kernel = 0; kernel < 2; ++kernel) {
        std::vector<int> sel(b.grids.size());
        for (size_t n = 0; n < b.grids.size(); ++n) {
            sel[n] = batch_variant(&b.grids[n], kernel, fields + 6 * n);
            if (sel[n] < 0) return fail(KL_ERR_INVALID, "grid %zu: no batched configuration fits", n);
        }
        merge_batch_groups(kernel, b.grids, fields, sel);
        for (size_t n = 0; n < b.grids.size(); ++n) {
            const kl_grid_t *g = &b.grids[n];
            const int vi = sel[n];
            const auto key = std::make_tuple(kernel, g->dtype, vi);
            auto it = gidx.find(key);
            if (it == gidx.end()) {
                it = gidx.emplace(key, b.groups.size()).first;
                Group gr;
                gr.kernel = kernel;
                gr.dtype = g->dtype;
                gr.variant = vi;
                b.groups.push_back(gr);
            }
            Group &gr = b.groups[it->second];
            const Variant &v = variants(kernel, g->dtype)[vi];
            const int nbx = (int)cdivu(g->itot, 64 * v.vx), nby = (int)cdivu(g->jtot, v.by),
                      nbz = (int)cdivu(g->ktot, v.kb);
            for (int tz = 0; tz < nbz; ++tz)
                for (int ty = 0; ty < nby; ++ty)
                    for (int tx = 0; tx < nbx; ++tx) gr.tiles.push_back(make_int4((int)n, tx, ty, tz));
        }
    }
    for (Group &gr : b.groups) {
        if ((e = upload(&gr.d_tiles, gr.tiles.data(), gr.tiles.size() * sizeof(int4))) != hipSuccess)
            return hip_fail(e, "tiles");
        const Variant &v = variants(gr.kernel, gr.dtype)[gr.variant];
        gr.nblocks = (int)std::min<int64_t>((int64_t)gr.tiles.size(), (int64_t)ncu * v.occupancy());
        b.ntiles += (int64_t)gr.tiles.size();
    }
    // zeroing tiles: 32 rows each
    if (b.zero) {
        for (size_t n = 0; n < b.grids.size(); ++n) {
            const kl_grid_t *g = &b.grids[n];
            const int rows = g->jtot * g->ktot;
            for (int r0 = 0; r0 < rows; r0 += 32)
                b.ztiles[g->dtype].push_back(make_int4((int)n, r0, std::min(rows, r0 + 32), 0));
        }
        for (int d = 0; d < 2; ++d) {
            if (b.ztiles[d].empty()) continue;
            if ((e = upload(&b.d_ztiles[d], b.ztiles[d].data(), b.ztiles[d].size() * sizeof(int4))) != hipSuccess)
                return hip_fail(e, "zero tiles");
            b.zblocks[d] = (int)std::min<int64_t>((int64_t)b.ztiles[d].size(), (int64_t)ncu * 8);
        }
    }
    // capture the graph on a private stream
    hipStream_t cs;
    if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e, "stream");
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    int rc = KL_OK;
    if (e != hipSuccess) rc = hip_fail(e, "begin capture");
    for (int d = 0; d < 2 && rc == KL_OK; ++d) {
        if (!b.zero || b.ztiles[d].empty()) continue;
        e = launch_zero_batch(d, b.d_desc[d], b.d_ztiles[d], (int)b.ztiles[d].size(), b.zblocks[d], cs);
        if (e != hipSuccess) rc = hip_fail(e, "zero launch");
        ++b.nkernels;
    }
    for (int kernel = 0; kernel < 2 && rc == KL_OK; ++kernel) {
        for (Group &gr : b.groups) {
            if (gr.kernel != kernel || rc != KL_OK) continue;
            const Variant &v = variants(gr.kernel, gr.dtype)[gr.variant];
            e = v.batch(b.d_desc[gr.dtype], gr.d_tiles, (int)gr.tiles.size(), gr.nblocks, cs);
            if (e != hipSuccess) rc = hip_fail(e, v.name);
            ++b.nkernels;
        }
    }
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    if (rc == KL_OK && e != hipSuccess) rc = hip_fail(e, "end capture");
    b.graph = graph;
    if (rc == KL_OK) {
        e = hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0);
        if (e != hipSuccess) rc = hip_fail(e, "graph instantiate");
    }
    (void)hipStreamDestroy(cs);
    return rc;
}

}  // namespace
}  // namespace kl

using namespace kl;

extern "C" {

int kl_batch_create(const kl_grid_t *grids, void *const *fields, int32_t n, double visc, int32_t zero_tendencies,
                    void *stream, void **batch)
{
    clear_error();
    (void)stream;
    if (!grids || !fields || !batch || n < 1) return fail(KL_ERR_INVALID, "bad batch arguments");
    *batch = nullptr;
    for (int i = 0; i < n; ++i) {
        int rc = check_grid(&grids[i]);
        if (rc) return fail(rc, "grid %d: %s", i, kl_last_error());
        for (int f = 0; f < 6; ++f)
            if (!fields[6 * i + f]) return fail(KL_ERR_INVALID, "grid %d field %d is NULL", i, f);
    }
    Batch *b = new (std::nothrow) Batch();
    if (!b) return fail(KL_ERR_NOMEM, "batch");
    b->grids.assign(grids, grids + n);
    b->visc = visc;
    b->zero = zero_tendencies != 0;
    const int rc = build(*b, fields);
    if (rc != KL_OK) {
        delete b;
        return rc;
    }
    *batch = b;
    return KL_OK;
}

int kl_batch_run(void *batch, void *stream)
{
    clear_error();
    if (!batch) return fail(KL_ERR_INVALID, "batch is NULL");
    Batch *b = (Batch *)batch;
    const hipError_t e = hipGraphLaunch(b->exec, (hipStream_t)stream);
    return e == hipSuccess ? KL_OK : hip_fail(e, "graph launch");
}

int kl_batch_info(void *batch, int32_t *n_kernels, int64_t *n_tiles)
{
    clear_error();
    if (!batch) return fail(KL_ERR_INVALID, "batch is NULL");
    Batch *b = (Batch *)batch;
    if (n_kernels) *n_kernels = b->nkernels;
    if (n_tiles) *n_tiles = b->ntiles;
    return KL_OK;
}

int kl_batch_destroy(void *batch)
{
    clear_error();
    if (!batch) return fail(KL_ERR_INVALID, "batch is NULL");
    delete (Batch *)batch;
    return KL_OK;
}

}  // extern "C"
