// Batched form: many independent grids advanced by persistent tile-walking
// kernels captured once in a HIP graph.
//
// Every grid runs advec_u followed by diff_uvw as one fused pass (the tile of
// kl_advec_diff: 9 values per point moved instead of 14, bitwise the result
// of the two separate kernels).  Each grid gets its configuration from the
// wisdom files like a single-grid launch (nearest problem size on this GPU,
// Section "Kernel Selection and Compilation"); grids whose selected
// configuration has no persistent form use an LDS z-march configuration
// sized to the grid.  The configuration selected for the most grid points
// then takes every grid it can serve, the next one the rest it can serve, and
// so on (all configurations give the same bits).  Grids are grouped by
// (dtype, configuration); every group becomes one persistent kernel whose
// blocks draw tiles from a work queue over the group's tile list, so the
// graph holds: [zero tendencies] -> the fused groups (one launch when one
// configuration serves every grid).
//
// A configuration that is fastest for one grid launched alone (where the
// launch is short and latency decides) need not be fastest inside a batch
// (where the GPU is full and bytes per tile decide), so a batch can also be
// tuned as a whole: kl_batch_tune times the batch with each configuration
// serving every grid it can and appends the fastest to
// advec_diff_batch.wisdom under the batch's signature (its multiset of
// grid shapes, boundary modes and dtype).  kl_batch_create takes a record
// with the batch's signature, for this GPU if there is one, else for this
// architecture, else any, before the per-grid selection.
#include <hip/hip_runtime.h>
#include <stdio.h>

#include <algorithm>
#include <chrono>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "json.hpp"
#include "kl_internal.hpp"
#include "variants.hpp"

namespace kl {
namespace {

struct Group {
    int kernel, dtype, variant;
    std::vector<int4> tiles;
    std::vector<int64_t> cost;  // grid points of each tile
    void *d_tiles = nullptr;
    int *d_queue = nullptr;  // work queue of the persistent kernel (two ints)
    int nblocks = 0;
};

struct Batch {
    std::vector<kl_grid_t> grids;
    std::vector<void *> fields;  // 6 per grid
    double visc = 0;
    bool zero = false;
    uint32_t flags = 0;        // KL_BATCH_* steps besides the tendencies
    double *sums = nullptr;    // caller's device array of 3 doubles per grid (KL_BATCH_SUMS)
    int forced[2] = {-1, -1};  // configuration serving every grid it can, per dtype (-1: per-grid selection)
    void *d_desc[2] = {nullptr, nullptr};  // StencilArgs<float>[] and StencilArgs<double>[], indexed by grid
    std::vector<int4> ztiles[2];
    void *d_ztiles[2] = {nullptr, nullptr};
    int zblocks[2] = {0, 0};
    std::vector<Group> groups;
    // ghost fill jobs and their blocks, per dtype
    void *d_fjobs[2] = {nullptr, nullptr}, *d_fblocks[2] = {nullptr, nullptr};
    int nfblocks[2] = {0, 0};
    // conservation-sum jobs per dtype and vector width, their pass-1 blocks, and the partials
    void *d_sjobs[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    void *d_sblocks[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    int nsjobs[2][2] = {{0, 0}, {0, 0}};
    int nsblocks[2][2] = {{0, 0}, {0, 0}};
    double *d_partials = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t ntiles = 0;
    int nkernels = 0;

    // release everything build() made, so that it can run again
    void release()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        for (int d = 0; d < 2; ++d) {
            if (d_desc[d]) (void)hipFree(d_desc[d]);
            if (d_ztiles[d]) (void)hipFree(d_ztiles[d]);
            d_desc[d] = nullptr;
            d_ztiles[d] = nullptr;
            ztiles[d].clear();
            zblocks[d] = 0;
        }
        for (auto &g : groups) {
            if (g.d_tiles) (void)hipFree(g.d_tiles);
            if (g.d_queue) (void)hipFree(g.d_queue);
        }
        for (int d = 0; d < 2; ++d) {
            for (void **p : {&d_fjobs[d], &d_fblocks[d], &d_sjobs[d][0], &d_sjobs[d][1], &d_sblocks[d][0],
                             &d_sblocks[d][1]}) {
                if (*p) (void)hipFree(*p);
                *p = nullptr;
            }
            nfblocks[d] = 0;
            nsjobs[d][0] = nsjobs[d][1] = 0;
            nsblocks[d][0] = nsblocks[d][1] = 0;
        }
        if (d_partials) (void)hipFree(d_partials);
        d_partials = nullptr;
        groups.clear();
        ntiles = 0;
        nkernels = 0;
    }

    ~Batch() { release(); }
};

}  // namespace

// Configuration of grid g for `kernel` in batched form.
int batch_variant(const kl_grid_t *g, int kernel, void *const f[6])
{
    const auto &vs = variants(kernel, g->dtype);
    const void *ptrs[6] = {f[0], f[1], f[2], f[3], f[4], f[5]};
    const int nptr = kernel_nptr(kernel);
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
    const int nptr = kernel_nptr(kernel);
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

// Whether configuration v can run grid g in a persistent kernel: it has a
// persistent form, fits the layout and pointers, and its wave segment (64 vx
// points) is no wider than the grid's rows.
bool serves(const Variant &v, const kl_grid_t *g, void *const *f)
{
    const void *ptrs[6] = {f[0], f[1], f[2], f[3], f[4], f[5]};
    return v.batch && 64 * v.vx <= std::max(64, g->itot) && variant_eligible(v, g, ptrs, 6);
}

// Signature of the grids of one dtype: FNV-1a over their sorted (itot, jtot,
// ktot, bc, gc) tuples, so that the same grids in any order match.
uint64_t batch_signature(const std::vector<kl_grid_t> &grids, int dtype, int64_t *npts, int *ngrids)
{
    std::vector<std::tuple<int, int, int, int, int>> key;
    *npts = 0;
    for (const kl_grid_t &g : grids)
        if (g.dtype == dtype) {
            key.emplace_back(g.itot, g.jtot, g.ktot, g.bc, g.gc);
            *npts += (int64_t)g.itot * g.jtot * g.ktot;
        }
    std::sort(key.begin(), key.end());
    *ngrids = (int)key.size();
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](int64_t x) {
        for (int q = 0; q < 8; ++q) {
            h ^= (uint64_t)((x >> (8 * q)) & 0xff);
            h *= 1099511628211ull;
        }
    };
    mix((int64_t)key.size());
    for (const auto &t : key) {
        mix(std::get<0>(t));
        mix(std::get<1>(t));
        mix(std::get<2>(t));
        mix(std::get<3>(t));
        mix(std::get<4>(t));
    }
    return h;
}

std::string batch_wisdom_path(const std::string &dir) { return dir + "/advec_diff_batch.wisdom"; }

std::string hex64(uint64_t x)
{
    char buf[24];
    snprintf(buf, sizeof buf, "%016llx", (unsigned long long)x);
    return buf;
}

// Configuration index recorded for this signature and dtype (this GPU, else
// this architecture, else any GPU; the later record wins within a level), or
// -1.  Records naming a configuration this build lacks are skipped.
int batch_wisdom_lookup(const std::string &dir, int dtype, uint64_t sig)
{
    std::ifstream in(batch_wisdom_path(dir));
    if (!in) return -1;
    DeviceIdent dev;
    const bool have_dev = current_device_ident(&dev) == KL_OK;
    const auto &vs = variants(KL_KERNEL_ADVEC_DIFF, dtype);
    int choice[3] = {-1, -1, -1};  // per level; -2 for a "per_grid" record
    std::string line;
    while (std::getline(in, line)) {
        JVal v;
        if (!parse_json(line, v) || v.kind != JVal::OBJ) continue;
        const JVal *k = v.get("kernel"), *dt = v.get("dtype"), *sg = v.get("signature"), *var = v.get("variant"),
                   *dn = v.get("device"), *ar = v.get("arch"), *cu = v.get("cu_count");
        if (!k || k->kind != JVal::STR || k->str != "advec_diff_batch") continue;
        if (!dt || dt->kind != JVal::STR || dt->str != (dtype == KL_F32 ? "f32" : "f64")) continue;
        if (!sg || sg->kind != JVal::STR || sg->str != hex64(sig)) continue;
        if (!var || var->kind != JVal::STR) continue;
        int idx = var->str == "per_grid" ? -2 : -1;  // -2: the per-grid selection was fastest
        for (size_t n = 0; n < vs.size(); ++n)
            if (var->str == vs[n].name && vs[n].batch) idx = (int)n;
        if (idx == -1) continue;
        const bool same_gpu = have_dev && dn && dn->kind == JVal::STR && dn->str == dev.name &&
                              (!cu || cu->kind != JVal::NUM || (int)cu->num == dev.cu_count);
        const bool same_arch = have_dev && ar && ar->kind == JVal::STR && ar->str == dev.arch;
        choice[same_gpu ? 0 : same_arch ? 1 : 2] = idx;
    }
    for (int l = 0; l < 3; ++l)
        if (choice[l] != -1) return choice[l] == -2 ? -1 : choice[l];
    return -1;
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
    {
        const int kernel = KL_KERNEL_ADVEC_DIFF;
        std::vector<int> sel(b.grids.size());
        for (size_t n = 0; n < b.grids.size(); ++n) {
            const kl_grid_t *g = &b.grids[n];
            const int fv = b.forced[g->dtype];
            if (fv >= 0 && serves(variants(kernel, g->dtype)[fv], g, fields + 6 * n)) {
                sel[n] = fv;
                continue;
            }
            sel[n] = batch_variant(g, kernel, fields + 6 * n);
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
            const int tw = 64 * v.vx;
            const int nbx = (int)cdivu(g->itot, tw), nby = (int)cdivu(g->jtot, v.by), nbz = (int)cdivu(g->ktot, v.kb);
            for (int tz = 0; tz < nbz; ++tz)
                for (int ty = 0; ty < nby; ++ty)
                    for (int tx = 0; tx < nbx; ++tx) {
                        gr.tiles.push_back(make_int4((int)n, tx, ty, tz));
                        gr.cost.push_back((int64_t)std::min(tw, g->itot - tx * tw) *
                                          std::min(v.by, g->jtot - ty * v.by) * std::min(v.kb, g->ktot - tz * v.kb));
                    }
        }
    }
    for (Group &gr : b.groups) {
        // The blocks draw tiles from a queue: the largest tiles go first, so
        // the walk ends on small ones and the blocks finish about level.  The
        // sort is stable, so the equal tiles of one grid stay in order and
        // neighbours (which share halo rows) are drawn close together.
        std::vector<size_t> ord(gr.tiles.size());
        for (size_t n = 0; n < ord.size(); ++n) ord[n] = n;
        std::stable_sort(ord.begin(), ord.end(), [&](size_t x, size_t y) { return gr.cost[x] > gr.cost[y]; });
        std::vector<int4> sorted(ord.size());
        for (size_t n = 0; n < ord.size(); ++n) sorted[n] = gr.tiles[ord[n]];
        gr.tiles.swap(sorted);
        if ((e = upload(&gr.d_tiles, gr.tiles.data(), gr.tiles.size() * sizeof(int4))) != hipSuccess)
            return hip_fail(e, "tiles");
        if ((e = hipMalloc((void **)&gr.d_queue, 2 * sizeof(int))) != hipSuccess) return hip_fail(e, "queue");
        if ((e = hipMemset(gr.d_queue, 0, 2 * sizeof(int))) != hipSuccess) return hip_fail(e, "queue");
        const Variant &v = variants(gr.kernel, gr.dtype)[gr.variant];
        gr.nblocks = persistent_blocks((int64_t)gr.tiles.size(), ncu, v.occupancy());
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
    // ghost fill and conservation-sum jobs, one per grid
    if (b.flags & KL_BATCH_FILL_GHOSTS) {
        std::vector<char> jobs[2];
        std::vector<int2> blocks[2];
        for (size_t n = 0; n < b.grids.size(); ++n) {
            const kl_grid_t *g = &b.grids[n];
            append_fill_job(make_args(g), fields[6 * n], fields[6 * n + 1], fields[6 * n + 2], jobs[g->dtype],
                            blocks[g->dtype]);
        }
        for (int d = 0; d < 2; ++d) {
            if (blocks[d].empty()) continue;
            if ((e = upload(&b.d_fjobs[d], jobs[d].data(), jobs[d].size())) != hipSuccess ||
                (e = upload(&b.d_fblocks[d], blocks[d].data(), blocks[d].size() * sizeof(int2))) != hipSuccess)
                return hip_fail(e, "fill jobs");
            b.nfblocks[d] = (int)blocks[d].size();
        }
    }
    if (b.flags & KL_BATCH_SUMS) {
        std::vector<char> jobs[2][2];
        std::vector<int2> blocks[2][2];
        for (size_t n = 0; n < b.grids.size(); ++n) {
            const kl_grid_t *g = &b.grids[n];
            const HostArgs a = make_args(g);
            void *const *f = fields + 6 * n;
            const int vec = reduce_vectorized(a, f[3], f[4], f[5]) ? 1 : 0;
            append_sum_job(a, f[3], f[4], f[5], (int)n, jobs[g->dtype][vec], blocks[g->dtype][vec]);
            ++b.nsjobs[g->dtype][vec];
        }
        for (int d = 0; d < 2; ++d)
            for (int v = 0; v < 2; ++v) {
                if (!b.nsjobs[d][v]) continue;
                if ((e = upload(&b.d_sjobs[d][v], jobs[d][v].data(), jobs[d][v].size())) != hipSuccess ||
                    (e = upload(&b.d_sblocks[d][v], blocks[d][v].data(), blocks[d][v].size() * sizeof(int2))) !=
                        hipSuccess)
                    return hip_fail(e, "sum jobs");
                b.nsblocks[d][v] = (int)blocks[d][v].size();
            }
        // the partials of blocks that own no rows stay +0.0 (they are never launched)
        const size_t pb = sums_partial_bytes((int)b.grids.size());
        if ((e = hipMalloc((void **)&b.d_partials, pb)) != hipSuccess) return hip_fail(e, "sum partials");
        if ((e = hipMemset(b.d_partials, 0, pb)) != hipSuccess) return hip_fail(e, "sum partials");
    }
    // the queue and partial-buffer clears above ran on the null stream: let
    // them finish before any replay can start on another stream
    if ((e = hipStreamSynchronize(nullptr)) != hipSuccess) return hip_fail(e, "batch set-up");
    // capture the graph on a private stream
    hipStream_t cs;
    if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e, "stream");
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    int rc = KL_OK;
    if (e != hipSuccess) rc = hip_fail(e, "begin capture");
    for (int d = 0; d < 2 && rc == KL_OK; ++d) {
        if (!b.nfblocks[d]) continue;
        e = launch_fill_batch(d, b.d_fjobs[d], b.d_fblocks[d], b.nfblocks[d], cs);
        if (e != hipSuccess) rc = hip_fail(e, "fill launch");
        ++b.nkernels;
    }
    for (int d = 0; d < 2 && rc == KL_OK; ++d) {
        if (!b.zero || b.ztiles[d].empty()) continue;
        e = launch_zero_batch(d, b.d_desc[d], b.d_ztiles[d], (int)b.ztiles[d].size(), b.zblocks[d], cs);
        if (e != hipSuccess) rc = hip_fail(e, "zero launch");
        ++b.nkernels;
    }
    for (Group &gr : b.groups) {
        if (rc != KL_OK) break;
        const Variant &v = variants(gr.kernel, gr.dtype)[gr.variant];
        e = v.batch(b.d_desc[gr.dtype], gr.d_tiles, (int)gr.tiles.size(), gr.nblocks, gr.d_queue, cs);
        if (e != hipSuccess) rc = hip_fail(e, v.name);
        ++b.nkernels;
    }
    if (b.flags & KL_BATCH_SUMS) {
        for (int d = 0; d < 2 && rc == KL_OK; ++d)
            for (int v = 0; v < 2 && rc == KL_OK; ++v) {
                if (!b.nsjobs[d][v]) continue;
                e = launch_sums_batch(d, v != 0, b.d_sjobs[d][v], b.d_sblocks[d][v], b.nsblocks[d][v], b.d_partials,
                                      cs);
                if (e != hipSuccess) rc = hip_fail(e, "sums launch");
                ++b.nkernels;
            }
        if (rc == KL_OK) {
            e = launch_sums_finish(b.d_partials, (int)b.grids.size(), b.sums, cs);
            if (e != hipSuccess) rc = hip_fail(e, "sums finish");
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
    return kl_batch_create_ex(grids, fields, n, visc, zero_tendencies ? KL_BATCH_ZERO_TENDENCIES : 0u, nullptr,
                              stream, batch);
}

int kl_batch_create_ex(const kl_grid_t *grids, void *const *fields, int32_t n, double visc, uint32_t flags,
                       double *sums, void *stream, void **batch)
{
    clear_error();
    (void)stream;
    if (!grids || !fields || !batch || n < 1) return fail(KL_ERR_INVALID, "bad batch arguments");
    const uint32_t known = KL_BATCH_ZERO_TENDENCIES | KL_BATCH_FILL_GHOSTS | KL_BATCH_SUMS;
    if (flags & ~known) return fail(KL_ERR_INVALID, "unknown batch flags 0x%x", flags & ~known);
    if ((flags & KL_BATCH_SUMS) && !sums) return fail(KL_ERR_INVALID, "KL_BATCH_SUMS needs a sums array");
    *batch = nullptr;
    for (int i = 0; i < n; ++i) {
        int rc = check_grid(&grids[i]);
        if (rc) return fail(rc, "grid %d: %s", i, kl_last_error());
        for (int f = 0; f < 6; ++f)
            if (!fields[6 * i + f]) return fail(KL_ERR_INVALID, "grid %d field %d is NULL", i, f);
        if ((flags & KL_BATCH_FILL_GHOSTS) && fill_cell_count(make_args(&grids[i])) >= ((int64_t)1 << 32))
            return fail(KL_ERR_INVALID, "grid %d: 2^32 or more ghost cells", i);
        if ((flags & KL_BATCH_SUMS) && (int64_t)grids[i].jtot * grids[i].ktot >= ((int64_t)1 << 31))
            return fail(KL_ERR_INVALID, "grid %d: 2^31 or more rows to sum", i);
    }
    Batch *b = new (std::nothrow) Batch();
    if (!b) return fail(KL_ERR_NOMEM, "batch");
    b->grids.assign(grids, grids + n);
    b->fields.assign(fields, fields + 6 * (size_t)n);
    b->visc = visc;
    b->zero = (flags & KL_BATCH_ZERO_TENDENCIES) != 0;
    b->flags = flags;
    b->sums = (flags & KL_BATCH_SUMS) ? sums : nullptr;
    for (int dt = 0; dt < 2; ++dt) {
        int64_t np;
        int ng;
        const uint64_t sig = batch_signature(b->grids, dt, &np, &ng);
        if (ng > 0) b->forced[dt] = batch_wisdom_lookup(wisdom_dir(), dt, sig);
    }
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

int kl_batch_group(void *batch, int32_t group, int32_t *dtype, char *name, size_t len, int64_t *n_tiles)
{
    clear_error();
    if (!batch) return fail(KL_ERR_INVALID, "batch is NULL");
    Batch *b = (Batch *)batch;
    if (group < 0 || group >= (int)b->groups.size()) return fail(KL_ERR_NOTFOUND, "group %d", group);
    const Group &gr = b->groups[group];
    if (dtype) *dtype = gr.dtype;
    if (name && len) snprintf(name, len, "%s", variants(gr.kernel, gr.dtype)[gr.variant].name);
    if (n_tiles) *n_tiles = (int64_t)gr.tiles.size();
    return KL_OK;
}

int kl_batch_tune(void *batch, const char *wisdom_dir_, double budget_s, void *stream, double *timings_out,
                  int32_t max_timings, int32_t *n_timings)
{
    clear_error();
    if (!batch) return fail(KL_ERR_INVALID, "batch is NULL");
    Batch *b = (Batch *)batch;
    hipStream_t s = (hipStream_t)stream;
    const std::string dir = wisdom_dir_ && *wisdom_dir_ ? std::string(wisdom_dir_) : wisdom_dir();
    if (n_timings) *n_timings = 0;
    DeviceIdent dev;
    int rc = current_device_ident(&dev);
    if (rc) return rc;
    const size_t ng = b->grids.size();
    uint64_t *dhash = nullptr;
    hipError_t e = hipMalloc((void **)&dhash, 3 * ng * sizeof(uint64_t));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc");
    std::vector<uint64_t> hh(3 * ng);
    hipEvent_t ev[2] = {nullptr, nullptr};
    for (auto &x : ev)
        if ((e = hipEventCreate(&x)) != hipSuccess) rc = hip_fail(e, "hipEventCreate");
    void *ws = workspace(reduce_scratch_bytes(), s);
    if (!ws && rc == KL_OK) rc = fail(KL_ERR_NOMEM, "tune workspace");

    // zero the tendencies of the grids of dtype dt, replay once, and return
    // the sum of the outputs' bit hashes
    auto run_and_hash = [&](int dt, uint64_t *sum) -> int {
        for (size_t n = 0; n < ng; ++n) {
            if (b->grids[n].dtype != dt) continue;
            const HostArgs a = make_args(&b->grids[n]);
            for (int q = 3; q < 6; ++q)
                if ((e = launch_zero_interior(a, b->fields[6 * n + q], s)) != hipSuccess) return hip_fail(e, "zero");
        }
        if ((e = hipGraphLaunch(b->exec, s)) != hipSuccess) return hip_fail(e, "graph launch");
        for (size_t n = 0; n < ng; ++n) {
            if (b->grids[n].dtype != dt) continue;
            const HostArgs a = make_args(&b->grids[n]);
            for (int q = 0; q < 3; ++q)
                if ((e = launch_hash(a, b->fields[6 * n + 3 + q], dhash + 3 * n + q, ws, s)) != hipSuccess)
                    return hip_fail(e, "hash");
        }
        if ((e = hipMemcpyAsync(hh.data(), dhash, hh.size() * sizeof(uint64_t), hipMemcpyDeviceToHost, s)) !=
                hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return hip_fail(e, "hash copy");
        uint64_t acc = 0;
        for (size_t n = 0; n < ng; ++n)
            if (b->grids[n].dtype == dt) acc += hh[3 * n] * 3 + hh[3 * n + 1] * 5 + hh[3 * n + 2] * 7;
        *sum = acc;
        return KL_OK;
    };
    auto time_replays = [&](double *ms) -> int {
        for (int w = 0; w < 2; ++w)
            if ((e = hipGraphLaunch(b->exec, s)) != hipSuccess) return hip_fail(e, "graph launch");
        const int reps = 10;
        if ((e = hipEventRecord(ev[0], s)) != hipSuccess) return hip_fail(e, "event");
        for (int r = 0; r < reps; ++r)
            if ((e = hipGraphLaunch(b->exec, s)) != hipSuccess) return hip_fail(e, "graph launch");
        if ((e = hipEventRecord(ev[1], s)) != hipSuccess || (e = hipEventSynchronize(ev[1])) != hipSuccess)
            return hip_fail(e, "event");
        float t = 0;
        if ((e = hipEventElapsedTime(&t, ev[0], ev[1])) != hipSuccess) return hip_fail(e, "event");
        *ms = t / reps;
        return KL_OK;
    };
    auto rebuild = [&]() -> int {
        b->release();
        return build(*b, b->fields.data());
    };

    const auto t_start = std::chrono::steady_clock::now();
    int nt = 0;
    for (int dt = 0; dt < 2 && rc == KL_OK; ++dt) {
        int64_t npts;
        int ngr;
        const uint64_t sig = batch_signature(b->grids, dt, &npts, &ngr);
        if (ngr == 0) continue;
        const auto &vs = variants(KL_KERNEL_ADVEC_DIFF, dt);
        // candidate -1 is the per-grid selection; then every persistent configuration
        std::vector<int> cand = {-1};
        for (size_t n = 0; n < vs.size(); ++n)
            if (vs[n].batch) cand.push_back((int)n);
        uint64_t ref = 0;
        double best_ms = 1e300, sel_ms = -1;
        int best = -1, evaluated = 0;
        for (size_t c = 0; c < cand.size() && rc == KL_OK; ++c) {
            if (c > 0 && std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count() > budget_s)
                break;
            b->forced[dt] = cand[c];
            if ((rc = rebuild())) break;
            uint64_t h = 0;
            if ((rc = run_and_hash(dt, &h))) break;
            double ms = -1;
            if (c == 0)
                ref = h;
            if (h == ref) {
                if ((rc = time_replays(&ms))) break;
                if (c == 0) sel_ms = ms;
                if (ms < best_ms) {
                    best_ms = ms;
                    best = cand[c];
                }
            }
            ++evaluated;
            if (timings_out && nt < max_timings) {
                timings_out[2 * nt] = cand[c];
                timings_out[2 * nt + 1] = ms;
                ++nt;
            }
        }
        if (rc) break;
        b->forced[dt] = best;
        std::ostringstream o;
        o << "{\"kernel\":\"advec_diff_batch\",\"dtype\":\"" << (dt == KL_F32 ? "f32" : "f64")
          << "\",\"signature\":\"" << hex64(sig) << "\",\"grids\":" << ngr << ",\"points\":" << npts
          << ",\"variant\":\"" << (best >= 0 ? vs[best].name : "per_grid") << "\",\"time_ms\":" << best_ms
          << ",\"per_grid_selection_ms\":" << sel_ms << ",\"evaluated\":" << evaluated << ","
          << provenance_json(dev) << "}";
        rc = wisdom_append_file(dir, "advec_diff_batch.wisdom", o.str());
    }
    if (rc == KL_OK) rc = rebuild();
    for (auto x : ev)
        if (x) (void)hipEventDestroy(x);
    (void)hipFree(dhash);
    if (n_timings) *n_timings = nt;
    return rc;
}

int kl_batch_destroy(void *batch)
{
    clear_error();
    if (!batch) return fail(KL_ERR_INVALID, "batch is NULL");
    delete (Batch *)batch;
    return KL_OK;
}

}  // extern "C"
