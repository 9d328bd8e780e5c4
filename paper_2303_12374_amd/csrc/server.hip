// Served form: a request loop with continuous batching.
//
// A request asks for `nsteps` forward-Euler steps of advec_u + diff_uvw on a
// grid it names; its fields are generated on the device from its seed and
// stay resident in the caller's arena until released.  A background thread
// runs ticks: between ticks it admits queued requests in arrival order while
// their footprint fits the memory budget (and the arena), and every tick
// advances all admitted requests by one fused step (advec_u + diff_uvw +
// forward Euler + ghost refill in one kernel, one persistent launch per
// configuration group), each request ping-ponging between two field
// buffers.  Requests therefore join and leave between ticks while others are
// running.  All per-point arithmetic is shared with the single-grid path, so
// a request's result does not depend on what it ran beside.  The host logic
// (arena, admission, tick loop, tickets) is served::Server of
// server_core.hpp; this file is its device executor and the C entry points.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "kl_internal.hpp"
#include "server_core.hpp"
#include "variants.hpp"

namespace kl {
namespace {

using served::ALIGN;
using served::Req;
using served::round_up;

// Vertical metrics of a served grid: centers-primary tanh stretch
// (gamma = 1.5, Lz = ktot / max(itot, jtot)) with z walls, uniform when
// z is periodic; ghosts by reflection, faces at midpoints of centers.
void served_metrics(const kl_request_t &q, std::vector<double> &dzi, std::vector<double> &dzhi, double *dzmin)
{
    const int kt = q.ktot, kc = kt + 2;
    const double Lz = (double)kt / (double)std::max(q.itot, q.jtot);
    const double gamma = q.bc == KL_BC_ZPERIODIC ? 0.0 : 1.5;
    std::vector<double> z(kc), zh(kc), dz(kc), dzh(kc);
    for (int k = 1; k <= kt; ++k) {
        const double s = (k - 0.5) / kt;
        z[k] = gamma == 0.0 ? (k - 0.5) * (Lz / kt) : Lz * (1.0 - tanh(gamma * (1.0 - s)) / tanh(gamma));
    }
    z[0] = -z[1];
    z[kt + 1] = 2.0 * Lz - z[kt];
    for (int k = 1; k <= kt + 1; ++k) zh[k] = 0.5 * (z[k - 1] + z[k]);
    zh[0] = -zh[2];
    for (int k = 1; k <= kt; ++k) dz[k] = zh[k + 1] - zh[k];
    dz[0] = dz[1];
    dz[kt + 1] = dz[kt];
    for (int k = 1; k <= kt + 1; ++k) dzh[k] = z[k] - z[k - 1];
    dzh[0] = dzh[1];
    dzi.resize(kc);
    dzhi.resize(kc);
    *dzmin = INFINITY;
    for (int k = 0; k < kc; ++k) {
        dzi[k] = 1.0 / dz[k];
        dzhi[k] = 1.0 / dzh[k];
        if (k >= 1 && k <= kt) *dzmin = std::min(*dzmin, dz[k]);
    }
}

struct DevBuf {
    void *d = nullptr;
    void *h = nullptr;
    size_t cap = 0;
    ~DevBuf()
    {
        if (d) (void)hipFree(d);
        if (h) (void)hipHostFree(h);
    }
    hipError_t ensure(size_t bytes)
    {
        if (bytes <= cap) return hipSuccess;
        if (d) (void)hipFree(d);
        if (h) (void)hipHostFree(h);
        d = h = nullptr;
        cap = std::max(bytes, (size_t)65536) * 2;
        hipError_t e = hipMalloc(&d, cap);
        if (e == hipSuccess) e = hipHostMalloc(&h, cap, hipHostMallocDefault);
        if (e != hipSuccess) cap = 0;
        return e;
    }
};

// Pinned host memory that kernels write directly (the checksums of the
// requests a tick finishes), grown on demand.
struct PinBuf {
    double *h = nullptr;
    size_t cap = 0;  // doubles
    ~PinBuf()
    {
        if (h) (void)hipHostFree(h);
    }
    hipError_t ensure(size_t n)
    {
        if (n <= cap) return hipSuccess;
        if (h) (void)hipHostFree(h);
        h = nullptr;
        cap = std::max(n, (size_t)4096) * 2;
        hipError_t e = hipHostMalloc((void **)&h, cap * sizeof(double), hipHostMallocDefault);
        if (e != hipSuccess) cap = 0;
        return e;
    }
};

// The served form's device work (the executor of served::Server): request
// set-up, one persistent fused-step launch per configuration group per tick,
// FP64 checksums of finished requests, and one event per tick slot, all on
// the server's own stream.
struct GpuExec {
    int device = 0, ncu = 256;
    hipStream_t stream = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    DevBuf tab[2];  // per-tick tables (descriptors, tiles), one per tick in flight
    // Checksums of the requests a tick finishes, written by the reduction's
    // last pass straight into pinned host memory of the tick's slot (reused
    // only after that tick has completed), so that publishing a finished
    // request takes no copy or synchronisation of its own.
    PinBuf sums[2];
    int cur_slot = 0;
    std::unordered_map<const Req *, const double *> pending;
    std::map<const Variant *, int> occ;  // resident blocks per CU of batched kernels
    // work queue of the persistent step kernels (two device ints): the kernels
    // run one after another on the server stream, and each returns it to zero
    int *d_queue = nullptr;

    hipError_t open()
    {
        hipError_t e = hipGetDevice(&device);
        hipDeviceProp_t prop;
        if (e == hipSuccess) e = hipGetDeviceProperties(&prop, device);
        if (e == hipSuccess) ncu = prop.multiProcessorCount;
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
        for (int n = 0; n < 2 && e == hipSuccess; ++n) e = hipEventCreateWithFlags(&ev[n], hipEventDisableTiming);
        if (e == hipSuccess) e = hipMalloc((void **)&d_queue, 2 * sizeof(int));
        if (e == hipSuccess) e = hipMemset(d_queue, 0, 2 * sizeof(int));
        return e;
    }

    ~GpuExec()
    {
        for (int n = 0; n < 2; ++n)
            if (ev[n]) (void)hipEventDestroy(ev[n]);
        if (stream) (void)hipStreamDestroy(stream);
        if (d_queue) (void)hipFree(d_queue);
    }

    void thread_init() { (void)hipSetDevice(device); }

    size_t footprint(const kl_request_t &q, int64_t *off, int64_t *js, int64_t *ks, int64_t *alloc)
    {
        kl_layout(q.itot, q.jtot, q.ktot, q.dtype, off, js, ks, alloc);
        const size_t s = q.dtype == KL_F32 ? 4 : 8;
        return 6 * round_up((size_t)*alloc * s) + 2 * round_up((size_t)(q.ktot + 2) * s);
    }

    // Lay out an admitted request in its arena block and queue its initial state.
    int init_request(Req &q, char *block)
    {
        int64_t off, js, ks, alloc;
        footprint(q.r, &off, &js, &ks, &alloc);
        const size_t s = q.r.dtype == KL_F32 ? 4 : 8;
        char *p = block;
        for (int n = 0; n < 6; ++n) {
            q.f[n] = p;
            p += round_up((size_t)alloc * s);
        }
        // dzi and dzhi back to back, as in the host copy: one upload
        char *dzi = p;
        char *dzhi = p + (size_t)(q.r.ktot + 2) * s;
        std::vector<double> mi, mhi;
        double dzmin;
        served_metrics(q.r, mi, mhi, &dzmin);
        const int kc = q.r.ktot + 2;
        q.metrics.resize(2 * kc * s);
        for (int k = 0; k < kc; ++k) {
            if (s == 4) {
                ((float *)q.metrics.data())[k] = (float)mi[k];
                ((float *)q.metrics.data())[kc + k] = (float)mhi[k];
            } else {
                ((double *)q.metrics.data())[k] = mi[k];
                ((double *)q.metrics.data())[kc + k] = mhi[k];
            }
        }
        q.g.itot = q.r.itot;
        q.g.jtot = q.r.jtot;
        q.g.ktot = q.r.ktot;
        q.g.gc = 1;
        q.g.off = off;
        q.g.jstride = js;
        q.g.kstride = ks;
        q.g.dxi = q.r.dtype == KL_F32 ? (double)(float)q.r.itot : (double)q.r.itot;
        q.g.dyi = q.r.dtype == KL_F32 ? (double)(float)q.r.jtot : (double)q.r.jtot;
        q.g.dzi = dzi;
        q.g.dzhi = dzhi;
        q.g.dtype = q.r.dtype;
        q.g.bc = q.r.bc;
        q.dt = q.r.dt > 0 ? q.r.dt : 0.1 * std::min(std::min(1.0 / q.r.itot, 1.0 / q.r.jtot), dzmin);
        hipError_t e = hipMemcpyAsync(dzi, q.metrics.data(), 2 * kc * s, hipMemcpyHostToDevice, stream);
        HostArgs a = make_args(&q.g);
        if (e == hipSuccess) e = launch_gen_uniform(a, q.r.seed, q.f[0], q.f[1], q.f[2], stream);
        if (e == hipSuccess) e = launch_fill_ghosts(a, q.f[0], q.f[1], q.f[2], stream);
        return e == hipSuccess ? KL_OK : hip_fail(e, "request init");
    }

    // Enqueue one tick on the server stream: every active request advances one
    // fused step from its current buffer into the other (the caller flips
    // each request's current buffer after this returns).  Tables go through
    // slot `slot`, which the previous use has released.
    int run_tick(int slot, const std::vector<Req *> &act, int64_t *launches)
    {
        cur_slot = slot;
        std::vector<StencilArgs<float>> df;
        std::vector<StencilArgs<double>> dd;
        std::vector<int> didx(act.size()), sel(act.size());
        std::vector<kl_grid_t> grids(act.size());
        std::vector<void *> fields(6 * act.size());
        std::map<std::tuple<int, int>, std::vector<int4>> groups;  // (dtype, configuration) -> tiles
        std::map<std::tuple<int, int>, std::vector<std::pair<int64_t, int4>>> sized;  // the same, with tile sizes
        for (size_t n = 0; n < act.size(); ++n) {
            Req &q = *act[n];
            void **f = fields.data() + 6 * n;
            for (int m = 0; m < 3; ++m) {
                f[m] = q.f[3 * q.cur + m];
                f[3 + m] = q.f[3 * (1 - q.cur) + m];
            }
            grids[n] = q.g;
            HostArgs a = make_args(&q.g);
            a.u = f[0];
            a.v = f[1];
            a.w = f[2];
            a.ut = f[3];
            a.vt = f[4];
            a.wt = f[5];
            a.visc = q.r.visc;
            a.dt = q.dt;
            if (q.g.dtype == KL_F32) {
                didx[n] = (int)df.size();
                df.push_back(device_args<float>(a));
            } else {
                didx[n] = (int)dd.size();
                dd.push_back(device_args<double>(a));
            }
            sel[n] = batch_variant(&q.g, KL_KERNEL_STEP, f);
            if (sel[n] < 0)
                return fail(KL_ERR_INVALID, "no step configuration for request %llu", (unsigned long long)q.ticket);
        }
        // as few groups (launches per tick) as the configurations allow; every
        // configuration gives the same bits, so a request may change group
        merge_batch_groups(KL_KERNEL_STEP, grids, fields.data(), sel);
        for (size_t n = 0; n < act.size(); ++n) {
            const Req &q = *act[n];
            const int vi = sel[n];
            const Variant &v = variants(KL_KERNEL_STEP, q.g.dtype)[vi];
            auto &tl = sized[std::make_tuple(q.g.dtype, vi)];
            const int tw = 64 * v.vx;
            const int nbx = (int)cdivu(q.g.itot, tw), nby = (int)cdivu(q.g.jtot, v.by), nbz = (int)cdivu(q.g.ktot, v.kb);
            for (int tz = 0; tz < nbz; ++tz)
                for (int ty = 0; ty < nby; ++ty)
                    for (int tx = 0; tx < nbx; ++tx)
                        tl.emplace_back((int64_t)std::min(tw, q.g.itot - tx * tw) * std::min(v.by, q.g.jtot - ty * v.by) *
                                            std::min(v.kb, q.g.ktot - tz * v.kb),
                                        make_int4(didx[n], tx, ty, tz));
        }
        // the blocks draw tiles from a queue: largest first (stable, so the tiles
        // of one request stay in order), as in the batched form
        for (auto &kv : sized) {
            std::stable_sort(kv.second.begin(), kv.second.end(),
                             [](const std::pair<int64_t, int4> &x, const std::pair<int64_t, int4> &y) {
                                 return x.first > y.first;
                             });
            auto &tl = groups[kv.first];
            for (const auto &t : kv.second) tl.push_back(t.second);
        }
        // pack tables: [desc f32][desc f64][group tiles...]
        size_t off = 0;
        auto place = [&](size_t bytes) {
            const size_t o = off;
            off += round_up(bytes);
            return o;
        };
        const size_t o_df = place(df.size() * sizeof(df[0])), o_dd = place(dd.size() * sizeof(dd[0]));
        std::vector<size_t> o_g;
        for (auto &kv : groups) o_g.push_back(place(kv.second.size() * sizeof(int4)));
        hipError_t e = tab[slot].ensure(off);
        if (e != hipSuccess) return hip_fail(e, "tick tables");
        char *h = (char *)tab[slot].h;
        char *d = (char *)tab[slot].d;
        memcpy(h + o_df, df.data(), df.size() * sizeof(df[0]));
        memcpy(h + o_dd, dd.data(), dd.size() * sizeof(dd[0]));
        {
            size_t gi = 0;
            for (auto &kv : groups) memcpy(h + o_g[gi++], kv.second.data(), kv.second.size() * sizeof(int4));
        }
        if ((e = hipMemcpyAsync(d, h, off, hipMemcpyHostToDevice, stream)) != hipSuccess) return hip_fail(e, "tables");
        const size_t o_desc[2] = {o_df, o_dd};
        size_t gi = 0;
        for (auto &kv : groups) {
            const int dt = std::get<0>(kv.first), vi = std::get<1>(kv.first);
            const Variant &v = variants(KL_KERNEL_STEP, dt)[vi];
            const int nt = (int)kv.second.size();
            auto oc = occ.find(&v);
            if (oc == occ.end()) oc = occ.emplace(&v, v.occupancy()).first;
            const int nb = persistent_blocks(nt, ncu, oc->second);
            if ((e = v.batch(d + o_desc[dt], d + o_g[gi], nt, nb, d_queue, stream)) != hipSuccess)
                return hip_fail(e, v.name);
            ++*launches;
            ++gi;
        }
        return KL_OK;
    }

    // Enqueue the FP64 checksums of requests whose last step was just enqueued.
    int enqueue_checksums(const std::vector<Req *> &done, int64_t *launches)
    {
        if (done.empty()) return KL_OK;
        void *ws = workspace(reduce_scratch_bytes(), stream);
        if (!ws) return fail(KL_ERR_NOMEM, "server workspace");
        PinBuf &pb = sums[cur_slot];
        const hipError_t ea = pb.ensure(9 * done.size());
        if (ea != hipSuccess) return hip_fail(ea, "checksum buffer");
        for (size_t n = 0; n < done.size(); ++n) {
            Req *q = done[n];
            void *const *cur = q->f + 3 * q->cur;
            double *out = pb.h + 9 * n;
            const hipError_t e = launch_reduce(make_args(&q->g), 1, cur[0], cur[1], cur[2], out, ws, stream);
            if (e != hipSuccess) return hip_fail(e, "checksum");
            pending[q] = out;
            ++*launches;
        }
        return KL_OK;
    }

    int record(int slot)
    {
        const hipError_t e = hipEventRecord(ev[slot], stream);
        return e == hipSuccess ? KL_OK : hip_fail(e, "tick event");
    }

    int wait(int slot)
    {
        const hipError_t e = hipEventSynchronize(ev[slot]);
        return e == hipSuccess ? KL_OK : hip_fail(e, "tick");
    }

    int fetch_checksum(Req &q)
    {
        auto it = pending.find(&q);
        if (it == pending.end()) return fail(KL_ERR_INVALID, "no checksum pending for request %llu",
                                             (unsigned long long)q.ticket);
        memcpy(q.checksum, it->second, 9 * sizeof(double));
        pending.erase(it);
        return KL_OK;
    }
};

typedef served::Server<GpuExec> Server;

}  // namespace
}  // namespace kl

using namespace kl;

extern "C" {

int kl_server_create(void *arena, size_t arena_bytes, size_t budget_bytes, void **srv)
{
    clear_error();
    if (!arena || !srv || arena_bytes == 0) return fail(KL_ERR_INVALID, "bad server arguments");
    if (budget_bytes == 0 || budget_bytes > arena_bytes) budget_bytes = arena_bytes;
    if ((uintptr_t)arena % ALIGN) return fail(KL_ERR_INVALID, "arena must be %zu-byte aligned", ALIGN);
    Server *S = new (std::nothrow) Server(arena, arena_bytes, budget_bytes);
    if (!S) return fail(KL_ERR_NOMEM, "server");
    const hipError_t e = S->exec.open();
    if (e != hipSuccess) {
        delete S;
        return hip_fail(e, "server create");
    }
    S->th = std::thread(served::server_loop<GpuExec>, S);
    *srv = S;
    return KL_OK;
}

int kl_submit(void *srv, const kl_request_t *req, uint64_t *ticket)
{
    clear_error();
    if (!srv || !req || !ticket) return fail(KL_ERR_INVALID, "NULL argument");
    return served::submit(*(Server *)srv, req, ticket);
}

int kl_poll(void *srv, uint64_t ticket, kl_result_t *out)
{
    clear_error();
    if (!srv || !out) return fail(KL_ERR_INVALID, "NULL argument");
    return served::poll(*(Server *)srv, ticket, out);
}

int kl_release(void *srv, uint64_t ticket)
{
    clear_error();
    if (!srv) return fail(KL_ERR_INVALID, "NULL server");
    return served::release(*(Server *)srv, ticket);
}

int kl_server_stats(void *srv, int64_t out[5])
{
    clear_error();
    if (!srv || !out) return fail(KL_ERR_INVALID, "NULL argument");
    served::stats(*(Server *)srv, out);
    return KL_OK;
}

int kl_server_destroy(void *srv)
{
    clear_error();
    if (!srv) return fail(KL_ERR_INVALID, "NULL server");
    Server *S = (Server *)srv;
    served::shutdown(*S);
    delete S;
    return KL_OK;
}

}  // extern "C"
