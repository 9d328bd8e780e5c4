// kl_tune: measure every eligible configuration of a kernel on one grid and
// append the fastest to the kernel's wisdom file (Section "Kernel Tuning":
// the paper drives Kernel Tuner over captured launches for a bounded time;
// here the configuration space is the small set of ahead-of-time compiled
// gfx950 configurations, so it is searched exhaustively within the budget).
#include <hip/hip_runtime.h>
#include <stdio.h>

#include <algorithm>
#include <chrono>
#include <sstream>
#include <string>
#include <vector>

#include "kl_internal.hpp"

using namespace kl;

namespace {

struct Guard {
    std::vector<hipEvent_t> ev;
    uint64_t *dhash = nullptr;
    ~Guard()
    {
        for (auto e : ev) (void)hipEventDestroy(e);
        if (dhash) (void)hipFree(dhash);
    }
};

// Zero the interiors of the outputs `kernel` accumulates into (ut; or ut, vt, wt).
int zero_tendencies(const kl_grid_t *g, int kernel, void *const *f, hipStream_t s)
{
    const HostArgs a = make_args(g);
    const int nout = kernel_nptr(kernel) == 4 ? 1 : 3;
    for (int n = 3; n < 3 + nout; ++n) {
        const hipError_t e = launch_zero_interior(a, f[n], s);
        if (e != hipSuccess) return hip_fail(e, "zero tendencies");
    }
    return KL_OK;
}

// Hashes of the outputs of `kernel` (ut; or ut, vt, wt) into host h[3].
int output_hashes(const kl_grid_t *g, int kernel, void *const *f, uint64_t *dhash, uint64_t h[3], hipStream_t s)
{
    void *ws = workspace(reduce_scratch_bytes(), s);
    if (!ws) return fail(KL_ERR_NOMEM, "tune workspace");
    const HostArgs a = make_args(g);
    const int nout = kernel_nptr(kernel) == 4 ? 1 : 3;
    for (int n = 0; n < nout; ++n) {
        hipError_t e = launch_hash(a, f[3 + n], dhash + n, ws, s);
        if (e != hipSuccess) return hip_fail(e, "hash");
    }
    hipError_t e = hipMemcpyAsync(h, dhash, sizeof(uint64_t) * nout, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hash copy");
    for (int n = nout; n < 3; ++n) h[n] = 0;
    return KL_OK;
}

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Advection kernel a diffusion kernel follows in a time step of its scheme.
int partner_of(int kernel)
{
    return kernel == KL_KERNEL_DIFF_UVW ? KL_KERNEL_ADVEC_U : (kernel == KL_KERNEL_DIFF_SMAG ? KL_KERNEL_ADVEC_U_2I5 : -1);
}

// Algorithmic values moved per grid point (read + written).
int values_per_point(int kernel)
{
    switch (kernel) {
    case KL_KERNEL_ADVEC_U:
    case KL_KERNEL_ADVEC_U_2I5: return 5;
    case KL_KERNEL_DIFF_UVW:
    case KL_KERNEL_ADVEC_DIFF: return 9;
    case KL_KERNEL_DIFF_SMAG: return 10;
    default: return 6;
    }
}

int tune_one(const kl_grid_t *g, int kernel, void *const *f, const std::string &dir, double budget_s,
             hipStream_t s, double *timings_out, int max_timings, int *n_timings, bool after_advec)
{
    Guard gd;
    hipError_t e = hipMalloc(&gd.dhash, 3 * sizeof(uint64_t));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc");
    const auto &vs = variants(kernel, g->dtype);
    const void *const *ptrs = (const void *const *)f;
    const int nptr = kernel_nptr(kernel);
    const double visc = 1e-5, dt = 1e-4;
    int rc;

    // reference output of the default configuration
    uint64_t ref[3];
    if ((rc = zero_tendencies(g, kernel, f, s))) return rc;
    if ((rc = run_variant(g, kernel, 0, f, visc, s, dt))) return rc;
    if ((rc = output_hashes(g, kernel, f, gd.dhash, ref, s))) return rc;

    // In pair mode a diffusion kernel is timed right after the selected
    // advection kernel of its scheme, as it runs in a time step, so the
    // memory-side cache state it starts from is the one advection leaves.
    // advec_u_2i5 needs three ghost cells; on a narrower grid diff_smag is
    // timed on its own.
    int pk = after_advec ? partner_of(kernel) : -1;
    if (pk == KL_KERNEL_ADVEC_U_2I5 && g->gc < 3) pk = -1;
    int adv = pk >= 0 ? select_variant(g, pk) : -1;
    if (adv > 0 && !variant_eligible(variants(pk, g->dtype)[adv], g, ptrs, 4)) adv = 0;
    auto before = [&]() { return adv >= 0 ? run_variant(g, pk, adv, f, visc, s, dt) : KL_OK; };
    const int reps = 15, warm = 3;
    gd.ev.resize(2 * reps);
    for (auto &ev : gd.ev)
        if ((e = hipEventCreate(&ev)) != hipSuccess) return hip_fail(e, "hipEventCreate");

    const double t0 = now_s();
    int best = 0;
    double best_ms = 1e300, default_ms = -1;
    int count = 0;
    for (int idx = 0; idx < (int)vs.size(); ++idx) {
        if (idx > 0 && now_s() - t0 > budget_s) break;
        if (!variant_eligible(vs[idx], g, ptrs, nptr)) continue;
        double ms = -1.0;
        uint64_t h[3];
        if ((rc = zero_tendencies(g, kernel, f, s))) return rc;
        if ((rc = run_variant(g, kernel, idx, f, visc, s, dt))) return rc;
        if ((rc = output_hashes(g, kernel, f, gd.dhash, h, s))) return rc;
        if (h[0] == ref[0] && h[1] == ref[1] && h[2] == ref[2]) {
            for (int r = 0; r < warm; ++r) {
                if ((rc = before())) return rc;
                if ((rc = run_variant(g, kernel, idx, f, visc, s, dt))) return rc;
            }
            for (int r = 0; r < reps; ++r) {
                if ((rc = before())) return rc;
                (void)hipEventRecord(gd.ev[2 * r], s);
                if ((rc = run_variant(g, kernel, idx, f, visc, s, dt))) return rc;
                (void)hipEventRecord(gd.ev[2 * r + 1], s);
            }
            if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "tune sync");
            std::vector<float> t(reps);
            for (int r = 0; r < reps; ++r) (void)hipEventElapsedTime(&t[r], gd.ev[2 * r], gd.ev[2 * r + 1]);
            std::sort(t.begin(), t.end());
            ms = t[reps / 2];
            if (idx == 0) default_ms = ms;
            if (ms < best_ms) {
                best_ms = ms;
                best = idx;
            }
        }
        if (timings_out && count < max_timings) {
            timings_out[2 * count] = idx;
            timings_out[2 * count + 1] = ms;
        }
        ++count;
    }
    if (n_timings) *n_timings = std::min(count, max_timings);

    DeviceIdent id;
    if ((rc = current_device_ident(&id))) return rc;
    const double npts = (double)g->itot * g->jtot * g->ktot;
    const int values = values_per_point(kernel);
    const double bytes = npts * values * (g->dtype == KL_F32 ? 4 : 8);
    const Variant &v = vs[best];
    std::ostringstream o;
    o.precision(6);
    o << "{\"kernel\":\"" << kernel_name(kernel) << "\",\"dtype\":\"" << (g->dtype == KL_F32 ? "f32" : "f64")
      << "\",\"problem_size\":[" << g->itot << "," << g->jtot << "," << g->ktot << "],"
      << "\"variant\":\"" << v.name << "\",\"params\":{\"family\":" << v.family << ",\"vx\":" << v.vx
      << ",\"bx\":" << v.bx << ",\"by\":" << v.by << ",\"kb\":" << v.kb << ",\"xcd\":" << v.xcd << "},"
      << "\"time_ms\":" << best_ms << ",\"default_ms\":" << default_ms << ",\"gbps\":" << bytes / (best_ms * 1e6)
      << ",\"bc\":" << g->bc << ",\"evaluated\":" << count << ",\"after_advec\":" << (after_advec ? 1 : 0) << ","
      << provenance_json(id) << "}";
    if ((rc = wisdom_append(dir, kernel, o.str()))) return rc;
    return KL_OK;
}

}  // namespace

// kl_tune mask bit of each kernel.
uint32_t tune_bit(int kernel)
{
    static const uint32_t bits[KL_NUM_KERNELS] = {KL_TUNE_ADVEC_U, KL_TUNE_DIFF_UVW, KL_TUNE_STEP,
                                                  KL_TUNE_ADVEC_U_2I5, KL_TUNE_DIFF_SMAG, KL_TUNE_ADVEC_DIFF};
    return bits[kernel];
}

extern "C" int kl_tune(const kl_grid_t *g, void *const fields[6], uint32_t kernel_mask, const char *wisdom_dir_,
                       double budget_s, void *stream, double *timings_out, int32_t max_timings, int32_t *n_timings)
{
    clear_error();
    int rc = check_grid(g);
    if (rc) return rc;
    if (!fields) return fail(KL_ERR_INVALID, "fields is NULL");
    const uint32_t kernels = KL_TUNE_ADVEC_U | KL_TUNE_DIFF_UVW | KL_TUNE_STEP | KL_TUNE_ADVEC_U_2I5 |
                             KL_TUNE_DIFF_SMAG | KL_TUNE_ADVEC_DIFF;
    if ((kernel_mask & kernels) == 0 || (kernel_mask & ~(kernels | KL_TUNE_PAIR)))
        return fail(KL_ERR_INVALID, "kernel_mask %u", kernel_mask);
    const int nf = (kernel_mask & KL_TUNE_DIFF_SMAG) ? 7 : 6;
    for (int n = 0; n < nf; ++n)
        if (!fields[n]) return fail(KL_ERR_INVALID, "field %d is NULL", n);
    const bool pair = (kernel_mask & KL_TUNE_PAIR) != 0;
    if (n_timings) *n_timings = 0;
    const std::string dir = wisdom_dir_ && *wisdom_dir_ ? std::string(wisdom_dir_) : wisdom_dir();
    bool first = true;
    for (int kernel = 0; kernel < KL_NUM_KERNELS; ++kernel) {
        if (!(kernel_mask & tune_bit(kernel))) continue;
        if (kernel == KL_KERNEL_ADVEC_U_2I5 && g->gc < 3)
            return fail(KL_ERR_INVALID, "advec_u_2i5 needs gc = 3 ghost cells in x and y");
        rc = tune_one(g, kernel, fields, dir, budget_s, (hipStream_t)stream, first ? timings_out : nullptr,
                      max_timings, first ? n_timings : nullptr, pair && partner_of(kernel) >= 0);
        clear_plans();  // a kernel tuned above is selected for the ones that follow
        if (rc) return rc;
        first = false;
    }
    clear_plans();
    return KL_OK;
}
