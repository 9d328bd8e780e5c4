// C-ABI entry points: argument checks, layout, the selection cache and
// dispatch of the tendency kernels, ghost fill, Euler step and reductions.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "kl_internal.hpp"

#define KL_VERSION_STRING "klstencil 0.1.0 (gfx950)"

namespace kl {

namespace {
thread_local std::string g_last_error;
}

int fail(int code, const char *fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(KL_ERR_DEVICE, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

void clear_error() { g_last_error.clear(); }

const std::vector<Variant> &variants(int kernel, int dtype)
{
    return dtype == KL_F32 ? variants_f32(kernel) : variants_f64(kernel);
}

int check_grid(const kl_grid_t *g)
{
    if (!g) return fail(KL_ERR_INVALID, "grid is NULL");
    if (g->gc != 1 && g->gc != 3) return fail(KL_ERR_INVALID, "ghost width gc=%d, must be 1 or 3", g->gc);
    if (g->dtype != KL_F32 && g->dtype != KL_F64) return fail(KL_ERR_INVALID, "dtype %d", g->dtype);
    if (g->bc < KL_BC_ZWALL_ZEROGRAD || g->bc > KL_BC_ZPERIODIC) return fail(KL_ERR_INVALID, "bc %d", g->bc);
    if (g->itot < 1 || g->jtot < 1 || g->ktot < 1)
        return fail(KL_ERR_INVALID, "interior sizes %d x %d x %d must be >= 1", g->itot, g->jtot, g->ktot);
    if (g->bc != KL_BC_ZPERIODIC && g->ktot < 2)
        return fail(KL_ERR_INVALID, "z walls need ktot >= 2 (got %d)", g->ktot);
    const int64_t gc = g->gc;
    if (g->jstride < (int64_t)g->itot + 2 * gc)
        return fail(KL_ERR_INVALID, "jstride %lld < itot+2*gc", (long long)g->jstride);
    if (g->kstride < g->jstride * ((int64_t)g->jtot + 2 * gc))
        return fail(KL_ERR_INVALID, "kstride %lld < jstride*(jtot+2*gc)", (long long)g->kstride);
    if (g->off < (gc - 1) * (g->jstride + 1))
        return fail(KL_ERR_INVALID, "off %lld < (gc-1)*(jstride+1): ghost cells before the buffer",
                    (long long)g->off);
    if (!g->dzi || !g->dzhi) return fail(KL_ERR_INVALID, "dzi/dzhi is NULL");
    return KL_OK;
}

HostArgs make_args(const kl_grid_t *g)
{
    HostArgs a;
    memset(&a, 0, sizeof a);
    a.itot = g->itot;
    a.jtot = g->jtot;
    a.ktot = g->ktot;
    a.kw0 = g->bc == KL_BC_ZPERIODIC ? 1 : 2;
    a.gc = g->gc;
    a.dtype = g->dtype;
    a.bc = g->bc;
    a.off = g->off;
    a.js = g->jstride;
    a.ks = g->kstride;
    a.dxi = g->dxi;
    a.dyi = g->dyi;
    a.dzi = g->dzi;
    a.dzhi = g->dzhi;
    return a;
}

bool variant_eligible(const Variant &v, const kl_grid_t *g, const void *const *ptrs, int nptr)
{
    if (v.vx > 1) {
        const int64_t vx = v.vx;
        if (g->itot % vx || (g->off + 1) % vx || g->jstride % vx || g->kstride % vx) return false;
        const uintptr_t align = (uintptr_t)vx * (g->dtype == KL_F32 ? 4 : 8);
        for (int n = 0; n < nptr; ++n)
            if (ptrs[n] && ((uintptr_t)ptrs[n] % align)) return false;
    }
    return true;
}

// ---------------------------------------------------------------------------
// per-device, per-stream workspace for reduction partials (never freed)
// ---------------------------------------------------------------------------
namespace {
std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, void *> g_ws;
constexpr size_t WS_BYTES = 512 * 1024;
}  // namespace

void *workspace(size_t bytes, hipStream_t s)
{
    if (bytes > WS_BYTES) return nullptr;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(g_ws_mu);
    auto key = std::make_pair(dev, s);
    auto it = g_ws.find(key);
    if (it != g_ws.end()) return it->second;
    void *p = nullptr;
    if (hipMalloc(&p, WS_BYTES) != hipSuccess) return nullptr;
    g_ws[key] = p;
    return p;
}

// ---------------------------------------------------------------------------
// selection cache: (kernel, dtype, itot, jtot, ktot, device) -> variant index
// ---------------------------------------------------------------------------
namespace {
std::mutex g_plan_mu;
std::map<std::tuple<int, int, int, int, int, int>, int> g_plans;
}  // namespace

void clear_plans()
{
    std::lock_guard<std::mutex> lk(g_plan_mu);
    g_plans.clear();
}

int select_variant(const kl_grid_t *g, int kernel)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = -1;
    const auto key = std::make_tuple(kernel, g->dtype, g->itot, g->jtot, g->ktot, dev);
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        auto it = g_plans.find(key);
        if (it != g_plans.end()) return it->second;
    }
    int index = 0;
    DeviceIdent id;
    if (current_device_ident(&id) == KL_OK) {
        std::string name;
        int level = 5;
        if (wisdom_select(wisdom_dir(), kernel, g->dtype, id, g->itot, g->jtot, g->ktot, &name, &level) ==
                KL_OK &&
            level < 5) {
            const auto &vs = variants(kernel, g->dtype);
            for (size_t n = 0; n < vs.size(); ++n)
                if (name == vs[n].name) index = (int)n;
        }
    }
    std::lock_guard<std::mutex> lk(g_plan_mu);
    g_plans[key] = index;
    return index;
}

int run_variant(const kl_grid_t *g, int kernel, int index, void *const *fields, double visc, hipStream_t s,
                double dt)
{
    const auto &vs = variants(kernel, g->dtype);
    if (index < 0 || index >= (int)vs.size()) return fail(KL_ERR_NOTFOUND, "variant index %d", index);
    if (kernel == KL_KERNEL_ADVEC_U_2I5 && g->gc < 3)
        return fail(KL_ERR_INVALID, "advec_u_2i5 needs gc = 3 ghost cells in x and y (grid has %d)", g->gc);
    const Variant &v = vs[index];
    const int nptr = kernel_nptr(kernel);
    if (!variant_eligible(v, g, (const void *const *)fields, nptr))
        return fail(KL_ERR_INVALID, "configuration %s not eligible for this grid/alignment", v.name);
    HostArgs a = make_args(g);
    a.dt = dt;
    a.u = fields[0];
    a.v = fields[1];
    a.w = fields[2];
    a.ut = fields[3];
    a.vt = fields[4];
    a.wt = fields[5];
    a.evisc = nptr > 6 ? fields[6] : nullptr;
    a.visc = visc;
    const hipError_t e = v.launch(a, s);
    if (e != hipSuccess) return hip_fail(e, v.name);
    return KL_OK;
}

}  // namespace kl

using namespace kl;

namespace {

int check_ptrs(const void *const *p, int n)
{
    for (int i = 0; i < n; ++i)
        if (!p[i]) return fail(KL_ERR_INVALID, "field pointer %d is NULL", i);
    return KL_OK;
}

// Launch `kernel` with the selected configuration, falling back to the
// default when the selected one does not fit this call's alignment.
int launch_selected(const kl_grid_t *g, int kernel, void *const *fields, double visc, hipStream_t s,
                    double dt = 0.0)
{
    int index = select_variant(g, kernel);
    const auto &vs = variants(kernel, g->dtype);
    const void *const *ptrs = (const void *const *)fields;
    const int nptr = kernel_nptr(kernel);
    if (!variant_eligible(vs[index], g, ptrs, nptr)) index = 0;
    if (!variant_eligible(vs[index], g, ptrs, nptr))
        return fail(KL_ERR_INVALID, "no configuration of %s fits this grid/alignment", kernel_name(kernel));
    const int rc = maybe_capture(g, kernel, fields, visc, dt, s);
    if (rc) return rc;
    return run_variant(g, kernel, index, fields, visc, s, dt);
}

bool kernel_ok(int32_t kernel) { return kernel >= 0 && kernel < KL_NUM_KERNELS; }

}  // namespace

extern "C" {

const char *kl_version(void) { return KL_VERSION_STRING; }

const char *kl_last_error(void) { return g_last_error.c_str(); }

int kl_layout_gc(int32_t itot, int32_t jtot, int32_t ktot, int32_t dtype, int32_t gc, int64_t *off,
                 int64_t *jstride, int64_t *kstride, int64_t *alloc_elems)
{
    clear_error();
    if (itot < 1 || jtot < 1 || ktot < 1) return fail(KL_ERR_INVALID, "sizes must be >= 1");
    if (dtype != KL_F32 && dtype != KL_F64) return fail(KL_ERR_INVALID, "dtype %d", dtype);
    if (gc != 1 && gc != 3) return fail(KL_ERR_INVALID, "gc %d must be 1 or 3", gc);
    if (!off || !jstride || !kstride || !alloc_elems) return fail(KL_ERR_INVALID, "NULL output");
    const int64_t line = 128 / (dtype == KL_F32 ? 4 : 8);  // elements per 128-byte line
    const int64_t js = ((int64_t)itot + 2 * gc + line - 1) / line * line;
    const int64_t o = (gc - 1) * js + line - 1;  // idx(1, j, k) on a line boundary
    const int64_t ks = js * ((int64_t)jtot + 2 * gc);
    *off = o;
    *jstride = js;
    *kstride = ks;
    *alloc_elems = o + ks * ((int64_t)ktot + 2) + 2 * line;
    return KL_OK;
}

int kl_layout(int32_t itot, int32_t jtot, int32_t ktot, int32_t dtype, int64_t *off, int64_t *jstride,
              int64_t *kstride, int64_t *alloc_elems)
{
    return kl_layout_gc(itot, jtot, ktot, dtype, 1, off, jstride, kstride, alloc_elems);
}

int kl_fill_ghosts(const kl_grid_t *g, void *u, void *v, void *w, void *stream)
{
    clear_error();
    int rc = check_grid(g);
    if (rc) return rc;
    const void *p[3] = {u, v, w};
    if ((rc = check_ptrs(p, 3))) return rc;
    const hipError_t e = launch_fill_ghosts(make_args(g), u, v, w, (hipStream_t)stream);
    return e == hipSuccess ? KL_OK : hip_fail(e, "fill_ghosts");
}

int kl_fill_scalar(const kl_grid_t *g, void *f, void *stream)
{
    clear_error();
    int rc = check_grid(g);
    if (rc) return rc;
    if (!f) return fail(KL_ERR_INVALID, "field pointer is NULL");
    const hipError_t e = launch_fill_scalar(make_args(g), f, (hipStream_t)stream);
    return e == hipSuccess ? KL_OK : hip_fail(e, "fill_scalar");
}

int kl_advec_u_2i5(const kl_grid_t *g, void *ut, const void *u, const void *v, const void *w, void *stream)
{
    clear_error();
    int rc = check_grid(g);
    if (rc) return rc;
    if (g->gc < 3) return fail(KL_ERR_INVALID, "advec_u_2i5 needs gc = 3 ghost cells in x and y (grid has %d)", g->gc);
    const void *p[4] = {u, v, w, ut};
    if ((rc = check_ptrs(p, 4))) return rc;
    void *f[6] = {(void *)u, (void *)v, (void *)w, ut, nullptr, nullptr};
    return launch_selected(g, KL_KERNEL_ADVEC_U_2I5, f, 0.0, (hipStream_t)stream);
}

int kl_diff_smag(const kl_grid_t *g, void *ut, void *vt, void *wt, const void *u, const void *v, const void *w,
                 const void *evisc, void *stream)
{
    clear_error();
    int rc = check_grid(g);
    if (rc) return rc;
    const void *p[7] = {u, v, w, ut, vt, wt, evisc};
    if ((rc = check_ptrs(p, 7))) return rc;
    void *f[7] = {(void *)u, (void *)v, (void *)w, ut, vt, wt, (void *)evisc};
    return launch_selected(g, KL_KERNEL_DIFF_SMAG, f, 0.0, (hipStream_t)stream);
}

int kl_advec_u(const kl_grid_t *g, void *ut, const void *u, const void *v, const void *w, void *stream)
{
    clear_error();
    int rc = check_grid(g);
    if (rc) return rc;
    const void *p[4] = {u, v, w, ut};
    if ((rc = check_ptrs(p, 4))) return rc;
    void *f[6] = {(void *)u, (void *)v, (void *)w, ut, nullptr, nullptr};
    return launch_selected(g, KL_KERNEL_ADVEC_U, f, 0.0, (hipStream_t)stream);
}

int kl_diff_uvw(const kl_grid_t *g, void *ut, void *vt, void *wt, const void *u, const void *v, const void *w,
                double visc, void *stream)
{
    clear_error();
    int rc = check_grid(g);
    if (rc) return rc;
    const void *p[6] = {u, v, w, ut, vt, wt};
    if ((rc = check_ptrs(p, 6))) return rc;
    void *f[6] = {(void *)u, (void *)v, (void *)w, ut, vt, wt};
    return launch_selected(g, KL_KERNEL_DIFF_UVW, f, visc, (hipStream_t)stream);
}

int kl_advec_diff(const kl_grid_t *g, void *ut, void *vt, void *wt, const void *u, const void *v, const void *w,
                  double visc, void *stream)
{
    clear_error();
    int rc = check_grid(g);
    if (rc) return rc;
    const void *p[6] = {u, v, w, ut, vt, wt};
    if ((rc = check_ptrs(p, 6))) return rc;
    void *f[6] = {(void *)u, (void *)v, (void *)w, ut, vt, wt};
    return launch_selected(g, KL_KERNEL_ADVEC_DIFF, f, visc, (hipStream_t)stream);
}

int kl_euler(const kl_grid_t *g, double dt, void *u, void *v, void *w, const void *ut, const void *vt,
             const void *wt, void *stream)
{
    clear_error();
    int rc = check_grid(g);
    if (rc) return rc;
    const void *p[6] = {u, v, w, ut, vt, wt};
    if ((rc = check_ptrs(p, 6))) return rc;
    HostArgs a = make_args(g);
    a.ut = (void *)ut;
    a.vt = (void *)vt;
    a.wt = (void *)wt;
    hipError_t e = launch_euler(a, dt, u, v, w, (hipStream_t)stream);
    // the fused refill covers one ghost layer; wider halos are refilled whole
    if (e == hipSuccess && g->gc != 1) e = launch_fill_ghosts(a, u, v, w, (hipStream_t)stream);
    return e == hipSuccess ? KL_OK : hip_fail(e, "euler");
}

int kl_step(const kl_grid_t *g, double visc, double dt, void *u, void *v, void *w, void *ut, void *vt, void *wt,
            void *stream)
{
    clear_error();
    int rc = check_grid(g);
    if (rc) return rc;
    const void *p[6] = {u, v, w, ut, vt, wt};
    if ((rc = check_ptrs(p, 6))) return rc;
    hipStream_t s = (hipStream_t)stream;
    HostArgs a = make_args(g);
    for (void *t : {ut, vt, wt}) {
        const hipError_t e = launch_zero_interior(a, t, s);
        if (e != hipSuccess) return hip_fail(e, "zero tendencies");
    }
    void *f[6] = {u, v, w, ut, vt, wt};
    if ((rc = launch_selected(g, KL_KERNEL_ADVEC_U, f, visc, s))) return rc;
    if ((rc = launch_selected(g, KL_KERNEL_DIFF_UVW, f, visc, s))) return rc;
    a.ut = ut;
    a.vt = vt;
    a.wt = wt;
    hipError_t e = launch_euler(a, dt, u, v, w, s);
    if (e == hipSuccess && g->gc != 1) e = launch_fill_ghosts(a, u, v, w, s);
    return e == hipSuccess ? KL_OK : hip_fail(e, "euler");
}

int kl_step_fused(const kl_grid_t *g, double visc, double dt, const void *u, const void *v, const void *w,
                  void *u_out, void *v_out, void *w_out, void *stream)
{
    clear_error();
    int rc = check_grid(g);
    if (rc) return rc;
    const void *p[6] = {u, v, w, u_out, v_out, w_out};
    if ((rc = check_ptrs(p, 6))) return rc;
    for (int a = 0; a < 3; ++a)
        for (int b = 3; b < 6; ++b)
            if (p[a] == p[b]) return fail(KL_ERR_INVALID, "fused step: input %d and output %d overlap", a, b - 3);
    void *f[6] = {(void *)u, (void *)v, (void *)w, u_out, v_out, w_out};
    if ((rc = launch_selected(g, KL_KERNEL_STEP, f, visc, (hipStream_t)stream, dt))) return rc;
    if (g->gc != 1) {  // the kernel writes one ghost layer; refill wider halos whole
        const hipError_t e = launch_fill_ghosts(make_args(g), u_out, v_out, w_out, (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e, "fill_ghosts");
    }
    return KL_OK;
}

int kl_reduce_fp64(const kl_grid_t *g, int32_t what, const void *f0, const void *f1, const void *f2, double *out,
                   void *stream)
{
    clear_error();
    int rc = check_grid(g);
    if (rc) return rc;
    if (what != 0 && what != 1) return fail(KL_ERR_INVALID, "what=%d", what);
    if (!out) return fail(KL_ERR_INVALID, "out is NULL");
    if (what == 0) {
        const void *p[3] = {f0, f1, f2};
        if ((rc = check_ptrs(p, 3))) return rc;
    }
    void *ws = workspace(reduce_scratch_bytes(), (hipStream_t)stream);
    if (!ws) return fail(KL_ERR_NOMEM, "reduction workspace");
    const hipError_t e = launch_reduce(make_args(g), what, f0, f1, f2, out, ws, (hipStream_t)stream);
    return e == hipSuccess ? KL_OK : hip_fail(e, "reduce");
}

int kl_generate_fields(const kl_grid_t *g, uint64_t seed, void *u, void *v, void *w, void *stream)
{
    clear_error();
    int rc = check_grid(g);
    if (rc) return rc;
    const void *p[3] = {u, v, w};
    if ((rc = check_ptrs(p, 3))) return rc;
    const hipError_t e = launch_gen_uniform(make_args(g), seed, u, v, w, (hipStream_t)stream);
    return e == hipSuccess ? KL_OK : hip_fail(e, "generate_fields");
}

int kl_hash_interior(const kl_grid_t *g, const void *f, uint64_t *out, void *stream)
{
    clear_error();
    int rc = check_grid(g);
    if (rc) return rc;
    if (!f || !out) return fail(KL_ERR_INVALID, "NULL pointer");
    void *ws = workspace(reduce_scratch_bytes(), (hipStream_t)stream);
    if (!ws) return fail(KL_ERR_NOMEM, "hash workspace");
    const hipError_t e = launch_hash(make_args(g), f, out, ws, (hipStream_t)stream);
    return e == hipSuccess ? KL_OK : hip_fail(e, "hash");
}

int kl_num_variants(int32_t kernel, int32_t dtype)
{
    clear_error();
    if (!kernel_ok(kernel) || (dtype != KL_F32 && dtype != KL_F64))
        return fail(KL_ERR_INVALID, "kernel %d / dtype %d", kernel, dtype);
    return (int)variants(kernel, dtype).size();
}

int kl_variant_name(int32_t kernel, int32_t dtype, int32_t index, char *buf, size_t len)
{
    const int n = kl_num_variants(kernel, dtype);
    if (n < 0) return n;
    if (index < 0 || index >= n) return fail(KL_ERR_NOTFOUND, "variant index %d", index);
    if (!buf || len == 0) return fail(KL_ERR_INVALID, "NULL buffer");
    snprintf(buf, len, "%s", variants(kernel, dtype)[index].name);
    return KL_OK;
}

int kl_variant_eligible(const kl_grid_t *g, int32_t kernel, int32_t index, const void *const fields[6])
{
    clear_error();
    int rc = check_grid(g);
    if (rc) return rc;
    const int n = kl_num_variants(kernel, g->dtype);
    if (n < 0) return n;
    if (index < 0 || index >= n) return fail(KL_ERR_NOTFOUND, "variant index %d", index);
    return variant_eligible(variants(kernel, g->dtype)[index], g, fields, fields ? kernel_nptr(kernel) : 0) ? 1 : 0;
}

int kl_launch_variant_dt(const kl_grid_t *g, int32_t kernel, int32_t index, void *const fields[6], double visc,
                         double dt, void *stream)
{
    clear_error();
    int rc = check_grid(g);
    if (rc) return rc;
    if (!kernel_ok(kernel)) return fail(KL_ERR_INVALID, "kernel %d", kernel);
    if (!fields) return fail(KL_ERR_INVALID, "fields is NULL");
    if ((rc = check_ptrs((const void *const *)fields, kernel_nptr(kernel)))) return rc;
    return run_variant(g, kernel, index, fields, visc, (hipStream_t)stream, dt);
}

int kl_launch_variant(const kl_grid_t *g, int32_t kernel, int32_t index, void *const fields[6], double visc,
                      void *stream)
{
    return kl_launch_variant_dt(g, kernel, index, fields, visc, 0.0, stream);
}

int kl_selected_variant(const kl_grid_t *g, int32_t kernel)
{
    clear_error();
    int rc = check_grid(g);
    if (rc) return rc;
    if (!kernel_ok(kernel)) return fail(KL_ERR_INVALID, "kernel %d", kernel);
    return select_variant(g, kernel);
}

int kl_clear_plan_cache(void)
{
    clear_plans();
    return KL_OK;
}

}  // extern "C"
