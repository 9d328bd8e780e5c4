// Capture and replay of kernel launches (Section "Kernel Capturing": a
// captured launch stores everything needed to run the kernel again,
// including its input data, so that it can be tuned offline on the
// application's own data; capturing is switched on by naming kernels in an
// environment variable).
//
// File format (".klcap"):
//   line 1:  "KLCAP 1"
//   line 2:  one JSON object (the header): kernel, dtype, problem_size, gc,
//            off / jstride / kstride of the captured layout, dxi, dyi, bc,
//            visc, dt, device provenance and "arrays": [{"name", "elems"}]
//   payload: the arrays in header order, raw little-endian elements of the
//            field dtype, back to back.
// The field arrays hold the cells [base, base + elems) of the caller's
// buffers, where base is the first cell of the ghost box rounded down to a
// 128-byte line; the header's "off" is relative to base, so the layout's
// alignment is kept.
#include <errno.h>
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>
#include <time.h>
#include <unistd.h>

#include <fstream>
#include <mutex>
#include <set>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "json.hpp"
#include "kl_internal.hpp"

namespace kl {
namespace {

const char *field_names[7] = {"u", "v", "w", "ut", "vt", "wt", "evisc"};

struct CaptureState {
    std::mutex mu;
    bool init = false;
    std::set<std::string> kernels;
    std::string dir = "captures";
    std::set<std::tuple<int, int, int, int, int>> done;
};

CaptureState &cap_state()
{
    static CaptureState c;
    return c;
}

void set_kernels(CaptureState &c, const char *list)
{
    c.kernels.clear();
    if (!list) return;
    std::stringstream ss(list);
    std::string name;
    while (std::getline(ss, name, ','))
        if (!name.empty()) c.kernels.insert(name);
}

void init_from_env(CaptureState &c)
{
    if (c.init) return;
    c.init = true;
    set_kernels(c, getenv("KL_CAPTURE"));
    const char *d = getenv("KL_CAPTURE_DIR");
    if (d && *d) c.dir = d;
}

int make_dirs(const std::string &dir)
{
    std::string cur;
    std::stringstream ss(dir);
    std::string part;
    if (!dir.empty() && dir[0] == '/') cur = "/";
    while (std::getline(ss, part, '/')) {
        if (part.empty()) continue;
        cur += part + "/";
        if (mkdir(cur.c_str(), 0755) != 0 && errno != EEXIST)
            return fail(KL_ERR_IO, "cannot create directory %s", cur.c_str());
    }
    return KL_OK;
}

// First captured cell (rounded down to a 128-byte line) and the cell count.
void field_span(const kl_grid_t *g, int64_t *base, int64_t *elems)
{
    const int64_t line = 128 / (g->dtype == KL_F32 ? 4 : 8);
    const int64_t gc = g->gc;
    const int64_t first = g->off + (1 - gc) + (1 - gc) * g->jstride;
    const int64_t last = g->off + (g->itot + gc) + (g->jtot + gc) * g->jstride + (int64_t)(g->ktot + 1) * g->kstride;
    *base = first / line * line;
    *elems = last - *base + 1;
}

int write_capture(const kl_grid_t *g, int kernel, void *const *fields, double visc, double dt, hipStream_t s,
                  const std::string &path)
{
    const int nf = kernel_nptr(kernel);
    for (int n = 0; n < nf; ++n)
        if (!fields[n]) return fail(KL_ERR_INVALID, "capture: field %d is NULL", n);
    const size_t es = g->dtype == KL_F32 ? 4 : 8;
    int64_t base, elems;
    field_span(g, &base, &elems);
    DeviceIdent id;
    int rc = current_device_ident(&id);
    if (rc) return rc;
    std::ostringstream h;
    h.precision(17);
    h << "{\"kernel\":\"" << kernel_name(kernel) << "\",\"kernel_id\":" << kernel << ",\"dtype\":\""
      << (g->dtype == KL_F32 ? "f32" : "f64") << "\",\"problem_size\":[" << g->itot << "," << g->jtot << ","
      << g->ktot << "],\"gc\":" << g->gc << ",\"off\":" << (g->off - base) << ",\"jstride\":" << g->jstride
      << ",\"kstride\":" << g->kstride << ",\"dxi\":" << g->dxi << ",\"dyi\":" << g->dyi << ",\"bc\":" << g->bc
      << ",\"visc\":" << visc << ",\"dt\":" << dt << ",\"arrays\":[{\"name\":\"dzi\",\"elems\":" << g->ktot + 2
      << "},{\"name\":\"dzhi\",\"elems\":" << g->ktot + 2 << "}";
    for (int n = 0; n < nf; ++n) h << ",{\"name\":\"" << field_names[n] << "\",\"elems\":" << elems << "}";
    h << "]," << provenance_json(id) << "}";
    FILE *fp = fopen(path.c_str(), "wb");
    if (!fp) return fail(KL_ERR_IO, "capture: cannot open %s for writing", path.c_str());
    const std::string head = "KLCAP 1\n" + h.str() + "\n";
    bool ok = fwrite(head.data(), 1, head.size(), fp) == head.size();
    std::vector<char> buf;
    const void *metric[2] = {g->dzi, g->dzhi};
    for (int m = 0; m < 2 && ok; ++m) {
        buf.resize((size_t)(g->ktot + 2) * es);
        hipError_t e = hipMemcpyAsync(buf.data(), metric[m], buf.size(), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            fclose(fp);
            return hip_fail(e, "capture copy");
        }
        ok = fwrite(buf.data(), 1, buf.size(), fp) == buf.size();
    }
    buf.resize((size_t)elems * es);
    for (int n = 0; n < nf && ok; ++n) {
        const char *src = (const char *)fields[n] + (size_t)base * es;
        hipError_t e = hipMemcpyAsync(buf.data(), src, buf.size(), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            fclose(fp);
            return hip_fail(e, "capture copy");
        }
        ok = fwrite(buf.data(), 1, buf.size(), fp) == buf.size();
    }
    if (fclose(fp) != 0) ok = false;
    return ok ? KL_OK : fail(KL_ERR_IO, "capture: write to %s failed", path.c_str());
}

// Read and check the two header lines; *payload = offset of the arrays.
int read_header(const std::string &path, JVal &hdr, std::string &text, long *payload)
{
    FILE *fp = fopen(path.c_str(), "rb");
    if (!fp) return fail(KL_ERR_IO, "capture: cannot open %s", path.c_str());
    std::string magic, line;
    int c;
    while ((c = fgetc(fp)) != EOF && c != '\n') magic += (char)c;
    while ((c = fgetc(fp)) != EOF && c != '\n') line += (char)c;
    *payload = ftell(fp);
    fclose(fp);
    if (magic != "KLCAP 1") return fail(KL_ERR_INVALID, "capture: %s is not a KLCAP 1 file", path.c_str());
    if (!parse_json(line, hdr) || hdr.kind != JVal::OBJ) return fail(KL_ERR_INVALID, "capture: bad header");
    text = line;
    return KL_OK;
}

double num(const JVal &o, const char *key, bool *ok)
{
    const JVal *v = o.get(key);
    if (!v || v->kind != JVal::NUM) {
        *ok = false;
        return 0;
    }
    return v->num;
}

// An integer-valued header number within [lo, hi]; *ok = false otherwise.
int64_t inum(const JVal &o, const char *key, int64_t lo, int64_t hi, bool *ok)
{
    bool here = true;
    const double x = num(o, key, &here);
    if (!here || !(x >= (double)lo && x <= (double)hi) || x != (double)(int64_t)x) {
        *ok = false;
        return 0;
    }
    return (int64_t)x;
}

// Read a capture's header and check it against the payload before anything
// is allocated or launched: the kernel name and id agree, the dtype is
// "f32" or "f64", the grid passes the library's own grid checks, the arrays
// are dzi, dzhi (ktot+2 elements each) and the kernel's fields in order,
// every field covers the whole ghost box of its layout (the cells a kernel
// may touch) and the file holds all of their bytes.  On success *g has
// every member but the metric pointers, and elems[a] the element count of
// array a.
int parse_capture(const char *path, kl_grid_t *g, int *kernel_out, long *payload, std::vector<int64_t> &elems)
{
    JVal hdr;
    std::string text;
    int rc = read_header(path, hdr, text, payload);
    if (rc) return rc;
    bool ok = true;
    const int kernel = (int)inum(hdr, "kernel_id", 0, KL_NUM_KERNELS - 1, &ok);
    const JVal *kn = hdr.get("kernel"), *dt = hdr.get("dtype"), *ps = hdr.get("problem_size"),
               *arrs = hdr.get("arrays");
    if (!ok || !kn || kn->kind != JVal::STR || !dt || dt->kind != JVal::STR || !ps || ps->kind != JVal::ARR ||
        ps->arr.size() != 3 || !arrs || arrs->kind != JVal::ARR)
        return fail(KL_ERR_INVALID, "capture %s: incomplete header", path);
    if (kn->str != kernel_name(kernel))
        return fail(KL_ERR_INVALID, "capture %s: kernel \"%s\" does not match kernel_id %d", path, kn->str.c_str(),
                    kernel);
    if (dt->str != "f32" && dt->str != "f64")
        return fail(KL_ERR_INVALID, "capture %s: dtype \"%s\" is neither f32 nor f64", path, dt->str.c_str());
    memset(g, 0, sizeof *g);
    g->dtype = dt->str == "f64" ? KL_F64 : KL_F32;
    const int64_t big = (int64_t)1 << 40;
    for (int d = 0; d < 3; ++d) {
        const JVal &x = ps->arr[d];
        if (x.kind != JVal::NUM || !(x.num >= 1 && x.num <= (double)INT32_MAX) || x.num != (double)(int64_t)x.num)
            return fail(KL_ERR_INVALID, "capture %s: problem_size[%d]", path, d);
    }
    g->itot = (int32_t)ps->arr[0].num;
    g->jtot = (int32_t)ps->arr[1].num;
    g->ktot = (int32_t)ps->arr[2].num;
    g->gc = (int32_t)inum(hdr, "gc", 0, 16, &ok);
    g->off = inum(hdr, "off", 0, big, &ok);
    g->jstride = inum(hdr, "jstride", 1, big, &ok);
    g->kstride = inum(hdr, "kstride", 1, big, &ok);
    g->dxi = num(hdr, "dxi", &ok);
    g->dyi = num(hdr, "dyi", &ok);
    g->bc = (int32_t)inum(hdr, "bc", 0, 16, &ok);
    if (!ok) return fail(KL_ERR_INVALID, "capture %s: incomplete or out-of-range header", path);
    // the library's grid checks (the metric pointers are not known yet)
    g->dzi = g->dzhi = (const void *)g;
    rc = check_grid(g);
    g->dzi = g->dzhi = nullptr;
    if (rc) return rc;
    const int nf = kernel_nptr(kernel);
    if ((int)arrs->arr.size() != 2 + nf)
        return fail(KL_ERR_INVALID, "capture %s: %zu arrays, kernel %s needs %d", path, arrs->arr.size(),
                    kernel_name(kernel), 2 + nf);
    // the last cell of the ghost box, relative to the captured base
    const int64_t gc = g->gc;
    const int64_t last = g->off + (g->itot + gc) + (g->jtot + gc) * g->jstride + (int64_t)(g->ktot + 1) * g->kstride;
    const size_t es = g->dtype == KL_F32 ? 4 : 8;
    elems.assign(2 + nf, 0);
    int64_t total = 0;
    for (int a = 0; a < 2 + nf; ++a) {
        const JVal &ar = arrs->arr[a];
        const JVal *nm = ar.kind == JVal::OBJ ? ar.get("name") : nullptr;
        const char *want = a == 0 ? "dzi" : (a == 1 ? "dzhi" : field_names[a - 2]);
        if (!nm || nm->kind != JVal::STR || nm->str != want)
            return fail(KL_ERR_INVALID, "capture %s: array %d must be \"%s\"", path, a, want);
        bool aok = true;
        elems[a] = inum(ar, "elems", 1, big, &aok);
        if (!aok) return fail(KL_ERR_INVALID, "capture %s: array %s: bad element count", path, want);
        if (a < 2 && elems[a] != (int64_t)g->ktot + 2)
            return fail(KL_ERR_INVALID, "capture %s: %s holds %lld values, ktot+2 = %d needed", path, want,
                        (long long)elems[a], g->ktot + 2);
        if (a >= 2 && elems[a] <= last)
            return fail(KL_ERR_INVALID, "capture %s: field %s holds %lld cells, its layout spans %lld", path, want,
                        (long long)elems[a], (long long)(last + 1));
        if (a > 2 && elems[a] != elems[2])
            return fail(KL_ERR_INVALID, "capture %s: field %s size differs from u", path, want);
        total += elems[a];
    }
    struct stat st;
    if (stat(path, &st) != 0) return fail(KL_ERR_IO, "capture %s: cannot stat", path);
    if ((int64_t)st.st_size < (int64_t)*payload + total * (int64_t)es)
        return fail(KL_ERR_IO, "capture %s: truncated payload (%lld bytes, header describes %lld)", path,
                    (long long)st.st_size, (long long)(*payload + total * (int64_t)es));
    *kernel_out = kernel;
    return KL_OK;
}

}  // namespace

// Called before every selected launch: captures the first launch per
// problem size of each kernel named in KL_CAPTURE (or kl_set_capture).
int maybe_capture(const kl_grid_t *g, int kernel, void *const *fields, double visc, double dt, hipStream_t s)
{
    CaptureState &c = cap_state();
    std::lock_guard<std::mutex> lk(c.mu);
    init_from_env(c);
    if (c.kernels.empty() || !c.kernels.count(kernel_name(kernel))) return KL_OK;
    const auto key = std::make_tuple(kernel, (int)g->dtype, (int)g->itot, (int)g->jtot, (int)g->ktot);
    if (c.done.count(key)) return KL_OK;
    c.done.insert(key);
    int rc = make_dirs(c.dir);
    if (rc) return rc;
    char name[256];
    snprintf(name, sizeof name, "/%s_%s_%dx%dx%d.klcap", kernel_name(kernel), g->dtype == KL_F32 ? "f32" : "f64",
             g->itot, g->jtot, g->ktot);
    return write_capture(g, kernel, fields, visc, dt, s, c.dir + name);
}

}  // namespace kl

using namespace kl;

extern "C" {

int kl_set_capture(const char *kernels, const char *dir)
{
    clear_error();
    CaptureState &c = cap_state();
    std::lock_guard<std::mutex> lk(c.mu);
    c.init = true;
    set_kernels(c, kernels);
    c.dir = dir && *dir ? std::string(dir) : std::string("captures");
    c.done.clear();
    return KL_OK;
}

int kl_capture(const kl_grid_t *g, int32_t kernel, void *const fields[6], double visc, double dt, const char *path,
               void *stream)
{
    clear_error();
    int rc = check_grid(g);
    if (rc) return rc;
    if (kernel < 0 || kernel >= KL_NUM_KERNELS) return fail(KL_ERR_INVALID, "kernel %d", kernel);
    if (!fields || !path || !*path) return fail(KL_ERR_INVALID, "NULL fields or path");
    return write_capture(g, kernel, fields, visc, dt, (hipStream_t)stream, path);
}

int kl_capture_info(const char *path, char *header, size_t len)
{
    clear_error();
    if (!path || !header || len == 0) return fail(KL_ERR_INVALID, "NULL argument");
    JVal hdr;
    std::string text;
    long payload;
    int rc = read_header(path, hdr, text, &payload);
    if (rc) return rc;
    snprintf(header, len, "%s", text.c_str());
    return KL_OK;
}

int kl_tune_capture(const char *path, const char *wisdom_dir, double budget_s, void *stream, double *timings_out,
                    int32_t max_timings, int32_t *n_timings)
{
    clear_error();
    if (!path) return fail(KL_ERR_INVALID, "NULL path");
    kl_grid_t g;
    int kernel;
    long payload;
    std::vector<int64_t> elems;
    int rc = parse_capture(path, &g, &kernel, &payload, elems);
    if (rc) return rc;
    const int nf = kernel_nptr(kernel);
    const size_t es = g.dtype == KL_F32 ? 4 : 8;
    const int64_t line = 128 / (int64_t)es;
    // device copies: metrics, then fields (with slack for aligned vector access)
    std::vector<void *> dev(2 + nf, nullptr);
    struct Free {
        std::vector<void *> &d;
        ~Free()
        {
            for (void *p : d)
                if (p) (void)hipFree(p);
        }
    } freer{dev};
    FILE *fp = fopen(path, "rb");
    if (!fp || fseek(fp, payload, SEEK_SET) != 0) {
        if (fp) fclose(fp);
        return fail(KL_ERR_IO, "capture %s: cannot read the payload", path);
    }
    std::vector<char> buf;
    for (int a = 0; a < 2 + nf; ++a) {
        buf.resize((size_t)elems[a] * es);
        if (fread(buf.data(), 1, buf.size(), fp) != buf.size()) {
            fclose(fp);
            return fail(KL_ERR_IO, "capture %s: truncated payload", path);
        }
        hipError_t e = hipMalloc(&dev[a], buf.size() + 2 * line * es);
        if (e == hipSuccess) e = hipMemcpy(dev[a], buf.data(), buf.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            fclose(fp);
            return hip_fail(e, "capture upload");
        }
    }
    fclose(fp);
    g.dzi = dev[0];
    g.dzhi = dev[1];
    void *fields[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    for (int n = 0; n < nf; ++n) fields[n] = dev[2 + n];
    // kl_tune takes six field pointers; the advection kernels' unused
    // tendency slots get full-size buffers of the same layout
    for (int n = nf; n < 6; ++n) {
        void *p = nullptr;
        const hipError_t e = hipMalloc(&p, (size_t)elems[2] * es + 2 * line * es);
        if (e != hipSuccess) return hip_fail(e, "hipMalloc");
        dev.push_back(p);
        fields[n] = p;
    }
    static const uint32_t bits[KL_NUM_KERNELS] = {KL_TUNE_ADVEC_U, KL_TUNE_DIFF_UVW, KL_TUNE_STEP,
                                                  KL_TUNE_ADVEC_U_2I5, KL_TUNE_DIFF_SMAG, KL_TUNE_ADVEC_DIFF};
    rc = kl_tune(&g, fields, bits[kernel], wisdom_dir, budget_s, stream, timings_out, max_timings, n_timings);
    const hipError_t e = hipDeviceSynchronize();
    if (rc) return rc;
    return e == hipSuccess ? KL_OK : hip_fail(e, "tune_capture sync");
}

}  // extern "C"
