// Wisdom files: one human-readable JSON-lines file per kernel holding the
// best configuration found by each tuning session for one GPU and problem
// size, with provenance (Section "Wisdom Files"), and the record-selection
// heuristic run on the first launch per problem size (Section "Kernel
// Selection and Compilation"):
//   1. a record for this GPU (device name, and compute-unit count where the
//      record states it) and this exact problem size;
//   2. else the record for this GPU whose problem size is closest
//      (Euclidean distance);
//   3. else the closest record for this GPU architecture;
//   4. else the closest record of any GPU;
//   5. else (no file, or no usable record) the default configuration.
// Records must also match the field dtype.  Among equally good records the
// one later in the file wins, so a re-tune supersedes an older result.
#include <errno.h>
#include <fcntl.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <sys/file.h>
#include <sys/stat.h>
#include <time.h>
#include <unistd.h>

#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "json.hpp"
#include "kl_internal.hpp"

namespace kl {

namespace {

struct Record {
    std::string device, arch, variant;
    int dtype;
    int cu_count;  // 0 when the record does not state it
    double size[3];
};

// Parse one wisdom line; false if it is not a usable record of `kernel`.
bool parse_record(const std::string &line, int kernel, Record &r)
{
    JVal v;
    if (!parse_json(line, v) || v.kind != JVal::OBJ) return false;
    const JVal *k = v.get("kernel"), *dt = v.get("dtype"), *ps = v.get("problem_size"),
               *dev = v.get("device"), *arch = v.get("arch"), *var = v.get("variant");
    if (!k || k->kind != JVal::STR || k->str != kernel_name(kernel)) return false;
    if (!dt || dt->kind != JVal::STR || (dt->str != "f32" && dt->str != "f64")) return false;
    if (!ps || ps->kind != JVal::ARR || ps->arr.size() != 3) return false;
    if (!dev || dev->kind != JVal::STR || !arch || arch->kind != JVal::STR) return false;
    if (!var || var->kind != JVal::STR) return false;
    for (int d = 0; d < 3; ++d) {
        if (ps->arr[d].kind != JVal::NUM) return false;
        r.size[d] = ps->arr[d].num;
    }
    r.dtype = dt->str == "f32" ? KL_F32 : KL_F64;
    const JVal *cu = v.get("cu_count");
    r.cu_count = cu && cu->kind == JVal::NUM ? (int)cu->num : 0;
    r.device = dev->str;
    r.arch = arch->str;
    r.variant = var->str;
    return true;
}

bool variant_known(int kernel, int dtype, const std::string &name)
{
    for (const Variant &v : variants(kernel, dtype))
        if (name == v.name) return true;
    return false;
}

std::mutex g_dir_mu;
std::string g_dir;  // empty: default

}  // namespace

const char *kernel_name(int kernel)
{
    switch (kernel) {
    case KL_KERNEL_ADVEC_U: return "advec_u";
    case KL_KERNEL_DIFF_UVW: return "diff_uvw";
    case KL_KERNEL_STEP: return "step";
    case KL_KERNEL_ADVEC_U_2I5: return "advec_u_2i5";
    case KL_KERNEL_ADVEC_DIFF: return "advec_diff";
    default: return "diff_smag";
    }
}

std::string wisdom_dir()
{
    std::lock_guard<std::mutex> lk(g_dir_mu);
    if (!g_dir.empty()) return g_dir;
    const char *env = getenv("KL_WISDOM_DIR");
    return env && *env ? std::string(env) : std::string("wisdom");
}

std::string wisdom_path(const std::string &dir, int kernel)
{
    return dir + "/" + kernel_name(kernel) + ".wisdom";
}

int current_device_ident(DeviceIdent *out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    out->name = prop.name;
    std::string arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    out->arch = colon == std::string::npos ? arch : arch.substr(0, colon);
    out->cu_count = prop.multiProcessorCount;
    return KL_OK;
}

int wisdom_select(const std::string &dir, int kernel, int dtype, const DeviceIdent &dev, int itot, int jtot,
                  int ktot, std::string *variant, int *level)
{
    *level = 5;
    *variant = "default";
    std::ifstream in(wisdom_path(dir, kernel));
    if (!in) return KL_OK;  // a missing file selects the default configuration
    const double want[3] = {(double)itot, (double)jtot, (double)ktot};
    double best[5] = {INFINITY, INFINITY, INFINITY, INFINITY, INFINITY};
    std::string choice[5];
    std::string line;
    while (std::getline(in, line)) {
        Record r;
        if (!parse_record(line, kernel, r)) continue;
        if (r.dtype != dtype || !variant_known(kernel, dtype, r.variant)) continue;
        double d2 = 0;
        for (int d = 0; d < 3; ++d) d2 += (r.size[d] - want[d]) * (r.size[d] - want[d]);
        // one board: the same device name and, where both sides state it, the same
        // compute-unit count (boards of one architecture can share a name)
        const bool same_gpu = r.device == dev.name &&
                              (dev.cu_count <= 0 || r.cu_count <= 0 || r.cu_count == dev.cu_count);
        const bool same_arch = r.arch == dev.arch;
        // level 1: same GPU, exact size; 2: same GPU; 3: same arch; 4: any
        const int lvl = (same_gpu && d2 == 0) ? 1 : same_gpu ? 2 : same_arch ? 3 : 4;
        for (int l = lvl; l <= 4; ++l) {
            if (l == 1 && lvl != 1) continue;
            if (d2 <= best[l]) {  // "<=": a later record wins ties
                best[l] = d2;
                choice[l] = r.variant;
            }
        }
    }
    for (int l = 1; l <= 4; ++l) {
        if (!choice[l].empty()) {
            *level = l;
            *variant = choice[l];
            return KL_OK;
        }
    }
    return KL_OK;
}

static int mkdirs(const std::string &dir)
{
    std::string cur;
    std::stringstream ss(dir);
    std::string part;
    if (!dir.empty() && dir[0] == '/') cur = "/";
    while (std::getline(ss, part, '/')) {
        if (part.empty()) continue;
        cur += part + "/";
        if (mkdir(cur.c_str(), 0755) != 0 && errno != EEXIST) return -1;
    }
    return 0;
}

int wisdom_append(const std::string &dir, int kernel, const std::string &json_line)
{
    return wisdom_append_file(dir, std::string(kernel_name(kernel)) + ".wisdom", json_line);
}

int wisdom_append_file(const std::string &dir, const std::string &file, const std::string &json_line)
{
    if (mkdirs(dir) != 0) return fail(KL_ERR_IO, "cannot create wisdom dir %s: %s", dir.c_str(), strerror(errno));
    const std::string path = dir + "/" + file;
    const int fd = open(path.c_str(), O_WRONLY | O_APPEND | O_CREAT, 0644);
    if (fd < 0) return fail(KL_ERR_IO, "cannot open %s: %s", path.c_str(), strerror(errno));
    flock(fd, LOCK_EX);
    const std::string line = json_line + "\n";
    const ssize_t n = write(fd, line.data(), line.size());
    fsync(fd);
    flock(fd, LOCK_UN);
    close(fd);
    if (n != (ssize_t)line.size()) return fail(KL_ERR_IO, "short write to %s", path.c_str());
    return KL_OK;
}

std::string provenance_json(const DeviceIdent &dev)
{
    char host[256] = {0};
    gethostname(host, sizeof host - 1);
    char date[64];
    const time_t now = time(nullptr);
    struct tm tmv;
    gmtime_r(&now, &tmv);
    strftime(date, sizeof date, "%Y-%m-%dT%H:%M:%SZ", &tmv);
    int rt = 0, drv = 0;
    (void)hipRuntimeGetVersion(&rt);
    (void)hipDriverGetVersion(&drv);
    std::ostringstream o;
    o << "\"device\":\"" << json_escape(dev.name) << "\",\"arch\":\"" << json_escape(dev.arch)
      << "\",\"cu_count\":" << dev.cu_count << ",\"date\":\"" << date << "\",\"hostname\":\"" << json_escape(host)
      << "\",\"hip_runtime\":" << rt << ",\"hip_driver\":" << drv << ",\"lib_version\":\""
      << json_escape(kl_version()) << "\"";
    return o.str();
}

}  // namespace kl

using namespace kl;

extern "C" {

int kl_set_wisdom_dir(const char *dir)
{
    {
        std::lock_guard<std::mutex> lk(g_dir_mu);
        g_dir = dir ? dir : "";
    }
    clear_plans();
    return KL_OK;
}

int kl_wisdom_lookup(const char *wisdom_dir_, int32_t kernel, int32_t dtype, const char *device_name,
                     const char *arch, int32_t cu_count, int32_t itot, int32_t jtot, int32_t ktot, char *variant,
                     size_t len, int32_t *level)
{
    clear_error();
    if (kernel < 0 || kernel >= KL_NUM_KERNELS) return fail(KL_ERR_INVALID, "kernel %d", kernel);
    if (dtype != KL_F32 && dtype != KL_F64) return fail(KL_ERR_INVALID, "dtype %d", dtype);
    if (!device_name || !arch || !variant || !level || len == 0) return fail(KL_ERR_INVALID, "NULL argument");
    DeviceIdent id{device_name, arch, cu_count};
    std::string name;
    int lvl = 5;
    const std::string dir = wisdom_dir_ && *wisdom_dir_ ? std::string(wisdom_dir_) : kl::wisdom_dir();
    const int rc = wisdom_select(dir, kernel, dtype, id, itot, jtot, ktot, &name, &lvl);
    if (rc) return rc;
    snprintf(variant, len, "%s", name.c_str());
    *level = lvl;
    return KL_OK;
}

}  // extern "C"
