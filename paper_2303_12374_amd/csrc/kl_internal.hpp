// Internal host-side declarations of libkl (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "kl.h"

namespace kl {

// dtype-agnostic launch arguments; launchers convert metrics to the field type.
struct HostArgs {
    int itot, jtot, ktot, kw0, dtype, bc;
    int gc;  // ghost cells per side in x and y
    int64_t off, js, ks;
    double dxi, dyi, visc;
    double dt;  // fused step only
    const void *dzi, *dzhi;
    void *ut, *vt, *wt;  // tendencies; for the fused step: the output fields
    const void *u, *v, *w;
    const void *evisc;  // diff_smag only
};

// Number of leading entries of a fields[] array a kernel reads:
// u, v, w, ut (advection); u, v, w, ut, vt, wt (diffusion, step); and evisc
// as the seventh for diff_smag.
inline int kernel_nptr(int kernel)
{
    return (kernel == KL_KERNEL_ADVEC_U || kernel == KL_KERNEL_ADVEC_U_2I5) ? 4
           : (kernel == KL_KERNEL_DIFF_SMAG ? 7 : 6);
}
constexpr int KL_NUM_KERNELS = 6;

typedef hipError_t (*LaunchFn)(const HostArgs &, hipStream_t);
// Persistent batched launch: descriptor table (StencilArgs<T>[]), tile table
// (int4 {grid, tx, ty, tz}[]), tile count, number of blocks, and a work queue
// (two device ints, zero at launch and zero again at the end) or null for
// the static round-robin assignment.
typedef hipError_t (*BatchFn)(const void *, const void *, int, int, int *, hipStream_t);
typedef int (*OccFn)();  // resident blocks per CU of the batched kernel

// Blocks of a persistent tile walk: every resident slot (ncu * occ), at most
// one per tile.
inline int persistent_blocks(int64_t ntiles, int ncu, int occ)
{
    const int64_t nb = ntiles < (int64_t)ncu * occ ? ntiles : (int64_t)ncu * occ;
    return (int)(nb > 0 ? nb : 1);
}

enum { FAMILY_PLAIN = 0, FAMILY_ZC = 1, FAMILY_ZL = 2 };

// One ahead-of-time compiled configuration of a tendency kernel.
struct Variant {
    const char *name;
    int kernel, dtype, family;
    int vx, bx, by, kb, xcd;  // x vector width, block shape, z-march length, XCD order
    LaunchFn launch;
    BatchFn batch;  // persistent tile-list form (LDS z-march family only), else null
    OccFn occupancy;
};

// Registry (index 0 of every list is the default configuration).
const std::vector<Variant> &variants(int kernel, int dtype);
const std::vector<Variant> &variants_f32(int kernel);
const std::vector<Variant> &variants_f64(int kernel);

// Errors: record a message for kl_last_error() and return `code`.
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int hip_fail(hipError_t e, const char *what);
void clear_error();

// Validation shared by the entry points.
int check_grid(const kl_grid_t *g);
HostArgs make_args(const kl_grid_t *g);
bool variant_eligible(const Variant &v, const kl_grid_t *g, const void *const *ptrs, int nptr);

// Library-owned per-device workspace (for reduction partials).
void *workspace(size_t bytes, hipStream_t s);

// Auxiliary kernels (aux.hip).
hipError_t launch_fill_ghosts(const HostArgs &a, void *u, void *v, void *w, hipStream_t s);
hipError_t launch_fill_scalar(const HostArgs &a, void *f, hipStream_t s);
// The y and z ghost cells of u, v, w from their interior (the ghost fill
// without the x ghost columns of interior rows): after a step that stored
// the new values and their x images only.
hipError_t launch_fill_yz_images(const HostArgs &a, void *u, void *v, void *w, hipStream_t s);
hipError_t launch_euler(const HostArgs &a, double dt, void *u, void *v, void *w, hipStream_t s);
hipError_t launch_zero_interior(const HostArgs &a, void *f, hipStream_t s);
hipError_t launch_reduce(const HostArgs &a, int what, const void *f0, const void *f1,
                         const void *f2, double *out, void *scratch, hipStream_t s);
hipError_t launch_hash(const HostArgs &a, const void *f, uint64_t *out, void *scratch,
                       hipStream_t s);
hipError_t launch_gen_uniform(const HostArgs &a, uint64_t seed, void *u, void *v, void *w,
                              hipStream_t s);
size_t reduce_scratch_bytes();
bool reduce_vectorized(const HostArgs &a, const void *f0, const void *f1, const void *f2);
// Batched ghost fill of u, v, w (one job per grid: append_fill_job adds the
// job and its 256-cell blocks {job, block}) and batched conservation sums
// (one job per grid, written to out[3 slot ..]; jobs of one launch share a
// dtype and reduce_vectorized; their pass-1 blocks {job, block} are those
// that own rows; partials: sums_partial_bytes(slots) bytes, zeroed once).
size_t fill_job_bytes();
int64_t fill_cell_count(const HostArgs &a);  // ghost cells of the velocity fill (must be < 2^32)
void append_fill_job(const HostArgs &a, void *u, void *v, void *w, std::vector<char> &jobs,
                     std::vector<int2> &blocks);
hipError_t launch_fill_batch(int dtype, const void *jobs, const void *blocks, int nblocks, hipStream_t s);
size_t sum_job_bytes();
size_t sums_partial_bytes(int nslots);
void append_sum_job(const HostArgs &a, const void *ut, const void *vt, const void *wt, int slot, std::vector<char> &jobs,
                    std::vector<int2> &blocks);
hipError_t launch_sums_batch(int dtype, bool vec, const void *jobs, const void *blocks, int nblocks, double *partials,
                             hipStream_t s);
hipError_t launch_sums_finish(const double *partials, int nslots, double *out, hipStream_t s);
// Batched row-tile kernels: descs = StencilArgs<T>[], tiles = int4 {grid, row0, row1, 0}[].
hipError_t launch_zero_batch(int dtype, const void *descs, const void *tiles, int ntiles, int nblocks,
                             hipStream_t s);
// Configuration of grid g for `kernel` in batched (persistent) form, or -1.
int batch_variant(const kl_grid_t *g, int kernel, void *const f[6]);
// Regroup grids (6 field pointers each) for fewer persistent kernels: see batch.hip.
void merge_batch_groups(int kernel, const std::vector<kl_grid_t> &grids, void *const *fields, std::vector<int> &sel);

// Wisdom (wisdom.cpp).
struct DeviceIdent {
    std::string name, arch;
    int cu_count;
};
int current_device_ident(DeviceIdent *out);
std::string wisdom_dir();
std::string wisdom_path(const std::string &dir, int kernel);
const char *kernel_name(int kernel);
int wisdom_select(const std::string &dir, int kernel, int dtype, const DeviceIdent &dev,
                  int itot, int jtot, int ktot, std::string *variant, int *level);
int wisdom_append(const std::string &dir, int kernel, const std::string &json_line);
int wisdom_append_file(const std::string &dir, const std::string &file, const std::string &json_line);
std::string provenance_json(const DeviceIdent &dev);

// Plan cache (api.cpp).
int select_variant(const kl_grid_t *g, int kernel);
int run_variant(const kl_grid_t *g, int kernel, int index, void *const *fields, double visc,
                hipStream_t s, double dt = 0.0);
void clear_plans();

// Capture (capture.cpp): write the launch to a capture file if its kernel is
// named in KL_CAPTURE / kl_set_capture and its problem size is new.
int maybe_capture(const kl_grid_t *g, int kernel, void *const *fields, double visc, double dt, hipStream_t s);

}  // namespace kl
