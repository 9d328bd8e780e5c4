/*
 * kl.h -- C ABI of libkl, staggered-grid stencil kernels for AMD Instinct
 * MI355X (gfx950).
 *
 * Problem statement (the paper's evaluation, Section "Application" and
 * Section "Tunable Parameters"): two kernels of a finite-difference CFD code
 * act on 3-D fields stored on a grid of configurable size, in float or
 * double.  "advec_u" advances the x-velocity u by advection; "diff_uvw"
 * advances u, v and w by diffusion.  The caller hands over the fields, the
 * grid dimensions, the grid spacings, the viscosity and the precision; the
 * library derives every launch parameter itself (Section "Code Example":
 * block and grid dimensions are computed by the library, not passed by the
 * user), uses a default configuration when a kernel was never tuned, and
 * otherwise selects a tuned configuration from wisdom records (Section
 * "Kernel Selection and Compilation").
 *
 * Discretisation fixed by this library (the paper names the kernels but
 * prints no formulas): Arakawa-C staggering with one ghost cell per side;
 * u at (xh_i, y_j, z_k), v at (x_i, yh_j, z_k), w at (x_i, y_j, zh_k);
 * I(a,b) = (a+b)/2;
 *   advec_u:  ut += -[ (I(u_i,u_{i+1})^2 - I(u_{i-1},u_i)^2) dxi
 *                    + (I(v_{i-1,j+1},v_{i,j+1}) I(u_j,u_{j+1})
 *                       - I(v_{i-1,j},v_{i,j}) I(u_{j-1},u_j)) dyi
 *                    + (I(w_{i-1,k+1},w_{i,k+1}) I(u_k,u_{k+1})
 *                       - I(w_{i-1,k},w_{i,k}) I(u_{k-1},u_k)) dzi[k] ]
 *   diff_uvw: phi_t += visc [ (phi_{i+1} - 2 phi + phi_{i-1}) dxi^2
 *                           + (phi_{j+1} - 2 phi + phi_{j-1}) dyi^2 + Z(phi) ]
 *     with Z = ((phi_{k+1}-phi) dzhi[k+1] - (phi-phi_{k-1}) dzhi[k]) dzi[k]
 *     for u and v, and Z = ((w_{k+1}-w) dzi[k] - (w-w_{k-1}) dzi[k-1]) dzhi[k]
 *     for w.  u and v are advanced on k in [1, ktot]; w on k in [2, ktot]
 *     with z walls and on [1, ktot] when z is periodic.
 *
 * The schemes the paper names for its two kernels (Section "Tunable
 * Parameters": advection of u "second order with fifth order
 * interpolation", diffusion as part of "second order Smagorinsky
 * diffusion") are also provided:
 *   advec_u_2i5: the flux form above with the advected u interpolated to
 *     each face by the fifth-order upwind-biased formula of Wicker and
 *     Skamarock (2002): face(U; a_-2..a_3) = U c6 - |U| d5 with
 *     c6 = (37(a0+a1) - 8(a_-1+a2) + (a_-2+a3))/60,
 *     d5 = (10(a1-a0) - 5(a2-a_-1) + (a3-a_-2))/60 (face between a0, a1;
 *     U the midpoint-interpolated advecting velocity).  In z the order drops
 *     to third, U c4 - |U| d3 with c4 = (7(a0+a1) - (a_-1+a2))/12,
 *     d3 = (3(a1-a0) - (a2-a_-1))/12, on faces 2 and ktot, and to the
 *     midpoint U (a0+a1)/2 on faces 1 and ktot+1.  Needs gc = 3.
 *   diff_smag: (ut, vt, wt) += div(nu (grad u + grad u^T)) with nu = evisc
 *     given at cell centers: normal stresses 2 nu d_i u_i at cell centers,
 *     shear stresses on cell edges with nu the mean of the four surrounding
 *     centers, z widths dz_k for u, v and dzh_k for w.  w is advanced on the
 *     same range as in diff_uvw.
 *
 * Conventions shared by every entry point:
 *  - Return value: KL_OK (0) or a negative kl_status_t.  The message of the
 *    last failure on the calling thread is kl_last_error().  No C++
 *    exception crosses this boundary.
 *  - Memory: every field, metric and output pointer is DEVICE memory owned
 *    by the caller, unless stated otherwise; the library never frees it.
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *    stream).  Kernel entry points are asynchronous; their return code only
 *    covers argument checks and launch errors, and a fault during execution
 *    surfaces at the caller's next synchronisation.
 *  - Tendency kernels ACCUMULATE (+=) into the interior cells of their
 *    outputs and never write ghost or padding cells; they read ghost cells
 *    of u, v, w, which the caller fills first (kl_fill_ghosts).  x is
 *    periodic in every mode, and a configuration may take an x neighbour
 *    across the periodic boundary from the interior cell rather than from
 *    its ghost copy: after the ghost fill both hold the same value.
 */
#ifndef KL_H_
#define KL_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { KL_F32 = 0, KL_F64 = 1 };

/* Boundary conditions.  x and y are always periodic.
 *  ZWALL_ZEROGRAD: u, v zero gradient at the z walls; w on the wall faces
 *                  copies the neighbouring inner face (w_1 = w_2,
 *                  w_{ktot+1} = w_ktot); the unused ghost w_0 = w_2.
 *  ZWALL_NOPEN:    u, v as above; w = 0 on the wall faces, w_0 = -w_2.
 *  ZPERIODIC:      periodic in z for all fields (uniform dz expected). */
enum { KL_BC_ZWALL_ZEROGRAD = 0, KL_BC_ZWALL_NOPEN = 1, KL_BC_ZPERIODIC = 2 };

typedef enum {
    KL_OK = 0,
    KL_ERR_INVALID = -1,  /* bad argument: sizes, strides, null pointers, enum values */
    KL_ERR_DEVICE = -2,   /* HIP runtime error (launch, copy, synchronisation) */
    KL_ERR_NOMEM = -3,    /* a library-side allocation failed */
    KL_ERR_BUDGET = -4,   /* a request does not fit the server's memory budget */
    KL_ERR_AGAIN = -5,    /* not finished yet (kl_poll) */
    KL_ERR_NOTFOUND = -6, /* unknown ticket / variant / record */
    KL_ERR_IO = -7        /* wisdom file could not be written */
} kl_status_t;

/* Kernels with tunable configurations.  KL_KERNEL_STEP is the fused time
 * step of kl_step_fused; KL_KERNEL_ADVEC_DIFF is advec_u followed by
 * diff_uvw in one pass (kl_advec_diff, and the batched form). */
enum {
    KL_KERNEL_ADVEC_U = 0,
    KL_KERNEL_DIFF_UVW = 1,
    KL_KERNEL_STEP = 2,
    KL_KERNEL_ADVEC_U_2I5 = 3,
    KL_KERNEL_DIFF_SMAG = 4,
    KL_KERNEL_ADVEC_DIFF = 5
};

/* kl_tune kernel_mask bits. */
enum {
    KL_TUNE_ADVEC_U = 1u,
    KL_TUNE_DIFF_UVW = 2u,
    KL_TUNE_STEP = 4u,
    KL_TUNE_PAIR = 8u, /* time each diffusion kernel right after its advection kernel */
    KL_TUNE_ADVEC_U_2I5 = 16u,
    KL_TUNE_DIFF_SMAG = 32u,
    KL_TUNE_ADVEC_DIFF = 64u
};

/* One grid.  Element (i, j, k) of every field is at index
 * off + i + j*jstride + k*kstride (elements of the field dtype), with
 * i in [1-gc, itot+gc] (interior [1, itot]), likewise j, and k in
 * [0, ktot+1] (one ghost level in z).  The same layout holds for u, v, w,
 * the tendencies ut, vt, wt and the eddy viscosity.
 * dzi[k] = 1/(zh_{k+1} - zh_k) and dzhi[k] = 1/(z_k - z_{k-1}) are device
 * arrays of ktot+2 entries in the field dtype; dxi = 1/dx and dyi = 1/dy are
 * rounded to the field dtype inside the kernels. */
typedef struct kl_grid {
    int32_t itot, jtot, ktot; /* interior points per axis, >= 1 (ktot >= 2 with z walls) */
    int32_t gc;               /* ghost cells per side in x and y: 1, or 3 (advec_u_2i5) */
    int64_t off, jstride, kstride;
    double dxi, dyi;
    const void *dzi, *dzhi;
    int32_t dtype;            /* KL_F32 or KL_F64 */
    int32_t bc;               /* KL_BC_* */
} kl_grid_t;

/* Library version string (static storage). */
const char *kl_version(void);

/* Message of the last failed call on this thread ("" if none). */
const char *kl_last_error(void);

/* The library's preferred padded layout for a grid: x-contiguous rows padded
 * to whole 128-byte lines with the first interior element of every row on a
 * 128-byte boundary, so that 16-byte vector accesses are aligned and the two
 * x-ghost cells of neighbouring rows share one line.  *alloc_elems is the
 * element count to allocate per field (it includes tail padding).  Host
 * pointers; no device work. */
int kl_layout(int32_t itot, int32_t jtot, int32_t ktot, int32_t dtype,
              int64_t *off, int64_t *jstride, int64_t *kstride, int64_t *alloc_elems);

/* kl_layout for gc ghost cells per side in x and y (gc = 1 or 3): rows of
 * itot + 2 gc cells padded to whole 128-byte lines, interior rows starting
 * on a line boundary, off = (gc-1) jstride + (line - 1) (line = 128 bytes in
 * elements) so that the first ghost cell (1-gc, 1-gc, 0) has a non-negative
 * index.  gc = 1 is kl_layout. */
int kl_layout_gc(int32_t itot, int32_t jtot, int32_t ktot, int32_t dtype, int32_t gc,
                 int64_t *off, int64_t *jstride, int64_t *kstride, int64_t *alloc_elems);

/* Fill the ghost cells of u, v and w from the interior by the boundary rules
 * of g->bc (and, in wall modes, the wall faces w_1 and w_{ktot+1}).  Reads
 * interior cells only, so all ghosts are filled in one pass. */
int kl_fill_ghosts(const kl_grid_t *g, void *u, void *v, void *w, void *stream);

/* Fill the ghost cells of one cell-center scalar (the eddy viscosity):
 * periodic in x and y, in z periodic (KL_BC_ZPERIODIC) or zero gradient
 * across the walls, as u and v. */
int kl_fill_scalar(const kl_grid_t *g, void *f, void *stream);

/* ut += advec_u(u, v, w) on the interior (formula above).  u, v, w must be
 * ghost-filled.  Runs the configuration selected for (dtype, itot, jtot,
 * ktot, device) from the wisdom files, else the default configuration. */
int kl_advec_u(const kl_grid_t *g, void *ut, const void *u, const void *v, const void *w,
               void *stream);

/* (ut, vt, wt) += visc * Laplacian(u, v, w) on each field's computed range
 * (formula above).  u, v, w must be ghost-filled.  Selection as kl_advec_u. */
int kl_diff_uvw(const kl_grid_t *g, void *ut, void *vt, void *wt,
                const void *u, const void *v, const void *w, double visc, void *stream);

/* kl_advec_u followed by kl_diff_uvw, as one pass over the grid: ut +=
 * advec_u, then ut += diff_u, vt += diff_v, wt += diff_w on each field's
 * computed range.  The additions are made in that order and rounded as in
 * the two separate calls, so the tendencies are bitwise those of
 * kl_advec_u; kl_diff_uvw, while the pass reads u, v, w, ut, vt, wt once
 * and writes ut, vt, wt once (9 values per point instead of 14).  The two
 * kernels are the paper's pair (Section "Experimental Evaluation"); fusing
 * them is this library's.  u, v, w must be ghost-filled; ut, vt, wt must not
 * overlap u, v, w.  Selection as kl_advec_u (wisdom file advec_diff.wisdom). */
int kl_advec_diff(const kl_grid_t *g, void *ut, void *vt, void *wt, const void *u, const void *v,
                  const void *w, double visc, void *stream);

/* ut += advec_u_2i5(u, v, w) on the interior (scheme above).  Requires
 * g->gc >= 3; u, v, w ghost-filled.  Selection as kl_advec_u (wisdom file
 * advec_u_2i5.wisdom). */
int kl_advec_u_2i5(const kl_grid_t *g, void *ut, const void *u, const void *v, const void *w,
                   void *stream);

/* (ut, vt, wt) += div(evisc (grad u + grad u^T)) on each field's computed
 * range (scheme above).  u, v, w and evisc must be ghost-filled
 * (kl_fill_ghosts, kl_fill_scalar).  Selection as kl_advec_u (wisdom file
 * diff_smag.wisdom). */
int kl_diff_smag(const kl_grid_t *g, void *ut, void *vt, void *wt, const void *u, const void *v,
                 const void *w, const void *evisc, void *stream);

/* Forward-Euler update f += dt * ft on each field's computed range, fused
 * with the ghost refill of the updated fields (every ghost cell is written
 * by the thread that updates its source cell). */
int kl_euler(const kl_grid_t *g, double dt, void *u, void *v, void *w,
             const void *ut, const void *vt, const void *wt, void *stream);

/* One time step: tendencies := 0, ut += advec_u, (ut,vt,wt) += diff_uvw,
 * Euler update with ghost refill.  u, v, w must be ghost-filled on entry and
 * are ghost-filled on return; ut, vt, wt are overwritten (interior only). */
int kl_step(const kl_grid_t *g, double visc, double dt, void *u, void *v, void *w,
            void *ut, void *vt, void *wt, void *stream);

/* One time step fused into a single pass over the grid: reads u, v, w
 * (ghost-filled, not modified) and writes the next state into u_out, v_out,
 * w_out, ghost cells included (some configurations store the y and z ghost
 * cells with a second, small kernel that copies them from the new values).
 * The arithmetic and its order are those of kl_step (tendencies
 * zeroed, advec_u, diff_uvw, forward Euler, ghost refill), so the result is
 * bitwise identical to kl_step's, while the kernel moves 6 values per point
 * instead of 26.  Inputs and outputs must not overlap; the outputs' padding
 * cells are not written.  Configuration from the wisdom file step.wisdom. */
int kl_step_fused(const kl_grid_t *g, double visc, double dt, const void *u, const void *v, const void *w,
                  void *u_out, void *v_out, void *w_out, void *stream);

/* FP64 reductions over the interior, accumulated in double for either field
 * dtype, in a fixed-shape two-pass tree (bitwise reproducible).
 *  what = 0 (conservation): f0, f1, f2 = ut, vt, wt; out[0] = sum ut*dz_k,
 *         out[1] = sum vt*dz_k, out[2] = sum wt*dzh_k over w's computed
 *         faces, with dz_k = 1/dzi[k] and dzh_k = 1/dzhi[k] in double.
 *  what = 1 (checksums): for each of f0, f1, f2 (NULL skips a field):
 *         out[3n] = sum f, out[3n+1] = sum f^2, out[3n+2] = max |f|.
 * `out` is a device array of 3 (what=0) or 9 (what=1) doubles, written
 * asynchronously on `stream`.  Uses a library-owned device workspace. */
int kl_reduce_fp64(const kl_grid_t *g, int32_t what, const void *f0, const void *f1,
                   const void *f2, double *out, void *stream);

/* kl_reduce_fp64 for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, hosts that forbid hipMalloc.  Same
 * arguments, kernels and result bits as kl_reduce_fp64; it calls no
 * hipMalloc or hipFree.  The pass-1 partials (4096 x 9 doubles, 288 KiB) go
 * to one fixed array in device memory per GPU, which the library holds until
 * the process ends.  That need does not depend on the grid, so no grid size
 * valid for kl_reduce_fp64 is refused for it; devices with ordinal >= 64 get
 * KL_ERR_INVALID.  Every call on one GPU shares that array: calls that
 * overlap on one GPU (two streams, two threads) race and may return wrong
 * sums; serialise them.  Nothing in the array needs to start at zero. */
int kl_reduce_fp64_noalloc(const kl_grid_t *g, int32_t what, const void *f0, const void *f1,
                           const void *f2, double *out, void *stream);

/* Fill the interiors of u, v, w with the library's seeded initial state:
 * U[-1,1) noise plus the mean flow (1, 0.5, 0).  The noise value of
 * interior point (i, j, k) of field f (0 u, 1 v, 2 w) comes from the
 * counter-based SplitMix64 generator (Steele, Lea and Flood, OOPSLA 2014):
 * counter = ((seed*8 + f) << 40) + (i-1) + itot*((j-1) + jtot*(k-1)), one
 * generator step from state `counter` gives z, r = (z >> 11) * 2^-53 and
 * the value is (2r - 1) + mean_f in double, rounded to the field dtype.
 * Ghost cells are not touched (call kl_fill_ghosts next). */
int kl_generate_fields(const kl_grid_t *g, uint64_t seed, void *u, void *v, void *w, void *stream);

/* Order-independent 64-bit hash of the bit patterns of one field's interior
 * (sum over cells of a SplitMix64 mix of the value's bits and its (i,j,k));
 * equal hashes of two fields mean bitwise-equal interiors with overwhelming
 * probability.  `out` is one device uint64. */
int kl_hash_interior(const kl_grid_t *g, const void *f, uint64_t *out, void *stream);

/* Streaming probe (a measurement aid, not a stencil): one kernel reads
 * `bytes` from each of src[0..nread-1] and writes `bytes` to each of
 * dst[0..nwrite-1] (each destination gets the XOR of the sources), 16 bytes
 * per lane per access, with non-temporal loads and stores when nontemporal
 * is non-zero.  It gives the HBM rate of a tendency kernel's access mix
 * without its stencil.  Built mixes (nread, nwrite): (1,1) copy, (2,1),
 * (3,3), (4,1), (6,3), (7,3).  Every array is device memory of at least
 * `bytes` bytes, 16-byte aligned; bytes is a positive multiple of 16384.
 * KL_ERR_INVALID otherwise.  Asynchronous on `stream`. */
int kl_stream_probe(int32_t nread, int32_t nwrite, const void *const *src, void *const *dst, int64_t bytes,
                    int32_t nontemporal, void *stream);

/* ---- configurations (the AOT variant registry) --------------------------- */

/* Number of compiled configurations of `kernel` (KL_KERNEL_*) for `dtype`;
 * index 0 is always the default configuration (one thread per point, blocks
 * of 256 threads along x, no tiling; the paper's default configuration,
 * Section "Tunable Parameters"). */
int kl_num_variants(int32_t kernel, int32_t dtype);

/* Name of configuration `index` into buf (NUL-terminated, truncated to len). */
int kl_variant_name(int32_t kernel, int32_t dtype, int32_t index, char *buf, size_t len);

/* 1 if configuration `index` can run on this grid and these pointers
 * (vector width divides itot and the layout/pointer alignment), else 0.
 * `fields` as in kl_launch_variant (may be NULL: layout checks only). */
int kl_variant_eligible(const kl_grid_t *g, int32_t kernel, int32_t index,
                        const void *const fields[6]);

/* Launch configuration `index` of `kernel` directly.  fields = {u, v, w, ut,
 * vt, wt} and, for KL_KERNEL_DIFF_SMAG, a seventh entry evisc; the
 * advection kernels use u, v, w, ut; the fused step reads u, v, w and writes
 * fields 3..5 (visc and the time step dt of kl_launch_variant_dt).  Same
 * semantics as the corresponding kl_advec_u / kl_diff_uvw / kl_step_fused /
 * kl_advec_u_2i5 / kl_diff_smag entry point.  KL_ERR_INVALID if the
 * configuration is not eligible. */
int kl_launch_variant(const kl_grid_t *g, int32_t kernel, int32_t index,
                      void *const fields[6], double visc, void *stream);
int kl_launch_variant_dt(const kl_grid_t *g, int32_t kernel, int32_t index,
                         void *const fields[6], double visc, double dt, void *stream);

/* Index of the configuration kl_advec_u / kl_diff_uvw would run for this
 * grid on the current device (consults the wisdom files on first use per
 * problem size and caches the choice). */
int kl_selected_variant(const kl_grid_t *g, int32_t kernel);

/* ---- tuning and wisdom (Sections "Kernel Tuning", "Wisdom Files",
 *      "Kernel Selection and Compilation") --------------------------------- */

/* Directory of the wisdom files (one JSON-lines file per kernel:
 * <dir>/advec_u.wisdom and <dir>/diff_uvw.wisdom).  NULL or "" restores the
 * default: $KL_WISDOM_DIR, else "./wisdom".  Clears the selection cache. */
int kl_set_wisdom_dir(const char *dir);

/* Forget all cached selections (the next launch per problem size re-reads
 * the wisdom files). */
int kl_clear_plan_cache(void);

/* Host-only (no GPU work): run the selection heuristic over the wisdom file
 * of `kernel` in `wisdom_dir` (NULL = current wisdom directory) for a given
 * device name, architecture (e.g. "gfx950"), compute-unit count, dtype and
 * problem size.  A record is "this GPU" when its device name matches and,
 * where both the record and cu_count state one (cu_count > 0), its
 * compute-unit count matches too: boards of one architecture can report the
 * same name.  *level receives 1 (this GPU, this size), 2 (this GPU, closest size by
 * Euclidean distance), 3 (this architecture, closest size), 4 (any record,
 * closest size) or 5 (no usable record: the default configuration);
 * `variant` receives the configuration name ("default" at level 5).  Lines
 * that do not parse, other dtypes and unknown configuration names are
 * skipped; among equally close records the later one in the file wins. */
int kl_wisdom_lookup(const char *wisdom_dir, int32_t kernel, int32_t dtype, const char *device_name,
                     const char *arch, int32_t cu_count, int32_t itot, int32_t jtot, int32_t ktot,
                     char *variant, size_t len, int32_t *level);

/* Tune the kernels in kernel_mask (KL_TUNE_* bits: advec_u, diff_uvw, the
 * fused step, advec_u_2i5, diff_smag, the fused advec_diff; KL_TUNE_PAIR: time each diffusion
 * kernel right after the selected advection kernel of its scheme, as in a
 * time step, so that the cache state it starts from is realistic) for this
 * grid on the current device: every eligible configuration is checked for
 * bitwise-equal output against the default configuration, then timed (hip
 * events, median of repetitions after warm-up) until budget_s seconds are
 * spent (the default configuration is always measured).  The fastest one is
 * appended as a record (kernel, dtype, problem size, device, architecture,
 * configuration, time, provenance) to the kernel's wisdom file in
 * wisdom_dir (NULL = current wisdom directory), and the selection cache is
 * cleared.  fields = {u, v, w, ut, vt, wt} (plus evisc as a seventh entry
 * when diff_smag is tuned): u, v, w (and evisc) must be ghost-filled;
 * ut, vt, wt are clobbered.  Synchronous (returns after the file is written).
 * If timings_out is not NULL it receives up to max_timings entries of
 * (configuration index, median ms) for kernel_mask's lowest kernel, or -1 ms
 * for a configuration that failed the bitwise check; *n_timings = count. */
int kl_tune(const kl_grid_t *g, void *const fields[6], uint32_t kernel_mask,
            const char *wisdom_dir, double budget_s, void *stream,
            double *timings_out, int32_t max_timings, int32_t *n_timings);

/* ---- capture and replay (Section "Kernel Capturing") --------------------- */

/* Capture launches: the first launch per problem size of each kernel named
 * in the comma-separated list `kernels` ("advec_u", "diff_uvw", "step",
 * "advec_u_2i5", "diff_smag"; NULL or "" switches capturing off) is written,
 * before it runs, to <dir>/<kernel>_<dtype>_<itot>x<jtot>x<ktot>.klcap
 * (dir NULL = "captures").  Without this call the environment variables
 * KL_CAPTURE (the list) and KL_CAPTURE_DIR are read on the first launch.
 * Capturing copies the launch's fields to the host and blocks the calling
 * thread until the copy is done; it is meant for tuning runs. */
int kl_set_capture(const char *kernels, const char *dir);

/* Write one capture of `kernel` with these fields (as in kl_launch_variant),
 * viscosity and time step to `path`.  File format: line 1 "KLCAP 1"; line 2
 * a JSON header (kernel, kernel_id, dtype, problem_size, gc, off, jstride,
 * kstride, dxi, dyi, bc, visc, dt, arrays = [{name, elems}], device
 * provenance); then the arrays dzi, dzhi and the kernel's fields as raw
 * elements of the field dtype.  Field arrays cover the cells from the first
 * ghost cell (rounded down to a 128-byte line) to the last; "off" is
 * relative to that base.  Synchronises `stream`. */
int kl_capture(const kl_grid_t *g, int32_t kernel, void *const fields[6], double visc, double dt,
               const char *path, void *stream);

/* Host-only: copy the JSON header of a capture file into header
 * (NUL-terminated, truncated to len).  KL_ERR_IO if unreadable,
 * KL_ERR_INVALID if it is not a capture. */
int kl_capture_info(const char *path, char *header, size_t len);

/* Replay a capture for tuning: upload its metrics and fields to library-
 * allocated device buffers, run kl_tune for its kernel on them (each
 * configuration checked bitwise against the default, timed, the fastest
 * appended to the wisdom file in wisdom_dir), free the buffers.  timings_out
 * / max_timings / n_timings as in kl_tune.  Synchronous. */
int kl_tune_capture(const char *path, const char *wisdom_dir, double budget_s, void *stream,
                    double *timings_out, int32_t max_timings, int32_t *n_timings);

/* ---- batched form: many independent grids in one captured graph ---------- */

/* Build a batch of n grids (fields[6*g + f] = {u, v, w, ut, vt, wt} of grid
 * g, device pointers owned by the caller) and capture, on `stream`, one HIP
 * graph that runs, for all grids: tendencies := 0 (when zero_tendencies),
 * then ut += advec_u followed by (ut,vt,wt) += diff_uvw fused in one pass
 * as in kl_advec_diff (bitwise the two separate kernels), as persistent
 * tile-walking kernels (one per configuration group: advec_diff
 * configurations taken from the wisdom files, then regrouped so that the
 * configuration selected for the most grid points serves every grid it
 * can, and so on; all give the same bits) whose blocks draw tiles from a
 * work queue, largest tiles first.  Every tile is computed once, by one
 * block, with the same arithmetic, so the results do not depend on which
 * block takes it.  The queue returns to zero at the end of every replay;
 * replays of one batch must not overlap (launch them on one stream).  The
 * grid descriptors are copied; the library owns the tile tables, the queues
 * and the graph. */
int kl_batch_create(const kl_grid_t *grids, void *const *fields, int32_t n, double visc,
                    int32_t zero_tendencies, void *stream, void **batch);

/* Steps of a batch's graph besides the tendencies (kl_batch_create_ex). */
enum {
    KL_BATCH_ZERO_TENDENCIES = 1u, /* ut, vt, wt := 0 before the tendencies */
    KL_BATCH_FILL_GHOSTS = 2u,     /* first: the ghost cells of u, v, w as kl_fill_ghosts (all grids, one kernel per dtype) */
    KL_BATCH_SUMS = 4u             /* last: each grid's conservation sums as kl_reduce_fp64(what = 0) */
};

/* kl_batch_create with the graph's other steps chosen by `flags`
 * (KL_BATCH_*): [ghost fill] -> [tendencies := 0] -> the fused tendency
 * groups -> [conservation sums].  The ghost fill gives every grid's u, v, w
 * the same ghost values, bit for bit, as kl_fill_ghosts.  With
 * KL_BATCH_SUMS, `sums` is a device array of 3 doubles per grid (grid g at
 * sums[3g .. 3g+2]: sum ut*dz_k, sum vt*dz_k, sum wt*dzh_k), written by every
 * replay with the bits kl_reduce_fp64(what = 0) gives for that grid; the
 * library owns the partials (4096 x 9 doubles per grid).  Unknown flag bits,
 * or KL_BATCH_SUMS without `sums`, are KL_ERR_INVALID.  kl_batch_create is
 * this call with flags = zero_tendencies ? KL_BATCH_ZERO_TENDENCIES : 0. */
int kl_batch_create_ex(const kl_grid_t *grids, void *const *fields, int32_t n, double visc, uint32_t flags,
                       double *sums, void *stream, void **batch);

/* Tune a batch as a whole (the batch-level form of kl_tune): time the
 * batch with its per-grid selection and then with each persistent
 * advec_diff configuration serving every grid it can (the mean of
 * 10 graph replays after 2 warm-ups, on `stream`), after checking that each
 * gives the same output bits as the per-grid selection (sum of the bit
 * hashes of every grid's ut, vt, wt after one replay on zeroed tendencies).
 * A configuration fastest for one grid launched alone, where latency
 * decides, need not be fastest inside a full batch, where bytes per tile
 * decide.  The fastest is appended to <wisdom_dir>/advec_diff_batch.wisdom
 * (NULL = current wisdom directory) under the batch's signature, a hash of
 * the sorted (itot, jtot, ktot, bc, gc) of its grids of one dtype, with the
 * variant name ("per_grid" when the per-grid selection won), the time, the
 * per-grid selection's time and provenance; kl_batch_create uses a record
 * with the batch's signature (this GPU, else this architecture, else any)
 * before the per-grid selection.  The batch is rebuilt with the winner.
 * Tunes each dtype of the batch in turn until budget_s seconds are spent
 * (the per-grid selection is always timed).  The tendencies of every grid
 * are clobbered.  timings_out (if not NULL) receives up to max_timings
 * pairs (configuration index, -1 for the per-grid selection; ms, or -1 for
 * a configuration whose bits differed), *n_timings their count.
 * Synchronous. */
int kl_batch_tune(void *batch, const char *wisdom_dir, double budget_s, void *stream, double *timings_out,
                  int32_t max_timings, int32_t *n_timings);

/* Configuration group `group` (0 .. n_kernels of kl_batch_info minus the
 * zeroing, ghost-fill and sum kernels) of a batch: its dtype, configuration name (into name,
 * truncated to len) and tile count (host pointers; any may be NULL).
 * KL_ERR_NOTFOUND past the last group. */
int kl_batch_group(void *batch, int32_t group, int32_t *dtype, char *name, size_t len, int64_t *n_tiles);

/* Replay the batch's graph on `stream` (asynchronous). */
int kl_batch_run(void *batch, void *stream);

/* Number of kernels in the batch's graph (zeroing, ghost fill and sums included) and tiles of its
 * fused tendency groups (host ints). */
int kl_batch_info(void *batch, int32_t *n_kernels, int64_t *n_tiles);

int kl_batch_destroy(void *batch);

/* ---- served form: continuous batching of stencil-step requests ----------- */

typedef struct kl_request {
    int32_t itot, jtot, ktot;
    int32_t dtype, bc;
    int32_t nsteps;      /* time steps to advance, >= 1 */
    double dt, visc;
    uint64_t seed;       /* initial u, v, w = U[-1,1) noise + mean flow (1, 0.5, 0) */
} kl_request_t;

typedef struct kl_result {
    int32_t state;       /* 0 queued, 1 running, 2 done, 3 failed */
    int32_t err;         /* kl_status_t of a failed request */
    int64_t t_arrive_ns, t_admit_ns, t_done_ns; /* CLOCK_MONOTONIC */
    double checksum[9];  /* kl_reduce_fp64(what=1) of the final u, v, w */
    void *fields[3];     /* device u, v, w (library arena), valid until kl_release */
    int64_t off, jstride, kstride; /* layout of fields */
} kl_result_t;

/* Create a server that owns a background thread and one stream of its own.
 * arena/arena_bytes: caller-owned device memory the server sub-allocates
 * all request fields from; budget_bytes (<= arena_bytes) caps the bytes held
 * by admitted requests.  Requests are admitted in arrival order while they
 * fit; every tick advances all admitted requests by one fused step (one
 * persistent launch per configuration group, two field buffers per request
 * used in turn), so requests join and leave between ticks.  The host
 * prepares the next tick while the current one runs. */
int kl_server_create(void *arena, size_t arena_bytes, size_t budget_bytes, void **srv);

/* Enqueue a request; *ticket identifies it.  KL_ERR_BUDGET if the request's
 * footprint alone exceeds the budget, KL_ERR_INVALID for bad sizes. */
int kl_submit(void *srv, const kl_request_t *req, uint64_t *ticket);

/* Status of a request into *out (host struct).  KL_OK once done (or failed:
 * see out->state), KL_ERR_AGAIN while queued or running, KL_ERR_NOTFOUND
 * for an unknown or released ticket. */
int kl_poll(void *srv, uint64_t ticket, kl_result_t *out);

/* Free a finished request's fields back to the arena. */
int kl_release(void *srv, uint64_t ticket);

/* Server counters: out[0] ticks, out[1] launches, out[2] requests done,
 * out[3] peak bytes in use, out[4] points*steps advanced. */
int kl_server_stats(void *srv, int64_t out[5]);

/* Stop the thread after the queue drains and free the server. */
int kl_server_destroy(void *srv);

#ifdef __cplusplus
}
#endif

#endif /* KL_H_ */
