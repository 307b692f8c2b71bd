/*
 * pv3d.h -- C ABI of libpv3d: GPU shadow-map shading losses of PV generators
 * on AMD Instinct MI355X (gfx950).
 *
 * Method: Robledo, Leloux & Lorenzo, arXiv:1410.5780, Sec. 2. The library
 * follows the paper's four steps:
 *   Step 1  import the 3D scene            -> pv3d_scene_load
 *   Step 2  define the PV system           -> pv3d_generator_define
 *   Step 3  evaluate the shadows           -> pv3d_evaluate (depth picture from
 *           the sun, limited to the generator; depth check of sub-cell samples)
 *   Step 4  translate shading into losses  -> pv3d_evaluate (beam removed from
 *           shaded areas, bypass-diode string model, integration over time)
 * plus a batched form (all suns of many jobs in one persistent launch) and a
 * serving form (jobs submitted while others run).
 *
 * Conventions shared by every call:
 *  - Coordinates are ENU metres (x east, y north, z up), binary64.
 *  - Every call returns pv3d_status: 0 on success, a negative code on error.
 *    Nothing throws or aborts across the ABI; pv3d_last_error() describes the
 *    last failure of the calling thread.
 *  - Input arrays are host memory and are copied before the call returns; the
 *    caller keeps ownership.
 *  - Output arrays are caller-allocated; pv3d_outputs.on_device tells whether
 *    they are host memory or device memory of the context's GPU.
 *  - Handles (scenes, generators, tickets) belong to the context and are freed
 *    by pv3d_destroy.
 *  - Limits: 16 <= map_n <= 16384; 1 <= k <= 255; n_cu, n_cv in [1, 4096] with
 *    k*n_cu and k*n_cv at most 4095;
 *    n_vert, n_tri < 2^31; at least one module; all modules share n_cu, n_cv.
 *
 * Threading: a context may be used from one thread at a time, except that
 * pv3d_poll / pv3d_wait / pv3d_cancel may be called from any thread while the
 * serving loop runs.
 */
#ifndef PV3D_H
#define PV3D_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pv3d_status;
#define PV3D_OK 0
#define PV3D_EINVAL (-1)     /* bad argument (NaN/Inf, sizes, unknown flags, non-unit sun) */
#define PV3D_ENOMEM (-2)     /* does not fit the context's HBM budget (or device memory) */
#define PV3D_ENOENT (-3)     /* unknown scene / generator / ticket handle */
#define PV3D_EDEVICE (-4)    /* HIP runtime error */
#define PV3D_ERANGE (-5)     /* a documented limit was exceeded */
#define PV3D_EBUSY (-6)      /* serving queue full, retry later */
#define PV3D_ECANCELED (-7)  /* job was cancelled */

typedef struct pv3d_ctx pv3d_ctx;

/* Create a context on HIP device `device`. hbm_budget_bytes caps the device
 * memory the context may hold (scenes, generators, work buffers); 0 means 90%
 * of the device's free memory. The context owns one HIP stream. */
pv3d_status pv3d_create(int32_t device, uint64_t hbm_budget_bytes, pv3d_ctx** out);

/* Free every scene, generator, job and buffer of the context (waits for the
 * device first). NULL is ignored. */
void pv3d_destroy(pv3d_ctx* ctx);

/* Text of the calling thread's last error; valid until its next call. */
const char* pv3d_last_error(const pv3d_ctx* ctx);

/* Step 1 (Sec. 2, "Import the 3D scene"): a triangle soup.
 * xyz: [n_vert][3] vertex positions; tri: [n_tri][3] vertex indices.
 * Both faces of a triangle cast shadows. Copied to device memory.
 * EINVAL: non-finite coordinate, index out of range, n_vert/n_tri < 0.
 * ENOMEM: does not fit the budget. */
pv3d_status pv3d_scene_load(pv3d_ctx* ctx, const double* xyz, int64_t n_vert,
                            const int32_t* tri, int64_t n_tri, uint64_t* scene_out);
pv3d_status pv3d_scene_release(pv3d_ctx* ctx, uint64_t scene);

/* Step 2 (Sec. 2, "Define the PV system"; Fig. 2): rectangular modules split
 * into cells, cells grouped into bypass-diode substrings, modules in series
 * strings.
 * Module m covers origin + a*edge_u + b*edge_v, a, b in [0, 1]; its front
 * face is the side edge_u x edge_v points to. It holds n_cu cells along
 * edge_u and n_cv along edge_v; cell (cu, cv) has index cv*n_cu + cu.
 * cell_substring: [n_cu*n_cv] substring (0 .. n_sub_per_module-1) of each
 *   cell, the same for every module; every substring must own a cell.
 * module_string: [n_mod] series string of each module (0 .. n_string-1, every
 *   string non-empty); within a string, modules count in array order.
 * add_as_occluders: 1 = each module is also drawn as two triangles
 *   (origin, +u, +u+v) and (origin, +u+v, +v) so modules shade each other.
 * EINVAL: degenerate module, mixed n_cu/n_cv, bad maps. */
typedef struct {
    double origin[3];
    double edge_u[3];
    double edge_v[3];
    int32_t n_cu, n_cv;
} pv3d_module;

pv3d_status pv3d_generator_define(pv3d_ctx* ctx, const pv3d_module* mods, int64_t n_mod,
                                  const int32_t* cell_substring, int32_t n_sub_per_module,
                                  const int32_t* module_string, int32_t add_as_occluders,
                                  uint64_t* gen_out);
pv3d_status pv3d_generator_release(pv3d_ctx* ctx, uint64_t gen);

/* Trackers (Sec. 3.4 evaluates a plant of two-axis trackers; the paper gives
 * no tracking law, so ideal tracking is taken: no angle limits, no
 * backtracking). A tracker turns the modules assigned to it about its pivot
 * as the sun moves. Its rest frame is u0 = axis x z, v0 = axis, n0 = z (axis:
 * horizontal unit vector, axis[2] == 0); the modules are given at rest in
 * world coordinates and keep their coordinates in the tracker's frame,
 * which for a sun s becomes
 *   kind 1 (one horizontal axis): v' = axis, n' = unit(s - (s.axis) axis), u' = v' x n'
 *   kind 2 (two axes):            n' = s, u' = unit(z x s) (u0 at the zenith), v' = n' x u'.
 * Modules with module_tracker[m] = -1 stay put. The rest of the definition is
 * pv3d_generator_define's.
 * Evaluation: pv3d_evaluate poses every module for every sun on the device
 * (n_sun x n_mod x 128 bytes, counted against the HBM budget); the batched
 * form poses each tracked job's modules in its job memory before its launch;
 * the serving loop rejects tracked generators (EINVAL).
 * EINVAL: kind not 1 or 2, axis not horizontal unit length within 1e-9,
 * pivot not finite, module_tracker out of [-1, n_tracker). */
typedef struct {
    int32_t kind;       /* 1 or 2 */
    int32_t reserved;   /* 0 */
    double pivot[3];
    double axis[3];
} pv3d_tracker;

pv3d_status pv3d_generator_define_tracked(pv3d_ctx* ctx, const pv3d_module* mods, int64_t n_mod,
                                          const int32_t* cell_substring, int32_t n_sub_per_module,
                                          const int32_t* module_string, int32_t add_as_occluders,
                                          const pv3d_tracker* trackers, int32_t n_tracker,
                                          const int32_t* module_tracker, uint64_t* gen_out);

/* Electrical model (Sec. 2 Step 4 turns the geometric shading into power with
 * a diode model of the cells and a system model, neither given in the paper).
 * By default a generator uses ideal bypass-diode strings: a substring carries
 * at most the irradiance of its weakest cell, at unit voltage, or is bypassed;
 * each string works at its best current. pv3d_generator_set_diode switches a
 * generator to the single-diode cell model instead: every cell follows
 *   I = Iph - I0 (exp((V + I Rs) / a) - 1) - (V + I Rs) / Rsh,
 *   Iph = isc_ref * G / g_ref  (G: the cell's irradiance, beam on the module
 *   times its unshaded fraction, plus the diffuse),
 * at a fixed temperature (a = n k T / q is given); each substring's bypass
 * diode holds the substring's voltage at no less than -v_bypass; substrings
 * are in series; each string works at its maximum power point, found by a
 * search over 65 evenly spaced currents in [0, largest cell photocurrent]
 * refined by 40 golden-section steps around every sampled maximum. power and
 * power_ref are then in W. The setting applies to evaluations started after
 * the call (per-sun, batched and serving). d = NULL returns to ideal strings.
 * EINVAL: non-finite parameters, isc_ref, g_ref, i0, a or rsh not > 0, rs or
 * v_bypass negative; ENOENT: unknown generator; EBUSY: a running serving job
 * reads the generator. */
typedef struct {
    double isc_ref;    /* cell photocurrent at g_ref, A */
    double g_ref;      /* irradiance of isc_ref, W/m^2 */
    double i0;         /* diode saturation current, A */
    double a;          /* modified ideality factor n k T / q, V */
    double rs;         /* series resistance, ohm */
    double rsh;        /* shunt resistance, ohm */
    double v_bypass;   /* bypass diode forward voltage, V */
} pv3d_diode;

pv3d_status pv3d_generator_set_diode(pv3d_ctx* ctx, uint64_t gen, const pv3d_diode* d);

/* Helper (host): sun unit vectors for day-of-year and local solar hour at a
 * latitude, with Cooper's declination and 15 degrees of hour angle per hour
 * (the paper only states that the solar position is defined, Sec. 2 Step 3).
 * sun_xyz_out: [n][3]; s_z <= 0 means the sun is not above the horizon. */
pv3d_status pv3d_sun_cooper(double lat_deg, const int32_t* day, const double* solar_hour,
                            int64_t n, double* sun_xyz_out);

/* Steps 3 and 4 (Sec. 2). flags: */
#define PV3D_EXPORT_DEPTH 1u   /* write every sun's depth picture to outputs.depth_maps */
#define PV3D_EXPORT_BITS 2u    /* write every sample's shaded flag to outputs.shaded_bits */
#define PV3D_SEPARATE_TEST 4u  /* depth-check samples in a second kernel that reads the
                                  materialised picture (default: inside the raster tile);
                                  results are identical, this route exists for cross-checks */
#define PV3D_FULL_RASTER 8u    /* raster every texel of the picture even when it is not
                                  exported (default: only texels that hold a sample); results
                                  are identical, this route exists for cross-checks */

typedef struct {
    int32_t map_n;     /* depth picture is map_n x map_n texels */
    int32_t k;         /* k x k sample points per cell (Sec. 2 Step 3 uses 3 x 3) */
    uint32_t flags;    /* PV3D_EXPORT_* */
    int32_t tile;      /* raster tile edge in texels: 0 = library's choice (64 up to map_n
                          8192, else 128; 64 in the batched form), else 32/64/128
                          (batched form: 32/64) */
    int32_t bin_limit; /* a triangle overlapping more tiles than this is not binned; every
                          tile checks it instead. 0 = library's choice (256), else 1..256 */
    int32_t reserved;  /* must be 0 */
} pv3d_params;

/* Outputs (all optional except power, power_ref, energy):
 * cell_counts: [n_sun][n_cells] shaded samples per cell (cells in module,
 *   then cell-index order); a cell's shaded fraction is count / k^2.
 * power, power_ref: [n_sun] generator power with and without shading
 *   (ideal strings: W per unit substring voltage, current proportional to
 *   irradiance; single-diode model: W).
 * energy: [2] sum over suns of power * dt_h and power_ref * dt_h, in sun
 *   order; the shading loss is 1 - energy[0] / energy[1].
 * depth_maps: [n_sun][map_n][map_n] 24-bit depths in uint32 (row j = image
 *   axis e2, column i = image axis e1); suns below the horizon read 2^24-1.
 * shaded_bits: [n_sun][n_cells][ceil(k*k/32)] uint32 words; bit t of word w
 *   is sample 32*w + t of the cell, sample index b*k + a (a along edge_u).
 * on_device: 1 = every pointer is device memory of this context's GPU; then
 *   the call is asynchronous in stream order on hip_stream. 0 = host memory;
 *   the call returns when the results are in place. */
typedef struct {
    uint32_t* cell_counts;
    double* power;
    double* power_ref;
    double* energy;
    uint32_t* depth_maps;
    uint32_t* shaded_bits;
    int32_t on_device;
} pv3d_outputs;

/* Evaluate one generator in one scene for a sweep of sun positions: the suns
 * above the horizon in groups of up to 32 per launch sequence (set-up,
 * binning, tile pass), then one loss launch over the sweep and the energy sums
 * in sun order. Results do not depend on the grouping.
 * sun_xyz: [n_sun][3] unit vectors toward the sun (|s| = 1 within 1e-9);
 * dni: [n_sun] direct normal irradiance; d_poa: [n_sun] diffuse irradiance on
 * the module plane; dt_h: [n_sun] hours each sun stands for. Host memory.
 * hip_stream: a stream created on this device, or NULL for the context stream.
 * NULL is not the null stream: the context stream is non-blocking, so work on
 * the null stream is not ordered with it. A caller working on the null stream
 * passes a stream of its own, made to wait for the null stream's work before
 * the call, and makes the null stream wait for it afterwards. The special
 * handles hipStreamLegacy and hipStreamPerThread are not accepted.
 * Consecutive groups take turns on two streams (hip_stream and one of the
 * context's), joined back into hip_stream. Calls of one context are ordered:
 * each waits for the previous evaluation's kernels before it reuses the
 * context's work buffers, whatever streams the two calls use.
 * EINVAL: bad params or inputs; ENOENT: bad handle; ENOMEM: budget. */
pv3d_status pv3d_evaluate(pv3d_ctx* ctx, uint64_t scene, uint64_t gen, const double* sun_xyz,
                          const double* dni, const double* d_poa, const double* dt_h,
                          int64_t n_sun, const pv3d_params* params, pv3d_outputs* out,
                          void* hip_stream);

/* pv3d_evaluate for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same evaluation with identical results, in work memory taken from a static
 * device array of 128 MiB (PV3D_NOALLOC_SCRATCH_BYTES) that the library holds
 * on every GPU it runs on until the process ends. The call itself allocates
 * nothing: no hipMalloc, hipFree, pinned host memory or events (stage timing
 * is off during the call). Scene and generator are loaded beforehand as
 * usual; the caller passes the inputs (host memory, copied before the call
 * returns) and the outputs, which must be device memory (out->on_device = 1;
 * EINVAL otherwise). The call is asynchronous on hip_stream (NULL: the
 * context stream) like pv3d_evaluate's device form.
 * The work memory grows with the scene's triangles times bin_limit and with
 * n_sun: an evaluation that does not fit even one sun at a time returns
 * ERANGE before anything is queued (a smaller bin_limit, which leaves the
 * results unchanged, or fewer suns per call fit more). Every call on one GPU,
 * from any context, shares the array and finds the last call's contents; the
 * library clears what must start at zero. Calls of one context are ordered
 * (each waits for the previous evaluation's kernels); calls from different
 * contexts on one GPU that overlap in time race on the array. */
#define PV3D_NOALLOC_SCRATCH_BYTES (128ull << 20)
pv3d_status pv3d_evaluate_noalloc(pv3d_ctx* ctx, uint64_t scene, uint64_t gen, const double* sun_xyz,
                                  const double* dni, const double* d_poa, const double* dt_h,
                                  int64_t n_sun, const pv3d_params* params, pv3d_outputs* out,
                                  void* hip_stream);

/* Work counts of the context's last pv3d_evaluate (waits for it to end):
 * out[0] suns, out[1] triangle set-up records summed over the suns (the scene
 * and module triangles inside the window after culling; a triangle cut at the
 * guard band counts once per piece), out[2] records handled by every tile
 * instead of binned, out[3] (record, tile) pairs binned. All zero before any
 * evaluation; the batched, serving and allocation-free forms do not update
 * them. */
pv3d_status pv3d_path_stats(pv3d_ctx* ctx, int64_t out[4]);

/* Diffuse shading (Sec. 4: obstacles also hide part of the diffuse sky, which
 * the paper's evaluation leaves out). An isotropic sky is seen through n_dir
 * fixed directions above the horizon, each standing for an equal share of it
 * (dirs: [n_dir][3] unit vectors with z > 0, host memory). Every direction is
 * evaluated as a sun of unit beam with params (the same picture and depth
 * test; export flags are ignored), and a cell's sky view factor is
 *   svf = sum_j w_j (1 - shaded_j / k^2) / sum_j w_j,  w_j = max(0, n . s_j),
 * summed in direction order, n the module's front normal; 1 when no
 * direction faces the module. svf_out: [n_cells] host memory. The call is
 * synchronous and works on the context stream. EINVAL: a direction not above
 * the horizon or not of unit length, bad params, a tracked generator (its
 * view of the sky changes with its pose); ENOENT: bad handle; ENOMEM. */
pv3d_status pv3d_sky_view(pv3d_ctx* ctx, uint64_t scene, uint64_t gen, const double* dirs, int64_t n_dir,
                          const pv3d_params* params, double* svf_out);

/* Attach per-cell sky view factors (svf: [n_cells] host memory, each in
 * [0, 1], copied) to a generator: from then on a cell's diffuse irradiance in
 * the shaded power is d_poa * svf[cell]; the reference power keeps the whole
 * sky. svf = NULL detaches them. Applies to evaluations started after the
 * call (per-sun, batched and serving); the call first waits for the device's
 * queued work, which may still read the factors it replaces. EINVAL: a value
 * outside [0, 1], a tracked generator; ENOENT: unknown generator; EBUSY: a
 * running serving job reads the generator. */
pv3d_status pv3d_generator_set_sky(pv3d_ctx* ctx, uint64_t gen, const double* svf);

/* One job = one (scene, generator, sweep) evaluation. Its input arrays must
 * stay valid until the call that takes the job returns; its outputs until the
 * job completes. */
typedef struct {
    uint64_t scene;
    uint64_t gen;
    const double* sun_xyz;
    const double* dni;
    const double* d_poa;
    const double* dt_h;
    int64_t n_sun;
    pv3d_params params;
    pv3d_outputs out;
} pv3d_job;

/* All suns above the horizon of all jobs in one persistent launch (the
 * per-job constants, the scene's bounding sphere and the sample tables, are
 * computed on the host and copied in). Workgroups take units of work (a sun's set-up, a range
 * of triangles, the bin scan, a range of bin entries, a tile, the sun's
 * losses) from per-slot queues in device memory; a slot holds one (job, sun)
 * item at a time and takes the next item when its sun is done, so uneven
 * scenes share the GPU without a return to the host. Per job, results
 * (counts, powers, energy) are identical to pv3d_evaluate with the same
 * params. flags may be 0 or PV3D_FULL_RASTER (EINVAL otherwise); tile is 0,
 * 32 or 64. A sun whose set-up records or bin entries exceed the slot's
 * capacity is evaluated again with the per-sun path after the launch, so the
 * result does not depend on the capacity. Returns when every job's outputs
 * are in place (the call synchronizes hip_stream). ENOMEM when the slots do
 * not fit the budget. */
pv3d_status pv3d_evaluate_batched(pv3d_ctx* ctx, const pv3d_job* jobs, int64_t n_jobs,
                                  void* hip_stream);

/* Autotuner of the batched form: times every candidate (tile edge 32 or 64 x
 * bin_limit, the number of tiles above which a triangle is not binned but
 * checked by every tile, 8, 16, 32, 64, 128 or 256) on up to n_probe of the
 * job's suns above the horizon (evenly spaced), through the persistent launch,
 * and writes the fastest into job->params.tile and job->params.bin_limit.
 * Every candidate gives identical results; only time differs. best_ms_out
 * (may be NULL) receives the winner's time for the probe suns. The job's
 * outputs are not written.
 * The choice is cached in the context by the job's class: map_n, k, flags,
 * the decade of its triangles (scene, plus the generator's modules when they
 * occlude) and the decade of its cells. A job of a class already tuned (or
 * loaded with pv3d_autotune_cache) takes the cached choice without timing,
 * and best_ms_out receives the time cached with it. */
pv3d_status pv3d_autotune(pv3d_ctx* ctx, pv3d_job* job, int32_t n_probe, double* best_ms_out);

/* The autotuner's cache: mode PV3D_TUNE_SAVE writes every cached class to the
 * JSON file at path (an array of objects with the keys map_n, k, flags,
 * tri_decade, cell_decade, tile, bin_limit, ms), PV3D_TUNE_LOAD adds the
 * classes of such a file to the context's cache (replacing classes it already
 * holds), PV3D_TUNE_CLEAR empties the cache (path may be NULL). ENOENT: the
 * file cannot be opened; EINVAL: unknown mode, a malformed file, or values
 * outside the autotuner's candidates. */
#define PV3D_TUNE_LOAD 0
#define PV3D_TUNE_SAVE 1
#define PV3D_TUNE_CLEAR 2
pv3d_status pv3d_autotune_cache(pv3d_ctx* ctx, const char* path, int32_t mode);

/* Memory and placement of the batched form: at most max_slots (item) slots
 * in flight, each with room for slot_records triangle set-up records (and 8
 * bin entries per record); 0 = library's choice (128 slots, 2^20 records). A
 * smaller budget per slot only sends more suns to the per-sun path. By
 * default each slot is served by the workgroups of one XCD (slot i by XCD
 * i % 8, when the device shows 8 XCD ids), so the slot's buffers stay in that
 * XCD's L2; PV3D_BATCH_ANY_XCD lets every XCD serve every slot. Results are
 * the same either way. EINVAL: negative values, max_slots above 4096, unknown
 * flags. */
#define PV3D_BATCH_ANY_XCD 1u
pv3d_status pv3d_batch_limits(pv3d_ctx* ctx, int32_t max_slots, int64_t slot_records, uint32_t flags);

/* Statistics of the last pv3d_evaluate_batched or pv3d_autotune launch:
 * out[0] items (suns) run, out[1] work units run, out[2] items evaluated
 * again with the per-sun path (capacity exceeded), out[3] workgroups of the
 * persistent launch, out[4] slots, out[5] elapsed microseconds of the
 * persistent launch (HIP events), out[6] XCD groups (8: slots served per
 * XCD, 1: by every XCD). */
pv3d_status pv3d_batch_stats(pv3d_ctx* ctx, int64_t out[7]);

/* Serving: submit a job to the context's serving loop (started by the first
 * submit, with a service thread of its own). At its start the loop takes, of
 * the context's unused HBM budget, its slots and then half of what is left
 * as the arena for job data (sweep, constants, and internal outputs). Jobs
 * are admitted in submission order as soon as their data fits the arena;
 * every sun of an admitted job becomes an item of the live persistent launch
 * that the loop keeps running while work is in flight, so jobs that arrive
 * while others run share the GPU with them (continuous batching). Per job,
 * results are identical to pv3d_evaluate with the same params (same rules
 * as pv3d_evaluate_batched: flags 0 or FULL_RASTER, tile 0/32/64). A sun
 * whose set-up records or bin entries exceed a slot's capacity is evaluated
 * again, alone, with the per-sun path when its job completes (its device power
 * reads NaN until then). The job's input arrays are copied before the call
 * returns. Host outputs are written
 * when the job completes; device outputs are written by the device while the
 * job runs. The job's scene and generator cannot be released until it ends
 * (EBUSY). Limits: at most 4096 modules and 65536 raster tiles per job.
 * The loop's persistent kernel runs on a stream with a hardware queue of its
 * own, so the loop's copies and the context's other streams never wait behind
 * a live launch. That stream (made with a CU mask, which takes no flags) is a
 * blocking one: work the caller puts on the null stream while a launch is
 * live waits for that launch to end, so a caller serving and computing at once
 * works on streams of its own. EBUSY: 65536 jobs wait already; ENOMEM: the job's data can never fit the
 * arena. ticket identifies the job. */
pv3d_status pv3d_submit(pv3d_ctx* ctx, const pv3d_job* job, uint64_t* ticket);
/* done = 1 once the job has ended (outputs in place, cancelled or failed). */
pv3d_status pv3d_poll(pv3d_ctx* ctx, uint64_t ticket, int32_t* done);
/* Block until the job has ended; ECANCELED if it was cancelled, the failure's
 * code if it failed. Forgets the ticket. */
pv3d_status pv3d_wait(pv3d_ctx* ctx, uint64_t ticket);
/* Cancel a job. A job not yet admitted never runs; an admitted one runs to
 * its end but its host outputs are not written (device outputs may be, until
 * pv3d_wait returns). Outputs are undefined either way. */
pv3d_status pv3d_cancel(pv3d_ctx* ctx, uint64_t ticket);
/* Serving statistics: out[0] jobs ended, out[1] persistent launches started
 * by the loop, out[2] items (suns) published, out[3] jobs waiting for
 * admission. */
pv3d_status pv3d_serve_stats(pv3d_ctx* ctx, int64_t out[4]);

/* Kernel timing, a profiling aid. With bit i of stage_mask set, the per-sun
 * path records a pair of HIP events on its stream around every launch of
 * stage i (0 tri_setup, 1 bin_scan: the tile counts and their scan,
 * 2 bin_scatter, 3 raster, 4 sample_test, 5 setup, 6 loss); mask 0 turns recording off and clears the sums.
 * pv3d_profile_read waits for the recorded work and returns, for one stage,
 * the summed event-measured duration in milliseconds and the launch count. */
#define PV3D_STAGE_TRI_SETUP 0
#define PV3D_STAGE_BIN_SCAN 1
#define PV3D_STAGE_BIN_SCATTER 2
#define PV3D_STAGE_RASTER 3
#define PV3D_STAGE_SAMPLE_TEST 4
#define PV3D_STAGE_SETUP 5
#define PV3D_STAGE_LOSS 6
#define PV3D_N_STAGES 7
pv3d_status pv3d_profile_enable(pv3d_ctx* ctx, uint32_t stage_mask);
pv3d_status pv3d_profile_read(pv3d_ctx* ctx, int32_t stage, double* total_ms, int64_t* launches);
/* The time during which at least one timed launch of the stage ran (the
 * union of their event intervals, so launches of the two lanes that overlap
 * count once: the stage's exclusive share of the sweep), in milliseconds, and
 * the suns those launches covered (a launch covers a group of up to 32 suns).
 * Meaningful when every launch is timed (pv3d_profile_sample 1). Waits for
 * the recorded work. EINVAL: bad stage. */
pv3d_status pv3d_profile_busy(pv3d_ctx* ctx, int32_t stage, double* busy_ms, int64_t* suns);
/* Record only every n-th launch of each profiled stage (n >= 1; 1 after
 * pv3d_create): the events sit between kernels of the stream and hold back
 * the overlap of the two lanes, so a sample disturbs a long sweep less than
 * timing every launch. launches (pv3d_profile_read) counts the timed ones.
 * EINVAL: n < 1. */
pv3d_status pv3d_profile_sample(pv3d_ctx* ctx, int32_t every);

#ifdef __cplusplus
}
#endif

#endif /* PV3D_H */
