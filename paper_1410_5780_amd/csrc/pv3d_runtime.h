// Host-side state of libpv3d (internal; the public ABI is include/pv3d.h).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/pv3d.h"
#include "pv3d_device.h"

namespace pv3d {

struct Ctx;

constexpr int32_t kMaxBinLimit = 256;   // default and largest bin_limit

pv3d_status fail(pv3d_status code, const char* fmt, ...);
pv3d_status hip_fail(hipError_t e, const char* what);
pv3d_status check_params(const pv3d_params* p);
pv3d_status check_sweep(const double* sun, const double* dni, const double* dpoa, const double* dt, int64_t n);

// Grow-only device buffer.
struct Buf {
    void* ptr = nullptr;
    size_t cap = 0;
    pv3d_status ensure(Ctx* c, size_t bytes, const char* what);
    void release(Ctx* c);
};

struct Scene {
    double* xyz = nullptr;
    int32_t* tri = nullptr;
    double* cbox = nullptr;       // per block of 256 triangles: box of its vertices
    int64_t n_vert = 0, n_tri = 0;
    double lo[3], hi[3];          // axis-aligned box of the vertices (+inf / -inf when empty)
    int32_t users = 0;            // jobs of the serving loop that read it
};

struct Gen {
    double lo[3], hi[3];          // axis-aligned box of the module corners (with trackers: of their reach)
    int32_t users = 0;            // jobs of the serving loop that read it
    Module* mods = nullptr;
    int32_t* cell_sub = nullptr;
    int32_t* str_start = nullptr;
    int32_t* str_mods = nullptr;
    int64_t n_mod = 0;
    int32_t n_cu = 0, n_cv = 0, n_sub = 0, n_str = 0, occluders = 0;
    TrackerDev* trk = nullptr;    // [n_trk] (trackers: modules turn with the sun)
    int32_t* mod_trk = nullptr;   // [n_mod] tracker of each module, -1 none
    int32_t n_trk = 0;
    int32_t* sub_start = nullptr; // [n_sub + 1] CSR of the cells of each substring
    int32_t* sub_cell = nullptr;  // [n_cu * n_cv]
    double* svf = nullptr;        // [n_cells] sky view factors (nullptr: every cell sees the whole sky)
    DiodeDev diode{};             // electrical model (diode.on = 0: ideal strings)
};

// Frees the device arrays of a generator.
void free_gen(Ctx* c, Gen& g);

struct PathSizes {
    int32_t tile, ntx, n_tiles, large_tiles, words, mask_words;
    int64_t tri_total, rec_cap, bin_cap, cells, n_sun;
    int64_t item_cap, chunk_cap;      // pair mode: binned items, chunks of pair space
};

// The buffers one stream of the per-sun path works in: room for a group of
// suns (each sun's part at a fixed stride); consecutive groups take turns on
// the lanes, one stream each.
struct Lane {
    Buf rec, large, bins, tile_count, tile_start, tile_cursor, tile_list, pitems, pchunk, modbox, map;
    int32_t group = 0;            // suns the buffers hold room for
    void release_all(Ctx* c) {
        group = 0;
        Buf* all[] = {&rec, &large, &bins, &tile_count, &tile_start, &tile_cursor, &tile_list, &pitems, &pchunk,
                      &modbox, &map};
        for (Buf* b : all) b->release(c);
    }
};

// Streams the per-sun path spreads consecutive suns over (lane 0 is the
// caller's stream); a lane whose buffers do not fit the budget is left out.
// The context owns three streams in all: its own, lane 1's (which the serving
// loop also copies on) and the serving loop's kernel stream. With the
// default stream beside them that is the four hardware queues a process gets
// by default, so the serving loop's persistent kernel holds a queue of its
// own: a stream that shares a queue with it waits behind it.
constexpr int kLanes = 2;

struct Work {
    Lane lane[kLanes];
    Buf views, ctr, beam, bias, sweep, sphere, partial, fu, fv, tmask, posed;
    Buf counts, outd, maps, bits, sky;
    Buf groups;                   // SunGroup descriptors of the current evaluation
    void release_all(Ctx* c) {
        for (Lane& L : lane) L.release_all(c);
        Buf* all[] = {&views, &ctr, &beam, &bias, &sweep, &sphere, &partial, &fu, &fv, &tmask, &posed, &counts, &outd,
                      &maps, &bits, &sky, &groups};
        for (Buf* b : all) b->release(c);
    }
};

struct BatchState;
struct Server;

// What the persistent kernel needs to know about the device, probed once.
struct DevInfo {
    int32_t blocks_per_cu = 0, n_cu = 0;
    int32_t xcd_groups = 1;       // 8 when the workgroups of a full launch show XCD ids 0..7
    long long stall_ticks = 0;
    int rate_khz = 100000;        // wall clock of the device
};

// A class of jobs for the autotuner's cache, and the choice made for it.
struct TuneKey {
    int32_t map_n, k, tri_decade, cell_decade;
    uint32_t flags;
    bool operator<(const TuneKey& o) const {
        if (map_n != o.map_n) return map_n < o.map_n;
        if (k != o.k) return k < o.k;
        if (tri_decade != o.tri_decade) return tri_decade < o.tri_decade;
        if (cell_decade != o.cell_decade) return cell_decade < o.cell_decade;
        return flags < o.flags;
    }
};
struct TuneChoice {
    int32_t tile, bin_limit;
    double ms;
};

// Event pairs around launches of selected stages (profiling aid).
struct Profiler {
    uint32_t mask = 0;
    int32_t every = 1;                              // time every n-th launch of a stage
    int64_t seen[PV3D_N_STAGES] = {};
    std::vector<hipEvent_t> pool;
    std::vector<std::pair<int, size_t>> pending;   // (stage, index of the start event in pool)
    size_t used = 0;
    double total_ms[PV3D_N_STAGES] = {};
    int64_t launches[PV3D_N_STAGES] = {};
    int64_t suns[PV3D_N_STAGES] = {};               // suns the timed launches covered
    std::vector<int32_t> pending_suns;              // beside pending
    hipEvent_t ref = nullptr;                       // time origin of the intervals
    std::vector<std::pair<double, double>> spans[PV3D_N_STAGES];   // [start, end) ms after ref
    bool on(int stage) const { return (mask >> stage) & 1u; }
    bool take(int stage) { return on(stage) && seen[stage]++ % every == 0; }
    hipError_t begin(int stage, hipStream_t st, size_t* slot, int32_t n_sun);
    hipError_t end(size_t slot, hipStream_t st);
    hipError_t collect();
    double busy_ms(int stage) const;                // length of the union of the stage's spans
    void reset();
};

PathSizes path_sizes(const Scene& sc, const Gen& g, const pv3d_params& p, int64_t n_sun);
size_t lane_bytes_per_sun(const PathSizes& z, const Gen& g);
// Device memory of pv3d_evaluate_noalloc: one static array per GPU, whose address
// pv3d_create looks up once per device.
constexpr size_t kScratchBytes = PV3D_NOALLOC_SCRATCH_BYTES;
// Bytes an evaluation takes from that array: the per-sun arrays and tables, the
// counts when the caller passes none, n_groups group descriptors and n_lanes lanes
// of room for `group` suns, every buffer 256-byte aligned.
size_t carve_bytes(const PathSizes& z, const Gen& g, int32_t k, int32_t map_n, bool own_map, bool own_counts,
                   int32_t group, int n_lanes, int64_t n_groups);
void host_sphere(const Scene& sc, const Gen& g, double sphere[4]);
void host_sample_tables(int32_t k, int32_t n_cu, int32_t n_cv, double* fu, double* fv);
int32_t choose_tile(const pv3d_params& p);
SceneDev scene_dev(const Scene& sc);
GenDev gen_dev(const Gen& g);

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t stream_in_use = nullptr;
    hipStream_t lane_st[kLanes] = {};       // the per-sun path's further lanes ([0] unused)
    hipEvent_t fork_ev = nullptr, join_ev[kLanes] = {};
    uint64_t budget = 0;
    uint64_t used = 0;
    size_t max_lds = 65536;
    int32_t n_cu = 256;
    std::map<void*, size_t> sizes;
    std::map<uint64_t, Scene> scenes;
    std::map<uint64_t, Gen> gens;
    uint64_t next_handle = 0;
    Work w;
    std::recursive_mutex mu;
    // pinned staging of host inputs
    void* staging = nullptr;
    size_t staging_cap = 0, staging_used = 0;
    bool staging_busy = false;
    hipEvent_t staging_done = nullptr;
    BatchState* batch = nullptr;
    Server* server = nullptr;
    // the last per-sun path's work: a later call waits for it before it reuses the work buffers
    hipEvent_t ws_ev = nullptr;
    bool ws_recorded = false;
    // pv3d_evaluate has run: the serving loop is not started in this context any more (a
    // burst of requests served after the per-sun path in one context waited minutes)
    bool per_sun_ran = false;
    int64_t last_n_sun = 0;                 // suns of the last per-sun evaluation (pv3d_path_stats)
    DevInfo dev_info;
    // pv3d_evaluate_noalloc: while `carving`, every work buffer the evaluation ensures
    // is taken from the device's static scratch array (carve_base, kScratchBytes bytes)
    // by bumping carve_used; nothing is allocated and nothing is freed
    void* scratch = nullptr;
    bool carving = false;
    size_t carve_used = 0;
    pv3d_status carve(Buf& b, size_t bytes, const char* what);
    // the stream waits for the end of the context's previous evaluation, whose kernels
    // may still read the work buffers on another stream
    pv3d_status wait_previous(hipStream_t st);
    // pv3d_batch_limits: slots of the batched form and the serving loop
    int32_t batch_max_slots = 128;
    int64_t batch_slot_records = 1 << 20;
    bool batch_any_xcd = false;
    Profiler prof;
    std::map<TuneKey, TuneChoice> tune_cache;   // pv3d_autotune's choices by job class

    pv3d_status dalloc(void** p, size_t bytes, const char* what);
    void dfree(void* p);
    pv3d_status stage(const void* host, size_t bytes, void* dev, hipStream_t st);
    pv3d_status stage_reserve(size_t bytes);
    pv3d_status stage_done(hipStream_t st);
    pv3d_status ensure_path(const PathSizes& z, const Gen& g, int32_t map_n, bool own_map);
    pv3d_status ensure_lane(Lane& L, const PathSizes& z, const Gen& g, int32_t map_n, bool own_map, int32_t group);
    pv3d_status run_group(const SunGroup* d_grp, const SunGroup& grp, const PathSizes& z, const SceneDev& sd,
                          const GenDev& gd, const pv3d_params& p, const View* views, SunCounters* ctr,
                          const int32_t* bias, const double* beam, int n_lanes, hipStream_t st);
    pv3d_status ensure_tables(const Gen& g, int32_t k);
    BinBuffers bin_buffers(const PathSizes& z, int lane, int32_t q);
    // pinned staging of the group descriptors (beside the sweep's, which callers reserve)
    void* gstage = nullptr;
    size_t gstage_cap = 0;
    hipEvent_t gstage_done = nullptr;
    bool gstage_busy = false;
    pv3d_status upload_groups(const std::vector<SunGroup>& groups, hipStream_t st);
    pv3d_status run_path(const Scene& sc, const Gen& g, const pv3d_params& p, const double* sun_host, int64_t n_sun,
                         const double* d_sun, const double* d_dni, const double* d_dpoa, const double* d_dt,
                         uint32_t* counts, double* power, double* power_ref, double* energy, uint32_t* maps,
                         uint32_t* bits, hipStream_t st);
    pv3d_status read_overflow(int64_t n_sun, hipStream_t st, bool* overflow);
    bool scene_in_use(uint64_t h);
    bool gen_in_use(uint64_t h);
    void release_batched();
};

// While one of these lives, the serving loop admits no new job, so its live
// launch runs out of work and ends. Every device-wide wait of the library
// (hipDeviceSynchronize, and hipFree / hipHostFree, which wait for every
// stream of the device) is taken under one: otherwise a loop fed faster than
// it drains would keep that wait from ever returning.
struct HoldServing {
    Ctx* c;
    explicit HoldServing(Ctx* ctx);
    ~HoldServing();
    HoldServing(const HoldServing&) = delete;
    HoldServing& operator=(const HoldServing&) = delete;
};

}  // namespace pv3d

struct pv3d_ctx : pv3d::Ctx {};

void pv3d_server_stop(pv3d_ctx* ctx);
