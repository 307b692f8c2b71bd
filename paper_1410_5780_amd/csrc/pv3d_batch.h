// Host pieces shared by the batched form and the serving loop of libpv3d:
// job checks, the layout of slot buffers, the job table entry, and what the
// device tells about its XCDs (internal; the public ABI is include/pv3d.h).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/pv3d.h"
#include "pv3d_device.h"
#include "pv3d_runtime.h"

namespace pv3d {

constexpr int32_t kMaxSlots = 128;          // items in flight
constexpr int64_t kSlotRecCap = 1 << 20;    // set-up records per slot (more: the sun goes to the per-sun path)
constexpr double kStallSeconds = 5.0;       // watchdog of the persistent launch

inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

pv3d_status device_info(Ctx* c, DevInfo* out);

// One batch through the persistent kernel (pv3d_evaluate_batched).
pv3d_status run_batch(Ctx* c, const pv3d_job* jobs, int64_t n_jobs, hipStream_t s);

// Host view of one job: sizes, and the device regions of its data.
struct HostJob {
    const Scene* sc;
    const Gen* g;
    pv3d_job job;
    int32_t tile, ntx, n_tiles, words, large_tiles, sparse, use_mask;
    int64_t cells, tri_all, n_items;
    double *d_sun, *d_dni, *d_dpoa, *d_dt, *d_sphere, *d_fu, *d_fv;
    Module* d_posed;          // trackers: [n_sun][n_mod] modules posed per sun
    uint32_t* d_counts;
    double *d_power, *d_pref, *d_energy;
};

// Validate one job (params, sweep, handles, outputs) and fill its sizes.
// Tracked generators are taken only when allow_tracked (the batched form).
pv3d_status check_job(Ctx* c, const pv3d_job& j, int64_t idx, HostJob& h, bool allow_tracked = false);

// Bytes of a job's device data: sweep, sphere, sample tables, posed modules
// (trackers), and (when with_outputs) counts, powers and energy.
size_t job_bytes(const HostJob& h, bool with_counts, bool with_powers);

// Lay out the job's device data from p on (the regions listed in job_bytes).
void carve_job(HostJob& h, char* p, bool with_counts, bool with_powers);

// Host copy of the job's sphere and sample tables: [4 + k (n_cu + n_cv)] doubles.
void job_constants(const HostJob& h, std::vector<double>& tab);

// The job table entry of the persistent kernel.
PJob make_pjob(const HostJob& h);

// Slot buffers: one region per array kind, so every slot's tile counters
// clear in one call.
struct SlotGeom {
    int64_t rec_cap, bin_cap, max_tiles, max_mod;
    size_t per_rec, per_large, per_bins, per_t, per_list, per_mod, per_misc, slot_bytes;
};
SlotGeom slot_geom(int64_t rec_cap, int64_t bin_cap, int64_t max_tiles, int64_t max_mod);
// Fills out[0..n_slots) and returns the tile-counter region (per_t * n_slots bytes).
char* carve_slots(char* base, const SlotGeom& g, int64_t n_slots, std::vector<PSlotBufs>& out);

}  // namespace pv3d
