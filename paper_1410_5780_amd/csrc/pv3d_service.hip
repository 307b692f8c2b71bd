// Batched form of libpv3d: every (job, sun) item of a set of jobs in one
// persistent launch (k_persist), and the autotuner that picks its tile and
// bin sizes.
//
// Host side of a batch:
//   1. validate the jobs, copy their sweeps and constants (bounding sphere,
//      sample tables, computed on the host) to the device in one staging pass,
//      and zero their outputs (suns below the horizon keep zero power);
//   2. size the slots (work buffers of one item each) from the largest job
//      and the HBM budget, zero their tile counters, seed the first items;
//   3. one persistent launch over the list of suns above the horizon;
//   4. suns that exceeded a slot's capacity are evaluated again with the
//      per-sun path, and their jobs' energies summed again;
//   5. copy host outputs back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <iterator>
#include <string>
#include <memory>
#include <vector>

#include "../../include/pv3d.h"
#include "pv3d_batch.h"
#include "pv3d_device.h"
#include "pv3d_runtime.h"

using namespace pv3d;

namespace pv3d {

struct BatchState {
    Buf slotmem, slots, state, sched, jobs, items, jobdone, overflow, jobmem, energy_tmp;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int64_t stats[7] = {};
};

void Ctx::release_batched() {
    if (!batch) return;
    BatchState& b = *batch;
    Buf* all[] = {&b.slotmem, &b.slots, &b.state, &b.sched, &b.jobs, &b.items, &b.jobdone, &b.overflow, &b.jobmem, &b.energy_tmp};
    for (Buf* x : all) x->release(this);
    if (b.ev0) (void)hipEventDestroy(b.ev0);
    if (b.ev1) (void)hipEventDestroy(b.ev1);
    delete batch;
    batch = nullptr;
}

pv3d_status device_info(Ctx* c, DevInfo* out) {
    if (c->dev_info.n_cu == 0) {
        DevInfo d;
        hipError_t e;
        int32_t bpc = 0;
        if ((e = persist_blocks_per_cu(&bpc))) return hip_fail(e, "occupancy of the persistent kernel");
        hipDeviceProp_t prop;
        if ((e = hipGetDeviceProperties(&prop, c->device))) return hip_fail(e, "hipGetDeviceProperties");
        int rate_khz = 0;
        if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, c->device) != hipSuccess || rate_khz <= 0)
            rate_khz = 100000;
        d.blocks_per_cu = std::max(1, bpc);
        d.n_cu = std::max(1, prop.multiProcessorCount);
        d.rate_khz = rate_khz;
        d.stall_ticks = (long long)(kStallSeconds * 1000.0 * (double)rate_khz);
        // XCD ids the workgroups of a full-device launch run on
        uint32_t* d_mask = nullptr;
        if ((e = hipMalloc(&d_mask, 256))) return hip_fail(e, "hipMalloc");
        uint32_t mask = 0;
        e = hipMemsetAsync(d_mask, 0, 4, c->stream);
        if (!e) e = launch_xcc_probe(d_mask, 8 * d.n_cu, c->stream);
        if (!e) e = hipMemcpyAsync(&mask, d_mask, 4, hipMemcpyDeviceToHost, c->stream);
        if (!e) e = hipStreamSynchronize(c->stream);
        {
            HoldServing hold(c);            // hipFree waits for every stream of the device
            (void)hipFree(d_mask);
        }
        if (e) return hip_fail(e, "XCD probe");
        d.xcd_groups = mask == 0xFFu ? 8 : 1;
        c->dev_info = d;
    }
    *out = c->dev_info;
    return PV3D_OK;
}

static pv3d_status batch_state(Ctx* c, BatchState** out) {
    if (!c->batch) {
        std::unique_ptr<BatchState> b(new BatchState());
        hipError_t e;
        if ((e = hipEventCreate(&b->ev0)) || (e = hipEventCreate(&b->ev1))) return hip_fail(e, "hipEventCreate");
        c->batch = b.release();
    }
    *out = c->batch;
    return PV3D_OK;
}

pv3d_status check_job(Ctx* c, const pv3d_job& j, int64_t idx, HostJob& h, bool allow_tracked) {
    pv3d_status st;
    if ((st = check_params(&j.params))) return fail(st, "job %lld: %s", (long long)idx, pv3d_last_error(nullptr));
    if (j.params.flags & ~PV3D_FULL_RASTER)
        return fail(PV3D_EINVAL, "job %lld: the batched form takes flags 0 or FULL_RASTER", (long long)idx);
    if (j.params.tile != 0 && j.params.tile != 32 && j.params.tile != 64)
        return fail(PV3D_EINVAL, "job %lld: the batched form takes tile 0, 32 or 64", (long long)idx);
    if ((st = check_sweep(j.sun_xyz, j.dni, j.d_poa, j.dt_h, j.n_sun)))
        return fail(st, "job %lld: %s", (long long)idx, pv3d_last_error(nullptr));
    if (!j.out.power || !j.out.power_ref || !j.out.energy)
        return fail(PV3D_EINVAL, "job %lld: power, power_ref and energy are required", (long long)idx);
    auto si = c->scenes.find(j.scene);
    if (si == c->scenes.end()) return fail(PV3D_ENOENT, "job %lld: unknown scene %llu", (long long)idx, (unsigned long long)j.scene);
    auto gi = c->gens.find(j.gen);
    if (gi == c->gens.end()) return fail(PV3D_ENOENT, "job %lld: unknown generator %llu", (long long)idx, (unsigned long long)j.gen);
    const Gen& g = gi->second;
    if (g.n_trk > 0 && !allow_tracked)
        return fail(PV3D_EINVAL, "job %lld: the serving loop does not take tracked generators", (long long)idx);
    if ((int64_t)j.params.k * g.n_cu > 4095 || (int64_t)j.params.k * g.n_cv > 4095)
        return fail(PV3D_ERANGE, "job %lld: k * cells per module side exceeds 4095 samples", (long long)idx);
    memset(&h, 0, sizeof(h));
    h.sc = &si->second;
    h.g = &g;
    h.job = j;
    h.tile = j.params.tile ? j.params.tile : 64;
    h.ntx = (j.params.map_n + h.tile - 1) / h.tile;
    h.n_tiles = h.ntx * h.ntx;
    h.words = (h.n_tiles + 31) / 32;
    h.large_tiles = j.params.bin_limit ? j.params.bin_limit : kMaxBinLimit;
    h.sparse = (j.params.flags & PV3D_FULL_RASTER) ? 0 : 1;
    h.use_mask = h.sparse && h.words <= 512;
    h.cells = g.n_mod * g.n_cu * g.n_cv;
    h.tri_all = h.sc->n_tri + (g.occluders ? 2 * g.n_mod : 0);
    h.n_items = 0;
    for (int64_t t = 0; t < j.n_sun; t++)
        if (j.sun_xyz[3 * t + 2] > 0.0) h.n_items++;
    return PV3D_OK;
}

static size_t table_bytes(const HostJob& h) {
    return al256(8 * (size_t)h.job.params.k * std::max(h.g->n_cu, h.g->n_cv));
}

size_t job_bytes(const HostJob& h, bool with_counts, bool with_powers) {
    const size_t ns = (size_t)h.job.n_sun;
    size_t b = al256(48 * ns) + 256 + 2 * table_bytes(h);
    if (h.g->n_trk > 0) b += al256(sizeof(Module) * ns * (size_t)h.g->n_mod);
    if (with_counts) b += al256(4 * ns * (size_t)h.cells);
    if (with_powers) b += al256(16 * ns) + 256;
    return b;
}

void carve_job(HostJob& h, char* p, bool with_counts, bool with_powers) {
    const int64_t ns = h.job.n_sun;
    h.d_sun = reinterpret_cast<double*>(p);
    h.d_dni = h.d_sun + 3 * ns;
    h.d_dpoa = h.d_dni + ns;
    h.d_dt = h.d_dpoa + ns;
    p += al256(48 * (size_t)ns);
    h.d_sphere = reinterpret_cast<double*>(p);
    p += 256;
    const size_t tb = table_bytes(h);
    h.d_fu = reinterpret_cast<double*>(p);
    p += tb;
    h.d_fv = reinterpret_cast<double*>(p);
    p += tb;
    h.d_posed = nullptr;
    if (h.g->n_trk > 0) {
        h.d_posed = reinterpret_cast<Module*>(p);
        p += al256(sizeof(Module) * (size_t)ns * (size_t)h.g->n_mod);
    }
    if (with_counts) {
        h.d_counts = reinterpret_cast<uint32_t*>(p);
        p += al256(4 * (size_t)(ns * h.cells));
    }
    if (with_powers) {
        h.d_power = reinterpret_cast<double*>(p);
        h.d_pref = h.d_power + ns;
        p += al256(16 * (size_t)ns);
        h.d_energy = reinterpret_cast<double*>(p);
    }
}

void job_constants(const HostJob& h, std::vector<double>& tab) {
    const int32_t kk = h.job.params.k;
    tab.assign(4 + (size_t)kk * (h.g->n_cu + h.g->n_cv), 0.0);
    host_sphere(*h.sc, *h.g, tab.data());
    host_sample_tables(kk, h.g->n_cu, h.g->n_cv, tab.data() + 4, tab.data() + 4 + (size_t)kk * h.g->n_cu);
}

PJob make_pjob(const HostJob& h) {
    PJob J;
    memset(&J, 0, sizeof(J));
    J.sc = scene_dev(*h.sc);
    J.g = gen_dev(*h.g);
    J.g.mods_sun = h.d_posed;
    J.sun = h.d_sun;
    J.dni = h.d_dni;
    J.dpoa = h.d_dpoa;
    J.counts = h.d_counts;
    J.power = h.d_power;
    J.power_ref = h.d_pref;
    J.energy = h.d_energy;
    J.dt = h.d_dt;
    J.sphere = h.d_sphere;
    J.fu = h.d_fu;
    J.fv = h.d_fv;
    J.n_sun = h.job.n_sun;
    J.cells = h.cells;
    J.n = h.job.params.map_n;
    J.k = h.job.params.k;
    J.tile = h.tile;
    J.sparse = h.sparse;
    J.use_mask = h.use_mask;
    J.large_tiles = h.large_tiles;
    J.ntx = h.ntx;
    J.n_tiles = h.n_tiles;
    J.words = h.words;
    J.n_items = (int32_t)h.n_items;
    J.done_target = (uint32_t)h.n_items;
    return J;
}

SlotGeom slot_geom(int64_t rec_cap, int64_t bin_cap, int64_t max_tiles, int64_t max_mod) {
    SlotGeom g;
    g.rec_cap = rec_cap;
    g.bin_cap = bin_cap;
    g.max_tiles = max_tiles;
    g.max_mod = max_mod;
    g.per_rec = al256(80 * (size_t)rec_cap);
    g.per_large = al256(4 * (size_t)rec_cap);
    g.per_bins = al256(4 * (size_t)bin_cap);
    g.per_t = al256(4 * (size_t)(max_tiles + 1));
    g.per_list = al256(4 * (size_t)max_tiles);           // one item per tile, in tile order
    g.per_mod = al256(16 * (size_t)max_mod) + al256(8 * (size_t)max_mod) + al256(4 * (size_t)max_mod);
    g.per_misc = 256 /*view*/ + al256(4 * 512) /*mask*/ + 256 /*counters*/;
    g.slot_bytes = g.per_rec + g.per_large + g.per_bins + 3 * g.per_t + g.per_list + g.per_mod + g.per_misc;
    return g;
}

char* carve_slots(char* q, const SlotGeom& g, int64_t n_slots, std::vector<PSlotBufs>& out) {
    const size_t ns = (size_t)n_slots;
    char* r_rec = q; q += g.per_rec * ns;
    char* r_large = q; q += g.per_large * ns;
    char* r_bins = q; q += g.per_bins * ns;
    char* r_tc = q; q += g.per_t * ns;
    char* r_ts = q; q += g.per_t * ns;
    char* r_tcur = q; q += g.per_t * ns;
    char* r_tl = q; q += g.per_list * ns;
    char* r_mod = q; q += g.per_mod * ns;
    char* r_misc = q;
    out.resize(ns);
    for (size_t i = 0; i < ns; i++) {
        PSlotBufs& b = out[i];
        b.rec = reinterpret_cast<TriRec*>(r_rec + g.per_rec * i);
        b.large = reinterpret_cast<int32_t*>(r_large + g.per_large * i);
        b.bins = reinterpret_cast<int32_t*>(r_bins + g.per_bins * i);
        b.tile_count = reinterpret_cast<int32_t*>(r_tc + g.per_t * i);
        b.tile_start = reinterpret_cast<int32_t*>(r_ts + g.per_t * i);
        b.tile_cursor = reinterpret_cast<int32_t*>(r_tcur + g.per_t * i);
        b.tile_list = reinterpret_cast<int32_t*>(r_tl + g.per_list * i);
        char* m = r_mod + g.per_mod * i;
        b.modbox = reinterpret_cast<int4*>(m);
        b.beam = reinterpret_cast<double*>(m + al256(16 * (size_t)g.max_mod));
        b.bias = reinterpret_cast<int32_t*>(m + al256(16 * (size_t)g.max_mod) + al256(8 * (size_t)g.max_mod));
        char* x = r_misc + g.per_misc * i;
        b.view = reinterpret_cast<View*>(x);
        b.tmask = reinterpret_cast<uint32_t*>(x + 256);
        b.ctr = reinterpret_cast<SunCounters*>(x + 256 + al256(4 * 512));
    }
    return r_tc;
}

// One batch: every job's suns above the horizon through the persistent kernel.
pv3d_status run_batch(Ctx* c, const pv3d_job* jobs, int64_t n_jobs, hipStream_t s) {
    BatchState* B = nullptr;
    pv3d_status st;
    if ((st = batch_state(c, &B))) return st;
    DevInfo D;
    if ((st = device_info(c, &D))) return st;
    for (int i = 0; i < 7; i++) B->stats[i] = 0;
    std::vector<HostJob> H((size_t)n_jobs);
    int64_t n_items = 0, sweep_total = 0;
    for (int64_t i = 0; i < n_jobs; i++) {
        if ((st = check_job(c, jobs[i], i, H[(size_t)i], true))) return st;
        n_items += H[(size_t)i].n_items;
        sweep_total += jobs[i].n_sun;
    }
    if (n_items >= INT32_MAX) return fail(PV3D_ERANGE, "more than 2^31 suns in one batch");
    hipError_t e;

    // --- per-job device memory: sweep, sphere, sample tables, internal outputs
    size_t jm = 0;
    std::vector<size_t> off((size_t)n_jobs);
    for (int64_t i = 0; i < n_jobs; i++) {
        const HostJob& h = H[(size_t)i];
        off[(size_t)i] = jm;
        jm += job_bytes(h, !h.job.out.on_device || !h.job.out.cell_counts, !h.job.out.on_device);
    }
    if ((st = B->jobmem.ensure(c, std::max<size_t>(jm, 256), "batched job data"))) return st;
    if ((st = B->energy_tmp.ensure(c, 256, "energy scratch"))) return st;
    size_t tab_total = 0;
    for (const HostJob& h : H) tab_total += 2 * al256(8 * (size_t)h.job.params.k * std::max(h.g->n_cu, h.g->n_cv)) + 256;
    if ((st = c->stage_reserve(48 * (size_t)sweep_total + 256 * 4 * (size_t)n_jobs + tab_total))) return st;
    std::vector<double> tab;
    char* base = static_cast<char*>(B->jobmem.ptr);
    for (int64_t i = 0; i < n_jobs; i++) {
        HostJob& h = H[(size_t)i];
        const int64_t ns = h.job.n_sun;
        const bool own_counts = !h.job.out.on_device || !h.job.out.cell_counts;
        carve_job(h, base + off[(size_t)i], own_counts, !h.job.out.on_device);
        if (!own_counts) h.d_counts = h.job.out.cell_counts;
        if (h.job.out.on_device) {
            h.d_power = h.job.out.power;
            h.d_pref = h.job.out.power_ref;
            h.d_energy = h.job.out.energy;
        }
        if (ns > 0) {
            if ((st = c->stage(h.job.sun_xyz, 24 * (size_t)ns, h.d_sun, s))) return st;
            if ((st = c->stage(h.job.dni, 8 * (size_t)ns, h.d_dni, s))) return st;
            if ((st = c->stage(h.job.d_poa, 8 * (size_t)ns, h.d_dpoa, s))) return st;
            if ((st = c->stage(h.job.dt_h, 8 * (size_t)ns, h.d_dt, s))) return st;
        }
        // bounding sphere and sample tables, computed on the host (no launch per job)
        const int32_t kk = h.job.params.k;
        job_constants(h, tab);
        if ((st = c->stage(tab.data(), 32, h.d_sphere, s))) return st;
        if ((st = c->stage(tab.data() + 4, 8 * (size_t)kk * h.g->n_cu, h.d_fu, s))) return st;
        if ((st = c->stage(tab.data() + 4 + (size_t)kk * h.g->n_cu, 8 * (size_t)kk * h.g->n_cv, h.d_fv, s))) return st;
    }
    if ((st = c->stage_done(s))) return st;
    for (int64_t i = 0; i < n_jobs; i++) {
        HostJob& h = H[(size_t)i];
        const int64_t ns = h.job.n_sun;
        if (ns > 0) {
            if ((e = hipMemsetAsync(h.d_counts, 0, 4 * (size_t)(ns * h.cells), s))) return hip_fail(e, "clear counts");
            if ((e = hipMemsetAsync(h.d_power, 0, 8 * (size_t)ns, s))) return hip_fail(e, "clear power");
            if ((e = hipMemsetAsync(h.d_pref, 0, 8 * (size_t)ns, s))) return hip_fail(e, "clear power_ref");
        }
        if ((e = hipMemsetAsync(h.d_energy, 0, 16, s))) return hip_fail(e, "clear energy");
        // trackers: every module posed for every sun before the launch reads them
        if (h.d_posed && ns > 0 &&
            (e = launch_pose(h.d_sun, ns, h.g->mods, (int32_t)h.g->n_mod, h.g->trk, h.g->mod_trk, h.d_posed, s)))
            return hip_fail(e, "pose modules");
    }

    if (n_items > 0) {
        // --- slots
        int64_t worst_rec = 64, max_tiles = 1, max_mod = 1;
        int64_t worst_bins = 0;
        for (const HostJob& h : H) {
            if (h.n_items == 0) continue;
            const int64_t rec = 5 * h.tri_all + 64;
            worst_rec = std::max(worst_rec, rec);
            worst_bins = std::max(worst_bins, (int64_t)h.large_tiles * rec + h.g->n_mod * (int64_t)h.n_tiles);
            max_tiles = std::max<int64_t>(max_tiles, h.n_tiles);
            max_mod = std::max<int64_t>(max_mod, h.g->n_mod);
        }
        const int64_t rec_cap = std::min(worst_rec, c->batch_slot_records);
        const int64_t bin_cap = std::min(worst_bins, 8 * rec_cap + 64 * max_mod + 65536);
        const SlotGeom geo = slot_geom(rec_cap, bin_cap, max_tiles, max_mod);
        const uint64_t room = c->budget > c->used + B->slotmem.cap ? c->budget - c->used + B->slotmem.cap : 0;
        int64_t n_slots = std::min<int64_t>(std::min<int64_t>(n_items, c->batch_max_slots), (int64_t)(room / 2 / geo.slot_bytes));
        if (n_slots < 1) return fail(PV3D_ENOMEM, "one batch slot (%zu bytes) does not fit the HBM budget", geo.slot_bytes);
        const size_t ns = (size_t)n_slots;
        if ((st = B->slotmem.ensure(c, geo.slot_bytes * ns, "batch slots"))) return st;
        std::vector<PSlotBufs> slots;
        char* r_tc = carve_slots(static_cast<char*>(B->slotmem.ptr), geo, n_slots, slots);
        if ((e = hipMemsetAsync(r_tc, 0, geo.per_t * ns, s))) return hip_fail(e, "clear slot tile counts");

        // --- tables
        std::vector<PJob> pj((size_t)n_jobs);
        std::vector<PItem> items((size_t)n_items);
        int64_t k = 0;
        for (int64_t i = 0; i < n_jobs; i++) {
            const HostJob& h = H[(size_t)i];
            pj[(size_t)i] = make_pjob(h);
            for (int64_t t = 0; t < h.job.n_sun; t++)
                if (h.job.sun_xyz[3 * t + 2] > 0.0) items[(size_t)k++] = PItem{(int32_t)i, (int32_t)t};
        }
        std::vector<PSlotState> state(ns);
        memset(state.data(), 0, sizeof(PSlotState) * ns);
        for (size_t i = 0; i < ns; i++) {
            state[i].item = (int32_t)i;
            state[i].job = items[i].job;
            state[i].sun = items[i].sun;
            state[i].word = ((unsigned long long)kPhSetup << 56) | (1ull << 32);
        }
        PSched sched;
        memset(&sched, 0, sizeof(sched));
        sched.next_item = (uint32_t)ns;
        sched.n_items = (uint32_t)n_items;
        if ((st = B->slots.ensure(c, sizeof(PSlotBufs) * ns, "slot table"))) return st;
        if ((st = B->state.ensure(c, sizeof(PSlotState) * ns, "slot states"))) return st;
        if ((st = B->sched.ensure(c, sizeof(PSched), "scheduler"))) return st;
        if ((st = B->jobs.ensure(c, sizeof(PJob) * (size_t)n_jobs, "job table"))) return st;
        if ((st = B->items.ensure(c, sizeof(PItem) * (size_t)n_items, "item list"))) return st;
        if ((st = B->jobdone.ensure(c, 8 * (size_t)n_jobs, "job counters"))) return st;
        if ((st = B->overflow.ensure(c, 4 * (size_t)n_items, "overflow list"))) return st;
        const size_t tbytes = al256(sizeof(PSlotBufs) * ns) + al256(sizeof(PSlotState) * ns) + al256(sizeof(PSched)) +
                              al256(sizeof(PJob) * (size_t)n_jobs) + al256(sizeof(PItem) * (size_t)n_items) + 4096;
        if ((st = c->stage_reserve(tbytes))) return st;
        if ((st = c->stage(slots.data(), sizeof(PSlotBufs) * ns, B->slots.ptr, s))) return st;
        if ((st = c->stage(state.data(), sizeof(PSlotState) * ns, B->state.ptr, s))) return st;
        if ((st = c->stage(&sched, sizeof(PSched), B->sched.ptr, s))) return st;
        if ((st = c->stage(pj.data(), sizeof(PJob) * (size_t)n_jobs, B->jobs.ptr, s))) return st;
        if ((st = c->stage(items.data(), sizeof(PItem) * (size_t)n_items, B->items.ptr, s))) return st;
        if ((st = c->stage_done(s))) return st;
        if ((e = hipMemsetAsync(B->jobdone.ptr, 0, 8 * (size_t)n_jobs, s))) return hip_fail(e, "clear job counters");

        PLaunch P;
        memset(&P, 0, sizeof(P));
        P.jobs = static_cast<const PJob*>(B->jobs.ptr);
        P.items = static_cast<const PItem*>(B->items.ptr);
        P.slots = static_cast<const PSlotBufs*>(B->slots.ptr);
        P.state = static_cast<PSlotState*>(B->state.ptr);
        P.sched = static_cast<PSched*>(B->sched.ptr);
        P.job_done = static_cast<uint32_t*>(B->jobdone.ptr);
        P.job_overflow = reinterpret_cast<int32_t*>(static_cast<uint32_t*>(B->jobdone.ptr) + n_jobs);
        P.overflow_items = static_cast<int32_t*>(B->overflow.ptr);
        P.n_slots = (int32_t)n_slots;
        P.rec_cap = (int32_t)rec_cap;
        P.bin_cap = (int32_t)bin_cap;
        P.stall_ticks = D.stall_ticks;
        P.groups = c->batch_any_xcd ? 1 : D.xcd_groups;
        const int32_t grid = D.blocks_per_cu * D.n_cu;
        if ((e = hipEventRecord(B->ev0, s))) return hip_fail(e, "event");
        if ((e = launch_persist(P, grid, s))) return hip_fail(e, "persistent launch");
        if ((e = hipEventRecord(B->ev1, s))) return hip_fail(e, "event");
        PSched got;
        if ((e = hipMemcpyAsync(&got, B->sched.ptr, sizeof(PSched), hipMemcpyDeviceToHost, s))) return hip_fail(e, "read scheduler");
        if ((e = hipStreamSynchronize(s))) return hip_fail(e, "persistent launch");
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, B->ev0, B->ev1);
        if (got.abort) return fail(PV3D_EDEVICE, "persistent launch made no progress for %.0f s", kStallSeconds);
        if (got.items_done != (uint32_t)n_items)
            return fail(PV3D_EDEVICE, "persistent launch ended with %u of %lld items done", got.items_done, (long long)n_items);
        B->stats[0] = n_items;
        B->stats[1] = (int64_t)got.units;
        B->stats[2] = got.n_overflow;
        B->stats[3] = grid;
        B->stats[4] = n_slots;
        B->stats[5] = (int64_t)llround((double)ms * 1000.0);
        B->stats[6] = P.groups;

        // --- suns beyond a slot's capacity: the per-sun path, then the job's energy again
        if (got.n_overflow > 0) {
            std::vector<int32_t> ov(got.n_overflow);
            if ((e = hipMemcpyAsync(ov.data(), B->overflow.ptr, 4 * ov.size(), hipMemcpyDeviceToHost, s)) ||
                (e = hipStreamSynchronize(s)))
                return hip_fail(e, "read overflow list");
            std::vector<char> redo((size_t)n_jobs, 0);
            for (int32_t it : ov) {
                const PItem pi = items[(size_t)it];
                HostJob& h = H[(size_t)pi.job];
                const int64_t t = pi.sun;
                pv3d_params p1 = h.job.params;
                p1.tile = h.tile;
                if ((st = c->run_path(*h.sc, *h.g, p1, h.job.sun_xyz + 3 * t, 1, h.d_sun + 3 * t, h.d_dni + t, h.d_dpoa + t,
                                      h.d_dt + t, h.d_counts + t * h.cells, h.d_power + t, h.d_pref + t,
                                      static_cast<double*>(B->energy_tmp.ptr), nullptr, nullptr, s)))
                    return st;
                bool ovf = false;
                if ((st = c->read_overflow(1, s, &ovf))) return st;
                if (ovf) return fail(PV3D_ERANGE, "job %d, sun %lld overflows the per-sun path's buffers", pi.job, (long long)t);
                redo[(size_t)pi.job] = 1;
            }
            for (int64_t i = 0; i < n_jobs; i++)
                if (redo[(size_t)i]) {
                    const HostJob& h = H[(size_t)i];
                    if ((e = launch_energy(h.job.n_sun, h.d_power, h.d_pref, h.d_dt, h.d_energy, s))) return hip_fail(e, "energy");
                }
        }
    }

    // --- host outputs
    for (int64_t i = 0; i < n_jobs; i++) {
        const HostJob& h = H[(size_t)i];
        if (h.job.out.on_device) continue;
        const int64_t ns = h.job.n_sun;
        if (h.job.out.cell_counts && ns &&
            (e = hipMemcpyAsync(h.job.out.cell_counts, h.d_counts, 4 * (size_t)(ns * h.cells), hipMemcpyDeviceToHost, s)))
            return hip_fail(e, "copy counts");
        if (ns && (e = hipMemcpyAsync(h.job.out.power, h.d_power, 8 * (size_t)ns, hipMemcpyDeviceToHost, s))) return hip_fail(e, "copy power");
        if (ns && (e = hipMemcpyAsync(h.job.out.power_ref, h.d_pref, 8 * (size_t)ns, hipMemcpyDeviceToHost, s)))
            return hip_fail(e, "copy power_ref");
        if ((e = hipMemcpyAsync(h.job.out.energy, h.d_energy, 16, hipMemcpyDeviceToHost, s))) return hip_fail(e, "copy energy");
    }
    if ((e = hipStreamSynchronize(s))) return hip_fail(e, "synchronize");
    return PV3D_OK;
}

}  // namespace pv3d

extern "C" {

pv3d_status pv3d_evaluate_batched(pv3d_ctx* ctx, const pv3d_job* jobs, int64_t n_jobs, void* hip_stream) {
    if (!ctx) return fail(PV3D_EINVAL, "null context");
    if (n_jobs < 0 || (n_jobs > 0 && !jobs)) return fail(PV3D_EINVAL, "bad job list");
    if (n_jobs >= INT32_MAX) return fail(PV3D_ERANGE, "too many jobs");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    (void)hipSetDevice(ctx->device);
    hipStream_t s = hip_stream ? static_cast<hipStream_t>(hip_stream) : ctx->stream;
    ctx->stream_in_use = s;
    return run_batch(ctx, jobs, n_jobs, s);
}

}  // extern "C"

namespace pv3d {
// The autotuner's candidates: tile edges of the persistent launch, and bin limits.
constexpr int32_t kTuneTiles[2] = {32, 64};
constexpr int32_t kTuneLimits[6] = {8, 16, 32, 64, 128, 256};

static int32_t decade(int64_t n) {
    int32_t d = 0;
    for (int64_t v = std::max<int64_t>(n, 1); v >= 10; v /= 10) d++;
    return d;
}

// The class of a job: map size, samples per cell side, flags, and the decades of its
// triangles and cells.
static TuneKey tune_key(const pv3d_job& j, const HostJob& h) {
    return TuneKey{j.params.map_n, j.params.k, decade(h.tri_all), decade(h.cells), j.params.flags};
}
}  // namespace pv3d

extern "C" {

pv3d_status pv3d_autotune(pv3d_ctx* ctx, pv3d_job* job, int32_t n_probe, double* best_ms_out) {
    if (!ctx || !job) return fail(PV3D_EINVAL, "null argument");
    if (n_probe < 1) return fail(PV3D_EINVAL, "n_probe %d < 1", n_probe);
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    (void)hipSetDevice(ctx->device);
    HostJob h;
    ctx->stream_in_use = ctx->stream;
    pv3d_status st;
    if ((st = check_job(ctx, *job, 0, h, true))) return st;
    const TuneKey key = tune_key(*job, h);
    auto hit = ctx->tune_cache.find(key);
    if (hit != ctx->tune_cache.end()) {
        job->params.tile = hit->second.tile;
        job->params.bin_limit = hit->second.bin_limit;
        if (best_ms_out) *best_ms_out = hit->second.ms;
        return PV3D_OK;
    }
    // probe suns: evenly spaced among those above the horizon
    std::vector<int64_t> up;
    for (int64_t t = 0; t < job->n_sun; t++)
        if (job->sun_xyz[3 * t + 2] > 0.0) up.push_back(t);
    const int64_t np = std::min<int64_t>(n_probe, (int64_t)up.size());
    if (np == 0) {
        if (best_ms_out) *best_ms_out = 0.0;
        return PV3D_OK;                              // nothing to time: keep the job's params
    }
    std::vector<double> sun(3 * (size_t)np), dni((size_t)np), dp((size_t)np), dt((size_t)np);
    for (int64_t q = 0; q < np; q++) {
        const int64_t t = up[(size_t)((q * (int64_t)up.size()) / np)];
        for (int c = 0; c < 3; c++) sun[(size_t)(3 * q + c)] = job->sun_xyz[3 * t + c];
        dni[(size_t)q] = job->dni[t];
        dp[(size_t)q] = job->d_poa[t];
        dt[(size_t)q] = job->dt_h[t];
    }
    std::vector<uint32_t> counts((size_t)(np * h.cells));
    std::vector<double> pw((size_t)np), pr((size_t)np), en(2);
    pv3d_job probe = *job;
    probe.sun_xyz = sun.data();
    probe.dni = dni.data();
    probe.d_poa = dp.data();
    probe.dt_h = dt.data();
    probe.n_sun = np;
    probe.out.cell_counts = nullptr;
    probe.out.power = pw.data();
    probe.out.power_ref = pr.data();
    probe.out.energy = en.data();
    probe.out.depth_maps = nullptr;
    probe.out.shaded_bits = nullptr;
    probe.out.on_device = 0;
    double best = INFINITY;
    int32_t bt = 64, bl = kMaxBinLimit;
    for (int32_t tile : kTuneTiles)
        for (int32_t lim : kTuneLimits) {
            probe.params.tile = tile;
            probe.params.bin_limit = lim;
            if ((st = run_batch(ctx, &probe, 1, ctx->stream))) return st;     // warm
            if ((st = run_batch(ctx, &probe, 1, ctx->stream))) return st;
            const double ms = (double)ctx->batch->stats[5] / 1000.0;
            if (ms < best) {
                best = ms;
                bt = tile;
                bl = lim;
            }
        }
    job->params.tile = bt;
    job->params.bin_limit = bl;
    ctx->tune_cache[key] = TuneChoice{bt, bl, best};
    if (best_ms_out) *best_ms_out = best;
    return PV3D_OK;
}

pv3d_status pv3d_autotune_cache(pv3d_ctx* ctx, const char* path, int32_t mode) {
    if (!ctx) return fail(PV3D_EINVAL, "null context");
    if (mode != PV3D_TUNE_LOAD && mode != PV3D_TUNE_SAVE && mode != PV3D_TUNE_CLEAR)
        return fail(PV3D_EINVAL, "unknown cache mode %d", mode);
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (mode == PV3D_TUNE_CLEAR) {
        ctx->tune_cache.clear();
        return PV3D_OK;
    }
    if (!path) return fail(PV3D_EINVAL, "null path");
    if (mode == PV3D_TUNE_SAVE) {
        FILE* f = fopen(path, "w");
        if (!f) return fail(PV3D_ENOENT, "cannot open %s for writing", path);
        fprintf(f, "[\n");
        size_t i = 0;
        for (const auto& kv : ctx->tune_cache) {
            const TuneKey& k = kv.first;
            const TuneChoice& c = kv.second;
            fprintf(f, "  {\"map_n\": %d, \"k\": %d, \"flags\": %u, \"tri_decade\": %d, \"cell_decade\": %d, "
                       "\"tile\": %d, \"bin_limit\": %d, \"ms\": %.17g}%s\n",
                    k.map_n, k.k, k.flags, k.tri_decade, k.cell_decade, c.tile, c.bin_limit, c.ms,
                    ++i < ctx->tune_cache.size() ? "," : "");
        }
        fprintf(f, "]\n");
        const bool bad = ferror(f) != 0;
        if (fclose(f) != 0 || bad) return fail(PV3D_ENOENT, "writing %s failed", path);
        return PV3D_OK;
    }
    FILE* f = fopen(path, "r");
    if (!f) return fail(PV3D_ENOENT, "cannot open %s", path);
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
    fclose(f);
    // the objects of the array, in the layout PV3D_TUNE_SAVE writes (any spacing)
    std::map<TuneKey, TuneChoice> add;
    size_t at = text.find('[');
    if (at == std::string::npos) return fail(PV3D_EINVAL, "%s: no JSON array", path);
    for (;;) {
        const size_t open = text.find('{', at), close = text.find('}', at);
        if (open == std::string::npos) break;
        if (close == std::string::npos || close < open) return fail(PV3D_EINVAL, "%s: unbalanced object", path);
        const std::string obj = text.substr(open, close - open + 1);
        auto field = [&](const char* name, double* v) {
            const std::string pat = std::string("\"") + name + "\"";
            const size_t p = obj.find(pat);
            if (p == std::string::npos) return false;
            const size_t colon = obj.find(':', p + pat.size());
            if (colon == std::string::npos) return false;
            char* end = nullptr;
            *v = strtod(obj.c_str() + colon + 1, &end);
            return end != obj.c_str() + colon + 1 && std::isfinite(*v);
        };
        double v[8];
        const char* names[8] = {"map_n", "k", "flags", "tri_decade", "cell_decade", "tile", "bin_limit", "ms"};
        for (int i = 0; i < 8; i++)
            if (!field(names[i], &v[i])) return fail(PV3D_EINVAL, "%s: an entry lacks \"%s\"", path, names[i]);
        TuneKey key{(int32_t)v[0], (int32_t)v[1], (int32_t)v[3], (int32_t)v[4], (uint32_t)v[2]};
        TuneChoice c{(int32_t)v[5], (int32_t)v[6], v[7]};
        const bool tile_ok = std::find(std::begin(kTuneTiles), std::end(kTuneTiles), c.tile) != std::end(kTuneTiles);
        const bool lim_ok =
            std::find(std::begin(kTuneLimits), std::end(kTuneLimits), c.bin_limit) != std::end(kTuneLimits);
        if (!tile_ok || !lim_ok || key.map_n < 16 || key.map_n > 16384 || key.k < 1 || key.k > 255 || c.ms < 0.0)
            return fail(PV3D_EINVAL, "%s: an entry holds values outside the autotuner's candidates", path);
        add[key] = c;
        at = close + 1;
    }
    for (const auto& kv : add) ctx->tune_cache[kv.first] = kv.second;
    return PV3D_OK;
}

pv3d_status pv3d_batch_limits(pv3d_ctx* ctx, int32_t max_slots, int64_t slot_records, uint32_t flags) {
    if (!ctx) return fail(PV3D_EINVAL, "null context");
    if (max_slots < 0 || max_slots > 4096 || slot_records < 0 || slot_records > INT32_MAX / 8)
        return fail(PV3D_EINVAL, "batch limits out of range");
    if (flags & ~PV3D_BATCH_ANY_XCD) return fail(PV3D_EINVAL, "unknown batch flags 0x%x", flags);
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    ctx->batch_max_slots = max_slots ? max_slots : kMaxSlots;
    ctx->batch_slot_records = slot_records ? slot_records : kSlotRecCap;
    ctx->batch_any_xcd = (flags & PV3D_BATCH_ANY_XCD) != 0;
    return PV3D_OK;
}

pv3d_status pv3d_batch_stats(pv3d_ctx* ctx, int64_t out[7]) {
    if (!ctx || !out) return fail(PV3D_EINVAL, "null argument");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    for (int i = 0; i < 7; i++) out[i] = ctx->batch ? ctx->batch->stats[i] : 0;
    return PV3D_OK;
}

}  // extern "C"
