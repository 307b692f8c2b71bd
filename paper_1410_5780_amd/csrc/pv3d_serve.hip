// Serving loop of libpv3d: jobs submitted at any time share one live
// persistent launch (k_persist in serving mode), so work that arrives while
// other jobs are on the GPU starts as soon as a slot and memory are free.
//
// A service thread per context:
//   - admits pending jobs in submission order while their data fits the job
//     arena (the HBM budget of the loop), a job-table entry is free and the
//     item feed has room: uploads the job's sweep and constants with the copy
//     engine, writes its table entry, then publishes one item per sun in the
//     feed (host memory the kernel reads);
//   - keeps a live launch running while items are in flight (the launch
//     ends by itself after a short idle time and is started again when work
//     comes back);
//   - watches the completion tags the kernel writes into host memory,
//     copies host outputs back, and frees the job's memory.
// Nothing here allocates or frees device memory while a launch runs: the
// arena, the slots and the tables are taken once, when the loop starts.
// The thread never holds the server lock while it waits for the device, so
// submit, poll, wait and cancel never queue behind a copy. Its copies run on
// the context's lane-1 stream and the launch on a stream of its own, so that
// the launch holds a hardware queue no other work of the library waits in.
// While a HoldServing lives (another thread is about to wait for the whole
// device) no job is admitted, so the live launch runs out of work and ends.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/pv3d.h"
#include "pv3d_batch.h"
#include "pv3d_device.h"
#include "pv3d_runtime.h"

using namespace pv3d;

namespace pv3d {

constexpr int32_t kServeJobs = 1024;          // jobs in flight (job-table entries)
constexpr uint32_t kFeedCap = 1u << 20;       // items in flight
constexpr size_t kMaxPending = 1u << 16;      // submitted, not yet admitted
constexpr int32_t kServeSlots = 64;           // items on the device at once
constexpr int32_t kServeMaxMod = 4096;        // modules per job
constexpr int32_t kServeMaxTiles = 65536;     // raster tiles per job
constexpr double kIdleSeconds = 0.002;        // a live launch with nothing to do ends after this

enum SState { kPending, kLive, kDone, kCancelled, kFailed };

// First-fit allocator over the job arena.
struct Arena {
    size_t cap = 0;
    std::map<size_t, size_t> free_;           // offset -> bytes
    void reset(size_t c) {
        cap = c;
        free_.clear();
        if (c) free_[0] = c;
    }
    bool alloc(size_t bytes, size_t* off) {
        bytes = al256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                return true;
            }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = al256(bytes);
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct SJob {
    uint64_t ticket = 0;
    uint64_t scene = 0, gen = 0;
    HostJob h;                      // h.job: the caller's job, inputs redirected to `in`
    std::vector<double> in;         // owned copy of sun_xyz, dni, d_poa, dt_h
    SState state = kPending;
    pv3d_status result = PV3D_OK;
    bool cancel = false;
    int32_t jslot = -1;
    uint32_t seq = 0;
    size_t off = 0, bytes = 0;
};

struct Server {
    Ctx* c = nullptr;
    std::thread th;
    std::mutex mu;
    std::condition_variable cv, cv_done;
    bool quit = false;
    int32_t hold = 0;                // HoldServing guards alive: admit nothing
    std::deque<SJob*> pending;
    std::map<uint64_t, std::unique_ptr<SJob>> jobs;
    std::map<uint64_t, int32_t> users;       // scene / generator handle -> jobs that read it
    uint64_t next_ticket = 1;
    pv3d_status fatal = PV3D_OK;
    // device side
    hipStream_t kstream = nullptr;   // the persistent launch
    hipStream_t cstream = nullptr;   // copies: the context's lane-1 stream, not owned
    hipEvent_t kdone = nullptr;
    bool live = false;
    Buf arena_mem, slotmem, slotbufs, state, sched, jobtab, counters;
    Arena arena;
    SlotGeom geo{};
    int32_t n_slots = 0;
    DevInfo dev;
    // host memory the kernel reads and writes
    unsigned long long* feed = nullptr;
    uint32_t* pub = nullptr;
    uint32_t* stop = nullptr;
    uint32_t* report = nullptr;
    void* host_mem = nullptr;
    void* staging = nullptr;           // pinned: job uploads and output bounce
    void* staging_dev = nullptr;       // its device address
    size_t staging_cap = 0;
    uint32_t published = 0;
    int64_t inflight_items = 0;
    std::vector<int32_t> free_jslots;
    std::vector<uint32_t> done_base, ovf_base;
    std::vector<SJob*> slot_job;
    uint32_t next_seq = 1;
    int64_t stats_launches = 0, stats_done = 0, stats_items = 0;
};

static void use(Server* S, uint64_t h, int32_t d) {
    S->users[h] += d;
    if (S->users[h] <= 0) S->users.erase(h);
}

bool Ctx::scene_in_use(uint64_t h) {
    if (!server) return false;
    std::lock_guard<std::mutex> lk(server->mu);
    auto it = server->users.find(h);
    return it != server->users.end() && it->second > 0;
}
bool Ctx::gen_in_use(uint64_t h) { return scene_in_use(h); }

// Start the loop: slots, tables, the job arena (half of the budget left),
// host memory for the feed and the tags, streams, the service thread.
static pv3d_status start_server(Ctx* c);
static void service(Server* S);

static void free_server(Ctx* c, Server* S) {
    Buf* all[] = {&S->arena_mem, &S->slotmem, &S->slotbufs, &S->state, &S->sched, &S->jobtab, &S->counters};
    for (Buf* b : all) b->release(c);
    if (S->host_mem) (void)hipHostFree(S->host_mem);
    if (S->staging) (void)hipHostFree(S->staging);
    if (S->kdone) (void)hipEventDestroy(S->kdone);
    if (S->kstream) (void)hipStreamDestroy(S->kstream);
    delete S;
}

static pv3d_status start_server_parts(Ctx* c, Server* S);

static pv3d_status start_server(Ctx* c) {
    if (c->server) return PV3D_OK;
    Server* S = new Server();
    S->c = c;
    pv3d_status st = start_server_parts(c, S);
    if (st) {
        free_server(c, S);
        return st;
    }
    c->server = S;
    S->th = std::thread(service, S);
    return PV3D_OK;
}

static pv3d_status start_server_parts(Ctx* c, Server* S) {
    pv3d_status st;
    if ((st = device_info(c, &S->dev))) return st;
    hipError_t e;
    {
        // The persistent kernel's stream takes a hardware queue of its own (a stream made
        // with a CU mask always does; this one enables every CU). Beyond the few queues a
        // process gets, streams share queues, and a stream whose queue holds a live launch
        // waits behind it: the loop's copy stream landing there made every admission wait
        // for the launch to run dry (copies of up to 2 s, request rates down to 2 per s).
        std::vector<uint32_t> mask((size_t)(c->n_cu + 31) / 32, 0u);
        for (int32_t i = 0; i < c->n_cu; i++) mask[(size_t)i / 32] |= 1u << (i % 32);
        if ((e = hipExtStreamCreateWithCUMask(&S->kstream, (uint32_t)mask.size(), mask.data())))
            return hip_fail(e, "hipExtStreamCreateWithCUMask");
    }
    S->cstream = c->lane_st[kLanes - 1];
    if (!S->cstream) return fail(PV3D_EDEVICE, "the context has no copy stream for the serving loop");
    if ((e = hipEventCreateWithFlags(&S->kdone, hipEventDisableTiming))) return hip_fail(e, "hipEventCreate");
    const int64_t rec_cap = c->batch_slot_records;
    const int64_t bin_cap = 8 * rec_cap + 64 * (int64_t)kServeMaxMod + 65536;
    S->geo = slot_geom(rec_cap, bin_cap, kServeMaxTiles, kServeMaxMod);
    const uint64_t room = c->budget > c->used ? c->budget - c->used : 0;
    S->n_slots = (int32_t)std::min<int64_t>(std::min<int64_t>(kServeSlots, c->batch_max_slots),
                                            (int64_t)(room / 4 / S->geo.slot_bytes));
    if (S->n_slots < 1) return fail(PV3D_ENOMEM, "the serving loop's slots do not fit the HBM budget");
    const size_t ns = (size_t)S->n_slots;
    if ((st = S->slotmem.ensure(c, S->geo.slot_bytes * ns, "serving slots"))) return st;
    std::vector<PSlotBufs> slots;
    char* r_tc = carve_slots(static_cast<char*>(S->slotmem.ptr), S->geo, S->n_slots, slots);
    if ((st = S->slotbufs.ensure(c, sizeof(PSlotBufs) * ns, "slot table"))) return st;
    if ((st = S->state.ensure(c, sizeof(PSlotState) * ns, "slot states"))) return st;
    if ((st = S->sched.ensure(c, sizeof(PSched), "scheduler"))) return st;
    if ((st = S->jobtab.ensure(c, sizeof(PJob) * kServeJobs, "job table"))) return st;
    if ((st = S->counters.ensure(c, 8 * kServeJobs, "job counters"))) return st;
    if ((e = hipMemsetAsync(r_tc, 0, S->geo.per_t * ns, S->cstream))) return hip_fail(e, "clear tile counts");
    if ((e = hipMemsetAsync(S->state.ptr, 0, sizeof(PSlotState) * ns, S->cstream))) return hip_fail(e, "clear slots");
    if ((e = hipMemsetAsync(S->sched.ptr, 0, sizeof(PSched), S->cstream))) return hip_fail(e, "clear scheduler");
    if ((e = hipMemsetAsync(S->counters.ptr, 0, 8 * kServeJobs, S->cstream))) return hip_fail(e, "clear counters");
    if ((e = hipMemcpyAsync(S->slotbufs.ptr, slots.data(), sizeof(PSlotBufs) * ns, hipMemcpyHostToDevice, S->cstream)))
        return hip_fail(e, "slot table");
    if ((e = hipStreamSynchronize(S->cstream))) return hip_fail(e, "serving set-up");
    const uint64_t left = c->budget > c->used ? c->budget - c->used : 0;
    const size_t arena_bytes = (size_t)(left / 2) & ~(size_t)255;
    if (arena_bytes < (1u << 20)) return fail(PV3D_ENOMEM, "no HBM budget left for the serving loop's job data");
    if ((st = S->arena_mem.ensure(c, arena_bytes, "serving job arena"))) return st;
    S->arena.reset(arena_bytes);
    // host memory shared with the kernel: feed ring, published count, stop flag, tags
    const size_t hbytes = 8 * (size_t)kFeedCap + 256 + 256 + 4 * (size_t)kServeJobs;
    if ((e = hipHostMalloc(&S->host_mem, hbytes, hipHostMallocCoherent | hipHostMallocMapped)))
        return hip_fail(e, "hipHostMalloc");
    memset(S->host_mem, 0, hbytes);
    char* hp = static_cast<char*>(S->host_mem);
    S->feed = reinterpret_cast<unsigned long long*>(hp);
    S->pub = reinterpret_cast<uint32_t*>(hp + 8 * (size_t)kFeedCap);
    S->stop = reinterpret_cast<uint32_t*>(hp + 8 * (size_t)kFeedCap + 256);
    S->report = reinterpret_cast<uint32_t*>(hp + 8 * (size_t)kFeedCap + 512);
    S->free_jslots.clear();
    for (int32_t j = kServeJobs - 1; j >= 0; j--) S->free_jslots.push_back(j);
    S->done_base.assign(kServeJobs, 0);
    S->ovf_base.assign(kServeJobs, 0);
    S->slot_job.assign(kServeJobs, nullptr);
    return PV3D_OK;
}

static void* dev_ptr(void* host) {
    void* d = nullptr;
    if (hipHostGetDevicePointer(&d, host, 0) != hipSuccess) return host;
    return d;
}

// Copies of the loop go through the copy engines (no compute unit): the live
// launch holds every CU, and a copy done by a kernel would wait for it to end.
// Host memory takes part through the device address of pinned staging.
static hipError_t copy_nocu(void* dst, const void* src, size_t bytes, hipStream_t st) {
    if (bytes == 0) return hipSuccess;
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDeviceNoCU, st);
}

static pv3d_status ensure_staging(Server* S, size_t need) {
    if (need <= S->staging_cap) return PV3D_OK;
    if (S->staging) (void)hipHostFree(S->staging);
    S->staging = nullptr;
    S->staging_dev = nullptr;
    S->staging_cap = 0;
    const size_t cap = std::max(need + need / 2, (size_t)64 << 20);   // rarely regrown: a free may wait for the device
    hipError_t e = hipHostMalloc(&S->staging, cap, hipHostMallocDefault);
    if (e) return hip_fail(e, "hipHostMalloc staging");
    S->staging_dev = dev_ptr(S->staging);
    S->staging_cap = cap;
    return PV3D_OK;
}

// Upload a job and publish its items (server lock held on entry and on
// return, released while the copies run). False: it has to wait, or *err
// says why it failed.
static bool try_admit(Server* S, std::unique_lock<std::mutex>& lk, SJob* J, pv3d_status* err) {
    HostJob& h = J->h;
    const int64_t ns = h.job.n_sun;
    if (S->free_jslots.empty()) return false;
    if (S->inflight_items + ns > (int64_t)kFeedCap) return false;
    const bool dev_out = h.job.out.on_device != 0;
    const bool own_counts = !dev_out || !h.job.out.cell_counts;
    const size_t bytes = job_bytes(h, own_counts, !dev_out);
    size_t off = 0;
    if (!S->arena.alloc(bytes, &off)) return false;
    J->off = off;
    J->bytes = bytes;
    carve_job(h, static_cast<char*>(S->arena_mem.ptr) + off, own_counts, !dev_out);
    if (!own_counts) h.d_counts = h.job.out.cell_counts;
    if (dev_out) {
        h.d_power = h.job.out.power;
        h.d_pref = h.job.out.power_ref;
        h.d_energy = h.job.out.energy;
    }
    const int32_t j = S->free_jslots.back();
    S->free_jslots.pop_back();
    J->jslot = j;
    J->seq = S->next_seq++ & 0x7FFFFFFFu;
    if (J->seq == 0) J->seq = S->next_seq++ & 0x7FFFFFFFu;
    // staging: sweep, sphere, tables, and the job-table entry
    std::vector<double> tab;
    job_constants(h, tab);
    const int32_t kk = h.job.params.k;
    const size_t need = 48 * (size_t)ns + 8 * tab.size() + sizeof(PJob) + 1024;
    PJob pj = make_pjob(h);
    pj.n_items = (int32_t)ns;                           // every sun is an item: below the horizon it only writes zeros
    pj.done_target = S->done_base[(size_t)j] + (uint32_t)ns;
    pj.ovf_base = S->ovf_base[(size_t)j];
    pj.seq = J->seq;
    // only this thread touches the staging buffer and the reserved arena block
    lk.unlock();
    hipError_t e = hipSuccess;
    pv3d_status st = ensure_staging(S, need);
    if (!st) {
        char* sp = static_cast<char*>(S->staging);
        char* sd = static_cast<char*>(S->staging_dev);
        memcpy(sp, J->in.data(), 48 * (size_t)ns);          // sun (3 ns), dni, d_poa, dt: the device layout
        char* tp = sp + al256(48 * (size_t)ns);
        memcpy(tp, tab.data(), 8 * tab.size());
        char* jp = tp + al256(8 * tab.size());
        memcpy(jp, &pj, sizeof(PJob));
        const size_t to = (size_t)(tp - sp), jo = (size_t)(jp - sp);
        if (ns > 0) e = copy_nocu(h.d_sun, sd, 48 * (size_t)ns, S->cstream);
        if (!e) e = copy_nocu(h.d_sphere, sd + to, 32, S->cstream);
        if (!e) e = copy_nocu(h.d_fu, sd + to + 32, 8 * (size_t)kk * h.g->n_cu, S->cstream);
        if (!e) e = copy_nocu(h.d_fv, sd + to + 32 + 8 * (size_t)kk * h.g->n_cu, 8 * (size_t)kk * h.g->n_cv, S->cstream);
        if (!e) e = copy_nocu(static_cast<PJob*>(S->jobtab.ptr) + j, sd + jo, sizeof(PJob), S->cstream);
        if (!e) e = hipStreamSynchronize(S->cstream);
        if (e) st = hip_fail(e, "upload of a serving job");
    }
    lk.lock();
    if (st) {
        S->arena.release(J->off, J->bytes);
        S->free_jslots.push_back(j);
        J->jslot = -1;
        *err = st;
        return false;
    }
    if (ns == 0) {           // nothing to evaluate: zero energy
        J->state = kLive;
        S->slot_job[(size_t)j] = J;
        return true;
    }
    for (int64_t t = 0; t < ns; t++)
        S->feed[(S->published + (uint32_t)t) % kFeedCap] = ((unsigned long long)(uint32_t)j << 32) | (uint32_t)t;
    S->published += (uint32_t)ns;
    __atomic_store_n(S->pub, S->published, __ATOMIC_RELEASE);
    S->inflight_items += ns;
    S->stats_items += ns;
    J->state = kLive;
    S->slot_job[(size_t)j] = J;
    return true;
}

// A job's tag came back (server lock held by the caller; released while the
// device is waited for, and around work that needs the context).
static void finish(Server* S, std::unique_lock<std::mutex>& lk, SJob* J, bool overflow) {
    HostJob& h = J->h;
    const int64_t ns = h.job.n_sun;
    const int32_t j = J->jslot;
    pv3d_status st = PV3D_OK;
    hipError_t e = hipSuccess;
    const bool cancelled = J->cancel;    // host outputs of a cancelled job are not written
    lk.unlock();                     // J stays live until this returns: no other thread frees it
    if (ns == 0) {
        static const double zero[2] = {0.0, 0.0};
        if (h.job.out.on_device) {
            if ((st = ensure_staging(S, 16)) == PV3D_OK) {
                memcpy(S->staging, zero, 16);
                e = copy_nocu(h.job.out.energy, S->staging_dev, 16, S->cstream);
                if (!e) e = hipStreamSynchronize(S->cstream);
            }
        } else {
            memcpy(h.job.out.energy, zero, 16);
        }
    } else if (overflow) {
        // suns that exceeded a slot's capacity (their power marked NaN by the kernel): the
        // per-sun path evaluates each of them again, one sun per call, and the job's energy
        // is summed again
        std::lock_guard<std::recursive_mutex> cl(S->c->mu);
        S->c->stream_in_use = S->cstream;
        pv3d_params p1 = h.job.params;
        p1.tile = h.tile;
        std::vector<double> pw((size_t)ns);
        if ((st = ensure_staging(S, 8 * (size_t)ns)) == PV3D_OK) {
            e = copy_nocu(S->staging_dev, h.d_power, 8 * (size_t)ns, S->cstream);
            if (!e) e = hipStreamSynchronize(S->cstream);
            if (!e) memcpy(pw.data(), S->staging, 8 * (size_t)ns);
        }
        for (int64_t t = 0; t < ns && !st && !e; t++) {
            if (!std::isnan(pw[(size_t)t])) continue;
            st = S->c->run_path(*h.sc, *h.g, p1, h.job.sun_xyz + 3 * t, 1, h.d_sun + 3 * t, h.d_dni + t,
                                h.d_dpoa + t, h.d_dt + t, h.d_counts + t * h.cells, h.d_power + t, h.d_pref + t,
                                h.d_energy, nullptr, nullptr, S->cstream);
            bool ovf = false;
            if (!st) st = S->c->read_overflow(1, S->cstream, &ovf);
            if (!st && ovf) st = fail(PV3D_ERANGE, "a sun of a serving job overflows the per-sun path's buffers");
        }
        if (!st && !e) e = launch_energy(ns, h.d_power, h.d_pref, h.d_dt, h.d_energy, S->cstream);
        if (!st && !e) e = hipStreamSynchronize(S->cstream);
        uint32_t ov = 0;
        if (!st && !e && (st = ensure_staging(S, 4)) == PV3D_OK) {
            e = copy_nocu(S->staging_dev, static_cast<uint32_t*>(S->counters.ptr) + kServeJobs + j, 4, S->cstream);
            if (!e) e = hipStreamSynchronize(S->cstream);
            if (!e) memcpy(&ov, S->staging, 4);
        }
        if (!st && !e) S->ovf_base[(size_t)j] = ov;
    }
    if (!st && !e && !h.job.out.on_device && ns > 0 && !cancelled) {
        // one copy of the job's output region (counts, powers, energy lie in this order) into
        // pinned staging, then into the caller's arrays
        const char* first = h.job.out.cell_counts ? reinterpret_cast<const char*>(h.d_counts)
                                                  : reinterpret_cast<const char*>(h.d_power);
        const size_t span = (size_t)(reinterpret_cast<const char*>(h.d_energy) + 16 - first);
        if ((st = ensure_staging(S, span)) == PV3D_OK) {
            e = copy_nocu(S->staging_dev, first, span, S->cstream);
            if (!e) e = hipStreamSynchronize(S->cstream);
            if (!e) {
                const char* b = static_cast<const char*>(S->staging);
                auto at = [&](const void* dev) { return b + (reinterpret_cast<const char*>(dev) - first); };
                if (h.job.out.cell_counts) memcpy(h.job.out.cell_counts, at(h.d_counts), 4 * (size_t)(ns * h.cells));
                memcpy(h.job.out.power, at(h.d_power), 8 * (size_t)ns);
                memcpy(h.job.out.power_ref, at(h.d_pref), 8 * (size_t)ns);
                memcpy(h.job.out.energy, at(h.d_energy), 16);
            }
        }
    }
    lk.lock();
    if (e) st = hip_fail(e, "serving outputs");
    S->arena.release(J->off, J->bytes);
    S->done_base[(size_t)j] += (uint32_t)ns;
    S->slot_job[(size_t)j] = nullptr;
    S->free_jslots.push_back(j);
    S->inflight_items -= ns;
    use(S, J->scene, -1);
    use(S, J->gen, -1);
    J->result = st;
    J->state = J->cancel ? kCancelled : (st ? kFailed : kDone);
    S->stats_done++;
    S->cv_done.notify_all();
}

static void fail_live(Server* S, pv3d_status code) {
    for (int32_t j = 0; j < kServeJobs; j++) {
        SJob* J = S->slot_job[(size_t)j];
        if (!J) continue;
        J->result = code;
        J->state = kFailed;
        use(S, J->scene, -1);
        use(S, J->gen, -1);
        S->slot_job[(size_t)j] = nullptr;
    }
    S->cv_done.notify_all();
}

static bool any_live(Server* S) {
    for (SJob* J : S->slot_job)
        if (J) return true;
    return false;
}

static void service(Server* S) {
    (void)hipSetDevice(S->c->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        // 1. finished jobs
        for (int32_t j = 0; j < kServeJobs; j++) {
            SJob* J = S->slot_job[(size_t)j];
            if (!J) continue;
            bool done = J->h.job.n_sun == 0;
            bool ovf = false;
            if (!done) {
                const uint32_t tag = __atomic_load_n(S->report + j, __ATOMIC_ACQUIRE);
                done = (tag & 0x7FFFFFFFu) == J->seq;
                ovf = (tag >> 31) != 0;
            }
            if (done) finish(S, lk, J, ovf);
        }
        // 2. the launch ended: check it, and start another while items are in flight
        const hipError_t q = S->live ? hipEventQuery(S->kdone) : hipErrorNotReady;
        if (S->live && q != hipErrorNotReady) {
            S->live = false;
            PSched got;
            memset(&got, 0, sizeof(got));
            lk.unlock();
            bool ok = q == hipSuccess && ensure_staging(S, sizeof(PSched)) == PV3D_OK &&
                      copy_nocu(S->staging_dev, S->sched.ptr, sizeof(PSched), S->cstream) == hipSuccess &&
                      hipStreamSynchronize(S->cstream) == hipSuccess;
            if (ok) memcpy(&got, S->staging, sizeof(PSched));
            lk.lock();
            if (!ok || got.abort) {
                S->fatal = fail(PV3D_EDEVICE, "the serving launch stopped making progress");
                fail_live(S, S->fatal);
            }
            continue;                        // look at the tags once more before starting again
        }
        // 3. admissions, in submission order (none while a HoldServing lives)
        while (!S->pending.empty() && !S->fatal && S->hold == 0) {
            SJob* J = S->pending.front();
            if (J->cancel) {
                S->pending.pop_front();
                J->state = kCancelled;
                use(S, J->scene, -1);
                use(S, J->gen, -1);
                S->cv_done.notify_all();
                continue;
            }
            pv3d_status err = PV3D_OK;
            if (!try_admit(S, lk, J, &err)) {
                if (err) {
                    S->pending.pop_front();
                    J->result = err;
                    J->state = kFailed;
                    use(S, J->scene, -1);
                    use(S, J->gen, -1);
                    S->cv_done.notify_all();
                    continue;
                }
                break;
            }
            S->pending.pop_front();
        }
        if (S->fatal) {
            while (!S->pending.empty()) {
                SJob* J = S->pending.front();
                S->pending.pop_front();
                J->result = S->fatal;
                J->state = kFailed;
                use(S, J->scene, -1);
                use(S, J->gen, -1);
            }
            S->cv_done.notify_all();
        }
        const bool inflight = S->inflight_items > 0;
        if (!S->live && inflight && !S->fatal) {
            PLaunch P;
            memset(&P, 0, sizeof(P));
            P.jobs = static_cast<const PJob*>(S->jobtab.ptr);
            P.items = nullptr;
            P.slots = static_cast<const PSlotBufs*>(S->slotbufs.ptr);
            P.state = static_cast<PSlotState*>(S->state.ptr);
            P.sched = static_cast<PSched*>(S->sched.ptr);
            P.job_done = static_cast<uint32_t*>(S->counters.ptr);
            P.job_overflow = reinterpret_cast<int32_t*>(static_cast<uint32_t*>(S->counters.ptr) + kServeJobs);
            P.overflow_items = nullptr;
            P.n_slots = S->n_slots;
            P.rec_cap = (int32_t)S->geo.rec_cap;
            P.bin_cap = (int32_t)S->geo.bin_cap;
            P.groups = S->c->batch_any_xcd ? 1 : S->dev.xcd_groups;
            P.stall_ticks = S->dev.stall_ticks;
            P.serve = 1;
            P.feed_cap = kFeedCap;
            P.feed = static_cast<const unsigned long long*>(dev_ptr(S->feed));
            P.feed_pub = static_cast<const uint32_t*>(dev_ptr(S->pub));
            P.stop_flag = static_cast<const uint32_t*>(dev_ptr(S->stop));
            P.report = static_cast<uint32_t*>(dev_ptr(S->report));
            P.idle_ticks = (long long)(kIdleSeconds * 1000.0 * (double)S->dev.rate_khz);
            hipError_t e = launch_persist(P, S->dev.blocks_per_cu * S->dev.n_cu, S->kstream);
            if (!e) e = hipEventRecord(S->kdone, S->kstream);
            if (e) {
                S->fatal = hip_fail(e, "serving launch");
                fail_live(S, S->fatal);
            } else {
                S->live = true;
                S->stats_launches++;
            }
        }
        if (S->quit && S->pending.empty() && !any_live(S) && !S->live) break;
        if (!inflight && !S->live && S->pending.empty() && !S->quit) {
            S->cv.wait(lk);
        } else {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(50));
            lk.lock();
        }
    }
}

HoldServing::HoldServing(Ctx* ctx) : c(ctx) {
    Server* S = c->server;
    if (!S) {
        c = nullptr;
        return;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    S->hold++;
}

HoldServing::~HoldServing() {
    if (!c || !c->server) return;
    Server* S = c->server;
    std::lock_guard<std::mutex> lk(S->mu);
    S->hold--;
    S->cv.notify_all();
}

}  // namespace pv3d

void pv3d_server_stop(pv3d_ctx* ctx) {
    Server* S = ctx->server;
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->quit = true;
        for (SJob* J : S->pending) J->cancel = true;
        __atomic_store_n(S->stop, 1u, __ATOMIC_RELEASE);
        S->cv.notify_all();
    }
    if (S->th.joinable()) S->th.join();
    (void)hipStreamSynchronize(S->kstream);
    (void)hipStreamSynchronize(S->cstream);
    ctx->server = nullptr;
    free_server(ctx, S);
}

extern "C" {

pv3d_status pv3d_submit(pv3d_ctx* ctx, const pv3d_job* job, uint64_t* ticket) {
    if (!ctx || !job || !ticket) return fail(PV3D_EINVAL, "null argument");
    std::lock_guard<std::recursive_mutex> cl(ctx->mu);
    (void)hipSetDevice(ctx->device);
    std::unique_ptr<SJob> J(new SJob());
    pv3d_status st;
    if ((st = check_job(ctx, *job, 0, J->h))) return st;
    HostJob& h = J->h;
    if (h.g->n_mod > kServeMaxMod) return fail(PV3D_ERANGE, "the serving loop takes at most %d modules per job", kServeMaxMod);
    if (h.n_tiles > kServeMaxTiles) return fail(PV3D_ERANGE, "the serving loop takes at most %d raster tiles per job", kServeMaxTiles);
    if (h.job.n_sun > (int64_t)kFeedCap) return fail(PV3D_ERANGE, "the serving loop takes at most %u suns per job", kFeedCap);
    if ((st = start_server(ctx))) return st;
    Server* S = ctx->server;
    const bool dev_out = h.job.out.on_device != 0;
    if (job_bytes(h, !dev_out || !h.job.out.cell_counts, !dev_out) > S->arena.cap)
        return fail(PV3D_ENOMEM, "the job's data does not fit the serving loop's HBM budget");
    // own the inputs: the caller may reuse them once this returns
    const int64_t ns = h.job.n_sun;
    J->in.resize(6 * (size_t)ns);
    if (ns) {
        memcpy(J->in.data(), job->sun_xyz, 24 * (size_t)ns);
        memcpy(J->in.data() + 3 * ns, job->dni, 8 * (size_t)ns);
        memcpy(J->in.data() + 4 * ns, job->d_poa, 8 * (size_t)ns);
        memcpy(J->in.data() + 5 * ns, job->dt_h, 8 * (size_t)ns);
    }
    h.job.sun_xyz = J->in.data();
    h.job.dni = J->in.data() + 3 * ns;
    h.job.d_poa = J->in.data() + 4 * ns;
    h.job.dt_h = J->in.data() + 5 * ns;
    J->scene = job->scene;
    J->gen = job->gen;
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->fatal) return fail(S->fatal, "the serving loop has failed");
    if (S->pending.size() >= kMaxPending) return fail(PV3D_EBUSY, "serving queue full");
    const uint64_t t = S->next_ticket++;
    J->ticket = t;
    use(S, J->scene, 1);
    use(S, J->gen, 1);
    S->pending.push_back(J.get());
    S->jobs[t] = std::move(J);
    *ticket = t;
    S->cv.notify_all();
    return PV3D_OK;
}

pv3d_status pv3d_poll(pv3d_ctx* ctx, uint64_t ticket, int32_t* done) {
    if (!ctx || !done) return fail(PV3D_EINVAL, "null argument");
    Server* S = ctx->server;
    if (!S) return fail(PV3D_ENOENT, "unknown ticket %llu", (unsigned long long)ticket);
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) return fail(PV3D_ENOENT, "unknown ticket %llu", (unsigned long long)ticket);
    const SState s = it->second->state;
    *done = (s == kDone || s == kCancelled || s == kFailed) ? 1 : 0;
    return PV3D_OK;
}

pv3d_status pv3d_wait(pv3d_ctx* ctx, uint64_t ticket) {
    if (!ctx) return fail(PV3D_EINVAL, "null context");
    Server* S = ctx->server;
    if (!S) return fail(PV3D_ENOENT, "unknown ticket %llu", (unsigned long long)ticket);
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) return fail(PV3D_ENOENT, "unknown ticket %llu", (unsigned long long)ticket);
    SJob* J = it->second.get();
    S->cv_done.wait(lk, [&] { return J->state == kDone || J->state == kCancelled || J->state == kFailed; });
    const SState s = J->state;
    const pv3d_status r = J->result;
    S->jobs.erase(it);
    if (s == kCancelled) return fail(PV3D_ECANCELED, "job %llu was cancelled", (unsigned long long)ticket);
    if (s == kFailed) return fail(r ? r : PV3D_EDEVICE, "job %llu failed", (unsigned long long)ticket);
    return PV3D_OK;
}

pv3d_status pv3d_cancel(pv3d_ctx* ctx, uint64_t ticket) {
    if (!ctx) return fail(PV3D_EINVAL, "null context");
    Server* S = ctx->server;
    if (!S) return fail(PV3D_ENOENT, "unknown ticket %llu", (unsigned long long)ticket);
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) return fail(PV3D_ENOENT, "unknown ticket %llu", (unsigned long long)ticket);
    SJob* J = it->second.get();
    if (J->state == kPending || J->state == kLive) J->cancel = true;
    S->cv.notify_all();
    return PV3D_OK;
}

pv3d_status pv3d_serve_stats(pv3d_ctx* ctx, int64_t out[4]) {
    if (!ctx || !out) return fail(PV3D_EINVAL, "null argument");
    for (int i = 0; i < 4; i++) out[i] = 0;
    Server* S = ctx->server;
    if (!S) return PV3D_OK;
    std::lock_guard<std::mutex> lk(S->mu);
    out[0] = S->stats_done;
    out[1] = S->stats_launches;
    out[2] = S->stats_items;
    out[3] = (int64_t)S->pending.size();
    return PV3D_OK;
}

}  // extern "C"
