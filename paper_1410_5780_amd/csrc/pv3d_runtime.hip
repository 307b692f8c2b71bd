// Host runtime of libpv3d: the C ABI declared in include/pv3d.h.
//
// Owns the HIP stream, the device copies of scenes and generators, the work
// buffers of the per-sun path, and the HBM budget. Every step of the
// shading path runs in the kernels of pv3d_kernels.hip; the host validates
// arguments, sizes buffers and sequences launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pv3d.h"
#include "pv3d_device.h"
#include "pv3d_runtime.h"

using namespace pv3d;

namespace pv3d {

static thread_local std::string g_err;

pv3d_status fail(pv3d_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

pv3d_status hip_fail(hipError_t e, const char* what) {
    return fail(PV3D_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// A synchronous host-to-device copy on the context's own stream. hipMemcpy would go on the
// null stream, which waits for every blocking stream, the serving loop's kernel stream among
// them: a scene loaded while a launch is live would wait for that launch to end.
static hipError_t copy_in(Ctx* c, void* dev, const void* host, size_t bytes) {
    hipError_t e = hipMemcpyAsync(dev, host, bytes, hipMemcpyHostToDevice, c->stream);
    return e != hipSuccess ? e : hipStreamSynchronize(c->stream);
}

// ---------------------------------------------------------------------------
// device memory with budget accounting
// ---------------------------------------------------------------------------
pv3d_status Ctx::dalloc(void** p, size_t bytes, const char* what) {
    *p = nullptr;
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~(size_t)255;
    if (used + bytes > budget)
        return fail(PV3D_ENOMEM, "%s: %zu bytes exceed the HBM budget (%zu of %zu in use)", what, bytes,
                    (size_t)used, (size_t)budget);
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(PV3D_ENOMEM, "%s: hipMalloc(%zu): %s", what, bytes, hipGetErrorString(e));
    }
    sizes[*p] = bytes;
    used += bytes;
    return PV3D_OK;
}

void Ctx::dfree(void* p) {
    if (!p) return;
    auto it = sizes.find(p);
    if (it != sizes.end()) {
        used -= it->second;
        sizes.erase(it);
    }
    HoldServing hold(this);             // hipFree waits for every stream of the device
    (void)hipFree(p);
}

pv3d_status Buf::ensure(Ctx* c, size_t bytes, const char* what) {
    if (bytes <= cap && ptr) return PV3D_OK;
    if (c->carving) return c->carve(*this, bytes, what);
    if (ptr) {
        HoldServing hold(c);
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "synchronize before regrowing a work buffer");
        c->dfree(ptr);
        ptr = nullptr;
        cap = 0;
    }
    size_t want = std::max(bytes, cap + cap / 2);
    pv3d_status st = c->dalloc(&ptr, want, what);
    if (st != PV3D_OK) {
        st = c->dalloc(&ptr, bytes, what);
        if (st != PV3D_OK) return st;
        want = bytes;
    }
    cap = want;
    return PV3D_OK;
}

void Buf::release(Ctx* c) {
    if (ptr) c->dfree(ptr);
    ptr = nullptr;
    cap = 0;
}

static size_t align256(size_t b) { return (std::max<size_t>(b, 1) + 255) & ~(size_t)255; }

pv3d_status Ctx::carve(Buf& b, size_t bytes, const char* what) {
    const size_t want = align256(bytes);
    if (!scratch || carve_used + want > kScratchBytes)
        return fail(PV3D_ERANGE, "%s: %zu bytes do not fit the static scratch (%zu of %zu bytes taken)", what, want,
                    carve_used, kScratchBytes);
    b.ptr = static_cast<char*>(scratch) + carve_used;
    b.cap = want;
    carve_used += want;
    return PV3D_OK;
}

pv3d_status Ctx::wait_previous(hipStream_t st) {
    if (!ws_recorded) return PV3D_OK;
    hipError_t e = hipStreamWaitEvent(st, ws_ev, 0);
    return e == hipSuccess ? PV3D_OK : hip_fail(e, "wait for the previous evaluation");
}

pv3d_status Ctx::stage(const void* host, size_t bytes, void* dev, hipStream_t st) {
    // pinned staging so the caller's host arrays can be reused once we return
    if (staging_busy) {
        hipError_t e = hipEventSynchronize(staging_done);
        if (e != hipSuccess) return hip_fail(e, "wait for the staging buffer");
        staging_busy = false;
        staging_used = 0;
    }
    if (staging_used + bytes > staging_cap) {
        size_t need = staging_used + bytes;
        if (staging_used > 0) return fail(PV3D_EINVAL, "staging overflow");  // callers reserve first
        HoldServing hold(this);          // hipHostFree waits for every stream of the device
        if (staging) (void)hipHostFree(staging);
        staging = nullptr;
        size_t cap = std::max(need, (size_t)1 << 20);
        hipError_t e = hipHostMalloc(&staging, cap, hipHostMallocDefault);
        if (e != hipSuccess) return hip_fail(e, "hipHostMalloc staging");
        staging_cap = cap;
    }
    char* p = static_cast<char*>(staging) + staging_used;
    memcpy(p, host, bytes);
    staging_used += (bytes + 255) & ~(size_t)255;
    hipError_t e = hipMemcpyAsync(dev, p, bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync staging");
    return PV3D_OK;
}

pv3d_status Ctx::stage_reserve(size_t bytes) {
    if (staging_busy) {
        hipError_t e = hipEventSynchronize(staging_done);
        if (e != hipSuccess) return hip_fail(e, "wait for the staging buffer");
        staging_busy = false;
    }
    staging_used = 0;
    if (bytes > staging_cap) {
        HoldServing hold(this);          // hipHostFree waits for every stream of the device
        if (staging) (void)hipHostFree(staging);
        staging = nullptr;
        staging_cap = 0;
        size_t cap = std::max(bytes + 4096, (size_t)1 << 20);
        hipError_t e = hipHostMalloc(&staging, cap, hipHostMallocDefault);
        if (e != hipSuccess) return hip_fail(e, "hipHostMalloc staging");
        staging_cap = cap;
    }
    return PV3D_OK;
}

pv3d_status Ctx::stage_done(hipStream_t st) {
    hipError_t e = hipEventRecord(staging_done, st);
    if (e != hipSuccess) return hip_fail(e, "record staging event");
    staging_busy = true;
    return PV3D_OK;
}

// ---------------------------------------------------------------------------
// stage timing
// ---------------------------------------------------------------------------
hipError_t Profiler::begin(int stage, hipStream_t st, size_t* slot, int32_t n_sun) {
    if (used + 2 > pool.size()) {
        size_t grow = std::max<size_t>(1024, pool.size());
        for (size_t i = 0; i < grow; i++) {
            hipEvent_t ev;
            hipError_t e = hipEventCreate(&ev);
            if (e != hipSuccess) return e;
            pool.push_back(ev);
        }
    }
    *slot = used;
    used += 2;
    pending.emplace_back(stage, *slot);
    pending_suns.push_back(n_sun);
    return hipEventRecord(pool[*slot], st);
}

hipError_t Profiler::end(size_t slot, hipStream_t st) { return hipEventRecord(pool[slot + 1], st); }

hipError_t Profiler::collect() {
    for (size_t i = 0; i < pending.size(); i++) {
        const auto& pr = pending[i];
        hipError_t e = hipEventSynchronize(pool[pr.second + 1]);
        if (e != hipSuccess) return e;
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, pool[pr.second], pool[pr.second + 1]);
        if (e != hipSuccess) return e;
        total_ms[pr.first] += (double)ms;
        launches[pr.first] += 1;
        suns[pr.first] += pending_suns[i];
        float t0 = 0.f;
        if (ref && hipEventElapsedTime(&t0, ref, pool[pr.second]) == hipSuccess)
            spans[pr.first].emplace_back((double)t0, (double)t0 + (double)ms);
    }
    pending.clear();
    pending_suns.clear();
    used = 0;
    return hipSuccess;
}

double Profiler::busy_ms(int stage) const {
    std::vector<std::pair<double, double>> v = spans[stage];
    std::sort(v.begin(), v.end());
    double busy = 0.0, a = 0.0, b = 0.0;
    bool open = false;
    for (const auto& x : v) {
        if (!open || x.first > b) {
            if (open) busy += b - a;
            a = x.first;
            b = x.second;
            open = true;
        } else {
            b = std::max(b, x.second);
        }
    }
    if (open) busy += b - a;
    return busy;
}

void Profiler::reset() {
    pending.clear();
    pending_suns.clear();
    used = 0;
    for (int i = 0; i < PV3D_N_STAGES; i++) {
        total_ms[i] = 0.0;
        launches[i] = 0;
        suns[i] = 0;
        seen[i] = 0;
        spans[i].clear();
    }
}

// Launch `call` for `stage` (covering n_sun suns), bracketed by timing events when that
// stage is profiled.
template <typename F>
static hipError_t timed(Profiler& pf, int stage, hipStream_t st, F&& call, int32_t n_sun = 1) {
    if (!pf.take(stage)) return call();
    size_t slot = 0;
    hipError_t e = pf.begin(stage, st, &slot, n_sun);
    if (e != hipSuccess) return e;
    e = call();
    if (e != hipSuccess) return e;
    if (pf.used >= 1u << 16) {                     // bound the event pool: fold what is done
        e = pf.end(slot, st);
        if (e != hipSuccess) return e;
        return pf.collect();
    }
    return pf.end(slot, st);
}

// ---------------------------------------------------------------------------
// validation helpers
// ---------------------------------------------------------------------------
static bool finite3(const double* p) { return std::isfinite(p[0]) && std::isfinite(p[1]) && std::isfinite(p[2]); }

constexpr double kMaxCoord = 1.0e7;   // metres; keeps every light-space value far from overflow

pv3d_status check_sweep(const double* sun, const double* dni, const double* dpoa, const double* dt, int64_t n) {
    if (n < 0) return fail(PV3D_EINVAL, "n_sun < 0");
    if (n > 0 && (!sun || !dni || !dpoa || !dt)) return fail(PV3D_EINVAL, "null sweep array");
    for (int64_t t = 0; t < n; t++) {
        const double* s = sun + 3 * t;
        if (!finite3(s)) return fail(PV3D_EINVAL, "sun %lld is not finite", (long long)t);
        double l2 = (s[0] * s[0] + s[1] * s[1]) + s[2] * s[2];
        if (std::fabs(std::sqrt(l2) - 1.0) > 1e-9) return fail(PV3D_EINVAL, "sun %lld is not a unit vector", (long long)t);
        if (!std::isfinite(dni[t]) || dni[t] < 0 || !std::isfinite(dpoa[t]) || dpoa[t] < 0 || !std::isfinite(dt[t]))
            return fail(PV3D_EINVAL, "irradiance or dt of sun %lld out of range", (long long)t);
    }
    return PV3D_OK;
}

pv3d_status check_params(const pv3d_params* p) {
    if (!p) return fail(PV3D_EINVAL, "params is NULL");
    if (p->map_n < 16 || p->map_n > 16384) return fail(PV3D_EINVAL, "map_n %d outside [16, 16384]", p->map_n);
    if (p->k < 1 || p->k > 255) return fail(PV3D_EINVAL, "k %d outside [1, 255]", p->k);
    if (p->flags & ~(PV3D_EXPORT_DEPTH | PV3D_EXPORT_BITS | PV3D_SEPARATE_TEST | PV3D_FULL_RASTER))
        return fail(PV3D_EINVAL, "unknown flags 0x%x", p->flags);
    if (p->tile != 0 && p->tile != 32 && p->tile != 64 && p->tile != 128)
        return fail(PV3D_EINVAL, "tile %d not in {0, 32, 64, 128}", p->tile);
    if (p->bin_limit < 0 || p->bin_limit > kMaxBinLimit)
        return fail(PV3D_EINVAL, "bin_limit %d outside [0, %d]", p->bin_limit, kMaxBinLimit);
    if (p->reserved != 0) return fail(PV3D_EINVAL, "reserved field must be 0");
    return PV3D_OK;
}

// ---------------------------------------------------------------------------
// per-sun path
// ---------------------------------------------------------------------------
// 64-texel tiles up to 8192 texels a side: a 128-texel tile's LDS (about 75 KB) leaves room
// for two workgroups per CU, and the rooftop workload's year took 2.66 s with them against
// 1.22 s with 64-texel tiles. Above 8192 the tile counts of 64-texel tiles outgrow the LDS.
int32_t choose_tile(const pv3d_params& p) { return p.tile ? p.tile : (p.map_n <= 8192 ? 64 : 128); }

PathSizes path_sizes(const Scene& sc, const Gen& g, const pv3d_params& p, int64_t n_sun) {
    PathSizes z;
    z.tile = choose_tile(p);
    z.ntx = (p.map_n + z.tile - 1) / z.tile;
    z.n_tiles = z.ntx * z.ntx;
    z.large_tiles = p.bin_limit ? p.bin_limit : kMaxBinLimit;
    z.tri_total = sc.n_tri + (g.occluders ? 2 * g.n_mod : 0);
    // a clipped triangle becomes at most 5 (a triangle cut by four half-planes
    // is a polygon of at most 7 corners); a binned one touches <= large_tiles
    // tiles, a module's samples at most every tile
    z.rec_cap = 5 * z.tri_total + 64;
    z.bin_cap = (int64_t)z.large_tiles * z.rec_cap + (int64_t)g.n_mod * z.n_tiles;
    // pair mode: an item per binned record and module, and the same bound on pairs as on bin entries
    z.item_cap = z.rec_cap + g.n_mod;
    z.chunk_cap = z.bin_cap / kPairChunk + 1;
    z.cells = (int64_t)g.n_mod * g.n_cu * g.n_cv;
    z.mask_words = (z.n_tiles + 31) / 32;
    z.words = (p.k * p.k + 31) / 32;
    z.n_sun = n_sun;
    return z;
}

// Device bytes of one sun's part of a lane (records, large list, bins, tile counters and
// list, pair items and chunks, module boxes).
size_t lane_bytes_per_sun(const PathSizes& z, const Gen& g) {
    return sizeof(TriRec) * (size_t)z.rec_cap + 4 * (size_t)z.rec_cap + 4 * (size_t)z.bin_cap +
           4 * (size_t)(3 * (int64_t)z.n_tiles + 1) + 4 * (4 * (size_t)z.n_tiles + kListHead) +
           sizeof(PairItem) * (size_t)z.item_cap + 4 * (size_t)z.chunk_cap + 16 * (size_t)g.n_mod + 6 * 256;
}

// The per-sun arrays of an evaluation (views, counters, beam, bias, sweep, sphere,
// tile masks, bounds partials), in bytes.
constexpr int kPathBufs = 8;
static void path_buf_sizes(const PathSizes& z, const Gen& g, size_t b[kPathBufs]) {
    const size_t S = (size_t)std::max<int64_t>(z.n_sun, 1);
    b[0] = sizeof(View) * S;
    b[1] = sizeof(SunCounters) * S;
    b[2] = 8 * (size_t)std::max<int64_t>(z.n_sun * g.n_mod, 1);
    b[3] = 4 * (size_t)std::max<int64_t>(z.n_sun * g.n_mod, 1);
    b[4] = 8 * 6 * S;
    b[5] = 64;
    b[6] = 4 * (size_t)z.mask_words * S;
    b[7] = 8 * 6 * 1024;
}

// The buffers of a lane with room for `group` suns, one sun's part after the other, in bytes.
constexpr int kLaneBufs = 11;
static void lane_buf_sizes(const PathSizes& z, const Gen& g, int32_t map_n, bool own_map, int32_t group,
                           size_t b[kLaneBufs]) {
    const size_t G = (size_t)std::max(group, 1);
    b[0] = G * sizeof(TriRec) * (size_t)z.rec_cap;
    b[1] = G * 4 * (size_t)z.rec_cap;
    b[2] = G * 4 * (size_t)z.bin_cap;
    b[3] = G * 4 * (size_t)z.n_tiles;
    b[4] = G * 4 * (size_t)(z.n_tiles + 1);
    b[5] = G * 4 * (size_t)z.n_tiles;
    b[6] = G * 4 * (4 * (size_t)z.n_tiles + kListHead);
    b[7] = G * sizeof(PairItem) * (size_t)z.item_cap;
    b[8] = G * 4 * (size_t)z.chunk_cap;
    b[9] = G * 16 * (size_t)g.n_mod;
    b[10] = own_map ? 4 * (size_t)map_n * map_n : 0;
}

// Bytes of the static scratch one lane with room for `group` suns takes.
static size_t lane_carve_bytes(const PathSizes& z, const Gen& g, int32_t map_n, bool own_map, int32_t group) {
    size_t lb[kLaneBufs], lane = 0;
    lane_buf_sizes(z, g, map_n, own_map, group, lb);
    for (int i = 0; i < kLaneBufs; i++)
        if (i < kLaneBufs - 1 || own_map) lane += align256(lb[i]);
    return lane;
}

size_t carve_bytes(const PathSizes& z, const Gen& g, int32_t k, int32_t map_n, bool own_map, bool own_counts,
                   int32_t group, int n_lanes, int64_t n_groups) {
    size_t pb[kPathBufs], total = 0;
    path_buf_sizes(z, g, pb);
    for (size_t x : pb) total += align256(x);
    const size_t n_tab = (size_t)k * std::max(g.n_cu, g.n_cv);
    total += 2 * align256(8 * n_tab);                                  // sample tables
    if (g.n_trk > 0) total += align256(sizeof(Module) * (size_t)std::max<int64_t>(z.n_sun * g.n_mod, 1));
    if (own_counts) total += align256(4 * (size_t)std::max<int64_t>(z.n_sun * z.cells, 1));
    total += align256(sizeof(SunGroup) * (size_t)std::max<int64_t>(n_groups, 1));
    return total + (size_t)n_lanes * lane_carve_bytes(z, g, map_n, own_map, group);
}

pv3d_status Ctx::ensure_path(const PathSizes& z, const Gen& g, int32_t map_n, bool own_map) {
    pv3d_status st;
    if (z.rec_cap > INT32_MAX || z.bin_cap > INT32_MAX)
        return fail(PV3D_ERANGE, "scene too large for 32-bit bin indices");
    // (from the static scratch the lanes are taken once their group size is known)
    if (!carving && (st = ensure_lane(w.lane[0], z, g, map_n, own_map, 1))) return st;
    size_t b[kPathBufs];
    path_buf_sizes(z, g, b);
    Buf* bufs[kPathBufs] = {&w.views, &w.ctr, &w.beam, &w.bias, &w.sweep, &w.sphere, &w.tmask, &w.partial};
    static const char* const names[kPathBufs] = {"views", "counters", "module beam", "module bias", "sweep",
                                                 "bounding sphere", "tile masks", "bounds partials"};
    for (int i = 0; i < kPathBufs; i++)
        if ((st = bufs[i]->ensure(this, b[i], names[i]))) return st;
    return PV3D_OK;
}

// Room for `group` suns in each buffer of the lane, one sun's part after the other.
pv3d_status Ctx::ensure_lane(Lane& L, const PathSizes& z, const Gen& g, int32_t map_n, bool own_map, int32_t group) {
    pv3d_status st;
    size_t b[kLaneBufs];
    lane_buf_sizes(z, g, map_n, own_map, group, b);
    Buf* bufs[kLaneBufs] = {&L.rec, &L.large, &L.bins, &L.tile_count, &L.tile_start, &L.tile_cursor,
                            &L.tile_list, &L.pitems, &L.pchunk, &L.modbox, &L.map};
    static const char* const names[kLaneBufs] = {"triangle records", "large-triangle list", "tile bins",
                                                 "tile counts", "tile starts", "tile cursors", "tile work list",
                                                 "pair items", "pair chunks", "module tile boxes", "depth picture"};
    for (int i = 0; i < kLaneBufs; i++)
        if ((i < kLaneBufs - 1 || own_map) && (st = bufs[i]->ensure(this, b[i], names[i]))) return st;
    L.group = std::max(L.group, std::max(group, 1));
    return PV3D_OK;
}

// Sun q of a lane's group: its part of every lane buffer.
BinBuffers Ctx::bin_buffers(const PathSizes& z, int lane, int32_t q) {
    Lane& L = w.lane[lane];
    const size_t Q = (size_t)q;
    BinBuffers bb;
    bb.rec = static_cast<TriRec*>(L.rec.ptr) + Q * (size_t)z.rec_cap;
    bb.rec_cap = (int32_t)z.rec_cap;
    bb.large = static_cast<int32_t*>(L.large.ptr) + Q * (size_t)z.rec_cap;
    bb.tile_count = static_cast<int32_t*>(L.tile_count.ptr) + Q * (size_t)z.n_tiles;
    bb.tile_start = static_cast<int32_t*>(L.tile_start.ptr) + Q * (size_t)(z.n_tiles + 1);
    bb.tile_cursor = static_cast<int32_t*>(L.tile_cursor.ptr) + Q * (size_t)z.n_tiles;
    bb.bins = static_cast<int32_t*>(L.bins.ptr) + Q * (size_t)z.bin_cap;
    bb.modbox = static_cast<int4*>(L.modbox.ptr) + Q * (size_t)(z.item_cap - z.rec_cap);   // n_mod per sun
    bb.tile_list = nullptr;                // one workgroup per tile unless the sun takes the work list
    bb.list_ctr = nullptr;
    bb.split_at = 0;
    bb.pitems = static_cast<PairItem*>(L.pitems.ptr) + Q * (size_t)z.item_cap;
    bb.pchunk = static_cast<int32_t*>(L.pchunk.ptr) + Q * (size_t)z.chunk_cap;
    bb.pctr = nullptr;                     // per sun
    bb.item_cap = (int32_t)z.item_cap;
    bb.bin_cap = (int32_t)z.bin_cap;
    bb.tile = z.tile;
    bb.ntx = z.ntx;
    bb.n_tiles = z.n_tiles;
    bb.large_tiles = z.large_tiles;
    return bb;
}

// Bounding sphere of the scene vertices and module corners: centre and half
// diagonal of their axis-aligned box (the kernels' bounds reduction computes
// the same values from the same IEEE operations).
void host_sphere(const Scene& sc, const Gen& g, double sphere[4]) {
    double lo[3], hi[3];
    for (int c = 0; c < 3; c++) {
        lo[c] = std::fmin(sc.lo[c], g.lo[c]);
        hi[c] = std::fmax(sc.hi[c], g.hi[c]);
    }
    const double dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
    sphere[0] = (lo[0] + hi[0]) * 0.5;
    sphere[1] = (lo[1] + hi[1]) * 0.5;
    sphere[2] = (lo[2] + hi[2]) * 0.5;
    sphere[3] = 0.5 * std::sqrt((dx * dx + dy * dy) + dz * dz);
}

// Fractional sample positions along a module edge, (q + 1/2) / (k n).
void host_sample_tables(int32_t k, int32_t n_cu, int32_t n_cv, double* fu, double* fv) {
    for (int32_t i = 0; i < k * n_cu; i++) fu[i] = ((double)i + 0.5) / (double)(k * n_cu);
    for (int32_t i = 0; i < k * n_cv; i++) fv[i] = ((double)i + 0.5) / (double)(k * n_cv);
}

SceneDev scene_dev(const Scene& sc) {
    SceneDev d;
    d.xyz = sc.xyz;
    d.tri = sc.tri;
    d.cbox = sc.cbox;
    d.n_vert = sc.n_vert;
    d.n_tri = sc.n_tri;
    return d;
}

void free_gen(Ctx* c, Gen& g) {
    void** all[] = {(void**)&g.mods, (void**)&g.cell_sub, (void**)&g.str_start, (void**)&g.str_mods,
                    (void**)&g.trk, (void**)&g.mod_trk, (void**)&g.sub_start, (void**)&g.sub_cell, (void**)&g.svf};
    for (void** p : all) {
        c->dfree(*p);
        *p = nullptr;
    }
}

GenDev gen_dev(const Gen& g) {
    GenDev d;
    d.mods = g.mods;
    d.mods_sun = nullptr;
    d.n_mod = (int32_t)g.n_mod;
    d.n_cu = g.n_cu;
    d.n_cv = g.n_cv;
    d.n_sub = g.n_sub;
    d.n_str = g.n_str;
    d.occluders = g.occluders;
    d.cell_sub = g.cell_sub;
    d.str_start = g.str_start;
    d.str_mods = g.str_mods;
    d.sub_start = g.sub_start;
    d.sub_cell = g.sub_cell;
    d.svf = g.svf;
    d.diode = g.diode;
    return d;
}

// 64-texel tiles with more bin entries than this go to four workgroups, one per
// quadrant (each still walks all of the tile's triangles): the heaviest tiles,
// under tall occluders, otherwise finish long after the rest of the launch.
// C2 year: 397 ms at 32, 351 ms at 64, 335 ms at 128, 338 ms at 256 or with no
// split.
constexpr int32_t kSplitEntries = 128;

// Everything of one evaluation that lives on the device.
pv3d_status Ctx::run_path(const Scene& sc, const Gen& g, const pv3d_params& p, const double* sun_host,
                          int64_t n_sun, const double* d_sun, const double* d_dni, const double* d_dpoa,
                          const double* d_dt, uint32_t* counts, double* power, double* power_ref,
                          double* energy, uint32_t* maps, uint32_t* bits, hipStream_t st) {
    PathSizes z = path_sizes(sc, g, p, n_sun);
    pv3d_status rs = ensure_path(z, g, p.map_n, maps == nullptr && (p.flags & PV3D_SEPARATE_TEST));
    if (rs) return rs;
    hipError_t e;
    if ((rs = ensure_tables(g, p.k))) return rs;
    SceneDev sd = scene_dev(sc);
    GenDev gd = gen_dev(g);
    View* views = static_cast<View*>(w.views.ptr);
    SunCounters* ctr = static_cast<SunCounters*>(w.ctr.ptr);
    double* beam = static_cast<double*>(w.beam.ptr);
    int32_t* bias = static_cast<int32_t*>(w.bias.ptr);
    double* sphere = static_cast<double*>(w.sphere.ptr);
    const int64_t N2 = (int64_t)p.map_n * p.map_n;

    // the work buffers are shared by every call of the context: wait for the previous call's
    // kernels, which may still run on another stream
    if (ws_recorded && (e = hipStreamWaitEvent(st, ws_ev, 0))) return hip_fail(e, "wait for the previous evaluation");
    if ((e = hipMemsetAsync(ctr, 0, sizeof(SunCounters) * (size_t)std::max<int64_t>(n_sun, 1), st)))
        return hip_fail(e, "clear counters");
    // Suns go in groups of up to kMaxGroup per launch sequence (one group's set-up,
    // binning and tile pass in five launches), consecutive groups taking turns on up
    // to kLanes streams, so that one group's set-up and binning kernels, which leave
    // much of the GPU idle, run beside another group's tile pass and its drain. The
    // group shrinks until both lanes fit half of the budget left; a lane that still
    // does not fit is left out.
    const bool own_map = maps == nullptr && (p.flags & PV3D_SEPARATE_TEST);
    int64_t n_up = 0;
    for (int64_t s = 0; s < n_sun; s++)
        if (sun_host[3 * s + 2] > 0.0) n_up++;
    int32_t G = own_map ? 1 : kMaxGroup;                 // the materialised route keeps one picture per lane
    G = (int32_t)std::max<int64_t>(1, std::min<int64_t>(G, (n_up + kLanes - 1) / kLanes));
    if (carving) {
        // from the static scratch: the largest group whose lanes fit beside what is taken;
        // the descriptors and tracker poses first, so that a lane left out cannot starve them
        const size_t poses = g.n_trk > 0 ? align256(sizeof(Module) * (size_t)std::max<int64_t>(n_sun * g.n_mod, 1)) : 0;
        auto need = [&](int32_t Gc) {
            const int64_t n_groups = std::max<int64_t>((n_up + Gc - 1) / Gc, 1);
            return carve_used + align256(sizeof(SunGroup) * (size_t)n_groups) + poses +
                   (size_t)kLanes * lane_carve_bytes(z, g, p.map_n, own_map, Gc);
        };
        while (G > 1 && need(G) > kScratchBytes) G /= 2;
        if ((rs = w.groups.ensure(this, sizeof(SunGroup) * (size_t)std::max<int64_t>((n_up + G - 1) / G, 1),
                                  "group descriptors")))
            return rs;
        if (g.n_trk > 0 &&
            (rs = w.posed.ensure(this, sizeof(Module) * (size_t)std::max<int64_t>(n_sun * g.n_mod, 1), "posed modules")))
            return rs;
    } else {
        const size_t per_sun = lane_bytes_per_sun(z, g);
        const uint64_t room = budget > used ? budget - used : 0;
        // what the lanes hold already counts as room
        uint64_t held = 0;
        for (int l = 0; l < kLanes; l++)
            for (Buf* bf : {&w.lane[l].rec, &w.lane[l].large, &w.lane[l].bins, &w.lane[l].pitems, &w.lane[l].pchunk})
                held += bf->cap;
        while (G > 1 && (uint64_t)kLanes * (uint64_t)G * per_sun > (room + held) / 2) G /= 2;
    }
    if ((rs = ensure_lane(w.lane[0], z, g, p.map_n, own_map, G)) != PV3D_OK) {
        if (G == 1) return rs;
        G = 1;
        if ((rs = ensure_lane(w.lane[0], z, g, p.map_n, own_map, 1))) return rs;
    }
    int n_lanes = 1;
    while (n_lanes < kLanes && (int64_t)n_lanes * G < n_up && lane_st[n_lanes]) {
        const size_t taken = carve_used;
        if (ensure_lane(w.lane[n_lanes], z, g, p.map_n, own_map, G) != PV3D_OK) {
            if (carving) {                // give back what the lane took of the static scratch
                carve_used = taken;
                w.lane[n_lanes] = Lane{};
            }
            break;
        }
        n_lanes++;
    }
    // tile counts start at zero; the scan of every sun leaves them at zero again
    for (int l = 0; l < n_lanes; l++)
        if ((e = hipMemsetAsync(w.lane[l].tile_count.ptr, 0, 4 * (size_t)G * (size_t)z.n_tiles, st)))
            return hip_fail(e, "clear tile counts");
    if (counts && (e = hipMemsetAsync(counts, 0, 4 * (size_t)(n_sun * z.cells), st))) return hip_fail(e, "clear counts");
    if (bits && (e = hipMemsetAsync(bits, 0, 4 * (size_t)(n_sun * z.cells * z.words), st))) return hip_fail(e, "clear bits");
    if (maps && (e = launch_fill_u32(maps, kDepthMax, n_sun * N2, st))) return hip_fail(e, "fill depth maps");

    if (g.n_trk > 0) {
        // trackers: every module posed for every sun, and a sphere over the scene and the
        // trackers' reach (boxes known on the host since load and definition)
        if ((rs = w.posed.ensure(this, sizeof(Module) * (size_t)std::max<int64_t>(n_sun * g.n_mod, 1), "posed modules")))
            return rs;
        Module* posed = static_cast<Module*>(w.posed.ptr);
        if ((e = launch_pose(d_sun, n_sun, g.mods, (int32_t)g.n_mod, g.trk, g.mod_trk, posed, st)))
            return hip_fail(e, "pose modules");
        gd.mods_sun = posed;
        double lo[3], hi[3];
        for (int c = 0; c < 3; c++) {
            lo[c] = std::fmin(sc.lo[c], g.lo[c]);
            hi[c] = std::fmax(sc.hi[c], g.hi[c]);
        }
        if ((e = launch_box_sphere(lo, hi, sphere, st))) return hip_fail(e, "bounding sphere");
    } else {
        int32_t n_part = bounds_partials(sc.n_vert + 4 * g.n_mod);
        if ((e = launch_bounds(sd, gd, static_cast<double*>(w.partial.ptr), n_part, sphere, st)))
            return hip_fail(e, "bounds");
    }
    // the sparse route bins triangles only into tiles that hold samples
    const bool sparse = maps == nullptr && !(p.flags & (PV3D_SEPARATE_TEST | PV3D_FULL_RASTER));
    uint32_t* tmask = sparse ? static_cast<uint32_t*>(w.tmask.ptr) : nullptr;
    TileGrid tg{z.tile, z.ntx, z.n_tiles, z.mask_words};
    if (z.mask_words > 512) tmask = nullptr;
    if ((e = timed(prof, PV3D_STAGE_SETUP, st, [&] { return launch_setup(d_sun, n_sun, d_dni, gd, sphere, p.map_n, views, beam, bias, tg, tmask, st); }, (int32_t)n_sun)))
        return hip_fail(e, "setup");
    // the groups: descriptors of every sun, built here and copied to the device once
    const bool separate = (p.flags & PV3D_SEPARATE_TEST) != 0;
    std::vector<SunGroup> groups;
    std::vector<int> group_lane;
    for (int64_t s = 0; s < n_sun; s++) {
        if (!(sun_host[3 * s + 2] > 0.0)) continue;        // below the horizon: outputs stay zero
        if (groups.empty() || groups.back().n == G) {
            groups.emplace_back();
            memset(&groups.back(), 0, sizeof(SunGroup));
            group_lane.push_back((int)((groups.size() - 1) % (size_t)n_lanes));
        }
        SunGroup& grp = groups.back();
        const int lane = group_lane.back();
        const int32_t q = grp.n++;
        GroupSun& S = grp.sun[q];
        S.bb = bin_buffers(z, lane, q);
        if (sparse) {      // the scan lists the tiles with work, heaviest first; 64-texel ones split in quadrants
            int32_t* tl = static_cast<int32_t*>(w.lane[lane].tile_list.ptr) + (size_t)q * (4 * (size_t)z.n_tiles + kListHead);
            S.bb.list_ctr = tl;
            S.bb.tile_list = tl + kListHead;  // list_ctr: items, next item, first light item, XCD counters
            S.bb.split_at = z.tile == 64 ? kSplitEntries : 0;
        }
        S.bb.pctr = &ctr[s].pairs;
        S.out.map = maps ? maps + s * N2 : (separate ? static_cast<uint32_t*>(w.lane[lane].map.ptr) : nullptr);
        S.out.counts = counts + s * z.cells;
        S.out.bits = bits ? bits + s * z.cells * z.words : nullptr;
        S.out.test = separate ? 0 : 1;
        S.out.sparse = sparse ? 1 : 0;
        S.g = gd;
        if (gd.mods_sun) S.g.mods = gd.mods_sun + s * gd.n_mod;
        S.tmask = tmask ? tmask + s * z.mask_words : nullptr;
        S.s = s;
    }
    if (!groups.empty()) {
        if ((rs = w.groups.ensure(this, sizeof(SunGroup) * groups.size(), "group descriptors"))) return rs;
        if ((rs = upload_groups(groups, st))) return rs;
    }
    if (n_lanes > 1 && (e = hipEventRecord(fork_ev, st))) return hip_fail(e, "fork the lanes");
    for (int l = 1; l < n_lanes; l++)
        if ((e = hipStreamWaitEvent(lane_st[l], fork_ev, 0))) return hip_fail(e, "fork the lanes");
    const SunGroup* d_groups = static_cast<const SunGroup*>(w.groups.ptr);
    for (size_t gi = 0; gi < groups.size(); gi++) {
        const int lane = group_lane[gi];
        if ((rs = run_group(d_groups + gi, groups[gi], z, sd, gd, p, views, ctr, bias, beam, n_lanes,
                            lane ? lane_st[lane] : st)))
            return rs;
    }
    for (int l = 1; l < n_lanes; l++)
        if ((e = hipEventRecord(join_ev[l], lane_st[l])) || (e = hipStreamWaitEvent(st, join_ev[l], 0)))
            return hip_fail(e, "join the lanes");
    // One launch over every sun. With the single-diode model one sun's losses keep a workgroup
    // busy for milliseconds of arithmetic and the whole sweep side by side fills the GPU:
    // launched per group (8 suns, on the group's lane) the row plant's year took
    // 6.6 s instead of 0.41, in chunks of 512 suns between the groups 0.59 s.
    if ((e = timed(prof, PV3D_STAGE_LOSS, st, [&] { return launch_loss(0, n_sun, d_sun, beam, counts, d_dpoa, gd, p.k, power, power_ref, ctr, st); }, (int32_t)n_sun)))
        return hip_fail(e, "loss");
    if ((e = launch_energy(n_sun, power, power_ref, d_dt, energy, st))) return hip_fail(e, "energy");
    if ((e = hipEventRecord(ws_ev, st))) return hip_fail(e, "record the end of the evaluation");
    ws_recorded = true;
    return PV3D_OK;
}

// Copy the group descriptors to the device through pinned staging of their own.
pv3d_status Ctx::upload_groups(const std::vector<SunGroup>& groups, hipStream_t st) {
    const size_t bytes = sizeof(SunGroup) * groups.size();
    hipError_t e;
    if (carving) {   // no pinned staging to grow: a copy from pageable memory, staged before it returns
        if ((e = hipMemcpyAsync(w.groups.ptr, groups.data(), bytes, hipMemcpyHostToDevice, st)))
            return hip_fail(e, "copy descriptors");
        return PV3D_OK;
    }
    if (gstage_busy) {
        if ((e = hipEventSynchronize(gstage_done))) return hip_fail(e, "wait for the descriptor staging");
        gstage_busy = false;
    }
    if (bytes > gstage_cap) {
        HoldServing hold(this);          // hipHostFree waits for every stream of the device
        if (gstage) (void)hipHostFree(gstage);
        gstage = nullptr;
        gstage_cap = 0;
        const size_t cap = std::max(bytes + bytes / 2, (size_t)1 << 20);
        if ((e = hipHostMalloc(&gstage, cap, hipHostMallocDefault))) return hip_fail(e, "hipHostMalloc descriptors");
        gstage_cap = cap;
    }
    memcpy(gstage, groups.data(), bytes);
    if ((e = hipMemcpyAsync(w.groups.ptr, gstage, bytes, hipMemcpyHostToDevice, st))) return hip_fail(e, "copy descriptors");
    if ((e = hipEventRecord(gstage_done, st))) return hip_fail(e, "record descriptor copy");
    gstage_busy = true;
    return PV3D_OK;
}

// The launch sequence of one group of suns.
pv3d_status Ctx::run_group(const SunGroup* d_grp, const SunGroup& grp, const PathSizes& z, const SceneDev& sd,
                           const GenDev& gd, const pv3d_params& p, const View* views, SunCounters* ctr,
                           const int32_t* bias, const double* beam, int n_lanes, hipStream_t st) {
    hipError_t e;
    const int32_t ng = grp.n;
    const bool listed = grp.sun[0].bb.tile_list != nullptr;
    // pair mode: set-up lays the binned records and module boxes out in pair space;
    // counting and scatter then share every sun's pairs evenly over the grid
    const int32_t pair_grid = 4 * n_cu;
    if ((e = timed(prof, PV3D_STAGE_TRI_SETUP, st, [&] { return launch_tri_setup_group(d_grp, ng, views, sd, gd, bias, p.map_n, ctr, st); }, ng)))
        return hip_fail(e, "tri_setup");
    if ((e = timed(prof, PV3D_STAGE_BIN_SCAN, st, [&] {
             hipError_t r = launch_pair_count_group(d_grp, pair_grid, st);
             return r ? r : launch_bin_scan_group(d_grp, ng, z.n_tiles, st);
         }, ng)))
        return hip_fail(e, "bin_scan");
    if ((e = timed(prof, PV3D_STAGE_BIN_SCATTER, st, [&] { return launch_pair_scatter_group(d_grp, pair_grid, st); }, ng)))
        return hip_fail(e, "bin_scatter");
    // with several lanes the tile pass keeps to two workgroups per CU, leaving room for the other
    // lane's set-up and binning kernels beside it
    if ((e = timed(prof, PV3D_STAGE_RASTER, st, [&] {
             return launch_raster_group(d_grp, ng, listed, z.tile, z.n_tiles, views, ctr, p.map_n, bias, gd.n_mod,
                                        static_cast<double*>(w.fu.ptr), static_cast<double*>(w.fv.ptr), p.k, n_cu,
                                        n_lanes > 1 ? 2 : 0, st);
         }, ng)))
        return hip_fail(e, "raster");
    if (p.flags & PV3D_SEPARATE_TEST)
        for (int32_t q = 0; q < ng; q++) {
            const GroupSun& S = grp.sun[q];
            if ((e = timed(prof, PV3D_STAGE_SAMPLE_TEST, st, [&] {
                     return launch_sample_test(S.s, views, S.g, beam, bias, static_cast<double*>(w.fu.ptr),
                                               static_cast<double*>(w.fv.ptr), p.k, S.out.map, p.map_n, S.out.counts,
                                               S.out.bits, st);
                 })))
                return hip_fail(e, "sample_test");
        }
    return PV3D_OK;
}

pv3d_status Ctx::ensure_tables(const Gen& g, int32_t k) {
    pv3d_status st;
    size_t n = (size_t)k * std::max(g.n_cu, g.n_cv);
    if ((st = w.fu.ensure(this, 8 * n, "sample table u"))) return st;
    if ((st = w.fv.ensure(this, 8 * n, "sample table v"))) return st;
    hipError_t e = launch_sample_tables(static_cast<double*>(w.fu.ptr), static_cast<double*>(w.fv.ptr), k,
                                        g.n_cu, g.n_cv, stream_in_use);
    if (e != hipSuccess) return hip_fail(e, "sample tables");
    return PV3D_OK;
}

pv3d_status Ctx::read_overflow(int64_t n_sun, hipStream_t st, bool* overflow) {
    *overflow = false;
    std::vector<SunCounters> h((size_t)std::max<int64_t>(n_sun, 1));
    hipError_t e = hipMemcpyAsync(h.data(), w.ctr.ptr, sizeof(SunCounters) * (size_t)n_sun,
                                  hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return hip_fail(e, "read counters");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "synchronize");
    for (int64_t s = 0; s < n_sun; s++)
        if (h[(size_t)s].overflow) *overflow = true;
    return PV3D_OK;
}

// The work buffers of pv3d_evaluate_noalloc. Host code never passes `scratch`
// itself to the device (in host code the name stands for a host-side shadow):
// it uses the address hipGetSymbolAddress gives for each device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static std::mutex g_scratch_mu;
static std::map<int, void*> g_scratch_at;   // device -> address of its copy of scratch

// Address of the current device's copy of the static scratch, looked up once per device.
static pv3d_status scratch_address(int device, void** out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_at.find(device);
    if (it == g_scratch_at.end()) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "address of the static scratch");
        if (!ptr) return fail(PV3D_EDEVICE, "the static scratch has no device address");
        it = g_scratch_at.emplace(device, ptr).first;
    }
    *out = it->second;
    return PV3D_OK;
}

}  // namespace pv3d

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

pv3d_status pv3d_create(int32_t device, uint64_t hbm_budget_bytes, pv3d_ctx** out) {
    if (!out) return fail(PV3D_EINVAL, "out is NULL");
    *out = nullptr;
    int nd = 0;
    hipError_t e = hipGetDeviceCount(&nd);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= nd) return fail(PV3D_EINVAL, "device %d of %d", device, nd);
    if ((e = hipSetDevice(device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    size_t fr = 0, tot = 0;
    if ((e = hipMemGetInfo(&fr, &tot)) != hipSuccess) return hip_fail(e, "hipMemGetInfo");
    std::unique_ptr<pv3d_ctx> c(new pv3d_ctx());
    c->device = device;
    c->budget = hbm_budget_bytes ? hbm_budget_bytes : (uint64_t)(0.9 * (double)fr);
    if ((e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e, "hipStreamCreate");
    if ((e = hipEventCreateWithFlags(&c->staging_done, hipEventDisableTiming)) != hipSuccess)
        return hip_fail(e, "hipEventCreate");
    c->stream_in_use = c->stream;
    for (int l = 1; l < kLanes; l++) {
        if ((e = hipStreamCreateWithFlags(&c->lane_st[l], hipStreamNonBlocking)) != hipSuccess)
            return hip_fail(e, "hipStreamCreate");
        if ((e = hipEventCreateWithFlags(&c->join_ev[l], hipEventDisableTiming)) != hipSuccess)
            return hip_fail(e, "hipEventCreate");
    }
    if ((e = hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming)) != hipSuccess)
        return hip_fail(e, "hipEventCreate");
    if ((e = hipEventCreateWithFlags(&c->ws_ev, hipEventDisableTiming)) != hipSuccess)
        return hip_fail(e, "hipEventCreate");
    if ((e = hipEventCreateWithFlags(&c->gstage_done, hipEventDisableTiming)) != hipSuccess)
        return hip_fail(e, "hipEventCreate");
    if ((e = hipEventCreate(&c->prof.ref)) != hipSuccess) return hip_fail(e, "hipEventCreate");
    {
        pv3d_status st = scratch_address(device, &c->scratch);   // device is current
        if (st != PV3D_OK) return st;
    }
    {
        hipDeviceProp_t prop;
        if ((e = hipGetDeviceProperties(&prop, device)) != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
        c->max_lds = prop.sharedMemPerBlock;
        c->n_cu = prop.multiProcessorCount;
    }
    *out = c.release();
    return PV3D_OK;
}

void pv3d_destroy(pv3d_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    pv3d_server_stop(ctx);
    (void)hipDeviceSynchronize();
    for (auto& kv : ctx->scenes) {
        ctx->dfree(kv.second.xyz);
        ctx->dfree(kv.second.tri);
        if (kv.second.cbox) ctx->dfree(kv.second.cbox);
    }
    for (auto& kv : ctx->gens) free_gen(ctx, kv.second);
    ctx->w.release_all(ctx);
    ctx->release_batched();
    if (ctx->staging) (void)hipHostFree(ctx->staging);
    for (hipEvent_t ev : ctx->prof.pool) (void)hipEventDestroy(ev);
    (void)hipEventDestroy(ctx->staging_done);
    (void)hipStreamDestroy(ctx->stream);
    for (int l = 1; l < kLanes; l++) {
        if (ctx->lane_st[l]) (void)hipStreamDestroy(ctx->lane_st[l]);
        if (ctx->join_ev[l]) (void)hipEventDestroy(ctx->join_ev[l]);
    }
    if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
    if (ctx->ws_ev) (void)hipEventDestroy(ctx->ws_ev);
    if (ctx->gstage) (void)hipHostFree(ctx->gstage);
    if (ctx->gstage_done) (void)hipEventDestroy(ctx->gstage_done);
    if (ctx->prof.ref) (void)hipEventDestroy(ctx->prof.ref);
    delete ctx;
}

const char* pv3d_last_error(const pv3d_ctx* ctx) {
    (void)ctx;
    return pv3d::g_err.c_str();
}

pv3d_status pv3d_scene_load(pv3d_ctx* ctx, const double* xyz, int64_t n_vert, const int32_t* tri, int64_t n_tri,
                            uint64_t* scene_out) {
    if (!ctx || !scene_out) return fail(PV3D_EINVAL, "null argument");
    if (n_vert < 0 || n_tri < 0 || n_vert >= INT32_MAX || n_tri >= INT32_MAX / 8)
        return fail(PV3D_EINVAL, "bad sizes n_vert=%lld n_tri=%lld", (long long)n_vert, (long long)n_tri);
    if ((n_vert && !xyz) || (n_tri && !tri)) return fail(PV3D_EINVAL, "null array");
    for (int64_t i = 0; i < n_vert; i++) {
        if (!finite3(xyz + 3 * i)) return fail(PV3D_EINVAL, "vertex %lld is not finite", (long long)i);
        for (int c = 0; c < 3; c++)
            if (std::fabs(xyz[3 * i + c]) > kMaxCoord)
                return fail(PV3D_ERANGE, "vertex %lld beyond %.0e m", (long long)i, kMaxCoord);
    }
    for (int64_t i = 0; i < 3 * n_tri; i++)
        if (tri[i] < 0 || tri[i] >= n_vert) return fail(PV3D_EINVAL, "triangle index %lld out of range", (long long)i / 3);
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    (void)hipSetDevice(ctx->device);
    Scene s;
    s.n_vert = n_vert;
    s.n_tri = n_tri;
    for (int c = 0; c < 3; c++) {
        s.lo[c] = INFINITY;
        s.hi[c] = -INFINITY;
    }
    for (int64_t i = 0; i < n_vert; i++)
        for (int c = 0; c < 3; c++) {
            s.lo[c] = std::fmin(s.lo[c], xyz[3 * i + c]);
            s.hi[c] = std::fmax(s.hi[c], xyz[3 * i + c]);
        }
    pv3d_status st;
    if ((st = ctx->dalloc((void**)&s.xyz, 24 * (size_t)n_vert, "scene vertices"))) return st;
    if ((st = ctx->dalloc((void**)&s.tri, 12 * (size_t)n_tri, "scene triangles"))) {
        ctx->dfree(s.xyz);
        return st;
    }
    // vertex box of every block of kTriBlock triangles: the triangle set-up
    // skips a block whose box lies wholly outside a sun's window
    const int64_t n_blk = (n_tri + kTriBlock - 1) / kTriBlock;
    std::vector<double> cbox(6 * (size_t)n_blk);
    for (int64_t b = 0; b < n_blk; b++) {
        double* q = cbox.data() + 6 * b;
        for (int c = 0; c < 3; c++) {
            q[c] = INFINITY;
            q[3 + c] = -INFINITY;
        }
        for (int64_t t = b * kTriBlock; t < std::min<int64_t>(n_tri, (b + 1) * kTriBlock); t++)
            for (int v = 0; v < 3; v++)
                for (int c = 0; c < 3; c++) {
                    const double x = xyz[3 * (int64_t)tri[3 * t + v] + c];
                    q[c] = std::fmin(q[c], x);
                    q[3 + c] = std::fmax(q[3 + c], x);
                }
    }
    if (n_blk && (st = ctx->dalloc((void**)&s.cbox, 48 * (size_t)n_blk, "triangle block boxes"))) {
        ctx->dfree(s.xyz);
        ctx->dfree(s.tri);
        return st;
    }
    hipError_t e;
    if (n_vert && (e = copy_in(ctx, s.xyz, xyz, 24 * (size_t)n_vert))) return hip_fail(e, "copy vertices");
    if (n_tri && (e = copy_in(ctx, s.tri, tri, 12 * (size_t)n_tri))) return hip_fail(e, "copy triangles");
    if (n_blk && (e = copy_in(ctx, s.cbox, cbox.data(), 48 * (size_t)n_blk)))
        return hip_fail(e, "copy block boxes");
    uint64_t h = ++ctx->next_handle;
    ctx->scenes[h] = s;
    *scene_out = h;
    return PV3D_OK;
}

pv3d_status pv3d_scene_release(pv3d_ctx* ctx, uint64_t scene) {
    if (!ctx) return fail(PV3D_EINVAL, "null context");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto it = ctx->scenes.find(scene);
    if (it == ctx->scenes.end()) return fail(PV3D_ENOENT, "unknown scene %llu", (unsigned long long)scene);
    if (ctx->scene_in_use(scene)) return fail(PV3D_EBUSY, "scene %llu is used by a running job", (unsigned long long)scene);
    (void)hipSetDevice(ctx->device);
    HoldServing hold(ctx);
    (void)hipDeviceSynchronize();
    ctx->dfree(it->second.xyz);
    ctx->dfree(it->second.tri);
    if (it->second.cbox) ctx->dfree(it->second.cbox);
    ctx->scenes.erase(it);
    return PV3D_OK;
}

static pv3d_status define_upload(pv3d_ctx* ctx, Gen& g, const std::vector<Module>& hm, const int32_t* cell_substring,
                                 const std::vector<int32_t>& start, const std::vector<int32_t>& order,
                                 const std::vector<int32_t>& sub_start, const std::vector<int32_t>& sub_cell,
                                 const pv3d_tracker* trackers, int32_t n_trk, const int32_t* module_tracker);

static pv3d_status define_generator(pv3d_ctx* ctx, const pv3d_module* mods, int64_t n_mod,
                                   const int32_t* cell_substring, int32_t n_sub, const int32_t* module_string,
                                   int32_t add_as_occluders, const pv3d_tracker* trackers, int32_t n_trk,
                                   const int32_t* module_tracker, uint64_t* gen_out) {
    if (!ctx || !mods || !cell_substring || !module_string || !gen_out) return fail(PV3D_EINVAL, "null argument");
    if (n_trk < 0 || (n_trk > 0 && (!trackers || !module_tracker))) return fail(PV3D_EINVAL, "trackers");
    for (int32_t t = 0; t < n_trk; t++) {
        const pv3d_tracker& T = trackers[t];
        if (T.kind != 1 && T.kind != 2) return fail(PV3D_EINVAL, "tracker %d: kind %d", t, T.kind);
        if (T.reserved != 0) return fail(PV3D_EINVAL, "tracker %d: reserved field not 0", t);
        if (!finite3(T.pivot) || !finite3(T.axis)) return fail(PV3D_EINVAL, "tracker %d is not finite", t);
        const double aa = (T.axis[0] * T.axis[0] + T.axis[1] * T.axis[1]) + T.axis[2] * T.axis[2];
        if (T.axis[2] != 0.0 || !(std::fabs(aa - 1.0) <= 1e-9))
            return fail(PV3D_EINVAL, "tracker %d: the axis must be a horizontal unit vector", t);
        for (int c = 0; c < 3; c++)
            if (std::fabs(T.pivot[c]) > kMaxCoord) return fail(PV3D_ERANGE, "tracker %d beyond %.0e m", t, kMaxCoord);
    }
    if (n_trk > 0)
        for (int64_t m = 0; m < n_mod; m++)
            if (module_tracker[m] < -1 || module_tracker[m] >= n_trk)
                return fail(PV3D_EINVAL, "module %lld: tracker %d out of range", (long long)m, module_tracker[m]);
    if (n_mod < 1 || n_mod >= INT32_MAX / 8) return fail(PV3D_EINVAL, "n_mod %lld", (long long)n_mod);
    const int32_t n_cu = mods[0].n_cu, n_cv = mods[0].n_cv;
    if (n_cu < 1 || n_cv < 1 || n_cu > 4096 || n_cv > 4096) return fail(PV3D_EINVAL, "cells per module %d x %d", n_cu, n_cv);
    if (n_sub < 1 || n_sub > n_cu * n_cv) return fail(PV3D_EINVAL, "n_sub %d", n_sub);
    std::vector<Module> hm((size_t)n_mod);
    for (int64_t m = 0; m < n_mod; m++) {
        const pv3d_module& M = mods[m];
        if (M.n_cu != n_cu || M.n_cv != n_cv) return fail(PV3D_EINVAL, "module %lld: all modules must share n_cu, n_cv", (long long)m);
        if (!finite3(M.origin) || !finite3(M.edge_u) || !finite3(M.edge_v))
            return fail(PV3D_EINVAL, "module %lld is not finite", (long long)m);
        for (int c = 0; c < 3; c++)
            if (std::fabs(M.origin[c]) > kMaxCoord || std::fabs(M.edge_u[c]) > kMaxCoord || std::fabs(M.edge_v[c]) > kMaxCoord)
                return fail(PV3D_ERANGE, "module %lld beyond %.0e m", (long long)m, kMaxCoord);
        double cx = M.edge_u[1] * M.edge_v[2] - M.edge_u[2] * M.edge_v[1];
        double cy = M.edge_u[2] * M.edge_v[0] - M.edge_u[0] * M.edge_v[2];
        double cz = M.edge_u[0] * M.edge_v[1] - M.edge_u[1] * M.edge_v[0];
        if (!((cx * cx + cy * cy) + cz * cz > 0.0)) return fail(PV3D_EINVAL, "module %lld is degenerate", (long long)m);
        Module& D = hm[(size_t)m];
        memset(&D, 0, sizeof(D));
        for (int c = 0; c < 3; c++) {
            D.o[c] = M.origin[c];
            D.u[c] = M.edge_u[c];
            D.v[c] = M.edge_v[c];
        }
        // unit front normal u x v / |u x v|, the same IEEE operations the kernels use
        const double l = std::sqrt((cx * cx + cy * cy) + cz * cz);
        D.n[0] = cx / l;
        D.n[1] = cy / l;
        D.n[2] = cz / l;
    }
    std::vector<int32_t> seen((size_t)n_sub, 0);
    for (int32_t c = 0; c < n_cu * n_cv; c++) {
        if (cell_substring[c] < 0 || cell_substring[c] >= n_sub) return fail(PV3D_EINVAL, "cell %d: substring out of range", c);
        seen[(size_t)cell_substring[c]] = 1;
    }
    for (int32_t q = 0; q < n_sub; q++)
        if (!seen[(size_t)q]) return fail(PV3D_EINVAL, "substring %d owns no cell", q);
    int32_t n_str = 0;
    for (int64_t m = 0; m < n_mod; m++) {
        if (module_string[m] < 0 || module_string[m] >= n_mod) return fail(PV3D_EINVAL, "module %lld: bad string", (long long)m);
        n_str = std::max(n_str, module_string[m] + 1);
    }
    std::vector<int32_t> start((size_t)n_str + 1, 0), order((size_t)n_mod);
    for (int64_t m = 0; m < n_mod; m++) start[(size_t)module_string[m] + 1]++;
    for (int32_t q = 0; q < n_str; q++) {
        if (start[(size_t)q + 1] == 0) return fail(PV3D_EINVAL, "string %d has no module", q);
        if ((int64_t)start[(size_t)q + 1] * n_sub > 4096)
            return fail(PV3D_ERANGE, "string %d has more than 4096 substrings", q);
        start[(size_t)q + 1] += start[(size_t)q];
    }
    {
        std::vector<int32_t> cur(start.begin(), start.end() - 1);
        for (int64_t m = 0; m < n_mod; m++) order[(size_t)cur[(size_t)module_string[m]]++] = (int32_t)m;
    }
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    (void)hipSetDevice(ctx->device);
    Gen g;
    for (int c = 0; c < 3; c++) {
        g.lo[c] = INFINITY;
        g.hi[c] = -INFINITY;
    }
    // corners o, o+u, (o+u)+v, o+v of module m
    auto corner = [&](int64_t m, int q, int c) {
        const Module& D = hm[(size_t)m];
        return q == 0 ? D.o[c] : q == 1 ? D.o[c] + D.u[c] : q == 2 ? (D.o[c] + D.u[c]) + D.v[c] : D.o[c] + D.v[c];
    };
    for (int64_t m = 0; m < n_mod; m++) {
        if (n_trk > 0 && module_tracker[m] >= 0) continue;      // a tracker's reach counts instead
        for (int q = 0; q < 4; q++)
            for (int c = 0; c < 3; c++) {
                g.lo[c] = std::fmin(g.lo[c], corner(m, q, c));
                g.hi[c] = std::fmax(g.hi[c], corner(m, q, c));
            }
    }
    // a turn about the pivot keeps every corner within r of it: the cube P +- r
    for (int32_t t = 0; t < n_trk; t++) {
        double r = 0.0;
        for (int64_t m = 0; m < n_mod; m++) {
            if (module_tracker[m] != t) continue;
            for (int q = 0; q < 4; q++) {
                const double dx = corner(m, q, 0) - trackers[t].pivot[0], dy = corner(m, q, 1) - trackers[t].pivot[1],
                             dz = corner(m, q, 2) - trackers[t].pivot[2];
                const double l = std::sqrt((dx * dx + dy * dy) + dz * dz);
                r = l > r ? l : r;
            }
        }
        if (r > 0.0)
            for (int c = 0; c < 3; c++) {
                g.lo[c] = std::fmin(g.lo[c], trackers[t].pivot[c] - r);
                g.hi[c] = std::fmax(g.hi[c], trackers[t].pivot[c] + r);
            }
    }
    g.n_mod = n_mod;
    g.n_cu = n_cu;
    g.n_cv = n_cv;
    g.n_sub = n_sub;
    g.n_str = n_str;
    g.occluders = add_as_occluders ? 1 : 0;
    // cells of each substring, ascending (the order the string model adds them in)
    const int32_t cpm = n_cu * n_cv;
    std::vector<int32_t> sub_start((size_t)n_sub + 1, 0), sub_cell((size_t)cpm);
    for (int32_t c = 0; c < cpm; c++) sub_start[(size_t)cell_substring[c] + 1]++;
    for (int32_t q = 0; q < n_sub; q++) sub_start[(size_t)q + 1] += sub_start[(size_t)q];
    {
        std::vector<int32_t> cur(sub_start.begin(), sub_start.end() - 1);
        for (int32_t c = 0; c < cpm; c++) sub_cell[(size_t)cur[(size_t)cell_substring[c]]++] = c;
    }
    pv3d_status st = define_upload(ctx, g, hm, cell_substring, start, order, sub_start, sub_cell, trackers, n_trk,
                                   module_tracker);
    if (st) {
        free_gen(ctx, g);
        return st;
    }
    uint64_t h = ++ctx->next_handle;
    ctx->gens[h] = g;
    *gen_out = h;
    return PV3D_OK;
}

// Device arrays of a generator being defined (freed by the caller on failure).
static pv3d_status define_upload(pv3d_ctx* ctx, Gen& g, const std::vector<Module>& hm, const int32_t* cell_substring,
                                 const std::vector<int32_t>& start, const std::vector<int32_t>& order,
                                 const std::vector<int32_t>& sub_start, const std::vector<int32_t>& sub_cell,
                                 const pv3d_tracker* trackers, int32_t n_trk, const int32_t* module_tracker) {
    const int64_t n_mod = g.n_mod;
    const int32_t n_cu = g.n_cu, n_cv = g.n_cv, n_str = g.n_str, n_sub = g.n_sub;
    pv3d_status st;
    if ((st = ctx->dalloc((void**)&g.mods, sizeof(Module) * (size_t)n_mod, "modules"))) return st;
    if ((st = ctx->dalloc((void**)&g.cell_sub, 4 * (size_t)(n_cu * n_cv), "cell map"))) return st;
    if ((st = ctx->dalloc((void**)&g.str_start, 4 * (size_t)(n_str + 1), "string starts"))) return st;
    if ((st = ctx->dalloc((void**)&g.str_mods, 4 * (size_t)n_mod, "string modules"))) return st;
    if ((st = ctx->dalloc((void**)&g.sub_start, 4 * (size_t)(n_sub + 1), "substring starts"))) return st;
    if ((st = ctx->dalloc((void**)&g.sub_cell, 4 * (size_t)(n_cu * n_cv), "substring cells"))) return st;
    hipError_t e;
    if ((e = copy_in(ctx, g.mods, hm.data(), sizeof(Module) * (size_t)n_mod))) return hip_fail(e, "copy modules");
    if ((e = copy_in(ctx, g.cell_sub, cell_substring, 4 * (size_t)(n_cu * n_cv)))) return hip_fail(e, "copy cell map");
    if ((e = copy_in(ctx, g.str_start, start.data(), 4 * (size_t)(n_str + 1)))) return hip_fail(e, "copy strings");
    if ((e = copy_in(ctx, g.str_mods, order.data(), 4 * (size_t)n_mod))) return hip_fail(e, "copy strings");
    if ((e = copy_in(ctx, g.sub_start, sub_start.data(), 4 * (size_t)(n_sub + 1))))
        return hip_fail(e, "copy substrings");
    if ((e = copy_in(ctx, g.sub_cell, sub_cell.data(), 4 * (size_t)(n_cu * n_cv))))
        return hip_fail(e, "copy substrings");
    if (n_trk > 0) {
        std::vector<TrackerDev> td((size_t)n_trk);
        for (int32_t t = 0; t < n_trk; t++) {
            memset(&td[(size_t)t], 0, sizeof(TrackerDev));
            for (int c = 0; c < 3; c++) {
                td[(size_t)t].p[c] = trackers[t].pivot[c];
                td[(size_t)t].a[c] = trackers[t].axis[c];
            }
            td[(size_t)t].kind = trackers[t].kind;
        }
        if ((st = ctx->dalloc((void**)&g.trk, sizeof(TrackerDev) * (size_t)n_trk, "trackers"))) return st;
        if ((st = ctx->dalloc((void**)&g.mod_trk, 4 * (size_t)n_mod, "module trackers"))) return st;
        if ((e = copy_in(ctx, g.trk, td.data(), sizeof(TrackerDev) * (size_t)n_trk)))
            return hip_fail(e, "copy trackers");
        if ((e = copy_in(ctx, g.mod_trk, module_tracker, 4 * (size_t)n_mod)))
            return hip_fail(e, "copy module trackers");
        g.n_trk = n_trk;
    }
    return PV3D_OK;
}

pv3d_status pv3d_generator_define(pv3d_ctx* ctx, const pv3d_module* mods, int64_t n_mod, const int32_t* cell_substring,
                                  int32_t n_sub, const int32_t* module_string, int32_t add_as_occluders,
                                  uint64_t* gen_out) {
    return define_generator(ctx, mods, n_mod, cell_substring, n_sub, module_string, add_as_occluders, nullptr, 0,
                            nullptr, gen_out);
}

pv3d_status pv3d_generator_define_tracked(pv3d_ctx* ctx, const pv3d_module* mods, int64_t n_mod,
                                          const int32_t* cell_substring, int32_t n_sub, const int32_t* module_string,
                                          int32_t add_as_occluders, const pv3d_tracker* trackers, int32_t n_tracker,
                                          const int32_t* module_tracker, uint64_t* gen_out) {
    if (n_tracker < 1) return fail(PV3D_EINVAL, "a tracked generator needs at least one tracker");
    return define_generator(ctx, mods, n_mod, cell_substring, n_sub, module_string, add_as_occluders, trackers,
                            n_tracker, module_tracker, gen_out);
}

pv3d_status pv3d_generator_set_diode(pv3d_ctx* ctx, uint64_t gen, const pv3d_diode* d) {
    if (!ctx) return fail(PV3D_EINVAL, "null context");
    DiodeDev dd{};
    if (d) {
        const double v[7] = {d->isc_ref, d->g_ref, d->i0, d->a, d->rs, d->rsh, d->v_bypass};
        for (double x : v)
            if (!std::isfinite(x)) return fail(PV3D_EINVAL, "diode parameters must be finite");
        if (!(d->isc_ref > 0.0) || !(d->g_ref > 0.0) || !(d->i0 > 0.0) || !(d->a > 0.0) || !(d->rs >= 0.0) ||
            !(d->rsh > 0.0) || !(d->v_bypass >= 0.0))
            return fail(PV3D_EINVAL, "diode parameters out of range (isc_ref, g_ref, i0, a, rsh > 0; rs, v_bypass >= 0)");
        dd.isc = d->isc_ref;
        dd.gref = d->g_ref;
        dd.i0 = d->i0;
        dd.a = d->a;
        dd.rs = d->rs;
        dd.rsh = d->rsh;
        dd.vb = d->v_bypass;
        dd.on = 1;
    }
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto it = ctx->gens.find(gen);
    if (it == ctx->gens.end()) return fail(PV3D_ENOENT, "unknown generator %llu", (unsigned long long)gen);
    if (ctx->gen_in_use(gen)) return fail(PV3D_EBUSY, "generator %llu is used by a running job", (unsigned long long)gen);
    it->second.diode = dd;
    return PV3D_OK;
}

pv3d_status pv3d_generator_set_sky(pv3d_ctx* ctx, uint64_t gen, const double* svf) {
    if (!ctx) return fail(PV3D_EINVAL, "null context");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto it = ctx->gens.find(gen);
    if (it == ctx->gens.end()) return fail(PV3D_ENOENT, "unknown generator %llu", (unsigned long long)gen);
    Gen& g = it->second;
    if (g.n_trk > 0) return fail(PV3D_EINVAL, "sky view factors of a tracked generator change with its pose");
    if (ctx->gen_in_use(gen)) return fail(PV3D_EBUSY, "generator %llu is used by a running job", (unsigned long long)gen);
    const int64_t cells = g.n_mod * g.n_cu * g.n_cv;
    if (svf)
        for (int64_t c = 0; c < cells; c++)
            if (!(svf[c] >= 0.0 && svf[c] <= 1.0)) return fail(PV3D_EINVAL, "cell %lld: sky view factor not in [0, 1]", (long long)c);
    (void)hipSetDevice(ctx->device);
    HoldServing hold(ctx);
    (void)hipDeviceSynchronize();
    ctx->dfree(g.svf);
    g.svf = nullptr;
    if (!svf) return PV3D_OK;
    pv3d_status st;
    if ((st = ctx->dalloc((void**)&g.svf, 8 * (size_t)cells, "sky view factors"))) return st;
    hipError_t e = copy_in(ctx, g.svf, svf, 8 * (size_t)cells);
    if (e) {
        ctx->dfree(g.svf);
        g.svf = nullptr;
        return hip_fail(e, "copy sky view factors");
    }
    return PV3D_OK;
}

pv3d_status pv3d_sky_view(pv3d_ctx* ctx, uint64_t scene, uint64_t gen, const double* dirs, int64_t n_dir,
                          const pv3d_params* params, double* svf_out) {
    if (!ctx || !dirs || !svf_out || !params) return fail(PV3D_EINVAL, "null argument");
    if (n_dir < 1) return fail(PV3D_EINVAL, "n_dir %lld", (long long)n_dir);
    for (int64_t j = 0; j < n_dir; j++)
        if (!(dirs[3 * j + 2] > 0.0)) return fail(PV3D_EINVAL, "direction %lld is not above the horizon", (long long)j);
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto gi = ctx->gens.find(gen);
    if (gi == ctx->gens.end()) return fail(PV3D_ENOENT, "unknown generator %llu", (unsigned long long)gen);
    const Gen& g = gi->second;
    if (g.n_trk > 0) return fail(PV3D_EINVAL, "sky view factors of a tracked generator change with its pose");
    const int64_t cells = g.n_mod * g.n_cu * g.n_cv;
    // every direction is a sun of unit beam and no diffuse
    std::vector<double> in((size_t)(2 * n_dir), 0.0);
    for (int64_t j = 0; j < n_dir; j++) in[(size_t)j] = 1.0;
    pv3d_params p = *params;
    p.flags &= ~(PV3D_EXPORT_DEPTH | PV3D_EXPORT_BITS);
    pv3d_status st;
    if ((st = ctx->w.sky.ensure(ctx, 8 * (size_t)(2 * n_dir + 2 + 3 * n_dir + cells), "sky view"))) return st;
    double* d_pw = static_cast<double*>(ctx->w.sky.ptr);
    double* d_dirs = d_pw + 2 * n_dir + 2;
    double* d_svf = d_dirs + 3 * n_dir;
    pv3d_outputs o;
    memset(&o, 0, sizeof(o));
    o.power = d_pw;
    o.power_ref = d_pw + n_dir;
    o.energy = d_pw + 2 * n_dir;
    o.on_device = 1;
    if ((st = pv3d_evaluate(ctx, scene, gen, dirs, in.data(), in.data() + n_dir, in.data() + n_dir, n_dir, &p, &o,
                            nullptr)))
        return st;
    hipStream_t s = ctx->stream;
    bool ovf = false;
    if ((st = ctx->read_overflow(n_dir, s, &ovf))) return st;
    if (ovf) return fail(PV3D_ERANGE, "internal buffer overflow");
    hipError_t e;
    if ((e = hipMemcpyAsync(d_dirs, dirs, 24 * (size_t)n_dir, hipMemcpyHostToDevice, s))) return hip_fail(e, "copy directions");
    if ((e = launch_svf(g.mods, g.n_cu * g.n_cv, cells, d_dirs, n_dir, static_cast<const uint32_t*>(ctx->w.counts.ptr),
                        p.k, d_svf, s)))
        return hip_fail(e, "sky view launch");
    if ((e = hipMemcpyAsync(svf_out, d_svf, 8 * (size_t)cells, hipMemcpyDeviceToHost, s))) return hip_fail(e, "copy sky view");
    if ((e = hipStreamSynchronize(s))) return hip_fail(e, "sky view");
    return PV3D_OK;
}

pv3d_status pv3d_generator_release(pv3d_ctx* ctx, uint64_t gen) {
    if (!ctx) return fail(PV3D_EINVAL, "null context");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto it = ctx->gens.find(gen);
    if (it == ctx->gens.end()) return fail(PV3D_ENOENT, "unknown generator %llu", (unsigned long long)gen);
    if (ctx->gen_in_use(gen)) return fail(PV3D_EBUSY, "generator %llu is used by a running job", (unsigned long long)gen);
    (void)hipSetDevice(ctx->device);
    HoldServing hold(ctx);
    (void)hipDeviceSynchronize();
    free_gen(ctx, it->second);
    ctx->gens.erase(it);
    return PV3D_OK;
}

pv3d_status pv3d_sun_cooper(double lat_deg, const int32_t* day, const double* solar_hour, int64_t n, double* out) {
    if (n < 0 || (n && (!day || !solar_hour || !out))) return fail(PV3D_EINVAL, "bad arguments");
    const double deg = M_PI / 180.0;
    const double phi = lat_deg * deg;
    for (int64_t i = 0; i < n; i++) {
        double decl = 23.45 * std::sin(360.0 * (284.0 + (double)day[i]) / 365.0 * deg) * deg;
        double om = 15.0 * (solar_hour[i] - 12.0) * deg;
        out[3 * i + 0] = -std::cos(decl) * std::sin(om);
        out[3 * i + 1] = std::sin(decl) * std::cos(phi) - std::cos(decl) * std::sin(phi) * std::cos(om);
        out[3 * i + 2] = std::sin(decl) * std::sin(phi) + std::cos(decl) * std::cos(phi) * std::cos(om);
    }
    return PV3D_OK;
}

pv3d_status pv3d_evaluate(pv3d_ctx* ctx, uint64_t scene, uint64_t gen, const double* sun_xyz, const double* dni,
                          const double* d_poa, const double* dt_h, int64_t n_sun, const pv3d_params* params,
                          pv3d_outputs* out, void* hip_stream) {
    if (!ctx || !out) return fail(PV3D_EINVAL, "null argument");
    pv3d_status st;
    if ((st = check_params(params))) return st;
    if ((st = check_sweep(sun_xyz, dni, d_poa, dt_h, n_sun))) return st;
    if (!out->power || !out->power_ref || !out->energy) return fail(PV3D_EINVAL, "power, power_ref and energy are required");
    if ((params->flags & PV3D_EXPORT_DEPTH) && !out->depth_maps) return fail(PV3D_EINVAL, "EXPORT_DEPTH needs depth_maps");
    if ((params->flags & PV3D_EXPORT_BITS) && !out->shaded_bits) return fail(PV3D_EINVAL, "EXPORT_BITS needs shaded_bits");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto si = ctx->scenes.find(scene);
    if (si == ctx->scenes.end()) return fail(PV3D_ENOENT, "unknown scene %llu", (unsigned long long)scene);
    auto gi = ctx->gens.find(gen);
    if (gi == ctx->gens.end()) return fail(PV3D_ENOENT, "unknown generator %llu", (unsigned long long)gen);
    (void)hipSetDevice(ctx->device);
    hipStream_t s = hip_stream ? static_cast<hipStream_t>(hip_stream) : ctx->stream;
    ctx->stream_in_use = s;
    ctx->per_sun_ran = true;
    const Scene& sc = si->second;
    const Gen& g = gi->second;
    const pv3d_params& p = *params;
    if ((int64_t)p.k * g.n_cu > 4095 || (int64_t)p.k * g.n_cv > 4095)
        return fail(PV3D_ERANGE, "k * cells per module side exceeds 4095 samples");
    const int64_t cells = g.n_mod * g.n_cu * g.n_cv;
    const int64_t words = (p.k * p.k + 31) / 32;
    const bool want_maps = (p.flags & PV3D_EXPORT_DEPTH) != 0, want_bits = (p.flags & PV3D_EXPORT_BITS) != 0;
    const int64_t N2 = (int64_t)p.map_n * p.map_n;
    hipError_t e;

    // device views of the outputs: the caller's arrays, or context buffers copied back at the end
    uint32_t *d_counts, *d_maps = nullptr, *d_bits = nullptr;
    double *d_pw, *d_pr, *d_en;
    if (out->on_device) {
        if ((st = ctx->w.counts.ensure(ctx, 4 * (size_t)std::max<int64_t>(n_sun * cells, 1), "counts"))) return st;
        d_counts = out->cell_counts ? out->cell_counts : static_cast<uint32_t*>(ctx->w.counts.ptr);
        d_pw = out->power;
        d_pr = out->power_ref;
        d_en = out->energy;
        d_maps = want_maps ? out->depth_maps : nullptr;
        d_bits = want_bits ? out->shaded_bits : nullptr;
    } else {
        if ((st = ctx->w.counts.ensure(ctx, 4 * (size_t)std::max<int64_t>(n_sun * cells, 1), "counts"))) return st;
        if ((st = ctx->w.outd.ensure(ctx, 8 * (size_t)(2 * n_sun + 2), "power"))) return st;
        d_counts = static_cast<uint32_t*>(ctx->w.counts.ptr);
        d_pw = static_cast<double*>(ctx->w.outd.ptr);
        d_pr = d_pw + n_sun;
        d_en = d_pr + n_sun;
        if (want_maps) {
            if ((st = ctx->w.maps.ensure(ctx, 4 * (size_t)std::max<int64_t>(n_sun * N2, 1), "exported depth maps"))) return st;
            d_maps = static_cast<uint32_t*>(ctx->w.maps.ptr);
        }
        if (want_bits) {
            if ((st = ctx->w.bits.ensure(ctx, 4 * (size_t)std::max<int64_t>(n_sun * cells * words, 1), "exported bits"))) return st;
            d_bits = static_cast<uint32_t*>(ctx->w.bits.ptr);
        }
    }
    PathSizes z = path_sizes(sc, g, p, n_sun);
    if ((st = ctx->ensure_path(z, g, p.map_n, !want_maps && (p.flags & PV3D_SEPARATE_TEST)))) return st;
    double* d_sweep = static_cast<double*>(ctx->w.sweep.ptr);
    double *d_sun = d_sweep, *d_dni = d_sweep + 3 * n_sun, *d_dpoa = d_dni + n_sun, *d_dt = d_dpoa + n_sun;
    // the previous evaluation (perhaps on another stream) may still read the sweep buffer
    if ((st = ctx->wait_previous(s))) return st;
    if (n_sun > 0) {
        if ((st = ctx->stage_reserve(8 * 6 * (size_t)n_sun + 4 * 256))) return st;
        if ((st = ctx->stage(sun_xyz, 24 * (size_t)n_sun, d_sun, s))) return st;
        if ((st = ctx->stage(dni, 8 * (size_t)n_sun, d_dni, s))) return st;
        if ((st = ctx->stage(d_poa, 8 * (size_t)n_sun, d_dpoa, s))) return st;
        if ((st = ctx->stage(dt_h, 8 * (size_t)n_sun, d_dt, s))) return st;
        if ((st = ctx->stage_done(s))) return st;
    }
    if ((st = ctx->run_path(sc, g, p, sun_xyz, n_sun, d_sun, d_dni, d_dpoa, d_dt, d_counts, d_pw, d_pr, d_en,
                            d_maps, d_bits, s)))
        return st;
    ctx->last_n_sun = n_sun;
    if (!out->on_device) {
        bool ovf = false;
        if ((st = ctx->read_overflow(n_sun, s, &ovf))) return st;
        if (ovf) return fail(PV3D_ERANGE, "internal buffer overflow");
        if (out->cell_counts && n_sun &&
            (e = hipMemcpyAsync(out->cell_counts, d_counts, 4 * (size_t)(n_sun * cells), hipMemcpyDeviceToHost, s)))
            return hip_fail(e, "copy counts");
        if (n_sun && (e = hipMemcpyAsync(out->power, d_pw, 8 * (size_t)n_sun, hipMemcpyDeviceToHost, s))) return hip_fail(e, "copy power");
        if (n_sun && (e = hipMemcpyAsync(out->power_ref, d_pr, 8 * (size_t)n_sun, hipMemcpyDeviceToHost, s)))
            return hip_fail(e, "copy power_ref");
        if ((e = hipMemcpyAsync(out->energy, d_en, 16, hipMemcpyDeviceToHost, s))) return hip_fail(e, "copy energy");
        if (want_maps && n_sun &&
            (e = hipMemcpyAsync(out->depth_maps, d_maps, 4 * (size_t)(n_sun * N2), hipMemcpyDeviceToHost, s)))
            return hip_fail(e, "copy depth maps");
        if (want_bits && n_sun &&
            (e = hipMemcpyAsync(out->shaded_bits, d_bits, 4 * (size_t)(n_sun * cells * words), hipMemcpyDeviceToHost, s)))
            return hip_fail(e, "copy bits");
        if ((e = hipStreamSynchronize(s))) return hip_fail(e, "synchronize");
    } else {
        if ((e = hipGetLastError())) return hip_fail(e, "launch");
    }
    return PV3D_OK;
}

pv3d_status pv3d_evaluate_noalloc(pv3d_ctx* ctx, uint64_t scene, uint64_t gen, const double* sun_xyz,
                                  const double* dni, const double* d_poa, const double* dt_h, int64_t n_sun,
                                  const pv3d_params* params, pv3d_outputs* out, void* hip_stream) {
    if (!ctx || !out) return fail(PV3D_EINVAL, "null argument");
    pv3d_status st;
    if ((st = check_params(params))) return st;
    if ((st = check_sweep(sun_xyz, dni, d_poa, dt_h, n_sun))) return st;
    if (!out->on_device) return fail(PV3D_EINVAL, "the no-allocation form writes device outputs only (on_device = 1)");
    if (!out->power || !out->power_ref || !out->energy) return fail(PV3D_EINVAL, "power, power_ref and energy are required");
    if ((params->flags & PV3D_EXPORT_DEPTH) && !out->depth_maps) return fail(PV3D_EINVAL, "EXPORT_DEPTH needs depth_maps");
    if ((params->flags & PV3D_EXPORT_BITS) && !out->shaded_bits) return fail(PV3D_EINVAL, "EXPORT_BITS needs shaded_bits");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto si = ctx->scenes.find(scene);
    if (si == ctx->scenes.end()) return fail(PV3D_ENOENT, "unknown scene %llu", (unsigned long long)scene);
    auto gi = ctx->gens.find(gen);
    if (gi == ctx->gens.end()) return fail(PV3D_ENOENT, "unknown generator %llu", (unsigned long long)gen);
    const Scene& sc = si->second;
    const Gen& g = gi->second;
    const pv3d_params& p = *params;
    if ((int64_t)p.k * g.n_cu > 4095 || (int64_t)p.k * g.n_cv > 4095)
        return fail(PV3D_ERANGE, "k * cells per module side exceeds 4095 samples");
    const bool want_maps = (p.flags & PV3D_EXPORT_DEPTH) != 0, want_bits = (p.flags & PV3D_EXPORT_BITS) != 0;
    const bool own_map = !want_maps && (p.flags & PV3D_SEPARATE_TEST);
    const bool own_counts = out->cell_counts == nullptr;
    PathSizes z = path_sizes(sc, g, p, n_sun);
    if (z.rec_cap > INT32_MAX || z.bin_cap > INT32_MAX) return fail(PV3D_ERANGE, "scene too large for 32-bit bin indices");
    int64_t n_up = 0;
    for (int64_t i = 0; i < n_sun; i++)
        if (sun_xyz[3 * i + 2] > 0.0) n_up++;
    // the smallest layout: one lane with room for one sun
    const size_t least = carve_bytes(z, g, p.k, p.map_n, own_map, own_counts, 1, 1, n_up);
    if (least > kScratchBytes)
        return fail(PV3D_ERANGE,
                    "the evaluation needs %zu bytes of work memory and the static scratch holds %zu "
                    "(a smaller bin_limit, fewer triangles or fewer suns per call need less)",
                    least, kScratchBytes);
    (void)hipSetDevice(ctx->device);
    if (!ctx->scratch) return fail(PV3D_EDEVICE, "no static scratch on device %d", ctx->device);
    hipStream_t s = hip_stream ? static_cast<hipStream_t>(hip_stream) : ctx->stream;
    ctx->stream_in_use = s;
    ctx->per_sun_ran = true;
    // the evaluation works in buffers carved from the scratch; the context's own
    // work buffers are set aside and come back untouched. No timing: its events
    // would be created here.
    struct Carved {
        Ctx* c;
        Work saved;
        uint32_t mask;
        explicit Carved(Ctx* ctx) : c(ctx), saved(ctx->w), mask(ctx->prof.mask) {
            c->w = Work{};
            c->prof.mask = 0;
            c->carving = true;
            c->carve_used = 0;
        }
        ~Carved() {
            c->carving = false;
            c->w = saved;
            c->prof.mask = mask;
        }
    } carved(ctx);
    hipError_t e;
    uint32_t* d_counts = out->cell_counts;
    if (own_counts) {
        if ((st = ctx->w.counts.ensure(ctx, 4 * (size_t)std::max<int64_t>(n_sun * z.cells, 1), "counts"))) return st;
        d_counts = static_cast<uint32_t*>(ctx->w.counts.ptr);
    }
    if ((st = ctx->ensure_path(z, g, p.map_n, own_map))) return st;
    double* d_sweep = static_cast<double*>(ctx->w.sweep.ptr);
    double *d_sun = d_sweep, *d_dni = d_sweep + 3 * n_sun, *d_dpoa = d_dni + n_sun, *d_dt = d_dpoa + n_sun;
    // the scratch is the previous call's work memory until that call's kernels end
    if ((st = ctx->wait_previous(s))) return st;
    if (n_sun > 0) {
        const double* src[4] = {sun_xyz, dni, d_poa, dt_h};
        double* dst[4] = {d_sun, d_dni, d_dpoa, d_dt};
        const size_t bytes[4] = {24 * (size_t)n_sun, 8 * (size_t)n_sun, 8 * (size_t)n_sun, 8 * (size_t)n_sun};
        for (int i = 0; i < 4; i++)
            if ((e = hipMemcpyAsync(dst[i], src[i], bytes[i], hipMemcpyHostToDevice, s))) return hip_fail(e, "copy the sweep");
    }
    if ((st = ctx->run_path(sc, g, p, sun_xyz, n_sun, d_sun, d_dni, d_dpoa, d_dt, d_counts, out->power,
                            out->power_ref, out->energy, want_maps ? out->depth_maps : nullptr,
                            want_bits ? out->shaded_bits : nullptr, s)))
        return st;
    if ((e = hipGetLastError())) return hip_fail(e, "launch");
    return PV3D_OK;
}

pv3d_status pv3d_path_stats(pv3d_ctx* ctx, int64_t out[4]) {
    if (!ctx || !out) return fail(PV3D_EINVAL, "null argument");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    for (int i = 0; i < 4; i++) out[i] = 0;
    const int64_t n = ctx->last_n_sun;
    if (n <= 0 || !ctx->w.ctr.ptr) return PV3D_OK;
    (void)hipSetDevice(ctx->device);
    hipError_t e;
    if (ctx->ws_recorded && (e = hipEventSynchronize(ctx->ws_ev))) return hip_fail(e, "wait for the evaluation");
    std::vector<SunCounters> h((size_t)n);
    // on the context's own stream: the null stream would also wait for a live serving launch
    if ((e = hipMemcpyAsync(h.data(), ctx->w.ctr.ptr, sizeof(SunCounters) * (size_t)n, hipMemcpyDeviceToHost,
                            ctx->stream)) ||
        (e = hipStreamSynchronize(ctx->stream)))
        return hip_fail(e, "read the sun counters");
    out[0] = n;
    for (const SunCounters& c : h) {
        out[1] += c.n_rec;
        out[2] += c.n_large;
        out[3] += (int64_t)(c.pairs & 0xFFFFFFFFull);
    }
    return PV3D_OK;
}

pv3d_status pv3d_profile_enable(pv3d_ctx* ctx, uint32_t stage_mask) {
    if (!ctx) return fail(PV3D_EINVAL, "null context");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (stage_mask >> PV3D_N_STAGES) return fail(PV3D_EINVAL, "unknown stage bits 0x%x", stage_mask);
    (void)hipSetDevice(ctx->device);
    hipError_t e = ctx->prof.collect();
    if (e != hipSuccess) return hip_fail(e, "collect timings");
    if (stage_mask == 0) ctx->prof.reset();
    if (stage_mask != 0 && ctx->prof.mask == 0) {
        // the origin of the launch intervals; the context stream is idle between calls
        for (auto& v : ctx->prof.spans) v.clear();
        if ((e = hipEventRecord(ctx->prof.ref, ctx->stream)) != hipSuccess) return hip_fail(e, "record time origin");
        if ((e = hipEventSynchronize(ctx->prof.ref)) != hipSuccess) return hip_fail(e, "record time origin");
    }
    ctx->prof.mask = stage_mask;
    return PV3D_OK;
}

pv3d_status pv3d_profile_sample(pv3d_ctx* ctx, int32_t every) {
    if (!ctx) return fail(PV3D_EINVAL, "null context");
    if (every < 1) return fail(PV3D_EINVAL, "every %d", every);
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    ctx->prof.every = every;
    return PV3D_OK;
}

pv3d_status pv3d_profile_busy(pv3d_ctx* ctx, int32_t stage, double* busy_ms, int64_t* suns) {
    if (!ctx || !busy_ms || !suns) return fail(PV3D_EINVAL, "null argument");
    if (stage < 0 || stage >= PV3D_N_STAGES) return fail(PV3D_EINVAL, "stage %d", stage);
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    (void)hipSetDevice(ctx->device);
    hipError_t e = ctx->prof.collect();
    if (e != hipSuccess) return hip_fail(e, "collect timings");
    *busy_ms = ctx->prof.busy_ms(stage);
    *suns = ctx->prof.suns[stage];
    return PV3D_OK;
}

pv3d_status pv3d_profile_read(pv3d_ctx* ctx, int32_t stage, double* total_ms, int64_t* launches) {
    if (!ctx || !total_ms || !launches) return fail(PV3D_EINVAL, "null argument");
    if (stage < 0 || stage >= PV3D_N_STAGES) return fail(PV3D_EINVAL, "stage %d", stage);
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    (void)hipSetDevice(ctx->device);
    hipError_t e = ctx->prof.collect();
    if (e != hipSuccess) return hip_fail(e, "collect timings");
    *total_ms = ctx->prof.total_ms[stage];
    *launches = ctx->prof.launches[stage];
    return PV3D_OK;
}

}  // extern "C"
