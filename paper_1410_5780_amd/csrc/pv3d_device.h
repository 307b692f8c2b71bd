// Device-side data layout and kernel entry points of libpv3d (gfx950).
//
// Light space of one sun (Sec. 2, Step 3 of arXiv:1410.5780): an orthographic
// view along d = -s whose window is the generator's footprint seen from the
// sun. x, y are texel coordinates along the image axes e1, e2; z is depth in
// units of 2^-24 of the range [near side of the scene's bounding sphere,
// generator's farthest corner]. Pixel (i, j) is sampled at its centre
// (i + 1/2, j + 1/2); the depth picture keeps the nearest depth per pixel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pv3d {

constexpr int kSubBits = 8;                    // vertices snap to 1/256 texel
constexpr uint32_t kDepthMax = 0xFFFFFFu;      // 24-bit depth, 2^24 - 1 = farthest
constexpr double kGuard = 2097152.0;           // 2^21 texels: clip square for huge triangles
constexpr int kWave = 64;

// Per-sun view: 128 bytes.
struct View {
    double e1[3], e2[3], d[3];
    double ox, oy, itx, ity;   // texel x = (p.e1 - ox) * itx, y = (p.e2 - oy) * ity
    double znear, izd;         // depth z = (p.d - znear) * izd
    int32_t valid;             // 0: nothing drawn or tested (sun down / all modules back-lit)
    int32_t pad;
};

// Per-module generator data, 128 bytes: geometry and unit front normal.
struct Module {
    double o[3], u[3], v[3];
    double n[3];
    double pad[4];
};

// Set-up triangle ready for raster: 80 bytes.
// Edge k at pixel (i, j): E = e0[k] + 256 * (a[k] * i + b[k] * j); the pixel
// centre is inside when all three are >= 0 (the -1 of non top-left edges is
// folded into e0). Depth: floor((z0 + i * gx + j * gy) / 2^16), clamped.
struct TriRec {
    int64_t e0[3];
    int64_t z0, gx, gy;
    int32_t a[3], b[3];
    int16_t ilo, ihi, jlo, jhi;   // covered pixels lie in [ilo, ihi] x [jlo, jhi]
};
static_assert(sizeof(TriRec) == 80, "TriRec layout");

// Per-sun scratch counters, one slot per sun.
struct SunCounters {
    int32_t n_rec;      // set-up triangles written
    int32_t n_large;    // triangles handled by every tile instead of binned
    int32_t overflow;   // 1 if a buffer was too small for this sun
    int32_t pad;
    unsigned long long pairs;   // pair mode: items << 32 | (item, tile) pairs taken
};

// An item of the per-sun path's pair mode: a binned record (id >= 0) or a
// module's sample box (id = -(m + 1)), owning pairs [start, start + box
// size) of the sun's (item, tile-in-box) pair space.
struct PairItem {
    int32_t id, start;
    uint32_t xr, yr;    // tile box: x0 | x1 << 16, y0 | y1 << 16
};
constexpr int kPairChunk = 256;     // pairs per chunk of the counting and scatter passes

// Where one sun's triangle set-up and binning write. A bin entry is a
// triangle record id (>= 0) or a module -(m + 1) whose samples may fall in
// the tile.
struct BinBuffers {
    TriRec* rec;
    int32_t rec_cap;
    int32_t* large;        // [rec_cap] record ids of triangles every tile checks
    int32_t* tile_count;   // [n_tiles] (zero between suns)
    int32_t* tile_start;   // [n_tiles + 1]
    int32_t* tile_cursor;  // [n_tiles]
    int32_t* bins;         // [bin_cap]
    int4* modbox;          // [n_mod] tile range (x0, x1, y0, y1) of each module's samples; x0 > x1: none
    int32_t* tile_list;    // [4 n_tiles] work items of the tile pass, heaviest first (nullptr: one per tile)
    int32_t* list_ctr;     // [3] items listed, next item to take, first light item (the scan sets all three)
    int32_t split_at;      // list order: < 0 tile order; else heaviest first, tiles with more
                           // entries than split_at > 0 as four quadrant items
    // pair mode (pitems != nullptr): the triangle set-up only lays out items
    // in pair space; counting and scatter then take the pairs in chunks
    PairItem* pitems;      // [item_cap]
    int32_t* pchunk;       // [bin_cap / kPairChunk + 1] item holding the first pair of each chunk
    unsigned long long* pctr;   // this sun's SunCounters::pairs
    int32_t item_cap;
    int32_t bin_cap;
    int32_t tile;          // tile edge in texels
    int32_t ntx;           // tiles per row
    int32_t n_tiles;
    int32_t large_tiles;   // triangles touching more tiles than this go to the large list
};

// A work item of the tile pass: tile << 3 | part, part 0..3 a 32 x 32 quadrant
// (of a 64-texel tile) and kWholeTile the whole tile.
constexpr int32_t kWholeTile = 4;

// What the tile kernel writes for one sun.
struct TileOut {
    uint32_t* map;         // depth picture to export, or nullptr
    uint32_t* counts;      // [n_cells] shaded samples (accumulated; zero beforehand)
    uint32_t* bits;        // [n_cells][words] shaded flags (accumulated), or nullptr
    int32_t test;          // 1: depth-check the samples inside the tile
    int32_t sparse;        // 1: evaluate the picture only at sample texels (no export)
};

// Tile grid of one evaluation: tile edge, tiles per row, tile count, and the
// 32-bit words of a per-sun mask with one bit per tile.
struct TileGrid {
    int32_t tile, ntx, n_tiles, words;
};

// Generator as the kernels see it.
// A tracker (Sec. 3.4; ideal tracking): pivot, horizontal unit axis, kind
// 1 (one axis) or 2 (two axes).
struct TrackerDev {
    double p[3], a[3];
    int32_t kind, pad;
};

// Single-diode cell model (Step 4's diode model, parameters given): the
// photocurrent at irradiance G is isc * G / gref; a = n k T / q; rs, rsh the
// series and shunt resistances; vb the bypass diode's forward voltage.
// on = 0: ideal bypass-diode strings instead.
struct DiodeDev {
    double isc, gref, i0, a, rs, rsh, vb;
    int32_t on, pad;
};

struct GenDev {
    const Module* mods;
    const Module* mods_sun;     // trackers: [n_sun][n_mod] modules posed per sun (nullptr: fixed modules)
    int32_t n_mod, n_cu, n_cv, n_sub, n_str;
    int32_t occluders;
    const int32_t* cell_sub;    // [n_cu*n_cv]
    const int32_t* str_start;   // [n_str + 1] CSR of modules per string
    const int32_t* str_mods;    // [n_mod]
    const int32_t* sub_start;   // [n_sub + 1] CSR of the cells of each substring of a module
    const int32_t* sub_cell;    // [n_cu*n_cv] cell indices, ascending within each substring
    const double* svf;          // [n_cells] share of the diffuse sky each cell sees (nullptr: all of it)
    DiodeDev diode;
};

struct SceneDev {
    const double* xyz;
    const int32_t* tri;
    const double* cbox;     // [ceil(n_tri / 256)][6] vertex box (lo xyz, hi xyz) of each block of 256 triangles
    int64_t n_vert, n_tri;
};
constexpr int kTriBlock = 256;

// ---- group launches of the per-sun path ----------------------------------
// Up to kMaxGroup consecutive suns share each launch of the per-sun path
// (triangle set-up, pair count, scan, pair scatter, tile pass), so the five
// dependent launches and their ramp-up and drain are paid once per group,
// and every launch has a group's work to spread over the GPU. Each sun keeps
// its own bins, records and outputs; nothing is shared between the suns of a
// group, so every result is the one the sun gets alone.
constexpr int kMaxGroup = 32;

// Head of a sun's work list: item count, next item, first light item (words 0-2), then a
// light-tile counter per XCD at words kXcdStride (j + 1), 128 bytes apart; the items follow
// at word kListHead.
constexpr int kXcds = 8;
constexpr int kXcdStride = 32;
constexpr int kListHead = kXcdStride * (kXcds + 1);

// One sun of a group: the descriptors live in device memory, so the kernels
// take this sun's buffers by reference without copying them.
struct GroupSun {
    BinBuffers bb;           // its records, bins, tile counters, work list and pair space
    TileOut out;             // its counts, flags and picture
    GenDev g;                // the generator as it sees it (trackers: its posed modules)
    const uint32_t* tmask;   // its tile mask (nullptr: every tile)
    int64_t s;               // its index in the sweep
};

struct SunGroup {
    int32_t n;               // suns in the group, 1..kMaxGroup
    int32_t pad[3];
    GroupSun sun[kMaxGroup];
};

// ---- persistent launch: every (job, sun) item of a batch in one launch ----
// Phases of one item, in order; a phase is split into units that any
// workgroup may take.
enum : int32_t {
    kPhIdle = 0,      // slot holds no item
    kPhSetup = 1,     // 1 unit: view, module terms, tile mask
    kPhTri = 2,       // a unit per kTriPerUnit triangles (and modules): set-up and tile counts
    kPhScan = 3,      // 1 unit: scan of the tile counts, list of non-empty tiles, capacity check
    kPhScatter = 4,   // a unit per kScatterPerUnit records: bins
    kPhTile = 5,      // a unit per listed tile: raster and sample depth check
    kPhLoss = 6,      // 1 unit: string powers of the sun
    kPhAdmit = 7,     // serving: a workgroup is putting a newly published item into the slot
};
constexpr int32_t kTriPerUnit = 1024;
constexpr int32_t kScatterPerUnit = 2048;

// One job as the persistent kernel sees it (device pointers).
struct PJob {
    SceneDev sc;
    GenDev g;
    const double* sun;       // [n_sun][3]
    const double* dni;       // [n_sun]
    const double* dpoa;      // [n_sun]
    uint32_t* counts;        // [n_sun][cells], zero beforehand
    double* power;           // [n_sun], zero beforehand (suns below the horizon stay zero)
    double* power_ref;       // [n_sun]
    double* energy;          // [2]
    const double* dt;        // [n_sun]
    const double* sphere;    // scene bounding sphere (centre, radius)
    const double* fu;        // sample tables
    const double* fv;
    int64_t n_sun, cells;
    int32_t n, k, tile, sparse, use_mask, large_tiles, ntx, n_tiles, words, n_items;
    uint32_t done_target;    // job_done value once every item of the job is done
    uint32_t ovf_base;       // job_overflow value when the job started (more: a sun overflowed)
    uint32_t seq;            // serving: completion tag written to the report word
    int32_t pad2;
};

// (job, sun) of one item; the items of a job are consecutive.
struct PItem {
    int32_t job, sun;
};

// Work buffers of one slot (the item it holds).
struct PSlotBufs {
    TriRec* rec;
    int32_t* large;
    int32_t* bins;
    int32_t* tile_count;     // zero between items
    int32_t* tile_start;
    int32_t* tile_cursor;
    int32_t* tile_list;      // non-empty tiles of the item
    int4* modbox;
    View* view;
    double* beam;
    int32_t* bias;
    uint32_t* tmask;
    SunCounters* ctr;
};

// Queue state of one slot, alone in a 128-byte line. word packs the phase
// (bits 56-63), its unit count (bits 32-55) and the next unit to hand out
// (bits 0-31): a workgroup takes a unit with one atomic add and knows from
// the value it got which phase the unit belongs to.
struct alignas(128) PSlotState {
    unsigned long long word;
    uint32_t done;           // units of the current phase completed
    int32_t item;            // item held (its position in the launch's item order)
    int32_t n_list;          // tiles listed by the scan
    int32_t overflow;        // 1: a capacity was exceeded, the host evaluates the sun again
    int32_t job, sun;        // what the item is
    int32_t pad[24];
};
static_assert(sizeof(PSlotState) == 128, "PSlotState layout");

struct PSched {
    uint32_t next_item;          // next item to admit
    uint32_t items_done;
    uint32_t n_items;
    uint32_t abort;              // 1: the watchdog saw no progress; every workgroup leaves
    unsigned long long units;    // units completed (statistics, watchdog progress)
    uint32_t n_overflow;         // items listed in overflow_items
    // serving: device copies of the host's words, refreshed by a few polling workgroups
    uint32_t pub_dev;            // items published
    uint32_t stop_dev;           // stop asked
    int32_t busy;                // slots holding an item
};

struct PLaunch {
    const PJob* jobs;
    const PItem* items;
    const PSlotBufs* slots;
    PSlotState* state;
    PSched* sched;
    uint32_t* job_done;          // [n_jobs] items finished
    int32_t* job_overflow;       // [n_jobs] 1: an item was left to the host
    int32_t* overflow_items;     // [n_items]
    int32_t n_slots, rec_cap, bin_cap;
    int32_t groups;              // 8: slot i is served by the XCD whose id is i % 8; 1: by every XCD
    long long stall_ticks;       // wall-clock ticks without progress before the watchdog fires
    // serving: items arrive while the launch runs
    int32_t serve;               // 1: take items from feed instead of items
    uint32_t feed_cap;           // entries of the feed ring
    const unsigned long long* feed;   // host memory: ring of items, (job slot << 32) | sun
    const uint32_t* feed_pub;    // host memory: items published so far
    const uint32_t* stop_flag;   // host memory: nonzero asks the launch to end once idle
    uint32_t* report;            // host memory: [job slots] completion tag of the last job done
    long long idle_ticks;        // wall-clock ticks of idleness before the launch ends by itself
};

// ---- launch wrappers (pv3d_kernels.hip) -----------------------------------
hipError_t launch_bounds(const SceneDev& sc, const GenDev& g, double* partial, int32_t n_part,
                         double* sphere, hipStream_t st);
int32_t bounds_partials(int64_t n_points);
hipError_t launch_sample_tables(double* fu, double* fv, int32_t k, int32_t n_cu, int32_t n_cv,
                                hipStream_t st);
hipError_t launch_setup(const double* sun, int64_t n_sun, const double* dni, const GenDev& g,
                        const double* sphere, int32_t n, View* views, double* beam, int32_t* bias,
                        const TileGrid& tg, uint32_t* tmask, hipStream_t st);
hipError_t launch_pose(const double* sun, int64_t n_sun, const Module* rest, int32_t n_mod, const TrackerDev* trk,
                       const int32_t* mod_trk, Module* posed, hipStream_t st);
hipError_t launch_box_sphere(const double lo[3], const double hi[3], double* sphere, hipStream_t st);
// Group launches: grp points to the group's descriptor in device memory, n_sun is grp->n
// (known on the host), the arguments after it are shared by every sun of the group.
hipError_t launch_tri_setup_group(const SunGroup* grp, int32_t n_sun, const View* views, const SceneDev& sc,
                                  const GenDev& g, const int32_t* bias, int32_t n, SunCounters* ctr, hipStream_t st);
hipError_t launch_pair_count_group(const SunGroup* grp, int32_t grid, hipStream_t st);
hipError_t launch_bin_scan_group(const SunGroup* grp, int32_t n_sun, int32_t n_tiles, hipStream_t st);
hipError_t launch_pair_scatter_group(const SunGroup* grp, int32_t grid, hipStream_t st);
hipError_t launch_raster_group(const SunGroup* grp, int32_t n_sun, bool listed, int32_t tile, int32_t n_tiles,
                               const View* views, const SunCounters* ctr, int32_t n, const int32_t* bias,
                               int32_t n_mod, const double* fu, const double* fv, int32_t k, int32_t n_cu,
                               int32_t cap_per_cu, hipStream_t st);
hipError_t launch_sample_test(int64_t s, const View* views, const GenDev& g, const double* beam,
                              const int32_t* bias, const double* fu, const double* fv, int32_t k,
                              const uint32_t* map, int32_t n, uint32_t* counts, uint32_t* bits,
                              hipStream_t st);
// Losses of suns [s0, s1) (every array indexed by the sun's own index).
hipError_t launch_loss(int64_t s0, int64_t s1, const double* sun, const double* beam, const uint32_t* counts,
                       const double* d_poa, const GenDev& g, int32_t k, double* power,
                       double* power_ref, const SunCounters* ctr, hipStream_t st);
hipError_t launch_energy(int64_t n_sun, const double* power, const double* power_ref,
                         const double* dt, double* energy, hipStream_t st);
hipError_t launch_svf(const Module* mods, int32_t cpm, int64_t n_cells, const double* dirs, int64_t n_dir,
                      const uint32_t* counts, int32_t k, double* svf, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st);
hipError_t persist_blocks_per_cu(int32_t* blocks);
hipError_t launch_xcc_probe(uint32_t* mask, int32_t grid, hipStream_t st);
hipError_t launch_persist(const PLaunch& P, int32_t grid, hipStream_t st);

}  // namespace pv3d
